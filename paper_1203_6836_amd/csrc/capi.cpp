// C-ABI of the sp2qmd library: argument checking, scratch management and the
// host-side sequencing of the HIP kernels.  Every numerical step runs on the
// GPU; the host only enqueues kernels and reads small control records.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <map>
#include <tuple>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sp2qmd.h"
#include "f32_internal.h"
#include "fermi_internal.h"
#include "gemm_internal.h"
#include "noalloc_internal.h"
#include "nonorth_internal.h"
#include "sp2_internal.h"
#include "split_internal.h"
#include "tb_internal.h"

using namespace sp2;

namespace {

// eV / A / amu / fs unit system
constexpr double kAccAFs2 = 9.648533212e-3;  // 1 eV/(A amu) in A/fs^2
constexpr double kKeEv = 103.6426965;        // 1 amu A^2/fs^2 in eV

}  // namespace

// One autotuned launch configuration of the product kernel of a precision.
struct TuneChoice {
    int tile_group = 8;   // super-tile size of the tile order
    int stage_cfg = 0;    // INT8X: K-stage configuration of dense products
    int split_cap = 16;   // FP64: most chunks of a split tile
    int tile = 0;         // FP64: output tile side, 128 or 32 (0 = 32 up to kSmallLd, else 128)
    float ms = 0.f;       // measured ms per product
};

struct sp2_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // token of the host thread inside a call on this context (0: none); a
    // call from another thread meanwhile returns SP2_EBUSY
    std::atomic<unsigned long long> owner{0};
    // device staging of host-memory matrices (sp2_density_matrix_mem,
    // tb_hamiltonian_mem): H, D
    double* stage = nullptr;
    size_t stagecap = 0;
    // SP2 scratch
    double* xbuf = nullptr;   // 2 * ld * ld
    size_t xcap = 0;          // elements per buffer
    double* part = nullptr;
    size_t partcap = 0;
    State* st = nullptr;
    State* st_host = nullptr; // pinned
    double* scal = nullptr;   // device scalars
    double* scal_host = nullptr;
    double* chk = nullptr;    // H check partials (2 per check workgroup)
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    SplitScratch split;       // reduced-precision operands
    bool profile = false;
    std::vector<hipEvent_t> pev;  // 4 per product launch when profiling
    // TB scratch
    double* V = nullptr;
    double* eatom = nullptr;
    double* qtmp = nullptr;
    size_t natcap = 0;
    int* env = nullptr;        // per-panel surviving column-block ranges and block masks (thresholded X)
    size_t envcap = 0;
    int* tz = nullptr;         // per X buffer and upper tile: known all zero (thresholded int8)
    size_t tzcap = 0;
    // non-orthogonal and finite-temperature solves: N x N work buffers (Z,
    // Y / H_perp, T / D_perp, W) plus reduction slots
    double* nobuf = nullptr;
    size_t nocap = 0;
    // non-orthogonal finite-temperature solves: Z, H_perp, D_perp kept
    // across the Fermi-operator and entropy calls (which use nobuf)
    double* ftbuf = nullptr;
    size_t ftcap = 0;
    double* f64tail = nullptr; // chunk accumulators of split last-wave FP64 tiles
    size_t f64tailcap = 0;
    // qmd_evaluate scratch: H[n], D, zero charges, forces
    double* eH = nullptr;
    double* eD = nullptr;
    size_t ecap = 0;           // bytes of each of eH, eD
    double* ezero = nullptr;
    double* eF = nullptr;
    size_t eatcap = 0;         // atoms
    // launch configuration chosen by sp2_autotune (or loaded from a table),
    // per (padded N, precision, slices, levels)
    std::map<std::tuple<int, int, int, int>, TuneChoice> tuned;
    std::string arch;          // device architecture name (gfx...), the tables' key
    int cus = 0;
    // device address of the allocation-free solve's static scratch (NULL if
    // the lookup at creation failed; sscratch_err then holds the HIP error)
    void* sscratch = nullptr;
    hipError_t sscratch_err = hipSuccess;
};

int sp2_ctx_device_of(const sp2_ctx* c) { return c->device; }

static sp2_status fail(sp2_ctx* c, sp2_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

#define HIPCHK(c, expr)                                                                    \
    do {                                                                                   \
        hipError_t _e = (expr);                                                            \
        if (_e != hipSuccess)                                                              \
            return fail((c), SP2_EDEVICE, std::string(#expr " failed: ") + hipGetErrorString(_e)); \
    } while (0)

// One call at a time per context: the first call of a thread takes the
// context, nested calls of the same thread pass, a call of another thread
// meanwhile returns SP2_EBUSY (without touching the error string, which the
// owner may be writing).
static unsigned long long thread_token() {
    static std::atomic<unsigned long long> next{1};
    thread_local unsigned long long t = next.fetch_add(1);
    return t;
}
struct CtxGuard {
    sp2_ctx* c;
    bool owner = false, ok = true;
    explicit CtxGuard(sp2_ctx* ctx) : c(ctx) {
        if (!c) return;
        unsigned long long expected = 0;
        const unsigned long long me = thread_token();
        if (c->owner.compare_exchange_strong(expected, me)) owner = true;
        else ok = expected == me;
    }
    ~CtxGuard() {
        if (owner) c->owner.store(0);
    }
    CtxGuard(const CtxGuard&) = delete;
    CtxGuard& operator=(const CtxGuard&) = delete;
};
#define CTX_ENTER(ctx)                   \
    CtxGuard _ctx_guard(ctx);            \
    if (!_ctx_guard.ok) return SP2_EBUSY

static sp2_status grow(sp2_ctx* c, void** p, size_t* cap, size_t need_bytes) {
    if (*cap >= need_bytes && *p) return SP2_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    if (hipMalloc(p, need_bytes) != hipSuccess) {
        *p = nullptr;
        return fail(c, SP2_ENOMEM, "device allocation of " + std::to_string(need_bytes) + " bytes failed");
    }
    *cap = need_bytes;
    return SP2_OK;
}

// Chunk buffer of the FP64 product's K split (two workgroups per CU, one
// chunk each at most): the sparse last wave of large products and every tile
// of small ones.
static sp2_status f64_tail_buffer(sp2_ctx* c, int ld, int tail_split, double** buf, size_t* bytes) {
    (void)ld;
    *buf = nullptr;
    *bytes = 0;
    if (tail_split == 0) return SP2_OK;
    const size_t need = (size_t)2 * device_cus() * kF64Chunk * sizeof(double);
    sp2_status s = grow(c, (void**)&c->f64tail, &c->f64tailcap, need);
    if (s != SP2_OK) return s;
    *buf = c->f64tail;
    *bytes = c->f64tailcap;
    return SP2_OK;
}

extern "C" {

void sp2_options_default(sp2_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precision = SP2_PREC_FP64;
    o->max_iter = 100;
    o->idem_tol = 1e-10;
    o->stall_tol = 1e-2;
    o->fp64_head = 0;
    o->slices = 5;
    o->fp32_tail = 3;
    o->tau = 0.0;
    o->threshold = 0;
    o->tile_group = -1;
    o->tail_split = -1;
    o->dense_fill = 0.95;
}

const char* sp2_strerror(int s) {
    switch (s) {
        case SP2_OK: return "ok";
        case SP2_EINVAL: return "invalid argument";
        case SP2_ENOMEM: return "device out of memory";
        case SP2_EDEVICE: return "HIP runtime error";
        case SP2_ENOCONV: return "SP2 did not converge within max_iter";
        case SP2_EGAP: return "no resolvable gap at the Fermi level (theta(mu0 I - H) undefined)";
        case SP2_EBUDGET: return "request exceeds the memory budget";
        case SP2_EBUSY: return "context busy with a call from another thread";
        case SP2_ETIMEOUT: return "timed out";
        case SP2_EDIVERGE: return "XL-BOMD auxiliary charges diverged from q";
        default: return "unknown status";
    }
}

const char* sp2_last_error(const sp2_ctx* c) { return c ? c->err.c_str() : "null context"; }

sp2_status sp2_ctx_create(sp2_ctx** out, int device, void* stream) {
    if (!out) return SP2_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return SP2_EDEVICE;
    if (device < 0 || device >= ndev) return SP2_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return SP2_EDEVICE;
    sp2_ctx* c = new sp2_ctx();
    c->device = device;
    c->stream = (hipStream_t)stream;
    if (hipMalloc((void**)&c->st, sizeof(State)) != hipSuccess ||
        hipHostMalloc((void**)&c->st_host, sizeof(State), hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void**)&c->scal, 64 * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&c->chk, 2 * kCheckGrid * sizeof(double)) != hipSuccess ||
        hipHostMalloc((void**)&c->scal_host, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess ||
        hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
        sp2_ctx_destroy(c);
        return SP2_EDEVICE;
    }
    // set-up of the allocation-free solve: the static scratch's address on
    // this device (the device is current)
    c->sscratch_err = static_scratch_init(device, &c->sscratch);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        c->arch = prop.gcnArchName;
        c->arch = c->arch.substr(0, c->arch.find(':'));
        c->cus = prop.multiProcessorCount;
    }
    // an autotuner table named by the environment (missing file: no table)
    if (const char* path = std::getenv("SP2QMD_TUNE_TABLE")) (void)sp2_tune_load(c, path);
    *out = c;
    return SP2_OK;
}

void sp2_ctx_destroy(sp2_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    void* dev[] = {c->xbuf, c->part, c->st, c->scal, c->chk, c->V, c->eatom, c->qtmp, c->env, c->tz,
                   c->eH, c->eD, c->ezero, c->eF, c->f64tail, c->nobuf, c->ftbuf, c->stage};
    for (void* p : dev)
        if (p) (void)hipFree(p);
    split_free(c->split);
    if (c->st_host) (void)hipHostFree(c->st_host);
    if (c->scal_host) (void)hipHostFree(c->scal_host);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    for (hipEvent_t e : c->pev) (void)hipEventDestroy(e);
    delete c;
}

sp2_status sp2_ctx_set_stream(sp2_ctx* c, void* stream) {
    CTX_ENTER(c);
    if (!c) return SP2_EINVAL;
    c->stream = (hipStream_t)stream;
    return SP2_OK;
}

sp2_status sp2_ctx_set_profiling(sp2_ctx* c, int on) {
    CTX_ENTER(c);
    if (!c) return SP2_EINVAL;
    if (on && c->pev.empty()) {
        if (hipSetDevice(c->device) != hipSuccess) return SP2_EDEVICE;
        c->pev.resize(5 * kMaxIter, nullptr);
        for (hipEvent_t& e : c->pev)
            if (hipEventCreate(&e) != hipSuccess) return SP2_EDEVICE;
    }
    c->profile = on != 0;
    return SP2_OK;
}

}  // extern "C"

// ----------------------------------------------------------------- SP2 solve
static sp2_status check_options(sp2_ctx* c, const sp2_options& o, int N) {
    if (o.precision < SP2_PREC_FP64 || o.precision > SP2_PREC_FP32)
        return fail(c, SP2_EINVAL, "unknown precision");
    if (o.max_iter < 1 || o.max_iter > kMaxIter)
        return fail(c, SP2_EINVAL, "max_iter must be in [1, 128]");
    if (!(o.idem_tol > 0.0) || !(o.stall_tol > 0.0)) return fail(c, SP2_EINVAL, "tolerances must be > 0");
    if (o.precision == SP2_PREC_INT8X && (o.slices < 2 || o.slices > kMaxSlices))
        return fail(c, SP2_EINVAL, "slices must be in [2, 6]");
    if (o.precision == SP2_PREC_INT8X && o.levels != 0 && o.levels != o.slices &&
        !(o.levels == o.slices + 1 && o.slices < kMaxSlices))
        return fail(c, SP2_EINVAL, "levels must be 0, slices or slices + 1 (slices < 6)");
    if (o.fp64_head < 0) return fail(c, SP2_EINVAL, "fp64_head must be >= 0");
    if (o.precision == SP2_PREC_BF16X2 && o.fp32_tail < 0) return fail(c, SP2_EINVAL, "fp32_tail must be >= 0");
    if (!(o.tau >= 0.0)) return fail(c, SP2_EINVAL, "tau must be >= 0");
    if (o.tile_group < -1 || o.tile_group > 64) return fail(c, SP2_EINVAL, "tile_group must be in [-1, 64]");
    if (o.tail_split < -1 || o.tail_split > 1) return fail(c, SP2_EINVAL, "tail_split must be -1, 0 or 1");
    if (o.threshold < 0 || o.threshold > 1) return fail(c, SP2_EINVAL, "threshold must be 0 (block) or 1 (element)");
    if (!(o.dense_fill >= 0.0)) return fail(c, SP2_EINVAL, "dense_fill must be >= 0");
    if (o.tau > 0.0 && (o.precision == SP2_PREC_BF16X2 || o.precision == SP2_PREC_FP32))
        return fail(c, SP2_EINVAL, "block thresholding runs with FP64 or INT8X products");
    (void)N;
    return SP2_OK;
}

// Whether a solve with these options forms any product on the FP64 kernel:
// the FP64 mode, and the FP64 head of INT8X and BF16X2.
static bool fp64_products(const sp2_options& o) {
    return o.precision == SP2_PREC_FP64 ||
           ((o.precision == SP2_PREC_INT8X || o.precision == SP2_PREC_BF16X2) && o.fp64_head > 0);
}

// Device scratch of one SP2 solve: the two padded X buffers (2 ld^2 doubles),
// the partial-sum slots, the chunk accumulators of the FP64 product's K split
// (NULL: no split), and for thresholded solves the panel ranges and the
// zero-tile flags with the work list.
struct SolveScratch {
    double* xbuf = nullptr;
    double* part = nullptr;
    double* f64tail = nullptr;
    size_t f64tail_bytes = 0;
    int* env = nullptr;
    int* tz = nullptr;
};

static int padded_ld(int N) { return ((N + kTile - 1) / kTile) * kTile; }

// Digit-product levels of an INT8X solve (0 = slices), 0 for the other
// precisions.
static int int8_levels(const sp2_options& o) {
    if (o.precision != SP2_PREC_INT8X) return 0;
    return o.levels > 0 ? o.levels : o.slices;
}

// The autotuned configuration for (padded N, precision, slices, levels): the
// entry of that size, else the one of the nearest tuned size within a factor
// of 2 (the N bucket; a 32 x 32 tile entry only up to kSmallMaxLd), else the
// defaults.
static TuneChoice tuned_choice(const sp2_ctx* c, int ld, int precision, int slices, int levels) {
    auto it = c->tuned.find(std::make_tuple(ld, precision, slices, levels));
    if (it != c->tuned.end()) return it->second;
    TuneChoice best;
    double dist = 1e300;
    for (const auto& kv : c->tuned) {
        if (std::get<1>(kv.first) != precision || std::get<2>(kv.first) != slices ||
            std::get<3>(kv.first) != levels || (kv.second.tile == 32 && ld > kSmallMaxLd))
            continue;
        const double d = std::fabs(std::log((double)std::get<0>(kv.first) / ld));
        if (d <= std::log(2.0) && d < dist) {
            dist = d;
            best = kv.second;
        }
    }
    return best;
}

// Partial-sum slots any kernel of a solve of size N writes at most.
static size_t solve_part_slots(int N) {
    const int ld = padded_ld(N);
    const int nt = ld / kTile;
    return std::max<size_t>({(size_t)(N + 3) / 4 * 2, (size_t)ld / 4 * 3, (size_t)tri_tiles(nt) * 3, 1024,
                             (size_t)kDotBlocks, split_part_slots(ld) * 3,
                             ld <= kSmallMaxLd ? (size_t)tri_tiles(ld / 32) * 3 : 0});
}

static sp2_status sp2_solve_in(sp2_ctx* c, int N, const double* H, int n_occ, const sp2_options& o, double* D,
                               sp2_stats* stats, const SolveScratch& sc);

// Enqueue and run one SP2 solve of H (device, N x N) into D (device), with
// scratch owned by the context (grown on demand).
static sp2_status sp2_solve(sp2_ctx* c, int N, const double* H, int n_occ, const sp2_options& o, double* D,
                            sp2_stats* stats) {
    const int ld = padded_ld(N);
    const size_t ld2 = (size_t)ld * ld;
    const int nt = ld / kTile;
    sp2_status s;
    size_t xbytes = c->xcap * sizeof(double) * 2;
    if ((s = grow(c, (void**)&c->xbuf, &xbytes, 2 * ld2 * sizeof(double))) != SP2_OK) return s;
    c->xcap = xbytes / (2 * sizeof(double));
    size_t pbytes = c->partcap * sizeof(double);
    if ((s = grow(c, (void**)&c->part, &pbytes, solve_part_slots(N) * sizeof(double))) != SP2_OK) return s;
    c->partcap = pbytes / sizeof(double);
    const bool int8x = o.precision == SP2_PREC_INT8X;
    // BF16X2 and FP32: the BF16 planes and the FP32 copy of X_n
    const bool f32ops = o.precision == SP2_PREC_BF16X2 || o.precision == SP2_PREC_FP32;
    if (int8x || f32ops) {
        if ((s = (sp2_status)split_reserve(c->split, ld, int8x ? o.slices : 0, f32ops)) != SP2_OK)
            return fail(c, SP2_ENOMEM, "device allocation for split operands failed");
    }
    SolveScratch sc;
    sc.xbuf = c->xbuf;
    sc.part = c->part;
    // the FP64 product runs in FP64 mode and in the FP64 head of INT8X and
    // BF16X2
    if (fp64_products(o))
        if ((s = f64_tail_buffer(c, ld, o.tail_split, &sc.f64tail, &sc.f64tail_bytes)) != SP2_OK) return s;
    if (o.tau > 0.0) {
        size_t eb = c->envcap;
        if ((s = grow(c, (void**)&c->env, &eb, env_bytes(ld))) != SP2_OK) return s;
        c->envcap = eb;
        sc.env = c->env;
    }
    // zero-tile flags: int8 products from the first product on (the FP64
    // product does not keep them)
    if (o.tau > 0.0 && int8x && o.fp64_head == 0) {
        size_t zb = c->tzcap;
        // 2 T flags, then the product's work list (T entries) and its 2 counters
        if ((s = grow(c, (void**)&c->tz, &zb, ((size_t)3 * tri_tiles(nt) + 2) * sizeof(int))) != SP2_OK) return s;
        c->tzcap = zb;
        sc.tz = c->tz;
    }
    return sp2_solve_in(c, N, H, n_occ, o, D, stats, sc);
}

static sp2_status sp2_solve_in(sp2_ctx* c, int N, const double* H, int n_occ, const sp2_options& o, double* D,
                               sp2_stats* stats, const SolveScratch& sc) {
    const int ld = padded_ld(N);
    const size_t ld2 = (size_t)ld * ld;
    const int nt = ld / kTile;
    double* buf0 = sc.xbuf;
    double* buf1 = sc.xbuf + ld2;
    double* part = sc.part;
    const bool int8x = o.precision == SP2_PREC_INT8X;
    const bool bf16x = o.precision == SP2_PREC_BF16X2;
    const bool fp32 = o.precision == SP2_PREC_FP32;
    const bool f64p = fp64_products(o);
    // int8 products from the first one on, no threshold: the products write
    // their upper tiles only and the encode reads the upper triangle
    const bool upper = int8x && o.tau == 0.0 && o.fp64_head == 0;
    c->split.upper = upper;
    const TuneChoice tc = tuned_choice(c, ld, o.precision, int8x ? o.slices : 0, int8_levels(o));
    const int tile_group = o.tile_group >= 0 ? o.tile_group : tc.tile_group;
    c->split.tile_group = tile_group;
    c->split.stage_cfg = tc.stage_cfg;
    c->split.tail_split = o.tail_split;
    c->split.levels = int8_levels(o);
    // FP64 products: the tuned split cap and output tile (the 32 x 32 tile
    // kernel in pure FP64 solves only: it writes one partial slot per 32 x 32
    // tile, and does not keep the row maxima of the int8 encode)
    const TuneChoice f64c = tuned_choice(c, ld, SP2_PREC_FP64, 0, 0);
    const bool f64_small =
        !(int8x || bf16x) && ((f64c.tile == 32 && ld <= kSmallMaxLd) || (f64c.tile == 0 && ld <= kSmallLd));

    CtrlArgs a;
    a.n_occ = (double)n_occ;
    a.idem_tol = o.idem_tol;
    // with a threshold the floor of e_n grows with N; below 0.1 every
    // eigenvalue is within 0.113 of 0 or 1, where two products of opposite
    // branches shrink its deviation by more than half.  The int8 products'
    // rounding floor is detected the same way (an error that fails to halve
    // over two products has reached it)
    a.stall_tol = o.tau > 0.0 ? std::max(o.stall_tol, 0.1) : o.stall_tol;
    a.stall_ratio = (o.tau > 0.0 || int8x || fp32) ? 0.5 : 1.0;
    a.max_iter = o.max_iter;
    a.fp64_head = (int8x || bf16x) ? o.fp64_head : -1;
    a.fp32_tail = o.fp32_tail;
    a.mixed = int8x ? 1 : (bf16x ? 2 : (fp32 ? 3 : 0));
    const double nb = (double)((N + 31) / 32);
    a.total_blocks = o.tau > 0.0 ? nb * nb : 0.0;

    double* f64tail = sc.f64tail;
    const size_t f64tail_bytes = sc.f64tail_bytes;
    int* env = sc.env;
    int* tz = sc.tz;
    c->split.env = int8x ? env : nullptr;
    c->split.tz = tz;
    // thresholded int8 products from the first one on (work-list path): the
    // dense tile kernel takes over while X_n's kept fraction is at least
    // dense_fill
    const bool dense_switch = int8x && tz && env && o.dense_fill <= 1.0;
    c->split.dense_switch = dense_switch;
    a.dense_fill = dense_switch ? o.dense_fill : 2.0;
    hipStream_t st = c->stream;
    HIPCHK(c, hipEventRecord(c->ev0, st));
    int ns = 0, nchk = 0;
    HIPCHK(c, launch_check_h(H, N, c->chk, &nchk, st));
    HIPCHK(c, launch_gershgorin(H, N, part, &ns, st));
    HIPCHK(c, launch_bounds(part, ns, c->chk, nchk, c->st, st));
    if (o.tau > 0.0)   // X_0 formed and thresholded in one pass over H
        HIPCHK(c, launch_block_threshold(buf0, buf1, ld, N, o.tau, o.threshold, c->st, part, &ns, 1, st, env, tz,
                                         nullptr, false, H));
    else
        HIPCHK(c, launch_init(H, N, ld, buf0, c->st, part, &ns, st, upper ? c->split.rmax : nullptr));
    HIPCHK(c, launch_ctrl_init(part, ns, c->st, a, st));

    int launched = 0;
    bool finished = false;
    while (launched < o.max_iter) {
        const int chunk = std::min(launched == 0 ? 24 : 8, o.max_iter - launched);
        for (int k = 0; k < chunk; ++k) {
            const int g = launched + k;
            hipEvent_t* pe = c->profile ? &c->pev[5 * g] : nullptr;
            if (pe) HIPCHK(c, hipEventRecord(pe[0], st));
            if (int8x || bf16x) HIPCHK(c, launch_split_encode(c->split, buf0, buf1, ld, c->st, st));
            if (bf16x || fp32) HIPCHK(c, launch_encode_f32(buf0, buf1, ld, c->st, c->split.x32, st));
            if (pe) HIPCHK(c, hipEventRecord(pe[1], st));
            if (f64p)
                HIPCHK(c, launch_gemm_f64(buf0, buf1, ld, c->st, part, &ns, st, env, tile_group, f64tail,
                                          f64tail_bytes, f64c.split_cap, f64_small));
            if (pe) HIPCHK(c, hipEventRecord(pe[2], st));
            if (int8x || bf16x) HIPCHK(c, launch_split_gemm(c->split, buf0, buf1, ld, c->st, part, &ns, st, env));
            if (bf16x || fp32)
                HIPCHK(c, launch_gemm_f32(buf0, buf1, ld, c->st, c->split.x32, part, &ns, tile_group, st));
            if (pe) HIPCHK(c, hipEventRecord(pe[3], st));
            if (o.tau > 0.0)
                HIPCHK(c, launch_block_threshold(buf0, buf1, ld, N, o.tau, o.threshold, c->st, part, &ns, 0, st,
                                                 env, tz, tz ? tz + (size_t)2 * tri_tiles(nt) : nullptr,
                                                 dense_switch));
            if (pe) HIPCHK(c, hipEventRecord(pe[4], st));
            HIPCHK(c, launch_ctrl_step(part, ns, c->st, a, st));
        }
        launched += chunk;
        HIPCHK(c, hipMemcpyAsync(c->st_host, c->st, sizeof(State), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        if (c->st_host->done) {
            finished = true;
            break;
        }
    }
    (void)finished;
    const State& h = *c->st_host;
    if (h.done == 1 || h.done == 2)
        HIPCHK(c, upper ? launch_finalize_upper(buf0, buf1, ld, N, D, c->st, st)
                        : launch_finalize(buf0, buf1, ld, N, D, c->st, st));
    HIPCHK(c, hipEventRecord(c->ev1, st));
    HIPCHK(c, hipEventSynchronize(c->ev1));
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->iterations = h.iter;
        stats->status = h.done - 1;   // 0 converged, 1 stalled, 2 max_iter, 3 gap, 4 invalid H
        stats->fp64_products = h.fp64_products;
        stats->head_switch = h.head_switch;
        stats->eps_min = h.eps_min;
        stats->eps_max = h.eps_max;
        stats->idem_err = h.iter > 0 ? h.idem[h.iter - 1] : 0.0;
        stats->trace = h.t1;
        stats->branch_bits[0] = h.bits[0];
        stats->branch_bits[1] = h.bits[1];
        stats->ms = ms;
        stats->fill_min = h.fill_min;
        stats->fill_max = h.fill_max;
        for (int k = 0; k < kMaxIter && k < 128; ++k) {
            stats->idem_hist[k] = (float)h.idem[k];
            stats->fill_hist[k] = h.fill[k];
        }
        if (c->profile) {
            for (int g = 0; g < h.iter; ++g) {
                float t01 = 0.f, t12 = 0.f, t23 = 0.f, t34 = 0.f;
                HIPCHK(c, hipEventElapsedTime(&t01, c->pev[5 * g], c->pev[5 * g + 1]));
                HIPCHK(c, hipEventElapsedTime(&t12, c->pev[5 * g + 1], c->pev[5 * g + 2]));
                HIPCHK(c, hipEventElapsedTime(&t23, c->pev[5 * g + 2], c->pev[5 * g + 3]));
                HIPCHK(c, hipEventElapsedTime(&t34, c->pev[5 * g + 3], c->pev[5 * g + 4]));
                stats->post_ms += t34;
                // exactly one of the two product kernels did work in launch g
                if (t12 >= t23) {
                    stats->prod_ms[0] += t12;
                    stats->prod_count[0] += 1;
                } else {
                    stats->encode_ms += t01;
                    stats->prod_ms[1] += t23;
                    stats->prod_count[1] += 1;
                }
            }
        }
    }
    if (h.done == 3) return fail(c, SP2_ENOCONV, "SP2 reached max_iter without converging");
    if (h.done == 4)
        return fail(c, SP2_EGAP, "no resolvable HOMO-LUMO gap at the Fermi level: the occupied set is not unique");
    if (h.done == 5) return fail(c, SP2_EINVAL, "H is not finite and symmetric (|H - H^T| > 1e-12 max|H|)");
    return SP2_OK;
}

extern "C" sp2_status sp2_density_matrix(sp2_ctx* c, int N, const double* H, int n_occ, const sp2_options* opt,
                                         double* D_out, sp2_stats* stats) {
    CTX_ENTER(c);
    if (!c) return SP2_EINVAL;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (N < 1 || N > 65536) return fail(c, SP2_EINVAL, "N must be in [1, 65536]");
    if (!H || !D_out) return fail(c, SP2_EINVAL, "null matrix pointer");
    if (n_occ <= 0 || n_occ >= N) return fail(c, SP2_EINVAL, "need 0 < n_occ < N");
    sp2_options o;
    if (opt) o = *opt;
    else sp2_options_default(&o);
    sp2_status s = check_options(c, o, N);
    if (s != SP2_OK) return s;
    HIPCHK(c, hipSetDevice(c->device));
    return sp2_solve(c, N, H, n_occ, o, D_out, stats);
}

// Device staging buffer of at least `elems` doubles (grown on demand).
static sp2_status stage_buffer(sp2_ctx* c, size_t elems, double** out) {
    size_t cap = c->stagecap;
    sp2_status s = grow(c, (void**)&c->stage, &cap, elems * sizeof(double));
    if (s != SP2_OK) return s;
    c->stagecap = cap;
    *out = c->stage;
    return SP2_OK;
}

// sp2_density_matrix with H and D_out in host or device memory: host arrays
// are staged through the context's device buffer (H in, D out after a
// successful solve, then the stream is synchronised).
extern "C" sp2_status sp2_density_matrix_mem(sp2_ctx* c, int N, const double* H, sp2_memkind kind, int n_occ,
                                             const sp2_options* opt, double* D_out, sp2_stats* stats) {
    CTX_ENTER(c);
    if (!c) return SP2_EINVAL;
    if (kind == SP2_MEM_DEVICE) return sp2_density_matrix(c, N, H, n_occ, opt, D_out, stats);
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (kind != SP2_MEM_HOST) return fail(c, SP2_EINVAL, "unknown memory kind");
    if (N < 1 || N > 65536) return fail(c, SP2_EINVAL, "N must be in [1, 65536]");
    if (!H || !D_out) return fail(c, SP2_EINVAL, "null matrix pointer");
    HIPCHK(c, hipSetDevice(c->device));
    const size_t n2 = (size_t)N * N;
    double* Hd = nullptr;
    sp2_status s = stage_buffer(c, 2 * n2, &Hd);
    if (s != SP2_OK) return s;
    double* Dd = Hd + n2;
    HIPCHK(c, hipMemcpyAsync(Hd, H, n2 * sizeof(double), hipMemcpyHostToDevice, c->stream));
    if ((s = sp2_density_matrix(c, N, Hd, n_occ, opt, Dd, stats)) != SP2_OK) return s;
    HIPCHK(c, hipMemcpyAsync(D_out, Dd, n2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SP2_OK;
}

// Allocation-free variant of sp2_density_matrix: FP64 products, no threshold,
// N <= kStaticMaxN, every scratch array carved from the static device array
// (X buffers, partial slots, then the K-split chunk accumulators in the rest).
// Calls no allocating routine: the context's control state, pinned read-back
// record and events were made by sp2_ctx_create.
extern "C" sp2_status sp2_density_matrix_noalloc(sp2_ctx* c, int N, const double* H, int n_occ,
                                                 const sp2_options* opt, double* D_out, sp2_stats* stats) {
    CTX_ENTER(c);
    if (!c) return SP2_EINVAL;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (N < 1 || N > kStaticMaxN)
        return fail(c, SP2_EINVAL, "sp2_density_matrix_noalloc: N must be in [1, " + std::to_string(kStaticMaxN) +
                                       "] (the static scratch holds X buffers up to that size)");
    if (!H || !D_out) return fail(c, SP2_EINVAL, "null matrix pointer");
    if (n_occ <= 0 || n_occ >= N) return fail(c, SP2_EINVAL, "need 0 < n_occ < N");
    sp2_options o;
    if (opt) o = *opt;
    else sp2_options_default(&o);
    sp2_status s = check_options(c, o, N);
    if (s != SP2_OK) return s;
    if (o.precision != SP2_PREC_FP64)
        return fail(c, SP2_EINVAL, "sp2_density_matrix_noalloc: only FP64 products (precision 0)");
    if (o.tau != 0.0) return fail(c, SP2_EINVAL, "sp2_density_matrix_noalloc: no threshold (tau must be 0)");
    if (!c->sscratch)
        return fail(c, SP2_EDEVICE, std::string("static scratch address lookup failed: ") +
                                        hipGetErrorString(c->sscratch_err));
    HIPCHK(c, hipSetDevice(c->device));
    const size_t ld = (size_t)padded_ld(N);
    const auto up256 = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t xbytes = up256(2 * ld * ld * sizeof(double));
    const size_t pbytes = up256(solve_part_slots(N) * sizeof(double));
    if (xbytes + pbytes > kStaticScratchBytes)
        return fail(c, SP2_EINVAL, "sp2_density_matrix_noalloc: size exceeds the static scratch");
    unsigned char* base = static_cast<unsigned char*>(c->sscratch);
    SolveScratch sc;
    sc.xbuf = reinterpret_cast<double*>(base);
    sc.part = reinterpret_cast<double*>(base + xbytes);
    if (o.tail_split != 0) {
        sc.f64tail = reinterpret_cast<double*>(base + xbytes + pbytes);
        sc.f64tail_bytes = kStaticScratchBytes - xbytes - pbytes;
    }
    return sp2_solve_in(c, N, H, n_occ, o, D_out, stats, sc);
}

extern "C" sp2_status sp2_int8_mfma_rate(sp2_ctx* c, double* ops_per_s) {
    CTX_ENTER(c);
    if (!c) return SP2_EINVAL;
    if (!ops_per_s) return fail(c, SP2_EINVAL, "sp2_int8_mfma_rate: NULL output");
    HIPCHK(c, hipSetDevice(c->device));
    int cus = 0;
    HIPCHK(c, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
    const int grid = 4 * cus;     // 16 waves per CU, 4 per SIMD
    const int iters = 80000;      // ~20 ms at the published peak
    const double ops = (double)grid * 4 * iters * kInt8RateOpsPerIter;
    float best = 0.f;
    for (int r = 0; r < 4; ++r) {  // the first launch warms up
        HIPCHK(c, hipEventRecord(c->ev0, c->stream));
        HIPCHK(c, launch_int8_rate(grid, iters, c->scal, c->stream));
        HIPCHK(c, hipEventRecord(c->ev1, c->stream));
        HIPCHK(c, hipEventSynchronize(c->ev1));
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
        if (r > 0 && (best == 0.f || ms < best)) best = ms;
    }
    *ops_per_s = ops / (best * 1e-3);
    return SP2_OK;
}

extern "C" sp2_status sp2_autotune(sp2_ctx* c, int N, int precision, int slices, int levels,
                                   sp2_tune_result* out) {
    CTX_ENTER(c);
    if (!c) return SP2_EINVAL;
    if (N < 1 || N > 65536) return fail(c, SP2_EINVAL, "N must be in [1, 65536]");
    sp2_options o;
    sp2_options_default(&o);
    o.precision = precision;
    if (precision == SP2_PREC_INT8X) {
        o.slices = slices;
        o.levels = levels;
    }
    sp2_status s = check_options(c, o, N);
    if (s != SP2_OK) return s;
    const int nl = int8_levels(o);
    HIPCHK(c, hipSetDevice(c->device));
    const int ld = ((N + kTile - 1) / kTile) * kTile;
    const size_t ld2 = (size_t)ld * ld;
    const int nt = ld / kTile;
    size_t xbytes = c->xcap * sizeof(double) * 2;
    if ((s = grow(c, (void**)&c->xbuf, &xbytes, 2 * ld2 * sizeof(double))) != SP2_OK) return s;
    c->xcap = xbytes / (2 * sizeof(double));
    size_t pbytes = c->partcap * sizeof(double);
    if ((s = grow(c, (void**)&c->part, &pbytes, solve_part_slots(ld) * sizeof(double))) != SP2_OK)
        return s;
    c->partcap = pbytes / sizeof(double);
    const bool int8x = precision == SP2_PREC_INT8X, bf16x = precision == SP2_PREC_BF16X2;
    const bool fp32 = precision == SP2_PREC_FP32;
    if (int8x || bf16x || fp32) {
        if (split_reserve(c->split, ld, int8x ? slices : 0, bf16x || fp32) != 0)
            return fail(c, SP2_ENOMEM, "device allocation for split operands failed");
        c->split.upper = int8x;
        c->split.levels = nl;
        c->split.env = nullptr;
        c->split.tz = nullptr;
        c->split.dense_switch = false;
    }
    double* buf0 = c->xbuf;
    double* buf1 = c->xbuf + ld2;
    hipStream_t st = c->stream;
    // a symmetric operand with the bit activity of real data (the clock of the
    // device depends on it), row maxima 1/2 for the int8 encode, and a state
    // that enables the product of this precision
    HIPCHK(c, launch_fill_test_matrix(buf0, ld, st));
    if (int8x) {
        std::vector<unsigned long long> half(2 * (size_t)ld);
        const double h = 0.5;
        unsigned long long bits;
        std::memcpy(&bits, &h, sizeof(bits));
        std::fill(half.begin(), half.end(), bits);
        HIPCHK(c, hipMemcpy(c->split.rmax, half.data(), half.size() * sizeof(bits), hipMemcpyHostToDevice));
    }
    std::memset(c->st_host, 0, sizeof(State));
    c->st_host->phase = precision == SP2_PREC_FP64 ? 0 : (precision == SP2_PREC_FP32 ? 2 : 1);
    HIPCHK(c, hipMemcpyAsync(c->st, c->st_host, sizeof(State), hipMemcpyHostToDevice, st));
    double* f64tail = nullptr;
    size_t f64tail_bytes = 0;
    if (precision == SP2_PREC_FP64) {
        sp2_status s = f64_tail_buffer(c, ld, -1, &f64tail, &f64tail_bytes);
        if (s != SP2_OK) return s;
    }
    // candidates: tile order G x (INT8X) K-stage configuration or (FP64) the
    // most chunks of a split tile
    std::vector<TuneChoice> cand;
    for (int g : {0, 4, 8, 16, 32}) {
        if (!(g == 0 || g < nt)) continue;
        TuneChoice t;
        t.tile_group = g;
        t.tile = 128;
        if (int8x) {
            for (int cfg = 0; cfg < 3; ++cfg) {
                if (cfg == 2 && slices > 5) continue;
                t.stage_cfg = cfg;
                cand.push_back(t);
            }
        } else if (precision == SP2_PREC_FP64) {
            for (int cap : {8, 16}) {
                t.split_cap = cap;
                cand.push_back(t);
            }
        } else {
            cand.push_back(t);
        }
    }
    // FP64 up to kSmallMaxLd: the 32 x 32 output tile (no tile order, no split)
    if (precision == SP2_PREC_FP64 && ld <= kSmallMaxLd) {
        TuneChoice t;
        t.tile_group = 0;
        t.tile = 32;
        cand.push_back(t);
    }
    // about 40 ms of products per candidate, at least 3
    const double est_ms = (precision == SP2_PREC_FP64 ? 1.0 / 40e9
                           : precision == SP2_PREC_FP32 ? 1.0 / 80e9
                                                        : 1.0 / 1.2e12) * (double)ld * ld * ld;
    const int reps = std::max(3, std::min(40, (int)(40.0 / std::max(est_ms, 1e-3))));
    auto launch = [&](const TuneChoice& t) -> sp2_status {
        int ns = 0;
        c->split.tile_group = t.tile_group;
        c->split.stage_cfg = t.stage_cfg;
        if (precision == SP2_PREC_FP64) {
            HIPCHK(c, launch_gemm_f64(buf0, buf1, ld, c->st, c->part, &ns, st, nullptr, t.tile_group, f64tail,
                                      f64tail_bytes, t.split_cap, t.tile == 32));
        } else if (fp32) {
            HIPCHK(c, launch_encode_f32(buf0, buf1, ld, c->st, c->split.x32, st));
            HIPCHK(c, launch_gemm_f32(buf0, buf1, ld, c->st, c->split.x32, c->part, &ns, t.tile_group, st));
        } else {
            HIPCHK(c, launch_split_encode(c->split, buf0, buf1, ld, c->st, st));
            HIPCHK(c, launch_split_gemm(c->split, buf0, buf1, ld, c->st, c->part, &ns, st, nullptr));
        }
        return SP2_OK;
    };
    TuneChoice best;
    best.ms = 1e30f;
    sp2_tune_result r{};
    std::vector<float> cms(cand.size());
    for (size_t k = 0; k < cand.size(); ++k) {
        if ((s = launch(cand[k])) != SP2_OK) return s;   // warm-up
        HIPCHK(c, hipEventRecord(c->ev0, st));
        for (int q = 0; q < reps; ++q)
            if ((s = launch(cand[k])) != SP2_OK) return s;
        HIPCHK(c, hipEventRecord(c->ev1, st));
        HIPCHK(c, hipEventSynchronize(c->ev1));
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
        ms /= reps;
        if (k < 16) {
            r.candidates[k][0] = cand[k].tile_group;
            r.candidates[k][1] = cand[k].stage_cfg;
            r.candidates[k][2] = cand[k].split_cap;
            r.candidates[k][3] = cand[k].tile;
            r.ms_per_product[k] = ms;
            r.n_candidates = (int)k + 1;
        }
        cms[k] = ms;
        if (ms < best.ms) {
            best = cand[k];
            best.ms = ms;
        }
    }
    // From N = 4096 on operand panels no longer fit the L2 of an XCD and the
    // tile order sets how often they are fetched again; orders whose times
    // differ by less than the run-to-run spread (0.3 %) are then told apart
    // by those re-reads, least first: G = 8 (12 distinct panels per run of
    // 32 tiles), 16 (18), 4, 32, row-major
    if (ld >= 4096) {
        auto rank = [](int g) { return g == 8 ? 0 : g == 16 ? 1 : g == 4 ? 2 : g == 32 ? 3 : 4; };
        const float lim = best.ms * 1.003f;
        TuneChoice pick = best;
        for (size_t k = 0; k < cand.size(); ++k) {
            if (cms[k] > lim || cand[k].tile != 128) continue;
            const int rk = rank(cand[k].tile_group), rp = rank(pick.tile_group);
            if (rk < rp || (rk == rp && cms[k] < pick.ms)) {
                pick = cand[k];
                pick.ms = cms[k];
            }
        }
        best = pick;
    }
    c->split.tile_group = best.tile_group;
    c->split.stage_cfg = best.stage_cfg;
    c->tuned[std::make_tuple(ld, precision, int8x ? slices : 0, nl)] = best;
    r.tile_group = best.tile_group;
    r.stage_cfg = best.stage_cfg;
    r.split_cap = best.split_cap;
    r.tile = best.tile;
    if (out) *out = r;
    return SP2_OK;
}

// Table format: a header line, then one line per tuned configuration:
//   <arch> <compute units> <padded N> <precision> <slices> <levels> <tile_group> <stage_cfg> <split_cap> <tile>
//   <ms>
// (tile: the FP64 output tile side, 128 or 32; 128 for the other precisions)
extern "C" sp2_status sp2_tune_save(const sp2_ctx* c, const char* path) {
    if (!c || !path) return SP2_EINVAL;
    std::ofstream f(path);
    if (!f) return SP2_EINVAL;
    f << "# sp2qmd autotuner table: arch cus ld precision slices levels tile_group stage_cfg split_cap tile "
         "ms_per_product\n";
    for (const auto& kv : c->tuned)
        f << c->arch << ' ' << c->cus << ' ' << std::get<0>(kv.first) << ' ' << std::get<1>(kv.first) << ' '
          << std::get<2>(kv.first) << ' ' << std::get<3>(kv.first) << ' ' << kv.second.tile_group << ' '
          << kv.second.stage_cfg << ' ' << kv.second.split_cap << ' ' << kv.second.tile << ' ' << kv.second.ms
          << '\n';
    return f ? SP2_OK : SP2_EINVAL;
}

extern "C" sp2_status sp2_tune_load(sp2_ctx* c, const char* path) {
    CTX_ENTER(c);
    if (!c || !path) return SP2_EINVAL;
    std::ifstream f(path);
    if (!f) return fail(c, SP2_EINVAL, std::string("cannot read autotuner table ") + path);
    std::string line;
    int loaded = 0;
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#') continue;
        std::istringstream in(line);
        std::string arch;
        int cus, ld, prec, slices, levels;
        TuneChoice t;
        if (!(in >> arch >> cus >> ld >> prec >> slices >> levels >> t.tile_group >> t.stage_cfg >> t.split_cap >>
              t.tile >> t.ms))
            return fail(c, SP2_EINVAL, "malformed autotuner table line: " + line);
        // entries of another device type, or out of range, are skipped
        if (arch != c->arch || cus != c->cus) continue;
        if (ld < kTile || ld % kTile || prec < SP2_PREC_FP64 || prec > SP2_PREC_FP32 || t.tile_group < 0 ||
            t.tile_group > 64 || t.stage_cfg < 0 || t.stage_cfg > 2 || (t.stage_cfg == 2 && slices > 5) ||
            t.split_cap < 2 || t.split_cap > 16 || levels < 0 || levels > slices + 1 ||
            !(t.tile == 128 || (t.tile == 32 && prec == SP2_PREC_FP64 && ld <= kSmallMaxLd)))
            continue;
        c->tuned[std::make_tuple(ld, prec, slices, levels)] = t;
        ++loaded;
    }
    (void)loaded;
    return SP2_OK;
}
// ------------------------------------------------ non-orthogonal formulation
// Row-major C = alpha A B + beta C for N x N matrices: a row-major matrix read
// as column-major is its transpose, so this is the column-major product
// C^T = alpha B^T A^T + beta C^T.
// C = alpha A B + beta C_in + gamma I for a symmetric A (so that A B = A^T B,
// the form the FP64 product kernel reads), N x N, leading dimension N; sym
// when A B is symmetric (A and B symmetric and commuting, or a congruence
// M^T B M): then only the upper tiles are formed and mirrored, and C is
// exactly symmetric.  The K split of sparse last waves uses the context's
// FP64 chunk buffer.
static sp2_status prod(sp2_ctx* c, int N, const double* A, const double* B, double* C, bool sym,
                       double alpha = 1.0, double gamma = 0.0, double beta = 0.0, const double* Cin = nullptr) {
    double* chunk = nullptr;
    size_t chunk_bytes = 0;
    sp2_status s = f64_tail_buffer(c, 0, -1, &chunk, &chunk_bytes);
    if (s != SP2_OK) return s;
    GemmTN g{A, B, Cin, C, N, alpha, beta, gamma};
    HIPCHK(c, launch_gemm_tn(g, sym, 8, chunk, chunk_bytes, c->stream));
    return SP2_OK;
}

constexpr int kNsMaxIter = 40;

// Loewdin factor Z = S^(-1/2) (Eq. Congr) of an N x N overlap by the coupled
// Newton-Schulz iteration, in the context's nobuf: *Z is the factor, *F1 ..
// *F3 the other three N x N work buffers (free for the caller until nobuf
// is next grown); *iters the iterations.
static sp2_status loewdin_factor(sp2_ctx* c, int N, const double* S, double** Zout, double** F1, double** F2,
                                 double** F3, int* iters) {
    sp2_status s;
    const size_t n2 = (size_t)N * N;
    size_t nb = c->nocap;
    if ((s = grow(c, (void**)&c->nobuf, &nb, (4 * n2 + kNsBlocks + 64) * sizeof(double))) != SP2_OK) return s;
    c->nocap = nb;
    double* Zm = c->nobuf;
    double* Y = Zm + n2;
    double* T = Y + n2;
    double* W = T + n2;
    double* part = W + n2;
    double* res = part + kNsBlocks;
    unsigned long long* mx = reinterpret_cast<unsigned long long*>(res + 8);
    hipStream_t st = c->stream;
    HIPCHK(c, launch_zero_word(mx, st));
    HIPCHK(c, launch_row_abs_max(S, N, mx, st));
    HIPCHK(c, launch_ns_init(S, N, mx, Y, Zm, st));
    const double tol = 1e-11 * N;   // ||Z_k Y_k - I||_F: about 1e-11 per element
    double prev = 1e300;
    int it = 0;
    bool converged = false;
    for (; it < kNsMaxIter; ++it) {
        if ((s = prod(c, N, Zm, Y, T, true)) != SP2_OK) return s;        // T = Z_k Y_k (polynomials in S)
        HIPCHK(c, launch_ns_step(T, N, part, st));                      // residual; T = (3 I - T) / 2
        HIPCHK(c, launch_sum_sqrt(part, kNsBlocks, res, st));
        HIPCHK(c, hipMemcpyAsync(c->scal_host, res, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        const double r = c->scal_host[0];
        if (!(r == r)) return fail(c, SP2_EINVAL, "overlap matrix gives a non-finite inverse factor");
        if (r < tol || (it >= 4 && r >= prev && r < 1e-6 * N)) {   // converged, or at its rounding floor
            converged = true;
            break;
        }
        prev = r;
        if ((s = prod(c, N, Y, T, W, true)) != SP2_OK) return s;         // Y_{k+1} = Y_k T_k
        std::swap(Y, W);
        if ((s = prod(c, N, T, Zm, W, true)) != SP2_OK) return s;        // Z_{k+1} = T_k Z_k
        std::swap(Zm, W);
    }
    *iters = it + 1;
    if (!converged) return fail(c, SP2_ENOCONV, "inverse factor of S did not converge (S not positive definite?)");
    HIPCHK(c, launch_scale_inv_sqrt(Zm, N, mx, st));
    *Zout = Zm;
    *F1 = Y;
    *F2 = T;
    *F3 = W;
    return SP2_OK;
}

extern "C" sp2_status sp2_density_matrix_nonorth(sp2_ctx* c, int N, const double* H, const double* S, int n_occ,
                                                  const sp2_options* opt, double* D_out, sp2_stats* stats,
                                                  int* factor_iterations) {
    CTX_ENTER(c);
    if (!c) return SP2_EINVAL;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (factor_iterations) *factor_iterations = 0;
    if (N < 1 || N > 65536 || !H || !S || !D_out) return fail(c, SP2_EINVAL, "bad non-orthogonal solve arguments");
    if (n_occ <= 0 || n_occ >= N) return fail(c, SP2_EINVAL, "need 0 < n_occ < N");
    sp2_options o;
    if (opt) o = *opt;
    else sp2_options_default(&o);
    sp2_status s = check_options(c, o, N);
    if (s != SP2_OK) return s;
    HIPCHK(c, hipSetDevice(c->device));
    double *Zm, *Y, *T, *W;
    int it = 0;
    s = loewdin_factor(c, N, S, &Zm, &Y, &T, &W, &it);
    if (factor_iterations) *factor_iterations = it;
    if (s != SP2_OK) return s;
    hipStream_t st = c->stream;
    // H_perp = Z^T H Z (Z symmetric): W = H Z, then H_perp = W^T Z, formed
    // as a symmetric product (exactly symmetric)
    double* Hp = Y;
    double* Dp = T;
    if ((s = prod(c, N, H, Zm, W, false)) != SP2_OK) return s;
    if ((s = prod(c, N, W, Zm, Hp, true)) != SP2_OK) return s;
    // rho_perp = theta(mu0 I - H_perp) by SP2, then rho = Z rho_perp Z^T the same way
    if ((s = sp2_solve(c, N, Hp, n_occ, o, Dp, stats)) != SP2_OK) return s;
    if ((s = prod(c, N, Dp, Zm, W, false)) != SP2_OK) return s;
    if ((s = prod(c, N, W, Zm, D_out, true)) != SP2_OK) return s;
    HIPCHK(c, hipStreamSynchronize(st));
    return SP2_OK;
}

// ---------------------------------------------- finite electronic temperature
// One pass of the recursive Fermi-operator expansion at chemical potential mu:
// X_0 = I/2 - beta (H - mu I) / 2^(n+2), then n steps
// X_{k+1} = X_k^2 (X_k^2 + (I - X_k)^2)^(-1), each made exactly symmetric.
// delta0 bounds |x - 1/2| over the spectrum of X_0 (from the Gershgorin
// interval); under the step, a bound d becomes 2 d / (1 + 4 d^2), which sets
// the Newton-Schulz start and update count of each inverse.
// buf holds five N x N matrices; returns the one holding X_n.
static sp2_status fermi_pass(sp2_ctx* c, int N, const double* H, double mu, double beta, int n_steps, double delta0,
                             double* buf, double** Xn, long long* products) {
    const size_t n2 = (size_t)N * N;
    double* X = buf;
    double* X2 = buf + n2;
    double* A = buf + 2 * n2;
    double* Y = buf + 3 * n2;
    double* R = buf + 4 * n2;
    hipStream_t st = c->stream;
    sp2_status s;
    HIPCHK(c, launch_fermi_init(H, N, mu, beta / std::ldexp(1.0, n_steps + 2), X, st));
    double delta = delta0;
    for (int k = 0; k < n_steps; ++k) {
        const double db = std::min(0.5, delta * 1.01 + 1e-9);   // margin for rounding
        const double rho = 2.0 * db * db / (1.0 + 2.0 * db * db);
        int updates = 0;   // error rho^2 after Y_1, squared by each update
        for (double err = rho * rho; err > kFermiInvErr && updates < kFermiInvUpdates; err *= err) ++updates;
        // every factor is a polynomial in H: the products are symmetric
        if ((s = prod(c, N, X, X, X2, true)) != SP2_OK) return s;
        HIPCHK(c, launch_fermi_a(X2, X, N, 2.0 / (1.0 + 2.0 * db * db), A, Y, st));   // A, Y_1
        double* W = X;                                        // X is free until X_{k+1}
        for (int j = 0; j < updates; ++j) {
            if ((s = prod(c, N, A, Y, R, true, -1.0, 2.0)) != SP2_OK) return s;   // R = 2 I - A Y
            if ((s = prod(c, N, Y, R, W, true)) != SP2_OK) return s;               // Y <- Y (2 I - A Y)
            std::swap(Y, W);
        }
        if ((s = prod(c, N, X2, Y, W, true)) != SP2_OK) return s;      // X_{k+1} = X_k^2 A^(-1)
        X = W;
        *products += 2 + 2 * updates;
        delta = std::min(0.5, 2.0 * delta / (1.0 + 4.0 * delta * delta));
    }
    *Xn = X;
    return SP2_OK;
}

extern "C" sp2_status sp2_fermi_density_matrix(sp2_ctx* c, int N, const double* H, double n_occ, double kT,
                                                int n_steps, int max_newton, double tol, double* mu,
                                                double* D_out, int* newton_iterations, long long* products) {
    CTX_ENTER(c);
    if (!c) return SP2_EINVAL;
    if (newton_iterations) *newton_iterations = 0;
    if (products) *products = 0;
    long long nprod = 0;
    if (N < 1 || N > 32768 || !H || !D_out || !mu) return fail(c, SP2_EINVAL, "bad Fermi-operator arguments");
    if (!(kT > 0.0) || !std::isfinite(kT)) return fail(c, SP2_EINVAL, "need a finite kT > 0");
    if (n_steps < 1 || n_steps > 60) return fail(c, SP2_EINVAL, "need 1 <= n_steps <= 60");
    if (max_newton < 0 || max_newton > 1000) return fail(c, SP2_EINVAL, "need 0 <= max_newton <= 1000");
    if (max_newton > 0 && (!(n_occ > 0.0) || !(n_occ < N) || !(tol > 0.0)))
        return fail(c, SP2_EINVAL, "need 0 < n_occ < N and tol > 0");
    if (max_newton == 0 && !std::isfinite(*mu)) return fail(c, SP2_EINVAL, "a fixed mu must be finite");
    HIPCHK(c, hipSetDevice(c->device));
    sp2_status s;
    const size_t n2 = (size_t)N * N;
    size_t nb = c->nocap;
    if ((s = grow(c, (void**)&c->nobuf, &nb, (5 * n2 + 2 * kFermiBlocks + 8) * sizeof(double))) != SP2_OK) return s;
    c->nocap = nb;
    double* part = c->nobuf + 5 * n2;
    double* res = part + 2 * kFermiBlocks;
    // the Gershgorin pass writes a (min, max) pair per 4 rows into c->part
    size_t pbytes = c->partcap * sizeof(double);
    if ((s = grow(c, (void**)&c->part, &pbytes, std::max<size_t>((size_t)(N + 3) / 4 * 2, 1024) * sizeof(double))) !=
        SP2_OK)
        return s;
    c->partcap = pbytes / sizeof(double);
    hipStream_t st = c->stream;
    // validity of H and its Gershgorin interval
    int ns = 0, nchk = 0;
    HIPCHK(c, launch_check_h(H, N, c->chk, &nchk, st));
    HIPCHK(c, launch_gershgorin(H, N, c->part, &ns, st));
    HIPCHK(c, launch_bounds(c->part, ns, c->chk, nchk, c->st, st));
    HIPCHK(c, hipMemcpyAsync(c->st_host, c->st, sizeof(State), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (c->st_host->done == 5) return fail(c, SP2_EINVAL, "H is not finite and symmetric");
    const double e_lo = c->st_host->eps_min, e_hi = c->st_host->eps_max;
    const double beta = 1.0 / kT;
    // the root stays bracketed: below e_lo - 40 kT every Fermi factor is under
    // e^-40 (Tr < n_occ), above e_hi + 40 kT over 1 - e^-40 (Tr > n_occ)
    double lo = e_lo - 40.0 * kT, hi = e_hi + 40.0 * kT;
    double m = max_newton == 0 ? *mu : (std::isfinite(*mu) && *mu > lo && *mu < hi) ? *mu : 0.5 * (e_lo + e_hi);
    // X_0 has its spectrum in [0, 1] (and A in [1/2, 1]) when
    // beta |e - mu| <= 2^(n+1) over the Gershgorin interval
    const double reach = std::ldexp(1.0, n_steps + 1) / beta;
    if (!(std::max(e_hi - m, m - e_lo) <= reach) || (max_newton > 0 && !(hi - lo <= reach)))
        return fail(c, SP2_EINVAL, "beta |e - mu| can exceed 2^(n_steps + 1): more steps needed");
    const int evals = max_newton == 0 ? 1 : max_newton;
    for (int it = 0; it < evals; ++it) {
        double* X = nullptr;
        const double delta0 = beta * std::max(e_hi - m, m - e_lo) / std::ldexp(1.0, n_steps + 2);
        if ((s = fermi_pass(c, N, H, m, beta, n_steps, delta0, c->nobuf, &X, &nprod)) != SP2_OK) return s;
        if (newton_iterations) *newton_iterations = it + 1;
        if (products) *products = nprod;
        if (max_newton == 0) {
            HIPCHK(c, hipMemcpyAsync(D_out, X, n2 * sizeof(double), hipMemcpyDeviceToDevice, st));
            HIPCHK(c, hipStreamSynchronize(st));
            return SP2_OK;
        }
        HIPCHK(c, launch_trace_fro(X, N, part, st));
        HIPCHK(c, launch_sum_pairs(part, kFermiBlocks, res, st));
        HIPCHK(c, hipMemcpyAsync(c->scal_host, res, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        const double t = c->scal_host[0], fr = c->scal_host[1];
        if (!std::isfinite(t) || !std::isfinite(fr)) return fail(c, SP2_EDEVICE, "non-finite Fermi-operator trace");
        if (std::fabs(t - n_occ) < tol || it + 1 == evals) {
            HIPCHK(c, hipMemcpyAsync(D_out, X, n2 * sizeof(double), hipMemcpyDeviceToDevice, st));
            HIPCHK(c, hipStreamSynchronize(st));
            *mu = m;
            if (std::fabs(t - n_occ) < tol) return SP2_OK;
            return fail(c, SP2_ENOCONV, "Newton on mu did not reach Tr D = n_occ");
        }
        // Newton with dTr X / dmu ~ beta Tr[X (I - X)] (the Fermi function's
        // derivative); a step out of the bracket bisects it instead
        if (t < n_occ) lo = m;
        else hi = m;
        const double d = beta * (t - fr);
        const double nm = d > 0.0 ? m - (t - n_occ) / d : NAN;
        const double next = (nm > lo && nm < hi) ? nm : 0.5 * (lo + hi);
        if (next == m) {   // X_0 cannot resolve a finer mu
            HIPCHK(c, hipMemcpyAsync(D_out, X, n2 * sizeof(double), hipMemcpyDeviceToDevice, st));
            HIPCHK(c, hipStreamSynchronize(st));
            *mu = m;
            return fail(c, SP2_ENOCONV, "tol is below the resolution of Tr D in mu");
        }
        m = next;
    }
    return SP2_OK;
}

// Electronic entropy S / k_B = -2 sum_i [f_i ln f_i + (1 - f_i) ln(1 - f_i)]
// (Eq. Entropy) of the Fermi occupations f_i = (exp(beta (e_i - mu)) + 1)^(-1)
// of H's eigenvalues, as Tr s(beta (H - mu I)) expanded in Chebyshev
// polynomials of Ht = (H - c I) / w over the Gershgorin interval [c - w, c + w].
// s(x) = ln(1 + e^-|x|) + |x| / (1 + e^|x|) is analytic within pi / beta of the
// real axis, so the coefficients fall geometrically.  The moments Tr T_k(Ht)
// come from T_0 .. T_K alone: Tr T_2k = 2 <T_k, T_k> - N and
// Tr T_(2k+1) = 2 <T_(k+1), T_k> - Tr T_1, one product per k.
constexpr int kEntropyNodes = 8192;   // Chebyshev-Gauss nodes of the coefficients
constexpr double kEntropyCoefTol = 1e-13;

static double fermi_entropy_term(double x) {   // s(x) per state, spin not counted
    const double a = std::fabs(x);
    const double e = std::exp(-a);
    return std::log1p(e) + a * e / (1.0 + e);
}

extern "C" sp2_status sp2_fermi_entropy(sp2_ctx* c, int N, const double* H, double mu, double kT, double* S_out,
                                         int* moments) {
    CTX_ENTER(c);
    if (!c) return SP2_EINVAL;
    if (moments) *moments = 0;
    if (N < 1 || N > 32768 || !H || !S_out) return fail(c, SP2_EINVAL, "bad entropy arguments");
    if (!(kT > 0.0) || !std::isfinite(kT) || !std::isfinite(mu)) return fail(c, SP2_EINVAL, "need finite mu and kT > 0");
    HIPCHK(c, hipSetDevice(c->device));
    sp2_status s;
    const size_t n2 = (size_t)N * N;
    const int kmax = kEntropyNodes / 2;
    size_t nb = c->nocap;
    if ((s = grow(c, (void**)&c->nobuf, &nb, (3 * n2 + kmax + 8) * sizeof(double))) != SP2_OK) return s;
    c->nocap = nb;
    size_t pbytes = c->partcap * sizeof(double);
    if ((s = grow(c, (void**)&c->part, &pbytes,
                  std::max<size_t>({(size_t)(N + 3) / 4 * 2, (size_t)kDotBlocks, 1024}) * sizeof(double))) != SP2_OK)
        return s;
    c->partcap = pbytes / sizeof(double);
    hipStream_t st = c->stream;
    int ns = 0, nchk = 0;
    HIPCHK(c, launch_check_h(H, N, c->chk, &nchk, st));
    HIPCHK(c, launch_gershgorin(H, N, c->part, &ns, st));
    HIPCHK(c, launch_bounds(c->part, ns, c->chk, nchk, c->st, st));
    HIPCHK(c, hipMemcpyAsync(c->st_host, c->st, sizeof(State), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (c->st_host->done == 5) return fail(c, SP2_EINVAL, "H is not finite and symmetric");
    const double beta = 1.0 / kT;
    const double ctr = 0.5 * (c->st_host->eps_min + c->st_host->eps_max);
    const double w = std::max(0.5 * (c->st_host->eps_max - c->st_host->eps_min) * (1.0 + 1e-12), 1e-300);
    // coefficients a_k = (2 / M) sum_j s(beta (w t_j + ctr - mu)) cos(k theta_j), t_j = cos theta_j
    std::vector<double> g(kEntropyNodes), a(kmax);
    const double pi = 3.14159265358979323846;
    for (int j = 0; j < kEntropyNodes; ++j)
        g[j] = fermi_entropy_term(beta * (w * std::cos(pi * (j + 0.5) / kEntropyNodes) + ctr - mu));
    // cos(k theta_j) by rotating (cos, sin)(k theta_j) by theta_j, recomputed
    // exactly every 32 orders (rounding stays near 32 ulp)
    std::vector<double> ck(kEntropyNodes), sk(kEntropyNodes), c1(kEntropyNodes), s1(kEntropyNodes);
    for (int j = 0; j < kEntropyNodes; ++j) {
        c1[j] = std::cos(pi * (j + 0.5) / kEntropyNodes);
        s1[j] = std::sin(pi * (j + 0.5) / kEntropyNodes);
    }
    int m = 0;
    for (int k = 0; k < kmax && k < m + 64; ++k) {   // stop after 64 coefficients below the tolerance
        double acc = 0.0;
        if (k % 32 == 0) {
            for (int j = 0; j < kEntropyNodes; ++j) {   // k theta_j reduced mod 2 pi in integers
                const long long r = ((long long)k * (2 * j + 1)) % (4LL * kEntropyNodes);
                ck[j] = std::cos(pi * (double)r / (2.0 * kEntropyNodes));
                sk[j] = std::sin(pi * (double)r / (2.0 * kEntropyNodes));
            }
        } else {
            for (int j = 0; j < kEntropyNodes; ++j) {
                const double cn = ck[j] * c1[j] - sk[j] * s1[j];
                sk[j] = sk[j] * c1[j] + ck[j] * s1[j];
                ck[j] = cn;
            }
        }
        for (int j = 0; j < kEntropyNodes; ++j) acc += g[j] * ck[j];
        a[k] = 2.0 * acc / kEntropyNodes;
        if (std::fabs(a[k]) > kEntropyCoefTol) m = k + 1;
    }
    if (m + 8 >= kmax)
        return fail(c, SP2_EINVAL, "kT too small against the spectral width for the entropy's Chebyshev expansion");
    m = std::max(m, 2);
    const int K = (m + 1) / 2;   // T_0 .. T_K give the moments 0 .. 2K
    double* Ht = c->nobuf;
    double* Tp = Ht + n2;   // T_(k-1)
    double* Tc = Tp + n2;   // T_k
    double* mom = Tc + n2;  // <T_k, T_k>, <T_(k+1), T_k> pairs
    HIPCHK(c, launch_cheb_init(H, N, ctr, 1.0 / w, Ht, Tp, st));   // Tp = T_0 = I
    HIPCHK(c, hipMemcpyAsync(Tc, Ht, n2 * sizeof(double), hipMemcpyDeviceToDevice, st));   // T_1
    HIPCHK(c, launch_dot(Tp, Tc, n2, c->part, &ns, mom, st));   // Tr T_1
    for (int k = 1; k <= K; ++k) {
        // <T_k, T_k> (moment 2k); then T_(k+1) = 2 Ht T_k - T_(k-1) over T_(k-1)
        HIPCHK(c, launch_dot(Tc, Tc, n2, c->part, &ns, mom + 2 * k, st));
        if (k == K) break;
        if ((s = prod(c, N, Ht, Tc, Tp, true, 2.0, 0.0, -1.0, Tp)) != SP2_OK) return s;
        std::swap(Tp, Tc);
        HIPCHK(c, launch_dot(Tc, Tp, n2, c->part, &ns, mom + 2 * k + 1, st));   // <T_(k+1), T_k>
    }
    std::vector<double> h(2 * K + 1);
    HIPCHK(c, hipMemcpyAsync(h.data(), mom, (2 * K + 1) * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    // moments: mu_0 = N, mu_1 = Tr T_1, mu_2k = 2 <T_k, T_k> - N, mu_(2k+1) = 2 <T_(k+1), T_k> - mu_1
    double S = 0.5 * a[0] * N;
    for (int k = 1; k < std::min(m, 2 * K + 1); ++k) {
        const double mk = k == 1 ? h[0] : (k % 2 == 0 ? 2.0 * h[k] - N : 2.0 * h[k] - h[0]);
        S += a[k] * mk;
    }
    if (!std::isfinite(S)) return fail(c, SP2_EDEVICE, "non-finite entropy");
    *S_out = 2.0 * S;
    if (moments) *moments = m;
    return SP2_OK;
}

// Finite electronic temperature in the non-orthogonal basis: the Fermi
// operator of H_perp = Z^T H Z (Z the Loewdin factor) at the canonical mu,
// rho = Z f(H_perp) Z^T, the energy-weighted W = Z f(H_perp) H_perp Z^T of
// the free-energy forces, and the entropy of the occupations.
extern "C" sp2_status sp2_fermi_density_matrix_nonorth(sp2_ctx* c, int N, const double* H, const double* S,
                                                        double n_occ, double kT, int n_steps, int max_newton,
                                                        double tol, double* mu, double* D_out, double* W_out,
                                                        double* entropy_out, int* newton_iterations) {
    CTX_ENTER(c);
    if (!c) return SP2_EINVAL;
    if (newton_iterations) *newton_iterations = 0;
    if (N < 1 || N > 32768 || !H || !S || !D_out || !mu)
        return fail(c, SP2_EINVAL, "bad non-orthogonal Fermi-operator arguments");
    HIPCHK(c, hipSetDevice(c->device));
    const size_t n2 = (size_t)N * N;
    sp2_status s;
    size_t fb = c->ftcap;
    if ((s = grow(c, (void**)&c->ftbuf, &fb, 3 * n2 * sizeof(double))) != SP2_OK) return s;
    c->ftcap = fb;
    double* Zf = c->ftbuf;
    double* Hp = Zf + n2;
    double* Dp = Hp + n2;
    double *Zm, *F1, *F2, *F3;
    int it = 0;
    if ((s = loewdin_factor(c, N, S, &Zm, &F1, &F2, &F3, &it)) != SP2_OK) return s;
    hipStream_t st = c->stream;
    // Z and H_perp = Z^T H Z kept outside nobuf, which the Fermi operator and
    // the entropy reuse
    HIPCHK(c, hipMemcpyAsync(Zf, Zm, n2 * sizeof(double), hipMemcpyDeviceToDevice, st));
    if ((s = prod(c, N, H, Zf, F1, false)) != SP2_OK) return s;
    if ((s = prod(c, N, F1, Zf, Hp, true)) != SP2_OK) return s;
    if ((s = sp2_fermi_density_matrix(c, N, Hp, n_occ, kT, n_steps, max_newton, tol, mu, Dp, newton_iterations,
                                      nullptr)) != SP2_OK)
        return s;
    if (entropy_out && (s = sp2_fermi_entropy(c, N, Hp, *mu, kT, entropy_out, nullptr)) != SP2_OK) return s;
    double* tmp = c->nobuf;   // at least 3 N x N after the calls above
    // rho = Z D_perp Z^T
    if ((s = prod(c, N, Dp, Zf, tmp, false)) != SP2_OK) return s;
    if ((s = prod(c, N, tmp, Zf, D_out, true)) != SP2_OK) return s;
    if (W_out) {
        // W = Z (D_perp H_perp) Z^T; D_perp and H_perp commute, so their
        // product is symmetric
        if ((s = prod(c, N, Dp, Hp, tmp, true)) != SP2_OK) return s;
        if ((s = prod(c, N, tmp, Zf, Dp, false)) != SP2_OK) return s;
        if ((s = prod(c, N, Dp, Zf, W_out, true)) != SP2_OK) return s;
    }
    HIPCHK(c, hipStreamSynchronize(st));
    return SP2_OK;
}

extern "C" sp2_status sp2_mulliken_overlap(sp2_ctx* c, int n_atoms, const double* D, const double* S, double z_val,
                                           double* q_out) {
    CTX_ENTER(c);
    if (!c) return SP2_EINVAL;
    if (n_atoms < 1 || n_atoms > 16384 || !D || !S || !q_out)
        return fail(c, SP2_EINVAL, "bad mulliken arguments");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_mulliken_overlap(D, S, n_atoms, z_val, q_out, c->stream));
    return SP2_OK;
}

extern "C" sp2_status sp2_mulliken(sp2_ctx* c, int n_atoms, const double* D, double z_val, double* q_out) {
    CTX_ENTER(c);
    if (!c) return SP2_EINVAL;
    if (n_atoms < 1 || n_atoms > 16384 || !D || !q_out) return fail(c, SP2_EINVAL, "bad mulliken arguments");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_mulliken(D, n_atoms, z_val, q_out, c->stream));
    return SP2_OK;
}

extern "C" sp2_status sp2_band_energy(sp2_ctx* c, int N, const double* D, const double* H, double* e_host) {
    CTX_ENTER(c);
    if (!c) return SP2_EINVAL;
    if (N < 1 || N > 65536 || !D || !H || !e_host) return fail(c, SP2_EINVAL, "bad band-energy arguments");
    HIPCHK(c, hipSetDevice(c->device));
    sp2_status s;
    size_t pbytes = c->partcap * sizeof(double);
    if ((s = grow(c, (void**)&c->part, &pbytes, (size_t)std::max(1024, kDotBlocks) * sizeof(double))) != SP2_OK)
        return s;
    c->partcap = pbytes / sizeof(double);
    int ns = 0;
    HIPCHK(c, launch_dot(D, H, (size_t)N * N, c->part, &ns, c->scal, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->scal_host, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *e_host = 2.0 * c->scal_host[0];
    return SP2_OK;
}

// ------------------------------------------------------------ tight binding
// Quintic tail coefficients: B0..B2 match value, slope, curvature of the
// exponential at r1; B3..B5 make value, slope, curvature vanish at rcut.
static Radial make_radial(double amp, double r0, double decay, double r1, double rcut) {
    Radial f;
    f.amp = amp;
    f.r0 = r0;
    f.decay = decay;
    f.r1 = r1;
    f.rcut = rcut;
    for (double& b : f.B) b = 0.0;
    if (r1 < rcut) {
        const double z = amp * std::exp(-(r1 - r0) / decay);
        const double b0 = z, b1 = -z / decay, b2 = 0.5 * z / (decay * decay);
        const double d = rcut - r1;
        const double c0 = -(b0 + b1 * d + b2 * d * d);
        const double c1 = -(b1 + 2.0 * b2 * d);
        const double c2 = -2.0 * b2;
        // u = B3 d^3, v = B4 d^4, w = B5 d^5:
        // u + v + w = c0; 3u + 4v + 5w = c1 d; 6u + 12v + 20w = c2 d^2
        const double a1 = c1 * d - 3.0 * c0;
        const double a2 = c2 * d * d - 6.0 * c0;
        const double w = 0.5 * (a2 - 6.0 * a1);
        const double v = a1 - 2.0 * w;
        const double u = c0 - v - w;
        f.B[0] = b0;
        f.B[1] = b1;
        f.B[2] = b2;
        f.B[3] = u / (d * d * d);
        f.B[4] = v / (d * d * d * d);
        f.B[5] = w / (d * d * d * d * d);
    }
    return f;
}

static bool params_ok(const tb_params* p) {
    return p && p->lam > 0 && p->r_cut > 0 && p->r_tail > 0 && p->r_tail <= p->r_cut &&
           (p->pair_a == 0.0 || p->pair_rho > 0) && std::isfinite(p->t0) && std::isfinite(p->hubbard_u);
}

static TBArgs make_tbargs(const tb_params* p) {
    TBArgs a;
    a.eps_s = p->eps_s;
    a.eps_p = p->eps_p;
    a.hubbard_u = p->hubbard_u;
    a.coulomb_k = p->coulomb_k;
    a.hop = make_radial(p->t0, p->r0, p->lam, p->r_tail, p->r_cut);
    a.pair = make_radial(p->pair_a, p->pair_r0, p->pair_a != 0.0 ? p->pair_rho : 1.0, p->r_tail, p->r_cut);
    return a;
}

static sp2_status ensure_atoms(sp2_ctx* c, int nat) {
    if ((size_t)nat <= c->natcap) return SP2_OK;
    void* ps[] = {c->V, c->eatom, c->qtmp};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    c->V = c->eatom = c->qtmp = nullptr;
    c->natcap = 0;
    if (hipMalloc((void**)&c->V, nat * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&c->eatom, nat * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&c->qtmp, nat * sizeof(double)) != hipSuccess)
        return fail(c, SP2_ENOMEM, "atom scratch allocation failed");
    c->natcap = nat;
    return SP2_OK;
}

extern "C" sp2_status tb_hamiltonian(sp2_ctx* c, const tb_params* p, int n_atoms, const double* xyz,
                                     const double* n_aux, double* H_out) {
    CTX_ENTER(c);
    if (!c) return SP2_EINVAL;
    if (!params_ok(p)) return fail(c, SP2_EINVAL, "bad tb_params");
    if (n_atoms < 1 || n_atoms > 16384 || !xyz || !H_out) return fail(c, SP2_EINVAL, "bad tb_hamiltonian arguments");
    HIPCHK(c, hipSetDevice(c->device));
    sp2_status s = ensure_atoms(c, n_atoms);
    if (s != SP2_OK) return s;
    const TBArgs a = make_tbargs(p);
    const double* V = nullptr;
    if (n_aux) {
        HIPCHK(c, launch_potential(xyz, n_aux, n_atoms, p->hubbard_u, p->coulomb_k, c->V, c->stream));
        V = c->V;
    }
    HIPCHK(c, launch_hamiltonian(xyz, n_atoms, a, V, H_out, c->stream));
    return SP2_OK;
}

// tb_hamiltonian with xyz, n_aux and H_out in host or device memory (host
// arrays staged through the context's device buffer; the stream is
// synchronised before returning).
extern "C" sp2_status tb_hamiltonian_mem(sp2_ctx* c, const tb_params* p, int n_atoms, const double* xyz,
                                         const double* n_aux, double* H_out, sp2_memkind kind) {
    CTX_ENTER(c);
    if (!c) return SP2_EINVAL;
    if (kind == SP2_MEM_DEVICE) return tb_hamiltonian(c, p, n_atoms, xyz, n_aux, H_out);
    if (kind != SP2_MEM_HOST) return fail(c, SP2_EINVAL, "unknown memory kind");
    if (n_atoms < 1 || n_atoms > 16384 || !xyz || !H_out) return fail(c, SP2_EINVAL, "bad tb_hamiltonian arguments");
    HIPCHK(c, hipSetDevice(c->device));
    const size_t n2 = (size_t)16 * n_atoms * n_atoms;   // N = 4 n_atoms
    double* Hd = nullptr;
    sp2_status s = stage_buffer(c, n2 + 4 * (size_t)n_atoms, &Hd);
    if (s != SP2_OK) return s;
    double* xd = Hd + n2;
    double* nd = n_aux ? xd + 3 * (size_t)n_atoms : nullptr;
    HIPCHK(c, hipMemcpyAsync(xd, xyz, 3 * (size_t)n_atoms * sizeof(double), hipMemcpyHostToDevice, c->stream));
    if (n_aux)
        HIPCHK(c, hipMemcpyAsync(nd, n_aux, (size_t)n_atoms * sizeof(double), hipMemcpyHostToDevice, c->stream));
    if ((s = tb_hamiltonian(c, p, n_atoms, xd, nd, Hd)) != SP2_OK) return s;
    HIPCHK(c, hipMemcpyAsync(H_out, Hd, n2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SP2_OK;
}

extern "C" sp2_status tb_overlap(sp2_ctx* c, const tb_params* p, double s0, double lam_s, int n_atoms,
                                 const double* xyz, double* S_out) {
    CTX_ENTER(c);
    if (!c) return SP2_EINVAL;
    if (!params_ok(p) || !(s0 >= 0.0) || !(lam_s > 0.0)) return fail(c, SP2_EINVAL, "bad overlap parameters");
    if (n_atoms < 1 || n_atoms > 16384 || !xyz || !S_out) return fail(c, SP2_EINVAL, "bad tb_overlap arguments");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_overlap(xyz, n_atoms, make_radial(s0, p->r0, lam_s, p->r_tail, p->r_cut), S_out, c->stream));
    return SP2_OK;
}

// Non-orthogonal H[n] = h + (S L + L S)/2, L = V_i = (gamma n)_i on the orbitals
// of atom i (h alone when n_aux is NULL).
extern "C" sp2_status tb_hamiltonian_nonorth(sp2_ctx* c, const tb_params* p, int n_atoms, const double* xyz,
                                             const double* n_aux, const double* S, double* H_out) {
    CTX_ENTER(c);
    if (!c) return SP2_EINVAL;
    if (!params_ok(p)) return fail(c, SP2_EINVAL, "bad tb_params");
    if (n_atoms < 1 || n_atoms > 16384 || !xyz || !S || !H_out)
        return fail(c, SP2_EINVAL, "bad tb_hamiltonian_nonorth arguments");
    HIPCHK(c, hipSetDevice(c->device));
    sp2_status s = ensure_atoms(c, n_atoms);
    if (s != SP2_OK) return s;
    HIPCHK(c, launch_hamiltonian(xyz, n_atoms, make_tbargs(p), nullptr, H_out, c->stream));
    if (n_aux) {
        HIPCHK(c, launch_potential(xyz, n_aux, n_atoms, p->hubbard_u, p->coulomb_k, c->V, c->stream));
        HIPCHK(c, launch_overlap_shift(H_out, S, c->V, n_atoms, c->stream));
    }
    return SP2_OK;
}

// Forces and energy; V must already hold gamma n (computed here).
static sp2_status forces_impl(sp2_ctx* c, const tb_params* p, int nat, const double* xyz, const double* D,
                              const double* q, const double* n, double* F, double* U_dev) {
    const TBArgs a = make_tbargs(p);
    HIPCHK(c, launch_potential(xyz, n, nat, p->hubbard_u, p->coulomb_k, c->V, c->stream));
    HIPCHK(c, launch_forces(xyz, nat, a, D, q, n, c->V, F, c->eatom, U_dev, c->stream));
    return SP2_OK;
}

// Non-orthogonal forces at constant n: the orthogonal terms with the overlap
// charges q, plus sum_ab M_ab dS_ab/dR_k with M = 2 W - (V_a + V_b) D_ab, W
// the energy-weighted density matrix (Wen; NULL: D H D, its form for an
// idempotent D); U to the device slot U_dev.
static sp2_status tb_forces_nonorth_impl(sp2_ctx* c, const tb_params* p, double s0, double lam_s, int n_atoms,
                                         const double* xyz, const double* D, const double* H, const double* q,
                                         const double* n, double* F, double* U_dev, const double* Wen = nullptr) {
    sp2_status s = ensure_atoms(c, n_atoms);
    if (s != SP2_OK) return s;
    const int N = 4 * n_atoms;
    const size_t n2 = (size_t)N * N;
    size_t nb = c->nocap;
    if ((s = grow(c, (void**)&c->nobuf, &nb, (4 * n2 + kNsBlocks + 64) * sizeof(double))) != SP2_OK) return s;
    c->nocap = nb;
    double* W1 = c->nobuf;
    double* W2 = W1 + n2;
    // orthogonal terms (band with h, Coulomb with q, pair) and U; V = gamma n
    if ((s = forces_impl(c, p, n_atoms, xyz, D, q, n, F, U_dev)) != SP2_OK) return s;
    // energy-weighted density matrix D H D (= (H D)^T D), or the one given,
    // then M in place
    if (Wen) {
        HIPCHK(c, hipMemcpyAsync(W2, Wen, n2 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    } else {
        if ((s = prod(c, N, H, D, W1, false)) != SP2_OK) return s;
        if ((s = prod(c, N, W1, D, W2, true)) != SP2_OK) return s;
    }
    HIPCHK(c, launch_force_matrix(W2, D, c->V, n_atoms, c->stream));
    HIPCHK(c, launch_forces_overlap(xyz, n_atoms, make_radial(s0, p->r0, lam_s, p->r_tail, p->r_cut), W2, F,
                                    c->stream));
    return SP2_OK;
}

extern "C" sp2_status tb_forces_nonorth(sp2_ctx* c, const tb_params* p, double s0, double lam_s, int n_atoms,
                                        const double* xyz, const double* D, const double* H, const double* q,
                                        const double* n_aux, double* F_out, double* U_host) {
    CTX_ENTER(c);
    if (!c) return SP2_EINVAL;
    if (!params_ok(p) || !(s0 >= 0.0) || !(lam_s > 0.0)) return fail(c, SP2_EINVAL, "bad overlap parameters");
    if (n_atoms < 1 || n_atoms > 16384 || !xyz || !D || !H || !q || !n_aux || !F_out)
        return fail(c, SP2_EINVAL, "bad tb_forces_nonorth arguments");
    HIPCHK(c, hipSetDevice(c->device));
    sp2_status s = ensure_atoms(c, n_atoms);
    if (s != SP2_OK) return s;
    if ((s = tb_forces_nonorth_impl(c, p, s0, lam_s, n_atoms, xyz, D, H, q, n_aux, F_out, c->scal)) != SP2_OK)
        return s;
    if (U_host) {
        HIPCHK(c, hipMemcpyAsync(c->scal_host, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        *U_host = c->scal_host[0];
    }
    return SP2_OK;
}

extern "C" sp2_status tb_forces(sp2_ctx* c, const tb_params* p, int n_atoms, const double* xyz, const double* D,
                                const double* q, const double* n_aux, double* F_out, double* U_host) {
    CTX_ENTER(c);
    if (!c) return SP2_EINVAL;
    if (!params_ok(p)) return fail(c, SP2_EINVAL, "bad tb_params");
    if (n_atoms < 1 || n_atoms > 16384 || !xyz || !D || !q || !n_aux)
        return fail(c, SP2_EINVAL, "bad tb_forces arguments");
    HIPCHK(c, hipSetDevice(c->device));
    sp2_status s = ensure_atoms(c, n_atoms);
    if (s != SP2_OK) return s;
    if ((s = forces_impl(c, p, n_atoms, xyz, D, q, n_aux, F_out, c->scal)) != SP2_OK) return s;
    if (U_host) {
        HIPCHK(c, hipMemcpyAsync(c->scal_host, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        *U_host = c->scal_host[0];
    }
    return SP2_OK;
}

extern "C" sp2_status qmd_evaluate(sp2_ctx* c, const tb_params* p, int n_atoms, const double* xyz,
                                   const double* n_aux, int n_occ, const sp2_options* opt, double* q_out,
                                   double* e_band_host, double* e_pot_host, double* F_out, sp2_stats* stats) {
    CTX_ENTER(c);
    if (!c) return SP2_EINVAL;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (!params_ok(p)) return fail(c, SP2_EINVAL, "bad tb_params");
    if (n_atoms < 1 || n_atoms > 16384 || !xyz || !q_out) return fail(c, SP2_EINVAL, "bad qmd_evaluate arguments");
    const int N = 4 * n_atoms;
    if (n_occ <= 0 || n_occ >= N) return fail(c, SP2_EINVAL, "need 0 < n_occ < 4 n_atoms");
    sp2_options o;
    if (opt) o = *opt;
    else sp2_options_default(&o);
    sp2_status s = check_options(c, o, N);
    if (s != SP2_OK) return s;
    HIPCHK(c, hipSetDevice(c->device));
    if ((s = ensure_atoms(c, n_atoms)) != SP2_OK) return s;
    const size_t mat = (size_t)N * N * sizeof(double);
    if (c->ecap < mat) {
        size_t a = c->ecap, b = c->ecap;
        if ((s = grow(c, (void**)&c->eH, &a, mat)) != SP2_OK) return s;
        if ((s = grow(c, (void**)&c->eD, &b, mat)) != SP2_OK) return s;
        c->ecap = mat;
    }
    if ((size_t)n_atoms > c->eatcap) {
        size_t a = c->eatcap * sizeof(double), b = 3 * c->eatcap * sizeof(double);
        if ((s = grow(c, (void**)&c->ezero, &a, n_atoms * sizeof(double))) != SP2_OK) return s;
        if ((s = grow(c, (void**)&c->eF, &b, 3 * n_atoms * sizeof(double))) != SP2_OK) return s;
        c->eatcap = n_atoms;
    }
    hipStream_t st = c->stream;
    const double* n = n_aux;
    if (!n) {
        HIPCHK(c, hipMemsetAsync(c->ezero, 0, n_atoms * sizeof(double), st));
        n = c->ezero;
    }
    if ((s = tb_hamiltonian(c, p, n_atoms, xyz, n, c->eH)) != SP2_OK) return s;
    if ((s = sp2_solve(c, N, c->eH, n_occ, o, c->eD, stats)) != SP2_OK) return s;
    HIPCHK(c, launch_mulliken(c->eD, n_atoms, p->z_val, q_out, st));
    int ns = 0;
    if (e_band_host) HIPCHK(c, launch_dot(c->eD, c->eH, (size_t)N * N, c->part, &ns, c->scal + 1, st));
    if (F_out || e_pot_host)
        if ((s = forces_impl(c, p, n_atoms, xyz, c->eD, q_out, n, F_out ? F_out : c->eF, c->scal)) != SP2_OK)
            return s;
    if (e_band_host || e_pot_host) {
        HIPCHK(c, hipMemcpyAsync(c->scal_host, c->scal, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        if (e_pot_host) *e_pot_host = c->scal_host[0];
        if (e_band_host) *e_band_host = 2.0 * c->scal_host[1];
    }
    return SP2_OK;
}

// ------------------------------------------------------------------ XL-BOMD
struct xlbomd {
    sp2_ctx* c;
    tb_params p;
    xlbomd_options o;
    int nat;
    int n_occ;            // doubly occupied states: z_val n_atoms / 2
    double *xyz, *vel, *F, *q, *hist, *H, *D, *dev, *dscal;
    double* S = nullptr;  // overlap (non-orthogonal basis only)
    double* Wen = nullptr;  // energy-weighted density matrix (non-orthogonal basis at kT > 0)
    double mu = NAN;      // chemical potential of the last Fermi operator (kT > 0)
    double ts = 0.0;      // kT S of the last Fermi operator
    int head;
    long step;
    double U;
    int scf_iterations;
    double scf_residual;
    long long dm_count;   // density matrices built
};

static sp2_status md_evaluate(xlbomd* m, int* iters, bool with_forces = true, float* fill = nullptr) {
    sp2_ctx* c = m->c;
    const int nat = m->nat, N = 4 * nat;
    const double* n_t = m->hist + (size_t)m->head * nat;
    sp2_status s = tb_hamiltonian(c, &m->p, nat, m->xyz, n_t, m->H);
    if (s != SP2_OK) return s;
    sp2_stats st;
    if (m->o.kT > 0.0 && m->S) {
        // finite electronic temperature in the non-orthogonal basis: overlap,
        // H[n] with it, the Fermi operator of H_perp (canonical mu), its
        // entropy, charges with S and the free-energy forces with W
        if ((s = tb_overlap(c, &m->p, m->o.overlap_s0, m->o.overlap_lam, nat, m->xyz, m->S)) != SP2_OK) return s;
        if ((s = tb_hamiltonian_nonorth(c, &m->p, nat, m->xyz, n_t, m->S, m->H)) != SP2_OK) return s;
        int passes = 0;
        double Se = 0.0;
        if ((s = sp2_fermi_density_matrix_nonorth(c, N, m->H, m->S, (double)m->n_occ, m->o.kT, m->o.fermi_steps,
                                                  m->o.fermi_max_newton, m->o.fermi_tol, &m->mu, m->D, m->Wen,
                                                  &Se, &passes)) != SP2_OK)
            return s;
        m->ts = m->o.kT * Se;
        m->dm_count += 1;
        if (iters) *iters = passes;
        if (fill) *fill = 1.0f;
        HIPCHK(c, launch_mulliken_overlap(m->D, m->S, nat, m->p.z_val, m->q, c->stream));
        if (!with_forces) return SP2_OK;
        return tb_forces_nonorth_impl(c, &m->p, m->o.overlap_s0, m->o.overlap_lam, nat, m->xyz, m->D, m->H, m->q,
                                      n_t, m->F, m->dscal, m->Wen);
    }
    if (m->o.kT > 0.0) {
        // finite electronic temperature: the Fermi operator at the canonical mu
        // (from the previous step's), its entropy, charges and forces
        int passes = 0;
        if ((s = sp2_fermi_density_matrix(c, N, m->H, (double)m->n_occ, m->o.kT, m->o.fermi_steps,
                                          m->o.fermi_max_newton, m->o.fermi_tol, &m->mu, m->D, &passes, nullptr)) !=
            SP2_OK)
            return s;
        double S = 0.0;
        if ((s = sp2_fermi_entropy(c, N, m->H, m->mu, m->o.kT, &S, nullptr)) != SP2_OK) return s;
        m->ts = m->o.kT * S;
        m->dm_count += 1;
        if (iters) *iters = passes;
        if (fill) *fill = 1.0f;
        HIPCHK(c, launch_mulliken(m->D, nat, m->p.z_val, m->q, c->stream));
        if (!with_forces) return SP2_OK;
        return forces_impl(c, &m->p, nat, m->xyz, m->D, m->q, n_t, m->F, m->dscal);
    }
    if (m->S) {
        // non-orthogonal basis: overlap at these positions, H[n] with it, the
        // density matrix through the Loewdin factor, charges and forces with S
        if ((s = tb_overlap(c, &m->p, m->o.overlap_s0, m->o.overlap_lam, nat, m->xyz, m->S)) != SP2_OK) return s;
        if ((s = tb_hamiltonian_nonorth(c, &m->p, nat, m->xyz, n_t, m->S, m->H)) != SP2_OK) return s;
        if ((s = sp2_density_matrix_nonorth(c, N, m->H, m->S, m->n_occ, &m->o.sp2, m->D, &st, nullptr)) != SP2_OK)
            return s;
        m->dm_count += 1;
        if (iters) *iters = st.iterations;
        if (fill) *fill = m->o.sp2.tau > 0.0 ? (float)st.fill_min : 1.0f;
        HIPCHK(c, launch_mulliken_overlap(m->D, m->S, nat, m->p.z_val, m->q, c->stream));
        if (!with_forces) return SP2_OK;
        return tb_forces_nonorth_impl(c, &m->p, m->o.overlap_s0, m->o.overlap_lam, nat, m->xyz, m->D, m->H, m->q,
                                      n_t, m->F, m->dscal);
    }
    s = sp2_solve(c, N, m->H, m->n_occ, m->o.sp2, m->D, &st);
    if (s != SP2_OK) return s;
    m->dm_count += 1;
    if (iters) *iters = st.iterations;
    if (fill) *fill = m->o.sp2.tau > 0.0 ? (float)st.fill_min : 1.0f;
    HIPCHK(c, launch_mulliken(m->D, nat, m->p.z_val, m->q, c->stream));
    if (!with_forces) return SP2_OK;
    return forces_impl(c, &m->p, nat, m->xyz, m->D, m->q, n_t, m->F, m->dscal);
}

extern "C" sp2_status xlbomd_create(sp2_ctx* c, const tb_params* p, const xlbomd_options* o, int n_atoms,
                                    const double* xyz_host, const double* vel_host, const double* n0_host,
                                    xlbomd** out) {
    CTX_ENTER(c);
    if (!c) return SP2_EINVAL;
    if (!out || !params_ok(p) || !o || !xyz_host || !vel_host)
        return fail(c, SP2_EINVAL, "bad xlbomd_create arguments");
    if (o->scf_max_iter < 0 || (o->scf_max_iter == 0 && !n0_host))
        return fail(c, SP2_EINVAL, "scf_max_iter == 0 needs n0");
    if (o->scf_max_iter > 0 && (!(o->scf_beta > 0.0 && o->scf_beta <= 1.0) || !(o->scf_tol > 0.0)))
        return fail(c, SP2_EINVAL, "SCF start needs 0 < scf_beta <= 1 and scf_tol > 0");
    *out = nullptr;
    if (n_atoms < 2 || n_atoms > 16384) return fail(c, SP2_EINVAL, "n_atoms out of range");
    // neutral atoms with z_val valence electrons in doubly occupied states
    const double electrons = p->z_val * n_atoms;
    const long n_occ = std::lround(electrons / 2.0);
    if (!(std::fabs(electrons - 2.0 * (double)n_occ) < 1e-9) || n_occ <= 0 || n_occ >= 4L * n_atoms)
        return fail(c, SP2_EINVAL, "z_val * n_atoms must be an even electron count below 8 n_atoms");
    if (o->K < 1 || o->K > 8 || !(o->dt_fs > 0) || !(p->mass > 0) || !(o->diverge_q >= 0))
        return fail(c, SP2_EINVAL, "bad xlbomd options");
    if (!(o->kT >= 0.0) || !std::isfinite(o->kT) ||
        (o->kT > 0.0 && (o->fermi_steps < 1 || o->fermi_steps > 60)))
        return fail(c, SP2_EINVAL, "kT > 0 needs 1 <= fermi_steps <= 60");
    if (!(o->overlap_s0 >= 0.0) || (o->overlap_s0 > 0.0 && !(o->overlap_lam > 0.0)))
        return fail(c, SP2_EINVAL, "bad overlap parameters");
    if (!(o->fermi_tol >= 0.0) || !std::isfinite(o->fermi_tol) || o->fermi_max_newton < 0 ||
        o->fermi_max_newton > 1000)
        return fail(c, SP2_EINVAL, "need fermi_tol >= 0 and 0 <= fermi_max_newton <= 1000");
    sp2_status s = check_options(c, o->sp2, 4 * n_atoms);
    if (s != SP2_OK) return s;
    HIPCHK(c, hipSetDevice(c->device));
    if ((s = ensure_atoms(c, n_atoms)) != SP2_OK) return s;
    xlbomd* m = new xlbomd();
    m->c = c;
    m->p = *p;
    m->o = *o;
    // finite-T defaults: Tr D to 1e-9 per 512 orbitals (X_0 quantises the
    // trace at about 1e-10 per 512 orbitals for 16 recursion steps), 100 passes
    if (m->o.fermi_tol == 0.0) m->o.fermi_tol = 1e-9 * std::max(1.0, (double)(4 * n_atoms) / 512.0);
    if (m->o.fermi_max_newton == 0) m->o.fermi_max_newton = 100;
    m->nat = n_atoms;
    m->n_occ = (int)n_occ;
    const size_t N = 4 * (size_t)n_atoms;
    const int L = o->K + 1;
    double** bufs[] = {&m->xyz, &m->vel, &m->F, &m->q, &m->dev};
    bool ok = true;
    for (double** b : bufs) ok = ok && hipMalloc((void**)b, 3 * n_atoms * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc((void**)&m->hist, (size_t)L * n_atoms * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc((void**)&m->H, N * N * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc((void**)&m->D, N * N * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc((void**)&m->dscal, 8 * sizeof(double)) == hipSuccess;
    if (o->overlap_s0 > 0.0) ok = ok && hipMalloc((void**)&m->S, N * N * sizeof(double)) == hipSuccess;
    if (o->overlap_s0 > 0.0 && o->kT > 0.0)
        ok = ok && hipMalloc((void**)&m->Wen, N * N * sizeof(double)) == hipSuccess;
    if (!ok) {
        xlbomd_destroy(m);
        return fail(c, SP2_ENOMEM, "xlbomd allocation failed");
    }
    hipStream_t st = c->stream;
    HIPCHK(c, hipMemcpyAsync(m->xyz, xyz_host, 3 * n_atoms * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(m->vel, vel_host, 3 * n_atoms * sizeof(double), hipMemcpyHostToDevice, st));
    m->head = 0;
    m->scf_iterations = 0;
    m->scf_residual = 0.0;
    if (o->scf_max_iter == 0) {
        for (int k = 0; k < L; ++k)
            HIPCHK(c, hipMemcpyAsync(m->hist + (size_t)k * n_atoms, n0_host, n_atoms * sizeof(double),
                                     hipMemcpyHostToDevice, st));
    } else {
        // self-consistent start: n <- n + beta (q[n] - n) from the guess n0 (or 0)
        if (n0_host)
            HIPCHK(c, hipMemcpyAsync(m->hist, n0_host, n_atoms * sizeof(double), hipMemcpyHostToDevice, st));
        else
            HIPCHK(c, hipMemsetAsync(m->hist, 0, n_atoms * sizeof(double), st));
        bool conv = false;
        for (int it = 0; it < o->scf_max_iter; ++it) {
            if ((s = md_evaluate(m, nullptr, false)) != SP2_OK) {
                xlbomd_destroy(m);
                return s;
            }
            HIPCHK(c, launch_maxdiff(m->q, m->hist, n_atoms, m->dev, m->dscal + 1, st));
            HIPCHK(c, hipMemcpyAsync(c->scal_host, m->dscal + 1, sizeof(double), hipMemcpyDeviceToHost, st));
            HIPCHK(c, hipStreamSynchronize(st));
            m->scf_iterations = it + 1;
            m->scf_residual = c->scal_host[0];
            if (m->scf_residual < o->scf_tol) {
                conv = true;
                break;
            }
            HIPCHK(c, launch_mix(m->hist, m->q, n_atoms, o->scf_beta, st));
        }
        if (!conv) {
            xlbomd_destroy(m);
            return fail(c, SP2_ENOCONV, "SCF start did not converge");
        }
        for (int k = 0; k < L; ++k)   // n = q for the whole history
            HIPCHK(c, hipMemcpyAsync(m->hist + (size_t)k * n_atoms, m->q, n_atoms * sizeof(double),
                                     hipMemcpyDeviceToDevice, st));
    }
    m->step = 0;
    if ((s = md_evaluate(m, nullptr)) != SP2_OK) {
        xlbomd_destroy(m);
        return s;
    }
    HIPCHK(c, hipStreamSynchronize(st));
    *out = m;
    return SP2_OK;
}

extern "C" sp2_status xlbomd_run(xlbomd* m, int n_steps, xlbomd_record* log) {
    CTX_ENTER(m ? m->c : nullptr);
    if (!m) return SP2_EINVAL;
    sp2_ctx* c = m->c;
    if (n_steps < 0) return fail(c, SP2_EINVAL, "n_steps < 0");
    HIPCHK(c, hipSetDevice(c->device));
    const int nat = m->nat, K = m->o.K, L = K + 1;
    const double hacc = 0.5 * m->o.dt_fs * kAccAFs2 / m->p.mass;
    XLArgs xa;
    xa.kappa = m->o.kappa;
    xa.alpha = m->o.alpha;
    for (int k = 0; k < 9; ++k) xa.c[k] = k <= K ? m->o.c[k] : 0.0;
    hipStream_t st = c->stream;
    for (int step = 0; step < n_steps; ++step) {
        HIPCHK(c, launch_kick_drift(m->xyz, m->vel, m->F, 3 * nat, hacc, m->o.dt_fs, st));
        HIPCHK(c, launch_xl_charges(m->hist, nat, K, m->head, m->q, xa, st));
        m->head = (m->head + K) % L;
        int iters = 0;
        float fill = 1.0f;
        sp2_status s = md_evaluate(m, &iters, true, &fill);
        if (s != SP2_OK) return s;
        HIPCHK(c, launch_maxdiff(m->q, m->hist + (size_t)m->head * nat, nat, m->dev, m->dscal + 1, st));
        HIPCHK(c, launch_kick_drift(m->xyz, m->vel, m->F, 3 * nat, hacc, 0.0, st));
        HIPCHK(c, launch_sqsum(m->vel, 3 * nat, m->dscal + 2, st));
        HIPCHK(c, hipMemcpyAsync(c->scal_host, m->dscal, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        m->step += 1;
        const double U = c->scal_host[0] - m->ts;   // free energy at kT > 0
        const double ke = 0.5 * m->p.mass * kKeEv * c->scal_host[2];
        m->U = U;
        if (log) {
            log[step].epot = U;
            log[step].ekin = ke;
            log[step].etot = U + ke;
            log[step].max_q_minus_n = c->scal_host[1];
            log[step].sp2_iterations = iters;
            log[step].fill_min = fill;
        }
        if (m->o.diverge_q > 0.0 && !(c->scal_host[1] <= m->o.diverge_q))
            return fail(c, SP2_EDIVERGE, "auxiliary charges diverged: max|q - n| = " +
                                             std::to_string(c->scal_host[1]) + " e after step " +
                                             std::to_string(m->step) +
                                             " (kappa outside the stability bound, or too long a time step)");
    }
    return SP2_OK;
}

extern "C" sp2_status xlbomd_counters(const xlbomd* m, long long* steps, long long* density_matrices) {
    if (!m) return SP2_EINVAL;
    if (steps) *steps = m->step;
    if (density_matrices) *density_matrices = m->dm_count;
    return SP2_OK;
}

extern "C" sp2_status xlbomd_info(const xlbomd* m, int* scf_iterations, double* scf_residual) {
    if (!m) return SP2_EINVAL;
    if (scf_iterations) *scf_iterations = m->scf_iterations;
    if (scf_residual) *scf_residual = m->scf_residual;
    return SP2_OK;
}

extern "C" sp2_status xlbomd_get(xlbomd* m, double* xyz_host, double* vel_host, double* q_host, double* n_host) {
    CTX_ENTER(m ? m->c : nullptr);
    if (!m) return SP2_EINVAL;
    sp2_ctx* c = m->c;
    HIPCHK(c, hipSetDevice(c->device));
    const size_t b = m->nat * sizeof(double);
    hipStream_t st = c->stream;
    if (xyz_host) HIPCHK(c, hipMemcpyAsync(xyz_host, m->xyz, 3 * b, hipMemcpyDeviceToHost, st));
    if (vel_host) HIPCHK(c, hipMemcpyAsync(vel_host, m->vel, 3 * b, hipMemcpyDeviceToHost, st));
    if (q_host) HIPCHK(c, hipMemcpyAsync(q_host, m->q, b, hipMemcpyDeviceToHost, st));
    if (n_host) HIPCHK(c, hipMemcpyAsync(n_host, m->hist + (size_t)m->head * m->nat, b, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    return SP2_OK;
}

namespace {
// Checkpoint layout: header, then xyz, vel, F (3 n_atoms each), q (n_atoms)
// and the K + 1 history slots of n (n_atoms each), all FP64.
struct XlCheckpoint {
    uint32_t magic;      // 'XLBS'
    uint32_t version;
    int32_t n_atoms;
    int32_t K;
    int64_t step;
    int32_t head;
    int32_t fermi_steps; // recursion steps of the Fermi operator (kT > 0)
    double U;
    double mu;           // chemical potential of the last Fermi operator (NaN at kT = 0)
    double ts;           // kT S of the last Fermi operator
    double kT;           // electronic temperature of the integrator
    double overlap_s0;   // > 0: non-orthogonal basis
};
static_assert(sizeof(XlCheckpoint) == 72, "checkpoint header layout");
constexpr uint32_t kXlMagic = 0x53424c58u;
constexpr uint32_t kXlVersion = 2;
size_t checkpoint_bytes(int nat, int K) {
    return sizeof(XlCheckpoint) + (size_t)(10 + K + 1) * nat * sizeof(double);
}
}  // namespace

extern "C" sp2_status xlbomd_get_state(const xlbomd* m, void* buf, size_t* bytes) {
    if (!m || !bytes) return SP2_EINVAL;
    sp2_ctx* c = m->c;
    const size_t need = checkpoint_bytes(m->nat, m->o.K);
    if (!buf) {
        *bytes = need;
        return SP2_OK;
    }
    if (*bytes < need) {
        *bytes = need;
        return fail(c, SP2_EINVAL, "checkpoint buffer too small");
    }
    HIPCHK(c, hipSetDevice(c->device));
    XlCheckpoint h{};
    h.magic = kXlMagic;
    h.version = kXlVersion;
    h.n_atoms = m->nat;
    h.K = m->o.K;
    h.step = m->step;
    h.head = m->head;
    h.fermi_steps = m->o.kT > 0.0 ? m->o.fermi_steps : 0;
    h.U = m->U;
    h.mu = m->mu;
    h.ts = m->ts;
    h.kT = m->o.kT;
    h.overlap_s0 = m->o.overlap_s0;
    char* out = static_cast<char*>(buf);
    std::memcpy(out, &h, sizeof(h));
    double* d = reinterpret_cast<double*>(out + sizeof(h));
    const size_t na = m->nat;
    hipStream_t st = c->stream;
    HIPCHK(c, hipMemcpyAsync(d, m->xyz, 3 * na * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipMemcpyAsync(d + 3 * na, m->vel, 3 * na * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipMemcpyAsync(d + 6 * na, m->F, 3 * na * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipMemcpyAsync(d + 9 * na, m->q, na * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipMemcpyAsync(d + 10 * na, m->hist, (size_t)(m->o.K + 1) * na * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    *bytes = need;
    return SP2_OK;
}

extern "C" sp2_status xlbomd_set_state(xlbomd* m, const void* buf, size_t bytes) {
    CTX_ENTER(m ? m->c : nullptr);
    if (!m || !buf) return SP2_EINVAL;
    sp2_ctx* c = m->c;
    XlCheckpoint h;
    if (bytes < sizeof(h)) return fail(c, SP2_EINVAL, "checkpoint too short");
    std::memcpy(&h, buf, sizeof(h));
    if (h.magic != kXlMagic || h.version != kXlVersion) return fail(c, SP2_EINVAL, "not an xlbomd checkpoint");
    if (h.n_atoms != m->nat || h.K != m->o.K)
        return fail(c, SP2_EINVAL, "checkpoint is for a different system size or history length");
    if (bytes != checkpoint_bytes(m->nat, m->o.K) || h.head < 0 || h.head > h.K || h.step < 0)
        return fail(c, SP2_EINVAL, "corrupt checkpoint");
    // the same electronic model: temperature, Fermi recursion and basis
    if (h.kT != m->o.kT || h.overlap_s0 != m->o.overlap_s0 ||
        (m->o.kT > 0.0 && (h.fermi_steps != m->o.fermi_steps || !std::isfinite(h.mu))))
        return fail(c, SP2_EINVAL, "checkpoint is for a different electronic temperature, Fermi recursion or basis");
    HIPCHK(c, hipSetDevice(c->device));
    const double* d = reinterpret_cast<const double*>(static_cast<const char*>(buf) + sizeof(h));
    const size_t na = m->nat;
    hipStream_t st = c->stream;
    HIPCHK(c, hipMemcpyAsync(m->xyz, d, 3 * na * 8, hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(m->vel, d + 3 * na, 3 * na * 8, hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(m->F, d + 6 * na, 3 * na * 8, hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(m->q, d + 9 * na, na * 8, hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(m->hist, d + 10 * na, (size_t)(h.K + 1) * na * 8, hipMemcpyHostToDevice, st));
    HIPCHK(c, hipStreamSynchronize(st));
    m->step = h.step;
    m->head = h.head;
    m->U = h.U;
    m->mu = h.mu;
    m->ts = h.ts;
    return SP2_OK;
}

extern "C" void xlbomd_destroy(xlbomd* m) {
    if (!m) return;
    (void)hipSetDevice(m->c->device);
    (void)hipStreamSynchronize(m->c->stream);
    double* bufs[] = {m->xyz, m->vel, m->F, m->q, m->dev, m->hist, m->H, m->D, m->dscal, m->S, m->Wen};
    for (double* b : bufs)
        if (b) (void)hipFree(b);
    delete m;
}

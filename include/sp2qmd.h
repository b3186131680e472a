/* sp2qmd — zero-temperature density matrices by SP2 purification on MI355X,
 * with the charge, energy, force and extended-Lagrangian (XL-BOMD) steps of
 * Niklasson & Cawkwell, "Fast method for quantum mechanical molecular
 * dynamics" (orthogonal self-consistent-charge tight binding, T_e = 0).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Matrices are dense, N x N, row-major, FP64, leading dimension N.
 * - Every array argument is a DEVICE pointer (hipMalloc'd or a torch CUDA
 *   tensor) on the context's device, unless the name ends in _host or the
 *   call takes an sp2_memkind that says where its matrices live.  The
 *   caller owns all arrays; the library never frees or retains them.  Inputs
 *   are only read; outputs are written only when SP2_OK is returned (stats
 *   structs are always filled).
 * - All work is enqueued on the context's stream.  Functions that return
 *   host values (stats, energies, *_host outputs) synchronise that stream
 *   before returning.
 * - Orbitals are atom-major: orbital index = 4 * atom + {s, px, py, pz}.
 * - No exception crosses this ABI.  On error a status < 0 is returned and a
 *   message is kept in the context (sp2_last_error).
 * - A context serves one call at a time: a call made from another host
 *   thread while one is in progress returns SP2_EBUSY and does nothing.
 */
#ifndef SP2QMD_H
#define SP2QMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SP2_OK = 0,
    SP2_EINVAL = -1,    /* bad argument (size, pointer, option)              */
    SP2_ENOMEM = -2,    /* device allocation failed                          */
    SP2_EDEVICE = -3,   /* HIP runtime error                                 */
    SP2_ENOCONV = -4,   /* SP2 reached max_iter without converging/stalling  */
    SP2_EGAP = -5,      /* no resolvable gap at the Fermi level: the set of
                           n_occ occupied states is not unique               */
    SP2_EBUDGET = -6,   /* serving: request larger than the memory budget    */
    SP2_EBUSY = -7,     /* the context is inside a call from another thread
                           (a context serves one call at a time; the error
                           string is left as it is)                          */
    SP2_ETIMEOUT = -8,  /* serving: wait timed out                           */
    SP2_EDIVERGE = -9   /* XL-BOMD: auxiliary charges ran away from q        */
} sp2_status;

/* Arithmetic of the SP2 products X_n^2 (the update, traces, branch and stop
 * decisions are FP64 in every mode). */
typedef enum {
    SP2_PREC_FP64 = 0,   /* FP64 MFMA products                                   */
    SP2_PREC_INT8X = 1,  /* FP64 master X split into `slices` int8 digit
                            planes, each row scaled so that its largest
                            element fills the top digit (8 bits per digit
                            while slices 2^14 N < 2^31, else 7); the digit
                            products of planes t, u with level t+u < levels
                            on int8 MFMA with exact int32 accumulation,
                            levels combined in FP64 (the Ozaki scheme)       */
    SP2_PREC_BF16X2 = 2, /* BF16 hi+lo split with FP32 MFMA accumulation, FP32
                            master, then `fp32_tail` FP32 products (as in
                            SP2_PREC_FP32) once the BF16 stage stalls            */
    SP2_PREC_FP32 = 3    /* FP32 operands (X_0 rounded to FP32) on FP32 MFMA with
                            FP32 accumulation, update in FP32; stops at the
                            FP32 rounding floor by the stall rule with r = 1/2.
                            No threshold (tau = 0)                           */
} sp2_precision;

typedef struct {
    int precision;       /* sp2_precision                                        */
    int max_iter;        /* products before SP2_ENOCONV (default 100)            */
    double idem_tol;     /* stop when ||X_n^2 - X_n||_F < idem_tol (1e-10)       */
    double stall_tol;    /* also stop when n >= 4, e_n >= r e_{n-2}, e_n <
                            stall_tol (idempotency error at its floor; 1e-2);
                            r = 1 for FP64 and BF16X2 products without a
                            threshold; r = 1/2 for INT8X and FP32 products
                            (their rounding floor) and whenever tau > 0, where the
                            bound is also max(stall_tol, 0.1) (the floor set
                            by the threshold keeps creeping down and grows
                            with N) */
    int fp64_head;       /* INT8X: first products done in FP64 (default 0)      */
    int slices;          /* INT8X: digit planes, 2..6 (default 5)                */
    int fp32_tail;       /* BF16X2: FP32 iterations after the BF16 stage stalls
                            (default 3)                                          */
    double tau;          /* threshold applied to X_0 and after every update
                            (Linear scaling section), 0 = dense; the rule is
                            set by `threshold`. Products skip the 32-column
                            blocks outside each panel's nonzero range         */
    int tile_group;      /* order of the 128x128 product tiles: G x G super-tiles
                            dealt to the XCDs (G > 0), 0 = plain row-major, -1
                            (default) = the value sp2_autotune chose (or a
                            loaded table holds) for this size and precision,
                            else 8; the tuned K-stage configuration, split
                            cap and FP64 output tile apply whatever
                            tile_group is (32 x 32 tiles have no order).  INT8X results
                            do not depend on these; FP64 products with a tail
                            split (see below) may differ in the last bits    */
    int tail_split;      /* N >= 4096: when the tiles of the last wave of
                            product workgroups would leave at least half of the
                            workgroup slots idle, split their K loops into
                            chunks run in parallel, then summed: INT8X up to 8
                            chunks, summed exactly (results do not depend on
                            it); FP64 up to 16 chunks, summed in chunk order
                            (results change at the rounding level).  FP64
                            products whose tiles fill at most half of the slots
                            (N <= 2816 on 256 CUs) split every tile into about
                            sqrt(1.4 K/16) chunks.  -1 (default): on; 0: never. */
    int threshold;       /* tau > 0: 0 (default) zero each 32x32 block whose
                            Frobenius norm is < tau; 1 zero each element with
                            |x| < tau (the paper's rule). Fill fractions count
                            the 32x32 blocks that still hold a nonzero       */
    int levels;          /* INT8X: digit-product levels kept, slices (the
                            triangle, slices (slices + 1) / 2 products) or
                            slices + 1 (slices - 1 more products: the
                            accuracy of operands rounded to 8 slices bits;
                            slices <= 5); 0 (default) = slices.  Four planes
                            with five levels (13 products) reach the 1e-6
                            Frobenius error per sqrt(N) of mixed precision at
                            13/15 of the five-plane cost                     */
    double dense_fill;   /* tau > 0, INT8X (fp64_head 0): while the kept
                            fraction of 32x32 blocks of X_n is at least
                            dense_fill, its product runs the dense kernel over
                            every upper tile (rows of X_n encoded whole)
                            instead of the work-list kernel over the kept
                            blocks; the same D either way (exact integer
                            sums of the same digits).  Default 0.95 (3-10 %
                            faster solves at N = 2048-8192 on 3-D lattices,
                            no change at N = 16384); > 1: always the
                            work-list kernel.  SP2_EINVAL below 0          */
} sp2_options;

typedef struct {
    int iterations;          /* products X_n^2 formed                            */
    int status;              /* 0 converged, 1 stalled, 2 max_iter, 3 gap,
                                4 invalid H                                      */
    int fp64_products;       /* of which in FP64                                 */
    int head_switch;         /* product index where the precision switched (-1)  */
    double eps_min, eps_max; /* Gershgorin bounds used for X_0                   */
    double idem_err;         /* ||X^2 - X||_F of the last product formed         */
    double trace;            /* Tr D                                             */
    uint64_t branch_bits[2]; /* bit n set: update n was X <- 2X - X^2            */
    double ms;               /* wall time of the solve on the stream (ms)        */
    double fill_min, fill_max; /* tau > 0: range of the fraction of 32x32 blocks
                                  holding a nonzero after each update (X_0 incl.) */
    float idem_hist[128];    /* ||X_n^2 - X_n||_F of product n                   */
    float fill_hist[128];    /* that fraction after update n (tau > 0)         */
    /* Filled only when profiling is on (sp2_ctx_set_profiling): summed HIP-event
     * durations of the product kernels that formed products, [0] FP64 product
     * kernel, [1] reduced-precision product kernel, and their launch counts;
     * encode_ms: operand encoding; post_ms: block-threshold passes. */
    double prod_ms[2];
    int prod_count[2];
    double encode_ms, post_ms;
} sp2_stats;

typedef struct sp2_ctx sp2_ctx;

/* Fill *opt with the defaults listed above (precision FP64). */
void sp2_options_default(sp2_options *opt);

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * enqueue on (NULL: the null stream).  Library scratch (padded X buffers,
 * partial sums, control state) is owned by the context and grows on demand. */
sp2_status sp2_ctx_create(sp2_ctx **out, int device, void *hip_stream);
/* Destroy a context; every xlbomd and sp2_server made on it must be
 * destroyed first. */
void sp2_ctx_destroy(sp2_ctx *ctx);
sp2_status sp2_ctx_set_stream(sp2_ctx *ctx, void *hip_stream);
/* on != 0: bracket every product kernel with HIP events on the context's
 * stream and report their durations in sp2_stats (small launch overhead). */
sp2_status sp2_ctx_set_profiling(sp2_ctx *ctx, int on);
const char *sp2_strerror(int status);
const char *sp2_last_error(const sp2_ctx *ctx);

/* Density matrix D = theta(mu0 I - H) with Tr D = n_occ by SP2 purification
 * (Linear scaling section; orthogonal T_e = 0 subsection: the step function
 * of the Hamiltonian).  H: N x N symmetric (device); D_out: N x N (device).
 * 0 < n_occ < N.  opt NULL = defaults.  stats may be NULL.
 * H must be finite and symmetric to within 1e-12 max|H_ij|, else SP2_EINVAL
 * (checked on the device before any product).
 * Returns SP2_ENOCONV if neither stop rule fired within max_iter products,
 * and SP2_EGAP when theta(mu0 I - H) is not defined at the available
 * resolution (the paper assumes a gap; reading for a degenerate level): the
 * iteration stopped at a projector whose trace is not n_occ, or at least
 * 100 products left eigenvalues of X_n far from 0 and 1
 * (||X_n^2 - X_n||_F >= 1/16), or H is a multiple of I.  On any error D_out
 * is not written. */
sp2_status sp2_density_matrix(sp2_ctx *ctx, int N, const double *H, int n_occ,
                              const sp2_options *opt, double *D_out,
                              sp2_stats *stats);

/* Where the matrices of sp2_density_matrix_mem and tb_hamiltonian_mem live. */
typedef enum {
    SP2_MEM_HOST = 0,    /* host memory (pageable or pinned)                     */
    SP2_MEM_DEVICE = 1   /* device memory of the context's device                */
} sp2_memkind;

/* sp2_density_matrix with H and D_out in memory of the given kind.  Host
 * arrays are copied through a device staging buffer owned by the context
 * (2 N^2 doubles, grown on demand): H in before the solve, D out after a
 * successful one; the call then synchronises the context's stream, so D_out
 * is ready when it returns.  Same errors as sp2_density_matrix (D_out is not
 * written on error); stats->ms times the solve without the copies.  Device
 * memory: exactly sp2_density_matrix. */
sp2_status sp2_density_matrix_mem(sp2_ctx *ctx, int N, const double *H, sp2_memkind kind, int n_occ,
                                  const sp2_options *opt, double *D_out, sp2_stats *stats);

/* Allocation-free variant of sp2_density_matrix, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, result and errors as
 * sp2_density_matrix, restricted to FP64 products (opt->precision 0) without
 * a threshold (opt->tau 0) and 1 <= N <= 1024; other options as there.  It
 * calls no hipMalloc/hipFree: its scratch (the two padded X buffers, partial
 * sums and the FP64 product's K-split accumulators) lives in one static
 * device array of 64 MiB that the library holds on every GPU it runs on until
 * the process ends; its device address is looked up by sp2_ctx_create.
 * N > 1024, another precision or tau != 0 give SP2_EINVAL.  Every call on a
 * GPU shares that GPU's array, which keeps the last call's contents (each
 * call writes all of it that it reads), so calls that overlap on one GPU
 * (several contexts or streams, or host threads) race and must be serialised
 * by the caller.  Results equal sp2_density_matrix's with the same options
 * (same kernels, same K split). */
sp2_status sp2_density_matrix_noalloc(sp2_ctx *ctx, int N, const double *H, int n_occ,
                                      const sp2_options *opt, double *D_out, sp2_stats *stats);

/* Autotuner of the SP2 product's launch configuration: times the product
 * kernel of the given precision (and slices and levels (0 = slices), for
 * INT8X) at size N on the
 * context's device for every candidate -- the tile order (G x G super-tiles,
 * G in {0 (row-major), 4, 8, 16, 32}) and, for INT8X, the K-stage
 * configuration of the LDS staging ring (stage_cfg 0: 64-byte K stages two
 * deep (32-byte three deep at six planes), 1: 32-byte stages three deep, 2:
 * 32-byte stages four deep, up to five planes), for FP64 the most chunks of a
 * tile split along K (8 or 16) and, up to a padded N of 2048, the output tile
 * shape (128 x 128 tiles of 4 waves, or 32 x 32 tiles whose 4 waves split K,
 * no tile order; without an entry pure FP64 solves take the 32 x 32 tile up
 * to a padded N of 1024) -- on a pseudo-random symmetric operand, and
 * keeps the fastest (from a padded N of 4096 on, among 128 x 128 candidates
 * within 0.3 % of the fastest, the one whose tile order re-reads the fewest
 * operand panels: G = 8, then 16, 4, 32, row-major) for later solves of the
 * same padded size and precision
 * that leave tile_group at -1 (and for sizes within a factor of 2 that have
 * no entry of their own).  out (may be NULL): the choice and the measured ms
 * per product of each candidate.  Uses the context's scratch; INT8X results
 * do not depend on the choice, FP64 results at the rounding level. */
typedef struct {
    int tile_group;          /* chosen super-tile size (0 = row-major)            */
    int stage_cfg;           /* INT8X: chosen K-stage configuration              */
    int split_cap;           /* FP64: chosen most chunks of a split tile          */
    int tile;                /* chosen output tile side: 128, or 32 (FP64 only)   */
    int n_candidates;
    int candidates[16][4];   /* (tile_group, stage_cfg, split_cap, tile) each     */
    float ms_per_product[16];
} sp2_tune_result;
sp2_status sp2_autotune(sp2_ctx *ctx, int N, int precision, int slices, int levels, sp2_tune_result *out);

/* Persisted autotuner table.  sp2_tune_save writes every configuration the
 * context holds (tuned or loaded) to the text file at path, one line per
 * (device architecture, compute units, padded N, precision, slices, levels);
 * sp2_tune_load adds a file's entries for this context's device type (other
 * architectures and out-of-range entries are skipped).  sp2_ctx_create loads
 * the table named by the environment variable SP2QMD_TUNE_TABLE when it is
 * set and readable.  SP2_EINVAL: NULL arguments, an unreadable or unwritable
 * file, a malformed line. */
sp2_status sp2_tune_save(const sp2_ctx *ctx, const char *path);
sp2_status sp2_tune_load(sp2_ctx *ctx, const char *path);

/* Measurement aid, not a step of the path: the rate of the int8 product
 * kernel's instruction (v_mfma_i32_32x32x32_i8; 2 ops per multiply-add) this
 * device sustains with no memory traffic, the measured denominator beside
 * the published peak in a roofline.  The rate depends on the data through the
 * power-limited clock (zero operands run far faster), so every SIMD runs four
 * accumulator chains on pseudo-random balanced 7-bit digits, the range of the
 * digit planes, that change every product.  About 20 ms of work per launch
 * on the context's stream; *ops_per_s gets the best of three launches after
 * one warm-up.  SP2_EINVAL for a NULL output. */
sp2_status sp2_int8_mfma_rate(sp2_ctx *ctx, double *ops_per_s);

/* Net Mulliken charges of an orthogonal basis (net-charge equation of the
 * SCC-TB subsection, S = I): q_i = 2 sum_{alpha in atom i} D_{i alpha,i alpha}
 * - z_val (electron excess).  D: (4 n_atoms)^2 device; q_out: n_atoms device. */
sp2_status sp2_mulliken(sp2_ctx *ctx, int n_atoms, const double *D, double z_val,
                        double *q_out);

/* Band energy 2 Tr[D H] (doubly occupied orbitals, Eq. DFT_POT) returned on
 * the host.  D, H: N x N device. */
sp2_status sp2_band_energy(sp2_ctx *ctx, int N, const double *D, const double *H,
                           double *e_host);

/* Density matrix in a non-orthogonal basis (Non-orthogonal formulation
 * subsection: H_perp = Z^T H Z with the congruence factor Z^T S Z = I of
 * Eq. Congr, the T_e = 0 density matrix of H_perp as in Eq. DM_perp, and the
 * de-orthogonalised rho = Z rho_perp Z^T).  Z is the Loewdin factor
 * S^(-1/2), built by a coupled Newton-Schulz iteration whose products
 * (polynomials in S) are formed as symmetric FP64 MFMA products of upper
 * tiles; each transform is one full product and one symmetric one
 * (W = H Z, H_perp = W^T Z), so H_perp and rho are exactly symmetric;
 * rho_perp is an SP2 solve with *opt (any
 * precision and threshold), whose statistics go to *stats.  rho satisfies
 * Tr[rho S] = n_occ and rho S rho = rho.
 * H, S: N x N row-major FP64 device arrays (S symmetric positive definite;
 * the caller keeps ownership); D_out: N x N device; factor_iterations (host,
 * may be NULL): Newton-Schulz steps taken.  Scratch: 4 N^2 doubles owned by
 * the context.  Errors: SP2_EINVAL (arguments, non-finite factor), SP2_ENOCONV
 * (the factor did not converge in 40 steps: S not positive definite or badly
 * conditioned), and those of sp2_density_matrix.  Blocks the host until D_out
 * is written. */
sp2_status sp2_density_matrix_nonorth(sp2_ctx *ctx, int N, const double *H, const double *S,
                                      int n_occ, const sp2_options *opt, double *D_out,
                                      sp2_stats *stats, int *factor_iterations);

/* Net Mulliken charges in a non-orthogonal basis: q_i = 2 sum_{alpha in i}
 * (D S)_{i alpha, i alpha} - z_val (the charges whose derivative the
 * non-orthogonal force equation uses).  D, S: (4 n_atoms)^2 device, S
 * symmetric; q_out: n_atoms device. */
sp2_status sp2_mulliken_overlap(sp2_ctx *ctx, int n_atoms, const double *D, const double *S,
                                double z_val, double *q_out);

/* Density matrix at finite electronic temperature (Eq. EL_4c with kT > 0):
 * D = (exp(beta (H - mu I)) + 1)^(-1), beta = 1/kT, by the recursive
 * Fermi-operator expansion: X_0 = I/2 - beta (H - mu I) / 2^(n_steps + 2),
 * then n_steps times X <- X^2 (X^2 + (I - X)^2)^(-1) (every product is of
 * polynomials in H, formed as a symmetric FP64 MFMA product of upper tiles,
 * so each X is exactly symmetric; the inverse by Newton-Schulz).  Its
 * exponent carries a relative error of about (beta |e - mu| / 2^n_steps)^2
 * / 12 per eigenvalue e; FP64 rounding sets a floor near 1e-11 for
 * n_steps >= 16.
 *
 * H: N x N device, row-major, finite and symmetric (EINVAL otherwise).  kT in
 * the units of H (> 0).  n_steps in [1, 60] with beta |e - mu| <=
 * 2^(n_steps + 1) over H's Gershgorin interval, and over the bracket below
 * when mu is solved for (EINVAL otherwise).
 *
 * max_newton == 0: *mu (in) is the fixed chemical potential and D_out = X_n
 * at it.  max_newton > 0: canonical mu with |Tr D - n_occ| < tol
 * (0 < n_occ < N, fractional allowed) by Newton steps with
 * dTr/dmu ~ beta Tr[D (I - D)], safeguarded by bisection of the bracket
 * [e_min - 40 kT, e_max + 40 kT] (Gershgorin bounds; a step leaving it
 * bisects it), from *mu if inside it, else from the middle of the Gershgorin
 * interval; *mu (out) is the result.  X_0 resolves mu to about
 * 2^(n_steps + 2) 2^-54 kT, so tol below dTr/dmu times that is not reached.
 * ENOCONV if max_newton passes end short of tol or mu stops changing (D_out,
 * *mu then hold the last pass).
 *
 * D_out: N x N device, may not alias H.  newton_iterations (may be NULL):
 * passes made.  products (may be NULL): N x N FP64 matrix products made over
 * all passes (2 per step plus 2 per Newton-Schulz update; the updates per
 * inverse follow from a bound on X's spectrum, fewer in the first steps,
 * where X is near I/2).  N <= 32768 (five N x N FP64 work matrices).  Blocks
 * the host until D_out is written. */
sp2_status sp2_fermi_density_matrix(sp2_ctx *ctx, int N, const double *H, double n_occ, double kT,
                                    int n_steps, int max_newton, double tol, double *mu,
                                    double *D_out, int *newton_iterations, long long *products);

/* Electronic entropy (Eq. Entropy) in units of k_B:
 * S = -2 sum_i [f_i ln f_i + (1 - f_i) ln(1 - f_i)], f_i = (exp((e_i - mu)
 * / kT) + 1)^(-1) over the eigenvalues e_i of H (the occupations of the
 * Fermi operator at mu; the factor 2 counts spin).  Computed without
 * eigenvalues as Tr s((H - mu I) / kT) by a Chebyshev expansion over H's
 * Gershgorin interval: coefficients on the host (8192 Chebyshev-Gauss nodes,
 * kept while above 1e-13), moments Tr T_k from about half as many N x N
 * symmetric FP64 MFMA products as coefficients.  H: N x N device, finite and
 * symmetric (EINVAL otherwise); mu finite; kT > 0 in the units of H; EINVAL
 * when more than about 4000 coefficients would be needed (the count grows as
 * the Gershgorin width over kT: about 1000 at kT = 0.5 and 2200 at 0.25 on
 * the sp lattices, whose interval is about 30 eV wide).  S_out: host.  moments (may be NULL): the
 * coefficients used.  N <= 32768.  Blocks the host until done. */
sp2_status sp2_fermi_entropy(sp2_ctx *ctx, int N, const double *H, double mu, double kT, double *S_out,
                             int *moments);

/* Finite electronic temperature in a non-orthogonal basis (Non-orthogonal
 * formulation subsection, with the Fermi function of Eq. EL_4c and the
 * entropy of Eq. Entropy): H_perp = Z^T H Z with the Loewdin factor Z =
 * S^(-1/2) (Eq. Congr), D_perp = the Fermi operator of H_perp by
 * sp2_fermi_density_matrix (n_steps, max_newton, tol and mu as there; the
 * canonical mu makes Tr[D S] = n_occ), D = Z D_perp Z^T (Eq. DM_perp).
 * W_out (may be NULL): the energy-weighted density matrix Z D_perp H_perp
 * Z^T, which takes the place of D H D in the forces of the free energy
 * (tb_forces_nonorth uses D H D, the form for an idempotent D).
 * entropy_out (may be NULL, host): S / k_B of the occupations
 * (sp2_fermi_entropy of H_perp at the final mu).  H, S, D_out, W_out: device,
 * N x N row-major, caller-owned; N <= 32768.  Errors as the calls it makes
 * (SP2_ENOCONV when the factor of S or mu does not converge).  Blocks the
 * host until done. */
sp2_status sp2_fermi_density_matrix_nonorth(sp2_ctx *ctx, int N, const double *H, const double *S, double n_occ,
                                            double kT, int n_steps, int max_newton, double tol, double *mu,
                                            double *D_out, double *W_out, double *entropy_out,
                                            int *newton_iterations);

/* ---------------------------------------------------------------------
 * Tight-binding model, forces and XL-BOMD
 * ------------------------------------------------------------------- */

/* Parameters of the orthogonal sp tight-binding model (SCC-TB subsection):
 * hopping |t(r)| = t0 exp(-(r - r0)/lam) for r < r_tail, a quintic tail on
 * [r_tail, r_cut) matching value, slope and curvature at r_tail and vanishing
 * with them at r_cut (r_tail == r_cut: hard cut); bond-integral signs
 * ss-sigma < 0, sp-sigma > 0, pp-sigma > 0, pp-pi < 0; gamma_ii = hubbard_u,
 * gamma_ij = coulomb_k / r_ij; pair repulsion pair_a exp(-(r - pair_r0) /
 * pair_rho) with the same tail (pair_a = 0: none). */
typedef struct {
    double eps_s, eps_p;
    double t0, r0, lam;
    double r_cut, r_tail;
    double hubbard_u, coulomb_k;
    double pair_a, pair_r0, pair_rho;
    double mass;      /* amu, all atoms */
    double z_val;     /* valence electrons per neutral atom */
} tb_params;

/* H[n] = h(R) + diag over the four orbitals of atom i of V_i, V = gamma n
 * (Eq. DFTB_2 with S = I).  xyz: 3 n_atoms device (A); n_aux: n_atoms device
 * or NULL (then H = h); H_out: (4 n_atoms)^2 device. */
sp2_status tb_hamiltonian(sp2_ctx *ctx, const tb_params *p, int n_atoms,
                          const double *xyz, const double *n_aux, double *H_out);
/* tb_hamiltonian with xyz, n_aux (may be NULL) and H_out in memory of the
 * given kind; host arrays are staged through the context's device buffer and
 * the call synchronises the context's stream before returning. */
sp2_status tb_hamiltonian_mem(sp2_ctx *ctx, const tb_params *p, int n_atoms, const double *xyz,
                              const double *n_aux, double *H_out, sp2_memkind kind);

/* Overlap matrix of the non-orthogonal variant of the model (the paper's S of
 * the Non-orthogonal formulation subsection; its parameters are not given, so
 * the synthetic form is: identity blocks on the diagonal, and per pair within
 * r_cut the Slater-Koster block of overlap integrals of magnitude
 * s(r) = s0 exp(-(r - r0)/lam_s) with the hopping's tail from r_tail, with
 * the sign pattern opposite to the hopping's).  p supplies r0, r_tail, r_cut;
 * xyz: 3 n_atoms device (A); S_out: (4 n_atoms)^2 row-major device. */
sp2_status tb_overlap(sp2_ctx *ctx, const tb_params *p, double s0, double lam_s, int n_atoms,
                      const double *xyz, double *S_out);

/* Non-orthogonal H[n] = h + (S L + L S)/2, L the diagonal holding
 * V_i = sum_j gamma_ij n_j on the orbitals of atom i (the charge shift of the
 * non-orthogonal SCC-TB Hamiltonian, Eq. DFTB_2 with S != I); h alone when
 * n_aux is NULL.  S: (4 n_atoms)^2 device (from tb_overlap); n_aux: n_atoms
 * device or NULL; H_out: (4 n_atoms)^2 device. */
sp2_status tb_hamiltonian_nonorth(sp2_ctx *ctx, const tb_params *p, int n_atoms, const double *xyz,
                                  const double *n_aux, const double *S, double *H_out);

/* Non-orthogonal forces at constant auxiliary charges n (the role of the
 * non-orthogonal force equation, EL_Nonorth_a, at T_e = 0): with
 * U(R; n) = 2 Tr[D h] + sum_i q_i V_i - 1/2 n^T gamma n + E_pair and the
 * overlap charges q (sp2_mulliken_overlap), F_k = -dU/dR_k is the orthogonal
 * force of tb_forces with these q plus sum_ab M_ab dS_ab/dR_k, where
 * M = 2 D H D - (V_a + V_b) D_ab (the energy-weighted density matrix of the
 * generalized eigenproblem and the overlap inside H[n] and q; dS/dR_k is
 * evaluated from the positions).  D: the density matrix of H = H[n]
 * (sp2_density_matrix_nonorth); H, D: (4 n_atoms)^2 device; q, n_aux:
 * n_atoms device; s0, lam_s: the overlap parameters of tb_overlap; F_out:
 * 3 n_atoms device; U_host: host or NULL.  Uses two N^2 scratch buffers of
 * the context (two FP64 MFMA products form D H D = (H D)^T D). */
sp2_status tb_forces_nonorth(sp2_ctx *ctx, const tb_params *p, double s0, double lam_s, int n_atoms,
                             const double *xyz, const double *D, const double *H, const double *q,
                             const double *n_aux, double *F_out, double *U_host);

/* Forces at constant auxiliary charges n (Eq. EL_Orth_a with Eq. EL_Orth_c,
 * on-site term read with rho - rho0):
 *   F_k = -2 Tr[D dh/dR_k] - sum_ij (q_i n_j - n_i n_j / 2) dgamma_ij/dR_k
 *         - dE_pair/dR_k,
 * and the potential energy U = 2 Tr[D h] + q.V - n.V/2 + E_pair, V = gamma n
 * (Eq. HF_POT_2 in charge form).  D: (4 n_atoms)^2 device; q, n: n_atoms
 * device; F_out: 3 n_atoms device (may be NULL); U_host may be NULL. */
sp2_status tb_forces(sp2_ctx *ctx, const tb_params *p, int n_atoms,
                     const double *xyz, const double *D, const double *q,
                     const double *n_aux, double *F_out, double *U_host);

/* One Born-Oppenheimer evaluation at auxiliary charges n (n = q at
 * self-consistency): H[n] (Eq. DFTB_2, S = I), D = theta(mu0 I - H[n]) by
 * SP2, net Mulliken charges q[D] (SCC-TB subsection), band energy
 * 2 Tr[D H[n]] (Eq. DFT_POT), the potential energy U and the forces at
 * constant n as in tb_forces.  xyz: 3 n_atoms device; n_aux: n_atoms device
 * or NULL (n = 0); q_out: n_atoms device; F_out: 3 n_atoms device or NULL;
 * e_band_host, e_pot_host: host scalars or NULL; stats may be NULL.  The
 * H and D scratch is owned by the context.  Errors as sp2_density_matrix. */
sp2_status qmd_evaluate(sp2_ctx *ctx, const tb_params *p, int n_atoms, const double *xyz,
                        const double *n_aux, int n_occ, const sp2_options *opt, double *q_out,
                        double *e_band_host, double *e_pot_host, double *F_out,
                        sp2_stats *stats);

typedef struct {
    double dt_fs;     /* time step (fs)                                        */
    double kappa;     /* delta t^2 omega^2 of Eq. Verl_n                        */
    double alpha;     /* dissipation strength                                  */
    int K;            /* dissipation order, history length K + 1 (<= 8)        */
    double c[9];      /* c_0 .. c_K                                            */
    sp2_options sp2;  /* density-matrix options for the one solve per step     */
    double scf_beta;  /* SCF start: linear mixing n += beta (q - n) ...         */
    double scf_tol;   /* ... until max_i |q_i - n_i| < scf_tol ...              */
    int scf_max_iter; /* ... or SP2_ENOCONV after this many density matrices;
                         0: no SCF, n0 is used as given                        */
    double diverge_q; /* stop with SP2_EDIVERGE after a step whose
                         max_i |q_i - n_i| exceeds this (e), the sign of kappa
                         outside the stability bound of Eq. Verl_n or of a too
                         long time step; 0: no check                           */
    double overlap_s0;  /* > 0: non-orthogonal basis with the overlap of
                           tb_overlap(s0, overlap_lam): H[n], the density
                           matrix, charges and forces of the non-orthogonal
                           entry points each step; 0 (zero-initialised
                           options): orthogonal                              */
    double overlap_lam;
    double kT;          /* > 0: finite electronic temperature (units of H):
                           the density matrix is the Fermi operator of
                           sp2_fermi_density_matrix (canonical mu, Newton from
                           the previous step's mu, |Tr D - n_occ| < fermi_tol),
                           and the record's epot is the free energy
                           U - kT S with S of sp2_fermi_entropy; 0: SP2.
                           With overlap_s0 > 0: the density matrix, W and
                           entropy of sp2_fermi_density_matrix_nonorth, the
                           forces of the free energy with that W           */
    int fermi_steps;    /* recursion steps of the Fermi operator (1..60)      */
    double fermi_tol;   /* kT > 0: |Tr D - n_occ| bound of the mu solve per
                           step; 0: 1e-9 max(1, N / 512) (X_0 quantises the
                           trace at about 1e-10 per 512 orbitals)            */
    int fermi_max_newton; /* kT > 0: mu passes per step before SP2_ENOCONV;
                           0: 100                                            */
} xlbomd_options;

typedef struct {
    double etot, epot, ekin;   /* eV                                           */
    double max_q_minus_n;      /* max_i |q_i - n_i| at the step                 */
    int sp2_iterations;
    float fill_min;            /* smallest kept-block fraction over the step's
                                  SP2 updates (1 if tau == 0)                  */
} xlbomd_record;

typedef struct xlbomd xlbomd;

/* Create an XL-BOMD integrator (General remarks subsection: velocity Verlet
 * for the nuclei, Eq. Verl_n for the auxiliary charges, one density matrix
 * per step, no SCF during the run).  xyz, vel (A, A/fs) and n0 are HOST
 * arrays copied in.  Start (General remarks): with scf_max_iter > 0 the
 * charges are first converged self-consistently on the GPU from the guess n0
 * (zeros when n0_host is NULL) and n = q is set for the whole history; with
 * scf_max_iter == 0, n0_host (required) is the history as given.  Atoms are
 * neutral with p->z_val valence electrons in doubly occupied states: n_occ =
 * z_val n_atoms / 2 (SP2_EINVAL unless that is a whole number in (0, 4 n_atoms)). */
sp2_status xlbomd_create(sp2_ctx *ctx, const tb_params *p, const xlbomd_options *o,
                         int n_atoms, const double *xyz_host, const double *vel_host,
                         const double *n0_host, xlbomd **out);
/* SCF iterations and final residual max|q - n| of the start (0 if n0 given). */
sp2_status xlbomd_info(const xlbomd *md, int *scf_iterations, double *scf_residual);
/* Steps taken and density matrices constructed since creation (the start
 * builds one per SCF iteration plus one; each step builds exactly one). */
sp2_status xlbomd_counters(const xlbomd *md, long long *steps, long long *density_matrices);
/* Advance n_steps; log (host, n_steps entries) may be NULL. */
sp2_status xlbomd_run(xlbomd *md, int n_steps, xlbomd_record *log);
/* Copy current positions, velocities, charges q and n_t to host arrays (any may be NULL). */
sp2_status xlbomd_get(xlbomd *md, double *xyz_host, double *vel_host,
                      double *q_host, double *n_host);
/* Checkpoint: the complete integrator state (positions, velocities, forces,
 * charges q, the K + 1 auxiliary-charge history of Eq. Verl_n, step count
 * and, at kT > 0, the chemical potential that starts the next step's mu
 * solve and the last kT S) as a versioned byte image in caller memory.  With
 * buf NULL, *bytes is set to the size needed; a smaller *bytes gives
 * SP2_EINVAL (and the size).
 * Layout (version 2, native byte order): a 72-byte header {uint32 magic
 * 'XLBS', uint32 version, int32 n_atoms, int32 K, int64 step, int32 head,
 * int32 fermi_steps (0 at kT = 0), double U, double mu (NaN at kT = 0),
 * double kT S, double kT, double overlap_s0}, then FP64 arrays
 * xyz[3 n_atoms], vel[3 n_atoms], F[3 n_atoms], q[n_atoms], n history
 * [(K + 1) n_atoms] (slot `head` is n_t). */
sp2_status xlbomd_get_state(const xlbomd *md, void *buf, size_t *bytes);
/* Resume from a checkpoint of an integrator with the same n_atoms, K, kT,
 * fermi_steps and basis (overlap_s0), SP2_EINVAL otherwise; continuing is
 * then bit-identical to continuing the original. */
sp2_status xlbomd_set_state(xlbomd *md, const void *buf, size_t bytes);
void xlbomd_destroy(xlbomd *md);

/* ---------------------------------------------------------------------
 * Serving: continuous batching of SP2 solves (int8 digit-plane products)
 * ------------------------------------------------------------------- */

typedef struct {
    uint64_t hbm_budget_bytes; /* device arena for admitted requests (default 8 GiB) */
    int max_slots;             /* systems in flight at once, 1..64 (default 32)      */
    int slices;                /* int8 digit planes, 2..6 (default 5)                */
    int max_iter;              /* products per solve (default 100)                   */
    double idem_tol;           /* converged when ||X^2 - X||_F < idem_tol (1e-10)    */
    int iters_per_tick;        /* products per scheduler tick, 1..16 (default 8):
                                  more amortize the host round trip of a tick,
                                  a finished system waits out the rest of its
                                  tick (its launches return at once)            */
    int levels;                /* digit-product levels, as sp2_options.levels: 0
                                  (default) = slices, or slices + 1 (slices <= 5) */
} sp2_server_options;

typedef struct sp2_server sp2_server;

void sp2_server_options_default(sp2_server_options *opt);

/* Start a server on the context's device with its own stream and scheduler
 * thread.  Requests are admitted in arrival order whenever a slot is free and
 * their device footprint (about 37 N^2 bytes for 5 planes) fits in the arena;
 * every tick advances all admitted systems by one product in grouped,
 * graph-replayed launches, and finished systems are retired and replaced
 * between ticks.  Each result is independent of the other requests in flight. */
sp2_status sp2_server_create(sp2_ctx *ctx, const sp2_server_options *opt, sp2_server **out);

/* Queue one solve of the symmetric N x N host matrix H_host (copied before
 * returning) with trace n_occ.  SP2_EBUDGET if it can never fit the arena.
 * Thread-safe. */
sp2_status sp2_server_submit(sp2_server *srv, int N, const double *H_host, int n_occ,
                             uint64_t *ticket);

/* Wait for a ticket (timeout_s < 0: forever) and copy D (N x N) and, when N is
 * a multiple of 4, the Mulliken charges (N / 4) to host arrays (either may be
 * NULL).  Returns the solve's status; SP2_ETIMEOUT leaves the ticket valid.
 * stats->ms is the latency from submit to result in host memory.  Thread-safe. */
sp2_status sp2_server_wait(sp2_server *srv, uint64_t ticket, double timeout_s,
                           double *D_out_host, double *q_out_host, sp2_stats *stats);

/* Latency percentiles (submit to result in host memory) over all completed
 * requests, and completed requests per second since the first submit. */
sp2_status sp2_server_report(sp2_server *srv, double *p50_ms, double *p99_ms,
                             double *solves_per_s);

/* Stop the scheduler (after the systems in flight finish) and free everything;
 * queued requests that were not admitted are dropped. */
void sp2_server_destroy(sp2_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* SP2QMD_H */

"""Python binding of libsp2qmd (argument marshalling only).

Every computation runs in the HIP library; this module converts torch CUDA
tensors to device pointers, fills the C structs of ``include/sp2qmd.h`` and
raises on error statuses.  If the library is not built, importing the module
still works but every call raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsp2qmd.so")

SP2_OK, SP2_EINVAL, SP2_ENOMEM, SP2_EDEVICE, SP2_ENOCONV, SP2_EGAP = 0, -1, -2, -3, -4, -5
# kappa of the K = 5 dissipative auxiliary-charge step (Eq. Verl_n) before its
# rescaling: the paper's runs use half of it at zero electronic temperature and
# three quarters at finite temperature, which damps the free energy's random walk.
KAPPA_K5 = 1.82
KAPPA_ZERO_T = 0.5 * KAPPA_K5
KAPPA_FINITE_T = 0.75 * KAPPA_K5
SP2_EBUDGET, SP2_EBUSY, SP2_ETIMEOUT, SP2_EDIVERGE = -6, -7, -8, -9
SP2_MEM_HOST, SP2_MEM_DEVICE = 0, 1
# bytes before the FP64 arrays (xyz, vel, F, q, n history) of an xlbomd checkpoint
XL_CHECKPOINT_HEADER = 72
PREC_FP64, PREC_INT8X, PREC_BF16X2, PREC_FP32 = 0, 1, 2, 3
PRECISIONS = {"fp64": PREC_FP64, "int8x": PREC_INT8X, "bf16x2": PREC_BF16X2, "fp32": PREC_FP32}


class Sp2Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("idem_tol", ctypes.c_double), ("stall_tol", ctypes.c_double),
                ("fp64_head", ctypes.c_int), ("slices", ctypes.c_int),
                ("fp32_tail", ctypes.c_int), ("tau", ctypes.c_double),
                ("tile_group", ctypes.c_int), ("tail_split", ctypes.c_int),
                ("threshold", ctypes.c_int), ("levels", ctypes.c_int), ("dense_fill", ctypes.c_double)]


class TuneResult(ctypes.Structure):
    _fields_ = [("tile_group", ctypes.c_int), ("stage_cfg", ctypes.c_int), ("split_cap", ctypes.c_int),
                ("tile", ctypes.c_int), ("n_candidates", ctypes.c_int), ("candidates", (ctypes.c_int * 4) * 16),
                ("ms_per_product", ctypes.c_float * 16)]


class Sp2Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("status", ctypes.c_int),
                ("fp64_products", ctypes.c_int), ("head_switch", ctypes.c_int),
                ("eps_min", ctypes.c_double), ("eps_max", ctypes.c_double),
                ("idem_err", ctypes.c_double), ("trace", ctypes.c_double),
                ("branch_bits", ctypes.c_uint64 * 2), ("ms", ctypes.c_double),
                ("fill_min", ctypes.c_double), ("fill_max", ctypes.c_double),
                ("idem_hist", ctypes.c_float * 128), ("fill_hist", ctypes.c_float * 128),
                ("prod_ms", ctypes.c_double * 2), ("prod_count", ctypes.c_int * 2),
                ("encode_ms", ctypes.c_double), ("post_ms", ctypes.c_double)]

    def to_dict(self):
        n = self.iterations
        bits = [(self.branch_bits[k >> 6] >> (k & 63)) & 1 for k in range(max(n - 1, 0))]
        return {"iterations": n, "status": ["converged", "stalled", "max_iter", "gap", "invalid"][self.status],
                "fp64_products": self.fp64_products, "head_switch": self.head_switch,
                "eps_min": self.eps_min, "eps_max": self.eps_max, "idem_err": self.idem_err,
                "trace": self.trace, "branches": bits, "ms": self.ms,
                "fill_min": self.fill_min, "fill_max": self.fill_max,
                "idem_hist": [float(self.idem_hist[k]) for k in range(n)],
                "fill_hist": [float(self.fill_hist[k]) for k in range(n)],
                "prod_ms": [self.prod_ms[0], self.prod_ms[1]],
                "prod_count": [self.prod_count[0], self.prod_count[1]],
                "encode_ms": self.encode_ms, "post_ms": self.post_ms}


class TBParams(ctypes.Structure):
    _fields_ = [(f, ctypes.c_double) for f in
                ("eps_s", "eps_p", "t0", "r0", "lam", "r_cut", "r_tail", "hubbard_u",
                 "coulomb_k", "pair_a", "pair_r0", "pair_rho", "mass", "z_val")]


class XLOptions(ctypes.Structure):
    _fields_ = [("dt_fs", ctypes.c_double), ("kappa", ctypes.c_double),
                ("alpha", ctypes.c_double), ("K", ctypes.c_int),
                ("c", ctypes.c_double * 9), ("sp2", Sp2Options),
                ("scf_beta", ctypes.c_double), ("scf_tol", ctypes.c_double), ("scf_max_iter", ctypes.c_int),
                ("diverge_q", ctypes.c_double), ("overlap_s0", ctypes.c_double), ("overlap_lam", ctypes.c_double),
                ("kT", ctypes.c_double), ("fermi_steps", ctypes.c_int),
                ("fermi_tol", ctypes.c_double), ("fermi_max_newton", ctypes.c_int)]


class XLRecord(ctypes.Structure):
    _fields_ = [("etot", ctypes.c_double), ("epot", ctypes.c_double),
                ("ekin", ctypes.c_double), ("max_q_minus_n", ctypes.c_double),
                ("sp2_iterations", ctypes.c_int), ("fill_min", ctypes.c_float)]


class ServerOptions(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_slots", ctypes.c_int),
                ("slices", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("idem_tol", ctypes.c_double), ("iters_per_tick", ctypes.c_int), ("levels", ctypes.c_int)]


_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int
_SIGS = {
    "sp2_options_default": (None, [ctypes.POINTER(Sp2Options)]),
    "sp2_ctx_create": (_I, [ctypes.POINTER(_P), _I, _P]),
    "sp2_ctx_destroy": (None, [_P]),
    "sp2_ctx_set_stream": (_I, [_P, _P]),
    "sp2_ctx_set_profiling": (_I, [_P, _I]),
    "sp2_strerror": (ctypes.c_char_p, [_I]),
    "sp2_last_error": (ctypes.c_char_p, [_P]),
    "sp2_density_matrix": (_I, [_P, _I, _P, _I, ctypes.POINTER(Sp2Options), _P,
                                ctypes.POINTER(Sp2Stats)]),
    "sp2_density_matrix_noalloc": (_I, [_P, _I, _P, _I, ctypes.POINTER(Sp2Options), _P,
                                        ctypes.POINTER(Sp2Stats)]),
    "sp2_density_matrix_mem": (_I, [_P, _I, _P, _I, _I, ctypes.POINTER(Sp2Options), _P,
                                    ctypes.POINTER(Sp2Stats)]),
    "tb_hamiltonian_mem": (_I, [_P, ctypes.POINTER(TBParams), _I, _P, _P, _P, _I]),
    "sp2_mulliken": (_I, [_P, _I, _P, _D, _P]),
    "sp2_autotune": (_I, [_P, _I, _I, _I, _I, ctypes.POINTER(TuneResult)]),
    "sp2_tune_save": (_I, [_P, ctypes.c_char_p]),
    "sp2_tune_load": (_I, [_P, ctypes.c_char_p]),
    "sp2_int8_mfma_rate": (_I, [_P, ctypes.POINTER(_D)]),
    "sp2_band_energy": (_I, [_P, _I, _P, _P, ctypes.POINTER(_D)]),
    "sp2_density_matrix_nonorth": (_I, [_P, _I, _P, _P, _I, ctypes.POINTER(Sp2Options), _P,
                                        ctypes.POINTER(Sp2Stats), ctypes.POINTER(_I)]),
    "sp2_mulliken_overlap": (_I, [_P, _I, _P, _P, ctypes.c_double, _P]),
    "sp2_fermi_entropy": (_I, [_P, _I, _P, _D, _D, ctypes.POINTER(_D), ctypes.POINTER(_I)]),
    "sp2_fermi_density_matrix": (_I, [_P, _I, _P, _D, _D, _I, _I, _D, ctypes.POINTER(_D), _P,
                                      ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_longlong)]),
    "sp2_fermi_density_matrix_nonorth": (_I, [_P, _I, _P, _P, _D, _D, _I, _I, _D, ctypes.POINTER(_D), _P, _P,
                                              ctypes.POINTER(_D), ctypes.POINTER(_I)]),
    "tb_overlap": (_I, [_P, ctypes.POINTER(TBParams), ctypes.c_double, ctypes.c_double, _I, _P, _P]),
    "tb_hamiltonian_nonorth": (_I, [_P, ctypes.POINTER(TBParams), _I, _P, _P, _P, _P]),
    "tb_forces_nonorth": (_I, [_P, ctypes.POINTER(TBParams), ctypes.c_double, ctypes.c_double, _I, _P, _P, _P,
                               _P, _P, _P, ctypes.POINTER(ctypes.c_double)]),
    "tb_hamiltonian": (_I, [_P, ctypes.POINTER(TBParams), _I, _P, _P, _P]),
    "tb_forces": (_I, [_P, ctypes.POINTER(TBParams), _I, _P, _P, _P, _P, _P,
                       ctypes.POINTER(_D)]),
    "qmd_evaluate": (_I, [_P, ctypes.POINTER(TBParams), _I, _P, _P, _I, ctypes.POINTER(Sp2Options), _P,
                          ctypes.POINTER(_D), ctypes.POINTER(_D), _P, ctypes.POINTER(Sp2Stats)]),
    "xlbomd_create": (_I, [_P, ctypes.POINTER(TBParams), ctypes.POINTER(XLOptions), _I,
                           _P, _P, _P, ctypes.POINTER(_P)]),
    "xlbomd_run": (_I, [_P, _I, ctypes.POINTER(XLRecord)]),
    "xlbomd_get": (_I, [_P, _P, _P, _P, _P]),
    "xlbomd_info": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_D)]),
    "xlbomd_counters": (_I, [_P, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong)]),
    "xlbomd_get_state": (_I, [_P, _P, ctypes.POINTER(ctypes.c_size_t)]),
    "xlbomd_set_state": (_I, [_P, _P, ctypes.c_size_t]),
    "xlbomd_destroy": (None, [_P]),
    "sp2_server_options_default": (None, [ctypes.POINTER(ServerOptions)]),
    "sp2_server_create": (_I, [_P, ctypes.POINTER(ServerOptions), ctypes.POINTER(_P)]),
    "sp2_server_submit": (_I, [_P, _I, _P, _I, ctypes.POINTER(ctypes.c_uint64)]),
    "sp2_server_wait": (_I, [_P, ctypes.c_uint64, _D, _P, _P, ctypes.POINTER(Sp2Stats)]),
    "sp2_server_report": (_I, [_P, ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "sp2_server_destroy": (None, [_P]),
}

_lib = None


def lib():
    """Load libsp2qmd.so; raises if it is not built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run python -m paper_1203_6836_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class Sp2Error(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def _host_ptr(a):
    """Pointer to a C-contiguous float64 numpy array (host memory)."""
    if a is None:
        return None
    import numpy as np
    if not isinstance(a, np.ndarray) or a.dtype != np.float64 or not a.flags["C_CONTIGUOUS"]:
        raise TypeError("expected a C-contiguous float64 numpy array")
    return ctypes.c_void_p(a.ctypes.data)


def _ptr(t):
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 tensor")
    return ctypes.c_void_p(t.data_ptr())


def options(precision="fp64", **kw) -> Sp2Options:
    o = Sp2Options()
    lib().sp2_options_default(ctypes.byref(o))
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def tb_params(model) -> TBParams:
    """TBParams from any object with the synth.TBModel fields."""
    p = TBParams()
    for f, _ in TBParams._fields_:
        setattr(p, f, float(getattr(model, f)))
    return p


class Context:
    """A library context bound to a device and a stream (torch's current by default)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self._h = ctypes.c_void_p()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
        st = lib().sp2_ctx_create(ctypes.byref(self._h), int(device), ctypes.c_void_p(handle))
        if st != SP2_OK:
            raise Sp2Error(st, "sp2_ctx_create: " + lib().sp2_strerror(st).decode())
        self.device = device
        # servers and integrators hold the context: they are closed before it
        import weakref
        self._children = weakref.WeakSet()

    def _check(self, st, what):
        if st != SP2_OK:
            raise Sp2Error(st, f"{what}: {lib().sp2_last_error(self._h).decode()}")

    def close(self):
        if self._h:
            for child in list(getattr(self, "_children", ())):
                child.close()
            lib().sp2_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- entry points (same names as the C-ABI) ----
    def sp2_ctx_set_profiling(self, on: bool):
        self._check(lib().sp2_ctx_set_profiling(self._h, 1 if on else 0), "sp2_ctx_set_profiling")

    def sp2_density_matrix(self, H, n_occ: int, opts: Sp2Options | None = None, D_out=None):
        import torch
        N = H.shape[0]
        if H.shape != (N, N):
            raise ValueError("H must be square")
        if D_out is None:
            D_out = torch.empty_like(H)
        stats = Sp2Stats()
        st = lib().sp2_density_matrix(self._h, N, _ptr(H), int(n_occ),
                                      ctypes.byref(opts) if opts is not None else None,
                                      _ptr(D_out), ctypes.byref(stats))
        self._check(st, "sp2_density_matrix")
        return D_out, stats.to_dict()

    def sp2_density_matrix_noalloc(self, H, n_occ: int, opts: Sp2Options | None = None, D_out=None):
        """As sp2_density_matrix, with the library's static device scratch (FP64, tau 0, N <= 1024)."""
        import torch
        N = H.shape[0]
        if H.shape != (N, N):
            raise ValueError("H must be square")
        if D_out is None:
            D_out = torch.empty_like(H)
        stats = Sp2Stats()
        st = lib().sp2_density_matrix_noalloc(self._h, N, _ptr(H), int(n_occ),
                                              ctypes.byref(opts) if opts is not None else None,
                                              _ptr(D_out), ctypes.byref(stats))
        self._check(st, "sp2_density_matrix_noalloc")
        return D_out, stats.to_dict()

    def sp2_density_matrix_mem(self, H, n_occ: int, opts: Sp2Options | None = None, D_out=None):
        """H and D in host memory (numpy float64 arrays: SP2_MEM_HOST) or on
        the device (CUDA tensors: SP2_MEM_DEVICE)."""
        import numpy as np
        N = H.shape[0]
        if tuple(H.shape) != (N, N):
            raise ValueError("H must be square")
        host = isinstance(H, np.ndarray)
        if D_out is None:
            D_out = np.empty_like(H) if host else H.new_empty(H.shape)
        conv = _host_ptr if host else _ptr
        stats = Sp2Stats()
        st = lib().sp2_density_matrix_mem(self._h, N, conv(H), SP2_MEM_HOST if host else SP2_MEM_DEVICE,
                                          int(n_occ), ctypes.byref(opts) if opts is not None else None,
                                          conv(D_out), ctypes.byref(stats))
        self._check(st, "sp2_density_matrix_mem")
        return D_out, stats.to_dict()

    def sp2_density_matrix_status(self, H, n_occ: int, opts: Sp2Options | None = None):
        """Raw status + stats (for error-path tests)."""
        import torch
        D = torch.empty_like(H)
        stats = Sp2Stats()
        st = lib().sp2_density_matrix(self._h, H.shape[0], _ptr(H), int(n_occ),
                                      ctypes.byref(opts) if opts is not None else None,
                                      _ptr(D), ctypes.byref(stats))
        return st, stats.to_dict()

    def sp2_density_matrix_nonorth(self, H, S, n_occ: int, opts: Sp2Options | None = None, D_out=None):
        """rho = Z theta(mu0 I - Z^T H Z) Z^T with Z^T S Z = I; returns (rho, stats, factor steps)."""
        import torch
        N = H.shape[0]
        if H.shape != (N, N) or S.shape != (N, N):
            raise ValueError("H and S must be N x N")
        if D_out is None:
            D_out = torch.empty_like(H)
        stats = Sp2Stats()
        its = _I(0)
        st = lib().sp2_density_matrix_nonorth(self._h, N, _ptr(H), _ptr(S), int(n_occ),
                                              ctypes.byref(opts) if opts is not None else None,
                                              _ptr(D_out), ctypes.byref(stats), ctypes.byref(its))
        self._check(st, "sp2_density_matrix_nonorth")
        return D_out, stats.to_dict(), its.value

    def sp2_fermi_density_matrix(self, H, n_occ: float, kT: float, n_steps: int, mu=None,
                                 max_newton: int = 50, tol: float = 1e-10, D_out=None):
        """(D, mu, passes): the Fermi operator at temperature kT by the recursive expansion.

        max_newton == 0 keeps mu fixed (it must be given); otherwise mu is the
        canonical chemical potential, Newton from mu (None: the middle of the
        Gershgorin interval).  The N x N products the call made are left in
        ``self.last_fermi_products``.
        """
        import torch
        N = H.shape[0]
        if H.shape != (N, N):
            raise ValueError("H must be N x N")
        if D_out is None:
            D_out = torch.empty_like(H)
        m = _D(float("nan") if mu is None else float(mu))
        its = _I(0)
        prods = ctypes.c_longlong(0)
        st = lib().sp2_fermi_density_matrix(self._h, N, _ptr(H), float(n_occ), float(kT), int(n_steps),
                                            int(max_newton), float(tol), ctypes.byref(m), _ptr(D_out),
                                            ctypes.byref(its), ctypes.byref(prods))
        self.last_fermi_products = prods.value
        self._check(st, "sp2_fermi_density_matrix")
        return D_out, m.value, its.value

    def sp2_fermi_density_matrix_nonorth(self, H, S, n_occ: float, kT: float, n_steps: int, mu=None,
                                         max_newton: int = 50, tol: float = 1e-10, D_out=None, W_out=None):
        """(D, W, mu, S_entropy / k_B, passes): the Fermi operator in the
        non-orthogonal basis of overlap S, its energy-weighted density matrix
        and the entropy of its occupations (mu as in sp2_fermi_density_matrix)."""
        import torch
        N = H.shape[0]
        if H.shape != (N, N) or S.shape != (N, N):
            raise ValueError("H and S must be N x N")
        if D_out is None:
            D_out = torch.empty_like(H)
        if W_out is None:
            W_out = torch.empty_like(H)
        m = _D(float("nan") if mu is None else float(mu))
        ent = _D(0.0)
        its = _I(0)
        self._check(lib().sp2_fermi_density_matrix_nonorth(self._h, N, _ptr(H), _ptr(S), float(n_occ), float(kT),
                                                           int(n_steps), int(max_newton), float(tol),
                                                           ctypes.byref(m), _ptr(D_out), _ptr(W_out),
                                                           ctypes.byref(ent), ctypes.byref(its)),
                    "sp2_fermi_density_matrix_nonorth")
        return D_out, W_out, m.value, ent.value, its.value

    def sp2_fermi_entropy(self, H, mu: float, kT: float):
        """(S / k_B, coefficients): -2 sum_i [f ln f + (1 - f) ln(1 - f)] of the Fermi occupations at mu."""
        N = H.shape[0]
        if H.shape != (N, N):
            raise ValueError("H must be N x N")
        S = _D(0.0)
        m = _I(0)
        self._check(lib().sp2_fermi_entropy(self._h, N, _ptr(H), float(mu), float(kT), ctypes.byref(S),
                                            ctypes.byref(m)), "sp2_fermi_entropy")
        return S.value, m.value

    def tb_overlap(self, model, xyz, S_out=None):
        """S of the non-orthogonal variant (model.overlap_s0, model.overlap_lam)."""
        import torch
        nat = xyz.shape[0]
        if S_out is None:
            S_out = torch.empty((4 * nat, 4 * nat), dtype=torch.float64, device=xyz.device)
        p = tb_params(model)
        self._check(lib().tb_overlap(self._h, ctypes.byref(p), float(model.overlap_s0), float(model.overlap_lam),
                                     nat, _ptr(xyz), _ptr(S_out)), "tb_overlap")
        return S_out

    def tb_hamiltonian_nonorth(self, model, xyz, S, n_aux=None, H_out=None):
        """H[n] = h + (S L + L S)/2 of the non-orthogonal variant (h for n_aux None)."""
        import torch
        nat = xyz.shape[0]
        if H_out is None:
            H_out = torch.empty((4 * nat, 4 * nat), dtype=torch.float64, device=xyz.device)
        p = tb_params(model)
        self._check(lib().tb_hamiltonian_nonorth(self._h, ctypes.byref(p), nat, _ptr(xyz),
                                                 _ptr(n_aux) if n_aux is not None else None, _ptr(S),
                                                 _ptr(H_out)), "tb_hamiltonian_nonorth")
        return H_out

    def tb_forces_nonorth(self, model, xyz, D, H, q, n_aux, F_out=None):
        """(F, U): forces at constant n and the potential energy, non-orthogonal basis."""
        import torch
        nat = xyz.shape[0]
        if F_out is None:
            F_out = torch.empty((nat, 3), dtype=torch.float64, device=xyz.device)
        p = tb_params(model)
        U = ctypes.c_double()
        self._check(lib().tb_forces_nonorth(self._h, ctypes.byref(p), float(model.overlap_s0),
                                            float(model.overlap_lam), nat, _ptr(xyz), _ptr(D), _ptr(H),
                                            _ptr(q), _ptr(n_aux), _ptr(F_out), ctypes.byref(U)),
                    "tb_forces_nonorth")
        return F_out, U.value

    def sp2_mulliken_overlap(self, D, S, n_atoms: int, z_val: float = 4.0, q_out=None):
        import torch
        if q_out is None:
            q_out = torch.empty(n_atoms, dtype=torch.float64, device=D.device)
        self._check(lib().sp2_mulliken_overlap(self._h, int(n_atoms), _ptr(D), _ptr(S), float(z_val),
                                               _ptr(q_out)), "sp2_mulliken_overlap")
        return q_out

    def sp2_int8_mfma_rate(self) -> float:
        """Sustained rate (ops/s) of v_mfma_i32_32x32x32_i8 on this device with no
        memory traffic, on operands in the digit planes' range."""
        v = _D()
        self._check(lib().sp2_int8_mfma_rate(self._h, ctypes.byref(v)), "sp2_int8_mfma_rate")
        return v.value

    def sp2_autotune(self, N: int, precision="int8x", slices: int = 5, levels: int = 0):
        """Time the product kernel per launch configuration (tile order; K-stage
        configuration for int8x; split cap and, up to N = 2048, output tile for
        fp64) at size N; the choice is kept for later solves of that size and
        precision (tile_group = -1).  Candidates are keyed (tile_group,
        stage_cfg, split_cap, tile)."""
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        r = TuneResult()
        self._check(lib().sp2_autotune(self._h, int(N), prec, int(slices), int(levels), ctypes.byref(r)),
                    "sp2_autotune")
        return {"tile_group": r.tile_group, "stage_cfg": r.stage_cfg, "split_cap": r.split_cap, "tile": r.tile,
                "ms_per_product": {tuple(r.candidates[k]): r.ms_per_product[k] for k in range(r.n_candidates)}}

    def sp2_tune_save(self, path: str):
        self._check(lib().sp2_tune_save(self._h, str(path).encode()), "sp2_tune_save")

    def sp2_tune_load(self, path: str):
        self._check(lib().sp2_tune_load(self._h, str(path).encode()), "sp2_tune_load")

    def sp2_mulliken(self, D, n_atoms: int, z_val: float = 4.0, q_out=None):
        import torch
        if q_out is None:
            q_out = torch.empty(n_atoms, dtype=torch.float64, device=D.device)
        self._check(lib().sp2_mulliken(self._h, int(n_atoms), _ptr(D), float(z_val), _ptr(q_out)),
                    "sp2_mulliken")
        return q_out

    def sp2_band_energy(self, D, H) -> float:
        e = ctypes.c_double()
        self._check(lib().sp2_band_energy(self._h, D.shape[0], _ptr(D), _ptr(H), ctypes.byref(e)),
                    "sp2_band_energy")
        return e.value

    def tb_hamiltonian(self, model, xyz, n_aux=None, H_out=None):
        import torch
        nat = xyz.shape[0]
        if H_out is None:
            H_out = torch.empty((4 * nat, 4 * nat), dtype=torch.float64, device=xyz.device)
        p = tb_params(model)
        self._check(lib().tb_hamiltonian(self._h, ctypes.byref(p), nat, _ptr(xyz), _ptr(n_aux),
                                         _ptr(H_out)), "tb_hamiltonian")
        return H_out

    def tb_hamiltonian_mem(self, model, xyz, n_aux=None, H_out=None):
        """xyz, n_aux and H in host memory (numpy) or on the device (CUDA tensors)."""
        import numpy as np
        nat = xyz.shape[0]
        host = isinstance(xyz, np.ndarray)
        if H_out is None:
            H_out = (np.empty((4 * nat, 4 * nat)) if host else
                     xyz.new_empty((4 * nat, 4 * nat)))
        conv = _host_ptr if host else _ptr
        p = tb_params(model)
        self._check(lib().tb_hamiltonian_mem(self._h, ctypes.byref(p), nat, conv(xyz), conv(n_aux), conv(H_out),
                                             SP2_MEM_HOST if host else SP2_MEM_DEVICE), "tb_hamiltonian_mem")
        return H_out

    def tb_forces(self, model, xyz, D, q, n_aux, F_out=None):
        import torch
        nat = xyz.shape[0]
        if F_out is None:
            F_out = torch.empty((nat, 3), dtype=torch.float64, device=xyz.device)
        U = ctypes.c_double()
        p = tb_params(model)
        self._check(lib().tb_forces(self._h, ctypes.byref(p), nat, _ptr(xyz), _ptr(D), _ptr(q),
                                    _ptr(n_aux), _ptr(F_out), ctypes.byref(U)), "tb_forces")
        return F_out, U.value

    def qmd_evaluate(self, model, xyz, n_aux=None, n_occ=None, opts: Sp2Options | None = None,
                     want_forces=True):
        """One evaluation at auxiliary charges n_aux (device tensors; None = 0):
        returns (q, e_band, e_pot, F or None, stats)."""
        import torch
        nat = xyz.shape[0]
        if n_occ is None:
            n_occ = int(round(model.z_val * nat / 2))
        q = torch.empty(nat, dtype=torch.float64, device=xyz.device)
        F = torch.empty((nat, 3), dtype=torch.float64, device=xyz.device) if want_forces else None
        eb, ep = ctypes.c_double(), ctypes.c_double()
        st = Sp2Stats()
        p = tb_params(model)
        o = opts if opts is not None else options("fp64")
        self._check(lib().qmd_evaluate(self._h, ctypes.byref(p), nat, _ptr(xyz),
                                       None if n_aux is None else _ptr(n_aux), int(n_occ), ctypes.byref(o),
                                       _ptr(q), ctypes.byref(eb), ctypes.byref(ep),
                                       None if F is None else _ptr(F), ctypes.byref(st)), "qmd_evaluate")
        return q, eb.value, ep.value, F, st.to_dict()

    def xlbomd_create(self, model, xyz, vel, n0=None, dt_fs=0.25, kappa=0.91, alpha=0.018,
                      c=(-6.0, 14.0, -8.0, -3.0, 4.0, -1.0), sp2_opts=None,
                      scf_beta=0.3, scf_tol=1e-10, scf_max_iter=None, diverge_q=1.0, kT=0.0,
                      fermi_steps=16, fermi_tol=0.0, fermi_max_newton=0):
        """scf_max_iter None: 0 (use n0 as given) if n0 is given, else 500 (SCF from zeros).
        diverge_q: stop with SP2_EDIVERGE when max|q - n| exceeds it (0: never).
        kT > 0: finite electronic temperature (Fermi operator with fermi_steps
        recursion steps; epot is then the free energy U - kT S); the paper's
        finite-temperature runs use kappa=KAPPA_FINITE_T; fermi_tol and
        fermi_max_newton bound the mu solve per step (0: the library's
        defaults)."""
        if scf_max_iter is None:
            scf_max_iter = 0 if n0 is not None else 500
        return XLBOMD(self, model, xyz, vel, n0, dt_fs, kappa, alpha, c, sp2_opts,
                      scf_beta, scf_tol, scf_max_iter, diverge_q, kT, fermi_steps, fermi_tol, fermi_max_newton)


class XLBOMD:
    """Handle of an xlbomd integrator; host numpy arrays in, host numpy arrays out."""

    def __init__(self, ctx, model, xyz, vel, n0, dt_fs, kappa, alpha, c, sp2_opts,
                 scf_beta=0.3, scf_tol=1e-10, scf_max_iter=500, diverge_q=1.0, kT=0.0, fermi_steps=16,
                 fermi_tol=0.0, fermi_max_newton=0):
        self.ctx = ctx
        self.nat = len(xyz)
        o = XLOptions()
        o.dt_fs, o.kappa, o.alpha, o.K = dt_fs, kappa, alpha, len(c) - 1
        for k, ck in enumerate(c):
            o.c[k] = ck
        o.sp2 = sp2_opts if sp2_opts is not None else options("fp64")
        o.scf_beta, o.scf_tol, o.scf_max_iter = scf_beta, scf_tol, scf_max_iter
        o.diverge_q = diverge_q
        o.overlap_s0 = float(getattr(model, "overlap_s0", 0.0))
        o.overlap_lam = float(getattr(model, "overlap_lam", 0.5))
        o.kT, o.fermi_steps = float(kT), int(fermi_steps)
        o.fermi_tol, o.fermi_max_newton = float(fermi_tol), int(fermi_max_newton)
        p = tb_params(model)
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        vel = np.ascontiguousarray(vel, dtype=np.float64)
        n0 = None if n0 is None else np.ascontiguousarray(n0, dtype=np.float64)
        self._h = ctypes.c_void_p()
        st = lib().xlbomd_create(ctx._h, ctypes.byref(p), ctypes.byref(o), self.nat,
                                 xyz.ctypes.data_as(_P), vel.ctypes.data_as(_P),
                                 None if n0 is None else n0.ctypes.data_as(_P), ctypes.byref(self._h))
        ctx._check(st, "xlbomd_create")
        ctx._children.add(self)

    def xlbomd_run(self, n_steps: int):
        recs = (XLRecord * max(n_steps, 1))()
        self.ctx._check(lib().xlbomd_run(self._h, int(n_steps), recs), "xlbomd_run")
        return [{"etot": r.etot, "epot": r.epot, "ekin": r.ekin,
                 "max_q_minus_n": r.max_q_minus_n, "sp2_iterations": r.sp2_iterations,
                 "fill_min": r.fill_min}
                for r in recs[:n_steps]]

    def xlbomd_counters(self):
        """(steps, density matrices built) since creation."""
        a, b = ctypes.c_longlong(), ctypes.c_longlong()
        self.ctx._check(lib().xlbomd_counters(self._h, ctypes.byref(a), ctypes.byref(b)), "xlbomd_counters")
        return a.value, b.value

    def xlbomd_info(self):
        it, res = ctypes.c_int(), ctypes.c_double()
        self.ctx._check(lib().xlbomd_info(self._h, ctypes.byref(it), ctypes.byref(res)), "xlbomd_info")
        return it.value, res.value

    def xlbomd_get(self):
        xyz = np.empty((self.nat, 3))
        vel = np.empty((self.nat, 3))
        q = np.empty(self.nat)
        n = np.empty(self.nat)
        self.ctx._check(lib().xlbomd_get(self._h, xyz.ctypes.data_as(_P), vel.ctypes.data_as(_P),
                                         q.ctypes.data_as(_P), n.ctypes.data_as(_P)), "xlbomd_get")
        return xyz, vel, q, n

    def xlbomd_get_state(self) -> bytes:
        n = ctypes.c_size_t(0)
        self.ctx._check(lib().xlbomd_get_state(self._h, None, ctypes.byref(n)), "xlbomd_get_state")
        buf = ctypes.create_string_buffer(n.value)
        self.ctx._check(lib().xlbomd_get_state(self._h, ctypes.cast(buf, _P), ctypes.byref(n)),
                        "xlbomd_get_state")
        return buf.raw[:n.value]

    def xlbomd_set_state(self, state: bytes):
        buf = ctypes.create_string_buffer(bytes(state), len(state))
        self.ctx._check(lib().xlbomd_set_state(self._h, ctypes.cast(buf, _P), len(state)), "xlbomd_set_state")

    def close(self):
        if self._h:
            lib().xlbomd_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching SP2 server (host numpy matrices in and out)."""

    def __init__(self, ctx: Context, **kw):
        o = ServerOptions()
        lib().sp2_server_options_default(ctypes.byref(o))
        for k, v in kw.items():
            if not hasattr(o, k):
                raise KeyError(k)
            setattr(o, k, v)
        self.ctx = ctx
        self._h = ctypes.c_void_p()
        st = lib().sp2_server_create(ctx._h, ctypes.byref(o), ctypes.byref(self._h))
        if st != SP2_OK:
            raise Sp2Error(st, "sp2_server_create: " + lib().sp2_strerror(st).decode())
        ctx._children.add(self)

    def sp2_server_submit(self, H, n_occ: int) -> int:
        H = np.ascontiguousarray(H, dtype=np.float64)
        t = ctypes.c_uint64()
        st = lib().sp2_server_submit(self._h, H.shape[0], H.ctypes.data_as(_P), int(n_occ), ctypes.byref(t))
        if st != SP2_OK:
            raise Sp2Error(st, "sp2_server_submit: " + lib().sp2_strerror(st).decode())
        return t.value

    def sp2_server_wait(self, ticket: int, N: int, timeout_s: float = -1.0, want_D: bool = True):
        D = np.empty((N, N)) if want_D else None
        q = np.empty(N // 4) if N % 4 == 0 else None
        stats = Sp2Stats()
        st = lib().sp2_server_wait(self._h, ctypes.c_uint64(ticket), float(timeout_s),
                                   D.ctypes.data_as(_P) if D is not None else None,
                                   q.ctypes.data_as(_P) if q is not None else None, ctypes.byref(stats))
        if st != SP2_OK:
            raise Sp2Error(st, "sp2_server_wait: " + lib().sp2_strerror(st).decode())
        return D, q, stats.to_dict()

    def sp2_server_report(self):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        lib().sp2_server_report(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        return {"p50_ms": a.value, "p99_ms": b.value, "solves_per_s": c.value}

    def close(self):
        if self._h:
            lib().sp2_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""Oracle: exact zero-temperature density matrix by Jacobi + aufbau.

Test infrastructure only.  The density matrix of the orthogonal T_e = 0
formulation is the step function of the Hamiltonian, rho = theta(mu0 I - H),
with the step at the chemical potential separating occupied from unoccupied
states (Appendix, orthogonal T_e = 0 subsection; Eq. EL_4c at zero
temperature).  Written out: the projector onto the eigenvectors of the
N_occ lowest eigenvalues.  Orbitals are doubly occupied (Eq. DFT_POT), so
Tr rho = N_occ = number of electrons / 2.

Reading for a degenerate Fermi level (the paper is silent): the gap
eps_{N_occ+1} - eps_{N_occ} is reported; ties are broken by eigenvector
index (stable sort), so the projector is then not unique.

Pinned in tests/test_oracle_eig.py against closed forms and an independent
library eigensolver.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jacobi.c")
_LIB = os.path.join(_HERE, "liboracle_jacobi.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile jacobi.c with gcc into a shared library next to it."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        _lib.oracle_jacobi_eigh.restype = ctypes.c_int
        _lib.oracle_jacobi_eigh.argtypes = [
            ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_double, ctypes.c_int]
    return _lib


def jacobi_eigh(A, tol: float = 1e-15, max_sweeps: int = 60):
    """Eigenvalues (ascending) and eigenvectors (columns) of symmetric A."""
    A = np.array(A, dtype=np.float64, order="C", copy=True)
    n = A.shape[0]
    w = np.empty(n)
    V = np.empty((n, n))
    sweeps = _load().oracle_jacobi_eigh(n, A.ctypes.data, w.ctypes.data,
                                        V.ctypes.data, tol, max_sweeps)
    if sweeps < 0:
        raise RuntimeError("Jacobi did not converge")
    order = np.argsort(w, kind="stable")
    return w[order], V[:, order]


def density_matrix(H, n_occ: int):
    """rho = theta(mu0 I - H): projector on the n_occ lowest eigenvectors.

    Returns (rho, eigenvalues ascending, gap = eps[n_occ] - eps[n_occ-1]).
    """
    w, V = jacobi_eigh(H)
    Vo = V[:, :n_occ]
    rho = Vo @ Vo.T
    gap = float(w[n_occ] - w[n_occ - 1]) if n_occ < len(w) else float("inf")
    return rho, w, gap


def band_energy_from_eigenvalues(w, n_occ: int) -> float:
    """2 * sum of the n_occ lowest eigenvalues (doubly occupied, Eq. DFT_POT)."""
    return 2.0 * float(np.sum(w[:n_occ]))

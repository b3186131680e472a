"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module holds no arithmetic of the method itself: it only draws
positions, velocities and request streams from seeded generators and holds
the numeric model parameters that both sides read.  Everything that turns
those numbers into a Hamiltonian, a density matrix, charges or forces lives
separately in ``oracle/`` (CPU reference) and in the HIP library.

Workloads (stand-ins for the paper's hydrocarbon systems, whose LATTE
parameters and structures are not published):

* a jittered simple-cubic lattice of "carbon-like" atoms with four
  orthogonal valence orbitals (s, px, py, pz) each, spacing 1.5 A, Gaussian
  jitter sigma = 0.1 A per coordinate, atoms ordered x fastest, then y, then z,
  so orbital index = 4 * atom + {0: s, 1: px, 2: py, 3: pz};
* its gapped variant: closed-shell atoms with two valence electrons (s^2) and
  the p level at +4 eV on a 2.0 A lattice, a wire of 4 x 4 atoms in
  cross-section;
* Maxwell-Boltzmann velocities at a given temperature (centre-of-mass
  momentum removed);
* a Poisson stream of solve requests with uniformly drawn system sizes.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Physical constants (CODATA 2018) in the eV / A / amu / fs unit system.
KB_EV_PER_K = 8.617333262e-5          # Boltzmann constant, eV/K
COULOMB_EV_A = 14.399645478           # e^2 / (4 pi eps0), eV * A
ACC_A_FS2 = 9.648533212e-3            # 1 eV/(A*amu) expressed in A/fs^2
KE_EV = 103.6426965                   # 1 amu*A^2/fs^2 expressed in eV


@dataclasses.dataclass(frozen=True)
class TBModel:
    """Numeric parameters of the synthetic orthogonal sp tight-binding model.

    Hopping magnitude |t(r)| = t0 * exp(-(r - r0) / lam) for r < r_cut; on
    [r_tail, r_cut) a quintic tail replaces it when r_tail < r_cut (r_tail ==
    r_cut means a hard cut).  Bond-integral signs: ss-sigma = -|t|,
    sp-sigma = +|t|, pp-sigma = +|t|, pp-pi = -|t|.
    """
    eps_s: float = -8.0
    eps_p: float = -4.0
    t0: float = 2.0
    r0: float = 1.5
    lam: float = 0.5
    r_cut: float = 4.0
    r_tail: float = 4.0
    hubbard_u: float = 4.0
    coulomb_k: float = COULOMB_EV_A
    pair_a: float = 0.0        # pair repulsion amplitude, eV (0 = no pair term)
    pair_r0: float = 1.5
    pair_rho: float = 0.3
    mass: float = 12.0         # amu
    z_val: int = 4             # valence electrons per neutral atom
    # overlap of the non-orthogonal variant: s(r) = overlap_s0 exp(-(r - r0)/overlap_lam)
    # with the hopping's tail (0: orthogonal basis, S = I)
    overlap_s0: float = 0.0
    overlap_lam: float = 0.5

    def with_(self, **kw) -> "TBModel":
        return dataclasses.replace(self, **kw)


# Static configurations use the literal hard cut-off at 4 A; molecular
# dynamics uses the smooth tail on [3.5, 4.0] A so the energy is continuous,
# and a pair repulsion.  With gamma_ij = k_e / r the self-consistent charges
# order to +-4 e, so the repulsion must hold a +-4 e pair apart against a
# Coulomb attraction that diverges at r -> 0: with rho = 0.3 A no amplitude
# does both (at the zero-virial amplitude the pair energy falls all the way
# to r -> 0), while rho = 0.15 A puts a wall near 1 A.  The amplitude is the
# one for which the self-consistent unjittered 4 x 4 x 4 lattice has zero
# mean virial (computed by oracle/calibrate_pair.py).
STATIC_MODEL = TBModel()
MD_MODEL = TBModel(r_tail=3.5, pair_a=5.605396, pair_rho=0.15)


def lattice_positions(dims, spacing: float = 1.5, jitter: float = 0.1,
                      seed: int = 0, n_atoms: int | None = None) -> np.ndarray:
    """Jittered simple-cubic lattice, x fastest, then y, then z.

    Returns float64 array (n_atoms, 3) in Angstrom.  If ``n_atoms`` is given,
    only the first ``n_atoms`` lattice sites (in that order) are kept, before
    the jitter is drawn.
    """
    nx, ny, nz = (int(d) for d in dims)
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                             indexing="ij")
    sites = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    if n_atoms is not None:
        sites = sites[:n_atoms]
    rng = np.random.default_rng(seed)
    return sites * spacing + rng.normal(0.0, jitter, size=sites.shape)


def maxwell_velocities(n_atoms: int, temperature_k: float, mass_amu: float,
                       seed: int) -> np.ndarray:
    """Velocities in A/fs drawn from N(0, kT/M) per component, zero total momentum."""
    rng = np.random.default_rng(seed)
    # kT/M in eV/amu -> (A/fs)^2 via 1 amu*A^2/fs^2 = KE_EV eV
    sigma = math.sqrt(KB_EV_PER_K * temperature_k / (mass_amu * KE_EV))
    v = rng.normal(0.0, sigma, size=(n_atoms, 3))
    v -= v.mean(axis=0, keepdims=True)
    return v


def checkerboard_charges(dims, amplitude: float = 4.0) -> np.ndarray:
    """+-amplitude on the two sublattices of the cubic lattice (x fastest order).

    A starting guess for the self-consistent charges: the literal gamma of the
    model orders the charges this way at self-consistency.
    """
    nx, ny, nz = (int(d) for d in dims)
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    parity = ((ix + iy + iz) % 2).ravel()
    return np.where(parity == 0, amplitude, -amplitude).astype(np.float64)


def cube_dims_for(n_atoms: int):
    side = int(math.ceil(round(n_atoms ** (1.0 / 3.0), 9)))
    while side ** 3 < n_atoms:
        side += 1
    return (side, side, side)


@dataclasses.dataclass(frozen=True)
class Request:
    index: int
    arrival_s: float
    n_atoms: int
    seed: int

    @property
    def n_orb(self) -> int:
        return 4 * self.n_atoms

    def positions(self) -> np.ndarray:
        return lattice_positions(cube_dims_for(self.n_atoms), seed=self.seed,
                                 n_atoms=self.n_atoms)


def request_stream(n_requests: int = 512, rate_per_s: float = 200.0,
                   min_atoms: int = 32, max_atoms: int = 512,
                   size_seed: int = 5, arrival_seed: int = 4,
                   first_pos_seed: int = 1000):
    """Open-loop Poisson request stream with uniformly drawn system sizes."""
    sizes = np.random.default_rng(size_seed).integers(min_atoms, max_atoms + 1,
                                                      size=n_requests)
    gaps = np.random.default_rng(arrival_seed).exponential(1.0 / rate_per_s,
                                                           size=n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    return [Request(i, float(arrivals[i]), int(sizes[i]), first_pos_seed + i)
            for i in range(n_requests)]


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    dims: tuple
    seed: int
    spacing: float = 1.5
    electrons_per_atom: int = 4

    @property
    def n_atoms(self) -> int:
        return self.dims[0] * self.dims[1] * self.dims[2]

    @property
    def n_orb(self) -> int:
        return 4 * self.n_atoms

    @property
    def n_occ(self) -> int:
        # neutral atoms, doubly occupied orbitals
        return self.electrons_per_atom * self.n_atoms // 2

    def positions(self) -> np.ndarray:
        return lattice_positions(self.dims, spacing=self.spacing, seed=self.seed)


# The five workloads: a 256-orbital FP64 solve, a 4096-orbital XL-BOMD run,
# the 8192-orbital mixed-precision solve, the 16384-orbital elongated
# thresholded solve and the serving stream (``request_stream``).
SMALL = Workload("fp64_n256", (4, 4, 4), 0)
XLBOMD = Workload("xlbomd_n4096", (8, 8, 16), 1)
XLBOMD_VEL_SEED = 101
MIXED = Workload("mixed_n8192", (8, 16, 16), 2)
SPARSE = Workload("blocksparse_n16384", (8, 8, 64), 3)


# Gapped variant for the thresholded (linear-scaling) solver.  Atoms with two
# valence electrons (a closed s^2 shell) fill one orbital each: the Fermi
# level sits at quarter filling, between the s band and the p bands.  On the
# 1.5 A lattice the bands overlap (no gap); raising the p level to +4 eV and
# stretching the lattice to 2.0 A opens a gap of about 5 eV (band width about
# 21 eV), so D decays exponentially with distance, as in the insulating
# hydrocarbons of the paper.  The wire is 4 x 4 atoms in cross-section
# (64 orbitals per layer) and grows along z.
GAPPED_MODEL = TBModel(eps_p=4.0, z_val=2)
GAPPED_SPACING = 2.0
# For MD on the gapped wire: the smooth hopping tail of MD_MODEL and a pair
# repulsion whose amplitude gives the self-consistent unjittered 4 x 4 x 4
# lattice at 2.0 A zero virial (oracle/calibrate_pair.py).
GAPPED_MD_MODEL = GAPPED_MODEL.with_(r_tail=3.5, pair_a=3.373945, pair_rho=0.15)


# Non-orthogonal variant: the static model with overlap integrals of
# magnitude 0.05 at 1.5 A (dimensionless), decaying like the hopping; S stays
# well conditioned (smallest eigenvalue about 0.72 on these lattices).
NONORTH_MODEL = STATIC_MODEL.with_(overlap_s0=0.05)


def gapped_workload(n_layers: int, seed: int = 3) -> Workload:
    return Workload(f"gapped_wire_4x4x{n_layers}", (4, 4, int(n_layers)), seed, GAPPED_SPACING, 2)


def small_workload(dims, seed) -> Workload:
    return Workload(f"lattice_{dims[0]}x{dims[1]}x{dims[2]}_s{seed}", tuple(dims), seed)


# Seeded draws that select what a full-size comparison samples: Gaussian probe
# vectors (D V estimates ||D - D_ref||_F, since E|A v|^2 = ||A||_F^2 for
# v ~ N(0, I)), entries of H and 32 x 32 blocks of D.
PROBE_SEED, PROBES = 12, 2
H_SAMPLE_SEED, H_SAMPLES = 11, 4096
BLOCK_SEED, BLOCKS = 13, 8


def probe_vectors(n: int) -> np.ndarray:
    """(n, PROBES) standard normal probe vectors."""
    return np.random.default_rng(PROBE_SEED).standard_normal((n, PROBES))


def h_sample_index(n: int):
    """Row and column indices of sampled H entries: half uniform, half within
    64 orbitals of the diagonal."""
    rng = np.random.default_rng(H_SAMPLE_SEED)
    i = rng.integers(0, n, H_SAMPLES)
    j = np.where(np.arange(H_SAMPLES) % 2 == 0, rng.integers(0, n, H_SAMPLES),
                 np.clip(i + rng.integers(-64, 65, H_SAMPLES), 0, n - 1))
    return i, j


def block_index(nb: int):
    """Block-row and block-column indices of sampled 32 x 32 blocks of an
    nb x nb block grid: half within two blocks of the diagonal, half uniform."""
    rng = np.random.default_rng(BLOCK_SEED)
    bi = rng.integers(0, nb, BLOCKS)
    bj = np.where(np.arange(BLOCKS) < BLOCKS // 2, np.clip(bi + rng.integers(-2, 3, BLOCKS), 0, nb - 1),
                  rng.integers(0, nb, BLOCKS))
    return bi, bj


def permuted_groups(pos: np.ndarray, seed: int, group: int = 8) -> np.ndarray:
    """The same atoms with consecutive groups of `group` atoms (32 orbitals,
    one 32 x 32 block row, for group = 8) put in a seeded random order; the
    order inside a group is kept.  The groups are spatially compact (8
    neighbouring sites of a lattice row), so a Hamiltonian built from them is
    as block-sparse as the banded one, but its nonzero blocks are scattered
    over the whole matrix instead of lying in a band."""
    n = len(pos)
    ng = n // group
    order = np.random.default_rng(seed).permutation(ng)
    idx = (order[:, None] * group + np.arange(group)[None, :]).ravel()
    return np.concatenate([pos[idx], pos[ng * group:]])


PERMUTED_SEED = 31

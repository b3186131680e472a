"""Finite electronic temperature on the GPU: the Fermi operator by the
recursive expansion (rocBLAS GEMMs, Newton-Schulz inverses, canonical mu by
Newton) against the oracle's recursion at the same number of steps and against
the definition by eigendecomposition."""
import sys
import time

import numpy as np
import pytest

import synth
from oracle import fermi, observables, sp2 as osp2, tb as otb

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_1203_6836_amd as p
    c = p.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def lattice(dims, seed):
    w = synth.small_workload(dims, seed)
    return w, otb.hamiltonian(w.positions(), None, synth.STATIC_MODEL)


@pytest.mark.parametrize("dims,seed,kT,n", [((3, 3, 3), 1, 0.5, 10), ((3, 3, 3), 2, 0.5, 14),
                                            ((4, 4, 9), 3, 1.0, 12)])
def test_fixed_mu_matches_oracle_recursion(ctx, dims, seed, kT, n):
    w, H = lattice(dims, seed)
    say(f"case fermi fixed mu N={w.n_orb} kT={kT} n={n}")
    e = np.linalg.eigvalsh(H)
    mu = 0.5 * (e[w.n_occ - 1] + e[w.n_occ])
    ref = fermi.recursive_fermi(H, mu, kT, n)
    D, mu_out, passes = ctx.sp2_fermi_density_matrix(to_dev(H), w.n_occ, kT, n, mu=mu, max_newton=0)
    D = D.cpu().numpy()
    err = float(np.abs(D - ref).max())
    say(f"  max|D - oracle| {err:.2e}, passes {passes}")
    assert passes == 1 and mu_out == mu
    assert np.array_equal(D, D.T)
    assert err < 1e-10


@pytest.mark.parametrize("dims,seed,kT", [((3, 3, 3), 1, 0.5), ((4, 4, 8), 5, 0.25), ((4, 4, 9), 3, 2.0)])
def test_canonical_matches_oracle_and_definition(ctx, dims, seed, kT):
    w, H = lattice(dims, seed)
    say(f"case fermi canonical N={w.n_orb} kT={kT}")
    X, mu_ref, its_ref = fermi.recursive_fermi_canonical(H, w.n_occ, kT, 16, tol=1e-9)
    Dd, mu_def, _ = fermi.fermi_density(H, w.n_occ, kT)
    D, mu, passes = ctx.sp2_fermi_density_matrix(to_dev(H), w.n_occ, kT, 16, tol=1e-9)
    D = D.cpu().numpy()
    e_rec = float(np.abs(D - X).max())
    e_def = float(np.abs(D - Dd).max())
    say(f"  passes gpu={passes} oracle={its_ref}, mu {mu:.12f} (oracle {mu_ref:.12f}, definition {mu_def:.12f}), "
        f"max|D - recursion| {e_rec:.2e}, max|D - definition| {e_def:.2e}, Tr D - n_occ {np.trace(D) - w.n_occ:+.1e}")
    assert abs(passes - its_ref) <= 1
    assert abs(mu - mu_ref) < 1e-9 and abs(mu - mu_def) < 1e-8
    assert abs(np.trace(D) - w.n_occ) < 1e-9
    assert e_rec < 1e-9 and e_def < 1e-8


def test_low_temperature_limit_is_the_projector(ctx):
    """kT = 0.02 eV on the gapped wire (gap ~5 eV): D equals the zero-temperature
    projector (the oracle's SP2 result) to the Fermi tail's e^(-gap/2kT)."""
    w = synth.gapped_workload(2)
    H = otb.hamiltonian(w.positions(), None, synth.GAPPED_MODEL)
    say(f"case fermi low T N={w.n_orb}")
    P = osp2.sp2(H, w.n_occ).D
    D, mu, passes = ctx.sp2_fermi_density_matrix(to_dev(H), w.n_occ, 0.02, 20, tol=1e-9)
    D = D.cpu().numpy()
    err = float(np.abs(D - P).max())
    say(f"  mu {mu:.6f}, passes {passes}, max|D - projector| {err:.2e}")
    assert err < 1e-9


def test_fermi_rejects_bad_arguments(ctx):
    import paper_1203_6836_amd as p
    w, H = lattice((2, 2, 2), 1)
    Hd = to_dev(H)
    say("case fermi argument checks")
    for kw in ({"kT": 0.0, "n_steps": 12}, {"kT": 0.5, "n_steps": 0}, {"kT": 0.5, "n_steps": 2},
               {"kT": 0.5, "n_steps": 12, "max_newton": 0}):
        with pytest.raises(p.Sp2Error) as ei:
            ctx.sp2_fermi_density_matrix(Hd, w.n_occ, **kw)
        assert ei.value.status == p.SP2_EINVAL, kw
    Hb = H.copy()
    Hb[0, 1] += 1.0
    with pytest.raises(p.Sp2Error) as ei:
        ctx.sp2_fermi_density_matrix(to_dev(Hb), w.n_occ, 0.5, 12)
    assert ei.value.status == p.SP2_EINVAL
    e_lo = osp2.gershgorin(H)[0]
    with pytest.raises(p.Sp2Error) as ei:   # one pass from a mu near the bottom of the spectrum
        ctx.sp2_fermi_density_matrix(Hd, w.n_occ, 0.5, 12, mu=e_lo + 1.0, max_newton=1)
    assert ei.value.status == p.SP2_ENOCONV


def test_fermi_full_size_against_definition(ctx):
    """N = 2048 (512 atoms): the canonical Fermi operator at kT = 0.5 eV with 16
    steps against the definition (eigendecomposition on the host), and its
    GEMM rate."""
    import torch
    w, H = lattice((8, 8, 8), 7)
    say(f"case fermi N={w.n_orb}")
    Hd = to_dev(H)
    ctx.sp2_fermi_density_matrix(Hd, w.n_occ, 0.5, 16, tol=1e-8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    D, mu, passes = ctx.sp2_fermi_density_matrix(Hd, w.n_occ, 0.5, 16, tol=1e-8)
    torch.cuda.synchronize()
    s = time.perf_counter() - t0
    prods = ctx.last_fermi_products
    assert passes * 2 * 16 <= prods <= passes * 10 * 16
    tf = prods * 2.0 * w.n_orb ** 3 / s / 1e12
    Dd, mu_def, _ = fermi.fermi_density(H, w.n_occ, 0.5, solver="lapack")   # Jacobi is too slow at N = 2048
    err = float(np.abs(D.cpu().numpy() - Dd).max())
    say(f"  {s * 1e3:.1f} ms, {passes} passes, {prods} products, {tf:.1f} TF/s in GEMMs, mu - mu_def {mu - mu_def:+.1e}, "
        f"max|D - definition| {err:.2e}")
    assert err < 1e-7 and abs(mu - mu_def) < 1e-6


def test_finite_temperature_forces_match_oracle(ctx):
    """Forces and U at constant n with the Fermi D (kT = 0.5 eV): the GPU's
    Fermi operator fed to the GPU's force kernel against the oracle's
    definition and force expression (-dA/dR, A = U - T_e S, by the oracle's
    finite-difference pin)."""
    m = synth.MD_MODEL
    dims = (3, 3, 3)
    pos = synth.lattice_positions(dims, seed=21)
    nat = len(pos)
    n = np.random.default_rng(5).uniform(-0.2, 0.2, nat)
    n_occ = 2 * nat
    say(f"case fermi forces N={4 * nat} kT=0.5")
    A, Dd, mu_d = fermi.free_energy(pos, n, m, n_occ, 0.5)
    F_ref = observables.forces(pos, n, Dd, m)
    U_ref = observables.potential_energy(pos, n, Dd, m)
    xyz, nd = to_dev(pos), to_dev(n)
    H = ctx.tb_hamiltonian(m, xyz, nd)
    D, mu, _ = ctx.sp2_fermi_density_matrix(H, n_occ, 0.5, 16, tol=1e-9)
    q = ctx.sp2_mulliken(D, nat)
    F, U = ctx.tb_forces(m, xyz, D, q, nd)
    dF = float(np.abs(F.cpu().numpy() - F_ref).max())
    say(f"  mu {mu:.10f} (definition {mu_d:.10f}), max|dF| {dF:.2e} (max|F| {np.abs(F_ref).max():.1f}), "
        f"dU {U - U_ref:+.2e}")
    assert abs(mu - mu_d) < 1e-8
    assert dF < 1e-8 and abs(U - U_ref) < 1e-8


@pytest.mark.parametrize("dims,seed,kT", [((3, 3, 3), 1, 0.5), ((4, 4, 8), 5, 0.25), ((4, 4, 9), 3, 2.0)])
def test_entropy_matches_definition(ctx, dims, seed, kT):
    """S / k_B by Chebyshev moments on the GPU against the oracle's entropy of
    the eigenvalue occupations at the same mu."""
    import paper_1203_6836_amd as p
    w, H = lattice(dims, seed)
    say(f"case fermi entropy N={w.n_orb} kT={kT}")
    e = np.linalg.eigvalsh(H)
    mu = fermi.canonical_mu(e, w.n_occ, 1.0 / kT)
    S_ref = fermi.entropy(fermi.fermi_occupations(e, mu, 1.0 / kT))
    S, m = ctx.sp2_fermi_entropy(to_dev(H), mu, kT)
    say(f"  S {S:.12f} (oracle {S_ref:.12f}), rel {(S - S_ref) / S_ref:+.1e}, {m} coefficients")
    assert abs(S - S_ref) < 1e-10 * S_ref
    with pytest.raises(p.Sp2Error) as ei:
        ctx.sp2_fermi_entropy(to_dev(H), mu, 0.01)
    assert ei.value.status == p.SP2_EINVAL


def test_finite_temperature_xlbomd_matches_oracle(ctx):
    """XL-BOMD at kT = 0.5 eV (Fermi operator, its entropy in the free energy,
    forces of the Fermi D every step) on the 3 x 3 x 3 cluster, whose gap
    (0.16 eV) is well below kT: 20 steps from self-consistent finite-T charges
    against the oracle integrator with the Fermi operator by definition."""
    import paper_1203_6836_amd as p
    from oracle import xlbomd as oxl
    say("case fermi xlbomd 3x3x3 20 steps kT=0.5")
    m = synth.MD_MODEL
    pos = synth.lattice_positions((3, 3, 3), seed=21)
    nat, nocc = len(pos), 2 * len(pos)
    vel = synth.maxwell_velocities(nat, 300.0, m.mass, seed=5)
    n0 = np.zeros(nat)
    for _ in range(2000):   # finite-T SCF by linear mixing
        q = oxl.evaluate(pos, n0, m, nocc, want_forces=False, kT=0.5)["q"]
        if np.abs(q - n0).max() < 1e-11:
            break
        n0 = n0 + 0.1 * (q - n0)
    assert np.abs(q - n0).max() < 1e-11
    opts = oxl.XLOptions(kT=0.5, kappa=p.KAPPA_FINITE_T)   # the kappa rescaling of finite-T runs
    assert p.KAPPA_FINITE_T == 0.75 * oxl.K5_KAPPA
    ost, olog = oxl.run(oxl.init_state(pos, vel, m, nocc, opts, n0), m, nocc, opts, 20)
    md = ctx.xlbomd_create(m, pos, vel, n0, dt_fs=opts.dt_fs, kappa=opts.kappa, alpha=opts.alpha,
                           c=opts.c, sp2_opts=p.options("fp64"), kT=0.5, fermi_steps=16)
    glog = md.xlbomd_run(20)
    xyz, v, q, n = md.xlbomd_get()
    md.close()
    dx = float(np.abs(xyz - ost.pos).max())
    eg = np.array([r["etot"] for r in glog])
    eo = np.array([r["etot"] for r in olog])
    passes = [r["sp2_iterations"] for r in glog]
    say(f"  max|dx| {dx:.1e} A, max|dE_tot| {np.abs(eg - eo).max():.1e} eV, E_tot spread {np.ptp(eo) / nat:.1e} "
        f"eV/atom, Newton passes per step {passes[:3]}..{passes[-3:]}")
    np.testing.assert_allclose(xyz, ost.pos, atol=1e-9)
    np.testing.assert_allclose(v, ost.vel, atol=1e-9)
    # the step's canonical mu is solved to |Tr D - n_occ| < 1e-9, which bounds
    # how closely the charges, and the auxiliary charges built from them, agree
    np.testing.assert_allclose(n, ost.hist[0], atol=2e-8)
    assert np.abs(eg - eo).max() < 1e-7


def test_finite_temperature_checkpoint_resume_is_bit_identical(ctx):
    """A checkpoint of a kT > 0 integrator carries the chemical potential
    that starts the next step's mu solve: rewinding to it, or resuming it in a
    second integrator, continues bit-identically; a checkpoint of a kT = 0
    integrator is refused by a kT > 0 one and the other way round."""
    import paper_1203_6836_amd as p
    say("case fermi xlbomd checkpoint / resume 3x3x2 kT=0.5")
    m = synth.MD_MODEL
    pos = synth.lattice_positions((3, 3, 2), seed=4)
    nat = len(pos)
    vel = synth.maxwell_velocities(nat, 300.0, m.mass, seed=11)
    # zero start charges without an SCF: q - n stays large, so the divergence
    # check is off (the replay, not the physics, is under test)
    kw = dict(sp2_opts=p.options("fp64"), kT=0.5, fermi_steps=16, kappa=p.KAPPA_FINITE_T, diverge_q=0.0)
    md = ctx.xlbomd_create(m, pos, vel, np.zeros(nat), scf_max_iter=0, **kw)
    md.xlbomd_run(4)
    ck = md.xlbomd_get_state()
    assert len(ck) >= p.XL_CHECKPOINT_HEADER
    mu = np.frombuffer(ck[40:48], dtype=np.float64)[0]
    assert np.isfinite(mu)
    a = md.xlbomd_run(6)
    xa = md.xlbomd_get()
    md.xlbomd_set_state(ck)
    b = md.xlbomd_run(6)
    xb = md.xlbomd_get()
    md2 = ctx.xlbomd_create(m, pos + 0.03, np.zeros_like(vel), np.zeros(nat), scf_max_iter=0, **kw)
    md2.xlbomd_set_state(ck)
    c = md2.xlbomd_run(6)
    xc = md2.xlbomd_get()
    assert a == b == c
    for u, v, w in zip(xa, xb, xc):
        assert np.array_equal(u, v) and np.array_equal(u, w)
    md0 = ctx.xlbomd_create(m, pos, vel, np.zeros(nat), sp2_opts=p.options("fp64"), scf_max_iter=0,
                            diverge_q=0.0)
    ck0 = md0.xlbomd_get_state()
    for target, state in ((md, ck0), (md0, ck)):
        with pytest.raises(p.Sp2Error) as ei:
            target.xlbomd_set_state(state)
        assert ei.value.status == p.SP2_EINVAL
    md3 = ctx.xlbomd_create(m, pos, vel, np.zeros(nat), scf_max_iter=0, **{**kw, "fermi_steps": 14})
    with pytest.raises(p.Sp2Error) as ei:
        md3.xlbomd_set_state(ck)
    assert ei.value.status == p.SP2_EINVAL
    for h in (md, md2, md0, md3):
        h.close()


def test_finite_temperature_xlbomd_2048_orbitals_newton_passes(ctx):
    """XL-BOMD at kT = 0.5 eV on a 512-atom lattice (N = 2048) with the
    default trace tolerance, which scales with N above the floor X_0 sets:
    every step completes, and after the first the mu solve started from the
    previous step's mu takes few passes."""
    import paper_1203_6836_amd as p
    say("case fermi xlbomd 8x8x8 kT=0.5, 6 steps")
    m = synth.MD_MODEL
    dims = (8, 8, 8)
    pos = synth.lattice_positions(dims, seed=23)
    nat = len(pos)
    vel = synth.maxwell_velocities(nat, 300.0, m.mass, seed=24)
    # the charge-ordered state's gap (about 18 eV) is far above kT: the SCF
    # from the +-4 e checkerboard converges as at zero temperature
    md = ctx.xlbomd_create(m, pos, vel, synth.checkerboard_charges(dims), sp2_opts=p.options("fp64"), kT=0.5,
                           fermi_steps=16, kappa=p.KAPPA_FINITE_T, scf_beta=1.0, scf_tol=1e-7, scf_max_iter=100)
    it, res = md.xlbomd_info()
    rec = md.xlbomd_run(6)
    md.close()
    passes = [r["sp2_iterations"] for r in rec]
    say(f"  SCF {it} iterations (res {res:.1e}); Newton passes per step {passes}, "
        f"max|q-n| {max(r['max_q_minus_n'] for r in rec):.1e}")
    assert max(passes[1:]) <= 8

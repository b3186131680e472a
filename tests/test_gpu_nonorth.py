"""Non-orthogonal formulation on the GPU (Loewdin factor by Newton-Schulz on
the project's FP64 product kernel, SP2 or the Fermi operator of Z^T H Z,
rho = Z rho_perp Z^T, Mulliken charges with S) against the oracle."""
import sys
import time

import numpy as np
import pytest

import synth
from oracle import nonorth, tb as otb

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


def system(dims, seed, model=None):
    m = model or synth.NONORTH_MODEL
    w = synth.small_workload(dims, seed)
    pos = w.positions()
    return w, otb.hamiltonian(pos, None, m), nonorth.overlap(pos, m)


@pytest.mark.parametrize("dims,seed", [((3, 3, 3), 4), ((4, 4, 8), 5)])
def test_fp64_nonorth_matches_oracle(ctx, dims, seed):
    import paper_1203_6836_amd as p
    w, H, S = system(dims, seed)
    say(f"case nonorth fp64 N={w.n_orb}")
    rho_ref, _, _, r = nonorth.density_matrix(H, S, w.n_occ)
    Sd = to_dev(S)
    D, st, its = ctx.sp2_density_matrix_nonorth(to_dev(H), Sd, w.n_occ, p.options("fp64"))
    q = ctx.sp2_mulliken_overlap(D, Sd, w.n_atoms).cpu().numpy()
    D = D.cpu().numpy()
    err = np.linalg.norm(D - rho_ref) / np.sqrt(w.n_orb)
    dq = float(np.abs(q - nonorth.mulliken(rho_ref, S)).max())
    say(f"  factor steps {its}, SP2 iterations gpu={st['iterations']} oracle={r.iterations}, "
        f"err/sqrtN {err:.2e}, max|dq| {dq:.2e}, Tr[DS] - n_occ {np.trace(D @ S) - w.n_occ:+.1e}")
    assert st["iterations"] == r.iterations
    assert err <= 1e-9 and dq <= 1e-9
    assert abs(np.trace(D @ S) - w.n_occ) < 1e-8


@pytest.mark.parametrize("recipe", [{}, {"slices": 4, "levels": 5}])
def test_int8x_nonorth_matches_oracle(ctx, recipe):
    """Five planes (the library default) and four planes with five levels
    (the benchmark's recipe)."""
    import paper_1203_6836_amd as p
    w, H, S = system((8, 8, 8), 2)
    say(f"case nonorth int8x N={w.n_orb} {recipe}")
    rho_ref, _, _, _ = nonorth.density_matrix(H, S, w.n_occ, solver="lapack")   # N = 2048: library eigensolver
    Sd = to_dev(S)
    D, st, its = ctx.sp2_density_matrix_nonorth(to_dev(H), Sd, w.n_occ, p.options("int8x", **recipe))
    q = ctx.sp2_mulliken_overlap(D, Sd, w.n_atoms).cpu().numpy()
    D = D.cpu().numpy()
    err = np.linalg.norm(D - rho_ref) / np.sqrt(w.n_orb)
    dq = float(np.abs(q - nonorth.mulliken(rho_ref, S)).max())
    say(f"  factor steps {its}, SP2 iterations {st['iterations']}, err/sqrtN {err:.2e}, max|dq| {dq:.2e}")
    assert err <= 1e-6 and dq <= 1e-6


def test_identity_overlap_is_the_orthogonal_solve(ctx):
    """S = I: the factor is I after one step and the result is bitwise the
    orthogonal solve's."""
    import torch
    import paper_1203_6836_amd as p
    w, H, _ = system((4, 4, 4), 0)
    say("case nonorth with S = I vs orthogonal solve")
    Hd = to_dev(H)
    I = torch.eye(w.n_orb, dtype=torch.float64, device="cuda")
    D0, s0 = ctx.sp2_density_matrix(Hd, w.n_occ, p.options("fp64"))
    D1, s1, its = ctx.sp2_density_matrix_nonorth(Hd, I, w.n_occ, p.options("fp64"))
    assert its == 1 and s0["iterations"] == s1["iterations"]
    assert torch.equal(D0, D1)
    q0 = ctx.sp2_mulliken(D0, w.n_atoms)
    q1 = ctx.sp2_mulliken_overlap(D1, I, w.n_atoms)
    assert float((q0 - q1).abs().max()) < 1e-13


@pytest.mark.parametrize("dims,seed", [((3, 3, 3), 4), ((5, 4, 3), 9)])
def test_overlap_builder_matches_oracle(ctx, dims, seed):
    w = synth.small_workload(dims, seed)
    pos = w.positions()
    say(f"case tb_overlap N={w.n_orb}")
    S = ctx.tb_overlap(synth.NONORTH_MODEL, to_dev(pos)).cpu().numpy()
    ref = nonorth.overlap(pos, synth.NONORTH_MODEL)
    assert np.abs(S - ref).max() < 1e-14
    assert np.array_equal(S, S.T)


def test_nonorth_rejects_indefinite_overlap(ctx):
    import paper_1203_6836_amd as p
    w, H, S = system((3, 3, 3), 4)
    S = S.copy()
    S[0, 0] = -1.0                      # not positive definite
    st, _ = ctx.sp2_density_matrix_status(to_dev(H), w.n_occ)  # context still usable afterwards
    assert st == p.SP2_OK
    with pytest.raises(p.Sp2Error) as ei:
        ctx.sp2_density_matrix_nonorth(to_dev(H), to_dev(S), w.n_occ, p.options("fp64"))
    assert ei.value.status in (p.SP2_ENOCONV, p.SP2_EINVAL)


def test_nonorth_full_size_timing(ctx):
    """N = 8192 (the benchmark's lattice with the overlap model), int8: the
    transforms' cost beside the SP2 solve."""
    import torch
    import paper_1203_6836_amd as p
    w = synth.MIXED
    m = synth.NONORTH_MODEL
    xyz = to_dev(w.positions())
    H = ctx.tb_hamiltonian(m, xyz)
    S = ctx.tb_overlap(m, xyz)
    say(f"case nonorth int8x N={w.n_orb} timing (H and S built on the GPU)")
    ctx.sp2_density_matrix_nonorth(H, S, w.n_occ, p.options("int8x"))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    D, st, its = ctx.sp2_density_matrix_nonorth(H, S, w.n_occ, p.options("int8x"))
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    SD = S @ D
    tr = float(torch.trace(SD)) - w.n_occ
    idem = float(torch.linalg.norm(D @ SD - D)) / w.n_orb ** 0.5
    say(f"  {ms:.0f} ms total, SP2 {st['ms']:.0f} ms ({st['iterations']} products), factor steps {its}; "
        f"Tr[DS] - n_occ {tr:+.1e}, ||D S D - D||/sqrtN {idem:.1e}")
    assert abs(tr) < 1e-5 and idem < 1e-5


def test_nonorth_hamiltonian_and_forces_match_oracle(ctx):
    """The non-orthogonal H[n] and the forces at constant n (orthogonal terms with
    the overlap charges plus the overlap term) on the 3 x 3 x 2 cluster of the
    MD model with overlap, against the oracle (whose forces are pinned by finite
    differences of U)."""
    import paper_1203_6836_amd as p
    m = synth.MD_MODEL.with_(overlap_s0=0.05)
    pos = synth.lattice_positions((3, 3, 2), seed=4)
    nat = len(pos)
    nocc = 2 * nat
    n = np.random.default_rng(7).normal(0.0, 0.1, nat)
    say("case nonorth H[n], forces 3x3x2")
    xyz, nd = to_dev(pos), to_dev(n)
    S = ctx.tb_overlap(m, xyz)
    H = ctx.tb_hamiltonian_nonorth(m, xyz, S, nd)
    S_o = nonorth.overlap(pos, m)
    H_o = nonorth.hamiltonian(pos, n, m, S_o)
    assert np.abs(H.cpu().numpy() - H_o).max() < 1e-13
    D, st, _ = ctx.sp2_density_matrix_nonorth(H, S, nocc, p.options("fp64"))
    q = ctx.sp2_mulliken_overlap(D, S, nat)
    F, U = ctx.tb_forces_nonorth(m, xyz, D, H, q, nd)
    rho_o, _, _, r = nonorth.density_matrix(H_o, S_o, nocc)
    F_o = nonorth.forces(pos, n, rho_o, m, S_o)
    U_o = nonorth.potential_energy(pos, n, rho_o, m, S_o)
    dF = float(np.abs(F.cpu().numpy() - F_o).max())
    say(f"  SP2 iterations gpu={st['iterations']} oracle={r.iterations}; max|dF| {dF:.1e} "
        f"(max|F| {np.abs(F_o).max():.1f}), dU {abs(U - U_o):.1e}")
    assert dF < 1e-8
    assert U == pytest.approx(U_o, abs=1e-8)


def test_nonorth_xlbomd_trajectory_matches_oracle(ctx):
    """XL-BOMD in the non-orthogonal basis (overlap, H[n], density matrix
    through the Loewdin factor, overlap charges and forces every step): 20
    steps of the 2 x 2 x 2 cluster against the oracle integrator."""
    import paper_1203_6836_amd as p
    from oracle import xlbomd as oxl
    say("case nonorth xlbomd 2x2x2 20 steps")
    m = synth.MD_MODEL.with_(overlap_s0=0.05)
    pos = synth.lattice_positions((2, 2, 2), seed=21)
    nat, nocc = len(pos), 2 * len(pos)
    vel = synth.maxwell_velocities(nat, 300.0, m.mass, seed=5)
    qs, _ = oxl.scf(pos, m, nocc, beta=0.3, tol=1e-12, solver="jacobi")
    opts = oxl.XLOptions(solver="sp2")
    ost, olog = oxl.run(oxl.init_state(pos, vel, m, nocc, opts, qs), m, nocc, opts, 20)
    md = ctx.xlbomd_create(m, pos, vel, qs, dt_fs=opts.dt_fs, kappa=opts.kappa, alpha=opts.alpha,
                           c=opts.c, sp2_opts=p.options("fp64"))
    glog = md.xlbomd_run(20)
    xyz, v, q, n = md.xlbomd_get()
    md.close()
    dx = float(np.abs(xyz - ost.pos).max())
    de = float(np.abs(np.array([r["etot"] for r in glog]) - np.array([r["etot"] for r in olog])).max())
    say(f"  max|dx| {dx:.1e} A, max|dE_tot| {de:.1e} eV")
    np.testing.assert_allclose(xyz, ost.pos, atol=1e-9)
    np.testing.assert_allclose(v, ost.vel, atol=1e-9)
    np.testing.assert_allclose(n, ost.hist[0], atol=1e-9)
    assert de < 1e-7


@pytest.mark.parametrize("dims,seed,kT", [((3, 3, 3), 2, 0.5), ((4, 4, 4), 7, 0.25)])
def test_nonorth_fermi_operator_matches_oracle(ctx, dims, seed, kT):
    """Finite electronic temperature in the non-orthogonal basis: D = Z f(H_perp)
    Z^T at the canonical mu, the energy-weighted W = Z f(H_perp) H_perp Z^T and
    the entropy, against the oracle's definition (generalized eigenpairs);
    the recursion's error bound as for the orthogonal Fermi operator."""
    from oracle import fermi
    w, H, S = system(dims, seed)
    say(f"case nonorth fermi N={w.n_orb} kT={kT}")
    rho, W, mu_o, f = nonorth.fermi_density_matrix(H, S, w.n_occ, kT)
    D, Wg, mu, ent, passes = ctx.sp2_fermi_density_matrix_nonorth(to_dev(H), to_dev(S), w.n_occ, kT, 16, tol=1e-9)
    D, Wg = D.cpu().numpy(), Wg.cpu().numpy()
    eD, eW = float(np.abs(D - rho).max()), float(np.abs(Wg - W).max())
    ent_o = fermi.entropy(f)
    say(f"  passes {passes}, mu {mu:.10f} (oracle {mu_o:.10f}), max|D - rho| {eD:.1e}, max|W - W_o| {eW:.1e}, "
        f"S/kB {ent:.8f} (oracle {ent_o:.8f}), Tr[D S] - n_occ {np.trace(D @ S) - w.n_occ:+.1e}")
    assert abs(mu - mu_o) < 1e-8
    assert eD < 1e-8 and eW < 1e-7
    assert abs(np.trace(D @ S) - w.n_occ) < 1e-8
    assert abs(ent - ent_o) < 1e-8 * max(1.0, abs(ent_o))


def test_nonorth_finite_temperature_xlbomd_matches_oracle(ctx):
    """XL-BOMD at kT = 0.5 eV in the non-orthogonal basis (overlap, H[n], the
    Fermi operator of H_perp, its entropy in the free energy, the free-energy
    forces with the energy-weighted W): 20 steps of the 2 x 2 x 2 cluster from
    self-consistent finite-T charges against the oracle integrator."""
    import paper_1203_6836_amd as p
    from oracle import xlbomd as oxl
    say("case nonorth fermi xlbomd 2x2x2 20 steps kT=0.5")
    m = synth.MD_MODEL.with_(overlap_s0=0.05)
    pos = synth.lattice_positions((2, 2, 2), seed=21)
    nat, nocc = len(pos), 2 * len(pos)
    vel = synth.maxwell_velocities(nat, 300.0, m.mass, seed=5)
    n0 = np.zeros(nat)
    for _ in range(2000):   # finite-T SCF by linear mixing
        q = oxl.evaluate(pos, n0, m, nocc, want_forces=False, kT=0.5)["q"]
        if np.abs(q - n0).max() < 1e-11:
            break
        n0 = n0 + 0.1 * (q - n0)
    assert np.abs(q - n0).max() < 1e-11
    opts = oxl.XLOptions(kT=0.5, kappa=p.KAPPA_FINITE_T)
    ost, olog = oxl.run(oxl.init_state(pos, vel, m, nocc, opts, n0), m, nocc, opts, 20)
    md = ctx.xlbomd_create(m, pos, vel, n0, dt_fs=opts.dt_fs, kappa=opts.kappa, alpha=opts.alpha,
                           c=opts.c, sp2_opts=p.options("fp64"), kT=0.5, fermi_steps=16)
    glog = md.xlbomd_run(20)
    xyz, v, q, n = md.xlbomd_get()
    md.close()
    eg = np.array([r["etot"] for r in glog])
    eo = np.array([r["etot"] for r in olog])
    say(f"  max|dx| {np.abs(xyz - ost.pos).max():.1e} A, max|dE_tot| {np.abs(eg - eo).max():.1e} eV, "
        f"E_tot spread {np.ptp(eo) / nat:.1e} eV/atom")
    np.testing.assert_allclose(xyz, ost.pos, atol=1e-9)
    np.testing.assert_allclose(v, ost.vel, atol=1e-9)
    np.testing.assert_allclose(n, ost.hist[0], atol=2e-8)
    assert np.abs(eg - eo).max() < 1e-7


def quench(md, nat, max_steps=1500, ftol=1e-6):
    """Relax by quenched MD (velocities zeroed whenever F . v < 0; checkpoint
    layout: 40-byte header, then xyz, vel, F)."""
    import paper_1203_6836_amd as p
    hdr, b3 = p.XL_CHECKPOINT_HEADER, 3 * nat * 8
    fmax = np.inf
    for _ in range(max_steps):
        md.xlbomd_run(1)
        ck = bytearray(md.xlbomd_get_state())
        v = np.frombuffer(bytes(ck[hdr + b3:hdr + 2 * b3]), dtype=np.float64)
        F = np.frombuffer(bytes(ck[hdr + 2 * b3:hdr + 3 * b3]), dtype=np.float64)
        fmax = float(np.abs(F).max())
        if fmax < ftol:
            break
        if float(np.dot(F, v)) < 0.0:
            ck[hdr + b3:hdr + 2 * b3] = bytes(b3)
            md.xlbomd_set_state(bytes(ck))
    return fmax, np.frombuffer(bytes(ck[hdr:hdr + b3]), dtype=np.float64).reshape(nat, 3).copy()


def test_nonorth_xlbomd_energy_conservation(ctx):
    """1000 steps of 0.25 fs at 300 K in the non-orthogonal basis: the 8-atom
    cluster relaxed by quenched MD in that basis, then NVE from its SCF
    charges.  Bars: sigma of E_tot about its linear fit <= 1e-4 eV/atom and
    drift <= 2 sigma (the orthogonal run's bars), and sigma within a factor 2
    of the orthogonal model's on the same relaxed start.  (From the unrelaxed
    jittered cluster both bases fluctuate by ~6e-3 eV/atom.)"""
    import paper_1203_6836_amd as p
    from oracle import xlbomd as oxl
    say("case nonorth xlbomd 2x2x2: quench, then 1000 steps (and the orthogonal model alike)")
    pos = synth.lattice_positions((2, 2, 2), seed=21)
    nat = len(pos)
    sig = {}
    for s0 in (0.05, 0.0):
        m = synth.MD_MODEL.with_(overlap_s0=s0)
        md = ctx.xlbomd_create(m, pos, np.zeros((nat, 3)), synth.checkerboard_charges((2, 2, 2)),
                               sp2_opts=p.options("fp64"), scf_beta=0.3, scf_tol=1e-10, scf_max_iter=300)
        fmax, relaxed = quench(md, nat)
        md.close()
        assert fmax < 1e-6
        vel = synth.maxwell_velocities(nat, 300.0, m.mass, seed=5)
        qs, _ = oxl.scf(relaxed, m, 2 * nat, beta=0.3, tol=1e-12, solver="jacobi")
        md = ctx.xlbomd_create(m, relaxed, vel, qs, sp2_opts=p.options("fp64"))
        log = []
        while len(log) < 1000:
            log += md.xlbomd_run(200)
        md.close()
        et = np.array([r["etot"] for r in log])
        t = np.arange(len(log))
        fit = np.polyfit(t, et, 1)
        sigma = float((et - np.polyval(fit, t)).std())
        drift = abs(fit[0]) * len(log)
        say(f"  overlap_s0 {s0}: quench max|F| {fmax:.1e}; sigma {sigma:.2e} eV ({sigma / nat:.1e}/atom), "
            f"drift {drift:.1e} eV")
        assert sigma / nat <= 1e-4
        assert drift <= 2.0 * sigma
        sig[s0] = sigma
    assert sig[0.05] <= 2.0 * sig[0.0]


def test_nonorth_thresholded_gapped_wire_vs_oracle(ctx):
    """The SP2 of H_perp with the elementwise threshold (tau = 1e-5, int8 and
    FP64 products) on the gapped 4 x 4 x 16 wire with an overlap, against the
    oracle's thresholded non-orthogonal solve: FP64 step by step, int8 within
    the mixed-precision tolerance 1e-6 per sqrt(N) (measured 8.6e-11; the
    threshold itself moves rho by 1.9e-4)."""
    import paper_1203_6836_amd as p
    m = synth.GAPPED_MODEL.with_(overlap_s0=0.05)
    w = synth.gapped_workload(16)
    pos = w.positions()
    say(f"case nonorth tau=1e-5 element, gapped wire N={w.n_orb}")
    H = otb.hamiltonian0(pos, m)
    S = nonorth.overlap(pos, m)
    # N = 1024: the Loewdin factor from the library eigensolver
    ref, _, _, r = nonorth.density_matrix(H, S, w.n_occ, solver="lapack", tau=1e-5, threshold="element")
    dense, _, _, _ = nonorth.density_matrix(H, S, w.n_occ, solver="lapack")
    rn = np.sqrt(w.n_orb)
    err_thr = np.linalg.norm(ref - dense) / rn
    Hd, Sd = to_dev(H), to_dev(S)
    D64, s64, _ = ctx.sp2_density_matrix_nonorth(Hd, Sd, w.n_occ, p.options("fp64", tau=1e-5, threshold=1))
    D8, s8, _ = ctx.sp2_density_matrix_nonorth(Hd, Sd, w.n_occ, p.options("int8x", tau=1e-5, threshold=1))
    e64 = np.linalg.norm(D64.cpu().numpy() - ref) / rn
    e8 = np.linalg.norm(D8.cpu().numpy() - ref) / rn
    say(f"  iters oracle={r.iterations} fp64={s64['iterations']} int8={s8['iterations']}; err fp64 {e64:.1e}, "
        f"int8 {e8:.1e}, threshold's own {err_thr:.1e}, fill min {s8['fill_min']:.3f}")
    assert s64["iterations"] == r.iterations
    assert e64 <= 1e-9
    assert e8 <= 1e-6

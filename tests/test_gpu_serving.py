"""Continuous-batching server: results alone == in a mix, parity with the oracle, admission."""
import sys
import threading
import time

import numpy as np
import pytest

import synth
from oracle import observables, sp2 as osp2, tb as otb

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


def request_H(n_atoms, seed):
    pos = synth.lattice_positions(synth.cube_dims_for(n_atoms), seed=seed, n_atoms=n_atoms)
    return otb.hamiltonian(pos, None, synth.STATIC_MODEL)


@pytest.mark.parametrize("recipe", [{}, {"slices": 4, "levels": 5}])
def test_server_alone_equals_mix_and_direct(ctx, recipe):
    """A request served alone and in a mix gives bitwise the same D and q, the
    same as the direct int8 solve with the same digit recipe (five planes;
    four planes with five levels), and every result is within the
    mixed-precision tolerance of the oracle."""
    import torch
    import paper_1203_6836_amd as p
    say(f"case serving alone vs mix {recipe}")
    probe = request_H(40, 1000)           # N = 160 (ragged: ld = 256)
    others = [request_H(n, 2000 + k) for k, n in enumerate([32, 150, 77, 300, 64, 129])]
    srv = p.Server(ctx, max_slots=8, **recipe)
    t = srv.sp2_server_submit(probe, 80)
    D_alone, q_alone, st_alone = srv.sp2_server_wait(t, probe.shape[0])
    # in a mix: submit others first, the probe in the middle, more after
    tk = [srv.sp2_server_submit(H, H.shape[0] // 2) for H in others[:3]]
    tp = srv.sp2_server_submit(probe, 80)
    tk += [srv.sp2_server_submit(H, H.shape[0] // 2) for H in others[3:]]
    D_mix, q_mix, st_mix = srv.sp2_server_wait(tp, probe.shape[0])
    outs = [srv.sp2_server_wait(x, H.shape[0]) for x, H in zip(tk, others)]
    rep = srv.sp2_server_report()
    srv.close()
    say(f"  iters {st_alone['iterations']} / {st_mix['iterations']}; report {rep}")
    assert np.array_equal(D_alone, D_mix) and np.array_equal(q_alone, q_mix)
    # the same as the direct (non-served) int8 solve
    D_direct, _ = ctx.sp2_density_matrix(torch.from_numpy(probe).cuda(), 80, p.options("int8x", **recipe))
    assert np.array_equal(D_alone, D_direct.cpu().numpy())
    # every result in the mix within the tolerance of the oracle
    for (D, q, st), H in zip(outs, others):
        ref = osp2.sp2(H, H.shape[0] // 2)
        err = np.linalg.norm(D - ref.D) / np.sqrt(H.shape[0])
        dq = np.max(np.abs(q - observables.mulliken(ref.D)))
        assert err <= 1e-6 and dq <= 1e-6, (H.shape[0], err, dq)
    assert rep["p50_ms"] > 0 and rep["p99_ms"] >= rep["p50_ms"]


def test_server_levels_are_validated(ctx):
    import paper_1203_6836_amd as p
    with pytest.raises(p.Sp2Error):
        p.Server(ctx, slices=6, levels=7)
    with pytest.raises(p.Sp2Error):
        p.Server(ctx, slices=4, levels=3)


def test_server_admission_by_footprint(ctx):
    import paper_1203_6836_amd as p
    say("case serving admission with a small arena")
    Hs = [request_H(128, 3000 + k) for k in range(3)]     # N = 512, ~10 MB each
    srv = p.Server(ctx, hbm_budget_bytes=24 << 20, max_slots=4)   # room for two at a time
    big = request_H(400, 9)                                        # N = 1600: never fits
    with pytest.raises(p.Sp2Error) as ei:
        srv.sp2_server_submit(big, 800)
    assert ei.value.status == p.SP2_EBUDGET
    tks = [srv.sp2_server_submit(H, 256) for H in Hs]
    res = [srv.sp2_server_wait(t, 512, timeout_s=60.0) for t in tks]
    srv.close()
    for (D, q, st), H in zip(res, Hs):
        ref = osp2.sp2(H, 256)
        assert np.linalg.norm(D - ref.D) / np.sqrt(512) <= 1e-6


def test_server_poisson_stream(ctx):
    import paper_1203_6836_amd as p
    say("case serving poisson stream")
    reqs = synth.request_stream(n_requests=24, rate_per_s=200.0, max_atoms=256)
    Hs = [otb.hamiltonian(r.positions(), None, synth.STATIC_MODEL) for r in reqs]
    srv = p.Server(ctx)
    tickets = [None] * len(reqs)

    def submitter():
        t0 = time.perf_counter()
        for k, r in enumerate(reqs):
            dt = r.arrival_s - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            tickets[k] = srv.sp2_server_submit(Hs[k], 2 * r.n_atoms)

    th = threading.Thread(target=submitter)
    th.start()
    th.join()
    res = [srv.sp2_server_wait(t, 4 * r.n_atoms, want_D=False) for t, r in zip(tickets, reqs)]
    rep = srv.sp2_server_report()
    srv.close()
    say(f"  {rep}")
    assert all(st["status"] in ("converged", "stalled") for _, _, st in res)
    assert rep["solves_per_s"] > 0


def test_server_reports_gap_and_invalid_h(ctx):
    import paper_1203_6836_amd as p
    say("case serving: degenerate and invalid H next to a good one")
    good = request_H(40, 1000)
    degenerate = np.diag([-1.0, 0.0, 0.0, 1.0])
    asym = good.copy()
    asym[3, 100] += 1e-6
    srv = p.Server(ctx, max_slots=4)
    tg = srv.sp2_server_submit(good, 80)
    td = srv.sp2_server_submit(degenerate, 2)
    ta = srv.sp2_server_submit(asym, 80)
    D, q, st = srv.sp2_server_wait(tg, good.shape[0])
    for t, N, want in ((td, 4, p.SP2_EGAP), (ta, good.shape[0], p.SP2_EINVAL)):
        with pytest.raises(p.Sp2Error) as ei:
            srv.sp2_server_wait(t, N)
        assert ei.value.status == want
    srv.close()
    ref = osp2.sp2(good, 80)
    assert np.linalg.norm(D - ref.D) / np.sqrt(good.shape[0]) <= 1e-6


def test_server_largest_requests_against_oracle(ctx):
    """Requests at the top of the served size range (512 atoms, N = 2048, and
    a ragged 500-atom N = 2000) in a mix with small ones: each equals its
    solve alone, bitwise, and the oracle within 1e-6 (D per sqrt(N) and
    charges)."""
    import paper_1203_6836_amd as p
    say("case serving N=2048 and N=2000 in a mix")
    big = [request_H(512, 4000), request_H(500, 4001)]
    small = [request_H(n, 4100 + k) for k, n in enumerate([32, 200, 96, 333])]
    srv = p.Server(ctx, max_slots=8)
    alone = []
    for H in big:
        t = srv.sp2_server_submit(H, H.shape[0] // 2)
        alone.append(srv.sp2_server_wait(t, H.shape[0]))
    tk = [srv.sp2_server_submit(small[0], small[0].shape[0] // 2)]
    tb = [srv.sp2_server_submit(H, H.shape[0] // 2) for H in big]
    tk += [srv.sp2_server_submit(H, H.shape[0] // 2) for H in small[1:]]
    mixed = [srv.sp2_server_wait(t, H.shape[0]) for t, H in zip(tb, big)]
    for t, H in zip(tk, small):
        srv.sp2_server_wait(t, H.shape[0], want_D=False)
    srv.close()
    for (Da, qa, sa), (Dm, qm, sm), H in zip(alone, mixed, big):
        N = H.shape[0]
        ref = osp2.sp2(H, N // 2)
        err = np.linalg.norm(Dm - ref.D) / np.sqrt(N)
        dq = np.max(np.abs(qm - observables.mulliken(ref.D)))
        say(f"  N={N}: products {sm['iterations']} (oracle {ref.iterations}), err/sqrtN {err:.2e}, max|dq| {dq:.2e}")
        assert np.array_equal(Da, Dm) and np.array_equal(qa, qm)
        assert err <= 1e-6 and dq <= 1e-6

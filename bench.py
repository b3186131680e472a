"""Benchmark: SP2 density-matrix solves at N = 8192 on one MI355X.

One step = one whole solve of the 2048-atom (8 x 16 x 16 lattice) synthetic
tight-binding Hamiltonian, N = 8192 orbitals, n_occ = 4096: Gershgorin bounds,
X_0, every SP2 product with its fused update, the control steps, the copy-out
of D, then Mulliken charges and the band energy.  H is built on the GPU
(tb_hamiltonian) and resident in HBM before the timed region.

Reported (one JSON line): useful SP2 TFLOP/s (2 N^3 per product, the
GEMM-equivalent count) and solves/s of the reduced-precision path, the plain
FP64 GPU path beside it, the error of D against the FP64 path and against the
oracle's stored FP64 solve, a roofline record of the dominant kernel measured
with HIP events inside the timed region (2 N^3 per product over the kernel's
mean launch time; what the matrix cores issue is a separate field), and the
CPU oracle timed on a bounded sample (all host cores and one core).  Beside
it: the 256-orbital FP64 solve, the 1024-atom XL-BOMD run (ms per step,
total-energy statistics, the first steps against the oracle), the
16384-orbital block-thresholded solve (fill per update, errors against dense
FP64 and the oracle), the serving stream, the gapped-wire threshold scaling,
the non-orthogonal solve and the finite-temperature Fermi operator.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision int8x|fp64|bf16x2]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# digit recipe of every int8 solve of the benchmark (--slices, --levels)
INT8_RECIPE = {"slices": 4, "levels": 5}
PEAK = {"fp64": 78.6, "int8x": 5000.0, "bf16x2": 2500.0, "fp32": 157.3}   # TFLOP/s (TOP/s for int8), dense
PEAK_HBM_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


# Kernel sources whose text fixes each product kernel's memory traffic.
KERNEL_SOURCES = {
    "k_gemm_int8x": ["int8x.hip", "split_internal.h", "sp2_internal.h"],
    "k_gemm_f64": ["sp2_dense.hip", "sp2_internal.h"],
    "k_gemm_f32": ["gemm_f32.hip", "f32_internal.h", "sp2_internal.h"],
}


def kernel_source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1203_6836_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(kernel: str):
    """HBM bytes per launch of `kernel` at N = 8192 from its committed PMC summary
    (FETCH_SIZE + WRITE_SIZE, calibrated), or None when the summary is missing or
    the kernel's sources have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_counters_mixed_n8192.md")
    try:
        fields = {}
        with open(path) as f:
            for line in f:
                k, sep, v = line.strip().partition(": ")
                if sep:
                    fields[k] = v.strip()
        if fields.get("source_sha256") != kernel_source_hash(kernel):
            return None
        return int(fields["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(H_np, n_occ, H0_np, n_occ0, n_products=6):
    """The oracle as it stands, on the host: its SP2 loop (numpy/OpenBLAS FP64
    products) on a bounded sample of the benchmarked solve, n_products products
    on all host cores and one product on one core, and the whole small FP64
    solve (N = 256) on all cores and on one core.  Returns (record, D of the
    small solve)."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import sp2 as osp2
    cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()])
    N = H_np.shape[0]
    t0 = time.perf_counter()
    osp2.sp2(H_np, n_occ, max_iter=n_products)
    dt = time.perf_counter() - t0
    with threadpool_limits(limits=1):
        t1 = time.perf_counter()
        osp2.sp2(H_np, n_occ, max_iter=1)
        dt1 = time.perf_counter() - t1
    small = []
    for lim in (None, 1):
        with threadpool_limits(limits=lim):
            t2 = time.perf_counter()
            r0 = osp2.sp2(H0_np, n_occ0, tol=1e-10)
            small.append((time.perf_counter() - t2) * 1e3)
    N0 = H0_np.shape[0]
    rec = {"value": round(2.0 * N ** 3 * n_products / dt / 1e12, 4), "unit": "TFLOP/s",
           "cores": int(cores), "kind": "oracle",
           "sample": f"{n_products} SP2 products (X^2 via numpy/OpenBLAS FP64) of the same N={N} "
                     f"Hamiltonian, {dt:.1f} s, on {cpu_model()} ({os.cpu_count()} logical CPUs "
                     f"visible); GEMM-equivalent 2N^3 flops per product",
           "single_core": {"value": round(2.0 * N ** 3 / dt1 / 1e12, 4), "unit": "TFLOP/s", "cores": 1,
                           "sample": f"1 SP2 product of the same N={N} Hamiltonian, {dt1:.1f} s"},
           "fp64_n256_full_solve": {"ms_all_cores": round(small[0], 2), "ms_one_core": round(small[1], 2),
                                    "products": r0.iterations, "n": N0, "status": r0.status}}
    return rec, r0.D


def golden(name):
    """Stored oracle results of a full-size solve (written by
    tests/golden/make_oracle_golden.py), or None."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", name)
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def against_golden(D, g, n_atoms):
    """Error of a device D against the oracle's stored solve: ||D - D_ref||_F /
    sqrt(N) estimated from the probe vectors, charges from the diagonal (all
    atoms), and the largest deviation over the sampled 32 x 32 blocks."""
    import numpy as np
    import torch

    import synth
    N = D.shape[0]
    V = torch.from_numpy(synth.probe_vectors(N)).to(D.device)
    E = (D @ V).cpu().numpy() - g["DV"]
    est = float(np.linalg.norm(E) / np.sqrt(E.shape[1]) / np.sqrt(N))
    dd = torch.diagonal(D).cpu().numpy() - g["diag"]
    dq = float(np.max(np.abs(2.0 * dd.reshape(n_atoms, -1).sum(axis=1))))
    blk = 0.0
    for a, b, ref in zip(g["block_i"], g["block_j"], g["blocks"]):
        blk = max(blk, float(np.max(np.abs(D[32 * a:32 * a + 32, 32 * b:32 * b + 32].cpu().numpy() - ref))))
    return {"err_per_sqrtN_est": est, "max_dq": dq, "max_block_dev": blk}


def fp64_small(ctx, reps=20):
    """The 64-atom (4 x 4 x 4) FP64 solve, N = 256, n_occ = 128, tolerance 1e-10:
    milliseconds per solve (median of reps, launch-latency bound), products and
    the residuals of D (idempotency, trace, commutator with H)."""
    import numpy as np
    import torch

    import paper_1203_6836_amd as p
    import synth

    w = synth.SMALL
    H = ctx.tb_hamiltonian(synth.STATIC_MODEL, torch.from_numpy(w.positions()).cuda())
    D = torch.empty_like(H)
    opt = p.options("fp64")
    ctx.sp2_density_matrix(H, w.n_occ, opt, D_out=D)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = ctx.sp2_density_matrix(H, w.n_occ, opt, D_out=D)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    out = {"workload": "fp64_n256: 64-atom 4x4x4 lattice, N=256, n_occ=128, tol 1e-10",
           "ms_per_solve": round(float(np.median(ts)), 3), "products": st["iterations"],
           "idempotency": float(torch.linalg.norm(D @ D - D)), "trace_err": float(torch.trace(D)) - w.n_occ,
           "commutator": float(torch.linalg.norm(H @ D - D @ H))}
    log(f"  fp64_n256: {out}")
    return out, H, D


def energy_stats(et, dt_fs, n_atoms):
    """Span, fluctuation about the linear fit and drift of a total-energy series (per atom)."""
    import numpy as np
    t = np.arange(len(et)) * dt_fs
    a, b = np.polyfit(t, et, 1)
    sig = float(np.std(et - (a * t + b)))
    return {"etot_span_ev_per_atom": float(np.ptp(et)) / n_atoms, "sigma_ev_per_atom": sig / n_atoms,
            "drift_ev_per_atom": float(abs(a) * t[-1]) / n_atoms}


def xlbomd_c1(ctx, steps=200, quench_steps=400):
    """The 1024-atom XL-BOMD workload (8 x 8 x 16 lattice, 300 K, dt = 0.25 fs,
    K = 5, one SP2 solve per step, no SCF during the run): ms per MD step with
    FP64 and int8 products from the self-consistent start, the total-energy
    record of the literal jittered start (which relaxes and heats), the same
    statistics after a quenched relaxation, and the first ten steps against
    the oracle's stored trajectory."""
    import numpy as np

    import paper_1203_6836_amd as p
    import synth

    w = synth.XLBOMD
    m = synth.MD_MODEL
    pos = w.positions()
    vel = synth.maxwell_velocities(w.n_atoms, 300.0, m.mass, seed=synth.XLBOMD_VEL_SEED)
    guess = synth.checkerboard_charges(w.dims)
    out = {"workload": "xlbomd_n4096: 1024-atom 8x8x16 lattice, N=4096, 300 K, dt 0.25 fs, K=5",
           "steps": steps}
    for prec in ("fp64", "int8x"):
        log(f"xlbomd N=4096: {steps} steps, {prec}")
        recipe = INT8_RECIPE if prec == "int8x" else {}
        md = ctx.xlbomd_create(m, pos, vel, guess, sp2_opts=p.options(prec, **recipe), scf_beta=1.0,
                               scf_tol=1e-9, scf_max_iter=100)
        it, _ = md.xlbomd_info()
        t0 = time.perf_counter()
        rec = md.xlbomd_run(steps)
        ms = (time.perf_counter() - t0) * 1e3 / steps
        md.close()
        et = np.array([r["etot"] for r in rec])
        ek = np.array([r["ekin"] for r in rec])
        row = {"ms_per_step": round(ms, 3), "scf_iterations": it,
               "sp2_products_per_step": round(float(np.mean([r["sp2_iterations"] for r in rec])), 2),
               "max_q_minus_n": max(r["max_q_minus_n"] for r in rec),
               "ekin_first_ev": float(ek[0]), "ekin_max_ev": float(ek.max())}
        row.update(energy_stats(et, 0.25, w.n_atoms))
        row.update(recipe)
        out[prec] = row
        log(f"  {row}")
    # conservation from a relaxed start: quenched MD (velocities zeroed
    # whenever F . v < 0), then NVE at 300 K
    log(f"xlbomd N=4096: quench ({quench_steps} steps), then {steps} NVE steps")
    md = ctx.xlbomd_create(m, pos, np.zeros_like(vel), guess, sp2_opts=p.options("fp64"), scf_beta=1.0,
                           scf_tol=1e-9, scf_max_iter=100)
    fmax, relaxed = quench(md, w.n_atoms, quench_steps)
    md.close()
    md = ctx.xlbomd_create(m, relaxed, vel, guess, sp2_opts=p.options("fp64"), scf_beta=1.0, scf_tol=1e-9,
                           scf_max_iter=100)
    rec = md.xlbomd_run(steps)
    md.close()
    q = {"quench_steps": quench_steps, "max_force_after_quench": fmax}
    q.update(energy_stats(np.array([r["etot"] for r in rec]), 0.25, w.n_atoms))
    out["quenched_start"] = q
    log(f"  {q}")
    g = golden("c1_xlbomd_n4096.npz")
    if g is not None:
        md = ctx.xlbomd_create(m, pos, vel, g["scf_q"], sp2_opts=p.options("fp64"), scf_max_iter=0)
        rec = md.xlbomd_run(len(g["etot"]))
        xyz, v, qq, n = md.xlbomd_get()
        md.close()
        out["vs_oracle_10_steps"] = {
            "max_pos_dev_A": float(np.max(np.abs(xyz - g["pos"]))),
            "max_vel_dev_A_per_fs": float(np.max(np.abs(v - g["vel"]))),
            "max_n_dev": float(np.max(np.abs(n - g["hist"][0]))),
            "max_etot_dev_ev": float(np.max(np.abs(np.array([r["etot"] for r in rec]) - g["etot"])))}
        log(f"  vs oracle: {out['vs_oracle_10_steps']}")
    return out


def quench(md, nat, max_steps, ftol=1e-3):
    """Relax by quenched MD: after each step the velocities are zeroed whenever
    the power F . v is negative (checkpoint layout: header, then xyz,
    vel, F).  Returns (largest force component, relaxed positions)."""
    import numpy as np
    import paper_1203_6836_amd as p
    hdr, b3 = p.XL_CHECKPOINT_HEADER, 3 * nat * 8
    fmax = float("inf")
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
    xyz = np.frombuffer(bytes(ck[hdr:hdr + b3]), dtype=np.float64).reshape(nat, 3).copy()
    return fmax, xyz


def blocksparse_c3(ctx):
    """The thresholded solve of the elongated 8 x 8 x 64 lattice (N = 16384):
    32 x 32 blocks with Frobenius norm below 1e-5 dropped after every update,
    int8 (the benchmark's digit recipe) and FP64 products: ms per solve,
    kept-block fraction after every update, error against the dense FP64
    solve of the same H on the GPU and against the oracle's stored
    thresholded solve."""
    import torch

    import paper_1203_6836_amd as p
    import synth

    w = synth.SPARSE
    H = ctx.tb_hamiltonian(synth.STATIC_MODEL, torch.from_numpy(w.positions()).cuda())
    N = w.n_orb
    log(f"block-sparse N={N}: dense FP64 reference")
    Dd = torch.empty_like(H)
    t0 = time.perf_counter()
    _, sd = ctx.sp2_density_matrix(H, w.n_occ, p.options("fp64"), D_out=Dd)
    torch.cuda.synchronize()
    out = {"workload": "blocksparse_n16384: 4096-atom 8x8x64 lattice, N=16384, 32x32 blocks, tau=1e-5",
           "dense_fp64": {"ms_per_solve": round((time.perf_counter() - t0) * 1e3, 1),
                          "products": sd["iterations"]}}
    g = golden("c3_blocksparse_n16384.npz")
    D = torch.empty_like(H)
    for prec in ("int8x", "fp64"):
        recipe = INT8_RECIPE if prec == "int8x" else {}
        opt = p.options(prec, tau=1e-5, threshold=0, **recipe)
        log(f"block-sparse N={N}: {prec}")
        ctx.sp2_density_matrix(H, w.n_occ, opt, D_out=D)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = ctx.sp2_density_matrix(H, w.n_occ, opt, D_out=D)
        torch.cuda.synchronize()
        row = {"ms_per_solve": round((time.perf_counter() - t0) * 1e3, 1), "products": st["iterations"],
               "fill_per_update": [round(f, 5) for f in st["fill_hist"][:st["iterations"] - 1]],
               "err_vs_dense_fp64_per_sqrtN": float(torch.linalg.norm(D - Dd)) / N ** 0.5}
        row.update(recipe)
        if g is not None:
            row["vs_oracle"] = against_golden(D, g, w.n_atoms)
            row["vs_oracle"]["same_products"] = int(g["iterations"]) == st["iterations"]
            nf = min(len(g["fill"]), len(st["fill_hist"]))
            row["vs_oracle"]["max_fill_dev"] = max(abs(float(a) - float(b))
                                                   for a, b in zip(g["fill"][1:nf], st["fill_hist"][:nf - 1]))
        out[prec] = row
        log(f"  {prec}: {row['ms_per_solve']} ms, {row['products']} products, "
            f"err vs dense {row['err_vs_dense_fp64_per_sqrtN']:.2e}")
    del D, Dd, H
    torch.cuda.empty_cache()
    return out


def serving(ctx, n_requests, rate):
    """Serve a Poisson stream of SP2 solves (32-512 atoms each) open loop, then the
    same stream with serial plain-FP64 solves; latency = arrival -> result in host memory."""
    import threading

    import numpy as np
    import torch

    import paper_1203_6836_amd as p
    import synth

    reqs = synth.request_stream(n_requests=n_requests, rate_per_s=rate)
    log(f"serving: building {len(reqs)} Hamiltonians on the GPU")
    Hs = []
    for r in reqs:
        xyz = torch.from_numpy(r.positions()).cuda()
        Hs.append(ctx.tb_hamiltonian(synth.STATIC_MODEL, xyz).cpu().numpy())
    torch.cuda.synchronize()

    log("serving: continuous batching (int8 digit planes)")
    srv = p.Server(ctx, **INT8_RECIPE)
    lag = [0.0] * len(reqs)
    tickets = [None] * len(reqs)

    def submitter():
        t0 = time.perf_counter()
        for k, r in enumerate(reqs):
            dt = r.arrival_s - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            lag[k] = max(0.0, time.perf_counter() - t0 - r.arrival_s) * 1e3
            tickets[k] = srv.sp2_server_submit(Hs[k], 2 * r.n_atoms)

    th = threading.Thread(target=submitter)
    th.start()
    lat = []
    iters = []
    for k, r in enumerate(reqs):          # consume results as they complete
        while tickets[k] is None:
            time.sleep(0.0005)
        _, _, st = srv.sp2_server_wait(tickets[k], r.n_orb, want_D=True)
        # arrival -> result in host memory: submitter lag + (submit -> result) from the server
        lat.append(lag[k] + st["ms"])
        iters.append(st["iterations"])
    th.join()
    span = max(r.arrival_s + l * 1e-3 for r, l in zip(reqs, lat))
    rep = srv.sp2_server_report()
    srv.close()
    flops = sum(2.0 * r.n_orb ** 3 * it for r, it in zip(reqs, iters))

    # capacity: the same requests in a closed loop, four client threads each
    # keeping `window` of them in flight (a new one is submitted as each
    # completes; several clients so that copying H in and D out on the host
    # does not limit the server), timed until drained
    window, clients = 16, 4
    log(f"serving: saturated ({clients} clients x {window} requests in flight)")
    srv = p.Server(ctx, **INT8_RECIPE)

    def client(c):
        mine = list(range(c, len(reqs), clients))
        tk = {}
        for k in mine[:window]:
            tk[k] = srv.sp2_server_submit(Hs[k], 2 * reqs[k].n_atoms)
        nxt = min(window, len(mine))
        for k in mine:
            srv.sp2_server_wait(tk.pop(k), reqs[k].n_orb, want_D=True)
            if nxt < len(mine):
                j = mine[nxt]
                tk[j] = srv.sp2_server_submit(Hs[j], 2 * reqs[j].n_atoms)
                nxt += 1

    t0 = time.perf_counter()
    ths = [threading.Thread(target=client, args=(c,)) for c in range(clients)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    sat_s = time.perf_counter() - t0
    srv.close()

    log("serving: serial FP64 baseline")
    opts = p.options("fp64")
    finish_times = [0.0] * len(reqs)

    def run_serial():
        # solve requests in arrival order, each as soon as it has arrived
        t0 = time.perf_counter()
        for k, r in enumerate(reqs):
            dt = r.arrival_s - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            H = torch.from_numpy(Hs[k]).cuda()
            D, _ = ctx.sp2_density_matrix(H, 2 * r.n_atoms, opts)
            D.cpu()
            finish_times[k] = time.perf_counter() - t0

    run_serial()
    lat64 = [(finish_times[k] - r.arrival_s) * 1e3 for k, r in enumerate(reqs)]
    span64 = max(finish_times)
    pc = lambda v, q: float(np.percentile(np.array(v), q))
    return {"workload": f"{len(reqs)} requests, 32-512 atoms (N=128-2048), Poisson {rate:g}/s",
            "p50_ms": round(pc(lat, 50), 3), "p99_ms": round(pc(lat, 99), 3),
            "solves_per_s": round(len(reqs) / span, 2),
            "useful_tflops": round(flops / span / 1e12, 3),
            "server_report": {k: round(v, 3) for k, v in rep.items()},
            "saturated": {"in_flight": window * clients, "clients": clients,
                          "solves_per_s": round(len(reqs) / sat_s, 2),
                          "useful_tflops": round(flops / sat_s / 1e12, 3)},
            "baseline_serial_fp64": {"p50_ms": round(pc(lat64, 50), 3), "p99_ms": round(pc(lat64, 99), 3),
                                     "solves_per_s": round(len(reqs) / span64, 2)}}


def thresholded_scaling(ctx, layers=(128, 256, 512, 1024), dense_max=16384):
    """Gapped 4 x 4 x L wires (5 eV gap, D decays exponentially): int8
    products with the elementwise threshold tau = 1e-5, per-solve time,
    products, kept-block fraction and the time split over the steps, against
    the dense int8 solve up to dense_max orbitals."""
    import torch

    import paper_1203_6836_amd as p
    import synth

    rows = []
    for L in layers:
        w = synth.gapped_workload(L)
        log(f"thresholded scaling: gapped wire N={w.n_orb}")
        H = ctx.tb_hamiltonian(synth.GAPPED_MODEL, torch.from_numpy(w.positions()).cuda())
        D = torch.empty_like(H)
        opt = p.options("int8x", tau=1e-5, threshold=1, **INT8_RECIPE)
        ctx.sp2_density_matrix(H, w.n_occ, opt, D_out=D)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = ctx.sp2_density_matrix(H, w.n_occ, opt, D_out=D)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        ctx.sp2_ctx_set_profiling(True)
        _, sp = ctx.sp2_density_matrix(H, w.n_occ, opt, D_out=D)
        ctx.sp2_ctx_set_profiling(False)
        row = {"n": w.n_orb, "ms_per_solve": round(ms, 2), "products": st["iterations"],
               "fill_max": round(st["fill_max"], 5), "fill_min": round(st["fill_min"], 5),
               "trace_err": float(torch.trace(D)) - w.n_occ,
               "profiled_ms": {"products": round(sum(sp["prod_ms"]), 2), "encode": round(sp["encode_ms"], 2),
                               "threshold": round(sp["post_ms"], 2)}}
        if w.n_orb <= dense_max:
            Dd = torch.empty_like(H)
            ctx.sp2_density_matrix(H, w.n_occ, p.options("int8x", **INT8_RECIPE), D_out=Dd)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, sd = ctx.sp2_density_matrix(H, w.n_occ, p.options("int8x", **INT8_RECIPE), D_out=Dd)
            torch.cuda.synchronize()
            row["dense_ms_per_solve"] = round((time.perf_counter() - t0) * 1e3, 2)
            row["dense_products"] = sd["iterations"]
            row["err_vs_dense_per_sqrtN"] = float(torch.linalg.norm(D - Dd)) / w.n_orb ** 0.5
            del Dd
        log(f"  {row}")
        rows.append(row)
        del D, H
        torch.cuda.empty_cache()
    return {"workload": "gapped sp wire 4x4xL, 2.0 A, p level +4 eV, 2 electrons per atom",
            "precision": "int8x", **INT8_RECIPE, "tau": 1e-5, "threshold": "element", "rows": rows,
            "xlbomd": thresholded_md(ctx)}


def thresholded_md(ctx, layers=(128, 256), steps=20):
    """XL-BOMD steps on the gapped wire (2048 and 4096 atoms; one SP2 solve,
    charges, forces and the Verlet updates per step), int8 products, without
    and with the elementwise threshold tau = 1e-5: milliseconds per MD step.
    The closed-shell atoms start from zero charges (no SCF), at 300 K."""
    import numpy as np

    import paper_1203_6836_amd as p
    import synth

    out = []
    for L in layers:
        w = synth.gapped_workload(L)
        m = synth.GAPPED_MD_MODEL
        xyz = w.positions()
        vel = synth.maxwell_velocities(w.n_atoms, 300.0, m.mass, seed=31)
        row = {"n_atoms": w.n_atoms, "n": w.n_orb, "steps": steps}
        for name, opt in (("tau0", p.options("int8x", **INT8_RECIPE)),
                          ("tau1e-5", p.options("int8x", tau=1e-5, threshold=1, **INT8_RECIPE))):
            log(f"thresholded MD: {w.n_atoms} atoms, {name}")
            md = ctx.xlbomd_create(m, xyz, vel, np.zeros(w.n_atoms), sp2_opts=opt, scf_max_iter=0)
            md.xlbomd_run(2)                          # warm (allocation, first solves)
            t0 = time.perf_counter()
            rec = md.xlbomd_run(steps)
            ms = (time.perf_counter() - t0) * 1e3 / steps
            md.close()
            et = [r["etot"] for r in rec]
            row[name] = {"ms_per_step": round(ms, 2),
                         "sp2_products_per_step": round(float(np.mean([r["sp2_iterations"] for r in rec])), 1),
                         "fill_min": round(min(r["fill_min"] for r in rec), 4),
                         "etot_span_ev": float(max(et) - min(et))}
        row["speedup"] = round(row["tau0"]["ms_per_step"] / row["tau1e-5"]["ms_per_step"], 2)
        log(f"  {row}")
        out.append(row)
    return out


def nonorthogonal(ctx):
    """The non-orthogonal solve on the benchmark's lattice with the overlap
    model (N = 8192, int8 SP2 of H_perp): total time, the SP2 solve's share,
    Newton-Schulz steps of the Loewdin factor, and the S-metric invariants."""
    import torch

    import paper_1203_6836_amd as p
    import synth

    w = synth.MIXED
    m = synth.NONORTH_MODEL
    xyz = torch.from_numpy(w.positions()).cuda()
    log("non-orthogonal solve: N=8192")
    H = ctx.tb_hamiltonian(m, xyz)
    S = ctx.tb_overlap(m, xyz)
    D = torch.empty_like(H)
    opt = p.options("int8x", **INT8_RECIPE)
    ctx.sp2_density_matrix_nonorth(H, S, w.n_occ, opt, D_out=D)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st, its = ctx.sp2_density_matrix_nonorth(H, S, w.n_occ, opt, D_out=D)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    # invariants without a matrix product (Tr[D S] = sum D o S for symmetric S;
    # D S D = D on two seeded probe vectors)
    V = torch.from_numpy(synth.probe_vectors(w.n_orb)).cuda()
    DV = D @ V
    E = D @ (S @ DV) - DV
    out = {"n": w.n_orb, **INT8_RECIPE, "ms_per_solve": round(ms, 1), "sp2_ms": round(st["ms"], 1),
           "sp2_products": st["iterations"], "factor_steps": its,
           "trace_DS_minus_nocc": float((D * S).sum()) - w.n_occ,
           "idempotency_DSD_probe_rel": float(torch.linalg.norm(E) / torch.linalg.norm(DV))}
    log(f"  {out}")
    return out


def finite_temperature(ctx, dims=(8, 8, 16), kT=0.5, n_steps=16):
    """The Fermi operator at kT = 0.5 eV on a 1024-atom lattice (N = 4096) by
    the recursive expansion with canonical mu: time per solve, Newton passes,
    and the rate of its symmetric FP64 products over the whole solve."""
    import torch

    import synth

    w = synth.small_workload(dims, 7)
    xyz = torch.from_numpy(w.positions()).cuda()
    H = ctx.tb_hamiltonian(synth.STATIC_MODEL, xyz)
    N = w.n_orb
    log(f"finite temperature: N={N}, kT={kT} eV, {n_steps} steps")
    D = torch.empty_like(H)
    ctx.sp2_fermi_density_matrix(H, w.n_occ, kT, n_steps, tol=1e-8, D_out=D)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, mu, passes = ctx.sp2_fermi_density_matrix(H, w.n_occ, kT, n_steps, tol=1e-8, D_out=D)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    prods = ctx.last_fermi_products
    # every product is of polynomials in H, formed as a symmetric product of
    # upper tiles: N^2 (N + 1) flops issued, 2 N^3 in GEMM-equivalent terms
    tf = prods * 2.0 * N ** 3 / (ms * 1e-3) / 1e12
    tf_issued = prods * float(N) * N * (N + 1) / (ms * 1e-3) / 1e12
    t0 = time.perf_counter()
    S, coefs = ctx.sp2_fermi_entropy(H, mu, kT)
    ms_s = (time.perf_counter() - t0) * 1e3
    out = {"n": N, "kT_eV": kT, "n_steps": n_steps, "ms_per_solve": round(ms, 1), "newton_passes": passes,
           "products": prods,
           "mu": mu, "gemm_tflops_2n3": round(tf, 1), "gemm_tflops_issued": round(tf_issued, 1),
           "gemm_issued_frac_of_fp64_peak": round(tf_issued / PEAK["fp64"], 3),
           "trace_minus_nocc": float(torch.trace(D)) - w.n_occ,
           "entropy_kB": S, "entropy_coefficients": coefs, "entropy_ms": round(ms_s, 1)}
    log(f"  {out}")
    return out


def breakdown(st):
    """Product, encode and threshold kernel time of one profiled solve."""
    return {"fp64_products": round(st["prod_ms"][0], 2), "reduced_products": round(st["prod_ms"][1], 2),
            "encode": round(st["encode_ms"], 2), "threshold": round(st["post_ms"], 2),
            "wall": round(st["ms"], 2)}


def host_memory(ctx, H, nocc, opts):
    """The same solve with H and D in pinned host memory (sp2_density_matrix_mem):
    the PCIe-inclusive time per solve beside the solve alone."""
    import numpy as np
    import torch
    log("host-memory solve (H in, D out over PCIe)")
    N = H.shape[0]
    Hh = torch.empty((N, N), dtype=torch.float64, pin_memory=True)
    Hh.copy_(H)
    Dh = torch.empty((N, N), dtype=torch.float64, pin_memory=True)
    H_np, D_np = Hh.numpy(), Dh.numpy()
    ctx.sp2_density_matrix_mem(H_np, nocc, opts, D_out=D_np)     # warm-up (stages the buffers)
    t0 = time.perf_counter()
    _, st = ctx.sp2_density_matrix_mem(H_np, nocc, opts, D_out=D_np)
    ms = (time.perf_counter() - t0) * 1e3
    ok = bool(np.isfinite(D_np).all())
    out = {"ms_per_solve": round(ms, 2), "solve_ms": round(st["ms"], 2), "copies_ms": round(ms - st["ms"], 2),
           "bytes_over_pcie": 2 * 8 * N * N, "useful_tflops": round(2.0 * N ** 3 * st["iterations"] / (ms * 1e-3) / 1e12, 2),
           "products": st["iterations"], "finite": ok}
    log(f"  {out}")
    return out


def digit_products(slices, levels):
    """int8 digit products per SP2 product: planes t, u < slices with t + u < levels."""
    return sum(1 for t in range(slices) for u in range(slices) if t + u < (levels or slices))


def five_planes(ctx, H, nocc, n_atoms, g2, idem_tol, ms64):
    """The five-plane int8 recipe (15 digit products) on the same workload:
    time per solve and error against the oracle, beside the headline recipe."""
    import torch
    import paper_1203_6836_amd as p
    log("int8x five planes (15 digit products)")
    opts = p.options("int8x", slices=5, levels=5)
    opts.idem_tol = idem_tol
    D = torch.empty_like(H)
    ctx.sp2_autotune(H.shape[0], "int8x", 5, 5)
    ctx.sp2_density_matrix(H, nocc, opts, D_out=D)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = ctx.sp2_density_matrix(H, nocc, opts, D_out=D)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    out = {"slices": 5, "levels": 5, "digit_products": 15, "ms_per_solve": round(ms, 2),
           "products": st["iterations"], "speedup_vs_fp64": round(ms64 / ms, 3),
           "vs_oracle": against_golden(D, g2, n_atoms) if g2 is not None else None}
    log(f"  {out}")
    return out


def fp32_path(ctx, H, nocc, n_atoms, g2, idem_tol, ms64):
    """The FP32 products (FP32 MFMA, FP32 accumulation and update) on the same
    workload: time per solve, the product kernel's rate against the FP32
    matrix peak, and the error against the oracle's FP64 solve."""
    import torch
    import paper_1203_6836_amd as p
    log("fp32 path")
    N = H.shape[0]
    opts = p.options("fp32")
    opts.idem_tol = idem_tol
    D = torch.empty_like(H)
    ctx.sp2_autotune(N, "fp32")
    ctx.sp2_density_matrix(H, nocc, opts, D_out=D)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = ctx.sp2_density_matrix(H, nocc, opts, D_out=D)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    ctx.sp2_ctx_set_profiling(True)
    _, stp = ctx.sp2_density_matrix(H, nocc, opts, D_out=D)
    ctx.sp2_ctx_set_profiling(False)
    kms = stp["prod_ms"][1] / max(stp["prod_count"][1], 1)
    useful = 2.0 * float(N) ** 3
    sym_flops = float(N) * N * (N + 1)
    out = {"ms_per_solve": round(ms, 2), "products": st["iterations"], "status": st["status"],
           "speedup_vs_fp64": round(ms64 / ms, 3) if ms64 else None, "kernel": "k_gemm_f32",
           "kernel_ms_avg": round(kms, 4),
           "kernel_tflops_2n3": round(useful / (kms * 1e-3) / 1e12, 2),
           "mfma_issue_tflops": round(sym_flops / (kms * 1e-3) / 1e12, 2),
           "mfma_issue_frac_of_peak": round(sym_flops / (kms * 1e-3) / 1e12 / PEAK["fp32"], 4),
           "vs_oracle": against_golden(D, g2, n_atoms) if g2 is not None else None}
    log(f"  {out}")
    return out


def bf16x2_path(ctx, H, nocc, n_atoms, g2, ms64):
    """The configured BF16 hi + lo recipe (FP32 accumulation, then three FP32
    products on the FP32 kernel) on the same workload: time per solve and its
    error against the oracle's FP64 solve (it is not expected to reach 1e-6)."""
    import torch
    import paper_1203_6836_amd as p
    log("bf16x2 path")
    N = H.shape[0]
    opts = p.options("bf16x2")
    D = torch.empty_like(H)
    ctx.sp2_autotune(N, "bf16x2")
    ctx.sp2_density_matrix(H, nocc, opts, D_out=D)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = ctx.sp2_density_matrix(H, nocc, opts, D_out=D)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    out = {"ms_per_solve": round(ms, 2), "products": st["iterations"], "fp32_tail_from": st["head_switch"],
           "status": st["status"], "speedup_vs_fp64": round(ms64 / ms, 3) if ms64 else None,
           "vs_oracle": against_golden(D, g2, n_atoms) if g2 is not None else None}
    log(f"  {out}")
    return out


def fp32_n8192(ctx):
    """The FP32 leg alone on the mixed_n8192 workload (for profiling)."""
    import torch

    import synth
    w = synth.MIXED
    H = ctx.tb_hamiltonian(synth.STATIC_MODEL, torch.from_numpy(w.positions()).cuda())
    return fp32_path(ctx, H, w.n_occ, w.n_atoms, golden("c2_mixed_n8192.npz"), 1e-10, None)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="int8x", choices=["int8x", "fp64", "bf16x2", "fp32"])
    ap.add_argument("--slices", type=int, default=4, help="int8 digit planes")
    ap.add_argument("--levels", type=int, default=5,
                    help="int8 digit-product levels kept (slices or slices + 1)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tune-table", default=None, help="write the autotuner's table to this file")
    ap.add_argument("--probe-table", default=None,
                    help="with --traffic-probe: load this autotuner table (written by --tune-table) instead of "
                         "tuning, so that counter passes on one box all run the same launch configuration")
    ap.add_argument("--idem-tol", type=float, default=1e-10,
                    help="stop tolerance on ||X^2 - X||_F for both paths of the main solve")
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--no-scaling", action="store_true",
                    help="skip the thresholded gapped-wire scaling leg")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="only run the counter-calibration kernels and one solve per precision "
                         "(for rocprofv3 --pmc passes); prints no JSON")
    ap.add_argument("--only", choices=["finite_temperature", "nonorthogonal", "xlbomd_n4096",
                                       "blocksparse_n16384", "thresholded_scaling", "fp64_n256", "fp32_n8192"],
                    help="run only this leg and print its result as one JSON line (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1203_6836_amd as p
    import synth

    INT8_RECIPE.update(slices=args.slices, levels=args.levels)
    if args.only:
        ctx = p.Context(0)
        legs = {"finite_temperature": finite_temperature, "nonorthogonal": nonorthogonal,
                "xlbomd_n4096": xlbomd_c1, "blocksparse_n16384": blocksparse_c3,
                "thresholded_scaling": thresholded_scaling,
                "fp64_n256": lambda c: fp64_small(c)[0], "fp32_n8192": fp32_n8192}
        print(json.dumps({args.only: legs[args.only](ctx)}), flush=True)
        ctx.close()
        return
    w = synth.MIXED
    N, nocc = w.n_orb, w.n_occ
    ctx = p.Context(0)
    xyz = torch.from_numpy(w.positions()).cuda()
    H = ctx.tb_hamiltonian(synth.STATIC_MODEL, xyz)
    D = torch.empty_like(H)
    torch.cuda.synchronize()

    def solve(prec, Dout):
        opts = p.options(prec, slices=args.slices, levels=args.levels) if prec == "int8x" else p.options(prec)
        opts.idem_tol = args.idem_tol
        Dout, st = ctx.sp2_density_matrix(H, nocc, opts, D_out=Dout)
        q = ctx.sp2_mulliken(Dout, w.n_atoms)
        e = ctx.sp2_band_energy(Dout, H)
        return st, q, e

    # product tile order for this size (timed on the device; not in the timed region)
    if args.traffic_probe and args.probe_table:
        ctx.sp2_tune_load(args.probe_table)
        with open(args.probe_table) as f:
            log("traffic probe: launch configuration from " + args.probe_table + ": " +
                "; ".join(l.strip() for l in f if l.strip() and not l.startswith("#")))
    else:
        tune = {"fp64": ctx.sp2_autotune(N, "fp64")}
        if args.precision != "fp64":
            tune[args.precision] = ctx.sp2_autotune(N, args.precision, args.slices, args.levels)
        if args.tune_table and "fp32" not in tune:
            # the counter passes replay the FP32 solve with the same table
            ctx.sp2_autotune(N, "fp32")
        log("autotune: " + ", ".join(f"{k} tile_group {v['tile_group']} stage_cfg {v['stage_cfg']} split_cap "
                                     f"{v['split_cap']} tile {v['tile']}" for k, v in tune.items()))
        if args.tune_table:
            ctx.sp2_tune_save(args.tune_table)

    if args.traffic_probe:
        # calibration for the HBM byte counters: kernels of known traffic
        # (1 GiB written by a fill, 1 GiB read + 1 GiB written by an
        # elementwise add and by a device-to-device copy)
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        torch.add(a, 1.0, out=b)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        for prec in ("int8x", "fp64", "fp32"):
            log(f"traffic probe: one {prec} solve at N={N}")
            solve(prec, D)
            torch.cuda.synchronize()
        log("traffic probe done")
        ctx.close()
        return

    # ---- plain FP64 GPU path (reference speed and D_fp64) ----
    log(f"fp64 path: N={N}")
    D64 = torch.empty_like(H)
    solve("fp64", D64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.fp64_steps):
        st64, q64, e64 = solve("fp64", D64)
    torch.cuda.synchronize()
    ms64 = (time.perf_counter() - t0) * 1e3 / args.fp64_steps
    tflops64 = 2.0 * N ** 3 * st64["iterations"] / (ms64 * 1e-3) / 1e12
    log(f"  fp64: {ms64:.1f} ms/solve, {st64['iterations']} products, {tflops64:.2f} TFLOP/s")
    # one more solve with the product kernel bracketed by HIP events (outside the timing above)
    ctx.sp2_ctx_set_profiling(True)
    st64p, _, _ = solve("fp64", D64)
    ctx.sp2_ctx_set_profiling(False)
    kms64 = st64p["prod_ms"][0] / max(st64p["prod_count"][0], 1)

    prec = args.precision
    log(f"{prec} path: warmup {args.warmup}, steps {args.steps}")
    for _ in range(args.warmup):
        solve(prec, D)
    ctx.sp2_ctx_set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for _ in range(args.steps):
        st, q, e = solve(prec, D)
        stats.append(st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.sp2_ctx_set_profiling(False)
    ms = dt * 1e3 / args.steps
    iters = stats[-1]["iterations"]
    tflops = 2.0 * N ** 3 * iters / (ms * 1e-3) / 1e12

    # error of D against the FP64 GPU path and against the oracle's stored
    # FP64 solve of the same Hamiltonian (tests/golden/make_oracle_golden.py)
    err = float(torch.linalg.norm(D - D64)) / N ** 0.5
    dq = float((q - q64).abs().max())
    idem = float(torch.linalg.norm(D @ D - D))
    g2 = golden("c2_mixed_n8192.npz")
    vs_oracle = None
    if g2 is not None:
        vs_oracle = {prec: against_golden(D, g2, w.n_atoms), "fp64": against_golden(D64, g2, w.n_atoms),
                     "oracle_products": int(g2["iterations"])}

    # roofline of the dominant kernel, the product kernel of this precision:
    # algorithmic work 2 N^3 flops per SP2 product (the GEMM-equivalent count
    # of the metric, one unit for every precision) over the kernel's mean
    # launch time, against the peak of the instruction's own type
    k = 0 if prec == "fp64" else 1
    cnt = sum(s["prod_count"][k] for s in stats)
    kms = sum(s["prod_ms"][k] for s in stats) / max(cnt, 1)
    useful = 2.0 * float(N) ** 3
    sym_flops = float(N) * N * (N + 1)          # distinct entries of a symmetric product
    achieved = useful / (kms * 1e-3) / 1e12
    unit = "TOP/s" if prec == "int8x" else "TFLOP/s"
    kname = {"fp64": "k_gemm_f64", "int8x": "k_gemm_int8x", "bf16x2": "k_gemm_bf16x2", "fp32": "k_gemm_f32"}[prec]
    traffic = recorded_traffic(kname) if kname in KERNEL_SOURCES else None
    if prec == "int8x" and (args.slices, args.levels) != (4, 5):
        traffic = None                      # counters are taken with 4 planes, 5 levels
    roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK[prec], "unit": unit,
            "frac": round(achieved / PEAK[prec], 4), "traffic": traffic,
            "algorithmic_unit": "2 N^3 per SP2 product (GEMM-equivalent), every precision",
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
            "kernel": kname, "kernel_ms_avg": round(kms, 4), "launches": cnt}
    # what the matrix cores actually issue: the upper tiles only (N^2 (N + 1)
    # multiply-adds x 2), times the digit-plane products of the expansion
    issue_mult = {"int8x": digit_products(args.slices, args.levels), "bf16x2": 3, "fp64": 1, "fp32": 1}[prec]
    issued = issue_mult * sym_flops / (kms * 1e-3) / 1e12
    roof["mfma_issue"] = {"ops_per_launch": issue_mult * sym_flops, "rate": round(issued, 2), "unit": unit,
                          "frac_of_peak": round(issued / PEAK[prec], 4)}
    if prec == "int8x":
        # the instruction's sustained rate on digit-range operands, measured here
        # (the power-limited clock makes it data dependent)
        log("int8 matrix-core rate probe")
        pm = ctx.sp2_int8_mfma_rate() / 1e12
        roof["mfma_issue"]["peak_measured"] = round(pm, 1)
        roof["mfma_issue"]["frac_of_measured"] = round(issued / pm, 4)

    out = {
        "metric": "SP2 TFLOP/s & solves/s (mixed vs FP64) at N=8192; p50/p99 served latency",
        "value": round(tflops, 3), "unit": "TFLOP/s (useful, 2N^3 per SP2 product)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"int8x": "i8 (int32 accumulation, f64 combine)", "fp64": "f64",
                  "bf16x2": "bf16 (f32 accumulation)", "fp32": "f32"}[prec],
        "data": "synthetic",
        "config": {"workload": "mixed_n8192: 2048-atom 8x16x16 jittered sp tight-binding lattice, "
                               "N=8192, n_occ=4096", "precision": prec,
                   "slices": args.slices if prec == "int8x" else None,
                   "levels": args.levels if prec == "int8x" else None,
                   "digit_products": digit_products(args.slices, args.levels) if prec == "int8x" else None,
                   "tile_group": tune[prec]["tile_group"], "stage_cfg": tune[prec]["stage_cfg"],
                   "split_cap": tune[prec]["split_cap"], "tile": tune[prec]["tile"]},
        "autotune": {k: {"chosen": {"tile_group": v["tile_group"], "stage_cfg": v["stage_cfg"],
                                    "split_cap": v["split_cap"], "tile": v["tile"]},
                         "ms_per_product": {"G%d/cfg%d/cap%d/tile%d" % g: round(ms, 4)
                                            for g, ms in v["ms_per_product"].items()}}
                     for k, v in tune.items()},
        "solves_per_s": round(1e3 / ms, 4),
        "products": iters,
        "fp64_path": {"ms_per_solve": round(ms64, 2), "tflops": round(tflops64, 3),
                      "products": st64["iterations"],
                      "kernel": "k_gemm_f64", "kernel_ms_avg": round(kms64, 4),
                      "kernel_tflops_2n3": round(useful / (kms64 * 1e-3) / 1e12, 2),
                      "kernel_frac_2n3": round(useful / (kms64 * 1e-3) / 1e12 / PEAK["fp64"], 4),
                      "mfma_issue_tflops": round(sym_flops / (kms64 * 1e-3) / 1e12, 2),
                      "mfma_issue_frac_of_peak": round(sym_flops / (kms64 * 1e-3) / 1e12 / PEAK["fp64"], 4)},
        "speedup_vs_fp64": round(ms64 / ms, 3),
        # HIP-event sums of one profiled solve of each path (ms per solve)
        "solve_breakdown_ms": {prec: breakdown(stats[-1]), "fp64": breakdown(st64p)},
        "idem_tol": args.idem_tol,
        "idem_last": {prec: [float(f"{e:.3g}") for e in stats[-1]["idem_hist"][-6:]],
                      "fp64": [float(f"{e:.3g}") for e in st64["idem_hist"][-6:]]},
        "err_vs_fp64_per_sqrtN": err, "max_dq_vs_fp64": dq, "idempotency": idem,
        "vs_oracle": vs_oracle,
        "roofline": roof,
    }
    if prec == "int8x" and (args.slices, args.levels) != (5, 5):
        out["int8x_five_planes"] = five_planes(ctx, H, nocc, w.n_atoms, g2, args.idem_tol, ms64)
    if prec != "fp32":
        out["fp32_path"] = fp32_path(ctx, H, nocc, w.n_atoms, g2, args.idem_tol, ms64)
    if prec != "bf16x2":
        out["bf16x2_path"] = bf16x2_path(ctx, H, nocc, w.n_atoms, g2, ms64)
    hopts = p.options(prec, slices=args.slices, levels=args.levels) if prec == "int8x" else p.options(prec)
    hopts.idem_tol = args.idem_tol
    out["host_memory"] = host_memory(ctx, H, nocc, hopts)
    if args.serve_requests > 0 and prec == "int8x":
        out["serving"] = serving(ctx, args.serve_requests, args.serve_rate)
    log("fp64_n256 solve")
    small, H0, D0 = fp64_small(ctx)
    out["fp64_n256"] = small
    if not args.no_scaling:
        del D64
        torch.cuda.empty_cache()
        out["xlbomd_n4096"] = xlbomd_c1(ctx)
        out["blocksparse_n16384"] = blocksparse_c3(ctx)
        out["thresholded_scaling"] = thresholded_scaling(ctx)
        out["nonorthogonal"] = nonorthogonal(ctx)
        out["finite_temperature"] = finite_temperature(ctx)
    if not args.no_cpu:
        log("cpu baseline (oracle sample)")
        out["cpu_baseline"], D0_ref = cpu_baseline(H.cpu().numpy(), nocc, H0.cpu().numpy(), synth.SMALL.n_occ)
        d0 = D0.cpu().numpy() - D0_ref
        small["err_vs_oracle_per_sqrtN"] = float(np.linalg.norm(d0) / np.sqrt(d0.shape[0]))
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()

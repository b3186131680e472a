"""The boundary's memory kinds and its one-call-per-context rule, on the GPU."""
import sys
import threading
import time

import numpy as np
import pytest

import synth

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


@pytest.mark.parametrize("prec", ["fp64", "int8x"])
def test_host_memory_solve_equals_device_solve(ctx, prec):
    """H and D in host memory (staged by the library) give bitwise the D of
    the device-memory call (N = 720, ragged against the 128 tiles)."""
    import torch
    import paper_1203_6836_amd as p
    say(f"case host-memory solve {prec} N=720")
    pos = synth.lattice_positions((6, 6, 5), seed=12)
    xyz = np.ascontiguousarray(pos, dtype=np.float64)
    H_host = ctx.tb_hamiltonian_mem(synth.STATIC_MODEL, xyz)
    H_dev = ctx.tb_hamiltonian(synth.STATIC_MODEL, torch.from_numpy(xyz).cuda())
    assert isinstance(H_host, np.ndarray)
    assert np.array_equal(H_host, H_dev.cpu().numpy())
    nocc = 2 * len(pos)
    D_host, st_h = ctx.sp2_density_matrix_mem(H_host, nocc, p.options(prec))
    D_dev, st_d = ctx.sp2_density_matrix(H_dev, nocc, p.options(prec))
    assert isinstance(D_host, np.ndarray)
    assert st_h["iterations"] == st_d["iterations"]
    assert np.array_equal(D_host, D_dev.cpu().numpy())
    # device kind through the same entry point
    D_dev2, _ = ctx.sp2_density_matrix_mem(H_dev, nocc, p.options(prec))
    assert torch.equal(D_dev2, D_dev)


def test_host_memory_error_leaves_output(ctx):
    """On error (here n_occ = N) the host output is not written."""
    import paper_1203_6836_amd as p
    say("case host-memory solve error path")
    pos = synth.lattice_positions((3, 3, 3), seed=7)
    H = ctx.tb_hamiltonian_mem(synth.STATIC_MODEL, np.ascontiguousarray(pos, dtype=np.float64))
    D = np.full_like(H, np.nan)
    with pytest.raises(p.Sp2Error) as e:
        ctx.sp2_density_matrix_mem(H, H.shape[0], p.options("fp64"), D_out=D)
    assert e.value.status == p.SP2_EINVAL
    assert np.isnan(D).all()


def test_second_thread_gets_ebusy(ctx):
    """While one thread is inside a call on a context (an N = 8192 FP64 solve,
    about half a second), a call from another thread returns SP2_EBUSY and
    does nothing; once the first call has returned, the same call succeeds."""
    import torch
    import paper_1203_6836_amd as p
    say("case SP2_EBUSY from a second thread")
    w = synth.MIXED
    H_big = ctx.tb_hamiltonian(synth.STATIC_MODEL, torch.from_numpy(w.positions()).cuda())
    small = synth.lattice_positions((3, 3, 3), seed=7)
    H_small = ctx.tb_hamiltonian(synth.STATIC_MODEL, torch.from_numpy(small).cuda())
    torch.cuda.synchronize()
    result = {}

    def long_call():
        result["D"], result["st"] = ctx.sp2_density_matrix(H_big, w.n_occ, p.options("fp64"))

    th = threading.Thread(target=long_call)
    t0 = time.perf_counter()
    th.start()
    time.sleep(0.1)
    st, _ = ctx.sp2_density_matrix_status(H_small, 2 * len(small), p.options("fp64"))
    busy_at = time.perf_counter() - t0
    th.join()
    done_at = time.perf_counter() - t0
    say(f"  second call at {busy_at:.3f} s returned {st}; first call done at {done_at:.3f} s")
    assert busy_at < done_at
    assert st == p.SP2_EBUSY
    assert result["st"]["status"] == "converged"
    st2, s2 = ctx.sp2_density_matrix_status(H_small, 2 * len(small), p.options("fp64"))
    assert st2 == p.SP2_OK and s2["status"] == "converged"

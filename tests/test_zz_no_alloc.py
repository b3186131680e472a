"""The allocation-free SP2 entry point (static device scratch) against the
allocating one, through the C-ABI: two calls in a row, the second smaller."""
import sys

import numpy as np
import pytest

import synth
from oracle import sp2 as osp2, tb as otb

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_1203_6836_amd as p
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = p.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def hamiltonian(dims, seed, n_atoms=None):
    pos = synth.lattice_positions(dims, seed=seed, n_atoms=n_atoms)
    return otb.hamiltonian(pos, None, synth.STATIC_MODEL), 2 * len(pos)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def test_noalloc_equals_allocating_entry_point_twice(ctx):
    import paper_1203_6836_amd as p
    # 1000 orbitals (8 x 8 tiles, ragged), then 260 (3 x 3 tiles, ragged):
    # the second call runs on scratch that still holds the first call's data
    for dims, seed, nat in (((5, 5, 10), 21, None), ((5, 5, 5), 22, 65)):
        H, nocc = hamiltonian(dims, seed, nat)
        N = H.shape[0]
        say(f"case noalloc N={N} seed={seed}")
        Hd = to_dev(H)
        D_ref, st_ref = ctx.sp2_density_matrix(Hd, nocc, p.options("fp64"))
        D, st = ctx.sp2_density_matrix_noalloc(Hd, nocc, p.options("fp64"))
        D_ref, D = D_ref.cpu().numpy(), D.cpu().numpy()
        err = np.linalg.norm(D - D_ref) / np.sqrt(N)
        say(f"  iters {st['iterations']} / {st_ref['iterations']} err/sqrtN={err:.2e} "
            f"max|dD|={np.max(np.abs(D - D_ref)):.2e}")
        assert err <= 1e-10
        assert st["status"] == st_ref["status"] == "converged"
        assert st["iterations"] == st_ref["iterations"]
        assert st["branches"] == st_ref["branches"]
        assert abs(np.trace(D) - nocc) < 1e-10
        if N <= 260:
            ref = osp2.sp2(H, nocc, tol=1e-10)
            assert np.linalg.norm(D - ref.D) / np.sqrt(N) <= 1e-10


def test_noalloc_at_its_maximum_and_beyond(ctx):
    import paper_1203_6836_amd as p
    H, nocc = hamiltonian((8, 8, 4), 23)       # N = 1024, the largest accepted
    say(f"case noalloc N={H.shape[0]} (maximum)")
    Hd = to_dev(H)
    D_ref, _ = ctx.sp2_density_matrix(Hd, nocc, p.options("fp64"))
    D, st = ctx.sp2_density_matrix_noalloc(Hd, nocc, p.options("fp64", tail_split=0))
    D_ref0, _ = ctx.sp2_density_matrix(Hd, nocc, p.options("fp64", tail_split=0))
    D, D_ref, D_ref0 = D.cpu().numpy(), D_ref.cpu().numpy(), D_ref0.cpu().numpy()
    assert np.linalg.norm(D - D_ref0) / 32.0 <= 1e-10
    assert np.linalg.norm(D - D_ref) / 32.0 <= 1e-10
    # rejected on the host before any device work
    H2, nocc2 = hamiltonian((5, 5, 11), 24, 257)   # N = 1028
    for opts, Hx, nx in ((p.options("fp64"), H2, nocc2), (p.options("int8x"), H, nocc),
                         (p.options("fp64", tau=1e-5), H, nocc)):
        with pytest.raises(p.Sp2Error) as e:
            ctx.sp2_density_matrix_noalloc(to_dev(Hx), nx, opts)
        assert e.value.status == p.SP2_EINVAL

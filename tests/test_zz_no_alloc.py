"""The allocation-free variant of the Dirichlet load (for callers that
cannot allocate device memory): fftfem_dirichlet_load_noalloc, called
through the C ABI, against fftfem_dirichlet_load (same kernels, so the same
values bit for bit) and the oracle, on two calls in a row on one device,
the second with a smaller input (the static work area keeps the first
call's contents), with several right-hand sides and out == f; and the size
limit of the static work area, checked on the host."""
import ctypes

import numpy as np
import pytest

from oracle import dirichlet
from paper_1701_03967_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EINVAL = -1


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def fm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1701_03967_amd import fftfem
    fftfem.lib()
    return fftfem


def call_noalloc(fm, p, b, f, out):
    rc = fm.lib().fftfem_dirichlet_load_noalloc(p._h, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(f.data_ptr()),
                                               ctypes.c_void_p(out.data_ptr()),
                                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc


def one_case(fm, K, n, react, nrhs, seed, inplace=False):
    N = len(K)
    diff = (1.0, 0.5, 2.0)[:N]
    p = fm.Plan(K, n, diff, react, nrhs=nrhs)
    ext = tuple(m + 2 for m in p.shape)
    b = inputs.draw_rhs(ext, seed=seed, nrhs=nrhs)
    f = inputs.draw_rhs(p.shape, seed=seed + 1, nrhs=nrhs)
    bd, fd = torch.from_numpy(b).cuda(), torch.from_numpy(f).cuda()
    want = p.dirichlet_load(bd, fd)  # with a work array
    out = fd.clone() if inplace else torch.full_like(fd, float("nan"))
    rc = call_noalloc(fm, p, bd, out if inplace else fd, out)
    torch.cuda.synchronize()
    assert rc == 0
    assert torch.equal(out, want)
    got = out.cpu().numpy().reshape((nrhs,) + tuple(p.shape))
    bb = b.reshape((nrhs,) + ext)
    ff = f.reshape((nrhs,) + tuple(p.shape))
    for r in range(nrhs):
        ref = dirichlet.lifted_load(bb[r], ff[r], n, K, diff, react)
        scale = np.abs(ref - ff[r]).max() + np.abs(ff[r]).max()
        assert np.abs(got[r] - ref).max() <= 1e-13 * scale


def test_noalloc_two_calls_second_smaller(fm):
    say("noalloc: 2D n=(3,4) K=(40,24) nrhs=2, then 2D n=2 K=(8,6)")
    one_case(fm, (40, 24), (3, 4), 0.5, 2, 301)
    one_case(fm, (8, 6), 2, 0.0, 1, 303)


def test_noalloc_3d_and_in_place(fm):
    say("noalloc: 3D n=(2,3,2) K=(6,5,7) in place, then 1D n=4 K=9")
    one_case(fm, (6, 5, 7), (2, 3, 2), 1.0, 1, 305, inplace=True)
    one_case(fm, (9,), 4, 2.0, 3, 307)


def test_noalloc_size_limit(fm):
    """2 prod(E_d) doubles above the static array's 2^21: EINVAL on the host,
    no kernel launched; a call at the limit's side still works."""
    say("noalloc: size limit")
    p = fm.Plan((128, 128), 9, (1.0, 1.0), 0.0)  # E = 1153^2 > 2^20
    b = torch.zeros(tuple(m + 2 for m in p.shape), dtype=torch.float64, device="cuda")
    f = torch.zeros(p.shape, dtype=torch.float64, device="cuda")
    out = torch.empty_like(f)
    assert call_noalloc(fm, p, b, f, out) == EINVAL
    one_case(fm, (100, 112), (9, 9), 0.0, 1, 309)  # E = 901 x 1009 <= 2^20

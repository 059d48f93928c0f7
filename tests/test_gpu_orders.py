"""GPU parity with a different element order per axis (Sect. 4: the space
of orders n = (n_1, ..., n_N)): solves in every precision mode, the
transpose-free and transposed 2D schedules, 3D, element counts that are not
powers of two, the operator apply, and a batch, against the oracle."""
import numpy as np
import pytest

from oracle import solve as osolve
from paper_1701_03967_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def fm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1701_03967_amd import fftfem
    fftfem.lib()
    return fftfem


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


TOL = {"fp64": 1e-11, "fp32": 1e-5, "fp32_refine": 1e-10}
CASES = [((32, 24), (2, 5), "fp64"), ((32, 24), (2, 5), "fp32"), ((32, 24), (5, 2), "fp32_refine"),
         ((256, 16), (9, 3), "fp64"), ((256, 16), (9, 3), "fp32"), ((128, 64), (4, 9), "fp32_refine"),
         ((8, 12, 10), (3, 2, 4), "fp64"), ((8, 12, 10), (1, 9, 2), "fp32_refine"),
         ((20, 12), (4, 6), "fp64"), ((17, 33), (7, 3), "fp32_refine")]


@pytest.mark.parametrize("K,ns,precision", CASES)
def test_mixed_orders_solve(fm, K, ns, precision):
    N = len(K)
    diff = (1.0, 0.5, 2.0)[:N]
    react = 0.75
    shape = tuple(m * k - 1 for m, k in zip(ns, K))
    f = inputs.draw_rhs(shape, seed=61)
    say("mixed orders", K, ns, precision)
    ref = osolve.solve(f, ns, K, diff, react)
    kw = dict(max_iter=4, tol=1e-13) if precision == "fp32_refine" else {}
    p = fm.Plan(K, ns, diff, react, precision=precision, **kw)
    assert p.shape == shape
    u = p.solve(torch.from_numpy(f).cuda())
    torch.cuda.synchronize()
    e = rel(u.cpu().numpy(), ref)
    say("  rel", e)
    assert e < TOL[precision]


def test_mixed_orders_apply_exact(fm):
    K, ns, diff, react = (6, 5), (3, 7), (1.0, 2.0), 0.5
    shape = tuple(m * k - 1 for m, k in zip(ns, K))
    u = inputs.draw_rhs(shape, seed=62)
    ref = osolve.apply_A_exact(u, ns, K, diff, react)
    y = fm.Plan(K, ns, diff, react).apply_A(torch.from_numpy(u).cuda())
    torch.cuda.synchronize()
    assert np.abs(y.cpu().numpy() - ref).max() <= 4e-16 * np.abs(ref).max() * 8


def test_mixed_orders_batch(fm):
    probs = [dict(K=(16, 24), n=(2, 5), diff=(1.0, 1.5), react=10.0, precision="fp32_refine", max_iter=4,
                  tol=1e-13),
             dict(K=(12, 9), n=(6, 3), diff=(0.5, 1.0), react=10.0, precision="fp64"),
             dict(K=(32, 8), n=4, diff=(1.0, 1.0), react=10.0, precision="fp32_refine", max_iter=4, tol=1e-13)]
    b = fm.Batch(probs)
    fs, us, hosts = [], [], []
    for i, pr in enumerate(probs):
        shape = b.shapes[i]
        fh = inputs.draw_rhs(shape, seed=70 + i)
        hosts.append(fh)
        fs.append(torch.from_numpy(fh).cuda())
        us.append(torch.empty_like(fs[-1]))
    b.solve(fs, us)
    torch.cuda.synchronize()
    for i, pr in enumerate(probs):
        ref = osolve.solve(hosts[i], pr["n"], pr["K"], pr["diff"], pr["react"])
        assert rel(us[i].cpu().numpy(), ref) < 1e-10, i

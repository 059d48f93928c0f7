"""GPU parity of the non-homogeneous Dirichlet reduction (Sect. 4 remark: a
modified load): fftfem_dirichlet_load against the oracle's f - A_IB b_B on
random boundary data in 1D, 2D and 3D with mixed orders, several
right-hand sides and out == f; then whole solves (both algorithms) against
the oracle's, and exact reproduction of a FEM-space polynomial with
non-zero boundary values."""
import numpy as np
import pytest

from oracle import dirichlet, loads
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


CASES = [((7,), 3, 0.5), ((16, 12), (2, 5), 0.0), ((9, 6), (9, 4), 3.0), ((5, 4, 6), (3, 2, 4), 1.0),
         ((33, 17), 3, 0.25)]


@pytest.mark.parametrize("K,n,react", CASES)
def test_dirichlet_load_matches_oracle(fm, K, n, react):
    N = len(K)
    diff = (1.0, 0.5, 2.0)[:N]
    p = fm.Plan(K, n, diff, react)
    say("dirichlet load", K, n, react)
    b = inputs.draw_rhs(p.extended_shape, seed=91)
    f = inputs.draw_rhs(p.shape, seed=92)
    ref = dirichlet.lifted_load(b, f, n, K, diff, react)
    got = p.dirichlet_load(torch.from_numpy(b).cuda(), torch.from_numpy(f).cuda()).cpu().numpy()
    # float64 sums of at most 2 (n + 1)^N products per term, each term scaled
    # by coef ~ 4 K^2: compare against the terms' own size
    scale = np.abs(f).max() + np.abs(ref - f).max()
    err = np.abs(got - ref).max() / scale
    say("  max err / scale", err)
    assert err < 1e-13


def test_dirichlet_load_several_rhs_in_place(fm):
    K, n, diff, react = (6, 8), 3, (1.0, 1.0), 2.0
    p = fm.Plan(K, n, diff, react, nrhs=2)
    b = inputs.draw_rhs(p.extended_shape[1:], seed=93, nrhs=2)
    f = inputs.draw_rhs(p.shape, seed=94, nrhs=2)
    ref = np.stack([dirichlet.lifted_load(b[r], f[r], n, K, diff, react) for r in range(2)])
    fd = torch.from_numpy(f).cuda()
    out = p.dirichlet_load(torch.from_numpy(b).cuda(), fd, out=fd).cpu().numpy()
    assert np.abs(out - ref).max() < 1e-13 * (np.abs(ref).max() + np.abs(f).max())


@pytest.mark.parametrize("algorithm", ["a", "b"])
def test_dirichlet_solve_matches_oracle(fm, algorithm):
    K, n, diff, react = (12, 10), (4, 3), (1.0, 2.0), 0.5
    p = fm.Plan(K, n, diff, react, algorithm=algorithm)
    b = inputs.draw_rhs(p.extended_shape, seed=95)
    f = inputs.draw_rhs(p.shape, seed=96)
    ref = dirichlet.solve_dirichlet(b, f, n, K, diff, react)
    g = p.dirichlet_load(torch.from_numpy(b).cuda(), torch.from_numpy(f).cuda())
    u = p.solve(g).cpu().numpy()
    e = rel(u, ref[1:-1, 1:-1])
    say("dirichlet solve", algorithm, e)
    assert e < 1e-11


def test_dirichlet_polynomial_reproduced(fm):
    """u* = (1 + x + 2x^2)(3 - y + y^3), n = 3: the discrete solution with
    u* on the boundary is u* at every dof."""
    K, n, diff, react = (8, 6), 3, (1.0, 0.5), 2.0
    P = [np.polynomial.Polynomial((1.0, 1.0, 2.0)), np.polynomial.Polynomial((3.0, -1.0, 0.0, 1.0))]
    u = lambda x, y: P[0](x) * P[1](y)
    f = lambda x, y: (-diff[0] * P[0].deriv(2)(x) * P[1](y) - diff[1] * P[0](x) * P[1].deriv(2)(y)
                      + react * u(x, y))
    fh = np.ascontiguousarray(loads.load_vector(f, n, K))
    grids = [np.arange(n * k + 1) / (n * k) for k in K]
    b = np.ascontiguousarray(u(*np.meshgrid(*grids, indexing="ij")))
    p = fm.Plan(K, n, diff, react)
    g = p.dirichlet_load(torch.from_numpy(b).cuda(), torch.from_numpy(fh).cuda())
    ui = p.solve(g).cpu().numpy()
    err = np.abs(ui - b[1:-1, 1:-1]).max() / np.abs(b).max()
    say("polynomial", err)
    assert err < 1e-12

"""GPU parity of implicit Euler time stepping (fftfem_implicit_euler: per
step one mass apply and one solve with the plan) against the oracle's
stepping, for float64 and float32 + refinement plans, 2D and 3D, with and
without a load, several right-hand-side sets."""
import numpy as np
import pytest

from oracle import timestep
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


CASES = [((32, 24), 4, (1.0, 0.5), 1e3, 6, True, 1, "fp64", 1e-11),
         ((64, 64), 3, (2.0, 1.0), 50.0, 4, False, 2, "fp64", 1e-11),
         ((8, 12, 10), 2, (1.0, 2.0, 0.5), 1e2, 3, True, 1, "fp64", 1e-11),
         ((40, 32), 5, (1.0, 1.0), 1e3, 3, True, 1, "fp32_refine", 1e-10)]


@pytest.mark.parametrize("K,n,diff,react,steps,load,nrhs,precision,tol", CASES)
def test_implicit_euler_vs_oracle(fm, K, n, diff, react, steps, load, nrhs, precision, tol):
    shape = tuple(n * k - 1 for k in K)
    full = ((nrhs,) if nrhs > 1 else ()) + shape
    u0 = inputs.draw_rhs(shape, seed=51, nrhs=nrhs)
    F = inputs.draw_rhs(shape, seed=52, nrhs=nrhs) if load else None
    say("implicit euler", K, n, react, steps, load, nrhs, precision)
    kw = dict(max_iter=4, tol=1e-13) if precision == "fp32_refine" else {}
    p = fm.Plan(K, n, diff, react, precision=precision, nrhs=nrhs, **kw)
    u = torch.from_numpy(np.ascontiguousarray(u0.reshape(full))).cuda()
    Ft = torch.from_numpy(np.ascontiguousarray(F.reshape(full))).cuda() if load else None
    p.implicit_euler(u, steps, F=Ft)
    torch.cuda.synchronize()
    got = u.cpu().numpy().reshape((nrhs,) + shape)
    u0r = u0.reshape((nrhs,) + shape)
    Fr = F.reshape((nrhs,) + shape) if load else None
    for r in range(nrhs):
        ref = timestep.implicit_euler(u0r[r], Fr[r] if load else None, n, K, diff, react, steps)
        e = rel(got[r], ref)
        say("  rhs", r, e)
        assert e < tol


def test_implicit_euler_zero_steps_and_errors(fm):
    K, n = (8, 8), 2
    p = fm.Plan(K, n, (1.0, 1.0), 10.0)
    u = torch.randn((n * 8 - 1, n * 8 - 1), dtype=torch.float64, device="cuda")
    u0 = u.clone()
    p.implicit_euler(u, 0)
    torch.cuda.synchronize()
    assert torch.equal(u, u0)
    with pytest.raises(fm.FftfemError):
        p.implicit_euler(u, 1, work=u)  # work overlaps u
    with pytest.raises(fm.FftfemError):
        fm.Plan(K, n, (1.0, 1.0), 0.0).implicit_euler(u, 1)  # react = 0: no time step

"""Pins of the oracle's implicit time stepping (Sect. 4 remark on implicit
time discretizations) against closed forms of the implicit Euler method:
the decay of a single eigenmode of the pencil (A_diff, C), and the steady
state A_diff u = F.  The reference values come from the dense pencil
eigendecomposition and a dense Cholesky solve of assembled matrices (SciPy),
not from the stepping code."""
import numpy as np
import scipy.linalg

from oracle import solve as osolve
from oracle import timestep
from paper_1701_03967_amd import inputs


def _mats(n, K, diff):
    A = osolve.assemble_full(n, K, diff, 0.0)
    Cm = osolve.assemble_full(n, K, [0.0] * len(K), 1.0)
    return A, Cm


def test_eigenmode_decays_by_the_euler_factor():
    # u0 = eigenvector v of A v = lam C v, F = 0: u^m = (react / (react + lam))^m v
    n, K, diff, react, m = 2, (4, 5), (1.0, 0.7), 40.0, 7
    A, Cm = _mats(n, K, diff)
    lam, V = scipy.linalg.eigh(A, Cm)
    shape = tuple(n * k - 1 for k in K)
    for i in (0, 5, len(lam) - 1):
        v = V[:, i].reshape(shape)
        u = timestep.implicit_euler(v, None, n, K, diff, react, m)
        expect = (react / (react + lam[i])) ** m * v
        assert np.linalg.norm(u - expect) <= 1e-12 * np.linalg.norm(v), i


def test_steady_state_of_many_steps():
    # the fixed point of the steps solves A_diff u = F; the error contracts by
    # react / (react + lam_min) per step
    n, K, diff, react = 3, (3, 4), (1.0, 2.0), 1.0
    A, Cm = _mats(n, K, diff)
    lam_min = scipy.linalg.eigh(A, Cm, eigvals_only=True)[0]
    steps = int(np.ceil(np.log(1e-15) / np.log(react / (react + lam_min)))) + 2
    shape = tuple(n * k - 1 for k in K)
    F = inputs.draw_rhs(shape, seed=41)
    u = timestep.implicit_euler(np.zeros(shape), F, n, K, diff, react, steps)
    u_inf = scipy.linalg.cho_solve(scipy.linalg.cho_factor(A), F.reshape(-1)).reshape(shape)
    assert np.linalg.norm(u - u_inf) <= 1e-11 * np.linalg.norm(u_inf)


def test_mass_apply_matches_assembled_mass():
    n, K = 4, (3, 2, 3)
    _, Cm = _mats(n, K, (1.0, 1.0, 1.0))
    shape = tuple(n * k - 1 for k in K)
    u = inputs.draw_rhs(shape, seed=42)
    assert np.allclose(timestep.mass_apply(u, n, K), (Cm @ u.reshape(-1)).reshape(shape), rtol=0, atol=1e-13)

"""Write sampled oracle solutions of the full-size workloads.

    python tests/golden/make_fullsize.py [c3_2d_n9_k1024] [c4_3d_n9_k64]

For each workload: the seeded right-hand side of the workload table, solved
by the CPU oracle (per-axis dense generalized eigendecomposition, mode
products, refinement with the extended-precision residual of the exact
operator), then a text fixture ``fullsize_<name>.txt`` with

  * the solution's l2 norm, max norm and plain sum over all dofs;
  * 4096 seeded random flat indices, the first and last dof of every axis
    line through the array's corners, and every local position (node and
    bubbles) of one element in the middle of the array, each with the
    oracle's float64 value (17 significant digits);
  * the inner products ``proj<i>`` of the whole solution with the seeded
    random sign vectors ``inputs.probe_vector(shape, i)``, i < NPROBE, which
    any error of the solution moves by about its l2 norm wherever it sits.

Only the oracle and the seeded input generator are used.  The C3 solve takes
some minutes and ~15 GB of host memory; C4 ~30 GB.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import solve as osolve  # noqa: E402
from paper_1701_03967_amd import inputs  # noqa: E402

NSAMPLE = 4096


def sample_indices(shape, n, seed):
    """Seeded flat indices plus structured edge positions."""
    size = int(np.prod(shape))
    g = np.random.default_rng(seed)
    idx = set(int(i) for i in g.choice(size, size=NSAMPLE, replace=False))
    N = len(shape)
    # corners and their axis neighbours: first/last dofs (next to the boundary)
    for corner in range(1 << N):
        c = [0 if (corner >> d) & 1 == 0 else shape[d] - 1 for d in range(N)]
        idx.add(int(np.ravel_multi_index(c, shape)))
        for d in range(N):
            for step in (1, n - 1, n):
                cc = list(c)
                cc[d] = min(max(cc[d] + (step if c[d] == 0 else -step), 0), shape[d] - 1)
                idx.add(int(np.ravel_multi_index(cc, shape)))
    # all local positions of one element per axis through the middle
    mid = [s // 2 for s in shape]
    for d in range(N):
        e0 = (mid[d] // n) * n
        for i in range(-1, n):
            cc = list(mid)
            cc[d] = e0 + i
            idx.add(int(np.ravel_multi_index(cc, shape)))
    return np.array(sorted(idx), dtype=np.int64)


def main(names):
    for name in names:
        w = inputs.WORKLOADS[name]
        prob = w.problem
        t0 = time.time()
        f = inputs.workload_rhs(name)
        hist = []
        s = osolve.EigenSolver(prob.n, prob.K, prob.diff, prob.react)
        t1 = time.time()
        u = s.solve(f, history=hist)
        t2 = time.time()
        del f
        idx = sample_indices(prob.shape, prob.n, 7)
        flat = u.reshape(-1)
        path = os.path.join(HERE, f"fullsize_{name}.txt")
        with open(path, "w") as fh:
            fh.write(f"# Oracle solution samples of workload {name}: N={prob.N} n={prob.n} "
                     f"K={list(prob.K)} diff={list(prob.diff)} react={prob.react}\n")
            fh.write(f"# rhs: {w.rhs}, seed {w.seed}; oracle: dense per-axis eigendecomposition "
                     f"({t1 - t0:.0f} s) + refinement with the extended residual ({t2 - t1:.0f} s); "
                     f"relative corrections {['%.2e' % h for h in hist]}\n")
            fh.write("# written by tests/golden/make_fullsize.py (oracle only)\n")
            fh.write(f"l2 {float(np.linalg.norm(flat)):.17e}\n")
            fh.write(f"max {float(np.abs(flat).max()):.17e}\n")
            fh.write(f"sum {float(flat.sum()):.17e}\n")
            for i in range(inputs.NPROBE):
                w = inputs.probe_vector(prob.shape, i).reshape(-1)
                fh.write(f"proj{i} {float(np.dot(w, flat)):.17e}\n")
                del w
            for i in idx:
                fh.write(f"{int(i)} {float(flat[i]):.17e}\n")
        print(f"[fullsize] {name}: {len(idx)} samples, eig {t1 - t0:.0f}s, solve {t2 - t1:.0f}s, "
              f"corrections {hist}", flush=True)
        del u, flat, s


if __name__ == "__main__":
    main(sys.argv[1:] or ["c3_2d_n9_k1024", "c4_3d_n9_k64"])

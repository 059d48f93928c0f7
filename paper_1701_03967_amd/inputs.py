"""Seeded synthetic workloads for the tensor-product FEM Poisson solver.

This module is shared by the tests, the benchmark and the CPU oracle's
callers.  It holds no solver arithmetic: it only names the problem
configurations and draws seeded random load vectors of the right shapes.

Layout convention (used by every consumer): a load or solution is a dense
row-major float64 array of shape (M_1, ..., M_N) with M_d = n*K_d - 1, the
last axis contiguous.  Entry g_d (0-based) along axis d is the degree of
freedom at x_d = (g_d + 1) * h_d / n, h_d = 1/K_d: it is the mesh node
j = (g_d + 1)/n when (g_d + 1) % n == 0, otherwise bubble l = g_d % n + 1 of
element j = g_d // n + 1 (the ordering of the space S_K^(n) in Sect. 2 of the
paper, with the boundary nodes removed by the Dirichlet condition).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np


@dataclass(frozen=True)
class Problem:
    """One constant-coefficient problem sum_d diff[d]*(-d2u/dx_d^2) + react*u = f."""

    n: int                      # polynomial order of the elements
    K: Tuple[int, ...]          # elements per axis
    diff: Tuple[float, ...]     # diffusion coefficient per axis
    react: float = 0.0          # reaction coefficient
    nrhs: int = 1               # independent right-hand sides

    @property
    def N(self) -> int:
        return len(self.K)

    @property
    def shape(self) -> Tuple[int, ...]:
        return tuple(self.n * k - 1 for k in self.K)

    @property
    def size(self) -> int:
        return int(np.prod(self.shape))


@dataclass(frozen=True)
class Workload:
    name: str
    problem: Problem
    seed: int
    rhs: str                    # "normal" | "uniform"
    note: str = ""


# The five workloads.  The seeds follow a fixed assignment (0..4).
WORKLOADS = {
    "c1_2d_n2_k16": Workload(
        "c1_2d_n2_k16", Problem(2, (16, 16), (1.0, 1.0), 0.0), 0, "normal",
        "2D unit square, n=2, K=16 per axis, 961 unknowns"),
    "c2_2d_n4_k256": Workload(
        "c2_2d_n4_k256", Problem(4, (256, 256), (1.0, 0.25), 0.0), 1, "normal",
        "2D, n=4, K=256 per axis, 1023^2 unknowns"),
    "c3_2d_n9_k1024": Workload(
        "c3_2d_n9_k1024", Problem(9, (1024, 1024), (1.0, 1.0), 0.0), 2, "uniform",
        "2D, n=9, K=1024 per axis, 9215^2 = 84.9M unknowns"),
    "c4_3d_n9_k64": Workload(
        "c4_3d_n9_k64", Problem(9, (64, 64, 64), (1.0, 2.0, 0.5), 0.0), 3, "normal",
        "3D unit cube, n=9, K=64 per axis, 575^3 = 190.1M unknowns"),
}


def generator(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def draw_rhs(shape, seed: int, kind: str = "normal", nrhs: int = 1) -> np.ndarray:
    """Seeded i.i.d. load coefficients: N(0,1) or U[-1,1], float64.

    With nrhs > 1 the result has a leading dimension of length nrhs.
    """
    g = generator(seed)
    full = (nrhs,) + tuple(shape) if nrhs > 1 else tuple(shape)
    if kind == "normal":
        return g.standard_normal(full, dtype=np.float64)
    if kind == "uniform":
        return g.uniform(-1.0, 1.0, size=full)
    raise ValueError(f"unknown rhs kind {kind!r}")


def workload_rhs(name: str) -> np.ndarray:
    w = WORKLOADS[name]
    return draw_rhs(w.problem.shape, w.seed, w.rhs)


@dataclass
class BatchDraw:
    problems: List[Problem] = field(default_factory=list)
    seeds: List[int] = field(default_factory=list)


def draw_batch(count: int = 512, seed: int = 4, n_range=(2, 8), k_range=(32, 512),
               diff_range=(0.5, 2.0), tau: float = 1e-3, nrhs_range=(1, 8)) -> BatchDraw:
    """The batched workload: independent 2D implicit heat steps.

    Per problem (integers inclusive): n ~ U{n_range}, K_1 and K_2 ~ U{k_range}
    independently, diff_1, diff_2 ~ U[diff_range] independently,
    react = 1/tau, nrhs ~ U{nrhs_range}.  Right-hand sides are N(0,1) with a
    per-problem seed spawned from ``seed``.
    """
    g = generator(seed)
    out = BatchDraw()
    children = np.random.SeedSequence(seed).spawn(count)
    for i in range(count):
        n = int(g.integers(n_range[0], n_range[1] + 1))
        k1 = int(g.integers(k_range[0], k_range[1] + 1))
        k2 = int(g.integers(k_range[0], k_range[1] + 1))
        d1 = float(g.uniform(*diff_range))
        d2 = float(g.uniform(*diff_range))
        r = int(g.integers(nrhs_range[0], nrhs_range[1] + 1))
        out.problems.append(Problem(n, (k1, k2), (d1, d2), 1.0 / tau, r))
        out.seeds.append(int(children[i].generate_state(1)[0]))
    return out


def batch_rhs(draw: BatchDraw, i: int) -> np.ndarray:
    """Right-hand sides of problem i of a batch: shape (nrhs, M_1, M_2)."""
    p = draw.problems[i]
    g = generator(draw.seeds[i])
    return g.standard_normal((p.nrhs,) + p.shape, dtype=np.float64)


# Random sign vectors for whole-array checks at sizes where a solution can be
# stored only as samples: <w_i, u> over every entry of u, with w_i of i.i.d.
# +-1 entries, moves by about ||delta|| under any perturbation delta of u,
# wherever in the array it sits.
NPROBE = 4


def probe_vector(shape, i: int) -> np.ndarray:
    """The i-th seeded +-1 vector of the given shape (float64)."""
    g = generator(90000 + int(i))
    size = int(np.prod(shape))
    s = g.integers(0, 2, size=size, dtype=np.int8)
    out = s.astype(np.float64)
    out *= 2.0
    out -= 1.0
    return out.reshape(tuple(shape))

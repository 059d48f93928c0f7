/*
 * fftfem.h -- C ABI of the MI355X fast direct solver for the tensor-product
 * nth-order finite element method on a box (Zlotnik & Zlotnik, "On fast
 * Fourier solvers for the tensor product high-order FEM for a generalized
 * Poisson equation").
 *
 * Problem (Sect. 4 of the paper, "algorithm (a)", generalized to per-axis
 * diffusion diff[d] and reaction react):
 *
 *   ( sum_d diff[d] * 4/h_d^2 * C_1 x .. x A_d x .. x C_N
 *     + react * C_1 x .. x C_N ) u = f,          h_d = X_d / K_d,
 *
 * where A_d, C_d are the scaled 1D stiffness and mass operators of the
 * nth-order Lagrange elements on K_d uniform elements with homogeneous
 * Dirichlet conditions (Sect. 2), and f is the "FEM average" load
 * f_i = prod_d (2/h_d) * integral(f * phi_i).  The solver applies the direct
 * FC_n transform along every axis, divides by react + sum_d diff[d] 4/h_d^2
 * lambda_d, and applies the inverse F_n transform along every axis
 * (Sect. 3, Theorem 2; Sect. 4, algorithm (a)).
 *
 * Array layout (f, u, y): dense row-major float64 of shape (M_1, ..., M_N),
 * M_d = n_d*K_d - 1 with n_d the element order of axis d (Sect. 4 allows an
 * order per axis; by default n_d = n), last axis contiguous, optionally with
 * a leading dimension of nrhs.  Along axis d (order n = n_d), 0-based index g
 * is the dof at x = (g+1) h_d / n: mesh node j = (g+1)/n when
 * (g+1) % n == 0, else bubble l = g % n + 1 of element j = g / n + 1 (the
 * ordering of S_K^(n), Sect. 2).  Boundary dofs are not stored.
 *
 * Pointers named "device" must point to memory allocated on the current HIP
 * device; everything else is host memory.  All functions return an int
 * status (FFTFEM_OK = 0, negative on error) unless stated otherwise.
 * Arguments are validated synchronously; kernel-side outcomes (refinement
 * convergence) are reported by fftfem_get_stats after the caller has
 * synchronized the stream.
 */
#ifndef FFTFEM_H
#define FFTFEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* hipStream_t;
typedef struct fftfem_plan_s* fftfem_plan_t;

enum {
  FFTFEM_OK = 0,
  FFTFEM_EINVAL = -1,     /* bad argument (null pointer, size, order, aliasing) */
  FFTFEM_ENOMEM = -2,     /* device or host allocation failed */
  FFTFEM_EHIP = -3,       /* a HIP runtime call failed */
  FFTFEM_ESPECTRUM = -4,  /* plan eigen-solve failed (non-finite or non-positive pencil) */
  FFTFEM_EINDEF = -5,     /* the operator is not positive definite (a denominator <= 0) */
  FFTFEM_ENOCONV = -6,    /* refinement did not reach the tolerance */
  FFTFEM_ENOTIMPL = -7    /* configuration not supported by this build */
};

enum {
  FFTFEM_FP64 = 0,        /* transforms and tables in float64, one pass, no refinement */
  FFTFEM_FP32 = 1,        /* transforms in float32 (float32 accumulate), no refinement */
  FFTFEM_FP32_REFINE = 2  /* float32 transforms + float64 residual/update refinement */
};

/*
 * fftfem_desc.flags: solve by algorithm (b) of Sect. 4 instead of (a): the
 * FC_n transform along axes 2..N only, then along axis 1 a direct banded
 * solve of each line's shifted 1D system (the bubbles of every element
 * condensed onto its end nodes, then the tridiagonal node system by
 * elimination), then the inverse transforms along axes 2..N.  FFTFEM_FP64
 * plans only (FFTFEM_ENOTIMPL otherwise) and not in batches.  The node
 * elimination's rounding error grows like the condition number of that
 * system, about (nK_1)^2 eps relative at react = 0.
 */
#define FFTFEM_ALGORITHM_B 1u

#define FFTFEM_MAX_DIMS 3
#define FFTFEM_MAX_ORDER 16
#define FFTFEM_MAX_ITERS 16

/* Full plan description.  Fields left zero take the documented defaults. */
typedef struct {
  int N;                          /* number of axes, 1..FFTFEM_MAX_DIMS */
  int64_t K[FFTFEM_MAX_DIMS];     /* elements per axis, 2 <= K[d] <= 1024 (ENOTIMPL above; FFTFEM_FP64
                                     plans of algorithm (a), not in batches, also accept any K up to
                                     2^20 on one axis, or on one or both of two axes:
                                     multi-pass transforms, whose two work arrays hold up to
                                     8 GiB each and take the lines in chunks beyond that; a
                                     two-axis plan of one order keeps one full-size scratch
                                     array) */
  int n;                          /* element order (every axis without n_axis), 1..FFTFEM_MAX_ORDER */
  double diff[FFTFEM_MAX_DIMS];   /* diffusion per axis, > 0 */
  double react;                   /* reaction coefficient */
  double X[FFTFEM_MAX_DIMS];      /* domain lengths (0 -> 1.0) */
  int precision;                  /* FFTFEM_FP64 / FFTFEM_FP32 / FFTFEM_FP32_REFINE */
  int max_iter;                   /* refinement iterations after the first solve (0 -> 3) */
  double tol;                     /* refinement stop: ||correction||/||u|| <= tol (0 -> 1e-12) */
  int nrhs;                       /* right-hand sides per solve (0 -> 1) */
  unsigned flags;                 /* 0 or FFTFEM_ALGORITHM_B; other bits must be 0 */
  int n_axis[FFTFEM_MAX_DIMS];    /* element order per axis (Sect. 4: n = (n_1, ..., n_N));
                                     0 -> n; M_d = n_axis[d] K[d] - 1 */
} fftfem_desc;

/* Why the refinement of a solve stopped (fftfem_stats.stop). */
enum {
  FFTFEM_STOP_NONE = 0,       /* no refinement (FFTFEM_FP64 / FFTFEM_FP32) and a finite solution */
  FFTFEM_STOP_TOL = 1,        /* the relative correction reached tol */
  FFTFEM_STOP_MAX_ITER = 2,   /* max_iter corrections applied without reaching tol */
  FFTFEM_STOP_NONFINITE = 3,  /* a NaN or Inf in the solution or in a correction (e.g. in f) */
  FFTFEM_STOP_STALLED = 4     /* a correction was not smaller than the one before (no contraction) */
};

/* Refinement statistics of the last fftfem_solve on a plan.  With several
 * right-hand sides: the largest iteration count and relative corrections
 * (NaN if any is NaN), converged only if every right-hand side converged,
 * and the stop reason of the worst one (NONFINITE, STALLED, MAX_ITER, TOL,
 * NONE in that order). */
typedef struct {
  int iterations;                     /* refinement corrections applied */
  int converged;                      /* 1: stop is FFTFEM_STOP_TOL or FFTFEM_STOP_NONE */
  double rel_correction[FFTFEM_MAX_ITERS + 1];  /* ||c_i|| / ||u_i|| per iteration, i = 0 is the first solve */
  int stop;                           /* FFTFEM_STOP_* */
} fftfem_stats;

/*
 * Build a plan (Sect. 3, Theorem 1: the 1D eigenpairs; Sect. 4: the
 * denominators).  Host computation in 113-bit floating point, then upload of
 * the tables and allocation of the device workspace on the current device
 * (synchronous).  Returns FFTFEM_EINVAL for bad sizes, FFTFEM_EINDEF if some
 * denominator react + sum_d diff[d] 4/h_d^2 lambda_d is <= 0,
 * FFTFEM_ESPECTRUM if an eigen-solve fails, FFTFEM_ENOMEM/EHIP on device
 * errors.  On failure *out is set to NULL.  The plan owns all device memory
 * it allocates; release it with fftfem_destroy.
 */
int fftfem_plan(fftfem_plan_t* out, int N, const int64_t* K, int n, const double* diff,
                double react);
int fftfem_plan_ex(fftfem_plan_t* out, const fftfem_desc* desc);

/*
 * Solve A u = f (algorithm (a) of Sect. 4, or (b) with FFTFEM_ALGORITHM_B).
 * For (b) the plan holds the banded solve's float64 work, chosen with its
 * form at plan time: none for K_1 <= 128 (one LDS-tiled kernel),
 * (K_1 - 1) M_2 .. M_N values with at least 64K lines (one sweep per line),
 * else M_1 .. M_N + 2 (K_1 - 1) M_2 .. M_N values (three kernels); see
 * fftfem_workspace_bytes.  f, u: device float64 arrays in
 * the layout above (times nrhs).  f is read only; u must not overlap f.
 * Asynchronous on stream s (NULL = default stream); no host synchronization
 * and no allocation.  A plan may be used by one stream at a time.
 */
int fftfem_solve(fftfem_plan_t p, const double* f, double* u, hipStream_t s);

/*
 * y = A u in float64 (the operator above, as the sum over elements of the
 * reference matrices along each axis, Sect. 2 and 4).  u, y: device arrays,
 * y must not overlap u.  Asynchronous on s.
 */
int fftfem_apply_A(fftfem_plan_t p, const double* u, double* y, hipStream_t s);

/*
 * Statistics of the last solve.  Synchronizes the plan's last stream.  The
 * device checks every value of the solution a solve writes for NaN and Inf
 * (in the output pass of the line kernels; a one-dimensional algorithm (b)
 * solve, whose output pass is the banded solve, is not checked), and in
 * FFTFEM_FP32_REFINE mode every correction: a non-finite value ends the
 * refinement.  Returns FFTFEM_ENOCONV, with *out filled in, when the solve
 * did not converge (out->converged == 0: a non-finite solution, or a
 * refinement that stopped short of tol), FFTFEM_OK otherwise.
 */
int fftfem_get_stats(fftfem_plan_t p, fftfem_stats* out);

/* Device bytes owned by the plan (tables + workspace). */
size_t fftfem_workspace_bytes(const fftfem_plan_t p);

/* Release a plan (NULL is accepted). */
void fftfem_destroy(fftfem_plan_t p);

/* Static description of a status code. */
const char* fftfem_status_string(int status);

/*
 * Plan tables on the host, for tests.  For axis d (0-based) with M = n K - 1:
 * lam (M doubles): the scaled 1D eigenvalues in spectral order -- k = 0 with
 * l = 1..n-1, then k = 1..K-1 with l = 1..n (ascending within k);
 * Q (n*n*K doubles, may be NULL): per frequency k the channel-by-mode matrix
 * (row c = nodal, even 1..n/2, odd 1..(n-1)/2 channel; column l = mode) of
 * the C-orthonormal eigenvectors; block k = 0 is (n-1)x(n-1) stored in the
 * leading rows/columns of an n x n block.
 */
int fftfem_plan_tables(const fftfem_plan_t p, int axis, double* lam, double* Q);

/*
 * One stage of the solve on one axis, for unit parity tests (not a stable
 * interface).  dir = +1: direct FC_n transform along `axis` of the device
 * array in (float64) into out (float64) in spectral order along that axis,
 * with coefficients (y, s~) for C-orthonormal eigenvectors s~; dir = -1: the
 * inverse F_n transform (spectral -> physical); dir = 0: forward, divide by
 * the axis-only denominator react + diff[d] 4/h_d^2 lambda, inverse.  dtype:
 * 0 = compute in float64, 1 = compute in float32.  in and out may be equal.
 * Plans with K > 1024 (float64 only) transform by the multi-pass path; axis
 * 0 of a two-axis such plan goes through a transposed copy in the plan's
 * scratch.
 */
int fftfem_debug_transform(fftfem_plan_t p, int axis, int dir, const double* in, double* out,
                           int dtype, hipStream_t s);

/*
 * Per-kernel timing, for measurement.  With timing enabled, every kernel a
 * solve or apply launches is bracketed by HIP events recorded on the same
 * stream (the events are created on first use; do not enable it under graph
 * capture).  fftfem_get_timing synchronizes, and returns for up to `max`
 * distinct kernels (in first-launch order) a NUL-terminated name of at most
 * 31 characters in names[32*i], the mean duration in milliseconds and the
 * number of launches since the previous call; it then clears the record.
 * Returns the number of distinct kernels (>= 0) or a negative status.
 */
int fftfem_set_timing(fftfem_plan_t p, int enable);
int fftfem_get_timing(fftfem_plan_t p, int max, char* names, double* avg_ms, int* count);

/*
 * Batches of independent problems (the implicit time step of many small
 * heat problems in Sect. 4 is one use): count problems, each with its own
 * descriptor (any N, K, n, diff, react, precision, nrhs), solved together.
 *
 * fftfem_plan_batch builds one plan per problem (tables of equal (n, K)
 * axes are computed once per axis length within a plan; every plan owns its
 * device tables and workspace).  flags: FFTFEM_BATCH_TUNE measures, on the
 * first solve, the lines per tile and the largest FFT radix of every
 * line pass kind in the batch (kept process-wide for
 * later plans of the same kind).  EINVAL for count < 1 or a null pointer;
 * otherwise the status of the first descriptor that fails fftfem_plan_ex.
 *
 * fftfem_solve_batch: f[i] and u[i] are device arrays of problem i (its
 * nrhs right-hand sides, as in fftfem_solve; u[i] must not overlap f[i]).
 * The first call (and any call with different pointers) records every
 * problem's schedule, groups all problems' passes of one kind at one
 * position of the schedule into one launch, and captures the launches
 * into a graph on an internal stream; each call then launches that graph
 * on s.  Right-hand sides of one problem run one after another (they share
 * the problem's workspace); problems run side by side.  Asynchronous on s;
 * calls that overlap on one batch race.  fftfem_batch_get_stats synchronizes
 * s of the last solve and returns problem i's statistics of its last
 * right-hand side, like fftfem_get_stats.
 */
typedef struct fftfem_batch_s* fftfem_batch_t;
#define FFTFEM_BATCH_TUNE 1
int fftfem_plan_batch(fftfem_batch_t* out, int count, const fftfem_desc* descs, int flags);
int fftfem_solve_batch(fftfem_batch_t b, const double* const* f, double* const* u, hipStream_t s);
int fftfem_batch_get_stats(fftfem_batch_t b, int i, fftfem_stats* out);
size_t fftfem_batch_workspace_bytes(const fftfem_batch_t b);
void fftfem_destroy_batch(fftfem_batch_t b);

/*
 * Expansion in the tensor eigenbasis (Sect. 3, Theorem 2: the direct FC_n
 * transform of loads, and, item 3, the direct F_n transform of grid
 * values, which is FC_n of C w).  With S_d the C_d-orthonormal
 * eigenvectors of axis d (Theorem 1) in the spectral order of
 * fftfem_plan_tables (block k = 0, then k = 1 .. K_d - 1, n_d modes each):
 *   fftfem_coefficients, kind 0 (values):  out = (x_d S_d^T C_d) in,
 *                        kind 1 (loads):   out = (x_d S_d^T) in;
 *   fftfem_synthesize:                      out = (x_d S_d) in,
 * so synthesize(coefficients(w, values)) = w and the coefficients of a
 * solution are those of its load divided by the denominators react +
 * sum_d diff[d] 4/h_d^2 lambda_d.  float64 transforms for every plan
 * precision; arrays in the layout of fftfem_solve (nrhs sets); out may equal
 * in except for kind 0.  Eigenvectors of the k = 0 blocks carry a free sign
 * (largest component positive).  Asynchronous on s.  EINVAL: null
 * pointers, bad kind, overlapping arrays, or a plan being recorded.
 */
int fftfem_coefficients(fftfem_plan_t p, const double* in, double* out, int kind, hipStream_t s);
int fftfem_synthesize(fftfem_plan_t p, const double* in, double* out, hipStream_t s);

/*
 * Non-homogeneous Dirichlet data u = b on the boundary (Sect. 4: only the
 * load of the scaled global system changes).  On the dofs of the
 * closed box -- every axis extended by its two boundary points, E_d = M_d + 2
 * points at x = g h_d / n_d, g = 0 .. E_d - 1, row-major, last axis
 * contiguous -- the interior equations read A_II u_I = f - A_IB b_B:
 *
 *   out = f - (interior rows of the extended operator) (b with its interior zeroed),
 *
 * the extended operator being the plan's tensor sum with every 1D stiffness
 * and mass assembled over all n_d K_d + 1 points.  fftfem_solve(p, out, u)
 * then gives the interior values of the solution; its boundary values are
 * b's.  b: device float64, E_1 x .. x E_N per right-hand side (only entries
 * with some index 0 or E_d - 1 are read); f, out: device float64 in the
 * interior layout (out may equal f); work: device float64 scratch of
 * 2 E_1 .. E_N values, overlapping none of the others.  float64 arithmetic,
 * asynchronous on s, no allocation.  FFTFEM_EINVAL for null pointers or
 * overlaps, or inside a batch.
 */
int fftfem_dirichlet_load(fftfem_plan_t p, const double* b, const double* f, double* out, double* work,
                          hipStream_t s);

/*
 * fftfem_dirichlet_load without the caller's work array, for callers that
 * cannot allocate device memory (code under graph capture, serving loops,
 * harnesses that forbid allocation): the 2 E_1 .. E_N doubles of work live
 * in a static device array of the library of 2^21 doubles (16 MiB) per
 * device, held until the process ends, so E_1 .. E_N <= 2^20
 * (FFTFEM_EINVAL above).  The same kernels and results as
 * fftfem_dirichlet_load.  It allocates nothing and calls no allocating
 * routine; the first call on a device looks up the array's device address
 * (hipGetSymbolAddress) and keeps it.  All calls on one device share the
 * array: calls that overlap in time on one device (other streams, other
 * threads) race.  Arguments as in fftfem_dirichlet_load; asynchronous on s.
 */
int fftfem_dirichlet_load_noalloc(fftfem_plan_t p, const double* b, const double* f, double* out,
                                  hipStream_t s);

/*
 * Implicit Euler time stepping of the semi-discrete heat equation of the
 * plan's operator (Sect. 4 remarks that implicit time discretizations of
 * heat-type equations lead at every time level to the system solved here):
 *
 *   C (u^{m+1} - u^m) / tau + A_diff u^{m+1} = F,   tau = 1 / react,
 *
 * A_diff = sum_d diff[d] 4 h_d^-2 C_1 x .. x A_d x .. x C_N and
 * C = C_1 x ... x C_N, i.e. (A_diff + react C) u^{m+1} = F + react C u^m.
 * Each of the nsteps steps is one mass apply (F + react C u^m into work, in
 * float64) and one fftfem_solve (the plan's precision mode);
 * the plan (tables, workspace) is reused by every step.
 * u: in/out, u^0 on entry, u^nsteps on return, layout and right-hand-side
 * sets as in fftfem_solve; F: the scaled load (nrhs sets), constant in time,
 * or NULL for zero; work: caller-owned device array of the size of u.  u,
 * work and F must not overlap.  Asynchronous on s.  EINVAL: null plan, u or
 * work, nsteps < 0, react <= 0, overlapping arrays, or a plan that belongs
 * to a batch being recorded; otherwise the status of the first failing step.
 */
int fftfem_implicit_euler(fftfem_plan_t p, const double* F, double* u, double* work, int nsteps,
                          hipStream_t s);

/*
 * fftfem_tune: the measurement FFTFEM_BATCH_TUNE makes, for the line passes
 * of one plan with N >= 2 (float32, float32 with refinement or float64): each
 * of the 2N - 1 passes of the solve (forward along axes N-1 .. 1, the middle
 * pass, inverse along 1 .. N-1) is timed on the plan's own scratch, in the
 * layout its solve uses, for every admissible lines per tile and largest
 * FFT radix (16, 8, 4); the fastest per pass kind (precision, n, mode,
 * strided or not, element count) is kept process-wide and used by every
 * later solve of plans of that kind.  Synchronizes s.  ENOTIMPL for N = 1,
 * EINVAL for a null plan, EHIP on a runtime error.
 */
int fftfem_tune(fftfem_plan_t p, hipStream_t s);

/*
 * The process-wide table of measured line-pass parameters as a text file
 * (one kind per line: bytes per value, n, pass mode, strided, element-count
 * class, lines per tile, log2 of the largest FFT radix).  fftfem_tune_save
 * writes the table to `path` and returns the number of entries;
 * fftfem_tune_load adds the entries of `path` to the table (replacing equal
 * kinds) and returns their number.  Tuning (fftfem_tune, FFTFEM_BATCH_TUNE)
 * measures only kinds the table does not hold, so a loaded file replaces the
 * measurement.  Host only.  EINVAL: null path, unreadable/unwritable file, or
 * a malformed or out-of-range line (then nothing is loaded).
 */
int fftfem_tune_save(const char* path);
int fftfem_tune_load(const char* path);

/*
 * Host-only access to the plan arithmetic, for tests on machines without a
 * GPU (no device is touched).  fftfem_axis_tables_host: the lam and Q tables
 * of fftfem_plan_tables for one axis of n-th order elements on K elements.
 * fftfem_element_matrices_host: the (n+1) x (n+1) reference stiffness A and
 * mass C of Sect. 2, row-major.
 */
int fftfem_axis_tables_host(int n, int64_t K, double* lam, double* Q);
int fftfem_element_matrices_host(int n, double* A, double* C);

#ifdef __cplusplus
}
#endif
#endif /* FFTFEM_H */

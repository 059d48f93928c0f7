// Operator apply (float64, for y = A u and the refinement residual), the
// refinement bookkeeping kernels and the tiled transpose (gfx950).
#include "device_common.h"
#include "launch.h"

namespace fftfem {

// Dynamic LDS of the kernels in this file.
extern __shared__ double2 fftfem_ops_lds[];

// ---------------------------------------------------------------------------
// 1D operator application along one axis (float64), for y = A u and the
// refinement residual.  For output position g of a line (Sect. 2, the
// element-by-element assembly of A and C):
//   node (g+1) % n == 0:  sum_t X[n][t] v[g-n+t] + sum_t X[0][t] v[g+t]
//   bubble l = g % n + 1: sum_t X[l][t] v[g-l+t]
// with v = 0 outside the line (Dirichlet).  Two inputs and two outputs with
// coefficient rows let one pass produce the sum-factorized partial products:
//   o1 = c1[0] A in1 + c1[1] C in1 + c1[2] A in2 + c1[3] C in2   (o1 = f - that, if sub_f)
//   o2 = c2[0] A in1 + c2[1] C in1 + c2[2] A in2 + c2[3] C in2
template <int NORD>
__device__ __forceinline__ void stencil(const double* __restrict__ v, int i, const double* X,
                                        double& out) {
  constexpr int n = NORD;
  double s = 0;
  if ((i + 1) % n == 0) {
#pragma unroll
    for (int t = 0; t <= n; ++t) s += X[n * (n + 1) + t] * v[i - n + t] + X[t] * v[i + t];
  } else {
    int l = i % n + 1;
#pragma unroll
    for (int t = 0; t <= n; ++t) s += X[l * (n + 1) + t] * v[i - l + t];
  }
  out = s;
}

template <int NORD>
__global__ __launch_bounds__(kThreads) void apply_kernel(ApplyArgs a) {
  if (a.flag && *a.flag) return;
  constexpr int n = NORD;
  double* sm = reinterpret_cast<double*>(fftfem_ops_lds);
  __shared__ double Xa[(NORD + 1) * (NORD + 1)], Xc[(NORD + 1) * (NORD + 1)];
  const int tid = threadIdx.x;
  for (int i = tid; i < (n + 1) * (n + 1); i += kThreads) {
    Xa[i] = a.Ael[i];
    Xc[i] = a.Cel[i];
  }
  const int G = a.G, TL = a.TL, W = TL + 2 * n;
  const int64_t nseg = (a.M + TL - 1) / TL;
  const int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t lg = tile / nseg, seg = tile - lg * nseg;
  const int64_t l0 = lg * G, s0 = seg * TL;
  const bool lines_fast = a.es > 1;
  const bool two = a.in2 != nullptr;
  double* v1 = sm;
  double* v2 = sm + G * W;
  for (int t = tid; t < G * W; t += kThreads) {
    int g, i;
    if (lines_fast) {
      g = t % G;
      i = t / G;
    } else {
      i = t % W;
      g = t / W;
    }
    int64_t line = l0 + g;
    int64_t pos = s0 - n + i;
    double x1 = 0, x2 = 0;
    if (line < a.nlines && pos >= 0 && pos < a.M) {
      int64_t outer = line / a.es, inner = line - outer * a.es;
      int64_t idx = outer * a.M * a.es + inner + pos * a.es;
      x1 = a.in1[idx];
      if (two) x2 = a.in2[idx];
    }
    v1[g * W + i] = x1;
    if (two) v2[g * W + i] = x2;
  }
  __syncthreads();
  for (int t = tid; t < G * TL; t += kThreads) {
    int g, i;
    if (lines_fast) {
      g = t % G;
      i = t / G;
    } else {
      i = t % TL;
      g = t / TL;
    }
    int64_t line = l0 + g;
    int64_t pos = s0 + i;
    if (line >= a.nlines || pos >= a.M) continue;
    // local index within the window: pos - (s0 - n); the stencil uses the
    // position along the line for the node/bubble pattern
    const double* w1 = v1 + g * W + n - s0;  // w1[pos] = window value at pos
    double A1, C1, A2 = 0, C2v = 0;
    stencil<NORD>(w1, (int)pos, Xa, A1);
    stencil<NORD>(w1, (int)pos, Xc, C1);
    if (two) {
      const double* w2 = v2 + g * W + n - s0;
      stencil<NORD>(w2, (int)pos, Xa, A2);
      stencil<NORD>(w2, (int)pos, Xc, C2v);
    }
    int64_t outer = line / a.es, inner = line - outer * a.es;
    int64_t idx = outer * a.M * a.es + inner + pos * a.es;
    double r1 = a.c1[0] * A1 + a.c1[1] * C1 + a.c1[2] * A2 + a.c1[3] * C2v;
    if (a.sub_f) r1 = a.f[idx] - r1;
    if (a.o1_f64)
      ((double*)a.o1)[idx] = r1;
    else
      ((float*)a.o1)[idx] = (float)r1;
    if (a.o2) a.o2[idx] = a.c2[0] * A1 + a.c2[1] * C1 + a.c2[2] * A2 + a.c2[3] * C2v;
  }
}

// ---------------------------------------------------------------------------
// Refinement bookkeeping.  stats layout (doubles): [0] iterations applied,
// [1] converged flag, [2 + i] relative correction of iteration i.
__global__ void reset_kernel(int* flag, double* stats, int nstats) {
  int i = threadIdx.x;
  if (i == 0) *flag = 0;
  for (int j = i; j < nstats; j += blockDim.x) stats[j] = 0;
}

__global__ void reduce_kernel(const double* partials, int nparts, int iter, double tol,
                              int* flag, double* stats) {
  if (*flag) return;
  __shared__ double r0[kThreads], r1[kThreads];
  int tid = threadIdx.x;
  double a = 0, b = 0;
  for (int i = tid; i < nparts; i += kThreads) {
    a += partials[2 * i];
    b += partials[2 * i + 1];
  }
  r0[tid] = a;
  r1[tid] = b;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (tid < s) {
      r0[tid] += r0[tid + s];
      r1[tid] += r1[tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
    double rel = r1[0] > 0 ? sqrt(r0[0] / r1[0]) : 0.0;
    stats[2 + iter] = rel;
    stats[0] = iter;
    if (iter > 0 && rel <= tol) {
      stats[1] = 1;
      *flag = 1;
    }
  }
}

// ---------------------------------------------------------------------------
// Out-of-place transpose of a batch of R x C matrices: out[b][c][r] = in[b][r][c].
// 64 x 64 tiles through LDS (one padding column against bank conflicts);
// every global access is a contiguous 256-thread segment.
template <typename T>
__global__ __launch_bounds__(kThreads) void transpose_kernel(const T* __restrict__ in, T* __restrict__ out,
                                                             int64_t R, int64_t C, int64_t ntr, int64_t ntc) {
  constexpr int TS = 64;
  __shared__ T tile[TS][TS + 1];
  const int64_t bid = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t per = ntr * ntc;
  const int64_t b = bid / per;
  const int64_t rem = bid - b * per;
  const int64_t tr = rem / ntc, tc = rem - tr * ntc;
  const int64_t r0 = tr * TS, c0 = tc * TS;
  const T* src = in + b * R * C;
  T* dst = out + b * R * C;
  const int tx = threadIdx.x & (TS - 1), ty = threadIdx.x >> 6;  // 64 x 4
#pragma unroll
  for (int i = 0; i < TS; i += 4) {
    int64_t r = r0 + ty + i, c = c0 + tx;
    if (r < R && c < C) tile[ty + i][tx] = src[r * C + c];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < TS; i += 4) {
    int64_t c = c0 + ty + i, r = r0 + tx;
    if (r < R && c < C) dst[c * R + r] = tile[tx][ty + i];
  }
}

template <typename T>
hipError_t launch_transpose(const T* in, T* out, int64_t batch, int64_t R, int64_t C, hipStream_t s) {
  int64_t ntr = (R + 63) / 64, ntc = (C + 63) / 64;
  int64_t nb = batch * ntr * ntc;
  hipLaunchKernelGGL((transpose_kernel<T>), dim3((unsigned)nb), dim3(kThreads), 0, s, in, out, R, C, ntr, ntc);
  return hipGetLastError();
}
template hipError_t launch_transpose<float>(const float*, float*, int64_t, int64_t, int64_t, hipStream_t);
template hipError_t launch_transpose<double>(const double*, double*, int64_t, int64_t, int64_t, hipStream_t);

hipError_t launch_apply(int n, const ApplyArgs& a, int nblocks, size_t lds, hipStream_t s) {
  switch (n) {
#define FFTFEM_CASE(N)                                                                       \
  case N:                                                                                    \
    hipLaunchKernelGGL((apply_kernel<N>), dim3(nblocks), dim3(kThreads), lds, s, a);         \
    return hipGetLastError();
    FFTFEM_CASE(1)
    FFTFEM_CASE(2)
    FFTFEM_CASE(3)
    FFTFEM_CASE(4)
    FFTFEM_CASE(5)
    FFTFEM_CASE(6)
    FFTFEM_CASE(7)
    FFTFEM_CASE(8)
    FFTFEM_CASE(9)
#undef FFTFEM_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_reset(int* flag, double* stats, int nstats, hipStream_t s) {
  hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, s, flag, stats, nstats);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partials, int nparts, int iter, double tol, int* flag,
                         double* stats, hipStream_t s) {
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kThreads), 0, s, partials, nparts, iter, tol,
                     flag, stats);
  return hipGetLastError();
}

}  // namespace fftfem

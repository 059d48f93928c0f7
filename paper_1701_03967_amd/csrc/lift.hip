// Non-homogeneous Dirichlet data (Sect. 4 remark: a modified load), gfx950.
//
// With the dofs of the closed box (every axis extended by its two boundary
// points, E_d = n_d K_d + 1), the interior equations are
// A_II u_I = f - A_IB b_B.  A_IB b_B is the interior part of the extended
// tensor-sum operator applied to b with its interior set to zero; each term
// coef_t C x .. x A_t x .. x C (and react C x .. x C) is applied one axis at a
// time, each pass mapping the axis from its E_d extended points to its
// M_d = E_d - 2 interior rows by the element-wise 1D product.  One thread per
// output value; the axis' neighbours are strided by `inner`, so a wave's
// threads read consecutive values along the fastest axis.
#include <mutex>

#include "device_common.h"
#include "launch.h"

namespace fftfem {

// Work arrays of fftfem_dirichlet_load_noalloc: the axis passes' two
// intermediate arrays, in this file-scope device array instead of caller
// memory.  Each device holds its own copy for the life of the process.
static __device__ __align__(256) double scratch[kLiftScratchDoubles];

__global__ __launch_bounds__(kBlock) void lift_kernel(LiftArgs a) {
  const int n = a.n, K = a.K;
  const int64_t M = (int64_t)n * K - 1, E = (int64_t)n * K + 1;
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= a.outer * M * a.inner) return;
  const int64_t ii = t % a.inner, rest = t / a.inner;
  const int64_t i = rest % M, o = rest / M;
  const double* X = a.X;  // (n + 1) x (n + 1) element matrix, row-major
  auto x = [&](int64_t q) -> double {
    const int64_t flat = (o * E + q) * a.inner + ii;
    if (a.mask) {
      // extended input: interior points (every index in 1 .. E_d - 2) read as zero
      int64_t r = flat;
      bool interior = true;
      for (int d = a.N - 1; d >= 0; --d) {
        const int64_t c = r % a.ext[d];
        r /= a.ext[d];
        interior = interior && c >= 1 && c <= a.ext[d] - 2;
      }
      if (interior) return 0.0;
    }
    return a.in[flat];
  };
  double y = 0.0;
  if ((i + 1) % n != 0) {
    // bubble m (1 .. n - 1) of element e: row m of the element matrix
    const int64_t e = i / n;
    const int m = (int)(i % n) + 1;
    for (int k = 0; k <= n; ++k) y += X[m * (n + 1) + k] * x(e * n + k);
  } else {
    // node j: last row of element j - 1 plus first row of element j
    const int64_t j = (i + 1) / n;
    for (int k = 0; k <= n; ++k) y += X[n * (n + 1) + k] * x((j - 1) * n + k) + X[k] * x(j * n + k);
  }
  if (a.combine)
    a.out[t] = (a.f ? a.f[t] : a.out[t]) - a.scale * y;
  else
    a.out[t] = y;
}

hipError_t launch_lift(const LiftArgs& a, hipStream_t s) {
  if (a.n < 1 || a.K < 1 || a.outer < 1 || a.inner < 1) return hipErrorInvalidValue;
  const int64_t total = a.outer * ((int64_t)a.n * a.K - 1) * a.inner;
  const int64_t nb = (total + kBlock - 1) / kBlock;
  if (nb < 1) return hipSuccess;
  if (nb > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(lift_kernel, dim3((unsigned)nb), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

// Device address of `scratch` on the current device.  The array's name is a
// host-side stand-in in host code; its device address comes from
// hipGetSymbolAddress, taken once per device with that device current and
// kept.
hipError_t lift_scratch(double** ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static double* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = static_cast<double*>(p);
  }
  *ptr = addr[dev];
  return hipSuccess;
}

}  // namespace fftfem

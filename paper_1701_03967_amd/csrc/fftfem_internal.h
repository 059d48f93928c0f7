// Internal declarations shared by the host plan builder, the C ABI and the
// HIP kernels.  Not installed; the public interface is include/fftfem.h.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace fftfem {

// Per-axis tables produced on the host by the plan builder.
//
// Channel convention for one line of M = nK - 1 dofs (Sect. 2-3 of the paper):
//   nodal channel   x_j = y at node j, j = 1..K-1;
//   even channel m  (m = 1..n/2):      y_{j-1/2,m} + y_{j-1/2,n-m}  (just y_{j-1/2,m} if 2m = n);
//   odd channel m   (m = 1..(n-1)/2):  y_{j-1/2,m} - y_{j-1/2,n-m};   j = 1..K.
// Frequency k = 1..K-1 couples the nodal DST-I value at k, the even channels'
// DST-II value at k and the odd channels' DCT-II value at k; the bubble-only
// modes (k = 0) couple the even channels' DST-II value at k = K (alternating
// sum) and the odd channels' DCT-II value at k = 0 (plain sum).
// Q[k] (n x n, row = channel, column = mode) holds C-orthonormal eigenvectors
// of the projected pencil at frequency k, so that
//   forward:  w_l = sum_c Q[k][c][l] * chan_c(k)      (coefficients (y, s~))
//   inverse:  chan_c(k) = sum_l Q[k][c][l] * w_l.
struct AxisTables {
  int n = 0;
  int64_t K = 0;
  int64_t M = 0;
  double coef = 0.0;          // diff * 4 (K/X)^2
  std::vector<double> lam;    // M scaled eigenvalues, spectral order
  std::vector<double> Q;      // K blocks of n*n (block 0: (n-1)x(n-1) in the leading corner)
  std::vector<double> twf;    // K complex: exp(-2 pi i q / K)
  std::vector<double> twm;    // K complex: exp(-i pi k / (2K))
  std::vector<double> twd;    // K complex: exp(-i pi k / K)
  // K not a power of two with prime factors <= 7: the mixed-radix stages
  // (radices 16, 8, 4, 2 for the power of two, then 3, 5, 7; empty otherwise)
  std::vector<int> radices;
  // other K not a power of two: Bluestein's chirp-z tables (L = 0 otherwise)
  int64_t L = 0;              // power of two >= 2K - 1
  std::vector<double> chirp;  // K complex: exp(-i pi j^2 / K)
  std::vector<double> bhat;   // L complex: DFT_L of the conjugate chirp, / L
  std::vector<double> twl;    // L complex: exp(-2 pi i q / L)
  // condensed per-frequency solve of the fused middle pass (layout in
  // condensed_tables): ne^2 + no^2 + 3 (n - 1) + 2 values, unscaled
  std::vector<double> arrow;
  // banded solve along the axis (algorithm (b); layout in BandLayout), unscaled
  std::vector<double> band;
};

// Offsets into AxisTables::band (algorithm (b), the banded solve along an
// axis) for order n, nb = n - 1 bubbles: V (nb x nb, [bubble][mode],
// row-major: the mass-orthonormal eigenvectors of the element's bubble
// pencil in the physical bubble basis), lam (nb), then per mode V^T A_{B,0},
// V^T C_{B,0}, V^T A_{B,n}, V^T C_{B,n} (couplings to the element's left and
// right node), tL = 2 hAL hCL - hAL^2 / lam and tX = hAL hCR + hAR hCL -
// hAL hAR / lam, then C_00, C_0n and a0 = A_00 - sum_m hAL_m^2 / lam_m (the
// condensed stiffness' diagonal entry; its off-diagonal one is -a0).
struct BandLayout {
  int nb, V, lam, hAL, hCL, hAR, hCR, tL, tX, nn, size;
  explicit BandLayout(int n)
      : nb(n - 1), V(0), lam(nb * nb), hAL(lam + nb), hCL(hAL + nb), hAR(hCL + nb), hCR(hAR + nb),
        tL(hCR + nb), tX(tL + nb), nn(tX + nb), size(nn + 3) {}
};

// Offsets into AxisTables::arrow for order n.
struct ArrowLayout {
  int ne, no, nb, We, Wo, nu, gA, gC, cc, size;
  explicit ArrowLayout(int n)
      : ne(n / 2), no((n - 1) / 2), nb(n - 1), We(0), Wo(ne * ne), nu(Wo + no * no), gA(nu + nb),
        gC(gA + nb), cc(gC + nb), size(cc + 2) {}
};

// Builds the tables of one axis.  Returns 0 or a negative FFTFEM_* status.
int build_axis_tables(int n, int64_t K, double diff, double X, AxisTables* out);

// Reference-element matrices (n+1)^2, row-major, rounded from 113-bit values.
void element_matrices(int n, std::vector<double>* A, std::vector<double>* C);

// The same matrices as unevaluated sums hi + lo of doubles: 2 (n+1)^2 values
// each, the (n+1)^2 hi parts followed by the (n+1)^2 lo parts.
void element_matrices_dd(int n, std::vector<double>* A, std::vector<double>* C);

// Radices of a mixed-radix Stockham FFT of length K (K not a power of two,
// every prime factor <= 7); empty if K has a larger prime factor.
inline std::vector<int> mixed_radices(int64_t K) {
  std::vector<int> r;
  int64_t m = K;
  int twos = 0;
  while (m % 2 == 0) {
    m /= 2;
    ++twos;
  }
  int threes = 0, fives = 0, sevens = 0;
  while (m % 3 == 0) m /= 3, ++threes;
  while (m % 5 == 0) m /= 5, ++fives;
  while (m % 7 == 0) m /= 7, ++sevens;
  if (m != 1 || (threes + fives + sevens) == 0) return {};
  while (twos >= 4) r.push_back(16), twos -= 4;
  if (twos == 3) r.push_back(8);
  if (twos == 2) r.push_back(4);
  if (twos == 1) r.push_back(2);
  for (int i = 0; i < threes; ++i) r.push_back(3);
  for (int i = 0; i < fives; ++i) r.push_back(5);
  for (int i = 0; i < sevens; ++i) r.push_back(7);
  return r;
}

inline int num_even(int n) { return n / 2; }
inline int num_odd(int n) { return (n - 1) / 2; }

}  // namespace fftfem

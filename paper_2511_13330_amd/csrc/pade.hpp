// Pade degree / scaling selection and Neumann level count (shared by the
// 64 x 64 and block-tiled paths).
#pragma once
#include <hip/hip_runtime.h>

namespace lmag {

// theta_m (Higham 2005): largest ||A||_1 with backward error of r_m below the
// unit roundoff. Single precision uses m in {2, 3} (Pade-2 needs one product
// fewer than Pade-3 and covers the short slices of the spin workloads);
// double uses m in {3, 5, 7}. For these (m, theta) the denominator q_m(A) is
// column diagonally dominant (sum_j>=1 b_j theta^j < 1), so Gauss-Jordan needs
// no pivoting.
constexpr double c_theta32_2 = 8.093024022188482e-2;
constexpr double c_theta32_3 = 4.258730016922831e-1;
constexpr double c_theta64_3 = 1.495585217958292e-2, c_theta64_5 = 2.539398330063230e-1,
                 c_theta64_7 = 9.504178996162932e-1;

template <typename T>
__device__ __forceinline__ void choose_ms(double nrm, int& m, int& s) {
  s = 0;
  if constexpr (sizeof(T) == 4) {
    m = nrm <= c_theta32_2 ? 2 : 3;
    const double th = c_theta32_3;
    if (nrm > th) {
      s = (int)ceil(log2(nrm / th));
      while (s < 62 && ldexp(nrm, -s) > th) ++s;
    }
  } else {
    if (nrm <= c_theta64_3) m = 3;
    else if (nrm <= c_theta64_5) m = 5;
    else {
      m = 7;
      const double th = c_theta64_7;
      if (nrm > th) {
        s = (int)ceil(log2(nrm / th));
        while (s < 62 && ldexp(nrm, -s) > th) ++s;
      }
    }
  }
  if (!(nrm == nrm)) { m = 3; s = 0; }  // NaN input: propagate NaN, no scaling loop
  if (s < 0) s = 0;
  if (s > 62) s = 62;
}

// Levels K of the binary Neumann product Q^{-1} = (I+E)(I+E^2)...(I+E^{2^{K-1}}),
// E = I - q_m(A), from the bound ||E||_1 <= e = sum_{j>=1} b_j ||A||_1^j: the
// smallest K with e^{2^K} <= u (1 - e). 0 selects the Gauss-Jordan inverse.
template <typename T>
__device__ __forceinline__ int neumann_levels(double nA, const double* b, int m) {
  double e = 0.0, p = 1.0;
  for (int j = 1; j <= m; ++j) { p *= nA; e += b[j] * p; }
  const double u = sizeof(T) == 4 ? 5.9604644775390625e-8 : 1.1102230246251565e-16;
  const int kmax = sizeof(T) == 4 ? 4 : 5;
  if (!(e < 0.5)) return 0;
  double pe = e;   // e^(2^K)
  for (int K = 1; K <= kmax; ++K) {
    pe *= pe;
    if (pe <= u * (1.0 - e)) return K;
  }
  return 0;
}

// Power series of 1 / q_m(x), q_m(x) = sum_j (-1)^j b_j x^j (b_0 = 1):
// c_0 = 1, c_k = sum_{j=1}^{min(k,m)} (-1)^{j+1} b_j c_{k-j}.
__host__ __device__ inline void inv_series(const double* b, int m, double* c, int K) {
  c[0] = 1.0;
  for (int k = 1; k < K; ++k) {
    double v = 0.0;
    for (int j = 1; j <= m && j <= k; ++j) v += ((j & 1) ? b[j] : -b[j]) * c[k - j];
    c[k] = v;
  }
}

// Tail sum_{k > D} |c_k| x^k of the series of 1/q_m (48 terms; at the x where
// it is used the terms fall by more than a factor 4 per degree).
__host__ __device__ inline double inv_series_tail(const double* b, int m, int D, double x) {
  double c[48];
  inv_series(b, m, c, 48);
  double tail = 0.0, p = 1.0;
  for (int k = 1; k < 48; ++k) {
    p *= x;
    if (k > D) tail += fabs(c[k]) * p;
  }
  return tail;
}

// Power series of r_m(x) = p_m(x) / q_m(x), p_m(x) = sum_j b_j x^j:
// rho_k = sum_{j=0}^{min(k,m)} b_j c_{k-j} with c the series of 1/q_m. The
// [m/m] approximant matches e^x through degree 2m, so rho_k = 1/k! for k <= 2m.
__host__ __device__ inline void pade_series(const double* b, int m, double* rho, int K) {
  double c[48];
  inv_series(b, m, c, K < 48 ? K : 48);
  for (int k = 0; k < K && k < 48; ++k) {
    double v = 0.0;
    for (int j = 0; j <= m && j <= k; ++j) v += b[j] * c[k - j];
    rho[k] = v;
  }
}

// Tail sum_{k > D} |rho_k| x^k of the series of r_m (48 terms, as above).
__host__ __device__ inline double pade_series_tail(const double* b, int m, int D, double x) {
  double rho[48];
  pade_series(b, m, rho, 48);
  double tail = 0.0, p = 1.0;
  for (int k = 1; k < 48; ++k) {
    p *= x;
    if (k > D) tail += fabs(rho[k]) * p;
  }
  return tail;
}

// Largest ||A||_1 for which a truncated series has tail <= u / 2 in single
// precision: the degree-D series of r_m (of_r = true) or of 1/q_m. The tail
// increases with ||A||_1, so a slice may use the series exactly when its norm
// is at most this limit (bisection, host side).
inline double series_limit32(const double* b, int m, int D, bool of_r) {
  const double u = 5.9604644775390625e-8;
  double lo = 0.0, hi = 1.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    const double t = of_r ? pade_series_tail(b, m, D, mid) : inv_series_tail(b, m, D, mid);
    if (t <= 0.5 * u) lo = mid; else hi = mid;
  }
  return lo;
}

// Series degree used for each single-precision Pade degree. m = 2: r_2 itself
// at degree 4 (r_2 agrees with e^x through degree 4, so the truncation is the
// degree-4 Taylor polynomial; beyond theta_2 = 0.0809 it is not used), one
// product after A^2. m = 3: 1/q_3 at degree 5, A^4 and one product with A.
constexpr int series_degree(int m) { return m == 2 ? 4 : 5; }

// How a slice evaluates r_m(A) (code stored with the slice):
//   16 + D  single precision, D = series_degree(m): m = 2, r_2(A) by its
//           power series truncated at degree D; m = 3, r_3 = q_3^{-1} p_3 with
//           q_3^{-1} by its series truncated at degree D. Used when the tail
//           of that series at ||A||_1 is <= u / 2, i.e. when ||A||_1 <= the
//           limit for that m;
//   1..5    r_m = q_m^{-1} p_m, binary Neumann product with that many levels;
//   0       r_m = q_m^{-1} p_m, Gauss-Jordan.
template <typename T>
__device__ __forceinline__ int inverse_code(double nA, const double* b, int m, int allow_series,
                                            double ser_max2, double ser_max3) {
  if (sizeof(T) == 4 && allow_series && ((m == 2 && nA <= ser_max2) || (m == 3 && nA <= ser_max3)))
    return 16 + series_degree(m);
  return neumann_levels<T>(nA, b, m);
}

// Block-tiled path: single precision; Pade 2 (evaluated by its degree-4
// series, no scaling) or Pade 3 with scaling, as in the 64 x 64 kernels.
template <typename T>
__device__ __forceinline__ void big_choose_ms(double nrm, int& m, int& s) {
  choose_ms<T>(nrm, m, s);
}

template <typename T>
__device__ __forceinline__ int big_neumann_levels(double nA, const double* b3) {
  return neumann_levels<T>(nA, b3, 3);
}

}  // namespace lmag

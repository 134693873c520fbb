// Optimiser step for the pulse amplitudes: Adam (Kingma & Ba 2015, Alg. 1) on
// grad_scale * g, followed by projection onto [lo, hi] (the paper optimises the
// control coefficients with Adam, Sec. III-C). One thread per amplitude.
#include "tile.hpp"
#include "internal.hpp"

namespace lmag {

template <typename T>
__global__ void k_adam_project(AdamArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int64_t row = i / a.row_len;
  if (a.row_active && !a.row_active[row]) return;
  T* th = (T*)a.theta;
  T* m = (T*)a.m;
  T* v = (T*)a.v;
  const double g = a.grad_scale * (double)((const T*)a.grad)[i];
  const double mn = a.beta1 * (double)m[i] + (1.0 - a.beta1) * g;
  const double vn = a.beta2 * (double)v[i] + (1.0 - a.beta2) * g * g;
  const double mhat = mn / a.bc1, vhat = vn / a.bc2;
  double x = (double)th[i] - a.lr * mhat / (sqrt(vhat) + a.eps);
  x = fmin(fmax(x, a.lo), a.hi);
  m[i] = (T)mn;
  v[i] = (T)vn;
  th[i] = (T)x;
}

hipError_t launch_adam_project(int prec, const AdamArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  const dim3 g((unsigned)((a.n + 255) / 256));
  if (prec == 32) hipLaunchKernelGGL(k_adam_project<float>, g, dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_adam_project<double>, g, dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace lmag

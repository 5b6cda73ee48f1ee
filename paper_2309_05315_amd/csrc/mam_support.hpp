// Support step of the fixed-support approach (Sec. 2; the closed form of the
// free-support proposition, Prop. 4):
//
//   mass_r = sum_m alpha_m sum_s pi^(m)_rs,
//   xi_r   = sum_m alpha_m sum_s pi^(m)_rs zeta^(m)_s / mass_r   (mass_r > 0),
//
// from the plans pi^(m) = pi_hat^(m) of the iteration that just ran, rebuilt
// from the stored theta' = pi_hat - b^(m): pi_hat_rs = theta'_rs + b^(m)_r with
// b^(m)_r = t (p_r - p^(m)_r) / S^m of that iteration's starting marginals.
// An entry stored as exactly -b^(m)_r (rounded to the storage type) is an
// inactive one and counts as 0.
//
// Two passes, both in fixed orders (bitwise reproducible):
//   support_partial_kernel  one thread per row, one workgroup per (row block,
//       chunk of columns of one measure): the chunk's sums of pi_hat and of
//       pi_hat * zeta_s, streaming theta once (one coalesced load per column);
//   support_final_kernel    per row, the chunks' partials weighted by alpha_m in
//       chunk order, then the quotient.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mam {

constexpr int SUP_NT = 256;   // rows per workgroup of the partial pass
constexpr int SUP_MAXD = 3;   // largest point dimension

template <typename T>
struct SupArgs {
  const T* theta;
  int64_t ld;
  int64_t R;
  int32_t dim, nchunks;
  const int32_t* ch_m;       // chunk -> measure
  const int64_t* ch_j0;      // chunk -> first column (global)
  const int64_t* ch_j1;      // chunk -> one past its last column
  const double* alpha;       // chunk -> alpha of its measure
  const double* zeta;        // T x dim, column j's point at j*dim
  const double* p_prev;      // R: p of the iteration's start
  const double* pm_prev;     // M x R: p^(m) of the iteration's start
  const double* Sd;          // M
  const double* t;           // the iteration's t
  double* partial;           // nchunks x (dim+1) x R
  double* xi;                // R x dim, in/out
  double* mass;              // R, or null
};

template <typename T>
__global__ void __launch_bounds__(SUP_NT) support_partial_kernel(SupArgs<T> a) {
  const int64_t r = (int64_t)blockIdx.x * SUP_NT + threadIdx.x;
  const int c = blockIdx.y;
  if (r >= a.R) return;
  const int m = a.ch_m[c];
  const int64_t j0 = a.ch_j0[c], j1 = a.ch_j1[c];
  const int dim = a.dim;
  const double b = a.t[0] * (a.p_prev[r] - a.pm_prev[(size_t)m * a.R + r]) / a.Sd[m];
  const T nb = (T)(-b);
  double den = 0.0, num[SUP_MAXD] = {0.0, 0.0, 0.0};
  const T* __restrict__ th = a.theta + r;
  const double* __restrict__ z = a.zeta;
  int64_t j = j0;
  // eight columns' loads in flight per step
  for (; j + 8 <= j1; j += 8) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = th[(j + u) * a.ld];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double pi = v[u] == nb ? 0.0 : (double)v[u] + b;
      den += pi;
#pragma unroll
      for (int k = 0; k < SUP_MAXD; ++k)
        if (k < dim) num[k] += pi * z[(j + u) * dim + k];
    }
  }
  for (; j < j1; ++j) {
    const T v = th[j * a.ld];
    const double pi = v == nb ? 0.0 : (double)v + b;
    den += pi;
#pragma unroll
    for (int k = 0; k < SUP_MAXD; ++k)
      if (k < dim) num[k] += pi * z[j * dim + k];
  }
  double* out = a.partial + (size_t)c * (dim + 1) * a.R;
  out[r] = den;
#pragma unroll
  for (int k = 0; k < SUP_MAXD; ++k)
    if (k < dim) out[(size_t)(k + 1) * a.R + r] = num[k];
}

template <typename T>
__global__ void __launch_bounds__(256) support_final_kernel(SupArgs<T> a) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= a.R) return;
  const int dim = a.dim;
  double den = 0.0, num[SUP_MAXD] = {0.0, 0.0, 0.0};
  for (int c = 0; c < a.nchunks; ++c) {
    const double al = a.alpha[c];
    const double* in = a.partial + (size_t)c * (dim + 1) * a.R;
    den += al * in[r];
#pragma unroll
    for (int k = 0; k < SUP_MAXD; ++k)
      if (k < dim) num[k] += al * in[(size_t)(k + 1) * a.R + r];
  }
  if (a.mass) a.mass[r] = den;
  if (den > 0.0) {
#pragma unroll
    for (int k = 0; k < SUP_MAXD; ++k)
      if (k < dim) a.xi[r * dim + k] = num[k] / den;
  }
}

}  // namespace mam

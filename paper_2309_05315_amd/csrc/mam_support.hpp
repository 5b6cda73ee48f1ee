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
//   support_partial_kernel  V rows per thread (one 16-byte vector), one
//       workgroup per (row block, chunk of columns of one measure): the
//       chunk's sums of pi_hat and of pi_hat * zeta_s, streaming theta once;
//   support_final_kernel    per row, the chunks' partials weighted by alpha_m in
//       chunk order, then the quotient.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mam_kernels.hpp"

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

// V: rows per thread, 1 or one 16-byte vector (4 FP32 or 2 FP64 values; then
// ld is a multiple of V and theta 16-byte aligned, so a vector never leaves
// its column's ld entries; rows past R are loaded but not used).
template <typename T, int V>
__global__ void __launch_bounds__(SUP_NT) support_partial_kernel(SupArgs<T> a) {
  constexpr int U = 8;  // columns whose loads are in flight per step
  const int64_t r0 = ((int64_t)blockIdx.x * SUP_NT + threadIdx.x) * V;
  const int c = blockIdx.y;
  if (r0 >= a.R) return;
  const int m = a.ch_m[c];
  const int64_t j0 = a.ch_j0[c], j1 = a.ch_j1[c];
  const int dim = a.dim;
  const double t = a.t[0], Sm = a.Sd[m];
  const double* __restrict__ pmm = a.pm_prev + (size_t)m * a.R;
  double b[V];
  T nb[V];
#pragma unroll
  for (int e = 0; e < V; ++e) {
    const int64_t r = r0 + e < a.R ? r0 + e : r0;
    b[e] = t * (a.p_prev[r] - pmm[r]) / Sm;
    nb[e] = (T)(-b[e]);
  }
  double den[V], num[V][SUP_MAXD];
#pragma unroll
  for (int e = 0; e < V; ++e) {
    den[e] = 0.0;
#pragma unroll
    for (int k = 0; k < SUP_MAXD; ++k) num[e][k] = 0.0;
  }
  const T* __restrict__ th = a.theta + r0;
  const double* __restrict__ z = a.zeta;
  auto add = [&](const T (&v)[V], int64_t j) {
    double zk[SUP_MAXD];
#pragma unroll
    for (int k = 0; k < SUP_MAXD; ++k) zk[k] = k < dim ? z[j * dim + k] : 0.0;
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const double pi = v[e] == nb[e] ? 0.0 : (double)v[e] + b[e];
      den[e] += pi;
#pragma unroll
      for (int k = 0; k < SUP_MAXD; ++k)
        if (k < dim) num[e][k] += pi * zk[k];
    }
  };
  int64_t j = j0;
  for (; j + U <= j1; j += U) {
    T v[U][V];
#pragma unroll
    for (int u = 0; u < U; ++u) load_vec_nt<T, V>(th + (j + u) * a.ld, v[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) add(v[u], j + u);
  }
  for (; j < j1; ++j) {
    T v[V];
    load_vec_nt<T, V>(th + j * a.ld, v);
    add(v, j);
  }
#pragma unroll
  for (int e = 0; e < V; ++e) {
    if (r0 + e >= a.R) continue;
    double* out = a.partial + (size_t)c * (dim + 1) * a.R + r0 + e;
    out[0] = den[e];
#pragma unroll
    for (int k = 0; k < SUP_MAXD; ++k)
      if (k < dim) out[(size_t)(k + 1) * a.R] = num[e][k];
  }
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

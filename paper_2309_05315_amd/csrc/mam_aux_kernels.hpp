// Device code of the MAM library outside the column kernel: the marginal
// and average kernels that close each iteration, initialisation, input
// checks and the cost helper.  Included only by the host translation unit.
#pragma once

#include "mam_kernels.hpp"

namespace mam {

// p^(m)_r = sum over the segments of measure m (in schedule order).
__global__ void __launch_bounds__(256)
marginal_kernel(const double* __restrict__ partial, int R, const int32_t* __restrict__ mseg,
                const int32_t* __restrict__ seg_idx, double* __restrict__ pm, double* __restrict__ pm_prev,
                int save_prev) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  const int m = blockIdx.y;
  if (r >= R) return;
  double s = 0.0;
  const int e = mseg[m + 1];
  for (int i = mseg[m]; i < e; ++i) s += partial[(size_t)seg_idx[i] * R + r];
  const size_t o = (size_t)m * R + r;
  if (save_prev) pm_prev[o] = pm[o];
  pm[o] = s;
}

// p_r = sum_m a_m p^(m)_r and per-block partials of sum_r sum_m (p_r - p^(m)_r)^2 / S^m.
__global__ void __launch_bounds__(256)
average_kernel(const double* __restrict__ pm, int R, int M, const double* __restrict__ aw,
               const double* __restrict__ Sd, double* __restrict__ p, double* __restrict__ p_prev,
               int save_prev, double* __restrict__ d2part) {
  __shared__ double sh[4];
  const int r = blockIdx.x * 256 + threadIdx.x;
  double d2 = 0.0;
  if (r < R) {
    double pr = 0.0;
    for (int m = 0; m < M; ++m) pr += aw[m] * pm[(size_t)m * R + r];
    for (int m = 0; m < M; ++m) {
      const double e = pr - pm[(size_t)m * R + r];
      d2 += e * e / Sd[m];
    }
    if (save_prev) p_prev[r] = p[r];
    p[r] = pr;
  }
  d2 = wave_sum(d2);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = d2;
  __syncthreads();
  if (threadIdx.x == 0) d2part[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// theta^0_rs = q_s / R (Alg. 1 Step 0 with the library's default start).
template <typename T>
__global__ void __launch_bounds__(256)
fill_kernel(T* __restrict__ theta, int64_t ld, int R, const T* __restrict__ q, int64_t T_cols) {
  const int64_t total = T_cols * (int64_t)R;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
    const int64_t j = i / R;
    const int r = (int)(i - j * R);
    theta[j * ld + r] = (T)((double)q[j] / (double)R);
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
copy_kernel(T* __restrict__ theta, int64_t ld, int R, const T* __restrict__ src, int64_t T_cols) {
  const int64_t total = T_cols * (int64_t)R;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
    const int64_t j = i / R;
    const int r = (int)(i - j * R);
    theta[j * ld + r] = src[j * ld + r];
  }
}

// Row sums of the plans into the segment partials (used by initialisation).
template <typename T>
__global__ void __launch_bounds__(256)
rowsum_kernel(const T* __restrict__ theta, int64_t ld, int R, const int64_t* __restrict__ seg_j0,
              const int64_t* __restrict__ seg_j1, const int32_t* __restrict__ wg_seg,
              double* __restrict__ partial) {
  const int wg = blockIdx.x;
  for (int si = wg_seg[wg]; si < wg_seg[wg + 1]; ++si) {
    for (int r = threadIdx.x; r < R; r += 256) {
      double s = 0.0;
      for (int64_t j = seg_j0[si]; j < seg_j1[si]; ++j) s += (double)theta[j * ld + r];
      partial[(size_t)si * R + r] = s;
    }
  }
}

// Input validation: per-measure mass of q (fixed order) and a flag for any
// negative or non-finite weight, or non-finite cost entry.
template <typename T>
__global__ void __launch_bounds__(256)
check_q_kernel(const T* __restrict__ q, const int64_t* __restrict__ col_off, double* __restrict__ out,
               int M) {
  __shared__ double sh[4];
  const int m = blockIdx.x;
  double s = 0.0;
  bool bad = false;
  for (int64_t j = col_off[m] + threadIdx.x; j < col_off[m + 1]; j += 256) {
    const double v = (double)q[j];
    bad |= !(v >= 0.0) || __builtin_isinf(v);
    s += v;
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  if (bad) out[M] = 1.0;
  __syncthreads();
  if (threadIdx.x == 0) out[m] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

template <typename T>
__global__ void __launch_bounds__(256)
check_cost_kernel(const T* __restrict__ cost, int64_t cost_ld, int R, int64_t ncols,
                  double* __restrict__ flag) {
  const int64_t total = ncols * (int64_t)R;
  bool bad = false;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
    const int64_t j = i / R;
    const int r = (int)(i - j * R);
    const double v = (double)cost[j * cost_ld + r];
    bad |= !(v == v) || __builtin_isinf(v);
  }
  if (bad) flag[0] = 1.0;
}

__global__ void __launch_bounds__(256)
check_index_kernel(const int32_t* __restrict__ idx, int64_t n, int64_t ncols, double* __restrict__ flag) {
  bool bad = false;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    bad |= idx[i] < 0 || idx[i] >= ncols;
  if (bad) flag[0] = 1.0;
}

// Squared Euclidean cost; the max is reduced with an integer max on the bit
// pattern (non-negative doubles order like their bits), which is exact.
__global__ void __launch_bounds__(256)
sqdist_kernel(const double* __restrict__ xi, int R, const double* __restrict__ zeta, int64_t S,
              int dim, double* __restrict__ tmp_max, int want_max) {
  const int64_t total = (int64_t)R * S;
  double mx = 0.0;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
    const int64_t s = i / R;
    const int r = (int)(i - s * R);
    double d = 0.0;
    for (int k = 0; k < dim; ++k) {
      const double e = xi[(int64_t)r * dim + k] - zeta[s * dim + k];
      d += e * e;
    }
    mx = fmax(mx, d);
  }
  if (want_max) {
    mx = wave_max(mx);
    if ((threadIdx.x & 63) == 0)
      atomicMax(reinterpret_cast<unsigned long long*>(tmp_max),
                (unsigned long long)__double_as_longlong(mx));
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
cost_write_kernel(const double* __restrict__ xi, int R, const double* __restrict__ zeta, int64_t S,
                  int dim, const double* __restrict__ tmp_max, int normalize, T* __restrict__ out,
                  int64_t out_ld) {
  const int64_t total = (int64_t)R * S;
  const double scale = normalize ? tmp_max[0] : 1.0;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
    const int64_t s = i / R;
    const int r = (int)(i - s * R);
    double d = 0.0;
    for (int k = 0; k < dim; ++k) {
      const double e = xi[(int64_t)r * dim + k] - zeta[s * dim + k];
      d += e * e;
    }
    out[s * out_ld + r] = (T)(normalize ? d / scale : d);
  }
}

__global__ void __launch_bounds__(256)
fill_value_kernel(double* __restrict__ p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = v;
}

__global__ void zero_kernel(double* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

}  // namespace mam

// Device code of the MAM library outside the column kernel: the marginal
// and average kernels that close each iteration, initialisation, input
// checks and the cost helper.  Included only by the host translation unit.
#pragma once

#include "mam_adjoint.hpp"
#include "mam_kernels.hpp"
#include "mam_long.hpp"

namespace mam {

// p^(m)_r = sum over the segments of measure m, in schedule order.  The
// partials' offsets come as one list per measure, or per (measure, row tile)
// for long columns (mpoff[mseg[k] .. mseg[k+1]), k = the task's list);
// they are wave-uniform, and the partial loads are issued eight at a time so
// the loop is not a chain of dependent loads.  The additions keep the list
// order.
__global__ void __launch_bounds__(256)
marginal_kernel(const MargTask* __restrict__ tasks, const ProbAux* __restrict__ probs,
                const int32_t* __restrict__ mseg, const int64_t* __restrict__ mpoff,
                const double* __restrict__ partial, int save_prev, const int32_t* __restrict__ stop) {
  if (stop != nullptr && *stop != 0) return;  // early exit: the run has stopped
  const MargTask tk = tasks[blockIdx.x];
  const ProbAux& P = probs[tk.prob];
  const int R = uniform_i(P.R);
  const int r = tk.r0 + threadIdx.x;
  const int k = uniform_i(P.mbase) + tk.list;
  const int b = uniform_i(mseg[k]), e = uniform_i(mseg[k + 1]);
  constexpr int U = 8;
  double s = 0.0;
  const int rr = r < R ? r : tk.r0;  // rows past R read the task's first row (in bounds) and store nothing
  for (int i = b; i < e; i += U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t off = i + u < e ? uniform_l(mpoff[i + u]) : -1;
      v[u] = off >= 0 ? partial[off + rr] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i + u < e) s += v[u];
  }
  if (r >= R) return;
  const size_t o = (size_t)tk.m * R + r;
  double* const pm = gptr(P.pm);
  if (save_prev) gptr(P.pm_prev)[o] = pm[o];
  pm[o] = s;
}

// Short columns: the new marginals (close_marginal) of every task's rows.
__global__ void __launch_bounds__(256)
fixed_marginal_kernel(const MargTask* __restrict__ tasks, const ProbAux* __restrict__ probs, int save_prev,
                      const int32_t* __restrict__ stop) {
  // the stop flag and the task requested together (an early exit then adds
  // no memory latency in front of the work)
  const int stopv = stop != nullptr ? *stop : 0;
  const MargTask tk = tasks[blockIdx.x];
  if (stopv != 0) return;  // early exit: the run has stopped
  close_marginal(tk, probs[tk.prob], save_prev, threadIdx.x);
}

// Short columns, at the start: p^(m)_r = sum_s theta_rs in double (theta of
// the caller's start, or q_s/R).  A workgroup takes one task (a measure, 256
// rows); wave w sums the columns j0 + w, j0 + w + 4, ... in order, VEC rows
// per lane per load and U columns in flight, and the four waves' sums are
// added in wave order: a fixed order, so the result is reproducible.
template <typename T, int VEC>
__global__ void __launch_bounds__(256)
init_marginal_kernel(const MargTask* __restrict__ tasks, const ProbDev<T>* __restrict__ probs,
                     const ProbAux* __restrict__ aux) {
  constexpr int PASSES = 256 / (64 * VEC);  // row passes of a wave over the task's 256 rows
  constexpr int U = 8;
  __shared__ double part[4][256];
  const MargTask tk = tasks[blockIdx.x];
  const ProbDev<T>& P = probs[tk.prob];
  const int R = uniform_i(P.R);
  const int wv = uniform_i((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
  const T* const theta = gptr((const T*)uniform_l((int64_t)P.theta));
  const int64_t ld = uniform_l(P.ld);
  const int64_t j0 = uniform_l(gptr(P.col_off)[tk.m]), j1 = uniform_l(gptr(P.col_off)[tk.m + 1]);
  double s[PASSES][VEC];
  int rows[PASSES];
#pragma unroll
  for (int ps = 0; ps < PASSES; ++ps) {
    const int r0 = tk.r0 + (ps * 64 + lane) * VEC;
    rows[ps] = r0 < R ? r0 : tk.r0;  // vectors past R read the task's first rows and are not stored
#pragma unroll
    for (int v = 0; v < VEC; ++v) s[ps][v] = 0.0;
  }
  for (int64_t j = j0 + wv; j < j1; j += 4 * U) {
    T x[U][PASSES][VEC];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t jj = j + 4 * u < j1 ? j + 4 * u : j0;
#pragma unroll
      for (int ps = 0; ps < PASSES; ++ps) load_vec<T, VEC>(theta + jj * ld + rows[ps], x[u][ps]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (j + 4 * u < j1) {
#pragma unroll
        for (int ps = 0; ps < PASSES; ++ps)
#pragma unroll
          for (int v = 0; v < VEC; ++v) s[ps][v] += (double)x[u][ps][v];
      }
  }
#pragma unroll
  for (int ps = 0; ps < PASSES; ++ps)
#pragma unroll
    for (int v = 0; v < VEC; ++v) part[wv][(ps * 64 + lane) * VEC + v] = s[ps][v];
  __syncthreads();
  const int t = threadIdx.x, r = tk.r0 + t;
  if (r < R) gptr(aux[tk.prob].pm)[(size_t)tk.m * R + r] = ((part[0][t] + part[1][t]) + part[2][t]) + part[3][t];
}

// Short columns: Steps 3 and 1 of every task's block of 256 rows (close_rows).
__global__ void __launch_bounds__(256)
close_kernel(const AvgTask* __restrict__ tasks, const ProbAux* __restrict__ probs, int save_prev,
             const int32_t* __restrict__ stop) {
  __shared__ double sh[4];
  const int stopv = stop != nullptr ? *stop : 0;  // requested with the task
  const AvgTask tk = tasks[blockIdx.x];
  if (stopv != 0) return;  // early exit: the run has stopped
  close_rows(tk, probs[tk.prob], save_prev, threadIdx.x, sh);
}

// Step 1 for every task's block of 256 rows (close_average).
__global__ void __launch_bounds__(256)
average_kernel(const AvgTask* __restrict__ tasks, const ProbAux* __restrict__ probs, int save_prev,
               const int32_t* __restrict__ stop) {
  __shared__ double sh[4];
  const int stopv = stop != nullptr ? *stop : 0;  // requested with the task
  const AvgTask tk = tasks[blockIdx.x];
  if (stopv != 0) return;  // early exit: the run has stopped
  close_average(tk, probs[tk.prob], save_prev, threadIdx.x, sh);
}

// ---------------------------------------------------------------------------
// On-device stopping tests (Sec. 5, stopping criteria).  A run evaluates one
// test after every check iteration; once it holds, the stop flag is set and
// every later gated launch of the run (column, marginal, average and these
// kernels) returns at once, so the plans stay at the iterate that passed.
// ---------------------------------------------------------------------------
constexpr int STOP_DTHETA = 0;  // ||theta^{k+1} - theta^k||_inf (the column kernel's diagnostics)
constexpr int STOP_DP = 1;      // ||p^{k+1} - p^k||_2
constexpr int STOP_DIST = 2;    // dist_L(pi_hat^k)

struct StopState {
  int32_t stop;    // 1 once the test held
  int32_t pad;
  int64_t checks;  // checks evaluated since the reset
  double value;    // the test's value at the last check (NaN before any)
  double tol;
};

__global__ void stop_reset_kernel(StopState* __restrict__ st, double tol) {
  if (threadIdx.x == 0) {
    st->stop = 0;
    st->pad = 0;
    st->checks = 0;
    st->value = __builtin_nan("");
    st->tol = tol;
  }
}

// Per-block partial sums (256 rows a block) of the squared value of a test
// that the marginals decide.  After a check iteration p and p^(m) hold the
// new values, p_prev and pm_prev the ones the iteration started from, and
// t_out its damping.
//   STOP_DP:   sum_r (p_r - p_prev_r)^2
//   STOP_DIST: the row sums of pi_hat^(m) are ph^(m) = p^(m) + t (p_prev - pm_prev^(m))
//              (Step 2 subtracts t b^(m) from every column), and
//              dist_L(pi_hat)^2 = sum_m ||ph - ph^(m)||^2 / S^m, ph = sum_m a_m ph^(m).
__global__ void __launch_bounds__(256)
stop_partial_kernel(const ProbAux* __restrict__ probs, const double* __restrict__ t_out, int test,
                    double* __restrict__ part, const StopState* __restrict__ st) {
  if (st->stop != 0) return;
  __shared__ double sh[4];
  const ProbAux& P = probs[0];
  const int R = P.R, M = P.M;
  const int r = blockIdx.x * 256 + threadIdx.x;
  double v = 0.0;
  if (r < R) {
    const double* const pm = gptr(P.pm);
    const double* const pmp = gptr(P.pm_prev);
    const double pr = gptr(P.p)[r], pp = gptr(P.p_prev)[r];
    if (test == STOP_DP) {
      v = (pr - pp) * (pr - pp);
    } else {
      const double t = *t_out;
      double ph = 0.0;
      for (int m = 0; m < M; ++m)
        ph += P.aw[m] * (pm[(size_t)m * R + r] + t * (pp - pmp[(size_t)m * R + r]));
      for (int m = 0; m < M; ++m) {
        const double e = ph - (pm[(size_t)m * R + r] + t * (pp - pmp[(size_t)m * R + r]));
        v += e * e / P.Sd[m];
      }
    }
  }
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// Finish a check (one workgroup of 256): the test's value from the
// partials (fixed order) or from the column kernel's per-workgroup maxima
// of |theta^{k+1} - theta^k|; count the check; set the flag when
// value <= tol (a NaN value never stops), also in the host-visible word.
__global__ void __launch_bounds__(256)
stop_final_kernel(StopState* __restrict__ st, int test, const double* __restrict__ part, int nparts,
                  const double* __restrict__ diag, int nwg, int32_t* __restrict__ host_flag) {
  __shared__ double sh[4];
  if (st->stop != 0) return;
  double v;
  if (test == STOP_DTHETA) {
    double mx = 0.0;
    for (int i = threadIdx.x; i < nwg; i += 256) mx = fmax(mx, diag[(size_t)i * DIAG_STRIDE + 2]);
    mx = wave_max(mx);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
    __syncthreads();
    v = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
  } else {
    double s = 0.0;
    for (int i = 0; i < nparts; ++i) s += part[i];
    v = sqrt(s);
  }
  if (threadIdx.x == 0) {
    st->checks += 1;
    st->value = v;
    if (v <= st->tol) {
      st->stop = 1;
      if (host_flag) *reinterpret_cast<volatile int32_t*>(host_flag) = 1;
    }
  }
}

// ---- long-column iterations (the tile kernels are in mam_long.hpp) ----
// t^k from the d^2 partials (Alg. 1 Step 1), one workgroup, fixed order.
__global__ void __launch_bounds__(256)
damping_kernel(const double* __restrict__ d2part, int nb, double rho, double gamma, double* __restrict__ t_out,
               const int32_t* __restrict__ stop) {
  if (stop != nullptr && *stop != 0) return;
  __shared__ double sh[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) s += d2part[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double d2 = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    t_out[0] = (__builtin_isinf(gamma) || rho * sqrt(d2) <= gamma) ? 1.0 : gamma / (rho * sqrt(d2));
  }
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

// The R stored rows of T_cols columns at stride ld, src to dst (padding
// rows untouched): workgroups take columns in turn, a thread moves VEC
// elements per access with four accesses in flight.
template <typename T, int VEC>
__global__ void __launch_bounds__(256)
copy_kernel(T* __restrict__ dst, int64_t ld, int R, const T* __restrict__ src, int64_t T_cols) {
  constexpr int U = 4;
  for (int64_t j = blockIdx.x; j < T_cols; j += gridDim.x) {
    const T* __restrict__ s = src + j * ld;
    T* __restrict__ d = dst + j * ld;
    for (int r0 = (int)threadIdx.x * VEC; r0 < R; r0 += 256 * VEC * U) {
      T v[U][VEC];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int r = r0 + u * 256 * VEC;
        if (r + VEC <= R) load_vec<T, VEC>(s + r, v[u]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int r = r0 + u * 256 * VEC;
        if (r + VEC <= R) {
          store_vec<T, VEC>(d + r, v[u]);
        } else {
          for (int k = r; k < R; ++k) d[k] = s[k];  // the column's last rows
        }
      }
    }
  }
}

// Bandwidth probe: n16 blocks of 16 bytes from src to dst, non-temporal
// loads and stores, grid-stride (every workgroup steps over the whole range,
// so the blocks in flight at any time lie together in memory).
__global__ void __launch_bounds__(256)
stream_copy_kernel(const f4nt* __restrict__ src, f4nt* __restrict__ dst, int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
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

// ||xi_r - zeta_s||^2 as the sum of rounded squares in axis order (no fused
// multiply-add), so it equals the plain evaluation of the definition.
__device__ __forceinline__ double sq_dist(const double* __restrict__ xi, int r,
                                          const double* __restrict__ zeta, int64_t s, int dim) {
#pragma clang fp contract(off)
  double d = 0.0;
  for (int k = 0; k < dim; ++k) {
    const double e = xi[(int64_t)r * dim + k] - zeta[s * dim + k];
    d += e * e;
  }
  return d;
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
    const double d = sq_dist(xi, r, zeta, s, dim);
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
    const double d = sq_dist(xi, r, zeta, s, dim);
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

// ---- reverse mode (see mam_adjoint.hpp for the step) ----

// Transposed averaging of one reverse step, per row r:
//   bbar_m = 2 W_new - W_old - S^m V_m,  pbar = sum_m bbar_m / S^m,
//   V_m <- -bbar_m / S^m + a_m pbar,  W_old <- W_new,
// and the bound of |V| for the next step.
__global__ void __launch_bounds__(256)
adjoint_average_kernel(unsigned long long* __restrict__ wacc, double* __restrict__ wold, double* __restrict__ V,
                       const double* __restrict__ Sd, const double* __restrict__ aw, int R, int M,
                       unsigned long long* __restrict__ mx, int slot, double smax) {
  const AdjScale sc = adj_scale(mx, slot, smax);
  const int r = blockIdx.x * 256 + threadIdx.x;
  double vmx = 0.0;
  if (r < R) {
    // eight measures' loads in flight at a time (a row's values are a chain
    // of dependent steps otherwise); the sums keep the order m = 0, 1, ...
    constexpr int U = 8;
    double pbar = 0.0;
    for (int m0 = 0; m0 < M; m0 += U) {
      unsigned long long wa[U];
      double wo[U], vv[U], sd[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const size_t o = (size_t)(m0 + u) * R + r;
        const bool in = m0 + u < M;
        wa[u] = in ? wacc[o] : 0ull;
        wo[u] = in ? wold[o] : 0.0;
        vv[u] = in ? V[o] : 0.0;
        sd[u] = in ? Sd[m0 + u] : 1.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (m0 + u < M) {
          const size_t o = (size_t)(m0 + u) * R + r;
          // W_new from its fixed-point accumulator, which is cleared for the
          // next step (NaN when the step's bound was not finite); it is
          // written back over W_old
          const double wn = sc.ok ? adj_from_fixed(wa[u], sc.E) : __builtin_nan("");
          wacc[o] = 0ull;
          const double bb = 2.0 * wn - wo[u] - sd[u] * vv[u];
          wold[o] = wn;
          V[o] = bb;  // bbar_m, held until pbar is known
          pbar += bb / sd[u];
        }
      }
    }
    for (int m0 = 0; m0 < M; m0 += U) {
      double vv[U], sd[U], a[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool in = m0 + u < M;
        vv[u] = in ? V[(size_t)(m0 + u) * R + r] : 0.0;
        sd[u] = in ? Sd[m0 + u] : 1.0;
        a[u] = in ? aw[m0 + u] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (m0 + u < M) {
          const double v = -vv[u] / sd[u] + a[u] * pbar;
          V[(size_t)(m0 + u) * R + r] = v;
          vmx = fmax(vmx, adj_mag(v));
        }
      }
    }
  }
  adj_raise_block(mx + (slot + 1) % 3, vmx);
}

// Transposed averaging with the unbalanced damping.  Step 1 of Alg. 1 scales
// the correction by t = gamma / (rho d) when rho d > gamma (eq.
// (Unbalanced-prox)), so b^(m) = t e_m / S^m with e_m = p - p^(m) and t
// depends on every e_m through d^2 = sum_m ||e_m||^2 / S^m.  Given
// bbar_m = 2 W_new - W_old - S^m V_m, the adjoint of e_m is
//   ebar_m = t bbar_m / S^m - tbar t e_m / (S^m d^2),  tbar = sum_m <bbar_m, e_m> / S^m
// (second term only while t < 1), and V_m <- a_m sum_j ebar_j - ebar_m.
// First pass: bbar (W_old <- W_new) and the per-block partials of tbar
// (fixed order).
__global__ void __launch_bounds__(256)
adjoint_unbal1_kernel(unsigned long long* __restrict__ wacc, double* __restrict__ wold,
                      const double* __restrict__ V, const double* __restrict__ Sd,
                      const double* __restrict__ pm_k, const double* __restrict__ p_k,
                      double* __restrict__ bbar, double* __restrict__ tpart, int R, int M,
                      const unsigned long long* __restrict__ mx, int slot, double smax) {
  __shared__ double sh[4];
  const AdjScale sc = adj_scale(mx, slot, smax);
  const int r = blockIdx.x * 256 + threadIdx.x;
  double acc = 0.0;
  if (r < R) {
    // eight measures' loads in flight at a time; the sum keeps the order m = 0, 1, ...
    constexpr int U = 8;
    const double pr = p_k[r];
    for (int m0 = 0; m0 < M; m0 += U) {
      unsigned long long wa[U];
      double wo[U], vv[U], sd[U], pmv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const size_t o = (size_t)(m0 + u) * R + r;
        const bool in = m0 + u < M;
        wa[u] = in ? wacc[o] : 0ull;
        wo[u] = in ? wold[o] : 0.0;
        vv[u] = in ? V[o] : 0.0;
        sd[u] = in ? Sd[m0 + u] : 1.0;
        pmv[u] = in ? pm_k[o] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (m0 + u < M) {
          const size_t o = (size_t)(m0 + u) * R + r;
          // W_new (accumulator cleared; NaN when the bound was not finite)
          const double wn = sc.ok ? adj_from_fixed(wa[u], sc.E) : __builtin_nan("");
          wacc[o] = 0ull;
          const double bb = 2.0 * wn - wo[u] - sd[u] * vv[u];
          wold[o] = wn;
          bbar[o] = bb;
          acc += bb * (pr - pmv[u]) / sd[u];
        }
      }
    }
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) tpart[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// Second pass: tbar, d and t of the iteration (from its recorded d^2
// partials), then ebar and V per row, and the bound of |V| for the next step.
__global__ void __launch_bounds__(256)
adjoint_unbal2_kernel(const double* __restrict__ bbar, double* __restrict__ V,
                      const double* __restrict__ pm_k, const double* __restrict__ p_k,
                      const double* __restrict__ d2_k, int nd2, const double* __restrict__ tpart, int ntp,
                      const double* __restrict__ Sd, const double* __restrict__ aw, double rho, double gamma,
                      int R, int M, unsigned long long* __restrict__ mx, int slot) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  double vmx = 0.0;
  if (r < R) {
    double tb = 0.0, d2 = 0.0;
    for (int i = 0; i < ntp; ++i) tb += tpart[i];
    for (int i = 0; i < nd2; ++i) d2 += d2_k[i];
    const double d = sqrt(d2);
    const bool damped = !__builtin_isinf(gamma) && rho * d > gamma;
    const double t = damped ? gamma / (rho * d) : 1.0;
    const double c = damped ? tb * t / d2 : 0.0;
    double pbar = 0.0;
    for (int m = 0; m < M; ++m) {
      const size_t o = (size_t)m * R + r;
      pbar += (t * bbar[o] - c * (p_k[r] - pm_k[o])) / Sd[m];
    }
    for (int m = 0; m < M; ++m) {
      const size_t o = (size_t)m * R + r;
      const double eb = (t * bbar[o] - c * (p_k[r] - pm_k[o])) / Sd[m];
      const double v = aw[m] * pbar - eb;
      V[o] = v;
      vmx = fmax(vmx, adj_mag(v));
    }
  }
  adj_raise_block(mx + (slot + 1) % 3, vmx);
}

// Start of the reverse sweep: the bound slots and the W accumulators cleared.
__global__ void __launch_bounds__(256)
adjoint_reset_kernel(unsigned long long* __restrict__ wacc, int64_t n, unsigned long long* __restrict__ mx) {
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) wacc[i] = 0ull;
  if (blockIdx.x == 0 && threadIdx.x < kAdjSlots) mx[threadIdx.x] = 0ull;
}

// Then V_m = a_m * dL/dp_bar, W_old = 0, and the bound of |V| for the
// first reverse step (slot 0).
__global__ void __launch_bounds__(256)
adjoint_start_kernel(const double* __restrict__ gp, const double* __restrict__ aw, double* __restrict__ V,
                     double* __restrict__ wold, int R, int M, unsigned long long* __restrict__ mx) {
  const int64_t n = (int64_t)R * M;
  double vmx = 0.0;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int m = (int)(i / R);
    const int r = (int)(i - (int64_t)m * R);
    const double v = aw[m] * gp[r];
    V[i] = v;
    wold[i] = 0.0;
    vmx = fmax(vmx, adj_mag(v));
  }
  adj_raise_block(mx, vmx);
}

// qbar_s = qacc_s + (sum_r V^0_m,r) / R for the columns of measure m (one
// block per measure; the row sum in a fixed order).
template <typename T>
__global__ void __launch_bounds__(256)
grad_q_kernel(const double* __restrict__ V, const double* __restrict__ qacc, const int64_t* __restrict__ col_off,
              T* __restrict__ gq, int R) {
  __shared__ double sh[4];
  const int m = blockIdx.x;
  double s = 0.0;
  for (int r = threadIdx.x; r < R; r += 256) s += V[(size_t)m * R + r];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  const double add = (((sh[0] + sh[1]) + sh[2]) + sh[3]) / (double)R;
  for (int64_t j = col_off[m] + threadIdx.x; j < col_off[m + 1]; j += 256) gq[j] = (T)(qacc[j] + add);
}

// cbar of cost column c = -(1/rho) * sum of cacc over the plan columns that
// read column c (list in increasing order: fixed summation order).
template <typename T>
__global__ void __launch_bounds__(256)
grad_cost_kernel(const double* __restrict__ cacc, const int64_t* __restrict__ cptr, const int32_t* __restrict__ clist,
                 int64_t ncols, int R, double inv_rho, T* __restrict__ gc, int64_t cost_ld) {
  for (int64_t c = blockIdx.x; c < ncols; c += gridDim.x) {
    const int64_t b = cptr[c], e = cptr[c + 1];
    for (int r = threadIdx.x; r < R; r += 256) {
      double s = 0.0;
      for (int64_t i = b; i < e; ++i) s += cacc[(int64_t)clist[i] * R + r];
      gc[c * cost_ld + r] = (T)(-s * inv_rho);
    }
  }
}

// Long columns, sparse store (MAM_FLAG_SPARSE_STORE): set-up and parity.
// Every sub-tile dense (the plans are all in theta) and parity 0.
__global__ void __launch_bounds__(256) long_sparse_reset_kernel(int32_t* pcnt, int64_t n, int32_t* spar) {
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) pcnt[i] = -1;
  if (blockIdx.x == 0 && threadIdx.x == 0) spar[0] = 0;
}

// After an iteration's write kernel: the stored plans now use the other half
// of nbv.  Gated like the iteration's other kernels.
__global__ void long_sparse_flip_kernel(int32_t* spar, const int32_t* stop) {
  if (stop != nullptr && *stop != 0) return;
  if (threadIdx.x == 0) spar[0] ^= 1;
}

}  // namespace mam

// Device code of the MAM column kernel for gfx950 (CDNA4, wave64).
//
// One Douglas-Rachford iteration of Alg. 1 is three launches:
//
//   column kernel  : per plan column, fuses the broadcast correction and the
//                    reflection (w = theta + 2b - c/rho, Alg. 1 Step 2 and
//                    Prop. 2 eq. (row_sol)), the exact projection onto
//                    Delta_R(q_s) (Prop. 3), the update theta' = pi_hat - b,
//                    and the row sums of theta' (Step 3) as fixed-order
//                    per-segment partials.  It streams theta once in and once
//                    out and reads each cost column once: HBM bound.
//   marginal kernel: p^(m)_r = sum of the partials of measure m (fixed order).
//   average kernel : p = sum_m a_m p^(m) (eq. (pr)) and the partial sums of
//                    d^2 = sum_m ||p - p^(m)||^2 / S^m used by the t^k rule.
//
// The column kernel reads the d^2 partials at its start and forms t^k
// itself, so no extra launch sits between the average and the next columns.
//
// Threshold search.  For tau = q_s > 0 the projection is max(w - lambda, 0)
// with lambda the root of f(lambda) = sum_r max(w_r - lambda, 0) - tau, a
// convex, decreasing, piecewise-linear function.  Since one entry can carry
// at most tau, lambda >= w_max - tau, and only entries above w_max - tau can
// be active.  Starting from lambda_0 = w_max - tau (f >= 0 there), Newton's
// step on f is lambda_{k+1} = (sum_{w > lambda_k} w - tau) / |{w > lambda_k}|;
// it increases monotonically and stops on the exact root as soon as the
// active set no longer shrinks, so the loop ends after at most R+1 passes
// (in practice 2-3) with the same lambda as the sort-based formula, up to
// summation order.  The column stays in registers (held as w in double) for
// all passes; each pass is one compare/select/add per value plus a group
// reduction.
//
// All reductions have a fixed order, so results are bitwise reproducible
// run to run; there are no floating-point atomics.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mam.h"

namespace mam {

template <typename T> struct VecOf;
template <> struct VecOf<float>  { static constexpr int N = 4; using type = float4; };
template <> struct VecOf<double> { static constexpr int N = 2; using type = double2; };

template <typename T, int VEC>
__device__ __forceinline__ void load_vec(const T* __restrict__ src, T (&v)[VEC]) {
  if constexpr (VEC == 1) {
    v[0] = src[0];
  } else if constexpr (sizeof(T) == 4) {
    static_assert(VEC == 4, "float vectors are 16 bytes");
    const float4 x = *reinterpret_cast<const float4*>(src);
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
  } else {
    static_assert(VEC == 2, "double vectors are 16 bytes");
    const double2 x = *reinterpret_cast<const double2*>(src);
    v[0] = x.x; v[1] = x.y;
  }
}

template <typename T, int VEC>
__device__ __forceinline__ void store_vec(T* __restrict__ dst, const T (&v)[VEC]) {
  if constexpr (VEC == 1) {
    dst[0] = v[0];
  } else if constexpr (sizeof(T) == 4) {
    *reinterpret_cast<float4*>(dst) = make_float4(v[0], v[1], v[2], v[3]);
  } else {
    *reinterpret_cast<double2*>(dst) = make_double2(v[0], v[1]);
  }
}

// Row-sum accumulator: plain double for FP64 plans; compensated (Kahan)
// float pairs for FP32 plans, finished in double.
template <typename T> struct RowAcc;
template <> struct RowAcc<double> {
  double s;
  __device__ __forceinline__ void zero() { s = 0.0; }
  __device__ __forceinline__ void add(double x) { s += x; }
  __device__ __forceinline__ double value() const { return s; }
};
template <> struct RowAcc<float> {
  float s, c;  // running sum and the negated low part lost so far
  __device__ __forceinline__ void zero() { s = 0.0f; c = 0.0f; }
  __device__ __forceinline__ void add(float x) {
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
  }
  __device__ __forceinline__ double value() const { return (double)s - (double)c; }
};

__device__ __forceinline__ double uniform_d(double v) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(bits & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(bits >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return uniform_d(v);
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Reductions over one column group of NW waves.  NW == 1 needs no barrier;
// NW > 1 means the group is the whole workgroup, so __syncthreads is safe.
// 'slots' holds 2 parities x NW x 2 doubles; alternating parities make one
// barrier per reduction enough.
template <int NW>
struct GroupReduce {
  double* slots;
  int par;

  __device__ __forceinline__ double max(double v, int wv, int lane) {
    v = wave_max(v);
    if constexpr (NW == 1) {
      return v;
    } else {
      if (lane == 0) slots[(par * NW + wv) * 2] = v;
      __syncthreads();
      double r = slots[(par * NW) * 2];
#pragma unroll
      for (int i = 1; i < NW; ++i) r = fmax(r, slots[(par * NW + i) * 2]);
      par ^= 1;
      return r;
    }
  }

  __device__ __forceinline__ void sum2(double& s, double& c, int wv, int lane) {
    s = wave_sum(s);
    if constexpr (NW > 1) {
      if (lane == 0) {
        slots[(par * NW + wv) * 2] = s;
        slots[(par * NW + wv) * 2 + 1] = c;
      }
      __syncthreads();
      double rs = 0.0, rc = 0.0;
#pragma unroll
      for (int i = 0; i < NW; ++i) {
        rs += slots[(par * NW + i) * 2];
        rc += slots[(par * NW + i) * 2 + 1];
      }
      par ^= 1;
      s = rs;
      c = rc;
    }
  }
};

template <typename T>
struct ColArgs {
  T* theta;
  const T* cost;
  const T* q;
  const int32_t* cidx;
  int64_t ld, cost_ld;
  int32_t R, cost_mode;
  const double* pm;       // M x R marginals of the current plans
  const double* p;        // R, averaged marginal
  const double* d2part;   // nb partial sums of d^2
  int32_t nb, diag_on;
  double rho, inv_rho, gamma;
  const int64_t* col_off; // M+1
  const double* Sd;       // S^m as double
  const int32_t* seg_m;
  const int64_t* seg_j0;
  const int64_t* seg_j1;
  const int32_t* wg_seg;  // nwg+1
  double* partial;        // nseg x R
  double* t_out;          // 1
  double* diag;           // nwg x 4
  int32_t nwg, xcd_remap;
};

// XCD-aware block order: the hardware deals consecutive workgroup ids round
// robin over the 8 XCDs; remapping gives each XCD a contiguous run of
// segments so neighbouring columns (which share cost columns and L2 lines)
// stay on one XCD's L2.
__device__ __forceinline__ int logical_block(int bid, int nblocks, int remap) {
  if (!remap) return bid;
  const int nx = 8;
  const int per = (nblocks + nx - 1) / nx;
  const int x = bid % nx, k = bid / nx;
  const int full = nblocks - (per - 1) * nx;  // XCDs that receive 'per' blocks
  const int base = (x < full) ? x * per : full * per + (x - full) * (per - 1);
  return base + k;
}

// Dynamic LDS: VPT*NT doubles of b^(m) (each thread reads only its own
// slots: no sharing, no bank conflicts), then R doubles for the cross-group
// row-sum reduction when NG > 1.
template <int NT> struct GroupShape {
  // a 64-thread group is one wave: four of them share a workgroup;
  // larger groups are the whole workgroup
  static constexpr int NG = NT == 64 ? 4 : 1;
  static constexpr int WG = NT * NG;
};

template <typename T, int NT, int VPT, int VEC, bool DIAG>
__global__ void __launch_bounds__(GroupShape<NT>::WG)
column_kernel(ColArgs<T> a) {
  constexpr int WG = GroupShape<NT>::WG;
  constexpr int NG = GroupShape<NT>::NG;  // independent column groups per workgroup
  constexpr int NW = NT / 64;     // waves per group
  constexpr int NCH = VPT / VEC;  // vector chunks per thread
  static_assert(VPT % VEC == 0, "VPT must be a multiple of VEC");
  static_assert(NG == 1 || NW == 1, "multi-wave groups fill the workgroup");

  __shared__ double slots[2 * NW * 2];
  __shared__ double sh_t;
  __shared__ double sh_diag[WG / 64][3];
  extern __shared__ double lds_dyn[];
  double* lds_b = lds_dyn;               // [VPT][NT]
  double* lds_acc = lds_dyn + VPT * NT;  // [R], used when NG > 1

  const int gtid = threadIdx.x;
  const int g = gtid / NT;
  const int tid = gtid % NT;
  const int lane = gtid & 63;
  const int wv = tid >> 6;
  const int R = a.R;

  if (gtid == 0) {
    double d2 = 0.0;
    for (int i = 0; i < a.nb; ++i) d2 += a.d2part[i];
    const double d = sqrt(d2);
    const double t = (__builtin_isinf(a.gamma) || a.rho * d <= a.gamma) ? 1.0 : a.gamma / (a.rho * d);
    sh_t = t;
    if (blockIdx.x == 0) a.t_out[0] = t;
  }
  __syncthreads();
  const double t = sh_t;

  GroupReduce<NW> red{slots, 0};
  double dW = 0.0, dRes = 0.0, dTh = 0.0;

  const int wg = logical_block(blockIdx.x, gridDim.x, a.xcd_remap);
  const int sb = a.wg_seg[wg], se = a.wg_seg[wg + 1];
  for (int si = sb; si < se; ++si) {
    const int m = a.seg_m[si];
    const int64_t j0 = a.seg_j0[si], j1 = a.seg_j1[si];
    const double Sm = a.Sd[m];
    const int64_t off_m = a.col_off[m];
    const double* __restrict__ pmm = a.pm + (size_t)m * R;

    // b^(m) = t (p - p^(m)) / S^m for this thread's rows, kept in LDS
    __syncthreads();  // previous segment's readers are done
    if (g == 0) {
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const int r = (c * NT + tid) * VEC + v;
          lds_b[(c * VEC + v) * NT + tid] = (r < R) ? t * (a.p[r] - pmm[r]) / Sm : 0.0;
        }
      }
    }
    __syncthreads();
    RowAcc<T> acc[VPT];
#pragma unroll
    for (int k = 0; k < VPT; ++k) acc[k].zero();

    for (int64_t j = j0 + g; j < j1; j += NG) {
      T* __restrict__ thp = a.theta + j * a.ld;
      int64_t cc;
      if (a.cost_mode == MAM_COST_INDEXED) cc = a.cidx[j];
      else if (a.cost_mode == MAM_COST_SHARED) cc = j - off_m;
      else cc = j;
      const T* __restrict__ cp = a.cost + cc * a.cost_ld;

      // reflection w = theta + 2b - c/rho, widened to double
      double w[VPT];
      double mx = -INFINITY;
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const int r0 = (c * NT + tid) * VEC;
        if (r0 < R) {
          T tv[VEC], cv[VEC];
          load_vec<T, VEC>(thp + r0, tv);
          load_vec<T, VEC>(cp + r0, cv);
#pragma unroll
          for (int v = 0; v < VEC; ++v) {
            const int k = c * VEC + v;
            const double bk = lds_b[k * NT + tid];
            w[k] = (r0 + v < R) ? ((double)tv[v] + 2.0 * bk) - (double)cv[v] * a.inv_rho : -INFINITY;
            mx = fmax(mx, w[k]);
          }
        } else {
#pragma unroll
          for (int v = 0; v < VEC; ++v) w[c * VEC + v] = -INFINITY;
        }
      }
      mx = red.max(mx, wv, lane);

      // exact threshold: Newton from lambda_0 = w_max - tau
      const double tau = (double)a.q[j];
      double lam = INFINITY;
      if (tau > 0.0) {
        lam = mx - tau;
        double prev = 1e300;
        for (int it = 0; it <= R; ++it) {
          double s = 0.0, cnt = 0.0;
#pragma unroll
          for (int k = 0; k < VPT; ++k) {
            const bool act = w[k] > lam;
            s += act ? w[k] : 0.0;
            cnt += (double)__popcll(__ballot(act));
          }
          red.sum2(s, cnt, wv, lane);
          if (cnt == 0.0 || cnt >= prev) break;
          lam = (s - tau) / cnt;
          prev = cnt;
        }
      }

      // pi_hat = max(w - lambda, 0); theta' = pi_hat - b; row sums of theta'
      double colsum = 0.0;
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const int r0 = (c * NT + tid) * VEC;
        if (r0 < R) {
          T out[VEC];
          T oldv[VEC], cv[VEC];
          if constexpr (DIAG) {
            load_vec<T, VEC>(thp + r0, oldv);
            load_vec<T, VEC>(cp + r0, cv);
          }
#pragma unroll
          for (int v = 0; v < VEC; ++v) {
            const int k = c * VEC + v;
            const double ph = fmax(w[k] - lam, 0.0);
            out[v] = (T)(ph - lds_b[k * NT + tid]);
            if (DIAG && r0 + v < R) {
              colsum += ph;
              dW += (double)cv[v] * ph;
              dTh = fmax(dTh, fabs((double)out[v] - (double)oldv[v]));
            }
          }
          if (r0 + VEC <= R) {
            store_vec<T, VEC>(thp + r0, out);
          } else {
#pragma unroll
            for (int v = 0; v < VEC; ++v)
              if (r0 + v < R) thp[r0 + v] = out[v];
          }
#pragma unroll
          for (int v = 0; v < VEC; ++v)
            if (r0 + v < R) acc[c * VEC + v].add(out[v]);
        }
      }
      if constexpr (DIAG) {
        double zero = 0.0;
        red.sum2(colsum, zero, wv, lane);
        dRes = fmax(dRes, fabs(colsum - (tau > 0.0 ? tau : 0.0)));
      }
    }

    // fixed-order partial row sums of this segment
    if constexpr (NG == 1) {
#pragma unroll
      for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const int r = (c * NT + tid) * VEC + v;
          if (r < R) a.partial[(size_t)si * R + r] = acc[c * VEC + v].value();
        }
    } else {
      for (int gg = 0; gg < NG; ++gg) {
        if (g == gg) {
#pragma unroll
          for (int c = 0; c < NCH; ++c)
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
              const int r = (c * NT + tid) * VEC + v;
              if (r < R) lds_acc[r] = (gg == 0 ? 0.0 : lds_acc[r]) + acc[c * VEC + v].value();
            }
        }
        __syncthreads();
      }
      for (int r = gtid; r < R; r += WG) a.partial[(size_t)si * R + r] = lds_acc[r];
      __syncthreads();
    }
  }

  if constexpr (DIAG) {
    // dW sums per thread; dRes, dTh maxima.  Fixed order over waves.
    double s = wave_sum(dW);
    double r1 = wave_max(dRes), r2 = wave_max(dTh);
    if (lane == 0) {
      sh_diag[gtid >> 6][0] = s;
      sh_diag[gtid >> 6][1] = r1;
      sh_diag[gtid >> 6][2] = r2;
    }
    __syncthreads();
    if (gtid == 0) {
      double S0 = 0.0, m1 = 0.0, m2 = 0.0;
      for (int i = 0; i < WG / 64; ++i) {
        S0 += sh_diag[i][0];
        m1 = fmax(m1, sh_diag[i][1]);
        m2 = fmax(m2, sh_diag[i][2]);
      }
      a.diag[(size_t)wg * 4 + 0] = S0;
      a.diag[(size_t)wg * 4 + 1] = m1;
      a.diag[(size_t)wg * 4 + 2] = m2;
      a.diag[(size_t)wg * 4 + 3] = 0.0;
    }
  }
}

}  // namespace mam

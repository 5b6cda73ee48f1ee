// Device code of the reverse mode (adjoint) of the balanced MAM iteration.
//
// One iteration k of Alg. 1 (t = 1) maps theta^k to theta^{k+1} column by
// column:
//   b^(m)  = (p - p^(m)) / S^m,  p^(m) = row sums of theta^(m),  p = sum a_m p^(m)
//   w_s    = theta_s + 2 b^(m) - c_s / rho
//   theta'_s = P(w_s, q_s) - b^(m),   P = projection onto Delta_R(q_s) (Prop. 3).
// On the active set A of a column (w_r > lambda) the projection is
// w - lambda with lambda = (sum_A w - q_s)/|A|, so its Jacobian is
// J = D_A - 1_A 1_A^T / |A| (symmetric) and dP/dq_s = 1_A / |A|.
//
// Reverse step, given the adjoint X = dL/dtheta^{k+1} (R x T):
//   wbar_s  = J X_s         (X - mean_A X on A, zero elsewhere)
//   qbar_s += mean_A X_s,   cbar_s += -wbar_s / rho
//   bbar^(m) = sum_s (2 wbar_s - X_s)
//   pbar     = sum_m bbar^(m) / S^m
//   dL/dtheta^k_s = wbar_s + v^(m),   v^(m) = -bbar^(m)/S^m + a_m pbar.
// So every adjoint is U + (broadcast of one R-vector per measure) with U
// supported on the active sets: the state is the sparse U, the M vectors V
// and the row sums W^(m) = sum_s U_s; bbar^(m) = 2 W_new - W_old - S^m V.
// A step touches the forward's active-set bit masks, V, and U and the cost
// adjoint at active entries only.
//
// The loss side starts from X = broadcast of a_m * dL/dp_bar (U = 0); the
// start theta^0 = q/R adds sum_r X_rs / R to qbar_s.
#pragma once

#include "mam_kernels.hpp"

namespace mam {

struct AdjArgs {
  const int32_t* seg_m;
  const int64_t* seg_j0;
  const int64_t* seg_j1;
  const int64_t* seg_poff;
  const int32_t* wg_seg;
  double* partial;       // per-segment row sums of wbar
  const uint8_t* mk;     // active-set masks of iteration k (column j at mk + j*mld)
  const uint8_t* mk1;    // masks of iteration k+1, or null when U^{k+1} = 0
  int64_t mld;           // mask bytes per column
  double* U;             // R x T (ld R): wbar of the last reverse step, valid on its masks
  double* cacc;          // R x T (ld R): sum over steps of wbar
  double* qacc;          // T: sum over steps of mean_A X
  const double* V;       // M x R: broadcast part of X
  int32_t R, vec_shift, nwg, xcd_remap;
};

// Reverse column step.  Same column layout, groups and segments as the
// forward column kernel whose masks it reads: thread tid of a group holds
// bit k of a column's mask word for row ((k >> vs)*NT + tid) << vs | (k & (2^vs - 1)).
// Dynamic LDS: VPT*NT doubles of V^(m), then NG*VPT*NT doubles of row-sum
// accumulators (each row owned by one thread of a group: no atomics).
template <int NT, int VPT>
__global__ void __launch_bounds__(GroupShape<NT>::WG)
adjoint_kernel(AdjArgs a) {
  using W = typename MaskWord<VPT>::type;
  constexpr int WG = GroupShape<NT>::WG;
  constexpr int NG = GroupShape<NT>::NG;
  constexpr int NW = NT / 64;
  static_assert(VPT <= 16, "mask words hold at most 16 bits");

  __shared__ double red_s[2][NW > 1 ? NW : 1];
  __shared__ double red_n[2][NW > 1 ? NW : 1];
  extern __shared__ double lds_dyn[];
  double* lds_v = lds_dyn;                // [VPT][NT]
  double* lds_fix = lds_dyn + VPT * NT;   // [NG][VPT][NT]

  const int gtid = threadIdx.x;
  const int g = NG == 1 ? 0 : __builtin_amdgcn_readfirstlane(gtid / NT);
  const int tid = gtid % NT;
  const int lane = gtid & 63;
  const int wv = NW == 1 ? 0 : __builtin_amdgcn_readfirstlane(tid >> 6);
  double* fix = lds_fix + (size_t)g * VPT * NT;
  const int R = a.R, vs = a.vec_shift;
  auto row = [&](int k) { return (((k >> vs) * NT + tid) << vs) | (k & ((1 << vs) - 1)); };

  int par = 0;
  const int wg = logical_block(blockIdx.x, gridDim.x, a.xcd_remap);
  const int sb = uniform_i(a.wg_seg[wg]), se = uniform_i(a.wg_seg[wg + 1]);
  for (int si = sb; si < se; ++si) {
    const int m = uniform_i(a.seg_m[si]);
    const int64_t j0 = uniform_l(a.seg_j0[si]), j1 = uniform_l(a.seg_j1[si]);
    __syncthreads();  // previous segment's readers are done
    if (g == 0) {
#pragma unroll
      for (int k = 0; k < VPT; ++k) {
        const int r = row(k);
        lds_v[k * NT + tid] = r < R ? a.V[(size_t)m * R + r] : 0.0;
      }
    }
#pragma unroll
    for (int k = 0; k < VPT; ++k) fix[k * NT + tid] = 0.0;
    __syncthreads();

    // masks of the next column are loaded one column ahead
    W nk = 0, nk1 = 0;
    auto load_masks = [&](int64_t j) {
      nk = reinterpret_cast<const W*>(a.mk + j * a.mld)[tid];
      nk1 = a.mk1 ? reinterpret_cast<const W*>(a.mk1 + j * a.mld)[tid] : (W)0;
    };
    if (j0 + g < j1) load_masks(j0 + g);
    for (int64_t j = j0 + g; j < j1; j += NG) {
      const unsigned bk = nk, bk1 = nk1;
      if (j + NG < j1) load_masks(j + NG);
      double* __restrict__ Uc = a.U + j * (int64_t)R;
      double x[VPT];
      double s = 0.0;
      const bool wave_any = __ballot(bk != 0u) != 0ull;
      if (wave_any) {
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
          x[k] = 0.0;
          if ((bk >> k) & 1u) {
            double v = lds_v[k * NT + tid];
            if ((bk1 >> k) & 1u) v += Uc[row(k)];
            x[k] = v;
            s += v;
          }
        }
      }
      double n = (double)__popc(bk);
      // group sums of X over A and of |A| (fixed order)
      if (wave_any) {
        s = wave_reduce<OpSum>(s);
        n = wave_reduce<OpSum>(n);
      } else {
        s = 0.0;
        n = 0.0;
      }
      if constexpr (NW > 1) {
        if (lane == 0) {
          red_s[par][wv] = s;
          red_n[par][wv] = n;
        }
        __syncthreads();
        double ss = red_s[par][0], nn = red_n[par][0];
#pragma unroll
        for (int i = 1; i < NW; ++i) {
          ss += red_s[par][i];
          nn += red_n[par][i];
        }
        s = uniform_d(ss);
        n = uniform_d(nn);
        par ^= 1;
      }
      if (n == 0.0) continue;  // tau = 0 or an empty projection: no active entry
      const double mean = s / n;
      if (tid == 0) a.qacc[j] += mean;
      if (wave_any) {
        double* __restrict__ Cc = a.cacc + j * (int64_t)R;
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
          if ((bk >> k) & 1u) {
            const int r = row(k);
            const double wb = x[k] - mean;
            Uc[r] = wb;
            Cc[r] += wb;
            fix[k * NT + tid] += wb;
          }
        }
      }
    }

    // the segment's row sums of wbar, groups in order
    __syncthreads();
    for (int i = gtid; i < VPT * NT; i += WG) {
      const int k = i / NT, tt = i % NT;
      const int r = (((k >> vs) * NT + tt) << vs) | (k & ((1 << vs) - 1));
      if (r < R) {
        double f = lds_fix[i];
#pragma unroll
        for (int gg = 1; gg < NG; ++gg) f += lds_fix[(size_t)gg * VPT * NT + i];
        a.partial[uniform_l(a.seg_poff[si]) + r] = f;
      }
    }
  }
}

}  // namespace mam

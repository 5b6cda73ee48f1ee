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

#include <type_traits>

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
//
// A column has a handful of active entries (often one), spread over the
// group, so a thread usually holds none and rarely more than one.  The fast
// path keeps at most two active entries per thread in registers; a wave in
// which some thread has more takes a slow path that walks the bits (same
// summation order, so results do not depend on the path).  The work of a
// column is a dependent chain (mask -> gathers -> group sum -> writes), so
// columns are pipelined: masks are loaded four columns ahead and the V, U,
// cost-adjoint and q-adjoint entries gathered two columns ahead, so no
// read-modify-write waits on memory inside a column step.  V is read from
// global memory (it is a few tens of KB per measure and stays in L2).
//
// Dynamic LDS: NG*VPT*NT doubles of row-sum accumulators (each row owned by
// one thread of a group: no atomics).
template <int NT, int VPT>
__global__ void __launch_bounds__(GroupShape<NT>::WG)
adjoint_kernel(AdjArgs a) {
  // column slots in flight (gathers RING-1 columns ahead, masks RING+1):
  // four or five slots are no faster and five lower the resident workgroups
  constexpr int RING = 3;
  static_assert(RING >= 3, "masks are requested two steps before their gather");
  using W = typename MaskWord<VPT>::type;
  constexpr int WG = GroupShape<NT>::WG;
  constexpr int NG = GroupShape<NT>::NG;
  constexpr int NW = NT / 64;
  static_assert(VPT <= 16, "mask words hold at most 16 bits");

  extern __shared__ double lds_dyn[];
  double* lds_fix = lds_dyn;  // [NG][VPT][NT]

  const int gtid = threadIdx.x;
  const int g = NG == 1 ? 0 : __builtin_amdgcn_readfirstlane(gtid / NT);
  const int tid = gtid % NT;
  const int lane = gtid & 63;
  const int wv = NW == 1 ? 0 : __builtin_amdgcn_readfirstlane(tid >> 6);
  double* fix = lds_fix + (size_t)g * VPT * NT;
  const int R = a.R, vs = a.vec_shift;
  auto row = [&](int k) { return (((k >> vs) * NT + tid) << vs) | (k & ((1 << vs) - 1)); };

  // one column in flight: its masks, its first two active slots and the
  // loaded V, U and cost-adjoint entries there, and its q adjoint
  struct Gat {
    unsigned bk, bk1;
    int k0, k1;      // active slots (-1: none)
    double v0, u0, c0, v1, u1, c1, qa;
  };
  __shared__ double red_s[2][NW > 1 ? NW : 1];
  __shared__ double red_n[2][NW > 1 ? NW : 1];

  int par = 0;
  const int wg = logical_block(blockIdx.x, gridDim.x, a.xcd_remap);
  const int sb = uniform_i(a.wg_seg[wg]), se = uniform_i(a.wg_seg[wg + 1]);
  for (int si = sb; si < se; ++si) {
    const int m = uniform_i(a.seg_m[si]);
    const int64_t j0 = uniform_l(a.seg_j0[si]), j1 = uniform_l(a.seg_j1[si]);
    const double* __restrict__ Vm = a.V + (size_t)m * R;
    __syncthreads();  // previous segment's readers are done
#pragma unroll
    for (int k = 0; k < VPT; ++k) fix[k * NT + tid] = 0.0;
    __syncthreads();

    auto colj = [&](int64_t t) { return j0 + g + (int64_t)NG * t; };
    // every load below is issued by every lane of every step (addresses
    // clamped into the segment, unused values ignored): with a fixed number of
    // loads per step a wait covers only the loads it needs, never the ones
    // issued after them
    auto jclamp = [&](int64_t j) { return j < j1 ? j : j1 - 1; };
    const uint8_t* const mk1p = a.mk1 ? a.mk1 : a.mk;
    const bool has1 = a.mk1 != nullptr;
    unsigned mring[RING][2];  // raw mask words, slot = column mod RING
    Gat gr[RING];             // gathered entries, slot = column mod RING
    auto load_masks = [&](auto S, int64_t t) {
      constexpr int s = decltype(S)::value;
      const int64_t j = jclamp(colj(t));
      mring[s][0] = reinterpret_cast<const W*>(a.mk + j * a.mld)[tid];
      mring[s][1] = reinterpret_cast<const W*>(mk1p + j * a.mld)[tid];
    };
    // the column's masks (waiting for them) and the loads of its first two
    // active slots, X = V (+ U where also active at k+1) formed when used
    auto gather = [&](auto S, int64_t t) {
      constexpr int s = decltype(S)::value;
      Gat& c = gr[s];
      const bool in = colj(t) < j1;
      const int64_t j = jclamp(colj(t));
      c.bk = in ? mring[s][0] : 0u;
      c.bk1 = (in && has1) ? mring[s][1] : 0u;
      const unsigned b1 = c.bk & (c.bk - 1u);
      c.k0 = c.bk ? __builtin_ctz(c.bk) : -1;
      c.k1 = b1 ? __builtin_ctz(b1) : -1;
      const int r0 = c.k0 >= 0 ? row(c.k0) : 0, r1 = c.k1 >= 0 ? row(c.k1) : 0;
      const double* __restrict__ Uc = a.U + j * (int64_t)R;
      const double* __restrict__ Cc = a.cacc + j * (int64_t)R;
      c.v0 = Vm[r0];
      c.u0 = Uc[r0];
      c.c0 = Cc[r0];
      c.v1 = Vm[r1];
      c.u1 = Uc[r1];
      c.c1 = Cc[r1];
      c.qa = a.qacc[j];
    };

    auto process = [&](auto S, int64_t t) {
      constexpr int s = decltype(S)::value;
      const Gat& c = gr[s];
      const int64_t j = colj(t);
      double* __restrict__ Uc = a.U + j * (int64_t)R;
      const unsigned bk = c.bk, bk1 = c.bk1;
      const bool wave_any = __ballot(bk != 0u) != 0ull;
      const bool wave_slow = __ballot(__popc(bk) > 2) != 0ull;
      double x0 = 0.0, x1 = 0.0;
      if (c.k0 >= 0) {
        x0 = c.v0;
        if ((bk1 >> c.k0) & 1u) x0 += c.u0;
      }
      if (c.k1 >= 0) {
        x1 = c.v1;
        if ((bk1 >> c.k1) & 1u) x1 += c.u1;
      }
      double sum = 0.0;
      if (wave_slow) {
        for (unsigned b = bk; b; b &= b - 1) {
          const int r = row(__builtin_ctz(b));
          double v = Vm[r];
          if ((bk1 >> __builtin_ctz(b)) & 1u) v += Uc[r];
          sum += v;
        }
      } else {
        sum = x0 + x1;  // slot order, as the slow path
      }
      double n = (double)__popc(bk);
      // group sums of X over A and of |A| (fixed order)
      if (wave_any) {
        sum = wave_reduce<OpSum>(sum);
        n = wave_reduce<OpSum>(n);
      } else {
        sum = 0.0;
        n = 0.0;
      }
      if constexpr (NW > 1) {
        if (lane == 0) {
          red_s[par][wv] = sum;
          red_n[par][wv] = n;
        }
        __syncthreads();
        double ss = red_s[par][0], nn = red_n[par][0];
#pragma unroll
        for (int i = 1; i < NW; ++i) {
          ss += red_s[par][i];
          nn += red_n[par][i];
        }
        sum = uniform_d(ss);
        n = uniform_d(nn);
        par ^= 1;
      }
      if (n != 0.0) {  // n = 0: tau = 0 or an empty projection, nothing active
        const double mean = sum / n;
        if (tid == 0) a.qacc[j] = c.qa + mean;
        if (wave_any) {
          double* __restrict__ Cc = a.cacc + j * (int64_t)R;
          if (wave_slow) {
            // X is re-read: this column's U is written only below, entry by entry
            for (unsigned b = bk; b; b &= b - 1) {
              const int k = __builtin_ctz(b);
              const int r = row(k);
              double v = Vm[r];
              if ((bk1 >> k) & 1u) v += Uc[r];
              const double wb = v - mean;
              Uc[r] = wb;
              Cc[r] += wb;
              fix[k * NT + tid] += wb;
            }
          } else {
            if (c.k0 >= 0) {
              const int r = row(c.k0);
              const double wb = x0 - mean;
              Uc[r] = wb;
              Cc[r] = c.c0 + wb;
              fix[c.k0 * NT + tid] += wb;
            }
            if (c.k1 >= 0) {
              const int r = row(c.k1);
              const double wb = x1 - mean;
              Uc[r] = wb;
              Cc[r] = c.c1 + wb;
              fix[c.k1 * NT + tid] += wb;
            }
          }
        }
      }
    };

    // step t: masks of column t+RING+1 requested, column t+RING-1 gathered
    // (its masks arrived two steps ago), column t processed (gathered RING-1
    // steps ago); unrolled RING times so every slot index is static
    auto step = [&](auto U, int64_t t) {
      constexpr int u = decltype(U)::value;
      load_masks(std::integral_constant<int, (u + 1) % RING>{}, t + RING + 1);
      gather(std::integral_constant<int, (u + RING - 1) % RING>{}, t + RING - 1);
      process(U, t);
    };
    if (colj(0) < j1) {
      static_for<RING>([&](auto I) { load_masks(I, decltype(I)::value); });
      gather(std::integral_constant<int, 0>{}, 0);
      load_masks(std::integral_constant<int, 0>{}, RING);
      static_for<RING - 2>([&](auto I) {
        gather(std::integral_constant<int, decltype(I)::value + 1>{}, decltype(I)::value + 1);
      });
      for (int64_t t = 0;; t += RING) {
        bool done = false;
        static_for<RING>([&](auto I) {
          if (done) return;
          step(I, t + decltype(I)::value);
          if (colj(t + decltype(I)::value + 1) >= j1) done = true;
        });
        if (done) break;
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

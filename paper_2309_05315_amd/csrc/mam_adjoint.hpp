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
//
// Row sums W^(m) in fixed point.  A column contributes to a handful of rows
// (often one, and then wbar = X - X = 0 exactly), so the reverse column
// kernel adds each nonzero wbar to its row's 64-bit integer accumulator
// with an atomic: integer addition is associative, so W does not depend on
// the order in which columns finish (bitwise reproducible for any launch
// shape) and no per-segment partial rows are needed.  The scale 2^E of step
// i is fixed before the step from bounds kept on the device: |wbar| <= 2
// max|X|, |X| <= max|V| + max|U|, and a row sums at most S_max columns, so
// |W| * 2^E < 2^61 with 2 S_max (max|V| + max|U|) < 2^(61 - E).  Each term
// is rounded to a multiple of 2^-E: 2^-62 of the bound.  The bounds live in
// six slots (bits of non-negative doubles, so unsigned order is the order
// of the values; a NaN is recorded as +inf): slots 0-2 bound |V|, 3-5 bound
// |U|, and step i reads slot i mod 3.  Step i's column kernel raises the
// |U| bound of step i+1 and clears the slots step i+1 and i+2 will raise
// (no kernel of step i reads them); step i's averaging raises the |V| bound
// of step i+1.
#pragma once

#include <type_traits>

#include "mam_kernels.hpp"

namespace mam {

constexpr int kAdjSlots = 6;

struct AdjScale {
  int E;    // fixed-point values are round(x * 2^E)
  bool ok;  // false when a bound is not finite (the gradients are then NaN)
};

__device__ __forceinline__ AdjScale adj_scale(const unsigned long long* mx, int slot, double smax) {
  const double vm = __longlong_as_double((long long)mx[slot]);
  const double um = __longlong_as_double((long long)mx[3 + slot]);
  const double bound = 2.0 * smax * (vm + um);
  AdjScale s{0, true};
  if (!(bound <= __DBL_MAX__)) {
    s.ok = false;
  } else if (bound > 0.0) {
    int e = 0;
    (void)frexp(bound, &e);  // bound < 2^e
    s.E = 61 - e;
  }
  return s;
}

__device__ __forceinline__ unsigned long long adj_to_fixed(double x, int E) {
  return (unsigned long long)__double2ll_rn(ldexp(x, E));
}

__device__ __forceinline__ double adj_from_fixed(unsigned long long v, int E) {
  return ldexp((double)(long long)v, -E);
}

// |x| for the bound slots; NaN counts as +inf.
__device__ __forceinline__ double adj_mag(double x) {
  return x != x ? __builtin_huge_val() : fabs(x);
}

// Raise a bound slot to the block's largest magnitude (256 threads, every
// thread calls it).
__device__ __forceinline__ void adj_raise_block(unsigned long long* slot, double v) {
  __shared__ double sh[4];
  v = wave_reduce<OpMax>(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double b = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    if (b > 0.0) atomicMax(slot, (unsigned long long)__double_as_longlong(b));
  }
}

struct AdjArgs {
  const uint8_t* mk;          // active-set masks of iteration k (column j at mk + j*mld)
  const uint8_t* mk1;         // masks of iteration k+1, or null when U^{k+1} = 0
  int64_t mld;                // mask bytes per column (64 lanes x LB bytes)
  const int64_t* col_off;     // M+1 column offsets of the measures
  double* U;                  // R x T (ld R): wbar of the last reverse step, valid on its masks
  double* cacc;               // R x T (ld R): sum over steps of wbar
  double* qacc;               // T: sum over steps of mean_A X
  const double* V;            // M x R: broadcast part of X
  unsigned long long* wacc;   // M x R: fixed-point row sums of wbar (zero on entry)
  unsigned long long* mx;     // kAdjSlots magnitude bounds
  double smax;                // max_m S^m
  int64_t T;
  int32_t R, M;
  int32_t nt, vs, wshift;     // the forward's row mapping: threads per column,
                              // log2 vector width, log2 bits per mask word
  int32_t slot;               // reverse step mod 3
};

// Reverse column step: one wave per column, KC columns at a time (a
// grid-stride loop over batches of KC columns; launched with one batch per
// wave, which measured faster than resident waves that loop).
//
// The forward kernel stores a column's active set as one mask word per
// thread (bit k of thread tid = row ((k >> vs)*nt + tid) << vs | (k mod
// 2^vs)).  Here lane l reads LB consecutive bytes of the column's mask, the
// words of threads l*LB/wb ... (wb = bytes per word), so a column is one
// coalesced load per lane and no lane waits on another: no LDS and no
// barrier.  A lane usually holds no active entry and rarely more than one.
// The first two of a lane's entries are gathered (V, U, cost adjoint) right
// after the masks; a lane with more walks its bits (same order, so the
// result does not depend on the path).  Per column, the sums of X and of
// |A| over A are wave reductions in a fixed order, skipped when the column
// has a single active entry (then wbar = 0 and only q's adjoint moves).
template <int LB, int KC>
__global__ void __launch_bounds__(256) adjoint_kernel(AdjArgs a) {
  constexpr int NCH = LB >= 8 ? LB / 8 : 1;  // 64-bit chunks per lane
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * 4 + uniform_i((int)(threadIdx.x >> 6));
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  const int R = a.R, M = a.M, nt = a.nt, vs = a.vs, wsh = a.wshift;
  const int64_t T = a.T, mld = a.mld;
  const int64_t* __restrict__ col_off = gptr(a.col_off);
  const uint8_t* __restrict__ mk = gptr(a.mk);
  const uint8_t* __restrict__ mk1 = a.mk1 ? gptr(a.mk1) : nullptr;
  const double* __restrict__ V = gptr(a.V);
  double* __restrict__ U = gptr(a.U);
  double* __restrict__ Cacc = gptr(a.cacc);
  double* __restrict__ Qacc = gptr(a.qacc);
  unsigned long long* __restrict__ wacc = gptr(a.wacc);
  const AdjScale sc = adj_scale(gptr(a.mx), a.slot, a.smax);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    gptr(a.mx)[3 + (a.slot + 2) % 3] = 0ull;
    gptr(a.mx)[(a.slot + 1) % 3] = 0ull;
  }

  auto row_of = [&](int b) {  // bit b of this lane's bytes -> row
    const int gb = lane * (LB * 8) + b;
    const int tid = gb >> wsh, k = gb & ((1 << wsh) - 1);
    return (((k >> vs) * nt + tid) << vs) | (k & ((1 << vs) - 1));
  };
  auto load_mask = [&](const uint8_t* base, uint64_t (&w)[NCH]) {
    if constexpr (LB == 1) {
      w[0] = base[lane];
    } else if constexpr (LB == 2) {
      w[0] = reinterpret_cast<const uint16_t*>(base)[lane];
    } else if constexpr (LB == 4) {
      w[0] = reinterpret_cast<const uint32_t*>(base)[lane];
    } else {
      const uint64_t* p = reinterpret_cast<const uint64_t*>(base) + (int64_t)lane * NCH;
#pragma unroll
      for (int c = 0; c < NCH; ++c) w[c] = p[c];
    }
  };
  auto bit_of = [](const uint64_t (&w)[NCH], int b) -> bool { return (w[b >> 6] >> (b & 63)) & 1ull; };
  // measure of column j (wave-uniform), the m with col_off[m] <= j <
  // col_off[m+1]: the number of measures m' < M-1 with col_off[m'+1] <= j.
  // Up to 65 measures lane l holds col_off[l+1], so the count is one ballot;
  // beyond, a binary search over col_off.
  const bool few = M <= 65;
  const int64_t co0 = col_off[few ? (lane + 1 < M ? lane + 1 : M) : 0];
  const int64_t co = (few && lane < M - 1) ? co0 : INT64_MAX;
  auto measure_of = [&](int64_t j) {
    if (few) return (int)__popcll(__ballot(co <= j));
    int lo = 0, hi = M;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (col_off[mid] <= j) lo = mid;
      else hi = mid;
    }
    return lo;
  };

  double umx = 0.0;  // largest |wbar| this wave writes
  // the masks of a batch of KC columns (clamped to the last column)
  auto load_batch = [&](int64_t bt, uint64_t (&w0)[KC][NCH], uint64_t (&w1)[KC][NCH]) {
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      const int64_t j = bt * KC + kc < T ? bt * KC + kc : T - 1;
      load_mask(mk + j * mld, w0[kc]);
      if (mk1) {
        load_mask(mk1 + j * mld, w1[kc]);
      } else {
#pragma unroll
        for (int c = 0; c < NCH; ++c) w1[kc][c] = 0ull;
      }
    }
  };
  // a wave that loops requests the next batch's masks before this batch's
  // gathers are used
  uint64_t w0[KC][NCH], w1[KC][NCH];
  if (wave * KC < T) load_batch(wave, w0, w1);
  for (int64_t bt = wave; bt * KC < T; bt += nwaves) {
    const int64_t jb = bt * KC;
    // active slots and gathers
    int m[KC], pc[KC], b0[KC], b1[KC];
    double v0[KC], v1[KC], u0[KC], u1[KC], c0[KC], c1[KC], qa[KC];
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      const int64_t j = jb + kc;
      const bool in = j < T;
      const int mm = measure_of(j);
      m[kc] = mm;
      int n = 0;
      b0[kc] = -1;
      b1[kc] = -1;
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        uint64_t x = in ? w0[kc][c] : 0ull;
        n += __popcll(x);
        if (x && b0[kc] < 0) {
          b0[kc] = c * 64 + __builtin_ctzll(x);
          x &= x - 1ull;
        }
        if (x && b1[kc] < 0) b1[kc] = c * 64 + __builtin_ctzll(x);
      }
      pc[kc] = n;
      v0[kc] = v1[kc] = u0[kc] = u1[kc] = c0[kc] = c1[kc] = 0.0;
      if (n) {
        const int64_t jo = (in ? j : 0) * (int64_t)R;
        const double* __restrict__ Vm = V + (int64_t)mm * R;
        const int r0 = row_of(b0[kc]);
        v0[kc] = Vm[r0];
        u0[kc] = U[jo + r0];
        c0[kc] = Cacc[jo + r0];
        if (b1[kc] >= 0) {
          const int r1 = row_of(b1[kc]);
          v1[kc] = Vm[r1];
          u1[kc] = U[jo + r1];
          c1[kc] = Cacc[jo + r1];
        }
      }
      qa[kc] = Qacc[in ? j : T - 1];
    }
    uint64_t n0[KC][NCH], n1[KC][NCH];
    const bool more = (bt + nwaves) * KC < T;
    if (more) load_batch(bt + nwaves, n0, n1);

#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      const int64_t j = jb + kc;
      const unsigned long long any = __ballot(pc[kc] != 0);
      if (any == 0ull) continue;  // nothing active (or past the end): nothing moves
      const double* __restrict__ Vm = V + (int64_t)m[kc] * R;
      double* __restrict__ Uc = U + j * (int64_t)R;
      double* __restrict__ Cc = Cacc + j * (int64_t)R;
      unsigned long long* __restrict__ Wm = wacc + (int64_t)m[kc] * R;
      const int n = pc[kc];
      const double x0 = n ? v0[kc] + (bit_of(w1[kc], b0[kc]) ? u0[kc] : 0.0) : 0.0;
      const double x1 = n > 1 ? v1[kc] + (bit_of(w1[kc], b1[kc]) ? u1[kc] : 0.0) : 0.0;
      auto walk = [&](auto&& f) {  // every active bit of the lane, in order
#pragma unroll
        for (int c = 0; c < NCH; ++c)
          for (uint64_t x = w0[kc][c]; x; x &= x - 1ull) {
            const int b = c * 64 + __builtin_ctzll(x);
            const int r = row_of(b);
            f(r, Vm[r] + (bit_of(w1[kc], b) ? Uc[r] : 0.0));
          }
      };
      double sum, cnt;
      if (__ballot(n > 1) == 0ull && __popcll(any) == 1) {
        const int L = __builtin_ctzll(any);
        sum = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x0), L),
                               __builtin_amdgcn_readlane(__double2loint(x0), L));
        cnt = 1.0;
      } else {
        double s = x0 + x1;
        if (n > 2) {
          s = 0.0;
          walk([&](int, double x) { s += x; });
        }
        sum = wave_reduce<OpSum>(s);
        cnt = wave_reduce<OpSum>((double)n);
      }
      const double mean = sum / cnt;
      if (lane == 0) Qacc[j] = qa[kc] + mean;
      auto put = [&](int r, double wb, double cold) {
        Uc[r] = wb;
        if (wb != 0.0) {
          Cc[r] = cold + wb;
          atomicAdd(Wm + r, adj_to_fixed(wb, sc.E));
          umx = fmax(umx, adj_mag(wb));
        }
      };
      if (n > 2) {
        walk([&](int r, double x) { put(r, x - mean, Cc[r]); });
      } else if (n) {
        put(row_of(b0[kc]), x0 - mean, c0[kc]);
        if (n > 1) put(row_of(b1[kc]), x1 - mean, c1[kc]);
      }
    }
    if (more) {
#pragma unroll
      for (int kc = 0; kc < KC; ++kc)
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          w0[kc][c] = n0[kc][c];
          w1[kc][c] = n1[kc][c];
        }
    }
  }
  umx = wave_reduce<OpMax>(umx);
  if (lane == 0 && umx > 0.0)
    atomicMax(gptr(a.mx) + 3 + (a.slot + 1) % 3, (unsigned long long)__double_as_longlong(umx));
}

}  // namespace mam

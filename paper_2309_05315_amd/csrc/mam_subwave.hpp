// Column kernel for short columns with sub-wave groups: NT = 16 or 32 lanes
// per column, so one wave advances 64/NT columns at once.  For R up to a few
// hundred rows a whole wave per column leaves most lanes idle and repeats the
// column's fixed chain (loads, reductions, Newton step) per column; here each
// group of NT lanes does that chain for its own column, side by side with the
// other groups of the wave.
//
// The iteration is the one of the column kernel (mam_kernels.hpp): per plan
// column w = theta + 2b - c/rho in FP64 (Alg. 1 Step 2, Prop. 2 eq.
// (row_sol)), the exact projection onto Delta_R(q_s) by warm-started Newton
// steps with the same exactness certificate (Prop. 3), theta' = pi_hat - b,
// and the row sums of pi_hat, each entry rounded to 64-bit fixed point,
// into the marginal's accumulators at the end of every segment.  Only the reductions differ: they
// run over the group's NT lanes with DPP row operations (a butterfly, so every
// lane of the group ends with the same total), and every per-column value is
// held per lane, since the groups of a wave are at different columns.
//
// Segments and schedule tables are those of the column kernel with
// NG = 256/NT groups per workgroup; a group takes blocks of kb columns.  No
// diagnostics or active-set recording (the host takes the one-wave kernel
// for those).
#pragma once

#include "mam_kernels.hpp"

namespace mam {

// Sum / min / max over the NT lanes of a group (NT = 16: one DPP row; 32: two
// rows, combined through a swizzle that swaps lanes i and i^16).  Every lane
// of the group returns the same value.
template <int NT, class Op>
__device__ __forceinline__ double group_reduce(double v) {
  v = Op::f(v, dpp_move<0xb1, 0xf>(v, Op::id()));   // quad_perm [1,0,3,2]
  v = Op::f(v, dpp_move<0x4e, 0xf>(v, Op::id()));   // quad_perm [2,3,0,1]
  v = Op::f(v, dpp_move<0x141, 0xf>(v, Op::id()));  // row_half_mirror
  v = Op::f(v, dpp_move<0x140, 0xf>(v, Op::id()));  // row_mirror
  if constexpr (NT == 32) {
    constexpr int kSwap16 = 0x1f | (0x10 << 10);  // bit mode: and 0x1f, xor 0x10
    const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), kSwap16);
    const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), kSwap16);
    v = Op::f(v, __hiloint2double(hi, lo));
  }
  return v;
}

template <int NT>
__device__ __forceinline__ int group_sum_i(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0xb1, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x4e, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xf, 0xf, false);
  if constexpr (NT == 32) v += __builtin_amdgcn_ds_swizzle(v, 0x1f | (0x10 << 10));
  return v;
}

template <typename T, int NT, int VPT, int VEC, bool STREAM>
__global__ void __launch_bounds__(256) subwave_kernel(ColArgs<T> a) {
  static_assert(NT == 16 || NT == 32, "sub-wave groups have 16 or 32 lanes");
  static_assert(VPT % VEC == 0, "VPT must be a multiple of VEC");
  constexpr int NG = 256 / NT;   // column groups per workgroup
  constexpr int NCH = VPT / VEC;  // vector chunks per thread
  extern __shared__ double lds_dyn[];
  double* lds_b = lds_dyn;               // [VPT][NT], the segment's b (shared by the groups)
  // [NG][VPT][NT], each group's fixed-point row sums of pi_hat
  unsigned long long* lds_fix = reinterpret_cast<unsigned long long*>(lds_dyn + VPT * NT);

  const int gtid = threadIdx.x;
  const int g = gtid / NT;  // group (not wave-uniform)
  const int tid = gtid % NT;
  const int lane = gtid & 63;
  unsigned long long* const fix = lds_fix + (size_t)g * VPT * NT;

  const int wg = logical_block(blockIdx.x, gridDim.x, a.xcd_remap);
  // the stop flag and the segment range requested together
  const int stopv = a.stop != nullptr ? *gptr(a.stop) : 0;
  const int sb0 = a.wg_seg[wg], se0 = a.wg_seg[wg + 1];
  if (uniform_i(stopv) != 0) return;  // the run has stopped
  const int sb = uniform_i(sb0), se = uniform_i(se0);
  for (int si = sb; si < se; ++si) {
    const ProbDev<T>& P = a.probs[uniform_i(a.seg_p[si])];
    T* const theta = gptr((T*)uniform_l((int64_t)P.theta));
    const T* const cost = gptr((const T*)uniform_l((int64_t)P.cost));
    const T* const qv = gptr((const T*)uniform_l((int64_t)P.q));
    const int32_t* const cidx = gptr((const int32_t*)uniform_l((int64_t)P.cidx));
    const int64_t ld = uniform_l(P.ld), cost_ld = uniform_l(P.cost_ld);
    const int R = uniform_i(P.R), cost_mode = uniform_i(P.cost_mode), warm = uniform_i(P.warm);
    const bool relaxed = uniform_i(P.relaxed) != 0;
    const double inv_rho = uniform_d(P.inv_rho);
    double* const lamv = gptr((double*)uniform_l((int64_t)P.lam));
    const int m = uniform_i(a.seg_m[si]);
    const int64_t j0 = uniform_l(a.seg_j0[si]), j1 = uniform_l(a.seg_j1[si]);
    const int64_t stride = uniform_i(a.seg_st[si]);
    const double Sm = uniform_d(gptr(P.Sd)[m]);
    unsigned long long* const accm = gptr((unsigned long long*)uniform_l((int64_t)P.acc)) + (size_t)m * R;
    const double fxm = uniform_d(gptr(P.fx)[m]);
    const int64_t off_m = uniform_l(gptr(P.col_off)[m]);
    const double* __restrict__ pmm = gptr(P.pm) + (size_t)m * R;
    const double* __restrict__ pv = gptr(P.p);

    const double t = damping_t(gptr(P.d2part), uniform_i(P.nb), uniform_d(P.rho), uniform_d(P.gamma), lane);
    if (gtid == 0 && j0 == 0) gptr(P.t_out)[0] = t;

    // b^(m) at the group's rows (group 0 writes what every group reads); a
    // row past R gets b = -inf, so its w is -inf: never active
    __syncthreads();
    if (g == 0) {
#pragma unroll
      for (int k = 0; k < VPT; ++k) {
        const int r = ((k / VEC) * NT + tid) * VEC + (k % VEC);
        lds_b[k * NT + tid] = (r < R) ? t * (pv[r] - pmm[r]) / Sm : -__builtin_huge_val();
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < VPT; ++k) fix[k * NT + tid] = 0ull;
    T nb[VPT];
#pragma unroll
    for (int k = 0; k < VPT; ++k) nb[k] = (T)(-lds_b[k * NT + tid]);

    // this group's columns: blocks of kb (one column: sub-wave groups take
    // one column in flight), the block of group g at j0 + g*kb, the next one
    // 'stride' columns on
    const int kb = uniform_i(a.kb);
    const int sh = __builtin_ctz(kb);
    const int64_t gbase = j0 + (int64_t)g * kb;
    auto block_exists = [&](int64_t i) { return gbase + (i >> sh) * stride < j1; };
    auto col_of = [&](int64_t i, int64_t& j) -> bool {
      const int64_t base = gbase + (i >> sh) * stride;
      j = base + (i & (kb - 1));
      return base < j1 && j < (base + kb < j1 ? base + kb : j1);
    };
    auto cost_index = [&](int64_t j) -> int64_t {
      if (cost_mode == MAM_COST_INDEXED) return cidx[j];
      if (cost_mode == MAM_COST_SHARED) return j - off_m;
      return j;
    };
    // raw loads of a step: the group's column, or the segment's first
    // column when the group has none at this step (loaded and ignored)
    struct Buf {
      T th[VPT], c[VPT], q;
      double l;
    };
    auto issue = [&](int64_t i, Buf& b) {
      int64_t j;
      if (!col_of(i, j)) j = j0;
      b.q = qv[j];
      b.l = lamv[j];
      const T* __restrict__ thp = theta + j * ld;
      const T* __restrict__ cp = cost + cost_index(j) * cost_ld;
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const int r0 = (c * NT + tid) * VEC < R ? (c * NT + tid) * VEC : 0;
        T tv[VEC], cv[VEC];
        if constexpr (STREAM) load_vec_nt<T, VEC>(thp + r0, tv);
        else load_vec<T, VEC>(thp + r0, tv);
        load_vec<T, VEC>(cp + r0, cv);
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          b.th[c * VEC + v] = tv[v];
          b.c[c * VEC + v] = cv[v];
        }
      }
    };

    auto body = [&](int64_t i, const Buf& b) {
      int64_t j;
      const bool valid = col_of(i, j);
      double w[VPT];
#pragma unroll
      for (int k = 0; k < VPT; ++k) w[k] = ((double)b.th[k] + 2.0 * lds_b[k * NT + tid]) - (double)b.c[k] * inv_rho;
      const double tau = valid ? (double)b.q : 0.0;
      bool act = valid && tau > 0.0;
      double lam = (act && warm) ? b.l : __builtin_nan("");
      if (!act) lam = __builtin_huge_val();
      int mask = 0, nprev = -1;
      for (int it = 0; it < R + 4; ++it) {
        if (__ballot(act) == 0ull) break;
        const bool cold = lam != lam;
        double S = 0.0, lo = __builtin_huge_val(), hi = -__builtin_huge_val();
        int n = 0, bits = 0;
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
          const double x = w[k];
          const bool in = act && x > lam;
          if (__ballot(in) == 0ull) {
            hi = fmax(hi, x);
          } else {
            n += in;
            bits |= (int)in << k;
            S += in ? x : 0.0;
            lo = fmin(lo, in ? x : __builtin_huge_val());
            hi = fmax(hi, in ? -__builtin_huge_val() : x);
          }
        }
        S = group_reduce<NT, OpSum>(S);
        n = group_sum_i<NT>(n);
        const double mnA = (double)float_down(group_reduce<NT, OpMin>(lo));
        const double mxN = (double)float_up(group_reduce<NT, OpMax>(hi));
        double wmx = 0.0;  // w_max on a cold round (nothing is active then)
        if (__ballot(act && cold) != 0ull) wmx = group_reduce<NT, OpMax>(hi);
        if (act) {
          mask = bits;
          if (n == 0) {
            if (cold) {
              lam = wmx - tau;  // the exact lower bound w_max - tau
              nprev = 0x7fffffff;
            } else if (nprev < 0) {
              lam = __builtin_nan("");  // the warm start lay above w_max: a cold round
            } else {
              act = false;  // w_max - tau rounded to w_max: the column is 0
              mask = 0;
            }
          } else {
            const double ln = (S - tau) / (double)n;
            if (n == nprev || (mnA >= ln && mxN <= ln)) act = false;  // mask is the exact active set
            nprev = n;
            lam = ln;
          }
        }
      }
      // theta' = -b, patched at the active rows with max(w - lam, 0) - b
      const double lout = relaxed ? fmax(lam, 0.0) : lam;
      T out[VPT];
#pragma unroll
      for (int k = 0; k < VPT; ++k) out[k] = nb[k];
      if (__ballot(mask != 0) != 0ull) {
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
          if ((mask >> k) & 1) {
            const double ph = fmax(w[k] - lout, 0.0);
            out[k] = (T)(ph - lds_b[k * NT + tid]);
            fix[k * NT + tid] += to_fixed(ph, fxm);
          }
        }
      }
      if (valid) {
        T* __restrict__ thp = theta + j * ld;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          const int r0 = (c * NT + tid) * VEC;
          if (r0 < R) {
            T ov[VEC];
#pragma unroll
            for (int v = 0; v < VEC; ++v) ov[v] = out[c * VEC + v];
            if (r0 + VEC <= R) {
              if constexpr (STREAM) store_vec_nt<T, VEC>(thp + r0, ov);
              else store_vec<T, VEC>(thp + r0, ov);
            } else {
#pragma unroll
              for (int v = 0; v < VEC; ++v)
                if (r0 + v < R) thp[r0 + v] = ov[v];
            }
          }
        }
        if (tid == 0) lamv[j] = lam;
      }
    };

    // two buffers: the next step's loads are in flight while a step computes
    Buf b0, b1;
    if (__ballot(block_exists(0)) != 0ull) {
      issue(0, b0);
      for (int64_t i = 0;; i += 2) {
        issue(i + 1, b1);
        body(i, b0);
        if (__ballot(block_exists(i + 1)) == 0ull) break;
        issue(i + 2, b0);
        body(i + 1, b1);
        if (__ballot(block_exists(i + 2)) == 0ull) break;
      }
    }

    // the segment's row sums of pi_hat into the fixed-point accumulators
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
      const unsigned long long f = fix[k * NT + tid];
      if (f != 0ull) atomicAdd(accm + ((k / VEC) * NT + tid) * VEC + (k % VEC), f);
    }
  }
}

}  // namespace mam

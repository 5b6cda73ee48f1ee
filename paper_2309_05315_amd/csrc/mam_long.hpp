// Device code of MAM for long plan columns: R beyond what one workgroup
// holds in registers.  The free-support formulation (Theorem c: measures on
// one K^d grid with alpha_m = 1/M) has R = ((K-1)M+1)^d candidate support
// points, 349,281 for M = 10 images of 60 x 60 pixels.
//
// A column is cut into row tiles of RB = 256*VPT rows; inside a tile each of
// the four waves of a workgroup owns an interleaved quarter of the rows (a
// sub-tile).  Thread tid holds rows rb*RB + ((k/VEC)*256 + tid)*VEC + k%VEC,
// k < VPT.  One iteration of Alg. 1 is three kernels plus the marginal and
// averaging kernels of the short path:
//
//   scan       per (sub-tile, column): w = theta + 2b - c/rho, the sub-tile's
//              maximum w_loc, and every entry with w > w_loc - q_s appended
//              as (row, w) to the column's candidate list.  An entry left out
//              has w <= w_loc - q_s <= w_max - q_s <= lambda (one entry of a
//              projection onto Delta_R(q_s) carries at most q_s, Prop. 3), so
//              it is inactive.
//   threshold  per column: the exact threshold of Prop. 3 from the candidates
//              alone.  Newton steps on the piecewise-linear root with an
//              exactness certificate; every step is kept >= w_max - q_s, so
//              the left-out entries stay below it.
//   write      per (sub-tile, column): theta' = -b everywhere, patched with
//              max(w - lambda, 0) - b at the candidates above lambda, and the
//              row-sum partials of the tile (fixed order, no atomics).
//
// The candidate lists are the only cross-workgroup exchange: theta and c are
// read once and theta written once per iteration.  A column whose candidates
// exceed the list capacity is handled from theta and c directly: threshold
// rounds over the whole column, and a write pass that recomputes w before
// overwriting theta.  Summation orders are fixed: results are bitwise
// reproducible.
#pragma once

#include "mam_kernels.hpp"

namespace mam {

constexpr int LNT = 256;  // threads per workgroup of the tile kernels (4 waves)

template <typename T>
struct LongArgs {
  T* theta;
  const T* cost;
  const T* q;
  const int32_t* cidx;
  int64_t ld, cost_ld;
  int32_t R, cost_mode, M, nrb;  // nrb: row tiles per column
  int32_t cap, warm;             // candidate capacity per column; warm starts on
  double rho, inv_rho, gamma;
  double* t;                     // damping t^k of the iteration (set by damping_kernel)
  const double* p;               // R, averaged marginal
  const double* pm;              // M x R marginals
  const double* d2part;          // ceil(R/256) partial sums of d^2
  int32_t nb, pad;
  const double* Sd;              // S^m as double
  const int64_t* col_off;        // M+1
  // work items (row tile, measure, column range), in schedule order
  const int32_t* it_rb;
  const int32_t* it_m;
  const int64_t* it_j0;
  const int64_t* it_j1;
  const int64_t* it_poff;        // offset of the item's RB row-sum partials
  const int32_t* wg_it;          // items of workgroup w: [wg_it[w], wg_it[w+1])
  // candidates
  int32_t* cnt;                  // T: entries appended to column j this iteration
  int32_t* crow;                 // T*cap rows
  double* cw;                    // T*cap values of w
  int32_t* sub_off;              // (j*nrb + rb)*4 + wave: first entry of the sub-tile
  int32_t* sub_cnt;              //                        entries of the sub-tile
  double* lam;                   // T: threshold (previous one in, new one out)
  double* partial;
  const int32_t* stop;           // early-exit flag, or null
  int64_t T_cols;
};

template <typename T>
__device__ __forceinline__ const T* long_cost_col(const LongArgs<T>& a, int64_t j, int64_t off_m) {
  int64_t cc;
  if (a.cost_mode == MAM_COST_INDEXED) cc = a.cidx[j];
  else if (a.cost_mode == MAM_COST_SHARED) cc = j - off_m;
  else cc = j;
  return a.cost + cc * a.cost_ld;
}

// b^(m)_r = t (p_r - p^(m)_r) / S^m: every kernel forms it with this one
// expression, so all of them see the same value.
__device__ __forceinline__ double long_b(double t, const double* p, const double* pmm, int r, double Sm) {
  return t * (p[r] - pmm[r]) / Sm;
}

// ---- scan: w, sub-tile maxima, candidate lists ---------------------------
template <typename T, int VPT, int VEC>
__global__ void __launch_bounds__(LNT)
long_scan_kernel(LongArgs<T> a) {
  constexpr int NCH = VPT / VEC, RB = LNT * VPT;
  static_assert(VPT % VEC == 0 && VPT <= 16, "tile shape");
  if (a.stop != nullptr && uniform_i(*gptr(a.stop)) != 0) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = uniform_i(tid >> 6);
  const int R = a.R, cap = a.cap, nrb = a.nrb;
  const double t = uniform_d(*gptr(a.t)), inv_rho = a.inv_rho;
  const T* const theta = gptr(a.theta);
  const T* const qv = gptr(a.q);
  int32_t* const cnt = gptr(a.cnt);
  int32_t* const crow = gptr(a.crow);
  double* const cw = gptr(a.cw);
  const int ib = uniform_i(a.wg_it[blockIdx.x]), ie = uniform_i(a.wg_it[blockIdx.x + 1]);
  for (int it = ib; it < ie; ++it) {
    const int rb = uniform_i(a.it_rb[it]), m = uniform_i(a.it_m[it]);
    const int64_t j0 = uniform_l(a.it_j0[it]), j1 = uniform_l(a.it_j1[it]);
    const double Sm = uniform_d(gptr(a.Sd)[m]);
    const int64_t off_m = uniform_l(gptr(a.col_off)[m]);
    const double* __restrict__ pmm = gptr(a.pm) + (size_t)m * R;
    const double* __restrict__ pv = gptr(a.p);
    const int rbase = rb * RB;
    int row[VPT];
    double b[VPT];
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
      row[k] = rbase + ((k / VEC) * LNT + tid) * VEC + (k % VEC);
      b[k] = row[k] < R ? long_b(t, pv, pmm, row[k], Sm) : 0.0;
    }
    // raw theta and c of the next column in flight while this one is scanned
    T rt[VPT], rc[VPT], rq;
    auto issue = [&](int64_t j) {
      const T* __restrict__ thp = theta + j * a.ld;
      const T* __restrict__ cp = long_cost_col(a, j, off_m);
      rq = qv[j];
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const int r0 = row[c * VEC] < R ? row[c * VEC] : rbase;  // rows past R read the tile's first (masked)
        T tv[VEC], cv[VEC];
        load_vec_nt<T, VEC>(thp + r0, tv);
        load_vec<T, VEC>(cp + r0, cv);
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          rt[c * VEC + v] = tv[v];
          rc[c * VEC + v] = cv[v];
        }
      }
    };
    if (j0 < j1) issue(j0);
    for (int64_t j = j0; j < j1; ++j) {
      double w[VPT];
      double mx = -__builtin_huge_val();
#pragma unroll
      for (int k = 0; k < VPT; ++k) {
        const double x = ((double)rt[k] + 2.0 * b[k]) - (double)rc[k] * inv_rho;
        w[k] = row[k] < R ? x : -__builtin_huge_val();
        mx = fmax(mx, w[k]);
      }
      const double tau = uniform_d((double)rq);
      if (j + 1 < j1) issue(j + 1);
      mx = wave_max(mx);
      const double thr = mx - tau;
      int bits = 0;
      if (tau > 0.0) {
#pragma unroll
        for (int k = 0; k < VPT; ++k) bits |= (int)(w[k] > thr) << k;
      }
      // slot-major order inside the wave: position = entries of earlier
      // slots + earlier lanes of this slot
      unsigned long long bal[VPT];
      int n = 0;
#pragma unroll
      for (int k = 0; k < VPT; ++k) {
        bal[k] = __ballot((bits >> k) & 1);
        n += __popcll(bal[k]);
      }
      int off = 0;
      if (n > 0) {
        if (lane == 0) off = atomicAdd(cnt + j, n);
        off = __builtin_amdgcn_readlane(off, 0);
        int base = off;
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
          if ((bits >> k) & 1) {
            const int pos = base + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(bal[k] >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((unsigned)bal[k], 0u));
            if (pos < cap) {
              crow[j * cap + pos] = row[k];
              cw[j * cap + pos] = w[k];
            }
          }
          base += __popcll(bal[k]);
        }
      }
      if (lane == 0) {
        const int64_t s = (j * nrb + rb) * 4 + wv;
        gptr(a.sub_off)[s] = off;
        gptr(a.sub_cnt)[s] = n;
      }
    }
  }
}

// ---- threshold: one wave per column -------------------------------------
// Sums over the candidates in a fixed order: sub-tiles in order, and inside
// a sub-tile lane l takes entries l, l+64, ...; then a fixed wave tree.
template <typename T>
__global__ void __launch_bounds__(256)
long_threshold_kernel(LongArgs<T> a) {
  if (a.stop != nullptr && uniform_i(*gptr(a.stop)) != 0) return;
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + uniform_i(threadIdx.x >> 6);
  if (j >= a.T_cols) return;  // whole waves; no barriers below
  const int R = a.R, cap = a.cap, nsub = a.nrb * 4;
  const double tau = uniform_d((double)gptr(a.q)[j]);
  double* const lamv = gptr(a.lam);
  if (!(tau > 0.0)) {
    if (lane == 0) lamv[j] = __builtin_huge_val();  // q_s = 0: the column is 0
    return;
  }
  const int ntot = uniform_i(gptr(a.cnt)[j]);
  const bool listed = ntot <= cap;
  const int32_t* __restrict__ so = gptr(a.sub_off) + j * nsub;
  const int32_t* __restrict__ sc = gptr(a.sub_cnt) + j * nsub;
  const double* __restrict__ cwj = gptr(a.cw) + j * cap;
  // an unlisted column is recomputed from theta and c: its measure and b
  int m = 0;
  if (!listed) {
    while (m + 1 < a.M && gptr(a.col_off)[m + 1] <= j) ++m;
  }
  const double t = uniform_d(*gptr(a.t));
  const double Sm = gptr(a.Sd)[m];
  const int64_t off_m = gptr(a.col_off)[m];
  const double* __restrict__ pmm = gptr(a.pm) + (size_t)m * R;
  const double* __restrict__ pv = gptr(a.p);
  const T* __restrict__ thp = gptr(a.theta) + j * a.ld;
  const T* __restrict__ cp = long_cost_col(a, j, off_m);
  // visit every entry of the column that can be active, in the fixed order
  auto visit = [&](auto&& f) {
    if (listed) {
      for (int s = 0; s < nsub; ++s) {
        const int o = uniform_i(so[s]), c = uniform_i(sc[s]);
        for (int e = lane; e < c; e += 64) f(cwj[o + e]);
      }
    } else {
      for (int r = lane; r < R; r += 64)
        f(((double)thp[r] + 2.0 * long_b(t, pv, pmm, r, Sm)) - (double)cp[r] * a.inv_rho);
    }
  };
  double wmx = -__builtin_huge_val();
  visit([&](double x) { wmx = fmax(wmx, x); });
  wmx = wave_max(wmx);
  const double lo = wmx - tau;  // the root is >= w_max - tau
  const double lprev = lamv[j];
  double lam = (a.warm && lprev == lprev && lprev > lo) ? lprev : lo;
  int nprev = -1;
  for (int round = 0; round < R + 4; ++round) {
    double S = 0.0, mnA = __builtin_huge_val(), mxN = -__builtin_huge_val();
    double nd = 0.0;
    visit([&](double x) {
      if (x > lam) {
        S += x;
        nd += 1.0;
        mnA = fmin(mnA, x);
      } else {
        mxN = fmax(mxN, x);
      }
    });
    S = wave_sum(S);
    nd = wave_sum(nd);
    mnA = wave_reduce<OpMin>(mnA);
    mxN = wave_max(mxN);
    const int n = (int)nd;
    if (n == 0) {
      if (lam > lo) {  // a warm start at or above w_max: restart from the bound
        lam = lo;
        nprev = -1;
        continue;
      }
      // w_max - tau rounded to w_max (tau below half an ulp): the column is 0
      lam = __builtin_huge_val();
      break;
    }
    const double ln = (S - tau) / (double)n;
    if (ln >= lo && (n == nprev || (mnA >= ln && mxN <= ln))) {
      lam = ln;  // the set above lam is exactly the active set
      break;
    }
    nprev = n;
    lam = fmax(ln, lo);
  }
  if (lane == 0) lamv[j] = lam;
}

// ---- write: theta' and the tile's row-sum partials ----------------------
// Every row is written once, by its owner thread: the active rows of the
// column among the thread's slots are found first (from the wave's
// candidates, or from w recomputed for an unlisted column), then the
// thread's vectors are stored.  Dynamic LDS: VPT*256 doubles of row-sum
// patches (each row owned by one thread: no atomics).
template <typename T, int VPT, int VEC>
__global__ void __launch_bounds__(LNT)
long_write_kernel(LongArgs<T> a) {
  constexpr int NCH = VPT / VEC, RB = LNT * VPT;
  if (a.stop != nullptr && uniform_i(*gptr(a.stop)) != 0) return;
  extern __shared__ double lds_dyn[];
  double* fix = lds_dyn;  // [VPT][256]
  const int tid = threadIdx.x;
  const int wv = uniform_i(tid >> 6);
  const int R = a.R, cap = a.cap, nrb = a.nrb;
  const double t = uniform_d(*gptr(a.t)), inv_rho = a.inv_rho;
  T* const theta = gptr(a.theta);
  const int32_t* const cnt = gptr(a.cnt);
  const int32_t* const crow = gptr(a.crow);
  const double* const cw = gptr(a.cw);
  const double* const lamv = gptr(a.lam);
  const int ib = uniform_i(a.wg_it[blockIdx.x]), ie = uniform_i(a.wg_it[blockIdx.x + 1]);
  for (int it = ib; it < ie; ++it) {
    const int rb = uniform_i(a.it_rb[it]), m = uniform_i(a.it_m[it]);
    const int64_t j0 = uniform_l(a.it_j0[it]), j1 = uniform_l(a.it_j1[it]);
    const double Sm = uniform_d(gptr(a.Sd)[m]);
    const int64_t off_m = uniform_l(gptr(a.col_off)[m]);
    const double* __restrict__ pmm = gptr(a.pm) + (size_t)m * R;
    const double* __restrict__ pv = gptr(a.p);
    const int rbase = rb * RB;
    int row[VPT];
    double b[VPT];
    T nb[VPT];  // -b rounded to the storage type: every inactive entry's new value
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
      row[k] = rbase + ((k / VEC) * LNT + tid) * VEC + (k % VEC);
      b[k] = row[k] < R ? long_b(t, pv, pmm, row[k], Sm) : 0.0;
      nb[k] = (T)(-b[k]);
      fix[k * LNT + tid] = 0.0;  // each thread touches only its own slots
    }
    for (int64_t j = j0; j < j1; ++j) {
      T* __restrict__ thp = theta + j * a.ld;
      const double lam = uniform_d(lamv[j]);
      double w[VPT];
      int act = 0;  // bit k: slot k is active
#pragma unroll
      for (int k = 0; k < VPT; ++k) w[k] = -__builtin_huge_val();
      if (uniform_i(cnt[j]) <= cap) {
        // this wave's candidates; the owner of each active row takes it
        const int64_t s = (j * nrb + rb) * 4 + wv;
        const int o = uniform_i(gptr(a.sub_off)[s]), c = uniform_i(gptr(a.sub_cnt)[s]);
        for (int e = 0; e < c; ++e) {
          const double x = uniform_d(cw[j * cap + o + e]);
          if (!(x > lam)) continue;
          const int rr = uniform_i(crow[j * cap + o + e]) - rbase;
          if ((rr / VEC) % LNT == tid) {
            const int ks = (rr / (VEC * LNT)) * VEC + rr % VEC;
#pragma unroll
            for (int k = 0; k < VPT; ++k)
              if (k == ks) w[k] = x;
            act |= 1 << ks;
          }
        }
      } else {
        // no candidate list: w from theta and c, read before theta is overwritten
        const T* __restrict__ cp = long_cost_col(a, j, off_m);
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
          if (row[k] < R) {
            w[k] = ((double)thp[row[k]] + 2.0 * b[k]) - (double)cp[row[k]] * inv_rho;
            act |= (int)(w[k] > lam) << k;
          }
        }
      }
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const int r0 = row[c * VEC];
        T out[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const int k = c * VEC + v;
          out[v] = nb[k];
          if ((act >> k) & 1) {
            out[v] = (T)(fmax(w[k] - lam, 0.0) - b[k]);
            fix[k * LNT + tid] += (double)out[v] - (double)nb[k];
          }
        }
        if (r0 + VEC <= R) {
          store_vec_nt<T, VEC>(thp + r0, out);
        } else {
#pragma unroll
          for (int v = 0; v < VEC; ++v)
            if (r0 + v < R) thp[r0 + v] = out[v];
        }
      }
    }
    // the item's row sums: (#columns) * (-b) plus the patches
    const double ncols = (double)(j1 - j0);
    double* __restrict__ part = gptr(a.partial) + uniform_l(a.it_poff[it]);
#pragma unroll
    for (int k = 0; k < VPT; ++k)
      if (row[k] < R) part[row[k] - rbase] = ncols * (double)nb[k] + fix[k * LNT + tid];
  }
}

// Row sums of the plans into the item partials (initialisation).
template <typename T>
__global__ void __launch_bounds__(256)
long_rowsum_kernel(LongArgs<T> a, int rows_per_tile) {
  const int ib = a.wg_it[blockIdx.x], ie = a.wg_it[blockIdx.x + 1];
  for (int it = ib; it < ie; ++it) {
    const int rbase = a.it_rb[it] * rows_per_tile;
    const int rend = rbase + rows_per_tile < a.R ? rbase + rows_per_tile : a.R;
    for (int r = rbase + threadIdx.x; r < rend; r += 256) {
      double s = 0.0;
      for (int64_t j = a.it_j0[it]; j < a.it_j1[it]; ++j) s += (double)a.theta[j * a.ld + r];
      a.partial[a.it_poff[it] + (r - rbase)] = s;
    }
  }
}

}  // namespace mam

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
//   scan       per (column, sub-tile): w = theta + 2b - c/rho, the sub-tile's
//              maximum w_loc, and the entries with w > w_loc - q_s (at most
//              E of them kept, in fixed slots).  An entry left out has
//              w <= w_loc - q_s <= w_max - q_s <= lambda (one entry of a
//              projection onto Delta_R(q_s) carries at most q_s, Prop. 3), so
//              it is inactive.
//   threshold  per column (one wave): the exact threshold of Prop. 3 from the
//              kept entries of the sub-tiles with w_loc > w_max - q_s (no other
//              sub-tile can hold an active entry).  Newton steps on the
//              piecewise-linear root with an exactness certificate; every step
//              is kept >= w_max - q_s, so the left-out entries stay below it.
//   write      per (column, sub-tile): theta' = -b everywhere, patched with
//              max(w - lambda, 0) - b at the kept entries above lambda (none
//              unless w_loc > lambda), and the tile's row-sum partials (fixed
//              order, no atomics).
//
// The sub-tile headers and slots are the only cross-workgroup exchange: theta
// and c are read once and theta written once per iteration.  A sub-tile with
// more than E candidates is recomputed from theta and c where it is needed
// (threshold rounds, and the write pass before theta is overwritten).  Every
// sum has a fixed order: results are bitwise reproducible.
#pragma once

#include <utility>

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
  int32_t cap, warm;             // candidate slots per sub-tile; warm starts on
  int32_t relaxed, pad0;         // columns projected onto {u >= 0, sum u <= q_s}
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
  // per (column j, sub-tile s = rb*4 + wave), index h = j*nrb*4 + s
  double* hmax;                  // the sub-tile's maximum of w
  int32_t* hcnt;                 // its candidates (entries with w > hmax - q_s)
  int32_t* crow;                 // h*cap + e: row of candidate e < min(hcnt, cap)
  double* cw;                    //            its w
  double* lam;                   // T: threshold (previous one in, new one out)
  double* partial;
  const int32_t* stop;           // early-exit flag, or null
  int64_t T_cols;
  // grid cost (cost_mode MAM_COST_GRID): row r is point (i0, i1) of an
  // n0 x n1 grid (last axis fastest; gdim 1: i0 = r, gn1 = 1 and a second
  // axis of origin and spacing 0) with coordinates go[k] + i_k * gh[k], and
  // cost column s is the point gz[s*gdim ..]: c_rs = sum_k (x_rk - z_sk)^2,
  // rounded to the storage type
  int32_t gdim, gn1;
  double go[2], gh[2];
  const double* gz;
  // sparse store (MAM_FLAG_SPARSE_STORE): between iterations the plans are
  // held per (column j, sub-tile s) either as the dense rows in theta
  // (pcnt[s*T + j] < 0) or as pcnt[s*T + j] >= 0 patches (row, value), in
  // slots h*cap + e with h = j*nsub + s, over the value nbv[par][m][r] that
  // every other entry of measure m's row r holds
  int32_t sparse, pad1;
  int32_t* spar;                 // par: which half of nbv holds the stored plans
  int32_t* pcnt;
  int32_t* prow;                 // h*cap + e: row of patch e
  T* pval;                       //            its value
  T* nbv;                        // 2 x M x R
  // diagnostics of the iteration (the DIAG instances): per column j,
  // ldiag[4j..4j+3] = <c_s, pi_hat_s>, the column's measure residual, its
  // threshold rounds and active entries; per write workgroup w,
  // wdiag[w*DIAG_STRIDE + 2] = max |theta' - theta| over its entries (dense
  // store only)
  double* ldiag;
  double* wdiag;
};

// Coordinate k of grid index i: origin + i * spacing, each operation rounded
// (no fused multiply-add).
template <typename T>
__device__ __forceinline__ double grid_coord(const LongArgs<T>& a, int k, int i) {
#pragma clang fp contract(off)
  return a.go[k] + (double)i * a.gh[k];
}

// The grid cost of the point (x0, x1) and the column's point (z0, z1),
// evaluated in the order of its definition (each product and sum rounded, no
// fused multiply-add), then rounded to the storage type as a stored cost
// would be.  On a one-dimensional grid x1 = z1 = 0, so the second term is +0
// and c = d0^2 exactly.
template <typename T>
__device__ __forceinline__ double grid_cost_xy(double x0, double x1, double z0, double z1) {
#pragma clang fp contract(off)
  const double d0 = x0 - z0, d1 = x1 - z1;
  const double c = d0 * d0 + d1 * d1;
  return (double)(T)c;
}

// The column's point (z0, z1) of cost column j (z1 = 0 on a 1-D grid).
template <typename T>
__device__ __forceinline__ void grid_point(const LongArgs<T>& a, int64_t j, int64_t off_m, double* z0, double* z1) {
  const double* z = gptr(a.gz) + (j - off_m) * a.gdim;
  *z0 = z[0];
  *z1 = a.gdim == 2 ? z[1] : 0.0;
}

template <typename T>
__device__ __forceinline__ double grid_cost(const LongArgs<T>& a, int r, double z0, double z1) {
  const int i0 = r / a.gn1;
  return grid_cost_xy<T>(grid_coord(a, 0, i0), grid_coord(a, 1, r - i0 * a.gn1), z0, z1);
}

template <typename T>
__device__ __forceinline__ const T* long_cost_col(const LongArgs<T>& a, int64_t j, int64_t off_m) {
  int64_t cc;
  if (a.cost_mode == MAM_COST_INDEXED) cc = a.cidx[j];
  else if (a.cost_mode == MAM_COST_SHARED) cc = j - off_m;
  else cc = j;
  return a.cost + cc * a.cost_ld;
}

// The value of v in lane l (l wave-uniform).
__device__ __forceinline__ double read_lane(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float read_lane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// w = theta + 2b - c/rho (FP64) from 2b: one expression with one fused
// multiply-add, so the scan, threshold and write kernels form the same value
// for an entry.
__device__ __forceinline__ double long_w(double th, double b2, double c, double inv_rho) {
  return __builtin_fma(-c, inv_rho, th + b2);
}

// b^(m)_r = t (p_r - p^(m)_r) / S^m: every kernel forms it with this one
// expression, so all of them see the same value.
__device__ __forceinline__ double long_b(double t, const double* p, const double* pmm, int r, double Sm) {
  return t * (p[r] - pmm[r]) / Sm;
}

// Thread tt of the tile at rbase owns rows rbase + ((k/VEC)*LNT + tt)*VEC + k%VEC,
// k < VPT; row offset rr = r - rbase is slot k of thread (rr/VEC) % LNT.
__device__ __forceinline__ int slot_owner(int rr, int vec) { return (rr / vec) % LNT; }
__device__ __forceinline__ int slot_of(int rr, int vec) { return (rr / (vec * LNT)) * vec + rr % vec; }

// Sparse store: apply the pc <= cap patches (lane e holds row pr and value
// pv of patch e) to the values th of thread tt's rows, in patch order.
template <typename T, int VPT, int VEC>
__device__ __forceinline__ void apply_patches(int pc, int pr, T pv, int rbase, int tt, T (&th)[VPT]) {
  for (int e = 0; e < pc; ++e) {
    const int rr = __builtin_amdgcn_readlane(pr, e) - rbase;
    const T v = read_lane(pv, e);
    if (slot_owner(rr, VEC) == tt) {
      const int k = slot_of(rr, VEC);
#pragma unroll
      for (int kk = 0; kk < VPT; ++kk)
        if (kk == k) th[kk] = v;
    }
  }
}

// The stored plan values of thread tt's rows of the tile at rbase in column j
// (sub-tile si, measure m), 0 at rows past R: the dense rows, or the
// measure's common values with the sub-tile's patches.
template <typename T, int VPT, int VEC>
__device__ void stored_rows(const LongArgs<T>& a, int64_t j, int si, int rbase, int tt, int m, int par,
                            T (&th)[VPT]) {
  const int R = a.R;
  const int64_t h = j * (a.nrb * 4) + si;
  const int pc = a.sparse ? uniform_i(gptr(a.pcnt)[(int64_t)si * a.T_cols + j]) : -1;
  const T* __restrict__ src = pc < 0 ? gptr(a.theta) + j * a.ld : gptr(a.nbv) + ((size_t)par * a.M + m) * R;
#pragma unroll
  for (int k = 0; k < VPT; ++k) {
    const int r = rbase + ((k / VEC) * LNT + tt) * VEC + (k % VEC);
    th[k] = r < R ? src[r] : T(0);
  }
  if (pc > 0) {
    const int lane = threadIdx.x & 63;
    const int pr = lane < pc ? gptr(a.prow)[h * a.cap + lane] : 0;
    const T pv = lane < pc ? gptr(a.pval)[h * a.cap + lane] : T(0);
    apply_patches<T, VPT, VEC>(pc, pr, pv, rbase, tt, th);
  }
}

// ---- scan: w, sub-tile maxima, candidates -------------------------------
// GRID: the cost is formed from the row's grid point and the column's point
// instead of being read (only theta is streamed).  SP: the sparse-store
// instance; an unpatched entry of a sparse sub-tile has theta = the common
// value, so theta + 2b is a per-row constant of the item ('base', in
// registers) and w costs one fused multiply-add; 2b itself sits in LDS for
// dense sub-tiles and patched rows (dynamic LDS: VPT*256 doubles, each
// thread reading only its own slots).
template <typename T, int VPT, int VEC, bool GRID, bool SP>
__global__ void __launch_bounds__(LNT)
long_scan_kernel(LongArgs<T> a) {
  constexpr int NCH = VPT / VEC, RB = LNT * VPT;
  // columns in flight per wave: two where the registers allow it at two
  // waves per SIMD (FP32 tiles of 16 values in vectors), else one (and one
  // in the sparse-store instance, whose columns mostly load no theta)
  constexpr int PF = (!SP && sizeof(T) == 4 && VPT == 16 && VEC > 1) ? 2 : 1;
  static_assert(VPT % VEC == 0 && VPT <= 16, "tile shape");
  if (a.stop != nullptr && uniform_i(*gptr(a.stop)) != 0) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = uniform_i(tid >> 6);
  const int R = a.R, cap = a.cap, nsub = a.nrb * 4;
  const double t = uniform_d(*gptr(a.t)), inv_rho = a.inv_rho;
  const T* const theta = gptr(a.theta);
  const T* const qv = gptr(a.q);
  int32_t* const crow = gptr(a.crow);
  double* const cw = gptr(a.cw);
  constexpr bool sparse = SP;
  const int par = sparse ? uniform_i(*gptr(a.spar)) : 0;
  extern __shared__ double lds_dyn[];
  double* const lds_b2 = lds_dyn;  // SP: [VPT][LNT]
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
    // 2 b_r, or -inf for rows past R: their w is then -inf (theta and c are
    // finite), below every threshold, without a select per entry
    double b2[SP ? 1 : VPT];
    double base[SP ? VPT : 1];  // SP: common value + 2b of the row
    double gx0[GRID ? VPT : 1], gx1[GRID ? VPT : 1];  // grid coordinates of the rows
    const T* __restrict__ nbm = sparse ? gptr(a.nbv) + ((size_t)par * a.M + m) * R : nullptr;
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
      row[k] = rbase + ((k / VEC) * LNT + tid) * VEC + (k % VEC);
      const double b2k = row[k] < R ? 2.0 * long_b(t, pv, pmm, row[k], Sm) : -__builtin_huge_val();
      if constexpr (SP) {
        lds_b2[k * LNT + tid] = b2k;
        base[k] = (double)(row[k] < R ? nbm[row[k]] : T(0)) + b2k;
      } else {
        b2[k] = b2k;
      }
      if constexpr (GRID) {
        const int i0 = row[k] / a.gn1;
        gx0[k] = grid_coord(a, 0, i0);
        gx1[k] = grid_coord(a, 1, row[k] - i0 * a.gn1);
      }
    }
    // raw theta and c (or the column's point) of the next PF columns in
    // flight while one is scanned: PF buffers, used in turn; with the sparse
    // store, the column's patch count and lane e's patch instead of theta
    // when the sub-tile is not dense
    T rt[PF][VPT], rc[PF][GRID ? 1 : VPT], rq[PF];
    double rz[PF][2];
    int pcs[PF], prs[PF];
    T pvs[PF];
    // columns run in blocks: the whole item, or 64 columns with the sparse
    // store (lane l then holds the patch count of column jlo + l)
    int64_t jlo = j0, jhi = j1;
    int pcl = -1;
    auto issue = [&](auto S, int64_t j) {
      constexpr int s = decltype(S)::value;
      const T* __restrict__ thp = theta + j * a.ld;
      rq[s] = qv[j];
      if constexpr (GRID) grid_point(a, j, off_m, &rz[s][0], &rz[s][1]);
      const int pc = sparse ? __builtin_amdgcn_readlane(pcl, (int)(j - jlo)) : -1;
      pcs[s] = pc;
      if (pc >= 0) {
        const int64_t h = j * nsub + rb * 4 + wv;
        prs[s] = lane < pc ? gptr(a.prow)[h * cap + lane] : 0;
        pvs[s] = lane < pc ? gptr(a.pval)[h * cap + lane] : T(0);
      }
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const int r0 = row[c * VEC] < R ? row[c * VEC] : rbase;  // rows past R read the tile's first (masked)
        if (pc < 0) {
          T tv[VEC];
          load_vec_nt<T, VEC>(thp + r0, tv);
#pragma unroll
          for (int v = 0; v < VEC; ++v) rt[s][c * VEC + v] = tv[v];
        }
        if constexpr (!GRID) {
          T cv[VEC];
          load_vec<T, VEC>(long_cost_col(a, j, off_m) + r0, cv);
#pragma unroll
          for (int v = 0; v < VEC; ++v) rc[s][c * VEC + v] = cv[v];
        }
      }
    };
    // scan column j from buffer S; with NEXT, load column min(j + PF, j1 - 1)
    // into that buffer (past the item's end it loads its last column again:
    // unconditional loads keep the buffers in place across iterations)
    auto column = [&](auto S, auto NEXT, int64_t j) {
      constexpr int s = decltype(S)::value;
      double w[VPT];
      double mx = -__builtin_huge_val();
      const double z0 = uniform_d(rz[s][0]), z1 = uniform_d(rz[s][1]);
      auto cost_k = [&](int k) -> double {
        if constexpr (GRID) return grid_cost_xy<T>(gx0[k], gx1[k], z0, z1);
        else return (double)rc[s][k];
      };
      if constexpr (SP) {
        // theta + 2b of every entry: base for a sparse sub-tile, the dense
        // rows plus 2b from LDS otherwise; w is one fused multiply-add each
        const bool sp = pcs[s] >= 0;
        double bs[VPT];
        if (sp) {
#pragma unroll
          for (int k = 0; k < VPT; ++k) bs[k] = base[k];
        } else {
#pragma unroll
          for (int k = 0; k < VPT; ++k) bs[k] = (double)rt[s][k] + lds_b2[k * LNT + tid];
        }
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
          w[k] = __builtin_fma(-cost_k(k), inv_rho, bs[k]);
          mx = fmax(mx, w[k]);
        }
        if (sp) {
          // the patched rows (each patch raises its entry, so the maximum
          // only grows)
          for (int e = 0; e < pcs[s]; ++e) {
            const int rr = __builtin_amdgcn_readlane(prs[s], e) - rbase;
            const T v = read_lane(pvs[s], e);
            if (slot_owner(rr, VEC) == tid) {
              const int kp = slot_of(rr, VEC), r = rbase + rr;
              const double c = GRID ? grid_cost(a, r, z0, z1) : (double)long_cost_col(a, j, off_m)[r];
              const double wn = long_w((double)v, lds_b2[kp * LNT + tid], c, inv_rho);
#pragma unroll
              for (int kk = 0; kk < VPT; ++kk)
                if (kk == kp) w[kk] = wn;
              mx = fmax(mx, wn);
            }
          }
        }
      } else {
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
          w[k] = long_w((double)rt[s][k], b2[k], cost_k(k), inv_rho);
          mx = fmax(mx, w[k]);
        }
      }
      const double tau = uniform_d((double)rq[s]);
      if constexpr (decltype(NEXT)::value) issue(S, j + PF < jhi ? j + PF : jhi - 1);
      mx = wave_max(mx);
      const double thr = mx - tau;
      // slots in slot-major order inside the wave: position = candidates of
      // earlier slots + earlier lanes of this slot (rows past R have w = -inf
      // and are never candidates)
      const int64_t h = j * nsub + rb * 4 + wv;
      int n = 0;
      if (tau > 0.0) {
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
          const bool sel = w[k] > thr;
          const unsigned long long bal = __ballot(sel);
          if (sel) {
            const int pos = n + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
            if (pos < cap) {
              crow[h * cap + pos] = row[k];
              cw[h * cap + pos] = w[k];
            }
          }
          n += __popcll(bal);
        }
      }
      if (lane == 0) {
        gptr(a.hmax)[h] = mx;
        gptr(a.hcnt)[h] = n;
      }
    };
    using YES = std::true_type;
    using NO = std::false_type;
    const int64_t jstep = sparse ? 64 : j1 - j0;
    for (jlo = j0; jlo < j1; jlo += jstep) {
      jhi = jlo + jstep < j1 ? jlo + jstep : j1;
      if (sparse) pcl = jlo + lane < jhi ? gptr(a.pcnt)[(int64_t)(rb * 4 + wv) * a.T_cols + jlo + lane] : -1;
      // buffer i holds column j + i (clamped to the block's last column)
      static_for<PF>([&](auto I) { issue(I, jlo + I < jhi ? jlo + I : jhi - 1); });
      int64_t j = jlo;
      for (; j + PF - 1 < jhi; j += PF) static_for<PF>([&](auto I) { column(I, YES{}, j + I); });
      static_for<PF - 1>([&](auto I) {
        if (j + I < jhi) column(I, NO{}, j + I);
      });
    }
  }
}

// ---- threshold: one wave per column -------------------------------------
// Only sub-tiles with w_loc > w_max - q_s are visited, in index order; inside
// one, lane e takes kept entry e, or (more than E candidates) lane l
// recomputes the VPT values of thread 64*wave + l of the tile.  The wave
// sums in a fixed tree: the order is fixed.
template <typename T, int VPT, int VEC, bool DIAG>
__global__ void __launch_bounds__(256)
long_threshold_kernel(LongArgs<T> a) {
  constexpr int RB = LNT * VPT;
  if (a.stop != nullptr && uniform_i(*gptr(a.stop)) != 0) return;
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + uniform_i(threadIdx.x >> 6);
  if (j >= a.T_cols) return;  // whole waves; no barriers below
  const int R = a.R, cap = a.cap, nsub = a.nrb * 4;
  const double tau = uniform_d((double)gptr(a.q)[j]);
  double* const lamv = gptr(a.lam);
  if (!(tau > 0.0)) {
    if (lane == 0) {
      lamv[j] = __builtin_huge_val();  // q_s = 0: the column is 0
      if constexpr (DIAG) {
        double* const dj = gptr(a.ldiag) + j * 4;
        dj[0] = dj[1] = dj[2] = dj[3] = 0.0;
      }
    }
    return;
  }
  const double* __restrict__ hm = gptr(a.hmax) + j * nsub;
  const int32_t* __restrict__ hc = gptr(a.hcnt) + j * nsub;
  const double* __restrict__ cwj = gptr(a.cw) + j * nsub * (int64_t)cap;
  double wmx = -__builtin_huge_val();
  for (int s = lane; s < nsub; s += 64) wmx = fmax(wmx, hm[s]);
  wmx = wave_max(wmx);
  const double lo = wmx - tau;  // the root is >= w_max - tau
  // an overflowed sub-tile is recomputed from theta and c: the column's
  // measure and b
  int m = 0;
  while (m + 1 < a.M && gptr(a.col_off)[m + 1] <= j) ++m;
  const double t = uniform_d(*gptr(a.t));
  const double Sm = gptr(a.Sd)[m];
  const int64_t off_m = gptr(a.col_off)[m];
  const double* __restrict__ pmm = gptr(a.pm) + (size_t)m * R;
  const double* __restrict__ pv = gptr(a.p);
  const int par = a.sparse ? uniform_i(*gptr(a.spar)) : 0;
  const T* __restrict__ cp = long_cost_col(a, j, off_m);
  double z0 = 0.0, z1 = 0.0;
  if (a.gdim) grid_point(a, j, off_m, &z0, &z1);
  auto costv = [&](int r) { return a.gdim ? grid_cost(a, r, z0, z1) : (double)cp[r]; };
  auto visit = [&](auto&& f) {
    for (int s0 = 0; s0 < nsub; s0 += 64) {
      const int s = s0 + lane;
      unsigned long long rel = __ballot(s < nsub && hm[s < nsub ? s : 0] > lo);
      while (rel) {
        const int si = s0 + __builtin_ctzll(rel);
        rel &= rel - 1;
        const int n = uniform_i(hc[si]);
        if (n <= cap) {
          if (lane < n) f(cwj[(int64_t)si * cap + lane], gptr(a.crow)[(j * nsub + si) * (int64_t)cap + lane]);
        } else {
          const int rbase = (si >> 2) * RB, tt = (si & 3) * 64 + lane;
          T th[VPT];
          stored_rows<T, VPT, VEC>(a, j, si, rbase, tt, m, par, th);
#pragma unroll
          for (int k = 0; k < VPT; ++k) {
            const int r = rbase + ((k / VEC) * LNT + tt) * VEC + (k % VEC);
            if (r < R) f(long_w((double)th[k], 2.0 * long_b(t, pv, pmm, r, Sm), costv(r), a.inv_rho), r);
          }
        }
      }
    }
  };
  const double lprev = lamv[j];
  double lam = (a.warm && lprev == lprev && lprev > lo) ? lprev : lo;
  int nprev = -1, nrounds = 0, nact = 0;
  for (int round = 0; round < R + 4; ++round) {
    ++nrounds;
    double S = 0.0, mnA = __builtin_huge_val(), mxN = -__builtin_huge_val();
    double nd = 0.0;
    visit([&](double x, int) {
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
      nact = n;
      break;
    }
    nprev = n;
    lam = fmax(ln, lo);
  }
  // relaxed columns: max(w - max(lam, 0), 0) is the projection onto
  // {u >= 0, sum u <= q_s} (the write pass patches only entries above it)
  if (a.relaxed) lam = fmax(lam, 0.0);
  if (lane == 0) lamv[j] = lam;
  if constexpr (DIAG) {
    // the column's pi_hat = max(w - lam, 0) at the same entries and in the
    // same arithmetic as the write pass: its sum against q_s and against the
    // cost (fixed order: sub-tiles in order, lanes by the wave sum)
    double cs = 0.0, wc = 0.0;
    if (lam < __builtin_huge_val()) {
      visit([&](double x, int r) {
        if (x > lam) {
          const double ph = fmax(x - lam, 0.0);
          cs += ph;
          wc += costv(r) * ph;
        }
      });
    }
    cs = wave_sum(cs);
    wc = wave_sum(wc);
    if (lane == 0) {
      double* const dj = gptr(a.ldiag) + j * 4;
      dj[0] = wc;
      dj[1] = a.relaxed ? fmax(cs - tau, 0.0) : fabs(cs - tau);
      dj[2] = (double)nrounds;
      dj[3] = (double)(lam < __builtin_huge_val() ? nact : 0);
    }
  }
}

// ---- write: theta' and the tile's row-sum partials ----------------------
// Usually a column's sub-tile is stored as -b in whole vectors, and the few
// kept entries above lambda are then patched by the thread that owns the
// row (its own earlier store to the same address comes first).  An
// overflowed sub-tile above lambda is done vector by vector instead: theta
// and c are read, w formed, and the patched vector stored in one go.  The
// thresholds and sub-tile headers of 256 columns at a time are loaded into
// LDS together (one column per thread), so no column waits on memory for
// them.  Dynamic LDS: VPT*256 doubles of row-sum patches (each row owned by
// one thread: no atomics).
template <typename T, int VPT, int VEC, bool DIAG>
__global__ void __launch_bounds__(LNT)
long_write_kernel(LongArgs<T> a) {
  constexpr int NCH = VPT / VEC, RB = LNT * VPT;
  if (a.stop != nullptr && uniform_i(*gptr(a.stop)) != 0) return;
  double dth = 0.0;  // DIAG, dense store: max |theta' - theta| of this thread's entries
  extern __shared__ double lds_dyn[];
  double* fix = lds_dyn;  // [VPT][256]
  constexpr int WB = 128;  // columns whose thresholds and headers are staged at once
  __shared__ double s_lam[WB], s_max[4][WB];
  __shared__ int s_cnt[4][WB];
  const int tid = threadIdx.x;
  const int wv = uniform_i(tid >> 6);
  const int R = a.R, cap = a.cap, nsub = a.nrb * 4;
  const double t = uniform_d(*gptr(a.t)), inv_rho = a.inv_rho;
  T* const theta = gptr(a.theta);
  const double* const hm = gptr(a.hmax);
  const int32_t* const hc = gptr(a.hcnt);
  const int32_t* const crow = gptr(a.crow);
  const double* const cw = gptr(a.cw);
  const double* const lamv = gptr(a.lam);
  const bool sparse = a.sparse != 0;
  const int par = sparse ? uniform_i(*gptr(a.spar)) : 0;
  const int ib = uniform_i(a.wg_it[blockIdx.x]), ie = uniform_i(a.wg_it[blockIdx.x + 1]);
  for (int it = ib; it < ie; ++it) {
    const int rb = uniform_i(a.it_rb[it]), m = uniform_i(a.it_m[it]);
    const int64_t j0 = uniform_l(a.it_j0[it]), j1 = uniform_l(a.it_j1[it]);
    const double Sm = uniform_d(gptr(a.Sd)[m]);
    const int64_t off_m = uniform_l(gptr(a.col_off)[m]);
    const double* __restrict__ pmm = gptr(a.pm) + (size_t)m * R;
    const double* __restrict__ pv = gptr(a.p);
    const int rbase = rb * RB;
    const int sub = rb * 4 + wv;
    auto row = [&](int k) { return rbase + ((k / VEC) * LNT + tid) * VEC + (k % VEC); };
    T nb[VPT];  // -b rounded to the storage type: every inactive entry's new value
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
      nb[k] = (T)(-(row(k) < R ? long_b(t, pv, pmm, row(k), Sm) : 0.0));
      fix[k * LNT + tid] = 0.0;  // each thread touches only its own slots
    }
    // sparse store: the tile's new common values of measure m, written once
    // (by the item that starts at the measure's first column) into the half
    // of nbv the stored plans do not use yet
    if (sparse && j0 == off_m) {
      T* __restrict__ nbn = gptr(a.nbv) + ((size_t)(par ^ 1) * a.M + m) * R;
#pragma unroll
      for (int k = 0; k < VPT; ++k)
        if (row(k) < R) nbn[row(k)] = nb[k];
    }
    const T* __restrict__ nbo = sparse ? gptr(a.nbv) + ((size_t)par * a.M + m) * R : nullptr;
    for (int64_t jb = j0; jb < j1; jb += WB) {
      // thresholds and this tile's four sub-tile headers of 256 columns
      __syncthreads();  // the previous block's readers are done
      if (tid < WB && jb + tid < j1) {
        const int64_t jj = jb + tid;
        s_lam[tid] = lamv[jj];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          s_max[q][tid] = hm[jj * nsub + rb * 4 + q];
          s_cnt[q][tid] = hc[jj * nsub + rb * 4 + q];
        }
      }
      __syncthreads();
      const int64_t je = jb + WB < j1 ? jb + WB : j1;
    auto column = [&](int64_t j) {
      const double lam = uniform_d(s_lam[j - jb]), lmax = uniform_d(s_max[wv][j - jb]);
      const int n = uniform_i(s_cnt[wv][j - jb]);
      T* __restrict__ thp = theta + j * a.ld;
      const bool some = lmax > lam;  // some entry of this sub-tile is active
      const int64_t h = j * nsub + sub;
      int32_t* const pcj = sparse ? gptr(a.pcnt) + (int64_t)sub * a.T_cols + j : nullptr;
      if (some && n > cap) {
        // more candidates than slots: vector by vector, w from theta and c
        // (one vector at a time, so this rare path holds few registers); the
        // stored plans of a sparse sub-tile are the common values and its
        // patches, and the sub-tile is dense in theta afterwards
        const T* __restrict__ cp = long_cost_col(a, j, off_m);
        double z0 = 0.0, z1 = 0.0;
        if (a.gdim) grid_point(a, j, off_m, &z0, &z1);
        const int pc = sparse ? uniform_i(*pcj) : -1;
        const int lane = tid & 63;
        const int pr = lane < pc ? gptr(a.prow)[h * cap + lane] : 0;
        const T pvv = lane < pc ? gptr(a.pval)[h * cap + lane] : T(0);
#pragma unroll 1
        for (int c = 0; c < NCH; ++c) {
          const int r0 = rbase + (c * LNT + tid) * VEC;
          const int rl = r0 < R ? r0 : rbase;  // rows past R read the tile's first (masked)
          T tv[VEC], out[VEC];
          if (pc < 0) {
            load_vec<T, VEC>(thp + rl, tv);
          } else {
#pragma unroll
            for (int v = 0; v < VEC; ++v) tv[v] = r0 + v < R ? nbo[r0 + v] : T(0);
            for (int e = 0; e < pc; ++e) {
              const int rr = __builtin_amdgcn_readlane(pr, e) - rbase;
              const T val = read_lane(pvv, e);
              if (slot_owner(rr, VEC) == tid && slot_of(rr, VEC) / VEC == c) {
#pragma unroll
                for (int v = 0; v < VEC; ++v)
                  if (v == rr % VEC) tv[v] = val;
              }
            }
          }
#pragma unroll
          for (int v = 0; v < VEC; ++v) {
            out[v] = T(0);  // rows past R are not stored
            if (r0 + v < R) {
              const double bk = long_b(t, pv, pmm, r0 + v, Sm);
              const T nbk = (T)(-bk);  // the entry's value when inactive (nb of its slot)
              const double cc = a.gdim ? grid_cost(a, r0 + v, z0, z1) : (double)cp[r0 + v];
              const double w = long_w((double)tv[v], 2.0 * bk, cc, inv_rho);
              out[v] = nbk;
              if (w > lam) {
                const double ph = fmax(w - lam, 0.0);
                out[v] = (T)(ph - bk);
                fix[(c * VEC + v) * LNT + tid] += ph;  // theta' - (-b) before rounding
              }
            }
          }
          if constexpr (DIAG) {
#pragma unroll
            for (int v = 0; v < VEC; ++v)
              if (r0 + v < R) dth = fmax(dth, fabs((double)out[v] - (double)tv[v]));
          }
          if (r0 + VEC <= R) {
            store_vec_nt<T, VEC>(thp + r0, out);
          } else {
#pragma unroll
            for (int v = 0; v < VEC; ++v)
              if (r0 + v < R) thp[r0 + v] = out[v];
          }
        }
        if (sparse && lane == 0) *pcj = -1;
        return;
      }
      // DIAG, dense store: the entries' old values, and which of them the
      // patches below overwrite
      T old[VPT];
      unsigned pmask = 0u;
      if constexpr (DIAG) {
        if (!sparse) {
#pragma unroll
          for (int c = 0; c < NCH; ++c) {
            const int r0 = row(c * VEC);
            T ov[VEC];
            if (r0 + VEC <= R) {
              load_vec<T, VEC>(thp + r0, ov);
            } else {
#pragma unroll
              for (int v = 0; v < VEC; ++v) ov[v] = r0 + v < R ? thp[r0 + v] : T(0);
            }
#pragma unroll
            for (int v = 0; v < VEC; ++v) old[c * VEC + v] = ov[v];
          }
        }
      }
      if (!sparse) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          const int r0 = row(c * VEC);
          T out[VEC];
#pragma unroll
          for (int v = 0; v < VEC; ++v) out[v] = nb[c * VEC + v];
          if (r0 + VEC <= R) {
            store_vec_nt<T, VEC>(thp + r0, out);
          } else {
#pragma unroll
            for (int v = 0; v < VEC; ++v)
              if (r0 + v < R) thp[r0 + v] = out[v];
          }
        }
      }
      if (some) {
        // the kept entries above lambda (n <= cap <= 64): lane e reads entry
        // e and forms its patch, all at once; then, in entry order, the
        // owner of each row stores it (or, with the sparse store, the
        // patches are kept in slots) and adds it to the row sum
        const int e = tid & 63;
        const double xe = e < n ? cw[h * cap + e] : -__builtin_huge_val();
        const int re = e < n ? crow[h * cap + e] : rbase;
        const bool keep = xe > lam;
        const double bk = keep ? long_b(t, pv, pmm, re, Sm) : 0.0;
        const double dfix = fmax(xe - lam, 0.0);  // theta' - (-b) before rounding
        const T val = (T)(dfix - bk);
        unsigned long long sel = __ballot(keep);
        if (sparse) {
          const int pos = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(sel >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((unsigned)sel, 0u));
          if (keep) {
            gptr(a.prow)[h * cap + pos] = re;
            gptr(a.pval)[h * cap + pos] = val;
          }
          if (e == 0) *pcj = __popcll(sel);
        }
        while (sel != 0ull) {
          const int l = __builtin_ctzll(sel);
          sel &= sel - 1ull;
          const int rr = __builtin_amdgcn_readlane(re, l) - rbase;
          if (slot_owner(rr, VEC) == tid) {
            if (!sparse) thp[rbase + rr] = read_lane(val, l);
            fix[slot_of(rr, VEC) * LNT + tid] += read_lane(dfix, l);
            if constexpr (DIAG) {
              if (!sparse) {
                const int sl = slot_of(rr, VEC);
                const double nv = (double)read_lane(val, l);
#pragma unroll
                for (int k = 0; k < VPT; ++k)
                  if (k == sl) dth = fmax(dth, fabs(nv - (double)old[k]));
                pmask |= 1u << sl;
              }
            }
          }
        }
      }
      if constexpr (DIAG) {
        // every other entry of the sub-tile became -b
        if (!sparse) {
#pragma unroll
          for (int k = 0; k < VPT; ++k)
            if (row(k) < R && !((pmask >> k) & 1u)) dth = fmax(dth, fabs((double)nb[k] - (double)old[k]));
        }
      }
    };
      if (sparse) {
        // sparse store: only columns whose sub-tile has an active entry need
        // work; the others get a patch count of 0, 64 columns at a time
        const int lane = tid & 63;
        for (int64_t c0 = jb; c0 < je; c0 += 64) {
          const int64_t jl = c0 + lane;
          const bool in = jl < je;
          const bool act = in && s_max[wv][in ? jl - jb : 0] > s_lam[in ? jl - jb : 0];
          if (in && !act) gptr(a.pcnt)[(int64_t)sub * a.T_cols + jl] = 0;
          unsigned long long am = __ballot(act);
          while (am != 0ull) {
            const int64_t j = c0 + __builtin_ctzll(am);
            am &= am - 1ull;
            column(j);
          }
        }
      } else {
        for (int64_t j = jb; j < je; ++j) column(j);
      }
    }
    // the item's row sums: (#columns) * (-b) plus the patches, in double
    // from the unrounded updates (as in the short column kernel: the stored
    // -b of the inactive entries would add the same rounding error from
    // every column of the measure)
    const double ncols = (double)(j1 - j0);
    double* __restrict__ part = gptr(a.partial) + uniform_l(a.it_poff[it]);
#pragma unroll
    for (int k = 0; k < VPT; ++k)
      if (row(k) < R) part[row(k) - rbase] = fix[k * LNT + tid] - ncols * long_b(t, pv, pmm, row(k), Sm);
  }
  if constexpr (DIAG) {
    __shared__ double sh_dth[4];
    const double m = wave_max(dth);
    if ((tid & 63) == 0) sh_dth[tid >> 6] = m;
    __syncthreads();
    if (tid == 0)
      gptr(a.wdiag)[(size_t)blockIdx.x * DIAG_STRIDE + 2] =
          sparse ? __builtin_nan("") : fmax(fmax(sh_dth[0], sh_dth[1]), fmax(sh_dth[2], sh_dth[3]));
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

// ---- sparse store: write-back --------------------------------------------
// Write the stored plans back into theta: every sparse sub-tile is stored as
// its common values (whole vectors) and then its patches (each by the thread
// owning the row, after its own store), and marked dense.
template <typename T, int VPT, int VEC>
__global__ void __launch_bounds__(LNT)
long_materialize_kernel(LongArgs<T> a) {
  constexpr int NCH = VPT / VEC, RB = LNT * VPT;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = uniform_i(tid >> 6);
  const int R = a.R, cap = a.cap, nsub = a.nrb * 4;
  const int par = uniform_i(*gptr(a.spar));
  T* const theta = gptr(a.theta);
  const int ib = uniform_i(a.wg_it[blockIdx.x]), ie = uniform_i(a.wg_it[blockIdx.x + 1]);
  for (int it = ib; it < ie; ++it) {
    const int rb = uniform_i(a.it_rb[it]), m = uniform_i(a.it_m[it]);
    const int64_t j0 = uniform_l(a.it_j0[it]), j1 = uniform_l(a.it_j1[it]);
    const int rbase = rb * RB;
    const T* __restrict__ nbm = gptr(a.nbv) + ((size_t)par * a.M + m) * R;
    T nb[VPT];
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
      const int r = rbase + ((k / VEC) * LNT + tid) * VEC + (k % VEC);
      nb[k] = r < R ? nbm[r] : T(0);
    }
    for (int64_t j = j0; j < j1; ++j) {
      const int64_t h = j * nsub + rb * 4 + wv;
      int32_t* const pcj = gptr(a.pcnt) + (int64_t)(rb * 4 + wv) * a.T_cols + j;
      const int pc = uniform_i(*pcj);
      if (pc < 0) continue;
      T* __restrict__ thp = theta + j * a.ld;
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const int r0 = rbase + (c * LNT + tid) * VEC;
        T out[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) out[v] = nb[c * VEC + v];
        if (r0 + VEC <= R) {
          store_vec_nt<T, VEC>(thp + r0, out);
        } else {
#pragma unroll
          for (int v = 0; v < VEC; ++v)
            if (r0 + v < R) thp[r0 + v] = out[v];
        }
      }
      if (pc > 0) {
        const int pr = lane < pc ? gptr(a.prow)[h * cap + lane] : 0;
        const T pvv = lane < pc ? gptr(a.pval)[h * cap + lane] : T(0);
        for (int e = 0; e < pc; ++e) {
          const int r = __builtin_amdgcn_readlane(pr, e);
          const T val = read_lane(pvv, e);
          if (slot_owner(r - rbase, VEC) == tid) thp[r] = val;
        }
      }
      if (lane == 0) *pcj = -1;
    }
  }
}

}  // namespace mam

// Host side of the MAM library: C ABI, validation, column schedule,
// workspace layout and kernel launches.  See mam.h for the contract and
// mam_kernels.hpp for the device code.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "mam.h"
#include "mam_aux_kernels.hpp"
#include "mam_dispatch.hpp"

namespace {

thread_local std::string g_err;

mam_status fail(mam_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(MAM_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

#define LAUNCH_CHECK(name)                                                         \
  do {                                                                             \
    hipError_t e_ = hipGetLastError();                                             \
    if (e_ != hipSuccess)                                                          \
      return fail(MAM_EHIP, "launch of %s failed: %s", name, hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
constexpr int64_t kMaxLds = 160 * 1024;  // LDS per compute unit on gfx950
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t partial, pm, pm_prev, p, p_prev, d2part, tval, diag, check, lam;
  size_t seg_m, seg_j0, seg_j1, seg_idx, wg_seg, mseg, col_off, Sd, aw;
  size_t total;
};

}  // namespace

struct mam_problem {
  int dtype = MAM_F64;
  int cost_mode = MAM_COST_PER_COLUMN;
  int64_t R = 0, M = 0, T = 0, ld = 0, cost_ld = 0, cost_ncols = 0;
  double rho = 1.0, gamma = INFINITY;
  uint32_t flags = 0;
  std::vector<int64_t> S, col_off;
  std::vector<double> Sd, aw;

  // schedule
  int nt = 0, vpt = 0, ng = 0, nwg = 0, xcd_remap = 0, kc = 1;
  int nt_req = 0, nwg_req = 0, kc_req = 0;
  std::vector<int32_t> seg_m, wg_seg, mseg, seg_idx;
  bool blocked = false;
  int xcd_req = 0;    // >0 on, <0 off, 0 automatic (on for cost-block-major orders)
  int order_req = 0;  // 0 automatic, 1 measure-major, 2 cost-block-major
  std::vector<int64_t> seg_j0, seg_j1;
  int nb = 0;  // average-kernel blocks = d^2 partials
  Layout lay{};

  // bound state
  char* ws = nullptr;
  size_t ws_bytes = 0;
  void* theta = nullptr;
  const void* cost = nullptr;
  const int32_t* cidx = nullptr;
  const void* q = nullptr;
  int vec = 1;
  bool inited = false;
  bool tables_uploaded = false;
  int64_t iters_done = 0;
  bool diag_valid = false;

  // timing
  bool timing = false;
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
};

namespace {

int vec_width(int dtype) { return dtype == MAM_F32 ? 4 : 2; }
size_t elem_bytes(int dtype) { return dtype == MAM_F32 ? 4 : 8; }

int pow2_ceil(int64_t x) {
  int v = 1;
  while (v < x) v <<= 1;
  return v;
}

// Pick threads per column and values per thread.  A column of R rows is held
// in registers: NT threads x VPT values, VPT <= 16.
mam_status choose_shape(mam_problem* p) {
  const int64_t R = p->R;
  int nt = p->nt_req;
  if (nt == 0) {
    // The fewest threads per column that keep a thread at 16 (float) or 8
    // (double) values: a column group then fits twice per compute unit
    // (registers and LDS), which measured fastest on MI355X; one wave per
    // column whenever that suffices (no barriers in the threshold rounds).
    const int64_t target = p->dtype == MAM_F32 ? 16 : 8;
    nt = 64;
    while (nt < 1024 && (int64_t)nt * target < R) nt *= 2;
  }
  if (nt != 64 && nt != 128 && nt != 256 && nt != 512 && nt != 1024)
    return fail(MAM_EINVAL, "threads_per_column must be 64, 128, 256, 512 or 1024 (got %d)", nt);
  int64_t per = (R + nt - 1) / nt;
  int vpt = pow2_ceil(per);
  if (nt >= 128 && vpt < 4) vpt = 4;  // multi-wave groups hold at least 4 values per thread
  if (vpt > 16) return fail(MAM_EUNSUPPORTED, "R = %lld needs more than 16 values per thread at %d threads per column", (long long)R, nt);
  const int ng = nt == 64 ? 4 : 1;
  if ((int64_t)vpt * nt * 8 * (1 + ng) > kMaxLds)
    return fail(MAM_EUNSUPPORTED, "R = %lld at %d threads per column needs more than 160 KiB of LDS", (long long)R, nt);
  int kc = p->kc_req ? p->kc_req : 1;
  if (kc != 1 && kc != 2 && kc != 4) return fail(MAM_EINVAL, "columns_in_flight must be 1, 2 or 4 (got %d)", kc);
  p->nt = nt;
  p->vpt = vpt;
  p->kc = kc;
  p->ng = nt == 64 ? 4 : 1;
  return MAM_OK;
}

// Columns that share a cost column (the same s under a shared cost, the
// same index under an indexed cost) should be streamed close together in
// time so the cost column is fetched into L2 once.  The column order is a
// list of tasks (measure, contiguous column range): cost-block-major when
// the cost layout allows it (block = B cost columns, about 2 MiB), else
// measure-major.  Workgroups take equal shares of the concatenated order;
// every piece of a task a workgroup owns is one segment (one row-sum
// partial).
struct Task {
  int m;
  int64_t lo, hi;
};

int64_t cost_block(const mam_problem* p) {
  const int64_t col_bytes = p->R * (int64_t)elem_bytes(p->dtype);
  int64_t b = 1;
  while (b * 2 * col_bytes <= (int64_t)(2 << 20) && b < 4096) b *= 2;
  return b;
}

// Upper bound on the number of segments, fixed before the index is known.
int64_t segment_bound(const mam_problem* p, int nwg) {
  if (p->cost_mode == MAM_COST_PER_COLUMN) return p->M + nwg;
  const int64_t nkb = (p->cost_ncols + cost_block(p) - 1) / cost_block(p);
  return nkb * p->M + nwg;
}

std::vector<Task> task_order(const mam_problem* p, const std::vector<int32_t>* idx, bool* is_blocked) {
  std::vector<Task> tasks;
  // automatic: cost-block-major for a shared cost, measure-major for an
  // indexed cost (the faster of the two on the measured workloads)
  const int order = p->order_req ? p->order_req : (p->cost_mode == MAM_COST_SHARED ? 2 : 1);
  bool blocked = p->cost_mode == MAM_COST_SHARED && order == 2;
  if (p->cost_mode == MAM_COST_INDEXED && idx && order == 2) {
    blocked = true;
    for (int64_t m = 0; m < p->M && blocked; ++m)
      for (int64_t j = p->col_off[m] + 1; j < p->col_off[m + 1]; ++j)
        if ((*idx)[j] < (*idx)[j - 1]) {
          blocked = false;
          break;
        }
  }
  *is_blocked = blocked;
  if (!blocked) {
    for (int64_t m = 0; m < p->M; ++m) tasks.push_back({(int)m, p->col_off[m], p->col_off[m + 1]});
    return tasks;
  }
  const int64_t B = cost_block(p);
  const int64_t nkb = (p->cost_ncols + B - 1) / B;
  for (int64_t kb = 0; kb < nkb; ++kb) {
    for (int64_t m = 0; m < p->M; ++m) {
      const int64_t o = p->col_off[m], S = p->S[m];
      int64_t lo, hi;
      if (p->cost_mode == MAM_COST_SHARED) {
        lo = o + std::min(S, kb * B);
        hi = o + std::min(S, (kb + 1) * B);
      } else {
        const int32_t* b = idx->data() + o;
        lo = o + (std::lower_bound(b, b + S, (int32_t)std::min<int64_t>(kb * B, INT32_MAX)) - b);
        hi = o + (std::lower_bound(b, b + S, (int32_t)std::min<int64_t>((kb + 1) * B, INT32_MAX)) - b);
      }
      if (hi > lo) tasks.push_back({(int)m, lo, hi});
    }
  }
  return tasks;
}

void build_schedule(mam_problem* p, const std::vector<int32_t>* idx = nullptr) {
  const int64_t T = p->T;
  const int ng = p->ng;
  int nwg = p->nwg_req;
  if (nwg <= 0) {
    const int64_t cap = 1024;
    int64_t cpw = std::max<int64_t>(1, (T + ng * cap - 1) / (ng * cap));
    nwg = (int)std::min<int64_t>(cap, (T + ng * cpw - 1) / (ng * cpw));
  }
  nwg = (int)std::max<int64_t>(1, std::min<int64_t>(nwg, T));
  p->nwg = nwg;
  bool blocked = false;
  const std::vector<Task> tasks = task_order(p, idx, &blocked);
  p->blocked = blocked;
  p->xcd_remap = p->xcd_req > 0 ? 1 : (p->xcd_req < 0 ? 0 : (p->blocked ? 1 : 0));
  p->seg_m.clear();
  p->seg_j0.clear();
  p->seg_j1.clear();
  p->wg_seg.assign(nwg + 1, 0);
  size_t ti = 0;
  int64_t tpos = 0;  // columns of tasks[ti] already assigned
  for (int w = 0; w < nwg; ++w) {
    int64_t need = T * (w + 1) / nwg - T * w / nwg;
    p->wg_seg[w] = (int32_t)p->seg_m.size();
    while (need > 0 && ti < tasks.size()) {
      const Task& tk = tasks[ti];
      const int64_t take = std::min(need, tk.hi - tk.lo - tpos);
      p->seg_m.push_back(tk.m);
      p->seg_j0.push_back(tk.lo + tpos);
      p->seg_j1.push_back(tk.lo + tpos + take);
      need -= take;
      tpos += take;
      if (tpos == tk.hi - tk.lo) {
        ++ti;
        tpos = 0;
      }
    }
  }
  p->wg_seg[nwg] = (int32_t)p->seg_m.size();
  // each measure's segments, in schedule order, for the marginal kernel
  p->mseg.assign(p->M + 1, 0);
  for (int32_t m : p->seg_m) ++p->mseg[m + 1];
  for (int64_t m = 0; m < p->M; ++m) p->mseg[m + 1] += p->mseg[m];
  p->seg_idx.assign(p->seg_m.size(), 0);
  {
    std::vector<int32_t> fill(p->mseg.begin(), p->mseg.end() - 1);
    for (size_t k = 0; k < p->seg_m.size(); ++k) p->seg_idx[fill[p->seg_m[k]]++] = (int32_t)k;
  }
  p->nb = (int)((p->R + 255) / 256);

  const size_t nseg = (size_t)std::max<int64_t>(segment_bound(p, nwg), (int64_t)p->seg_m.size());
  const size_t R = (size_t)p->R, M = (size_t)p->M;
  Layout& L = p->lay;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
  L.partial = take(nseg * R * 8);
  L.pm = take(M * R * 8);
  L.pm_prev = take(M * R * 8);
  L.p = take(R * 8);
  L.p_prev = take(R * 8);
  L.d2part = take((size_t)p->nb * 8);
  L.tval = take(8);
  L.diag = take((size_t)nwg * mam::DIAG_STRIDE * 8);
  L.lam = take((size_t)p->T * 8);
  L.check = take((M + 2) * 8);
  L.seg_m = take(nseg * 4);
  L.seg_j0 = take(nseg * 8);
  L.seg_j1 = take(nseg * 8);
  L.seg_idx = take(nseg * 4);
  L.wg_seg = take((size_t)(nwg + 1) * 4);
  L.mseg = take((M + 1) * 4);
  L.col_off = take((M + 1) * 8);
  L.Sd = take(M * 8);
  L.aw = take(M * 8);
  L.total = o;
  p->tables_uploaded = false;
}

template <typename U>
U* at(mam_problem* p, size_t off) { return reinterpret_cast<U*>(p->ws + off); }

mam_status upload_tables(mam_problem* p, hipStream_t st) {
  if (p->tables_uploaded) return MAM_OK;
  const Layout& L = p->lay;
  HIP_TRY(hipMemcpyAsync(p->ws + L.seg_m, p->seg_m.data(), p->seg_m.size() * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(p->ws + L.seg_j0, p->seg_j0.data(), p->seg_j0.size() * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(p->ws + L.seg_j1, p->seg_j1.data(), p->seg_j1.size() * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(p->ws + L.wg_seg, p->wg_seg.data(), p->wg_seg.size() * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(p->ws + L.mseg, p->mseg.data(), p->mseg.size() * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(p->ws + L.seg_idx, p->seg_idx.data(), p->seg_idx.size() * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(p->ws + L.col_off, p->col_off.data(), p->col_off.size() * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(p->ws + L.Sd, p->Sd.data(), p->Sd.size() * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(p->ws + L.aw, p->aw.data(), p->aw.size() * 8, hipMemcpyHostToDevice, st));
  p->tables_uploaded = true;
  return MAM_OK;
}

// ---------------------------------------------------------------------------
// column-kernel dispatch
// ---------------------------------------------------------------------------
template <typename T>
mam_status launch_column(mam_problem* p, hipStream_t st, int diag) {
  const Layout& L = p->lay;
  mam::ColArgs<T> a;
  a.theta = static_cast<T*>(p->theta);
  a.cost = static_cast<const T*>(p->cost);
  a.q = static_cast<const T*>(p->q);
  a.cidx = p->cidx;
  a.ld = p->ld;
  a.cost_ld = p->cost_ld;
  a.R = (int32_t)p->R;
  a.cost_mode = p->cost_mode;
  a.pm = at<double>(p, L.pm);
  a.p = at<double>(p, L.p);
  a.d2part = at<double>(p, L.d2part);
  a.nb = p->nb;
  a.warm = (p->flags & MAM_FLAG_COLD) ? 0 : 1;
  a.rho = p->rho;
  a.inv_rho = 1.0 / p->rho;
  a.gamma = p->gamma;
  a.col_off = at<int64_t>(p, L.col_off);
  a.Sd = at<double>(p, L.Sd);
  a.seg_m = at<int32_t>(p, L.seg_m);
  a.seg_j0 = at<int64_t>(p, L.seg_j0);
  a.seg_j1 = at<int64_t>(p, L.seg_j1);
  a.wg_seg = at<int32_t>(p, L.wg_seg);
  a.partial = at<double>(p, L.partial);
  a.lam = at<double>(p, L.lam);
  a.t_out = at<double>(p, L.tval);
  a.diag = at<double>(p, L.diag);
  a.nwg = p->nwg;
  a.xcd_remap = p->xcd_remap;
  const int kc = p->vec == 1 ? 1 : p->kc;
  mam::ColFn<T> fn = mam::pick_column<T>(p->nt, p->vpt, p->vec, kc, diag);
  if (!fn) return fail(MAM_EUNSUPPORTED, "no column kernel for nt=%d vpt=%d vec=%d kc=%d", p->nt, p->vpt, p->vec, kc);
  const int wgsize = p->nt == 64 ? 256 : p->nt;
  const size_t shmem = (size_t)p->vpt * p->nt * 8 * (1 + p->ng);
  if (shmem > 65536) {
    // above the default dynamic-LDS limit: opt this kernel in once
    HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)shmem));
  }
  hipLaunchKernelGGL(fn, dim3(p->nwg), dim3(wgsize), shmem, st, a);
  LAUNCH_CHECK("column_kernel");
  return MAM_OK;
}

mam_status launch_marginals(mam_problem* p, hipStream_t st, int save_prev) {
  const Layout& L = p->lay;
  dim3 g1((unsigned)((p->R + 255) / 256), (unsigned)p->M);
  hipLaunchKernelGGL(mam::marginal_kernel, g1, dim3(256), 0, st, at<double>(p, L.partial), (int)p->R,
                     at<int32_t>(p, L.mseg), at<int32_t>(p, L.seg_idx), at<double>(p, L.pm),
                     at<double>(p, L.pm_prev), save_prev);
  LAUNCH_CHECK("marginal_kernel");
  hipLaunchKernelGGL(mam::average_kernel, dim3(p->nb), dim3(256), 0, st, at<double>(p, L.pm), (int)p->R,
                     (int)p->M, at<double>(p, L.aw), at<double>(p, L.Sd), at<double>(p, L.p),
                     at<double>(p, L.p_prev), save_prev, at<double>(p, L.d2part));
  LAUNCH_CHECK("average_kernel");
  return MAM_OK;
}

template <typename T>
mam_status launch_init(mam_problem* p, const void* theta0, hipStream_t st) {
  const Layout& L = p->lay;
  const int blocks = (int)std::min<int64_t>(8192, std::max<int64_t>(1, (p->T * p->R + 255) / 256));
  if (theta0) {
    hipLaunchKernelGGL(mam::copy_kernel<T>, dim3(blocks), dim3(256), 0, st, static_cast<T*>(p->theta), p->ld,
                       (int)p->R, static_cast<const T*>(theta0), p->T);
    LAUNCH_CHECK("copy_kernel");
  } else {
    hipLaunchKernelGGL(mam::fill_kernel<T>, dim3(blocks), dim3(256), 0, st, static_cast<T*>(p->theta), p->ld,
                       (int)p->R, static_cast<const T*>(p->q), p->T);
    LAUNCH_CHECK("fill_kernel");
  }
  hipLaunchKernelGGL(mam::fill_value_kernel, dim3((unsigned)std::min<int64_t>(4096, (p->T + 255) / 256)), dim3(256), 0,
                     st, at<double>(p, L.lam), p->T, (double)NAN);
  LAUNCH_CHECK("fill_value_kernel");
  hipLaunchKernelGGL(mam::rowsum_kernel<T>, dim3(p->nwg), dim3(256), 0, st, static_cast<const T*>(p->theta),
                     p->ld, (int)p->R, at<int64_t>(p, L.seg_j0), at<int64_t>(p, L.seg_j1),
                     at<int32_t>(p, L.wg_seg), at<double>(p, L.partial));
  LAUNCH_CHECK("rowsum_kernel");
  return launch_marginals(p, st, 0);
}

template <typename T>
mam_status launch_checks(mam_problem* p, hipStream_t st) {
  const Layout& L = p->lay;
  double* chk = at<double>(p, L.check);
  hipLaunchKernelGGL(mam::zero_kernel, dim3((unsigned)((p->M + 2 + 255) / 256)), dim3(256), 0, st, chk,
                     (int)(p->M + 2));
  LAUNCH_CHECK("zero_kernel");
  hipLaunchKernelGGL(mam::check_q_kernel<T>, dim3((unsigned)p->M), dim3(256), 0, st, static_cast<const T*>(p->q),
                     at<int64_t>(p, L.col_off), chk, (int)p->M);
  LAUNCH_CHECK("check_q_kernel");
  const int blocks = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (p->cost_ncols * p->R + 255) / 256));
  hipLaunchKernelGGL(mam::check_cost_kernel<T>, dim3(blocks), dim3(256), 0, st, static_cast<const T*>(p->cost),
                     p->cost_ld, (int)p->R, p->cost_ncols, chk + p->M + 1);
  LAUNCH_CHECK("check_cost_kernel");
  if (p->cost_mode == MAM_COST_INDEXED) {
    const int ib = (int)std::min<int64_t>(1024, (p->T + 255) / 256);
    hipLaunchKernelGGL(mam::check_index_kernel, dim3(ib), dim3(256), 0, st, p->cidx, p->T, p->cost_ncols,
                       chk + p->M + 1);
    LAUNCH_CHECK("check_index_kernel");
  }
  return MAM_OK;
}

hipEvent_t next_event(mam_problem* p) {
  if (p->ev_used == p->ev.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    p->ev.push_back(e);
  }
  return p->ev[p->ev_used++];
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int32_t mam_abi_version(void) { return 1; }

const char* mam_last_error(void) { return g_err.c_str(); }

mam_status mam_create(mam_problem** out, const mam_desc* d) {
  if (!out) return fail(MAM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!d) return fail(MAM_EINVAL, "desc is NULL");
  if (d->dtype != MAM_F32 && d->dtype != MAM_F64) return fail(MAM_EINVAL, "unknown dtype %d", d->dtype);
  if (d->cost_mode < MAM_COST_PER_COLUMN || d->cost_mode > MAM_COST_INDEXED)
    return fail(MAM_EINVAL, "unknown cost_mode %d", d->cost_mode);
  if (d->R < 1) return fail(MAM_EINVAL, "R must be >= 1 (got %lld)", (long long)d->R);
  if (d->M < 1) return fail(MAM_EINVAL, "M must be >= 1 (got %lld)", (long long)d->M);
  if (!d->S) return fail(MAM_EINVAL, "S is NULL");
  if (!(d->rho > 0.0) || !std::isfinite(d->rho)) return fail(MAM_EINVAL, "rho must be finite and > 0");
  if (!(d->gamma >= 0.0)) return fail(MAM_EINVAL, "gamma must be >= 0 (INFINITY = balanced)");
  if (d->R > 8192) return fail(MAM_EUNSUPPORTED, "R = %lld exceeds 8192", (long long)d->R);
  if (d->M > 65535) return fail(MAM_EUNSUPPORTED, "M = %lld exceeds 65535", (long long)d->M);
  const int64_t ld = d->ld ? d->ld : d->R;
  const int64_t cld = d->cost_ld ? d->cost_ld : d->R;
  if (ld < d->R) return fail(MAM_EINVAL, "ld (%lld) < R (%lld)", (long long)ld, (long long)d->R);
  if (cld < d->R) return fail(MAM_EINVAL, "cost_ld (%lld) < R (%lld)", (long long)cld, (long long)d->R);
  int64_t T = 0, smax = 0;
  for (int64_t m = 0; m < d->M; ++m) {
    if (d->S[m] < 1) return fail(MAM_EINVAL, "S[%lld] must be >= 1", (long long)m);
    T += d->S[m];
    smax = std::max(smax, d->S[m]);
  }
  if (d->cost_ncols < 1) return fail(MAM_EINVAL, "cost_ncols must be >= 1");
  if (d->cost_mode == MAM_COST_SHARED && smax > d->cost_ncols)
    return fail(MAM_EINVAL, "shared cost has %lld columns but a measure has %lld", (long long)d->cost_ncols,
                (long long)smax);
  if (d->cost_mode == MAM_COST_PER_COLUMN && d->cost_ncols < T)
    return fail(MAM_EINVAL, "per-column cost needs T = %lld columns (got %lld)", (long long)T,
                (long long)d->cost_ncols);

  mam_problem* p = new (std::nothrow) mam_problem();
  if (!p) return fail(MAM_ENOMEM, "host allocation failed");
  p->dtype = d->dtype;
  p->cost_mode = d->cost_mode;
  p->R = d->R;
  p->M = d->M;
  p->T = T;
  p->ld = ld;
  p->cost_ld = cld;
  p->cost_ncols = d->cost_ncols;
  p->rho = d->rho;
  p->gamma = d->gamma;
  p->flags = d->flags;
  p->vec = vec_width(d->dtype);  // until mam_bind checks the alignment
  p->S.assign(d->S, d->S + d->M);
  p->col_off.assign(d->M + 1, 0);
  for (int64_t m = 0; m < d->M; ++m) p->col_off[m + 1] = p->col_off[m] + d->S[m];
  p->Sd.resize(d->M);
  p->aw.resize(d->M);
  double inv_sum = 0.0;
  for (int64_t m = 0; m < d->M; ++m) {
    p->Sd[m] = (double)d->S[m];
    inv_sum += 1.0 / (double)d->S[m];
  }
  for (int64_t m = 0; m < d->M; ++m) p->aw[m] = (1.0 / (double)d->S[m]) / inv_sum;
  mam_status st = choose_shape(p);
  if (st != MAM_OK) {
    delete p;
    return st;
  }
  build_schedule(p);
  *out = p;
  return MAM_OK;
}

mam_status mam_set_schedule(mam_problem* p, const mam_schedule* s) {
  if (!p || !s) return fail(MAM_EINVAL, "NULL argument");
  if (p->ws) return fail(MAM_ESTATE, "schedule must be set before the workspace");
  const int nt0 = p->nt_req, kc0 = p->kc_req;
  p->nt_req = s->threads_per_column;
  p->kc_req = s->columns_in_flight;
  mam_status st = choose_shape(p);
  if (st != MAM_OK) {
    p->nt_req = nt0;
    p->kc_req = kc0;
    choose_shape(p);
    return st;
  }
  if (s->order < 0 || s->order > 2) return fail(MAM_EINVAL, "order must be 0, 1 or 2 (got %d)", s->order);
  p->nwg_req = s->workgroups;
  p->xcd_req = s->xcd_remap;
  p->order_req = s->order;
  build_schedule(p);
  return MAM_OK;
}

mam_status mam_get_schedule(const mam_problem* p, mam_schedule* s) {
  if (!p || !s) return fail(MAM_EINVAL, "NULL argument");
  s->threads_per_column = p->nt;
  s->values_per_thread = p->vpt;
  s->columns_in_flight = p->vec == 1 ? 1 : p->kc;
  s->workgroups = p->nwg;
  s->xcd_remap = p->xcd_remap;
  s->vector_width = p->vec;
  s->order = p->blocked ? 2 : 1;
  return MAM_OK;
}

size_t mam_workspace_bytes(const mam_problem* p) { return p ? p->lay.total : 0; }

mam_status mam_set_workspace(mam_problem* p, void* dev, size_t bytes) {
  if (!p) return fail(MAM_EINVAL, "NULL handle");
  if (!dev) return fail(MAM_ENOMEM, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(dev) % kAlign) return fail(MAM_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < p->lay.total)
    return fail(MAM_ENOMEM, "workspace has %zu bytes, needs %zu", bytes, p->lay.total);
  p->ws = static_cast<char*>(dev);
  p->ws_bytes = bytes;
  p->tables_uploaded = false;
  p->inited = false;
  return MAM_OK;
}

mam_status mam_bind(mam_problem* p, void* theta, const void* cost, const int32_t* cost_col_index, const void* q) {
  if (!p) return fail(MAM_EINVAL, "NULL handle");
  if (!theta || !cost || !q) return fail(MAM_EINVAL, "theta, cost and q must be non-NULL");
  if (p->cost_mode == MAM_COST_INDEXED && !cost_col_index)
    return fail(MAM_EINVAL, "MAM_COST_INDEXED needs cost_col_index");
  if (p->cost_mode != MAM_COST_INDEXED && cost_col_index)
    return fail(MAM_EINVAL, "cost_col_index given but cost_mode is not MAM_COST_INDEXED");
  const size_t eb = elem_bytes(p->dtype);
  if (reinterpret_cast<uintptr_t>(theta) % eb || reinterpret_cast<uintptr_t>(cost) % eb ||
      reinterpret_cast<uintptr_t>(q) % eb)
    return fail(MAM_EINVAL, "buffers must be aligned to their element size");
  p->theta = theta;
  p->cost = cost;
  p->cidx = cost_col_index;
  p->q = q;
  const int vn = vec_width(p->dtype);
  const bool aligned = reinterpret_cast<uintptr_t>(theta) % 16 == 0 && reinterpret_cast<uintptr_t>(cost) % 16 == 0 &&
                       p->ld % vn == 0 && p->cost_ld % vn == 0;
  p->vec = (aligned && p->vpt >= vn) ? vn : 1;
  p->inited = false;
  return MAM_OK;
}

mam_status mam_init(mam_problem* p, const void* theta0, void* stream) {
  if (!p) return fail(MAM_EINVAL, "NULL handle");
  if (!p->ws) return fail(MAM_ESTATE, "no workspace");
  if (!p->theta) return fail(MAM_ESTATE, "no buffers bound");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (p->cost_mode == MAM_COST_INDEXED) {
    // the column order depends on the index (sorted within each measure:
    // cost-block-major); it is read once here
    std::vector<int32_t> idx(p->T);
    HIP_TRY(hipMemcpyAsync(idx.data(), p->cidx, p->T * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int64_t j = 0; j < p->T; ++j)
      if (idx[j] < 0 || idx[j] >= p->cost_ncols)
        return fail(MAM_ENONFINITE, "cost_col_index[%lld] = %d is out of range", (long long)j, idx[j]);
    build_schedule(p, &idx);
  }
  mam_status s = upload_tables(p, st);
  if (s != MAM_OK) return s;
  s = p->dtype == MAM_F32 ? launch_checks<float>(p, st) : launch_checks<double>(p, st);
  if (s != MAM_OK) return s;
  std::vector<double> chk(p->M + 2);
  HIP_TRY(hipMemcpyAsync(chk.data(), p->ws + p->lay.check, (p->M + 2) * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (chk[p->M] != 0.0) return fail(MAM_ENONFINITE, "q holds a negative or non-finite weight");
  if (chk[p->M + 1] != 0.0) return fail(MAM_ENONFINITE, "cost holds a non-finite entry or the column index is out of range");
  if (std::isinf(p->gamma)) {
    const double tol = p->dtype == MAM_F32 ? 1e-6 : 1e-12;
    double lo = chk[0], hi = chk[0];
    for (int64_t m = 1; m < p->M; ++m) {
      lo = std::min(lo, chk[m]);
      hi = std::max(hi, chk[m]);
    }
    if (hi - lo > tol * std::max(std::fabs(hi), 1e-300))
      return fail(MAM_ENOTBALANCED, "balanced mode but masses range over [%.17g, %.17g]", lo, hi);
  }
  s = p->dtype == MAM_F32 ? launch_init<float>(p, theta0, st) : launch_init<double>(p, theta0, st);
  if (s != MAM_OK) return s;
  p->inited = true;
  p->iters_done = 0;
  p->diag_valid = false;
  return MAM_OK;
}

mam_status mam_iterate(mam_problem* p, int64_t iters, void* stream) {
  if (!p) return fail(MAM_EINVAL, "NULL handle");
  if (iters < 0) return fail(MAM_EINVAL, "iters must be >= 0");
  if (!p->inited) return fail(MAM_ESTATE, "mam_init has not run");
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (int64_t k = 0; k < iters; ++k) {
    const int diag = (p->flags & MAM_FLAG_DIAG) && k == iters - 1;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (p->timing) {
      e0 = next_event(p);
      e1 = next_event(p);
      if (!e0 || !e1) return fail(MAM_EHIP, "hipEventCreate failed");
      HIP_TRY(hipEventRecord(e0, st));
    }
    mam_status s = p->dtype == MAM_F32 ? launch_column<float>(p, st, diag) : launch_column<double>(p, st, diag);
    if (s != MAM_OK) return s;
    if (p->timing) HIP_TRY(hipEventRecord(e1, st));
    s = launch_marginals(p, st, diag);
    if (s != MAM_OK) return s;
    if (diag) p->diag_valid = true;
  }
  p->iters_done += iters;
  return MAM_OK;
}

mam_status mam_barycenter(mam_problem* p, double* p_dev, void* stream) {
  if (!p || !p_dev) return fail(MAM_EINVAL, "NULL argument");
  if (!p->inited) return fail(MAM_ESTATE, "mam_init has not run");
  HIP_TRY(hipMemcpyAsync(p_dev, p->ws + p->lay.p, p->R * 8, hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)));
  return MAM_OK;
}

mam_status mam_barycenter_host(mam_problem* p, double* p_host, void* stream) {
  if (!p || !p_host) return fail(MAM_EINVAL, "NULL argument");
  if (!p->inited) return fail(MAM_ESTATE, "mam_init has not run");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipMemcpyAsync(p_host, p->ws + p->lay.p, p->R * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return MAM_OK;
}

mam_status mam_marginals(mam_problem* p, double* pm_dev, void* stream) {
  if (!p || !pm_dev) return fail(MAM_EINVAL, "NULL argument");
  if (!p->inited) return fail(MAM_ESTATE, "mam_init has not run");
  HIP_TRY(hipMemcpyAsync(pm_dev, p->ws + p->lay.pm, p->M * p->R * 8, hipMemcpyDeviceToDevice,
                         static_cast<hipStream_t>(stream)));
  return MAM_OK;
}

mam_status mam_diagnostics(mam_problem* p, mam_diag* out, void* stream) {
  if (!p || !out) return fail(MAM_EINVAL, "NULL argument");
  if (!p->inited || !p->diag_valid) return fail(MAM_ESTATE, "no iteration ran with MAM_FLAG_DIAG");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t R = p->R, M = p->M;
  std::vector<double> pm(M * R), pmp(M * R), pv(R), pp(R), dg((size_t)p->nwg * mam::DIAG_STRIDE);
  double t = 0.0;
  const Layout& L = p->lay;
  HIP_TRY(hipMemcpyAsync(pm.data(), p->ws + L.pm, M * R * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(pmp.data(), p->ws + L.pm_prev, M * R * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(pv.data(), p->ws + L.p, R * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(pp.data(), p->ws + L.p_prev, R * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(dg.data(), p->ws + L.diag, dg.size() * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&t, p->ws + L.tval, 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  mam_diag r{};
  r.iterations = p->iters_done;
  r.t = t;
  double rounds = 0.0, active = 0.0, cols = 0.0;
  for (int w = 0; w < p->nwg; ++w) {
    const double* o = &dg[(size_t)w * mam::DIAG_STRIDE];
    r.W_hat += o[0];
    r.meas_resid = std::max(r.meas_resid, o[1]);
    r.dtheta_inf = std::max(r.dtheta_inf, o[2]);
    rounds += o[3];
    active += o[4];
    cols += o[5];
  }
  r.rounds_per_column = cols > 0 ? rounds / cols : 0.0;
  r.active_per_column = cols > 0 ? active / cols : 0.0;
  // row sums of pi_hat^(m) = p^(m),new + t (p_old - p^(m),old)
  std::vector<double> ph(M * R), phbar(R, 0.0);
  for (size_t m = 0; m < M; ++m)
    for (size_t r = 0; r < R; ++r) ph[m * R + r] = pm[m * R + r] + t * (pp[r] - pmp[m * R + r]);
  for (size_t m = 0; m < M; ++m)
    for (size_t r = 0; r < R; ++r) phbar[r] += p->aw[m] * ph[m * R + r];
  double d2 = 0.0;
  for (size_t m = 0; m < M; ++m) {
    double s = 0.0;
    for (size_t r = 0; r < R; ++r) {
      const double e = phbar[r] - ph[m * R + r];
      s += e * e;
    }
    d2 += s / p->Sd[m];
  }
  r.dist_L = std::sqrt(d2);
  double dp = 0.0, mass = 0.0;
  bool finite = true;
  for (size_t i = 0; i < R; ++i) {
    dp += (pv[i] - pp[i]) * (pv[i] - pp[i]);
    mass += pv[i];
    finite = finite && std::isfinite(pv[i]);
  }
  r.dp_norm = std::sqrt(dp);
  r.p_mass = mass;
  *out = r;
  if (!finite) return fail(MAM_ENONFINITE, "barycenter holds NaN or Inf");
  return MAM_OK;
}

mam_status mam_timing_enable(mam_problem* p, int32_t enable) {
  if (!p) return fail(MAM_EINVAL, "NULL handle");
  p->timing = enable != 0;
  p->ev_used = 0;
  return MAM_OK;
}

mam_status mam_timing_read(mam_problem* p, double* total_ms, int64_t* launches) {
  if (!p || !total_ms || !launches) return fail(MAM_EINVAL, "NULL argument");
  double tot = 0.0;
  for (size_t i = 0; i + 1 < p->ev_used; i += 2) {
    HIP_TRY(hipEventSynchronize(p->ev[i + 1]));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, p->ev[i], p->ev[i + 1]));
    tot += ms;
  }
  *total_ms = tot;
  *launches = (int64_t)(p->ev_used / 2);
  p->ev_used = 0;
  return MAM_OK;
}

void mam_destroy(mam_problem* p) {
  if (!p) return;
  for (hipEvent_t e : p->ev) hipEventDestroy(e);
  delete p;
}

mam_status mam_cost_sq_euclid(const double* xi, int64_t R, const double* zeta, int64_t S, int32_t dim,
                              int32_t normalize_max, void* out, int64_t out_ld, int32_t dtype, double* scratch,
                              void* stream) {
  if (!xi || !zeta || !out) return fail(MAM_EINVAL, "NULL buffer");
  if (R < 1 || S < 1 || dim < 1) return fail(MAM_EINVAL, "R, S and dim must be >= 1");
  if (R > INT32_MAX) return fail(MAM_EUNSUPPORTED, "R too large");
  if (out_ld < R) return fail(MAM_EINVAL, "out_ld < R");
  if (dtype != MAM_F32 && dtype != MAM_F64) return fail(MAM_EINVAL, "unknown dtype");
  if (normalize_max && !scratch) return fail(MAM_EINVAL, "normalize_max needs an 8-byte device scratch");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int blocks = (int)std::min<int64_t>(8192, std::max<int64_t>(1, (R * S + 255) / 256));
  if (normalize_max) {
    hipLaunchKernelGGL(mam::zero_kernel, dim3(1), dim3(64), 0, st, scratch, 1);
    LAUNCH_CHECK("zero_kernel");
    hipLaunchKernelGGL(mam::sqdist_kernel, dim3(blocks), dim3(256), 0, st, xi, (int)R, zeta, S, dim, scratch, 1);
    LAUNCH_CHECK("sqdist_kernel");
  }
  if (dtype == MAM_F32)
    hipLaunchKernelGGL(mam::cost_write_kernel<float>, dim3(blocks), dim3(256), 0, st, xi, (int)R, zeta, S, dim,
                       scratch, normalize_max, static_cast<float*>(out), out_ld);
  else
    hipLaunchKernelGGL(mam::cost_write_kernel<double>, dim3(blocks), dim3(256), 0, st, xi, (int)R, zeta, S, dim,
                       scratch, normalize_max, static_cast<double*>(out), out_ld);
  LAUNCH_CHECK("cost_write_kernel");
  return MAM_OK;
}

}  // extern "C"

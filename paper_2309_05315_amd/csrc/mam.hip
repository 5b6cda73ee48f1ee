// Host side of the MAM library: C ABI, validation, column schedules,
// workspace layout, kernel launches and graph capture.  See mam.h for the
// contract, mam_kernels.hpp and mam_aux_kernels.hpp for the device code.
//
// Internally every handle is a Plan of one or more independent problems.  A
// single problem (mam_create) is a plan of one; a batch (mam_batch_create)
// is a plan of many.  Problems are grouped by column shape (threads per
// column, values per thread); one iteration of the whole plan is one
// column-kernel launch per group, then one marginal and one averaging
// launch for all problems.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mam.h"
#include "mam_aux_kernels.hpp"
#include "mam_dispatch.hpp"
#include "mam_support.hpp"

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

#define TRY(expr)                      \
  do {                                 \
    mam_status s_ = (expr);            \
    if (s_ != MAM_OK) return s_;       \
  } while (0)

constexpr size_t kAlign = 256;
constexpr int64_t kMaxLds = 160 * 1024;  // LDS per compute unit on gfx950
constexpr int64_t kShortMaxR = 8192;      // longest column one workgroup holds in registers
constexpr int64_t kLongMaxR = 1 << 28;    // row indices of the long-column path are int32
constexpr int kDefaultTeam = 1;            // workgroups per team sweep (team_size 0)
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int vec_width(int dtype) { return dtype == MAM_F32 ? 4 : 2; }
size_t elem_bytes(int dtype) { return dtype == MAM_F32 ? 4 : 8; }

int pow2_ceil(int64_t x) {
  int v = 1;
  while (v < x) v <<= 1;
  return v;
}

// A contiguous column range of one measure.
struct Task {
  int m;
  int64_t lo, hi;
};

struct Prob {
  int64_t R = 0, M = 0, T = 0, ld = 0, cost_ld = 0, cost_ncols = 0;
  int cost_mode = MAM_COST_PER_COLUMN;
  double rho = 1.0, gamma = INFINITY;
  uint32_t flags = 0;
  std::vector<int64_t> S, col_off;
  std::vector<double> Sd, aw;
  // bound buffers
  void* theta = nullptr;
  const void* cost = nullptr;
  const int32_t* cidx = nullptr;
  const void* q = nullptr;
  bool aligned = true;
  std::vector<int32_t> idx;  // host copy of an indexed cost's column index
  // grid cost: dimension (0 = not set), points per axis, origin, spacing
  int gdim = 0;
  int64_t gn[2] = {1, 1};
  double go[2] = {0.0, 0.0}, gh[2] = {0.0, 0.0};
  // workspace offsets of the problem's own region
  size_t o_pm = 0, o_pm_prev = 0, o_p = 0, o_p_prev = 0, o_d2 = 0, o_t = 0, o_lam = 0, o_check = 0;
  size_t o_coloff = 0, o_Sd = 0, o_aw = 0;
  size_t o_acc = 0, o_fx = 0;  // short columns: fixed-point row sums of pi_hat; scales 2^E_m, then 2^-E_m
  int nb = 0;
  int group = 0;
  int mbase = 0;
};

struct Group {
  int nt = 64, vpt = 1, ng = 4, kc = 1, vec = 1;
  int nt_req = 0, kc_req = 0, nwg_req = 0, xcd_req = 0, order_req = 0, stream_req = 0, team_req = 0;
  int team = 1;  // workgroups sweeping one share of the columns together
  int nwg = 1, wg_base = 0, xcd_remap = 0, stream = 0;
  int nwg_auto = 0;  // workgroups the device holds at once (set at init), 0 = unknown
  int64_t Rmax = 0;
  bool blocked = false;
  std::vector<int> probs;
};

struct Layout {
  size_t partial = 0, diag = 0, seg_p = 0, seg_m = 0, seg_j0 = 0, seg_j1 = 0, seg_poff = 0, seg_idx = 0, seg_st = 0;
  size_t wg_seg = 0, mseg = 0, probdev = 0, probaux = 0, mtasks = 0, atasks = 0;
  size_t stop = 0, stop_part = 0;  // stopping-test state and row-block partials
  size_t total = 0;
};

// Reverse-mode state of a single-problem plan (mam_record / mam_backward).
// columns one wave of the reverse column kernel takes at a time
constexpr int kAdjCols = 2;

struct Adjoint {
  bool valid = false;
  int64_t K = 0, C = 1, nw = 0;  // iterations, window length, windows
  int64_t resident = -1;         // window whose masks the ring holds
  char* ws = nullptr;
  size_t bytes = 0;
  int64_t mld = 0;               // mask bytes per column
  size_t ckpt_bytes = 0;         // one checkpoint of theta
  size_t o_mask = 0, o_ckpt = 0, o_ckpt_pm = 0, o_U = 0, o_cacc = 0, o_qacc = 0, o_V = 0, o_wold = 0;
  size_t o_wacc = 0, o_mx = 0, o_cptr = 0, o_clist = 0, total = 0;
  // unbalanced problems: p, p^(m) and the d^2 partials of every recorded
  // iteration (same slot ring as the masks), and the two-pass buffers
  bool unbal = false;
  size_t o_pm_rec = 0, o_p_rec = 0, o_d2_rec = 0, o_bbar = 0, o_tpart = 0;
};

// Randomized variant: a partition of a single problem's measures into
// bundles, each with its own segment schedule (tables in a caller-provided
// bundle workspace; partials in the plan's buffer).
struct BundleSched {
  int nwg = 0;
  size_t nseg = 0;
  size_t o_seg_p = 0, o_seg_m = 0, o_seg_j0 = 0, o_seg_j1 = 0, o_seg_st = 0, o_wg_seg = 0, o_mtasks = 0;
  size_t nmtasks = 0;
};

struct Bundles {
  int nb = 0;
  char* ws = nullptr;
  std::vector<BundleSched> b;
};

// Long-column path (single problems with R beyond kShortMaxR, or forced by
// the schedule): work items (row tile, measure, column range) split evenly
// over the workgroups; per (column, wave sub-tile) a header (maximum of w,
// candidate count) and 'cap' candidate slots.
struct LongPlan {
  bool on = false, sets = false;
  int vpt = 16, rows = 4096, nrb = 0, cap = 0, vec = 1;
  int nwg = 1, nwg_req = 0, nwg_auto = 0, rows_req = 0, cap_req = 0;
  std::vector<int32_t> it_rb, it_m, wg_it;
  std::vector<int64_t> it_j0, it_j1, it_poff;
  size_t items_cap = 0;
  size_t o_it_rb = 0, o_it_m = 0, o_it_j0 = 0, o_it_j1 = 0, o_it_poff = 0, o_wg_it = 0;
  size_t o_hmax = 0, o_hcnt = 0, o_crow = 0, o_cw = 0;
  // sparse store (MAM_FLAG_SPARSE_STORE): patch counts, rows and values per
  // (column, sub-tile), the two halves of the common values, the parity
  bool sparse = false;
  size_t o_pcnt = 0, o_prow = 0, o_pval = 0, o_nbv = 0, o_spar = 0;
  // diagnostics: 4 doubles per column (threshold kernel), DIAG_STRIDE per
  // write workgroup
  size_t o_ldiag = 0, o_wdiag = 0;
};

struct Plan {
  int dtype = MAM_F64;
  bool batch = false;
  std::vector<Prob> P;
  std::vector<Group> G;
  // schedule tables
  std::vector<int32_t> seg_p, seg_m, wg_seg, mseg, seg_idx, seg_st;
  std::vector<int64_t> mpoff;  // partial offsets of every measure's segments, in schedule order
  std::vector<int64_t> seg_j0, seg_j1, seg_poff;
  std::vector<mam::MargTask> mtasks;
  std::vector<mam::AvgTask> atasks;
  size_t nseg_cap = 0, partial_cap = 0;
  int nwg_total = 0;
  Layout lay;
  // state
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool tables_uploaded = false;
  bool inited = false;
  bool default_start = false;
  int64_t iters_done = 0;
  Adjoint adj;
  Bundles bund;
  LongPlan lg;
  bool diag_valid = false;
  // graph of a fixed number of iterations
  int64_t graph_iters = 0;
  hipGraphExec_t gexec = nullptr;
  hipStream_t capture_stream = nullptr;
  // timing
  bool timing = false;
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
  // several shape groups run concurrently: one stream per group (default
  // priority), forked from and joined back into the caller's stream
  std::vector<hipStream_t> gstream;
  std::vector<hipEvent_t> gjoin;
  hipEvent_t gfork = nullptr;
  bool capturing = false;  // forks are worth their event calls only inside a graph
  // runs with an on-device stopping test: the gate flag every launch of such
  // a run checks (null otherwise), a host-visible copy of it, the graph of
  // one check period and the events that bound the periods in flight
  const int32_t* gate = nullptr;
  int32_t* host_flag = nullptr;
  hipGraphExec_t uexec = nullptr;
  int utest = -1;
  int64_t uevery = 0;
  std::vector<hipEvent_t> uev;

  ~Plan() {
    for (hipEvent_t e : uev) hipEventDestroy(e);
    if (uexec) hipGraphExecDestroy(uexec);
    if (host_flag) hipHostFree(host_flag);
    for (hipEvent_t e : ev) hipEventDestroy(e);
    for (hipEvent_t e : gjoin) hipEventDestroy(e);
    if (gfork) hipEventDestroy(gfork);
    for (hipStream_t s : gstream) hipStreamDestroy(s);
    if (gexec) hipGraphExecDestroy(gexec);
    if (capture_stream) hipStreamDestroy(capture_stream);
  }
};

template <typename U>
U* at(Plan* pl, size_t off) { return reinterpret_cast<U*>(pl->ws + off); }

// ---------------------------------------------------------------------------
// problem description and shapes
// ---------------------------------------------------------------------------
mam_status read_desc(const mam_desc* d, int index, Prob* out) {
  if (!d) return fail(MAM_EINVAL, "desc %d is NULL", index);
  if (d->dtype != MAM_F32 && d->dtype != MAM_F64) return fail(MAM_EINVAL, "unknown dtype %d", d->dtype);
  if (d->cost_mode < MAM_COST_PER_COLUMN || d->cost_mode > MAM_COST_GRID)
    return fail(MAM_EINVAL, "unknown cost_mode %d", d->cost_mode);
  if (d->R < 1) return fail(MAM_EINVAL, "R must be >= 1 (got %lld)", (long long)d->R);
  if (d->M < 1) return fail(MAM_EINVAL, "M must be >= 1 (got %lld)", (long long)d->M);
  if (!d->S) return fail(MAM_EINVAL, "S is NULL");
  if (!(d->rho > 0.0) || !std::isfinite(d->rho)) return fail(MAM_EINVAL, "rho must be finite and > 0");
  if (!(d->gamma >= 0.0)) return fail(MAM_EINVAL, "gamma must be >= 0 (INFINITY = balanced)");
  if (d->R > kLongMaxR) return fail(MAM_EUNSUPPORTED, "R = %lld exceeds %lld", (long long)d->R, (long long)kLongMaxR);
  if (d->M > 65535) return fail(MAM_EUNSUPPORTED, "M = %lld exceeds 65535", (long long)d->M);
  const int64_t ld = d->ld ? d->ld : d->R;
  // a grid cost is formed in the kernels: its buffer holds points, no stride
  const int64_t cld = (d->cost_ld && d->cost_mode != MAM_COST_GRID) ? d->cost_ld : d->R;
  if (ld < d->R) return fail(MAM_EINVAL, "ld (%lld) < R (%lld)", (long long)ld, (long long)d->R);
  if (cld < d->R) return fail(MAM_EINVAL, "cost_ld (%lld) < R (%lld)", (long long)cld, (long long)d->R);
  int64_t T = 0, smax = 0;
  for (int64_t m = 0; m < d->M; ++m) {
    if (d->S[m] < 1) return fail(MAM_EINVAL, "S[%lld] must be >= 1", (long long)m);
    T += d->S[m];
    smax = std::max(smax, d->S[m]);
  }
  if (d->cost_ncols < 1) return fail(MAM_EINVAL, "cost_ncols must be >= 1");
  if ((d->cost_mode == MAM_COST_SHARED || d->cost_mode == MAM_COST_GRID) && smax > d->cost_ncols)
    return fail(MAM_EINVAL, "shared cost has %lld columns but a measure has %lld", (long long)d->cost_ncols,
                (long long)smax);
  if (d->cost_mode == MAM_COST_PER_COLUMN && d->cost_ncols < T)
    return fail(MAM_EINVAL, "per-column cost needs T = %lld columns (got %lld)", (long long)T,
                (long long)d->cost_ncols);
  out->R = d->R;
  out->M = d->M;
  out->T = T;
  out->ld = ld;
  out->cost_ld = cld;
  out->cost_ncols = d->cost_ncols;
  out->cost_mode = d->cost_mode;
  out->rho = d->rho;
  out->gamma = d->gamma;
  out->flags = d->flags;
  out->S.assign(d->S, d->S + d->M);
  out->col_off.assign(d->M + 1, 0);
  for (int64_t m = 0; m < d->M; ++m) out->col_off[m + 1] = out->col_off[m] + d->S[m];
  out->Sd.resize(d->M);
  out->aw.resize(d->M);
  double inv_sum = 0.0;
  for (int64_t m = 0; m < d->M; ++m) {
    out->Sd[m] = (double)d->S[m];
    inv_sum += 1.0 / (double)d->S[m];
  }
  for (int64_t m = 0; m < d->M; ++m) out->aw[m] = (1.0 / (double)d->S[m]) / inv_sum;
  out->nb = (int)((d->R + 255) / 256);
  return MAM_OK;
}

// Column groups per workgroup of 256 threads for nt threads per column:
// sub-wave groups (16 or 32 lanes) and single waves share a workgroup.
int groups_per_wg(int nt) { return nt <= 64 ? 256 / nt : 1; }

// Threads per column and values per thread for R rows.  Default: the fewest
// threads that keep a thread at 16 (float) or 8 (double) values, so a column
// group fits twice per compute unit (registers and LDS); one wave per
// column whenever that suffices (no barriers in the threshold rounds).
// 16 or 32 threads per column (several columns per wave) only on request.
mam_status shape_for(int dtype, int64_t R, int nt_req, int* nt_out, int* vpt_out) {
  int nt = nt_req;
  if (nt == 0) {
    const int64_t target = dtype == MAM_F32 ? 16 : 8;
    nt = 64;
    while (nt < 1024 && (int64_t)nt * target < R) nt *= 2;
  }
  if (nt != 16 && nt != 32 && nt != 64 && nt != 128 && nt != 256 && nt != 512 && nt != 1024)
    return fail(MAM_EINVAL, "threads_per_column must be 16, 32, 64, 128, 256, 512 or 1024 (got %d)", nt);
  int vpt = pow2_ceil((R + nt - 1) / nt);
  if (nt >= 128 && vpt < 4) vpt = 4;  // multi-wave groups hold at least 4 values per thread
  if (vpt > 16)
    return fail(MAM_EUNSUPPORTED, "R = %lld needs more than 16 values per thread at %d threads per column",
                (long long)R, nt);
  if ((int64_t)vpt * nt * 8 * (1 + groups_per_wg(nt)) > kMaxLds)
    return fail(MAM_EUNSUPPORTED, "R = %lld at %d threads per column needs more than 160 KiB of LDS",
                (long long)R, nt);
  *nt_out = nt;
  *vpt_out = vpt;
  return MAM_OK;
}

mam_status group_shape(Plan* pl, Group& g) {
  int nt = 0, vpt = 0;
  TRY(shape_for(pl->dtype, g.Rmax, g.nt_req, &nt, &vpt));
  const int kc = g.kc_req ? g.kc_req : 1;
  if (kc != 1 && kc != 2 && kc != 4) return fail(MAM_EINVAL, "columns_in_flight must be 1, 2 or 4 (got %d)", kc);
  g.nt = nt;
  g.vpt = vpt;
  g.kc = kc;
  if (nt < 64 && kc != 1)
    return fail(MAM_EINVAL, "16 or 32 threads per column take one column in flight (got %d)", kc);
  g.ng = groups_per_wg(nt);
  g.vec = vec_width(pl->dtype);  // until binding checks the alignment
  return MAM_OK;
}

// ---------------------------------------------------------------------------
// column order and segments
//
// Columns sharing a cost column (the same s under a shared cost, the same
// index under an indexed cost) should be streamed close together in time so
// the cost column is fetched into L2 once.  A problem's column order is a
// list of tasks: cost-block-major when the cost layout allows it (block = B
// cost columns, about 2 MiB), else measure-major.  A group's workgroups
// take equal shares of its problems' concatenated orders; every piece of a
// task a workgroup owns is one segment (one row-sum partial).
// ---------------------------------------------------------------------------
int64_t cost_block(int dtype, const Prob& p) {
  const int64_t col_bytes = p.R * (int64_t)elem_bytes(dtype);
  int64_t b = 1;
  while (b * 2 * col_bytes <= (int64_t)(2 << 20) && b < 4096) b *= 2;
  return b;
}

int64_t task_bound(int dtype, const Prob& p) {
  if (p.cost_mode == MAM_COST_PER_COLUMN) return p.M;
  const int64_t B = cost_block(dtype, p);
  return std::max<int64_t>(p.M, ((p.cost_ncols + B - 1) / B) * p.M);
}

std::vector<Task> task_order(int dtype, const Prob& p, int order_req, bool* is_blocked) {
  std::vector<Task> tasks;
  // automatic: cost-block-major for a shared cost, measure-major for an
  // indexed cost (the faster of the two on the measured workloads)
  const int order = order_req ? order_req : (p.cost_mode == MAM_COST_SHARED ? 2 : 1);
  bool blocked = p.cost_mode == MAM_COST_SHARED && order == 2;
  if (p.cost_mode == MAM_COST_INDEXED && !p.idx.empty() && order == 2) {
    blocked = true;
    for (int64_t m = 0; m < p.M && blocked; ++m)
      for (int64_t j = p.col_off[m] + 1; j < p.col_off[m + 1]; ++j)
        if (p.idx[j] < p.idx[j - 1]) {
          blocked = false;
          break;
        }
  }
  *is_blocked = blocked;
  if (!blocked) {
    for (int64_t m = 0; m < p.M; ++m) tasks.push_back({(int)m, p.col_off[m], p.col_off[m + 1]});
    return tasks;
  }
  const int64_t B = cost_block(dtype, p);
  const int64_t nkb = (p.cost_ncols + B - 1) / B;
  for (int64_t kb = 0; kb < nkb; ++kb) {
    for (int64_t m = 0; m < p.M; ++m) {
      const int64_t o = p.col_off[m], S = p.S[m];
      int64_t lo, hi;
      if (p.cost_mode == MAM_COST_SHARED) {
        lo = o + std::min(S, kb * B);
        hi = o + std::min(S, (kb + 1) * B);
      } else {
        const int32_t* b = p.idx.data() + o;
        lo = o + (std::lower_bound(b, b + S, (int32_t)std::min<int64_t>(kb * B, INT32_MAX)) - b);
        hi = o + (std::lower_bound(b, b + S, (int32_t)std::min<int64_t>((kb + 1) * B, INT32_MAX)) - b);
      }
      if (hi > lo) tasks.push_back({(int)m, lo, hi});
    }
  }
  return tasks;
}

// Default workgroup count: as many as the device holds at once for this
// kernel (one wave of workgroups, equal shares, no tail), at most 1024.
int default_nwg(int64_t T, int ng, int req, int resident) {
  int nwg = req;
  if (nwg <= 0) {
    const int64_t cap = resident > 0 ? std::min(resident, 1024) : 1024;
    const int64_t cpw = std::max<int64_t>(1, (T + ng * cap - 1) / (ng * cap));
    nwg = (int)std::min<int64_t>(cap, (T + ng * cpw - 1) / (ng * cpw));
  }
  return (int)std::max<int64_t>(1, std::min<int64_t>(nwg, T));
}

// Columns a column group takes at a time: its columns in flight when
// several groups share a workgroup (so they share a segment's columns to
// within one step), a fixed block of kOneGroupBlock when the workgroup is
// one group.
int group_block(const Group& g) { return g.ng == 1 ? mam::kOneGroupBlock : g.kc; }

// Build the tables of every group.  The workspace capacity depends only on
// the problem sizes and workgroup counts (not on an indexed cost's index),
// so rebuilding after the index is known never grows it.
void build_long_schedule(Plan* pl);

// Team sweeps.  A group's workgroups form teams of 'team' workgroups; each
// team takes an equal contiguous share of the group's column order and
// deals it out in blocks of NG*kc columns, round robin over its workgroups,
// so the columns in flight at any time lie close together in memory (a
// sweep, which HBM serves faster than as many independent streams as there
// are workgroups).  Every piece of a task a workgroup takes blocks from is
// one segment, walked with a stride of team*NG*kc columns.  The marginals
// are accumulated per entry, so the number of segments costs nothing but
// one reload of b^(m) each.
void build_schedule(Plan* pl) {
  if (pl->lg.on) {
    build_long_schedule(pl);
    return;
  }
  pl->seg_p.clear();
  pl->seg_m.clear();
  pl->seg_j0.clear();
  pl->seg_j1.clear();
  pl->seg_poff.clear();
  pl->seg_st.clear();
  pl->wg_seg.clear();
  size_t cap_segs = 0;
  int wg_base = 0;
  for (Group& g : pl->G) {
    int64_t Tg = 0;
    for (int pi : g.probs) Tg += pl->P[pi].T;
    g.nwg = default_nwg(Tg, g.ng, g.nwg_req, g.nwg_auto);
    g.wg_base = wg_base;
    // concatenated task order of the group's problems
    std::vector<std::pair<int, Task>> tasks;
    bool all_blocked = true;
    size_t tasks_cap = 0;
    for (int pi : g.probs) {
      bool blocked = false;
      for (const Task& t : task_order(pl->dtype, pl->P[pi], g.order_req, &blocked)) tasks.push_back({pi, t});
      all_blocked = all_blocked && blocked;
      tasks_cap += (size_t)task_bound(pl->dtype, pl->P[pi]);
    }
    g.blocked = all_blocked;
    g.xcd_remap = g.xcd_req > 0 ? 1 : (g.xcd_req < 0 ? 0 : (g.blocked ? 1 : 0));
    // stream the plans past the caches when they cannot stay in the 256 MB
    // Infinity Cache from one iteration to the next anyway
    size_t plan_bytes = 0;
    for (int pi : g.probs) plan_bytes += (size_t)pl->P[pi].ld * (size_t)pl->P[pi].T * elem_bytes(pl->dtype);
    g.stream = g.stream_req > 0 ? 1 : (g.stream_req < 0 ? 0 : (plan_bytes > ((size_t)256 << 20) ? 1 : 0));
    g.team = std::max(1, std::min(g.nwg, g.team_req > 0 ? g.team_req : kDefaultTeam));
    const int nteams = (g.nwg + g.team - 1) / g.team;
    const int64_t blk = (int64_t)g.ng * group_block(g);  // a block for each of the ng groups
    // segments: at most one per block of a piece, so at most Tg/blk plus
    // the number of pieces (tasks split at the team shares, of which there
    // are at most 1024, the largest workgroup count): a bound that holds for
    // every later rebuild with another workgroup count
    cap_segs += (size_t)(Tg / blk) + tasks_cap + 1025;
    std::vector<std::vector<int64_t>> own(g.nwg);  // indices into the staged segments
    std::vector<int32_t> sp, sm, sst;
    std::vector<int64_t> sj0, sj1;
    size_t ti = 0;
    int64_t tpos = 0;
    for (int t = 0; t < nteams; ++t) {
      const int w0 = t * g.team, kt = std::min(g.team, g.nwg - w0);
      int64_t need = Tg * (t + 1) / nteams - Tg * t / nteams;
      int64_t dealt = 0;  // blocks of this share dealt so far
      while (need > 0 && ti < tasks.size()) {
        const int pi = tasks[ti].first;
        const Task& tk = tasks[ti].second;
        const int64_t take = std::min(need, tk.hi - tk.lo - tpos);
        const int64_t lo = tk.lo + tpos, hi = lo + take;
        const int64_t nblk = (take + blk - 1) / blk;
        for (int k = 0; k < kt; ++k) {
          const int64_t b0 = ((k - dealt) % kt + kt) % kt;  // this workgroup's first block of the piece
          if (b0 >= nblk) continue;
          own[w0 + k].push_back((int64_t)sp.size());
          sp.push_back(pi);
          sm.push_back(tk.m);
          sj0.push_back(lo + b0 * blk);
          sj1.push_back(hi);
          sst.push_back((int32_t)(kt * blk));
        }
        dealt += nblk;
        need -= take;
        tpos += take;
        if (tpos == tk.hi - tk.lo) {
          ++ti;
          tpos = 0;
        }
      }
    }
    for (int w = 0; w < g.nwg; ++w) {
      pl->wg_seg.push_back((int32_t)pl->seg_p.size());
      for (int64_t k : own[w]) {
        pl->seg_p.push_back(sp[k]);
        pl->seg_m.push_back(sm[k]);
        pl->seg_j0.push_back(sj0[k]);
        pl->seg_j1.push_back(sj1[k]);
        pl->seg_st.push_back(sst[k]);
      }
    }
    wg_base += g.nwg;
  }
  pl->wg_seg.push_back((int32_t)pl->seg_p.size());
  pl->nwg_total = wg_base;
  int nmeas = 0;
  for (Prob& p : pl->P) {
    p.mbase = nmeas;
    nmeas += (int)p.M;
  }
  // no segment partials: the marginals are accumulated per entry
  pl->mseg.assign(nmeas + 1, 0);
  pl->seg_idx.clear();
  pl->mpoff.clear();
  pl->mtasks.clear();
  pl->atasks.clear();
  for (size_t pi = 0; pi < pl->P.size(); ++pi) {
    const Prob& p = pl->P[pi];
    for (int64_t m = 0; m < p.M; ++m)
      for (int64_t r0 = 0; r0 < p.R; r0 += 256)
        pl->mtasks.push_back({(int32_t)pi, (int32_t)m, (int32_t)r0, (int32_t)m});
    for (int rb = 0; rb < p.nb; ++rb) pl->atasks.push_back({(int32_t)pi, rb});
  }
  if (!pl->ws) {
    pl->nseg_cap = std::max<size_t>(cap_segs, pl->seg_p.size());
    pl->partial_cap = 0;
  }
  pl->tables_uploaded = false;
}

// Long-column schedule.  Units (row tile rb, column j) in the order
// rb-major, then measure, then column are split into equal contiguous
// shares, one per workgroup; each piece inside one (rb, measure) is an item
// with its own RB-row partial.  The marginal kernel sums, for a row of tile
// rb, the items of (measure, rb): list index m*nrb + rb.
//
// Measure sets: with one cost shared by M measures of equal size, plan
// column s of every measure reads cost column s.  The M workgroups of a set
// then take the same (rb, s) units, one measure each, and sit on one XCD
// (the hardware deals workgroup b to XCD b mod 8), so a cost tile fetched
// by one of them is read by the others from that XCD's L2.
void build_long_schedule(Plan* pl) {
  LongPlan& lg = pl->lg;
  const Prob& p = pl->P[0];
  const int vn = vec_width(pl->dtype);
  lg.vpt = lg.rows_req ? lg.rows_req / 256 : (pl->dtype == MAM_F32 ? 16 : 8);
  lg.rows = 256 * lg.vpt;
  lg.nrb = (int)((p.R + lg.rows - 1) / lg.rows);
  lg.cap = lg.cap_req ? lg.cap_req : 64;
  if (!p.theta) lg.vec = vn;  // until binding checks the alignment
  const int64_t units = (int64_t)lg.nrb * p.T;
  const int64_t cap_wg = lg.nwg_auto > 0 ? std::min(lg.nwg_auto, 1024) : 1024;
  lg.nwg = (int)std::max<int64_t>(1, std::min<int64_t>(lg.nwg_req > 0 ? lg.nwg_req : cap_wg, units));
  lg.it_rb.clear();
  lg.it_m.clear();
  lg.it_j0.clear();
  lg.it_j1.clear();
  lg.it_poff.clear();
  lg.wg_it.clear();
  bool equal_S = true;
  for (int64_t k = 1; k < p.M; ++k) equal_S = equal_S && p.S[k] == p.S[0];
  const int64_t sets_per_xcd = cap_wg / 8 / std::max<int64_t>(p.M, 1);
  lg.sets = p.cost_mode == MAM_COST_SHARED && equal_S && p.M >= 2 && lg.nwg_req == 0 && sets_per_xcd >= 1 &&
            (int64_t)lg.nrb * p.S[0] >= 8 * sets_per_xcd;
  if (lg.sets) {
    const int64_t G = 8 * sets_per_xcd, M = p.M, S = p.S[0], su = (int64_t)lg.nrb * S;
    lg.nwg = (int)(G * M);
    for (int b = 0; b < lg.nwg; ++b) {
      // workgroup b: XCD b % 8, slot b / 8 = (set within the XCD) * M + measure
      const int64_t x = b % 8, k = b / 8, mm = k % M, g = (k / M) * 8 + x;
      lg.wg_it.push_back((int32_t)lg.it_rb.size());
      int64_t u = su * g / G;
      const int64_t u1 = su * (g + 1) / G;
      while (u < u1) {
        const int64_t rbu = u / S, s0 = u % S, take = std::min(u1 - u, S - s0);
        lg.it_rb.push_back((int32_t)rbu);
        lg.it_m.push_back((int32_t)mm);
        lg.it_j0.push_back(p.col_off[mm] + s0);
        lg.it_j1.push_back(p.col_off[mm] + s0 + take);
        lg.it_poff.push_back((int64_t)lg.it_rb.size() - 1);
        u += take;
      }
    }
  }
  int rb = lg.sets ? lg.nrb : 0, m = 0;
  int64_t pos = 0;  // columns of (rb, m) already given out
  for (int w = 0; w < lg.nwg && !lg.sets; ++w) {
    int64_t need = units * (w + 1) / lg.nwg - units * w / lg.nwg;
    lg.wg_it.push_back((int32_t)lg.it_rb.size());
    while (need > 0 && rb < lg.nrb) {
      const int64_t take = std::min(need, p.S[m] - pos);
      lg.it_rb.push_back(rb);
      lg.it_m.push_back(m);
      lg.it_j0.push_back(p.col_off[m] + pos);
      lg.it_j1.push_back(p.col_off[m] + pos + take);
      lg.it_poff.push_back((int64_t)lg.it_rb.size() - 1);  // scaled below
      need -= take;
      pos += take;
      if (pos == p.S[m]) {
        pos = 0;
        if (++m == p.M) {
          m = 0;
          ++rb;
        }
      }
    }
  }
  lg.wg_it.push_back((int32_t)lg.it_rb.size());
  for (auto& o : lg.it_poff) o *= lg.rows;
  const int nl = (int)p.M * lg.nrb;
  pl->mseg.assign(nl + 1, 0);
  for (size_t i = 0; i < lg.it_rb.size(); ++i) ++pl->mseg[lg.it_m[i] * lg.nrb + lg.it_rb[i] + 1];
  for (int k = 0; k < nl; ++k) pl->mseg[k + 1] += pl->mseg[k];
  pl->mpoff.assign(lg.it_rb.size(), 0);
  {
    std::vector<int32_t> fill(pl->mseg.begin(), pl->mseg.end() - 1);
    for (size_t i = 0; i < lg.it_rb.size(); ++i)
      pl->mpoff[fill[lg.it_m[i] * lg.nrb + lg.it_rb[i]]++] = lg.it_poff[i] - (int64_t)lg.it_rb[i] * lg.rows;
  }
  pl->mtasks.clear();
  pl->atasks.clear();
  for (int64_t mm = 0; mm < p.M; ++mm)
    for (int64_t r0 = 0; r0 < p.R; r0 += 256)
      pl->mtasks.push_back({0, (int32_t)mm, (int32_t)r0, (int32_t)(mm * lg.nrb + r0 / lg.rows)});
  for (int b = 0; b < p.nb; ++b) pl->atasks.push_back({0, b});
  pl->seg_p.clear();
  pl->seg_m.clear();
  pl->seg_j0.clear();
  pl->seg_j1.clear();
  pl->seg_poff.clear();
  pl->seg_st.clear();
  pl->wg_seg.assign(2, 0);
  pl->nwg_total = 1;
  if (!pl->ws) {
    lg.items_cap = (size_t)lg.nrb * (size_t)p.M + (size_t)std::max(lg.nwg, 1024);
    pl->nseg_cap = 1;
    pl->partial_cap = lg.items_cap * (size_t)lg.rows;
  }
  pl->tables_uploaded = false;
}

void build_layout(Plan* pl) {
  Layout& L = pl->lay;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t a = o;
    o = align_up(o + std::max<size_t>(bytes, 1));
    return a;
  };
  const size_t ns = pl->nseg_cap;
  L.partial = take(pl->partial_cap * 8);
  L.diag = take((size_t)pl->nwg_total * mam::DIAG_STRIDE * 8);
  L.seg_p = take(ns * 4);
  L.seg_m = take(ns * 4);
  L.seg_j0 = take(ns * 8);
  L.seg_j1 = take(ns * 8);
  L.seg_poff = take(ns * 8);
  L.seg_idx = take(ns * 8);  // holds mpoff
  L.seg_st = take(ns * 4);
  L.wg_seg = take((size_t)(pl->nwg_total + 1) * 4);
  size_t nmeas = 0;
  for (const Prob& p : pl->P) nmeas += (size_t)p.M;
  if (pl->lg.on) {
    nmeas *= (size_t)pl->lg.nrb;  // one partial list per (measure, row tile)
    L.seg_idx = take(pl->lg.items_cap * 8);
  }
  L.mseg = take((nmeas + 1) * 4);
  L.probdev = take(pl->P.size() * std::max(sizeof(mam::ProbDev<float>), sizeof(mam::ProbDev<double>)));
  L.probaux = take(pl->P.size() * sizeof(mam::ProbAux));
  L.mtasks = take(pl->mtasks.size() * sizeof(mam::MargTask));
  L.atasks = take(pl->atasks.size() * sizeof(mam::AvgTask));
  L.stop = take(sizeof(mam::StopState));
  L.stop_part = take((size_t)pl->P[0].nb * 8);
  if (pl->lg.on) {
    LongPlan& lg = pl->lg;
    const size_t T = (size_t)pl->P[0].T, ni = lg.items_cap;
    lg.o_it_rb = take(ni * 4);
    lg.o_it_m = take(ni * 4);
    lg.o_it_j0 = take(ni * 8);
    lg.o_it_j1 = take(ni * 8);
    lg.o_it_poff = take(ni * 8);
    lg.o_wg_it = take(((size_t)std::max(lg.nwg, 1024) + 1) * 4);
    lg.o_ldiag = take(T * 4 * 8);
    lg.o_wdiag = take((size_t)std::max(lg.nwg, 1024) * mam::DIAG_STRIDE * 8);
    const size_t nh = T * (size_t)lg.nrb * 4;  // (column, sub-tile) headers
    lg.o_hmax = take(nh * 8);
    lg.o_hcnt = take(nh * 4);
    lg.o_crow = take(nh * (size_t)lg.cap * 4);
    lg.o_cw = take(nh * (size_t)lg.cap * 8);
    lg.sparse = (pl->P[0].flags & MAM_FLAG_SPARSE_STORE) != 0;
    if (lg.sparse) {
      const size_t eb = elem_bytes(pl->dtype);
      lg.o_pcnt = take(nh * 4);
      lg.o_prow = take(nh * (size_t)lg.cap * 4);
      lg.o_pval = take(nh * (size_t)lg.cap * eb);
      lg.o_nbv = take(2 * (size_t)pl->P[0].M * (size_t)pl->P[0].R * eb);
      lg.o_spar = take(4);
    }
  }
  for (Prob& p : pl->P) {
    const size_t R = (size_t)p.R, M = (size_t)p.M;
    p.o_pm = take(M * R * 8);
    p.o_pm_prev = take(M * R * 8);
    p.o_p = take(R * 8);
    p.o_p_prev = take(R * 8);
    p.o_d2 = take((size_t)p.nb * 8);
    p.o_t = take(8);
    p.o_lam = take((size_t)p.T * 8);
    p.o_check = take((M + 2) * 8);
    p.o_coloff = take((M + 1) * 8);
    p.o_Sd = take(M * 8);
    p.o_aw = take(M * 8);
    if (!pl->lg.on) {
      p.o_acc = take(M * R * 8);
      p.o_fx = take(2 * M * 8);
    }
  }
  L.total = o;
}

// Plan with problems 'descs' and the default grouping by shape.
mam_status make_plan(Plan* pl, const mam_desc* descs, int n) {
  if (n < 1) return fail(MAM_EINVAL, "a batch needs at least one problem");
  pl->P.resize(n);
  for (int i = 0; i < n; ++i) {
    TRY(read_desc(&descs[i], i, &pl->P[i]));
    if (descs[i].dtype != descs[0].dtype) return fail(MAM_EINVAL, "all problems of a batch share one dtype");
  }
  pl->dtype = descs[0].dtype;
  for (int i = 0; i < n; ++i)
    if (pl->P[i].R > kShortMaxR && pl->batch)
      return fail(MAM_EUNSUPPORTED, "problem %d: R = %lld exceeds %lld in a batch", i, (long long)pl->P[i].R,
                  (long long)kShortMaxR);
  for (int i = 0; i < n; ++i)
    if (pl->P[i].cost_mode == MAM_COST_GRID && pl->batch)
      return fail(MAM_EUNSUPPORTED, "problem %d: a grid cost is for single problems", i);
  if (pl->P[0].R > kShortMaxR || pl->P[0].cost_mode == MAM_COST_GRID) {
    pl->lg.on = true;
    build_schedule(pl);
    build_layout(pl);
    return MAM_OK;
  }
  std::map<std::pair<int, int>, int> by_shape;
  for (int i = 0; i < n; ++i) {
    int nt = 0, vpt = 0;
    TRY(shape_for(pl->dtype, pl->P[i].R, 0, &nt, &vpt));
    auto key = std::make_pair(nt, vpt);
    if (!by_shape.count(key)) {
      by_shape[key] = (int)pl->G.size();
      pl->G.emplace_back();
    }
    Group& g = pl->G[by_shape[key]];
    g.probs.push_back(i);
    g.Rmax = std::max(g.Rmax, pl->P[i].R);
    pl->P[i].group = by_shape[key];
  }
  for (Group& g : pl->G) TRY(group_shape(pl, g));
  build_schedule(pl);
  build_layout(pl);
  return MAM_OK;
}

mam_status set_group_schedule(Plan* pl, int gi, const mam_schedule* s) {
  if (pl->ws) return fail(MAM_ESTATE, "schedule must be set before the workspace");
  if (s->rows_per_tile != 0 && s->rows_per_tile != 1024 && s->rows_per_tile != 2048 && s->rows_per_tile != 4096)
    return fail(MAM_EINVAL, "rows_per_tile must be 0, 1024, 2048 or 4096 (got %d)", s->rows_per_tile);
  if (s->candidate_slots < 0 || s->candidate_slots > 64)
    return fail(MAM_EINVAL, "candidate_slots must be in [0, 64] (got %d)", s->candidate_slots);
  if (s->rows_per_tile && pl->batch) return fail(MAM_EINVAL, "long-column tiles are for single problems");
  if (!pl->batch && (s->rows_per_tile > 0 || pl->P[0].R > kShortMaxR || pl->P[0].cost_mode == MAM_COST_GRID)) {
    if (s->workgroups < 0) return fail(MAM_EINVAL, "workgroups must be >= 0");
    pl->lg.on = true;
    pl->lg.rows_req = s->rows_per_tile;
    pl->lg.cap_req = s->candidate_slots;
    pl->lg.nwg_req = s->workgroups;
    build_schedule(pl);
    build_layout(pl);
    return MAM_OK;
  }
  pl->lg.on = false;
  if (s->order < 0 || s->order > 2) return fail(MAM_EINVAL, "order must be 0, 1 or 2 (got %d)", s->order);
  if (s->streaming < -1 || s->streaming > 1)
    return fail(MAM_EINVAL, "streaming must be -1, 0 or 1 (got %d)", s->streaming);
  if (s->team_size < 0 || s->team_size > 1024)
    return fail(MAM_EINVAL, "team_size must be in [0, 1024] (got %d)", s->team_size);
  Group& g = pl->G[gi];
  const Group saved = g;
  g.nt_req = s->threads_per_column;
  g.kc_req = s->columns_in_flight;
  mam_status st = group_shape(pl, g);
  if (st != MAM_OK) {
    g = saved;
    return st;
  }
  g.nwg_req = s->workgroups;
  g.xcd_req = s->xcd_remap;
  g.order_req = s->order;
  g.stream_req = s->streaming;
  g.team_req = s->team_size;
  build_schedule(pl);
  build_layout(pl);
  return MAM_OK;
}

void get_group_schedule(const Plan* pl, int gi, mam_schedule* s) {
  *s = mam_schedule{};
  if (pl->lg.on) {
    s->threads_per_column = 256;
    s->values_per_thread = pl->lg.vpt;
    s->columns_in_flight = 1;
    s->workgroups = pl->lg.nwg;
    s->xcd_remap = -1;
    s->vector_width = pl->lg.vec;
    s->order = 1;
    s->streaming = 1;
    s->rows_per_tile = pl->lg.rows;
    s->candidate_slots = pl->lg.cap;
    return;
  }
  const Group& g = pl->G[gi];
  s->threads_per_column = g.nt;
  s->values_per_thread = g.vpt;
  s->columns_in_flight = g.vec == 1 ? 1 : g.kc;
  s->workgroups = g.nwg;
  s->xcd_remap = g.xcd_remap;
  s->vector_width = g.vec;
  s->order = g.blocked ? 2 : 1;
  s->streaming = g.stream ? 1 : -1;
  s->team_size = g.team;
}

void drop_graphs(Plan* pl) {
  if (pl->gexec) {
    hipGraphExecDestroy(pl->gexec);
    pl->gexec = nullptr;
  }
  if (pl->uexec) {
    hipGraphExecDestroy(pl->uexec);
    pl->uexec = nullptr;
  }
}

mam_status set_workspace(Plan* pl, void* dev, size_t bytes) {
  if (!dev) return fail(MAM_ENOMEM, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(dev) % kAlign) return fail(MAM_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < pl->lay.total) return fail(MAM_ENOMEM, "workspace has %zu bytes, needs %zu", bytes, pl->lay.total);
  pl->ws = static_cast<char*>(dev);
  pl->ws_bytes = bytes;
  pl->tables_uploaded = false;
  pl->inited = false;
  return MAM_OK;
}

mam_status bind(Plan* pl, int i, void* theta, const void* cost, const int32_t* cidx, const void* q) {
  Prob& p = pl->P[i];
  if (!theta || !cost || !q) return fail(MAM_EINVAL, "theta, cost and q must be non-NULL");
  if (p.cost_mode == MAM_COST_INDEXED && !cidx) return fail(MAM_EINVAL, "MAM_COST_INDEXED needs cost_col_index");
  if (p.cost_mode != MAM_COST_INDEXED && cidx)
    return fail(MAM_EINVAL, "cost_col_index given but cost_mode is not MAM_COST_INDEXED");
  const size_t eb = elem_bytes(pl->dtype);
  const bool grid = p.cost_mode == MAM_COST_GRID;  // cost = the measures' points, doubles
  if (reinterpret_cast<uintptr_t>(theta) % eb || reinterpret_cast<uintptr_t>(cost) % (grid ? 8 : eb) ||
      reinterpret_cast<uintptr_t>(q) % eb)
    return fail(MAM_EINVAL, "buffers must be aligned to their element size");
  p.theta = theta;
  p.cost = cost;
  p.cidx = cidx;
  p.q = q;
  const int vn = vec_width(pl->dtype);
  p.aligned = reinterpret_cast<uintptr_t>(theta) % 16 == 0 && p.ld % vn == 0 &&
              (grid || (reinterpret_cast<uintptr_t>(cost) % 16 == 0 && p.cost_ld % vn == 0));
  if (pl->lg.on) {
    pl->lg.vec = p.aligned ? vn : 1;
  } else {
    Group& g = pl->G[p.group];
    bool all = true;
    for (int pi : g.probs) all = all && pl->P[pi].aligned;
    g.vec = (all && g.vpt >= vn) ? vn : 1;
  }
  pl->inited = false;
  pl->tables_uploaded = false;
  drop_graphs(pl);  // a captured graph holds the old buffers
  return MAM_OK;
}

// ---------------------------------------------------------------------------
// device tables
// ---------------------------------------------------------------------------
template <typename T>
void fill_probdev_one(Plan* pl, size_t i, mam::ProbDev<T>& d) {
  const Prob& p = pl->P[i];
  d.theta = static_cast<T*>(p.theta);
  d.cost = static_cast<const T*>(p.cost);
  d.q = static_cast<const T*>(p.q);
  d.cidx = p.cidx;
  d.acc = pl->lg.on ? nullptr : at<unsigned long long>(pl, p.o_acc);
  d.fx = pl->lg.on ? nullptr : at<double>(pl, p.o_fx);
  d.ld = p.ld;
  d.cost_ld = p.cost_ld;
  d.R = (int32_t)p.R;
  d.cost_mode = p.cost_mode;
  d.nb = p.nb;
  d.warm = (p.flags & MAM_FLAG_COLD) ? 0 : 1;
  d.relaxed = (p.flags & MAM_FLAG_RELAXED) ? 1 : 0;
  d.rho = p.rho;
  d.inv_rho = 1.0 / p.rho;
  d.gamma = p.gamma;
  d.pm = at<double>(pl, p.o_pm);
  d.p = at<double>(pl, p.o_p);
  d.d2part = at<double>(pl, p.o_d2);
  d.lam = at<double>(pl, p.o_lam);
  d.t_out = at<double>(pl, p.o_t);
  d.col_off = at<int64_t>(pl, p.o_coloff);
  d.Sd = at<double>(pl, p.o_Sd);
}

template <typename T>
void fill_probdev(Plan* pl, std::vector<mam::ProbDev<T>>& out) {
  out.resize(pl->P.size());
  for (size_t i = 0; i < pl->P.size(); ++i) fill_probdev_one<T>(pl, i, out[i]);
}


// Host staging for the table uploads; the copies complete before it is
// released (the upload synchronizes the stream).
mam_status upload_tables(Plan* pl, hipStream_t st) {
  if (pl->tables_uploaded) return MAM_OK;
  const Layout& L = pl->lay;
  auto put = [&](size_t off, const void* src, size_t bytes) -> mam_status {
    if (bytes) HIP_TRY(hipMemcpyAsync(pl->ws + off, src, bytes, hipMemcpyHostToDevice, st));
    return MAM_OK;
  };
  TRY(put(L.seg_p, pl->seg_p.data(), pl->seg_p.size() * 4));
  TRY(put(L.seg_m, pl->seg_m.data(), pl->seg_m.size() * 4));
  TRY(put(L.seg_j0, pl->seg_j0.data(), pl->seg_j0.size() * 8));
  TRY(put(L.seg_j1, pl->seg_j1.data(), pl->seg_j1.size() * 8));
  // every segment table must fit the capacity the layout reserved
  const size_t nseg = std::max({pl->seg_p.size(), pl->seg_m.size(), pl->seg_j0.size(), pl->seg_j1.size(),
                                pl->seg_poff.size(), pl->seg_st.size(), pl->mpoff.size()});
  if (nseg > pl->nseg_cap && !pl->lg.on)
    return fail(MAM_EHIP, "schedule of %zu segments exceeds its capacity %zu", nseg, pl->nseg_cap);
  if (pl->lg.on && (pl->seg_p.size() || pl->seg_st.size()))
    return fail(MAM_EHIP, "a long-column plan holds short-column segments");
  TRY(put(L.seg_poff, pl->seg_poff.data(), pl->seg_poff.size() * 8));
  TRY(put(L.seg_idx, pl->mpoff.data(), pl->mpoff.size() * 8));
  TRY(put(L.seg_st, pl->seg_st.data(), pl->seg_st.size() * 4));
  TRY(put(L.wg_seg, pl->wg_seg.data(), pl->wg_seg.size() * 4));
  TRY(put(L.mseg, pl->mseg.data(), pl->mseg.size() * 4));
  TRY(put(L.mtasks, pl->mtasks.data(), pl->mtasks.size() * sizeof(mam::MargTask)));
  TRY(put(L.atasks, pl->atasks.data(), pl->atasks.size() * sizeof(mam::AvgTask)));
  std::vector<mam::ProbAux> aux(pl->P.size());
  for (size_t i = 0; i < pl->P.size(); ++i) {
    Prob& p = pl->P[i];
    aux[i] = {at<double>(pl, p.o_pm), at<double>(pl, p.o_pm_prev), at<double>(pl, p.o_p), at<double>(pl, p.o_p_prev),
              at<double>(pl, p.o_d2), at<double>(pl, p.o_aw), at<double>(pl, p.o_Sd), (int32_t)p.R,
              (int32_t)p.M, p.mbase, p.nb,
              pl->lg.on ? nullptr : at<unsigned long long>(pl, p.o_acc),
              pl->lg.on ? nullptr : at<double>(pl, p.o_fx) + p.M, p.rho, p.gamma, at<double>(pl, p.o_t)};
    TRY(put(p.o_coloff, p.col_off.data(), p.col_off.size() * 8));
    TRY(put(p.o_Sd, p.Sd.data(), p.Sd.size() * 8));
    TRY(put(p.o_aw, p.aw.data(), p.aw.size() * 8));
  }
  TRY(put(L.probaux, aux.data(), aux.size() * sizeof(mam::ProbAux)));
  if (pl->lg.on) {
    const LongPlan& lg = pl->lg;
    TRY(put(lg.o_it_rb, lg.it_rb.data(), lg.it_rb.size() * 4));
    TRY(put(lg.o_it_m, lg.it_m.data(), lg.it_m.size() * 4));
    TRY(put(lg.o_it_j0, lg.it_j0.data(), lg.it_j0.size() * 8));
    TRY(put(lg.o_it_j1, lg.it_j1.data(), lg.it_j1.size() * 8));
    TRY(put(lg.o_it_poff, lg.it_poff.data(), lg.it_poff.size() * 8));
    TRY(put(lg.o_wg_it, lg.wg_it.data(), lg.wg_it.size() * 4));
  }
  std::vector<mam::ProbDev<float>> pdf;
  std::vector<mam::ProbDev<double>> pdd;
  if (pl->dtype == MAM_F32) {
    fill_probdev<float>(pl, pdf);
    TRY(put(L.probdev, pdf.data(), pdf.size() * sizeof(pdf[0])));
  } else {
    fill_probdev<double>(pl, pdd);
    TRY(put(L.probdev, pdd.data(), pdd.size() * sizeof(pdd[0])));
  }
  HIP_TRY(hipStreamSynchronize(st));
  pl->tables_uploaded = true;
  return MAM_OK;
}

// ---------------------------------------------------------------------------
// launches
// ---------------------------------------------------------------------------
mam_status group_streams(Plan* pl) {
  while (pl->gstream.size() < pl->G.size()) {
    hipStream_t s = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    pl->gstream.push_back(s);
    hipEvent_t e = nullptr;
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    pl->gjoin.push_back(e);
  }
  if (!pl->gfork) HIP_TRY(hipEventCreateWithFlags(&pl->gfork, hipEventDisableTiming));
  return MAM_OK;
}

template <typename T>
mam_status launch_columns(Plan* pl, hipStream_t st, int diag, uint8_t* rec, int64_t rec_ld) {
  const Layout& L = pl->lay;
  const bool fork = pl->G.size() > 1 && pl->capturing;
  if (fork) {
    TRY(group_streams(pl));
    HIP_TRY(hipEventRecord(pl->gfork, st));
  }
  for (size_t gi = 0; gi < pl->G.size(); ++gi) {
    const Group& g = pl->G[gi];
    hipStream_t gs = fork ? pl->gstream[gi] : st;
    if (fork) HIP_TRY(hipStreamWaitEvent(gs, pl->gfork, 0));
    mam::ColArgs<T> a;
    a.probs = at<mam::ProbDev<T>>(pl, L.probdev);
    a.seg_p = at<int32_t>(pl, L.seg_p);
    a.seg_m = at<int32_t>(pl, L.seg_m);
    a.seg_j0 = at<int64_t>(pl, L.seg_j0);
    a.seg_j1 = at<int64_t>(pl, L.seg_j1);
    a.seg_st = at<int32_t>(pl, L.seg_st);
    a.wg_seg = at<int32_t>(pl, L.wg_seg) + g.wg_base;
    a.diag = at<double>(pl, L.diag) + (size_t)g.wg_base * mam::DIAG_STRIDE;
    a.rec = rec;
    a.rec_ld = rec_ld;
    a.stop = pl->gate;
    a.nwg = g.nwg;
    a.xcd_remap = g.xcd_remap;
    a.kb = group_block(g);
    const int kc = g.vec == 1 ? 1 : g.kc;
    if (g.nt < 64 && (diag || rec))
      return fail(MAM_EUNSUPPORTED, "diagnostics and the reverse mode need 64 or more threads per column");
    mam::ColFn<T> fn = mam::pick_column<T>(g.nt, g.vpt, g.vec, kc, diag, g.stream);
    if (!fn) return fail(MAM_EUNSUPPORTED, "no column kernel for nt=%d vpt=%d vec=%d kc=%d", g.nt, g.vpt, g.vec, kc);
    const int wgsize = g.nt <= 64 ? 256 : g.nt;
    const size_t shmem = (size_t)g.vpt * g.nt * 8 * (1 + g.ng);
    if (shmem > 65536) {
      // above the default dynamic-LDS limit: opt this kernel in
      HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)shmem));
    }
    hipLaunchKernelGGL(fn, dim3(g.nwg), dim3(wgsize), shmem, gs, a);
    LAUNCH_CHECK("column_kernel");
    if (fork) HIP_TRY(hipEventRecord(pl->gjoin[gi], gs));
  }
  if (fork)
    for (size_t gi = 0; gi < pl->G.size(); ++gi) HIP_TRY(hipStreamWaitEvent(st, pl->gjoin[gi], 0));
  return MAM_OK;
}

// ---------------------------------------------------------------------------
// long-column iterations
// ---------------------------------------------------------------------------
template <typename T>
mam::LongArgs<T> long_args(Plan* pl) {
  const Prob& p = pl->P[0];
  const LongPlan& lg = pl->lg;
  mam::LongArgs<T> a{};
  a.theta = static_cast<T*>(p.theta);
  a.cost = static_cast<const T*>(p.cost);
  a.q = static_cast<const T*>(p.q);
  a.cidx = p.cidx;
  a.ld = p.ld;
  a.cost_ld = p.cost_ld;
  a.R = (int32_t)p.R;
  a.cost_mode = p.cost_mode;
  a.M = (int32_t)p.M;
  a.nrb = lg.nrb;
  a.cap = lg.cap;
  a.warm = (p.flags & MAM_FLAG_COLD) ? 0 : 1;
  a.relaxed = (p.flags & MAM_FLAG_RELAXED) ? 1 : 0;
  a.rho = p.rho;
  a.inv_rho = 1.0 / p.rho;
  a.gamma = p.gamma;
  a.t = at<double>(pl, p.o_t);
  a.p = at<double>(pl, p.o_p);
  a.pm = at<double>(pl, p.o_pm);
  a.d2part = at<double>(pl, p.o_d2);
  a.nb = p.nb;
  a.Sd = at<double>(pl, p.o_Sd);
  a.col_off = at<int64_t>(pl, p.o_coloff);
  a.it_rb = at<int32_t>(pl, lg.o_it_rb);
  a.it_m = at<int32_t>(pl, lg.o_it_m);
  a.it_j0 = at<int64_t>(pl, lg.o_it_j0);
  a.it_j1 = at<int64_t>(pl, lg.o_it_j1);
  a.it_poff = at<int64_t>(pl, lg.o_it_poff);
  a.wg_it = at<int32_t>(pl, lg.o_wg_it);
  a.hmax = at<double>(pl, lg.o_hmax);
  a.hcnt = at<int32_t>(pl, lg.o_hcnt);
  a.crow = at<int32_t>(pl, lg.o_crow);
  a.cw = at<double>(pl, lg.o_cw);
  a.lam = at<double>(pl, p.o_lam);
  a.partial = at<double>(pl, pl->lay.partial);
  a.stop = pl->gate;
  a.T_cols = p.T;
  a.gdim = p.cost_mode == MAM_COST_GRID ? p.gdim : 0;
  a.gn1 = (int32_t)(p.gdim == 2 ? p.gn[1] : 1);
  for (int k = 0; k < 2; ++k) {
    a.go[k] = p.go[k];
    a.gh[k] = p.gh[k];
  }
  a.gz = a.gdim ? static_cast<const double*>(p.cost) : nullptr;
  a.ldiag = at<double>(pl, lg.o_ldiag);
  a.wdiag = at<double>(pl, lg.o_wdiag);
  a.sparse = lg.sparse ? 1 : 0;
  if (lg.sparse) {
    a.spar = at<int32_t>(pl, lg.o_spar);
    a.pcnt = at<int32_t>(pl, lg.o_pcnt);
    a.prow = at<int32_t>(pl, lg.o_prow);
    a.pval = at<T>(pl, lg.o_pval);
    a.nbv = at<T>(pl, lg.o_nbv);
  }
  return a;
}

// t^k, then scan, threshold and write (the scan rewrites every header).
template <typename T>
mam_status launch_long_columns(Plan* pl, hipStream_t st, int diag) {
  const Prob& p = pl->P[0];
  const LongPlan& lg = pl->lg;
  mam::LongFns<T> fn = mam::pick_long<T>(lg.vpt, lg.vec, pl->P[0].cost_mode == MAM_COST_GRID);
  if (!fn.scan) return fail(MAM_EUNSUPPORTED, "no long-column kernels for vpt=%d vec=%d", lg.vpt, lg.vec);
  mam::LongArgs<T> a = long_args<T>(pl);
  hipLaunchKernelGGL(mam::damping_kernel, dim3(1), dim3(256), 0, st, a.d2part, p.nb, p.rho, p.gamma, a.t, a.stop);
  LAUNCH_CHECK("damping_kernel");
  if (lg.sparse) hipLaunchKernelGGL(fn.scan_sparse, dim3(lg.nwg), dim3(mam::LNT), (size_t)lg.vpt * mam::LNT * 8, st, a);
  else hipLaunchKernelGGL(fn.scan, dim3(lg.nwg), dim3(mam::LNT), 0, st, a);
  LAUNCH_CHECK("long_scan_kernel");
  hipLaunchKernelGGL(diag ? fn.thresh_diag : fn.thresh, dim3((unsigned)((p.T + 3) / 4)), dim3(256), 0, st, a);
  LAUNCH_CHECK("long_threshold_kernel");
  hipLaunchKernelGGL(diag ? fn.write_diag : fn.write, dim3(lg.nwg), dim3(mam::LNT), (size_t)lg.vpt * mam::LNT * 8, st,
                     a);
  LAUNCH_CHECK("long_write_kernel");
  if (lg.sparse) {
    hipLaunchKernelGGL(mam::long_sparse_flip_kernel, dim3(1), dim3(64), 0, st, a.spar, a.stop);
    LAUNCH_CHECK("long_sparse_flip_kernel");
  }
  return MAM_OK;
}

// Sparse store: every sub-tile dense (after theta^0 is in place), or the
// stored plans written back into theta (when a call returns).
template <typename T>
mam_status long_sparse_reset(Plan* pl, hipStream_t st) {
  const LongPlan& lg = pl->lg;
  const int64_t nh = pl->P[0].T * (int64_t)lg.nrb * 4;
  const int blocks = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (nh + 255) / 256));
  hipLaunchKernelGGL(mam::long_sparse_reset_kernel, dim3(blocks), dim3(256), 0, st, at<int32_t>(pl, lg.o_pcnt), nh,
                     at<int32_t>(pl, lg.o_spar));
  LAUNCH_CHECK("long_sparse_reset_kernel");
  return MAM_OK;
}

template <typename T>
mam_status long_writeback(Plan* pl, hipStream_t st) {
  const LongPlan& lg = pl->lg;
  mam::LongFns<T> fn = mam::pick_long<T>(lg.vpt, lg.vec, pl->P[0].cost_mode == MAM_COST_GRID);
  if (!fn.materialize) return fail(MAM_EUNSUPPORTED, "no long-column kernels for vpt=%d vec=%d", lg.vpt, lg.vec);
  hipLaunchKernelGGL(fn.materialize, dim3(lg.nwg), dim3(mam::LNT), 0, st, long_args<T>(pl));
  LAUNCH_CHECK("long_materialize_kernel");
  return MAM_OK;
}

mam_status sparse_writeback(Plan* pl, hipStream_t st) {
  if (!pl->lg.on || !pl->lg.sparse || !pl->inited) return MAM_OK;
  return pl->dtype == MAM_F32 ? long_writeback<float>(pl, st) : long_writeback<double>(pl, st);
}

template <typename T>
mam_status launch_long_rowsum(Plan* pl, hipStream_t st) {
  const LongPlan& lg = pl->lg;
  mam::LongFns<T> fn = mam::pick_long<T>(lg.vpt, lg.vec, pl->P[0].cost_mode == MAM_COST_GRID);
  if (!fn.rowsum) return fail(MAM_EUNSUPPORTED, "no long-column kernels for vpt=%d vec=%d", lg.vpt, lg.vec);
  hipLaunchKernelGGL(fn.rowsum, dim3(lg.nwg), dim3(256), 0, st, long_args<T>(pl), lg.rows);
  LAUNCH_CHECK("long_rowsum_kernel");
  return MAM_OK;
}

// Workgroups of the scan kernel the device holds at once.
template <typename T>
mam_status long_resident(Plan* pl, bool* changed) {
  mam::LongFns<T> fn = mam::pick_long<T>(pl->lg.vpt, pl->lg.vec, pl->P[0].cost_mode == MAM_COST_GRID);
  if (!fn.scan) return MAM_OK;
  int dev = 0, cus = 0, blocks = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void*>(fn.scan), mam::LNT, 0));
  const int res = std::max(1, blocks) * std::max(1, cus);
  if (res != pl->lg.nwg_auto) {
    pl->lg.nwg_auto = res;
    *changed = true;
  }
  return MAM_OK;
}

mam_status launch_average(Plan* pl, hipStream_t st, int save_prev) {
  const Layout& L = pl->lay;
  hipLaunchKernelGGL(mam::average_kernel, dim3((unsigned)pl->atasks.size()), dim3(256), 0, st,
                     at<mam::AvgTask>(pl, L.atasks), at<mam::ProbAux>(pl, L.probaux), save_prev, pl->gate);
  LAUNCH_CHECK("average_kernel");
  return MAM_OK;
}

// Steps 3 and 1 after the column kernels.  Short columns: with at most
// kFusedCloseM measures per problem, one row-parallel kernel (the new
// marginals from the fixed-point sums, then the average: one launch fewer);
// with more, the marginals of every (measure, row block) in parallel, then
// the average.  Long columns: the marginals from the row-tile partials, then
// the average.
constexpr int64_t kFusedCloseM = 8;
mam_status launch_marginals(Plan* pl, hipStream_t st, int save_prev) {
  const Layout& L = pl->lay;
  if (pl->lg.on) {
    hipLaunchKernelGGL(mam::marginal_kernel, dim3((unsigned)pl->mtasks.size()), dim3(256), 0, st,
                       at<mam::MargTask>(pl, L.mtasks), at<mam::ProbAux>(pl, L.probaux), at<int32_t>(pl, L.mseg),
                       at<int64_t>(pl, L.seg_idx), at<double>(pl, L.partial), save_prev, pl->gate);
    LAUNCH_CHECK("marginal_kernel");
    return launch_average(pl, st, save_prev);
  }
  int64_t mmax = 0;
  for (const Prob& p : pl->P) mmax = std::max(mmax, p.M);
  if (mmax <= kFusedCloseM) {
    hipLaunchKernelGGL(mam::close_kernel, dim3((unsigned)pl->atasks.size()), dim3(256), 0, st,
                       at<mam::AvgTask>(pl, L.atasks), at<mam::ProbAux>(pl, L.probaux), save_prev, pl->gate);
    LAUNCH_CHECK("close_kernel");
    return MAM_OK;
  }
  hipLaunchKernelGGL(mam::fixed_marginal_kernel, dim3((unsigned)pl->mtasks.size()), dim3(256), 0, st,
                     at<mam::MargTask>(pl, L.mtasks), at<mam::ProbAux>(pl, L.probaux), save_prev, pl->gate);
  LAUNCH_CHECK("fixed_marginal_kernel");
  return launch_average(pl, st, save_prev);
}


// Copy of a problem's plans (the R stored rows of each column), with 16-byte
// accesses when both buffers and the column stride allow them.
template <typename T>
mam_status launch_plan_copy(T* dst, const T* src, const Prob& p, hipStream_t st) {
  constexpr int VN = 16 / (int)sizeof(T);
  const bool vec = p.ld % VN == 0 && reinterpret_cast<uintptr_t>(dst) % 16 == 0 &&
                   reinterpret_cast<uintptr_t>(src) % 16 == 0;
  const int blocks = (int)std::min<int64_t>(4096, std::max<int64_t>(1, p.T));
  if (vec)
    hipLaunchKernelGGL((mam::copy_kernel<T, VN>), dim3(blocks), dim3(256), 0, st, dst, p.ld, (int)p.R, src, p.T);
  else
    hipLaunchKernelGGL((mam::copy_kernel<T, 1>), dim3(blocks), dim3(256), 0, st, dst, p.ld, (int)p.R, src, p.T);
  LAUNCH_CHECK("copy_kernel");
  return MAM_OK;
}

template <typename T>
mam_status launch_init(Plan* pl, const void* const* theta0, hipStream_t st) {
  const Layout& L = pl->lay;
  for (size_t i = 0; i < pl->P.size(); ++i) {
    Prob& p = pl->P[i];
    const int blocks = (int)std::min<int64_t>(8192, std::max<int64_t>(1, (p.T * p.R + 255) / 256));
    if (theta0 && theta0[i]) {
      TRY(launch_plan_copy<T>(static_cast<T*>(p.theta), static_cast<const T*>(theta0[i]), p, st));
    } else {
      hipLaunchKernelGGL(mam::fill_kernel<T>, dim3(blocks), dim3(256), 0, st, static_cast<T*>(p.theta), p.ld,
                         (int)p.R, static_cast<const T*>(p.q), p.T);
      LAUNCH_CHECK("fill_kernel");
    }
    hipLaunchKernelGGL(mam::fill_value_kernel, dim3((unsigned)std::min<int64_t>(4096, (p.T + 255) / 256)), dim3(256),
                       0, st, at<double>(pl, p.o_lam), p.T, (double)NAN);
    LAUNCH_CHECK("fill_value_kernel");
  }
  if (pl->lg.on) {
    TRY(launch_long_rowsum<T>(pl, st));
    return launch_marginals(pl, st, 0);
  }
  // short columns: the fixed-point accumulators start (and stay, between
  // iterations) at zero; the marginals of the start are plain row sums
  for (Prob& p : pl->P) {
    const int64_t n = p.M * p.R;
    hipLaunchKernelGGL(mam::fill_value_kernel, dim3((unsigned)std::min<int64_t>(4096, (n + 255) / 256)), dim3(256), 0,
                       st, at<double>(pl, p.o_acc), n, 0.0);
    LAUNCH_CHECK("fill_value_kernel");
  }
  // vector loads when every problem's plans are 16-byte aligned with a
  // leading dimension that is a multiple of the vector
  bool aligned = true;
  for (const Prob& p : pl->P) aligned = aligned && p.aligned;
  constexpr int VN = sizeof(T) == 4 ? 4 : 2;
  auto fn = aligned ? &mam::init_marginal_kernel<T, VN> : &mam::init_marginal_kernel<T, 1>;
  hipLaunchKernelGGL(fn, dim3((unsigned)pl->mtasks.size()), dim3(256), 0, st, at<mam::MargTask>(pl, L.mtasks),
                     at<mam::ProbDev<T>>(pl, L.probdev), at<mam::ProbAux>(pl, L.probaux));
  LAUNCH_CHECK("init_marginal_kernel");
  return launch_average(pl, st, 0);
}

template <typename T>
mam_status launch_checks(Plan* pl, hipStream_t st) {
  for (Prob& p : pl->P) {
    double* chk = at<double>(pl, p.o_check);
    hipLaunchKernelGGL(mam::zero_kernel, dim3((unsigned)((p.M + 2 + 255) / 256)), dim3(256), 0, st, chk,
                       (int)(p.M + 2));
    LAUNCH_CHECK("zero_kernel");
    hipLaunchKernelGGL(mam::check_q_kernel<T>, dim3((unsigned)p.M), dim3(256), 0, st, static_cast<const T*>(p.q),
                       at<int64_t>(pl, p.o_coloff), chk, (int)p.M);
    LAUNCH_CHECK("check_q_kernel");
    if (p.cost_mode == MAM_COST_GRID) {
      // the measures' points: cost_ncols rows of gdim doubles
      const int blocks = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (p.cost_ncols * p.gdim + 255) / 256));
      hipLaunchKernelGGL(mam::check_cost_kernel<double>, dim3(blocks), dim3(256), 0, st,
                         static_cast<const double*>(p.cost), (int64_t)p.gdim, p.gdim, p.cost_ncols, chk + p.M + 1);
    } else {
      const int blocks = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (p.cost_ncols * p.R + 255) / 256));
      hipLaunchKernelGGL(mam::check_cost_kernel<T>, dim3(blocks), dim3(256), 0, st, static_cast<const T*>(p.cost),
                         p.cost_ld, (int)p.R, p.cost_ncols, chk + p.M + 1);
    }
    LAUNCH_CHECK("check_cost_kernel");
  }
  return MAM_OK;
}

hipEvent_t next_event(Plan* pl) {
  if (pl->ev_used == pl->ev.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    pl->ev.push_back(e);
  }
  return pl->ev[pl->ev_used++];
}

// ---------------------------------------------------------------------------
// plan operations shared by single problems and batches
// ---------------------------------------------------------------------------
// Workgroups of each group's column kernel that the current device holds at
// once (occupancy of that instance times the compute units).
template <typename T>
mam_status resident_workgroups(Plan* pl, bool* changed) {
  int dev = 0, cus = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  for (Group& g : pl->G) {
    const int kc = g.vec == 1 ? 1 : g.kc;
    mam::ColFn<T> fn = mam::pick_column<T>(g.nt, g.vpt, g.vec, kc, 0, g.stream);
    if (!fn) continue;
    const int wgsize = g.nt <= 64 ? 256 : g.nt;
    const size_t shmem = (size_t)g.vpt * g.nt * 8 * (1 + g.ng);
    if (shmem > 65536)
      HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)shmem));
    int blocks = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void*>(fn), wgsize, shmem));
    const int res = std::max(1, blocks) * std::max(1, cus);
    if (res != g.nwg_auto) {
      g.nwg_auto = res;
      *changed = true;
    }
  }
  return MAM_OK;
}

mam_status plan_init(Plan* pl, const void* const* theta0, hipStream_t st) {
  if (!pl->ws) return fail(MAM_ESTATE, "no workspace");
  for (size_t i = 0; i < pl->P.size(); ++i)
    if (pl->P[i].cost_mode == MAM_COST_GRID && pl->P[i].gdim == 0)
      return fail(MAM_ESTATE, "problem %zu: MAM_COST_GRID needs mam_set_grid", i);
  for (size_t i = 0; i < pl->P.size(); ++i)
    if (!pl->P[i].theta) return fail(MAM_ESTATE, "problem %zu has no buffers bound", i);
  // an indexed cost's column order depends on its index: read it once here
  bool rebuilt = false;
  for (Prob& p : pl->P) {
    if (p.cost_mode != MAM_COST_INDEXED) continue;
    p.idx.resize(p.T);
    HIP_TRY(hipMemcpyAsync(p.idx.data(), p.cidx, p.T * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int64_t j = 0; j < p.T; ++j)
      if (p.idx[j] < 0 || p.idx[j] >= p.cost_ncols)
        return fail(MAM_ENONFINITE, "cost_col_index[%lld] = %d is out of range", (long long)j, p.idx[j]);
    rebuilt = true;
  }
  if (pl->lg.on)
    TRY(pl->dtype == MAM_F32 ? long_resident<float>(pl, &rebuilt) : long_resident<double>(pl, &rebuilt));
  else
    TRY(pl->dtype == MAM_F32 ? resident_workgroups<float>(pl, &rebuilt) : resident_workgroups<double>(pl, &rebuilt));
  if (rebuilt) build_schedule(pl);
  drop_graphs(pl);
  TRY(upload_tables(pl, st));
  TRY(pl->dtype == MAM_F32 ? launch_checks<float>(pl, st) : launch_checks<double>(pl, st));
  std::vector<double> fx;
  for (size_t i = 0; i < pl->P.size(); ++i) {
    Prob& p = pl->P[i];
    std::vector<double> chk(p.M + 2);
    HIP_TRY(hipMemcpyAsync(chk.data(), pl->ws + p.o_check, (p.M + 2) * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (!pl->lg.on) {
      // fixed-point scales of the marginal sums: 2^E_m with mass_m <= 2^(62 - E_m),
      // so no row sum of pi_hat (at most mass_m) exceeds 2^62; then 2^-E_m
      fx.assign(2 * p.M, 0.0);
      for (int64_t m = 0; m < p.M; ++m) {
        int e = 0;
        if (chk[m] > 0.0 && std::isfinite(chk[m])) std::frexp(chk[m], &e);  // mass = f 2^e, f in [0.5, 1)
        const int E = std::min(1000, 62 - e);
        fx[m] = std::ldexp(1.0, E);
        fx[p.M + m] = std::ldexp(1.0, -E);
      }
      HIP_TRY(hipMemcpyAsync(pl->ws + p.o_fx, fx.data(), fx.size() * 8, hipMemcpyHostToDevice, st));
      HIP_TRY(hipStreamSynchronize(st));  // fx is reused for the next problem
    }
    if (chk[p.M] != 0.0) return fail(MAM_ENONFINITE, "problem %zu: q holds a negative or non-finite weight", i);
    if (chk[p.M + 1] != 0.0) return fail(MAM_ENONFINITE, "problem %zu: cost holds a non-finite entry", i);
    if (std::isinf(p.gamma) && !(p.flags & MAM_FLAG_RELAXED)) {
      const double tol = pl->dtype == MAM_F32 ? 1e-6 : 1e-12;
      double lo = chk[0], hi = chk[0];
      for (int64_t m = 1; m < p.M; ++m) {
        lo = std::min(lo, chk[m]);
        hi = std::max(hi, chk[m]);
      }
      if (hi - lo > tol * std::max(std::fabs(hi), 1e-300))
        return fail(MAM_ENOTBALANCED, "problem %zu: balanced mode but masses range over [%.17g, %.17g]", i, lo, hi);
    }
  }
  TRY(pl->dtype == MAM_F32 ? launch_init<float>(pl, theta0, st) : launch_init<double>(pl, theta0, st));
  if (pl->lg.on && pl->lg.sparse)
    TRY(pl->dtype == MAM_F32 ? long_sparse_reset<float>(pl, st) : long_sparse_reset<double>(pl, st));
  pl->inited = true;
  pl->default_start = true;
  for (size_t i = 0; i < pl->P.size(); ++i)
    if (theta0 && theta0[i]) pl->default_start = false;
  pl->iters_done = 0;
  pl->diag_valid = false;
  return MAM_OK;
}

// save_prev < 0: keep the previous marginals when computing diagnostics
mam_status one_iteration(Plan* pl, hipStream_t st, int diag, uint8_t* rec = nullptr, int64_t rec_ld = 0,
                         int save_prev = -1) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (pl->timing) {
    e0 = next_event(pl);
    e1 = next_event(pl);
    if (!e0 || !e1) return fail(MAM_EHIP, "hipEventCreate failed");
    HIP_TRY(hipEventRecord(e0, st));
  }
  if (pl->lg.on) {
    if (rec) return fail(MAM_EUNSUPPORTED, "the reverse mode is not available for long columns");
    TRY(pl->dtype == MAM_F32 ? launch_long_columns<float>(pl, st, diag) : launch_long_columns<double>(pl, st, diag));
  } else {
    TRY(pl->dtype == MAM_F32 ? launch_columns<float>(pl, st, diag, rec, rec_ld)
                              : launch_columns<double>(pl, st, diag, rec, rec_ld));
  }
  if (pl->timing) HIP_TRY(hipEventRecord(e1, st));
  return launch_marginals(pl, st, save_prev < 0 ? diag : save_prev);
}

// Capture graph_iters iterations once on a stream of the library's own (a
// caller's legacy default stream cannot be captured); replays run on the
// caller's stream.
mam_status capture_graph(Plan* pl) {
  if (!pl->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&pl->capture_stream, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(pl->capture_stream, hipStreamCaptureModeThreadLocal));
  mam_status s = MAM_OK;
  pl->capturing = true;
  for (int64_t k = 0; k < pl->graph_iters && s == MAM_OK; ++k) s = one_iteration(pl, pl->capture_stream, 0);
  pl->capturing = false;
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(pl->capture_stream, &graph);
  if (s != MAM_OK) {
    if (graph) hipGraphDestroy(graph);
    return s;
  }
  if (e != hipSuccess) return fail(MAM_EHIP, "graph capture failed: %s", hipGetErrorString(e));
  const hipError_t e2 = hipGraphInstantiate(&pl->gexec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (e2 != hipSuccess) {
    pl->gexec = nullptr;
    return fail(MAM_EHIP, "graph instantiation failed: %s", hipGetErrorString(e2));
  }
  return MAM_OK;
}

mam_status plan_iterate(Plan* pl, int64_t iters, hipStream_t st) {
  if (iters < 0) return fail(MAM_EINVAL, "iters must be >= 0");
  if (!pl->inited) return fail(MAM_ESTATE, "mam_init has not run");
  const bool want_diag = !pl->batch && (pl->P[0].flags & MAM_FLAG_DIAG);
  int64_t k = 0;
  if (pl->graph_iters > 0 && !pl->timing) {
    // keep the last iteration outside the graph when it computes diagnostics
    const int64_t plain = want_diag ? 1 : 0;
    if (iters - plain >= pl->graph_iters) {
      if (!pl->gexec) TRY(capture_graph(pl));
      while (iters - k - plain >= pl->graph_iters) {
        HIP_TRY(hipGraphLaunch(pl->gexec, st));
        k += pl->graph_iters;
      }
    }
  }
  for (; k < iters; ++k) {
    const int diag = want_diag && k == iters - 1;
    TRY(one_iteration(pl, st, diag));
    if (diag) pl->diag_valid = true;
  }
  pl->iters_done += iters;
  return sparse_writeback(pl, st);
}

mam_status plan_graph(Plan* pl, int64_t iters) {
  if (iters < 0) return fail(MAM_EINVAL, "iterations per graph must be >= 0");
  if (pl->gexec) {
    hipGraphExecDestroy(pl->gexec);
    pl->gexec = nullptr;
  }
  pl->graph_iters = iters;
  return MAM_OK;
}

// ---------------------------------------------------------------------------
// runs with an on-device stopping test (Sec. 5, stopping criteria)
// ---------------------------------------------------------------------------
static_assert(offsetof(mam::StopState, stop) == 0, "the gate flag is the state's first word");
static_assert(MAM_STOP_DTHETA == mam::STOP_DTHETA && MAM_STOP_DP == mam::STOP_DP &&
                  MAM_STOP_DIST == mam::STOP_DIST,
              "stopping-test codes");

// One check period: every-1 plain iterations, then the check iteration
// (diagnostics of the column kernel for the theta test, previous marginals
// kept for the others) and the test itself, all gated by the stop flag.
mam_status until_period(Plan* pl, hipStream_t st, int test, int64_t every) {
  const Layout& L = pl->lay;
  for (int64_t k = 0; k + 1 < every; ++k) TRY(one_iteration(pl, st, 0));
  TRY(one_iteration(pl, st, test == MAM_STOP_DTHETA ? 1 : 0, nullptr, 0, 1));
  mam::StopState* ss = at<mam::StopState>(pl, L.stop);
  const Prob& pr = pl->P[0];
  if (test != MAM_STOP_DTHETA) {
    hipLaunchKernelGGL(mam::stop_partial_kernel, dim3((unsigned)pr.nb), dim3(256), 0, st,
                       at<mam::ProbAux>(pl, L.probaux), at<double>(pl, pr.o_t), test, at<double>(pl, L.stop_part),
                       ss);
    LAUNCH_CHECK("stop_partial_kernel");
  }
  // the per-workgroup maxima of |theta' - theta|: the column kernel's, or
  // the long write kernel's
  const double* dslots = pl->lg.on ? at<double>(pl, pl->lg.o_wdiag) : at<double>(pl, L.diag);
  const int nslots = pl->lg.on ? pl->lg.nwg : pl->nwg_total;
  hipLaunchKernelGGL(mam::stop_final_kernel, dim3(1), dim3(256), 0, st, ss, test, at<double>(pl, L.stop_part),
                     pr.nb, dslots, nslots, pl->host_flag);
  LAUNCH_CHECK("stop_final_kernel");
  return MAM_OK;
}

mam_status capture_until(Plan* pl, int test, int64_t every) {
  if (!pl->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&pl->capture_stream, hipStreamNonBlocking));
  if (pl->uexec) {
    hipGraphExecDestroy(pl->uexec);
    pl->uexec = nullptr;
  }
  HIP_TRY(hipStreamBeginCapture(pl->capture_stream, hipStreamCaptureModeThreadLocal));
  pl->capturing = true;
  const mam_status s = until_period(pl, pl->capture_stream, test, every);
  pl->capturing = false;
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(pl->capture_stream, &graph);
  if (s != MAM_OK) {
    if (graph) hipGraphDestroy(graph);
    return s;
  }
  if (e != hipSuccess) return fail(MAM_EHIP, "graph capture failed: %s", hipGetErrorString(e));
  const hipError_t e2 = hipGraphInstantiate(&pl->uexec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (e2 != hipSuccess) {
    pl->uexec = nullptr;
    return fail(MAM_EHIP, "graph instantiation failed: %s", hipGetErrorString(e2));
  }
  pl->utest = test;
  pl->uevery = every;
  return MAM_OK;
}

// Periods are enqueued with a bounded number in flight: before enqueuing
// period i the host waits for period i - ahead and reads the host-visible
// stop flag, so after the stop at most 'ahead' periods of gated (empty)
// launches follow.  The gate makes the iterate exact whatever was enqueued.
mam_status until_run(Plan* pl, int64_t max_iters, int test, double tol, int64_t every, hipStream_t st,
                     mam_stop_result* out) {
  const Layout& L = pl->lay;
  if (!pl->host_flag) {
    void* h = nullptr;
    HIP_TRY(hipHostMalloc(&h, 256, hipHostMallocCoherent));
    pl->host_flag = static_cast<int32_t*>(h);
  }
  *reinterpret_cast<volatile int32_t*>(pl->host_flag) = 0;
  mam::StopState* ss = at<mam::StopState>(pl, L.stop);
  hipLaunchKernelGGL(mam::stop_reset_kernel, dim3(1), dim3(64), 0, st, ss, tol);
  LAUNCH_CHECK("stop_reset_kernel");
  const int64_t periods = max_iters / every, tail = max_iters % every;
  const bool graph = pl->graph_iters > 0 && !pl->timing;
  if (graph && periods > 0 && (!pl->uexec || pl->utest != test || pl->uevery != every))
    TRY(capture_until(pl, test, every));
  const int64_t ahead = std::max<int64_t>(2, (32 + every - 1) / every);
  while ((int64_t)pl->uev.size() < ahead) {
    hipEvent_t e = nullptr;
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    pl->uev.push_back(e);
  }
  bool seen_stop = false;
  for (int64_t i = 0; i < periods; ++i) {
    if (i >= ahead) {
      HIP_TRY(hipEventSynchronize(pl->uev[(i - ahead) % ahead]));
      if (*reinterpret_cast<volatile int32_t*>(pl->host_flag) != 0) {
        seen_stop = true;
        break;
      }
    }
    if (graph) HIP_TRY(hipGraphLaunch(pl->uexec, st));
    else TRY(until_period(pl, st, test, every));
    HIP_TRY(hipEventRecord(pl->uev[i % ahead], st));
  }
  if (!seen_stop)
    for (int64_t k = 0; k < tail; ++k) TRY(one_iteration(pl, st, 0));
  mam::StopState hs{};
  HIP_TRY(hipMemcpyAsync(&hs, ss, sizeof(hs), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  out->converged = hs.stop != 0;
  out->checks = hs.checks;
  out->value = hs.value;
  out->iterations = hs.stop ? hs.checks * every : max_iters;
  pl->iters_done += out->iterations;
  // diagnostics stay valid when the last iteration run was a theta check
  pl->diag_valid = test == MAM_STOP_DTHETA && out->iterations > 0 && (hs.stop || (tail == 0 && periods > 0));
  return MAM_OK;
}

mam_status plan_iterate_until(Plan* pl, int64_t max_iters, int test, double tol, int64_t every,
                              mam_stop_result* out, hipStream_t st) {
  if (!out) return fail(MAM_EINVAL, "out is NULL");
  *out = mam_stop_result{0, 0, 0, (double)NAN};
  if (pl->batch) return fail(MAM_EUNSUPPORTED, "stopping tests run on single problems");
  if (!pl->inited) return fail(MAM_ESTATE, "mam_init has not run");
  if (max_iters < 0) return fail(MAM_EINVAL, "max_iters must be >= 0");
  if (every < 1) return fail(MAM_EINVAL, "check_every must be >= 1");
  if (test != MAM_STOP_DTHETA && test != MAM_STOP_DP && test != MAM_STOP_DIST)
    return fail(MAM_EINVAL, "unknown stopping test %d", test);
  if (std::isnan(tol)) return fail(MAM_EINVAL, "tol is NaN");
  if (test == MAM_STOP_DTHETA && pl->lg.on && pl->lg.sparse)
    return fail(MAM_EUNSUPPORTED, "the theta test is not available with the sparse store");
  pl->gate = at<int32_t>(pl, pl->lay.stop);  // StopState.stop is its first member
  const mam_status s = until_run(pl, max_iters, test, tol, every, st, out);
  pl->gate = nullptr;
  TRY(s);
  return sparse_writeback(pl, st);
}

mam_status plan_timing_read(Plan* pl, double* total_ms, int64_t* launches) {
  double tot = 0.0;
  for (size_t i = 0; i + 1 < pl->ev_used; i += 2) {
    HIP_TRY(hipEventSynchronize(pl->ev[i + 1]));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, pl->ev[i], pl->ev[i + 1]));
    tot += ms;
  }
  *total_ms = tot;
  *launches = (int64_t)(pl->ev_used / 2);
  pl->ev_used = 0;
  return MAM_OK;
}


// ---------------------------------------------------------------------------
// reverse mode
//
// mam_record runs K iterations from theta^0 = q/R, keeping theta at the
// start of every window of C iterations but the first (theta^0 is rebuilt
// from q) and the active-set masks of the last window.  mam_backward walks
// the windows from the last: it rebuilds a window's masks (restore its
// start, rerun its C iterations with recording) unless the ring holds them,
// then takes the window's reverse steps from its last iteration down.  The
// ring has C+1 slots (slot of iteration k = k mod (C+1)), so rerunning a
// window never overwrites the first mask of the window after it, which its
// last reverse step reads.
// ---------------------------------------------------------------------------
mam_status adjoint_layout(const Plan* pl, int64_t K, int64_t C, Adjoint* A) {
  if (pl->batch) return fail(MAM_EUNSUPPORTED, "the reverse mode is available for single problems");
  if (pl->lg.on) return fail(MAM_EUNSUPPORTED, "the reverse mode is not available for long columns");
  if (pl->P[0].flags & MAM_FLAG_RELAXED)
    return fail(MAM_EUNSUPPORTED, "the reverse mode is not available for relaxed measure constraints");
  if (K < 0) return fail(MAM_EINVAL, "iters must be >= 0");
  const Prob& p = pl->P[0];
  const Group& g = pl->G[0];
  A->K = K;
  A->C = (C <= 0 || C > K) ? std::max<int64_t>(K, 1) : C;
  A->nw = (K + A->C - 1) / A->C;
  A->mld = (int64_t)g.nt * (g.vpt <= 8 ? 1 : 2);
  A->ckpt_bytes = (size_t)p.ld * (size_t)p.T * elem_bytes(pl->dtype);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t a = o;
    o = align_up(o + std::max<size_t>(bytes, 1));
    return a;
  };
  const size_t R = (size_t)p.R, M = (size_t)p.M, T = (size_t)p.T;
  A->o_mask = take((size_t)(A->C + 1) * T * (size_t)A->mld);
  A->o_ckpt = take((size_t)std::max<int64_t>(A->nw - 1, 0) * A->ckpt_bytes);
  // the marginals of each checkpoint: the iteration's own (sums of the
  // unrounded updates), not the row sums of the stored plans
  A->o_ckpt_pm = take((size_t)std::max<int64_t>(A->nw - 1, 0) * (size_t)p.M * (size_t)p.R * 8);
  A->o_U = take(R * T * 8);
  A->o_cacc = take(R * T * 8);
  A->o_qacc = take(T * 8);
  A->o_V = take(M * R * 8);
  A->o_wold = take(M * R * 8);
  A->o_wacc = take(M * R * 8);
  A->o_mx = take(mam::kAdjSlots * 8);
  A->o_cptr = take((size_t)(p.cost_ncols + 1) * 8);
  A->o_clist = take(T * 4);
  A->unbal = !std::isinf(p.gamma);
  if (A->unbal) {
    const size_t slots = (size_t)(A->C + 1);
    A->o_pm_rec = take(slots * M * R * 8);
    A->o_p_rec = take(slots * R * 8);
    A->o_d2_rec = take(slots * (size_t)p.nb * 8);
    A->o_bbar = take(M * R * 8);
    A->o_tpart = take(((R + 255) / 256) * 8);
  }
  A->total = o;
  return MAM_OK;
}

uint8_t* mask_slot(Plan* pl, int64_t k) {
  Adjoint& A = pl->adj;
  return reinterpret_cast<uint8_t*>(A.ws + A.o_mask) + (size_t)(k % (A.C + 1)) * (size_t)pl->P[0].T * (size_t)A.mld;
}

template <typename T>
mam_status launch_copy(T* dst, const T* src, const Prob& p, hipStream_t st) {
  return launch_plan_copy<T>(dst, src, p, st);
}

// Iterations [k0, k1) with the masks of those at or after 'rec_from'
// recorded; theta is checkpointed at every window start k > 0 when 'ckpt'.
mam_status record_range(Plan* pl, int64_t k0, int64_t k1, int64_t rec_from, bool ckpt, hipStream_t st) {
  Adjoint& A = pl->adj;
  const Prob& p = pl->P[0];
  for (int64_t k = k0; k < k1; ++k) {
    if (ckpt && k > 0 && k % A.C == 0) {
      char* dst = A.ws + A.o_ckpt + (size_t)(k / A.C - 1) * A.ckpt_bytes;
      if (pl->dtype == MAM_F32)
        TRY(launch_copy<float>(reinterpret_cast<float*>(dst), static_cast<const float*>(p.theta), p, st));
      else
        TRY(launch_copy<double>(reinterpret_cast<double*>(dst), static_cast<const double*>(p.theta), p, st));
      const size_t MR = (size_t)p.M * (size_t)p.R;
      HIP_TRY(hipMemcpyAsync(A.ws + A.o_ckpt_pm + (size_t)(k / A.C - 1) * MR * 8, pl->ws + p.o_pm, MR * 8,
                             hipMemcpyDeviceToDevice, st));
    }
    if (A.unbal && k >= rec_from) {
      // the iteration's p^(m), p and d^2 partials, as its column kernel reads them
      const size_t sl = (size_t)(k % (A.C + 1));
      const size_t MR = (size_t)p.M * (size_t)p.R;
      HIP_TRY(hipMemcpyAsync(A.ws + A.o_pm_rec + sl * MR * 8, pl->ws + p.o_pm, MR * 8, hipMemcpyDeviceToDevice, st));
      HIP_TRY(hipMemcpyAsync(A.ws + A.o_p_rec + sl * (size_t)p.R * 8, pl->ws + p.o_p, (size_t)p.R * 8,
                             hipMemcpyDeviceToDevice, st));
      HIP_TRY(hipMemcpyAsync(A.ws + A.o_d2_rec + sl * (size_t)p.nb * 8, pl->ws + p.o_d2, (size_t)p.nb * 8,
                             hipMemcpyDeviceToDevice, st));
    }
    TRY(one_iteration(pl, st, 0, k >= rec_from ? mask_slot(pl, k) : nullptr, A.mld));
  }
  return MAM_OK;
}

mam_status plan_record(Plan* pl, int64_t K, int64_t C, void* ws, size_t bytes, hipStream_t st) {
  Adjoint A;
  TRY(adjoint_layout(pl, K, C, &A));
  const Prob& p = pl->P[0];
  if (!pl->inited) return fail(MAM_ESTATE, "mam_init has not run");
  if (!pl->default_start || pl->iters_done != 0)
    return fail(MAM_ESTATE, "mam_record needs a fresh mam_init with the default start (theta0 = NULL)");
  if (!ws) return fail(MAM_ENOMEM, "adjoint workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return fail(MAM_EINVAL, "adjoint workspace must be 256-byte aligned");
  if (bytes < A.total) return fail(MAM_ENOMEM, "adjoint workspace has %zu bytes, needs %zu", bytes, A.total);
  A.ws = static_cast<char*>(ws);
  A.bytes = bytes;
  // cost-column -> plan-column lists (increasing plan column)
  std::vector<int64_t> cptr(p.cost_ncols + 1, 0);
  std::vector<int32_t> clist(p.T);
  auto col_of = [&](int64_t j, int64_t m) -> int64_t {
    if (p.cost_mode == MAM_COST_INDEXED) return p.idx[j];
    if (p.cost_mode == MAM_COST_SHARED) return j - p.col_off[m];
    return j;
  };
  for (int64_t m = 0; m < p.M; ++m)
    for (int64_t j = p.col_off[m]; j < p.col_off[m + 1]; ++j) ++cptr[col_of(j, m) + 1];
  for (int64_t c = 0; c < p.cost_ncols; ++c) cptr[c + 1] += cptr[c];
  {
    std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
    for (int64_t m = 0; m < p.M; ++m)
      for (int64_t j = p.col_off[m]; j < p.col_off[m + 1]; ++j) clist[fill[col_of(j, m)]++] = (int32_t)j;
  }
  HIP_TRY(hipMemcpyAsync(A.ws + A.o_cptr, cptr.data(), cptr.size() * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(A.ws + A.o_clist, clist.data(), clist.size() * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  pl->adj = A;
  pl->adj.valid = false;
  TRY(record_range(pl, 0, K, (A.nw - 1) * A.C, true, st));
  pl->iters_done += K;
  pl->adj.resident = A.nw - 1;
  pl->adj.valid = true;
  return MAM_OK;
}

template <typename T>
mam_status backward_finish(Plan* pl, void* gq, void* gc, hipStream_t st) {
  Adjoint& A = pl->adj;
  const Prob& p = pl->P[0];
  hipLaunchKernelGGL(mam::grad_q_kernel<T>, dim3((unsigned)p.M), dim3(256), 0, st,
                     reinterpret_cast<const double*>(A.ws + A.o_V), reinterpret_cast<const double*>(A.ws + A.o_qacc),
                     at<int64_t>(pl, p.o_coloff), static_cast<T*>(gq), (int)p.R);
  LAUNCH_CHECK("grad_q_kernel");
  hipLaunchKernelGGL(mam::grad_cost_kernel<T>, dim3((unsigned)std::min<int64_t>(p.cost_ncols, 16384)), dim3(256), 0, st,
                     reinterpret_cast<const double*>(A.ws + A.o_cacc), reinterpret_cast<const int64_t*>(A.ws + A.o_cptr),
                     reinterpret_cast<const int32_t*>(A.ws + A.o_clist), p.cost_ncols, (int)p.R, 1.0 / p.rho,
                     static_cast<T*>(gc), p.cost_ld);
  LAUNCH_CHECK("grad_cost_kernel");
  return MAM_OK;
}

mam_status plan_backward(Plan* pl, const double* gp, void* gq, void* gc, hipStream_t st) {
  Adjoint& A = pl->adj;
  if (!A.valid) return fail(MAM_ESTATE, "mam_record has not run");
  if (!gp || !gq || !gc) return fail(MAM_EINVAL, "grad_p, grad_q and grad_cost must be non-NULL");
  const Prob& p = pl->P[0];
  const Group& g = pl->G[0];
  double* V = reinterpret_cast<double*>(A.ws + A.o_V);
  double* wold = reinterpret_cast<double*>(A.ws + A.o_wold);
  auto* wacc = reinterpret_cast<unsigned long long*>(A.ws + A.o_wacc);
  auto* mx = reinterpret_cast<unsigned long long*>(A.ws + A.o_mx);
  const int64_t MR = p.M * p.R;
  const unsigned mr_blocks = (unsigned)std::min<int64_t>(4096, (MR + 255) / 256);
  hipLaunchKernelGGL(mam::adjoint_reset_kernel, dim3(mr_blocks), dim3(256), 0, st, wacc, MR, mx);
  LAUNCH_CHECK("adjoint_reset_kernel");
  hipLaunchKernelGGL(mam::adjoint_start_kernel, dim3(mr_blocks), dim3(256), 0, st, gp, at<double>(pl, p.o_aw), V, wold,
                     (int)p.R, (int)p.M, mx);
  LAUNCH_CHECK("adjoint_start_kernel");
  const int64_t RT = p.R * p.T;
  hipLaunchKernelGGL(mam::fill_value_kernel, dim3((unsigned)std::min<int64_t>(8192, (RT + 255) / 256)), dim3(256), 0,
                     st, reinterpret_cast<double*>(A.ws + A.o_cacc), RT, 0.0);
  LAUNCH_CHECK("fill_value_kernel");
  hipLaunchKernelGGL(mam::fill_value_kernel, dim3((unsigned)std::min<int64_t>(4096, (p.T + 255) / 256)), dim3(256), 0,
                     st, reinterpret_cast<double*>(A.ws + A.o_qacc), p.T, 0.0);
  LAUNCH_CHECK("fill_value_kernel");

  // one wave per column, kAdjCols columns at a time; lane l reads mld/64
  // bytes of a column's mask
  const int lane_bytes = (int)(A.mld / 64);
  mam::AdjFn fn = mam::pick_adjoint(lane_bytes, kAdjCols);
  if (!fn || A.mld % 64) return fail(MAM_EUNSUPPORTED, "no reverse column kernel for %lld mask bytes per column",
                                     (long long)A.mld);
  double smax = 0.0;
  for (int64_t m = 0; m < p.M; ++m) smax = std::max(smax, (double)(p.col_off[m + 1] - p.col_off[m]));
  mam::AdjArgs a;
  a.mld = A.mld;
  a.col_off = at<int64_t>(pl, p.o_coloff);
  a.U = reinterpret_cast<double*>(A.ws + A.o_U);
  a.cacc = reinterpret_cast<double*>(A.ws + A.o_cacc);
  a.qacc = reinterpret_cast<double*>(A.ws + A.o_qacc);
  a.V = V;
  a.wacc = wacc;
  a.mx = mx;
  a.smax = smax;
  a.T = p.T;
  a.R = (int32_t)p.R;
  a.M = (int32_t)p.M;
  a.nt = g.nt;
  a.vs = g.vec == 4 ? 2 : (g.vec == 2 ? 1 : 0);
  a.wshift = g.vpt <= 8 ? 3 : 4;
  // one batch of columns per wave (measured faster than resident waves
  // looping over batches); the kernel loops only past 2^22 workgroups
  const int64_t nbatch = (p.T + kAdjCols - 1) / kAdjCols;
  const unsigned adj_blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((nbatch + 3) / 4, (int64_t)1 << 22));
  const unsigned nbr = (unsigned)((p.R + 255) / 256);
  int64_t step = 0;  // reverse steps taken: the bound slots rotate mod 3

  const bool timing = pl->timing;
  for (int64_t w = A.nw - 1; w >= 0; --w) {
    const int64_t k0 = w * A.C, k1 = std::min(A.K, k0 + A.C);
    if (A.resident != w) {
      // rebuild the window's masks from its start: theta^0 = q/R, or the
      // checkpoint's plans and marginals (then the thresholds start cold
      // and the average is formed again; the accumulators are zero between
      // iterations)
      if (w == 0) {
        const void* t0[1] = {nullptr};
        TRY(pl->dtype == MAM_F32 ? launch_init<float>(pl, t0, st) : launch_init<double>(pl, t0, st));
      } else {
        const char* src = A.ws + A.o_ckpt + (size_t)(w - 1) * A.ckpt_bytes;
        if (pl->dtype == MAM_F32)
          TRY(launch_copy<float>(static_cast<float*>(p.theta), reinterpret_cast<const float*>(src), p, st));
        else
          TRY(launch_copy<double>(static_cast<double*>(p.theta), reinterpret_cast<const double*>(src), p, st));
        const size_t MR = (size_t)p.M * (size_t)p.R;
        HIP_TRY(hipMemcpyAsync(pl->ws + p.o_pm, A.ws + A.o_ckpt_pm + (size_t)(w - 1) * MR * 8, MR * 8,
                               hipMemcpyDeviceToDevice, st));
        hipLaunchKernelGGL(mam::fill_value_kernel, dim3((unsigned)std::min<int64_t>(4096, (p.T + 255) / 256)),
                           dim3(256), 0, st, at<double>(pl, p.o_lam), p.T, (double)NAN);
        LAUNCH_CHECK("fill_value_kernel");
        TRY(launch_average(pl, st, 0));
      }
      pl->timing = false;
      const mam_status s = record_range(pl, k0, k1, k0, false, st);
      pl->timing = timing;
      TRY(s);
      A.resident = w;
    }
    for (int64_t k = k1 - 1; k >= k0; --k) {
      a.mk = mask_slot(pl, k);
      a.mk1 = k + 1 < A.K ? mask_slot(pl, k + 1) : nullptr;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (timing) {
        e0 = next_event(pl);
        e1 = next_event(pl);
        if (!e0 || !e1) return fail(MAM_EHIP, "hipEventCreate failed");
        HIP_TRY(hipEventRecord(e0, st));
      }
      a.slot = (int32_t)(step % 3);
      hipLaunchKernelGGL(fn, dim3(adj_blocks), dim3(256), 0, st, a);
      LAUNCH_CHECK("adjoint_kernel");
      if (timing) HIP_TRY(hipEventRecord(e1, st));
      if (!A.unbal) {
        hipLaunchKernelGGL(mam::adjoint_average_kernel, dim3(nbr), dim3(256), 0, st, wacc, wold, V,
                           at<double>(pl, p.o_Sd), at<double>(pl, p.o_aw), (int)p.R, (int)p.M, mx, a.slot, smax);
        LAUNCH_CHECK("adjoint_average_kernel");
      } else {
        const size_t sl = (size_t)(k % (A.C + 1));
        const size_t MRs = (size_t)p.M * (size_t)p.R;
        const double* pmk = reinterpret_cast<const double*>(A.ws + A.o_pm_rec) + sl * MRs;
        const double* pk = reinterpret_cast<const double*>(A.ws + A.o_p_rec) + sl * (size_t)p.R;
        const double* d2k = reinterpret_cast<const double*>(A.ws + A.o_d2_rec) + sl * (size_t)p.nb;
        double* bbar = reinterpret_cast<double*>(A.ws + A.o_bbar);
        double* tpart = reinterpret_cast<double*>(A.ws + A.o_tpart);
        hipLaunchKernelGGL(mam::adjoint_unbal1_kernel, dim3(nbr), dim3(256), 0, st, wacc, wold, V,
                           at<double>(pl, p.o_Sd), pmk, pk, bbar, tpart, (int)p.R, (int)p.M, mx, a.slot, smax);
        LAUNCH_CHECK("adjoint_unbal1_kernel");
        hipLaunchKernelGGL(mam::adjoint_unbal2_kernel, dim3(nbr), dim3(256), 0, st, bbar, V, pmk, pk, d2k, p.nb,
                           tpart, (int)nbr, at<double>(pl, p.o_Sd), at<double>(pl, p.o_aw), p.rho, p.gamma, (int)p.R,
                           (int)p.M, mx, a.slot);
        LAUNCH_CHECK("adjoint_unbal2_kernel");
      }
      ++step;
    }
  }
  TRY(pl->dtype == MAM_F32 ? backward_finish<float>(pl, gq, gc, st) : backward_finish<double>(pl, gq, gc, st));
  // the plans now hold an intermediate iterate
  pl->inited = false;
  return MAM_OK;
}


// ---------------------------------------------------------------------------
// randomized variant (bundles)
// ---------------------------------------------------------------------------
// Per bundle: workgroups take equal runs of the bundle's columns (its
// measures' column ranges, in measure order), split at measure boundaries.
struct BundleHost {
  std::vector<int32_t> seg_p, seg_m, wg_seg, seg_st;
  std::vector<int64_t> seg_j0, seg_j1;
  std::vector<mam::MargTask> mtasks;
};

mam_status bundle_check(const Plan* pl, const int32_t* bundle_of, int32_t nb) {
  if (pl->batch) return fail(MAM_EUNSUPPORTED, "bundles are available for single problems");
  if (!bundle_of) return fail(MAM_EINVAL, "bundle_of is NULL");
  const Prob& p = pl->P[0];
  if (nb < 1 || nb > p.M) return fail(MAM_EINVAL, "nb must be in [1, M] (got %d)", nb);
  std::vector<int> cnt(nb, 0);
  for (int64_t m = 0; m < p.M; ++m) {
    if (bundle_of[m] < 0 || bundle_of[m] >= nb)
      return fail(MAM_EINVAL, "bundle_of[%lld] = %d is outside [0, %d)", (long long)m, bundle_of[m], nb);
    ++cnt[bundle_of[m]];
  }
  for (int i = 0; i < nb; ++i)
    if (!cnt[i]) return fail(MAM_EINVAL, "bundle %d has no measure", i);
  return MAM_OK;
}

void bundle_build(const Plan* pl, const int32_t* bundle_of, int bi, BundleHost* h, int* nwg_out) {
  const Prob& p = pl->P[0];
  const Group& g = pl->G[0];
  std::vector<int64_t> ms;
  int64_t Tb = 0;
  for (int64_t m = 0; m < p.M; ++m)
    if (bundle_of[m] == bi) {
      ms.push_back(m);
      Tb += p.S[m];
    }
  const int nwg = default_nwg(Tb, g.ng, g.nwg_req, g.nwg_auto);
  // the bundle's columns as a list of (measure, first, end) runs
  std::vector<int64_t> starts(ms.size() + 1, 0);
  for (size_t i = 0; i < ms.size(); ++i) starts[i + 1] = starts[i] + p.S[ms[i]];
  for (int w = 0; w < nwg; ++w) {
    h->wg_seg.push_back((int32_t)h->seg_m.size());
    int64_t lo = Tb * w / nwg, hi = Tb * (w + 1) / nwg;
    while (lo < hi) {
      const size_t i = std::upper_bound(starts.begin(), starts.end(), lo) - starts.begin() - 1;
      const int64_t m = ms[i];
      const int64_t e = std::min(hi, starts[i + 1]);
      h->seg_p.push_back(0);
      h->seg_m.push_back((int32_t)m);
      h->seg_j0.push_back(p.col_off[m] + (lo - starts[i]));
      h->seg_j1.push_back(p.col_off[m] + (e - starts[i]));
      h->seg_st.push_back(g.ng * group_block(g));  // contiguous: the groups of one workgroup in turn
      lo = e;
    }
  }
  h->wg_seg.push_back((int32_t)h->seg_m.size());
  for (int64_t m : ms)
    for (int64_t r0 = 0; r0 < p.R; r0 += 256) h->mtasks.push_back({0, (int32_t)m, (int32_t)r0, (int32_t)m});
  *nwg_out = nwg;
}

// Bytes of the bundle workspace, and the offsets of every bundle's tables.
size_t bundle_layout(const Plan* pl, const int32_t* bundle_of, int32_t nb, Bundles* out) {
  const Prob& p = pl->P[0];
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t a = o;
    o = align_up(o + std::max<size_t>(bytes, 1));
    return a;
  };
  Bundles B;
  B.nb = nb;
  B.b.resize(nb);
  for (int i = 0; i < nb; ++i) {
    BundleHost h;
    int nwg = 0;
    bundle_build(pl, bundle_of, i, &h, &nwg);
    BundleSched& bs = B.b[i];
    bs.nwg = nwg;
    bs.nseg = h.seg_m.size();
    bs.nmtasks = h.mtasks.size();
    bs.o_seg_p = take(bs.nseg * 4);
    bs.o_seg_m = take(bs.nseg * 4);
    bs.o_seg_j0 = take(bs.nseg * 8);
    bs.o_seg_j1 = take(bs.nseg * 8);
    bs.o_seg_st = take(bs.nseg * 4);
    bs.o_wg_seg = take(((size_t)nwg + 1) * 4);
    bs.o_mtasks = take(bs.nmtasks * sizeof(mam::MargTask));
  }
  if (out) *out = B;
  return o;
}

mam_status plan_set_bundles(Plan* pl, const int32_t* bundle_of, int32_t nb, void* ws, size_t bytes, hipStream_t st) {
  if (pl->lg.on) return fail(MAM_EUNSUPPORTED, "the randomized variant is not available for long columns");
  TRY(bundle_check(pl, bundle_of, nb));
  if (!pl->inited) return fail(MAM_ESTATE, "mam_init has not run");
  if (!ws) return fail(MAM_ENOMEM, "bundle workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return fail(MAM_EINVAL, "bundle workspace must be 256-byte aligned");
  Bundles B;
  const size_t need = bundle_layout(pl, bundle_of, nb, &B);
  if (bytes < need) return fail(MAM_ENOMEM, "bundle workspace has %zu bytes, needs %zu", bytes, need);
  B.ws = static_cast<char*>(ws);
  for (int i = 0; i < nb; ++i) {
    BundleHost h;
    int nwg = 0;
    bundle_build(pl, bundle_of, i, &h, &nwg);
    const BundleSched& bs = B.b[i];
    auto put = [&](size_t off, const void* src, size_t n) -> mam_status {
      if (n) HIP_TRY(hipMemcpyAsync(B.ws + off, src, n, hipMemcpyHostToDevice, st));
      return MAM_OK;
    };
    TRY(put(bs.o_seg_p, h.seg_p.data(), h.seg_p.size() * 4));
    TRY(put(bs.o_seg_m, h.seg_m.data(), h.seg_m.size() * 4));
    TRY(put(bs.o_seg_j0, h.seg_j0.data(), h.seg_j0.size() * 8));
    TRY(put(bs.o_seg_j1, h.seg_j1.data(), h.seg_j1.size() * 8));
    TRY(put(bs.o_seg_st, h.seg_st.data(), h.seg_st.size() * 4));
    TRY(put(bs.o_wg_seg, h.wg_seg.data(), h.wg_seg.size() * 4));
    TRY(put(bs.o_mtasks, h.mtasks.data(), h.mtasks.size() * sizeof(mam::MargTask)));
    HIP_TRY(hipStreamSynchronize(st));  // host staging is released at the end of this loop body
  }
  pl->bund = B;
  return MAM_OK;
}

template <typename T>
mam_status launch_bundle_columns(Plan* pl, const BundleSched& bs, hipStream_t st) {
  const Layout& L = pl->lay;
  const Group& g = pl->G[0];
  char* bw = pl->bund.ws;
  mam::ColArgs<T> a;
  a.probs = at<mam::ProbDev<T>>(pl, L.probdev);
  a.seg_p = reinterpret_cast<const int32_t*>(bw + bs.o_seg_p);
  a.seg_m = reinterpret_cast<const int32_t*>(bw + bs.o_seg_m);
  a.seg_j0 = reinterpret_cast<const int64_t*>(bw + bs.o_seg_j0);
  a.seg_j1 = reinterpret_cast<const int64_t*>(bw + bs.o_seg_j1);
  a.seg_st = reinterpret_cast<const int32_t*>(bw + bs.o_seg_st);
  a.wg_seg = reinterpret_cast<const int32_t*>(bw + bs.o_wg_seg);
  a.diag = at<double>(pl, L.diag);
  a.rec = nullptr;
  a.rec_ld = 0;
  a.stop = nullptr;
  a.nwg = bs.nwg;
  a.xcd_remap = 0;
  a.kb = group_block(g);
  const int kc = g.vec == 1 ? 1 : g.kc;
  mam::ColFn<T> fn = mam::pick_column<T>(g.nt, g.vpt, g.vec, kc, 0, g.stream);
  if (!fn) return fail(MAM_EUNSUPPORTED, "no column kernel for nt=%d vpt=%d vec=%d kc=%d", g.nt, g.vpt, g.vec, kc);
  const int wgsize = g.nt <= 64 ? 256 : g.nt;
  const size_t shmem = (size_t)g.vpt * g.nt * 8 * (1 + g.ng);
  if (shmem > 65536)
    HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)shmem));
  hipLaunchKernelGGL(fn, dim3(bs.nwg), dim3(wgsize), shmem, st, a);
  LAUNCH_CHECK("column_kernel");
  return MAM_OK;
}

mam_status plan_iterate_bundles(Plan* pl, int64_t iters, const int32_t* seq, hipStream_t st) {
  if (iters < 0) return fail(MAM_EINVAL, "iters must be >= 0");
  if (!pl->inited) return fail(MAM_ESTATE, "mam_init has not run");
  if (!pl->bund.nb) return fail(MAM_ESTATE, "mam_set_bundles has not run");
  if (iters > 0 && !seq) return fail(MAM_EINVAL, "seq is NULL");
  for (int64_t k = 0; k < iters; ++k)
    if (seq[k] < 0 || seq[k] >= pl->bund.nb)
      return fail(MAM_EINVAL, "seq[%lld] = %d is not a bundle", (long long)k, seq[k]);
  const Layout& L = pl->lay;
  for (int64_t k = 0; k < iters; ++k) {
    const BundleSched& bs = pl->bund.b[seq[k]];
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (pl->timing) {
      e0 = next_event(pl);
      e1 = next_event(pl);
      if (!e0 || !e1) return fail(MAM_EHIP, "hipEventCreate failed");
      HIP_TRY(hipEventRecord(e0, st));
    }
    TRY(pl->dtype == MAM_F32 ? launch_bundle_columns<float>(pl, bs, st) : launch_bundle_columns<double>(pl, bs, st));
    if (pl->timing) HIP_TRY(hipEventRecord(e1, st));
    // new marginals of the bundle's measures only, then the average of all
    hipLaunchKernelGGL(mam::fixed_marginal_kernel, dim3((unsigned)bs.nmtasks), dim3(256), 0, st,
                       reinterpret_cast<const mam::MargTask*>(pl->bund.ws + bs.o_mtasks),
                       at<mam::ProbAux>(pl, L.probaux), 0, nullptr);
    LAUNCH_CHECK("fixed_marginal_kernel");
    hipLaunchKernelGGL(mam::average_kernel, dim3((unsigned)pl->atasks.size()), dim3(256), 0, st,
                       at<mam::AvgTask>(pl, L.atasks), at<mam::ProbAux>(pl, L.probaux), 0, nullptr);
    LAUNCH_CHECK("average_kernel");
  }
  pl->iters_done += iters;
  pl->diag_valid = false;
  return MAM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Support step (Prop. 4): chunks of at most C columns of one measure, enough
// of them for about 8192 workgroups of the partial pass; the workspace holds
// the chunk tables and the partials.
// ---------------------------------------------------------------------------
struct SupportLayout {
  int64_t C = 0;
  int nchunks = 0;
  size_t o_m = 0, o_j0 = 0, o_j1 = 0, o_al = 0, o_part = 0, total = 0;
};

SupportLayout support_layout(const Prob& p, int dim) {
  SupportLayout L;
  const int64_t row_blocks = (p.R + mam::SUP_NT - 1) / mam::SUP_NT;
  const int64_t want = std::max<int64_t>(p.M, (8192 + row_blocks - 1) / row_blocks);
  L.C = std::max<int64_t>(64, (p.T + want - 1) / want);
  int64_t n = 0;
  for (int64_t m = 0; m < p.M; ++m) n += (p.S[m] + L.C - 1) / L.C;
  L.nchunks = (int)n;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.o_m = take(n * 4);
  L.o_j0 = take(n * 8);
  L.o_j1 = take(n * 8);
  L.o_al = take(n * 8);
  L.o_part = take((size_t)n * (dim + 1) * p.R * 8);
  L.total = off;
  return L;
}

template <typename T>
mam_status launch_support(Plan* pl, const SupportLayout& L, char* ws, int dim, const double* zeta, double* xi,
                          double* mass, hipStream_t st) {
  const Prob& p = pl->P[0];
  mam::SupArgs<T> a;
  a.theta = static_cast<const T*>(p.theta);
  a.ld = p.ld;
  a.R = p.R;
  a.dim = dim;
  a.nchunks = L.nchunks;
  a.ch_m = reinterpret_cast<const int32_t*>(ws + L.o_m);
  a.ch_j0 = reinterpret_cast<const int64_t*>(ws + L.o_j0);
  a.ch_j1 = reinterpret_cast<const int64_t*>(ws + L.o_j1);
  a.alpha = reinterpret_cast<const double*>(ws + L.o_al);
  a.zeta = zeta;
  a.p_prev = at<double>(pl, p.o_p_prev);
  a.pm_prev = at<double>(pl, p.o_pm_prev);
  a.Sd = at<double>(pl, p.o_Sd);
  a.t = at<double>(pl, p.o_t);
  a.partial = reinterpret_cast<double*>(ws + L.o_part);
  a.xi = xi;
  a.mass = mass;
  // a 16-byte vector of rows per thread when ld and theta allow it
  constexpr int V = 16 / sizeof(T);
  const bool vec = p.ld % V == 0 && reinterpret_cast<uintptr_t>(p.theta) % 16 == 0;
  const int64_t rows_per_block = (int64_t)mam::SUP_NT * (vec ? V : 1);
  const dim3 grid((unsigned)((p.R + rows_per_block - 1) / rows_per_block), (unsigned)L.nchunks);
  if (vec) hipLaunchKernelGGL((mam::support_partial_kernel<T, V>), grid, dim3(mam::SUP_NT), 0, st, a);
  else hipLaunchKernelGGL((mam::support_partial_kernel<T, 1>), grid, dim3(mam::SUP_NT), 0, st, a);
  LAUNCH_CHECK("support_partial_kernel");
  hipLaunchKernelGGL(mam::support_final_kernel<T>, dim3((unsigned)((p.R + 255) / 256)), dim3(256), 0, st, a);
  LAUNCH_CHECK("support_final_kernel");
  return MAM_OK;
}

mam_status plan_support_update(Plan* pl, const double* alpha, const double* zeta, int dim, double* xi,
                               double* mass, void* ws, size_t bytes, hipStream_t st) {
  if (pl->batch) return fail(MAM_EUNSUPPORTED, "the support step is for single problems");
  if (!pl->inited) return fail(MAM_ESTATE, "mam_init has not run");
  if (!alpha || !zeta || !xi) return fail(MAM_EINVAL, "NULL argument");
  if (dim < 1 || dim > mam::SUP_MAXD) return fail(MAM_EINVAL, "dim must be in [1, %d] (got %d)", mam::SUP_MAXD, dim);
  const Prob& p = pl->P[0];
  for (int64_t m = 0; m < p.M; ++m)
    if (!(alpha[m] >= 0.0) || !std::isfinite(alpha[m]))
      return fail(MAM_EINVAL, "alpha[%lld] must be finite and >= 0", (long long)m);
  const SupportLayout L = support_layout(p, dim);
  if (!ws) return fail(MAM_ENOMEM, "support workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return fail(MAM_EINVAL, "support workspace must be 256-byte aligned");
  if (bytes < L.total) return fail(MAM_ENOMEM, "support workspace has %zu bytes, needs %zu", bytes, L.total);
  // one more iteration, keeping the marginals it starts from: its plans
  // pi_hat = theta' + b are the ones the support step uses
  TRY(one_iteration(pl, st, 0, nullptr, 0, 1));
  pl->iters_done += 1;
  TRY(sparse_writeback(pl, st));
  std::vector<int32_t> cm;
  std::vector<int64_t> cj0, cj1;
  std::vector<double> cal;
  for (int64_t m = 0; m < p.M; ++m) {
    for (int64_t s0 = 0; s0 < p.S[m]; s0 += L.C) {
      cm.push_back((int32_t)m);
      cj0.push_back(p.col_off[m] + s0);
      cj1.push_back(p.col_off[m] + std::min<int64_t>(s0 + L.C, p.S[m]));
      cal.push_back(alpha[m]);
    }
  }
  char* w = static_cast<char*>(ws);
  HIP_TRY(hipMemcpyAsync(w + L.o_m, cm.data(), cm.size() * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(w + L.o_j0, cj0.data(), cj0.size() * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(w + L.o_j1, cj1.data(), cj1.size() * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(w + L.o_al, cal.data(), cal.size() * 8, hipMemcpyHostToDevice, st));
  // the tables come from pageable vectors freed when this call returns: the
  // copies must have read them first
  HIP_TRY(hipStreamSynchronize(st));
  return pl->dtype == MAM_F32 ? launch_support<float>(pl, L, w, dim, zeta, xi, mass, st)
                              : launch_support<double>(pl, L, w, dim, zeta, xi, mass, st);
}

// ---------------------------------------------------------------------------
// Workspace of mam_solve_static: a file-scope device array, one copy per GPU
// the library runs on, held until the process ends.  Its name in host code
// stands for the symbol, not a device address: the address is looked up
// once per device with hipGetSymbolAddress (with that device current) and
// only that pointer is ever handed to kernels or copies.
// ---------------------------------------------------------------------------
constexpr size_t kStaticScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

mam_status static_scratch(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(MAM_EUNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(MAM_EHIP, "hipGetSymbolAddress of the static workspace failed on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return MAM_OK;
}

struct mam_problem {
  Plan plan;
};

struct mam_batch {
  Plan plan;
};

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
  mam_problem* p = new (std::nothrow) mam_problem();
  if (!p) return fail(MAM_ENOMEM, "host allocation failed");
  mam_status st = make_plan(&p->plan, d, 1);
  if (st != MAM_OK) {
    delete p;
    return st;
  }
  *out = p;
  return MAM_OK;
}

mam_status mam_set_schedule(mam_problem* p, const mam_schedule* s) {
  if (!p || !s) return fail(MAM_EINVAL, "NULL argument");
  return set_group_schedule(&p->plan, 0, s);
}

mam_status mam_get_schedule(const mam_problem* p, mam_schedule* s) {
  if (!p || !s) return fail(MAM_EINVAL, "NULL argument");
  get_group_schedule(&p->plan, 0, s);
  return MAM_OK;
}

size_t mam_workspace_bytes(const mam_problem* p) { return p ? p->plan.lay.total : 0; }

mam_status mam_set_workspace(mam_problem* p, void* dev, size_t bytes) {
  if (!p) return fail(MAM_EINVAL, "NULL handle");
  return set_workspace(&p->plan, dev, bytes);
}

mam_status mam_bind(mam_problem* p, void* theta, const void* cost, const int32_t* cost_col_index, const void* q) {
  if (!p) return fail(MAM_EINVAL, "NULL handle");
  return bind(&p->plan, 0, theta, cost, cost_col_index, q);
}

mam_status mam_init(mam_problem* p, const void* theta0, void* stream) {
  if (!p) return fail(MAM_EINVAL, "NULL handle");
  const void* t0[1] = {theta0};
  return plan_init(&p->plan, t0, static_cast<hipStream_t>(stream));
}

mam_status mam_iterate(mam_problem* p, int64_t iters, void* stream) {
  if (!p) return fail(MAM_EINVAL, "NULL handle");
  return plan_iterate(&p->plan, iters, static_cast<hipStream_t>(stream));
}

mam_status mam_set_grid(mam_problem* p, int32_t dim, const int64_t* n, const double* origin, const double* spacing) {
  if (!p || !n || !origin || !spacing) return fail(MAM_EINVAL, "NULL argument");
  Prob& pr = p->plan.P[0];
  if (pr.cost_mode != MAM_COST_GRID) return fail(MAM_EINVAL, "cost_mode is not MAM_COST_GRID");
  if (dim != 1 && dim != 2) return fail(MAM_EINVAL, "dim must be 1 or 2 (got %d)", dim);
  int64_t npts = 1;
  for (int k = 0; k < dim; ++k) {
    if (n[k] < 1) return fail(MAM_EINVAL, "n[%d] must be >= 1", k);
    if (!std::isfinite(origin[k]) || !std::isfinite(spacing[k]))
      return fail(MAM_EINVAL, "origin and spacing must be finite");
    npts *= n[k];
  }
  if (npts != pr.R) return fail(MAM_EINVAL, "the grid has %lld points but R = %lld", (long long)npts, (long long)pr.R);
  pr.gdim = dim;
  for (int k = 0; k < 2; ++k) {
    pr.gn[k] = k < dim ? n[k] : 1;
    pr.go[k] = k < dim ? origin[k] : 0.0;
    pr.gh[k] = k < dim ? spacing[k] : 0.0;
  }
  p->plan.inited = false;
  drop_graphs(&p->plan);
  return MAM_OK;
}

mam_status mam_iterate_until(mam_problem* p, int64_t max_iters, int32_t test, double tol, int64_t check_every,
                             mam_stop_result* out, void* stream) {
  if (!p) return fail(MAM_EINVAL, "NULL handle");
  return plan_iterate_until(&p->plan, max_iters, test, tol, check_every, out, static_cast<hipStream_t>(stream));
}

mam_status mam_graph(mam_problem* p, int64_t iters_per_launch) {
  if (!p) return fail(MAM_EINVAL, "NULL handle");
  return plan_graph(&p->plan, iters_per_launch);
}

mam_status mam_barycenter(mam_problem* p, double* p_dev, void* stream) {
  if (!p || !p_dev) return fail(MAM_EINVAL, "NULL argument");
  if (!p->plan.inited) return fail(MAM_ESTATE, "mam_init has not run");
  const Prob& pr = p->plan.P[0];
  HIP_TRY(hipMemcpyAsync(p_dev, p->plan.ws + pr.o_p, pr.R * 8, hipMemcpyDeviceToDevice,
                         static_cast<hipStream_t>(stream)));
  return MAM_OK;
}

mam_status mam_barycenter_host(mam_problem* p, double* p_host, void* stream) {
  if (!p || !p_host) return fail(MAM_EINVAL, "NULL argument");
  if (!p->plan.inited) return fail(MAM_ESTATE, "mam_init has not run");
  const Prob& pr = p->plan.P[0];
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipMemcpyAsync(p_host, p->plan.ws + pr.o_p, pr.R * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return MAM_OK;
}

mam_status mam_marginals(mam_problem* p, double* pm_dev, void* stream) {
  if (!p || !pm_dev) return fail(MAM_EINVAL, "NULL argument");
  if (!p->plan.inited) return fail(MAM_ESTATE, "mam_init has not run");
  const Prob& pr = p->plan.P[0];
  HIP_TRY(hipMemcpyAsync(pm_dev, p->plan.ws + pr.o_pm, pr.M * pr.R * 8, hipMemcpyDeviceToDevice,
                         static_cast<hipStream_t>(stream)));
  return MAM_OK;
}

mam_status mam_diagnostics(mam_problem* p, mam_diag* out, void* stream) {
  if (!p || !out) return fail(MAM_EINVAL, "NULL argument");
  Plan* pl = &p->plan;
  if (!pl->inited || !pl->diag_valid) return fail(MAM_ESTATE, "no iteration ran with MAM_FLAG_DIAG");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Prob& pr = pl->P[0];
  const size_t R = pr.R, M = pr.M;
  const bool lg = pl->lg.on;
  const int nslots = lg ? pl->lg.nwg : pl->nwg_total;
  std::vector<double> pm(M * R), pmp(M * R), pv(R), pp(R), dg((size_t)nslots * mam::DIAG_STRIDE);
  std::vector<double> cd(lg ? (size_t)pr.T * 4 : 0);
  double t = 0.0;
  HIP_TRY(hipMemcpyAsync(pm.data(), pl->ws + pr.o_pm, M * R * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(pmp.data(), pl->ws + pr.o_pm_prev, M * R * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(pv.data(), pl->ws + pr.o_p, R * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(pp.data(), pl->ws + pr.o_p_prev, R * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(dg.data(), pl->ws + (lg ? pl->lg.o_wdiag : pl->lay.diag), dg.size() * 8,
                         hipMemcpyDeviceToHost, st));
  if (lg) HIP_TRY(hipMemcpyAsync(cd.data(), pl->ws + pl->lg.o_ldiag, cd.size() * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&t, pl->ws + pr.o_t, 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  mam_diag r{};
  r.iterations = pl->iters_done;
  r.t = t;
  double rounds = 0.0, active = 0.0, cols = 0.0;
  if (lg) {
    // long columns: per-column figures of the threshold kernel (summed in
    // column order), and the write workgroups' maxima of the change (NaN
    // with the sparse store, which keeps no dense copy of the old plans)
    for (int64_t j = 0; j < pr.T; ++j) {
      const double* o = &cd[(size_t)j * 4];
      r.W_hat += o[0];
      r.meas_resid = std::max(r.meas_resid, o[1]);
      rounds += o[2];
      active += o[3];
    }
    cols = (double)pr.T;
    if (pl->lg.sparse) {
      r.dtheta_inf = NAN;
    } else {
      for (int w = 0; w < nslots; ++w) r.dtheta_inf = std::max(r.dtheta_inf, dg[(size_t)w * mam::DIAG_STRIDE + 2]);
    }
  } else {
    for (int w = 0; w < nslots; ++w) {
      const double* o = &dg[(size_t)w * mam::DIAG_STRIDE];
      r.W_hat += o[0];
      r.meas_resid = std::max(r.meas_resid, o[1]);
      r.dtheta_inf = std::max(r.dtheta_inf, o[2]);
      rounds += o[3];
      active += o[4];
      cols += o[5];
    }
  }
  r.rounds_per_column = cols > 0 ? rounds / cols : 0.0;
  r.active_per_column = cols > 0 ? active / cols : 0.0;
  // row sums of pi_hat^(m) = p^(m),new + t (p_old - p^(m),old)
  std::vector<double> ph(M * R), phbar(R, 0.0);
  for (size_t m = 0; m < M; ++m)
    for (size_t i = 0; i < R; ++i) ph[m * R + i] = pm[m * R + i] + t * (pp[i] - pmp[m * R + i]);
  for (size_t m = 0; m < M; ++m)
    for (size_t i = 0; i < R; ++i) phbar[i] += pr.aw[m] * ph[m * R + i];
  double d2 = 0.0;
  for (size_t m = 0; m < M; ++m) {
    double s = 0.0;
    for (size_t i = 0; i < R; ++i) {
      const double e = phbar[i] - ph[m * R + i];
      s += e * e;
    }
    d2 += s / pr.Sd[m];
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
  p->plan.timing = enable != 0;
  p->plan.ev_used = 0;
  return MAM_OK;
}

mam_status mam_timing_read(mam_problem* p, double* total_ms, int64_t* launches) {
  if (!p || !total_ms || !launches) return fail(MAM_EINVAL, "NULL argument");
  return plan_timing_read(&p->plan, total_ms, launches);
}

// ---- reverse mode ----------------------------------------------------------
size_t mam_adjoint_workspace_bytes(const mam_problem* p, int64_t iters, int64_t ckpt_every) {
  if (!p) return 0;
  Adjoint A;
  if (adjoint_layout(&p->plan, iters, ckpt_every, &A) != MAM_OK) return 0;
  return A.total;
}

mam_status mam_record(mam_problem* p, int64_t iters, int64_t ckpt_every, void* adj_ws, size_t bytes,
                      void* stream) {
  if (!p) return fail(MAM_EINVAL, "NULL handle");
  return plan_record(&p->plan, iters, ckpt_every, adj_ws, bytes, static_cast<hipStream_t>(stream));
}

mam_status mam_backward(mam_problem* p, const double* grad_p, void* grad_q, void* grad_cost, void* stream) {
  if (!p) return fail(MAM_EINVAL, "NULL handle");
  return plan_backward(&p->plan, grad_p, grad_q, grad_cost, static_cast<hipStream_t>(stream));
}

// ---- randomized variant ----------------------------------------------------
size_t mam_support_workspace_bytes(const mam_problem* p, int32_t dim) {
  if (!p || p->plan.P.empty() || dim < 1 || dim > mam::SUP_MAXD) return 0;
  return support_layout(p->plan.P[0], dim).total;
}

mam_status mam_support_update(mam_problem* p, const double* alpha, const double* zeta, int32_t dim, double* xi,
                              double* mass, void* ws, size_t bytes, void* stream) {
  if (!p) return fail(MAM_EINVAL, "NULL handle");
  return plan_support_update(&p->plan, alpha, zeta, dim, xi, mass, ws, bytes, static_cast<hipStream_t>(stream));
}

size_t mam_bundle_workspace_bytes(const mam_problem* p, const int32_t* bundle_of, int32_t nb) {
  if (!p || p->plan.lg.on || bundle_check(&p->plan, bundle_of, nb) != MAM_OK) return 0;
  return bundle_layout(&p->plan, bundle_of, nb, nullptr);
}

mam_status mam_set_bundles(mam_problem* p, const int32_t* bundle_of, int32_t nb, void* bundle_ws, size_t bytes,
                           void* stream) {
  if (!p) return fail(MAM_EINVAL, "NULL handle");
  return plan_set_bundles(&p->plan, bundle_of, nb, bundle_ws, bytes, static_cast<hipStream_t>(stream));
}

mam_status mam_iterate_bundles(mam_problem* p, int64_t iters, const int32_t* seq, void* stream) {
  if (!p) return fail(MAM_EINVAL, "NULL handle");
  return plan_iterate_bundles(&p->plan, iters, seq, static_cast<hipStream_t>(stream));
}

void mam_destroy(mam_problem* p) { delete p; }

mam_status mam_stream_copy(void* dst, const void* src, size_t bytes, int32_t workgroups, void* stream) {
  if (!dst || !src) return fail(MAM_EINVAL, "NULL buffer");
  if (bytes % 16 || reinterpret_cast<uintptr_t>(dst) % 16 || reinterpret_cast<uintptr_t>(src) % 16)
    return fail(MAM_EINVAL, "buffers and size must be multiples of 16 bytes");
  if (workgroups < 1) return fail(MAM_EINVAL, "workgroups must be >= 1");
  if (bytes == 0) return MAM_OK;
  hipLaunchKernelGGL(mam::stream_copy_kernel, dim3(workgroups), dim3(256), 0, static_cast<hipStream_t>(stream),
                     static_cast<const mam::f4nt*>(src), static_cast<mam::f4nt*>(dst), (int64_t)(bytes / 16));
  LAUNCH_CHECK("stream_copy_kernel");
  return MAM_OK;
}

mam_status mam_solve_static(const mam_desc* d, void* theta, const void* cost, const int32_t* cost_col_index,
                            const void* q, const void* theta0, int64_t iters, double* p_out, void* stream) {
  if (!d || !theta || !cost || !q || !p_out) return fail(MAM_EINVAL, "NULL argument");
  if (iters < 0) return fail(MAM_EINVAL, "iters must be >= 0");
  if (d->cost_mode == MAM_COST_GRID) return fail(MAM_EUNSUPPORTED, "a grid cost needs mam_set_grid: use a handle");
  mam_problem* raw = nullptr;
  TRY(mam_create(&raw, d));
  // the handle lives for this call only; the kernels queued on 'stream'
  // read only the caller's buffers and the static workspace, which outlive it
  std::unique_ptr<mam_problem, void (*)(mam_problem*)> h(raw, mam_destroy);
  const size_t need = mam_workspace_bytes(h.get());
  if (need > kStaticScratchBytes)
    return fail(MAM_ENOMEM, "this problem needs %zu bytes of workspace; the static workspace holds %zu",
                need, kStaticScratchBytes);
  void* ws = nullptr;
  TRY(static_scratch(&ws));
  TRY(mam_set_workspace(h.get(), ws, need));
  TRY(mam_bind(h.get(), theta, cost, cost_col_index, q));
  TRY(mam_init(h.get(), theta0, stream));
  TRY(mam_iterate(h.get(), iters, stream));
  return mam_barycenter(h.get(), p_out, stream);
}

// ---- batches ---------------------------------------------------------------
mam_status mam_batch_create(mam_batch** out, const mam_desc* descs, int32_t n) {
  if (!out) return fail(MAM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!descs) return fail(MAM_EINVAL, "descs is NULL");
  mam_batch* b = new (std::nothrow) mam_batch();
  if (!b) return fail(MAM_ENOMEM, "host allocation failed");
  b->plan.batch = true;
  mam_status st = make_plan(&b->plan, descs, n);
  if (st != MAM_OK) {
    delete b;
    return st;
  }
  *out = b;
  return MAM_OK;
}

int32_t mam_batch_groups(const mam_batch* b) { return b ? (int32_t)b->plan.G.size() : 0; }

int32_t mam_batch_group_of(const mam_batch* b, int32_t i) {
  if (!b || i < 0 || i >= (int32_t)b->plan.P.size()) return -1;
  return b->plan.P[i].group;
}

mam_status mam_batch_set_schedule(mam_batch* b, int32_t group, const mam_schedule* s) {
  if (!b || !s) return fail(MAM_EINVAL, "NULL argument");
  if (group < 0 || group >= (int32_t)b->plan.G.size()) return fail(MAM_EINVAL, "no group %d", group);
  return set_group_schedule(&b->plan, group, s);
}

mam_status mam_batch_get_schedule(const mam_batch* b, int32_t group, mam_schedule* s) {
  if (!b || !s) return fail(MAM_EINVAL, "NULL argument");
  if (group < 0 || group >= (int32_t)b->plan.G.size()) return fail(MAM_EINVAL, "no group %d", group);
  get_group_schedule(&b->plan, group, s);
  return MAM_OK;
}

size_t mam_batch_workspace_bytes(const mam_batch* b) { return b ? b->plan.lay.total : 0; }

mam_status mam_batch_set_workspace(mam_batch* b, void* dev, size_t bytes) {
  if (!b) return fail(MAM_EINVAL, "NULL handle");
  return set_workspace(&b->plan, dev, bytes);
}

mam_status mam_batch_bind(mam_batch* b, int32_t i, void* theta, const void* cost, const int32_t* cost_col_index,
                          const void* q) {
  if (!b) return fail(MAM_EINVAL, "NULL handle");
  if (i < 0 || i >= (int32_t)b->plan.P.size()) return fail(MAM_EINVAL, "no problem %d", i);
  return bind(&b->plan, i, theta, cost, cost_col_index, q);
}

mam_status mam_batch_init(mam_batch* b, void* stream) {
  if (!b) return fail(MAM_EINVAL, "NULL handle");
  return plan_init(&b->plan, nullptr, static_cast<hipStream_t>(stream));
}

mam_status mam_batch_iterate(mam_batch* b, int64_t iters, void* stream) {
  if (!b) return fail(MAM_EINVAL, "NULL handle");
  return plan_iterate(&b->plan, iters, static_cast<hipStream_t>(stream));
}

mam_status mam_batch_graph(mam_batch* b, int64_t iters_per_launch) {
  if (!b) return fail(MAM_EINVAL, "NULL handle");
  return plan_graph(&b->plan, iters_per_launch);
}

mam_status mam_batch_barycenter(mam_batch* b, int32_t i, double* p_dev, void* stream) {
  if (!b || !p_dev) return fail(MAM_EINVAL, "NULL argument");
  if (i < 0 || i >= (int32_t)b->plan.P.size()) return fail(MAM_EINVAL, "no problem %d", i);
  if (!b->plan.inited) return fail(MAM_ESTATE, "mam_batch_init has not run");
  const Prob& pr = b->plan.P[i];
  HIP_TRY(hipMemcpyAsync(p_dev, b->plan.ws + pr.o_p, pr.R * 8, hipMemcpyDeviceToDevice,
                         static_cast<hipStream_t>(stream)));
  return MAM_OK;
}

mam_status mam_batch_timing_enable(mam_batch* b, int32_t enable) {
  if (!b) return fail(MAM_EINVAL, "NULL handle");
  b->plan.timing = enable != 0;
  b->plan.ev_used = 0;
  return MAM_OK;
}

mam_status mam_batch_timing_read(mam_batch* b, double* total_ms, int64_t* launches) {
  if (!b || !total_ms || !launches) return fail(MAM_EINVAL, "NULL argument");
  return plan_timing_read(&b->plan, total_ms, launches);
}

void mam_batch_destroy(mam_batch* b) { delete b; }

// ---- cost helper -----------------------------------------------------------
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

// Device code of the MAM column kernel for gfx950 (CDNA4, wave64).
//
// One Douglas-Rachford iteration of Alg. 1 is three launches:
//
//   column kernel  : per plan column, fuses the broadcast correction and the
//                    reflection (w = theta + 2b - c/rho, Alg. 1 Step 2 and
//                    Prop. 2 eq. (row_sol)), the exact projection onto
//                    Delta_R(q_s) (Prop. 3) and the update theta' = pi_hat - b.
//                    The row sums of theta' (Step 3) are -S^m b plus the row
//                    sums of pi_hat, which is nonzero only at the active
//                    entries: each active entry's pi_hat is rounded to a
//                    64-bit fixed-point integer, each thread sums its rows'
//                    integers over a segment's columns and adds the sums to
//                    the marginal's accumulator.
//                    It streams theta once in and once out and reads each
//                    cost column once: HBM bound.
//   marginal kernel: p^(m)_r = (fixed-point sum) - S^m b^(m)_r.
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
// (2-3 from this cold start) with the same lambda as the sort-based formula,
// up to summation order.  Started from the column's threshold of the previous
// iteration, one pass usually both moves to and certifies the root.  The
// column stays in registers (held as w in double) for all passes; each pass
// is one compare/select/add per value plus a group reduction, and a wave none
// of whose values lies above the current threshold (most waves, since active
// sets are small) settles its part of a pass with one compare of each lane's
// largest w.
//
// Fixed-point row sums.  Every entry is rounded on its own and integer
// addition is associative, so the sums depend neither on the order in which
// columns finish nor on how the columns are split into segments: results are
// bitwise reproducible run to run and equal for every workgroup count,
// column order, team size, XCD mapping and number of columns in flight, with
// no floating-point atomics.  (The threshold's own sums follow the lanes'
// rows, so another thread shape can move them by a rounding.)  Measure m
// uses the scale 2^E_m with mass_m <= 2^(62 - E_m) (mass_m = sum_s q_s);
// every pi_hat row sum is at most mass_m, so no sum overflows 2^63, and each
// entry is rounded to the nearest multiple of 2^-E_m (a relative 2^-63 of
// the mass).  All other reductions have a fixed order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "mam.h"

namespace mam {

// f(integral_constant<int, 0>{}), ..., f(integral_constant<int, N - 1>{}):
// a loop over buffers whose index stays a compile-time constant.
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

template <typename T> struct VecOf;
template <> struct VecOf<float>  { static constexpr int N = 4; using type = float4; };
template <> struct VecOf<double> { static constexpr int N = 2; using type = double2; };

// Non-temporal forms for the plans: the stream of theta passes through the
// caches without displacing the cost columns that are reused.
typedef float f4nt __attribute__((ext_vector_type(4)));
typedef double d2nt __attribute__((ext_vector_type(2)));

template <typename T, int VEC>
__device__ __forceinline__ void load_vec_nt(const T* __restrict__ src, T (&v)[VEC]) {
  if constexpr (VEC == 1) {
    v[0] = __builtin_nontemporal_load(src);
  } else if constexpr (sizeof(T) == 4) {
    const f4nt x = __builtin_nontemporal_load(reinterpret_cast<const f4nt*>(src));
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
  } else {
    const d2nt x = __builtin_nontemporal_load(reinterpret_cast<const d2nt*>(src));
    v[0] = x.x; v[1] = x.y;
  }
}

template <typename T, int VEC>
__device__ __forceinline__ void store_vec_nt(T* __restrict__ dst, const T (&v)[VEC]) {
  if constexpr (VEC == 1) {
    __builtin_nontemporal_store(v[0], dst);
  } else if constexpr (sizeof(T) == 4) {
    f4nt x = {v[0], v[1], v[2], v[3]};
    __builtin_nontemporal_store(x, reinterpret_cast<f4nt*>(dst));
  } else {
    d2nt x = {v[0], v[1]};
    __builtin_nontemporal_store(x, reinterpret_cast<d2nt*>(dst));
  }
}

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

// ---------------------------------------------------------------------------
// Wave reductions with DPP (data-parallel primitives): butterfly steps inside
// rows of 16 lanes, then row broadcasts; the total lands in lane 63 and is
// read back as a wave-uniform scalar.  Fixed order: bitwise reproducible.
// ---------------------------------------------------------------------------
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_move(double v, double identity) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(identity), __double2loint(v), CTRL, ROWMASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(identity), __double2hiint(v), CTRL, ROWMASK, 0xf, false);
  return __hiloint2double(hi, lo);
}

struct OpSum {
  static constexpr double id() { return 0.0; }
  __device__ static double f(double a, double b) { return a + b; }
};
struct OpMax {
  static constexpr double id() { return -__builtin_huge_val(); }
  __device__ static double f(double a, double b) { return fmax(a, b); }
};
struct OpMin {
  static constexpr double id() { return __builtin_huge_val(); }
  __device__ static double f(double a, double b) { return fmin(a, b); }
};

__device__ __forceinline__ double read_lane63(double v) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_move_f(float v, float identity) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(identity), __float_as_int(v), CTRL, ROWMASK, 0xf, false));
}

struct OpMaxF {
  static constexpr float id() { return -__builtin_huge_valf(); }
  __device__ static float f(float a, float b) { return fmaxf(a, b); }
};
struct OpMinF {
  static constexpr float id() { return __builtin_huge_valf(); }
  __device__ static float f(float a, float b) { return fminf(a, b); }
};

template <class Op>
__device__ __forceinline__ float wave_reduce_f(float v) {
  v = Op::f(v, dpp_move_f<0xb1, 0xf>(v, Op::id()));
  v = Op::f(v, dpp_move_f<0x4e, 0xf>(v, Op::id()));
  v = Op::f(v, dpp_move_f<0x141, 0xf>(v, Op::id()));
  v = Op::f(v, dpp_move_f<0x140, 0xf>(v, Op::id()));
  v = Op::f(v, dpp_move_f<0x142, 0xa>(v, Op::id()));
  v = Op::f(v, dpp_move_f<0x143, 0xc>(v, Op::id()));
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ double uniform_d(double v) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float uniform_f(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform_l(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

template <class Op>
__device__ __forceinline__ double wave_reduce(double v) {
  v = Op::f(v, dpp_move<0xb1, 0xf>(v, Op::id()));   // quad_perm [1,0,3,2]
  v = Op::f(v, dpp_move<0x4e, 0xf>(v, Op::id()));   // quad_perm [2,3,0,1]
  v = Op::f(v, dpp_move<0x141, 0xf>(v, Op::id()));  // row_half_mirror
  v = Op::f(v, dpp_move<0x140, 0xf>(v, Op::id()));  // row_mirror
  v = Op::f(v, dpp_move<0x142, 0xa>(v, Op::id()));  // row_bcast:15 into rows 1, 3
  v = Op::f(v, dpp_move<0x143, 0xc>(v, Op::id()));  // row_bcast:31 into rows 2, 3
  return read_lane63(v);
}

// Pointers read from device tables are generic to the compiler, which then
// emits flat memory instructions; those also count against the LDS wait
// counter and so serialise LDS traffic behind HBM loads.  Every buffer the
// kernels touch through a table is global memory: the cast says so.
template <typename T>
__device__ __forceinline__ T* gptr(T* p) {
  const uint64_t bits = (uint64_t)p;
  return (T*)(__attribute__((address_space(1))) T*)bits;
}

__device__ __forceinline__ double wave_sum(double v) { return wave_reduce<OpSum>(v); }
__device__ __forceinline__ double wave_max(double v) { return wave_reduce<OpMax>(v); }

// t^k of Alg. 1 (Step 1) from the nb <= 64 partial sums of
// d^2 = sum_m ||p - p^(m)||^2 / S^m: every wave sums them in a fixed order
// (one partial per lane), so t is wave-uniform without LDS, and every kernel
// that needs t forms the same value.
__device__ __forceinline__ double damping_t(const double* d2part, int nb, double rho, double gam, int lane) {
  double d2 = lane < nb ? d2part[lane] : 0.0;
  d2 = wave_reduce<OpSum>(d2);
  return (__builtin_isinf(gam) || rho * sqrt(d2) <= gam) ? 1.0 : gam / (rho * sqrt(d2));
}

// The nearest float to x and its neighbours: float_up(x) >= x and
// float_down(x) <= x (the float conversion rounds to nearest; one step in the
// last place fixes the side), NaN for NaN.  The bounds of the threshold
// certificate need only the side, not the exact directed rounding.
__device__ __forceinline__ float float_up(double x) {
  const float f = (float)x;
  const int b = __float_as_int(f);
  return (double)f < x ? __int_as_float(f >= 0.0f ? b + 1 : b - 1) : f;
}
__device__ __forceinline__ float float_down(double x) {
  const float f = (float)x;
  const int b = __float_as_int(f);
  return (double)f > x ? __int_as_float(f > 0.0f ? b - 1 : (f == 0.0f ? (int)0x80000001 : b + 1)) : f;
}

// max(a, b) of two results of arithmetic, which are never signaling NaNs:
// the bare instruction (it returns the other operand for a quiet NaN, as
// fmax does).  fmax itself first quiets each operand the compiler cannot
// prove is the result of arithmetic, one more instruction per call.
__device__ __forceinline__ double max_arith(double a, double b) {
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// Fixed-point value of pi_hat >= 0 at scale fx = 2^E (round to nearest).
__device__ __forceinline__ unsigned long long to_fixed(double ph, double fx) {
  return __double2ull_rn(ph * fx);
}

// One problem as the marginal and average kernels see it.
struct ProbAux {
  double* pm;        // M x R
  double* pm_prev;   // M x R, marginals before the last iteration (diagnostics)
  double* p;         // R
  double* p_prev;    // R
  double* d2part;    // ceil(R/256) partial sums of d^2
  const double* aw;  // averaging weights a_m
  const double* Sd;  // S^m as double
  int32_t R, M;
  int32_t mbase;     // index of (this problem, measure 0) in the measure list
  int32_t nb;        // d^2 partials
  unsigned long long* acc;  // M x R fixed-point row sums of pi_hat (short columns)
  const double* fxinv;      // M inverse scales 2^-E_m of those sums
  double rho, gamma;
  const double* t;          // t^k of the iteration, as its column kernel formed it
};

struct MargTask {
  int32_t prob, m, r0;
  int32_t list;  // partial-offset list: the measure's, or (long columns) its row tile's
};

struct AvgTask {
  int32_t prob, rb;
};

// Short columns, Step 3: p^(m)_r = sum_s theta'_rs = sum_s pi_hat_rs - S^m b^(m)_r,
// with the pi_hat sum from the column kernel's fixed-point accumulator and
// b^(m)_r = t (p_r - p^(m)_r) / S^m formed from the marginals and the t^k
// the column kernel used (same inputs, same operations).  The accumulator
// is cleared for the next iteration.  Row tk.r0 + tidx; a whole wave calls
// it (t is a wave reduction).
__device__ __forceinline__ void close_marginal(const MargTask& tk, const ProbAux& P, int save_prev, int tidx) {
  const int R = uniform_i(P.R);
  const int r = tk.r0 + tidx;
  const double t = damping_t(gptr(P.d2part), uniform_i(P.nb), uniform_d(P.rho), uniform_d(P.gamma), tidx & 63);
  if (r >= R) return;
  const size_t o = (size_t)tk.m * R + r;
  double* const pm = gptr(P.pm);
  unsigned long long* const acc = gptr(P.acc);
  const double Sm = gptr(P.Sd)[tk.m];
  const double old = pm[o];
  const double b = t * (gptr(P.p)[r] - old) / Sm;
  const double s = (double)acc[o] * gptr(P.fxinv)[tk.m] - Sm * b;
  acc[o] = 0ull;
  if (save_prev) gptr(P.pm_prev)[o] = old;
  pm[o] = s;
}

// p_r = sum_m a_m p^(m)_r, and the block's partial sum of
// sum_r sum_m (p_r - p^(m)_r)^2 / S^m.
// Called by all 256 threads of a workgroup (tidx = thread index; sh: four
// doubles of LDS).
__device__ __forceinline__ void close_average(const AvgTask& tk, const ProbAux& P, int save_prev, int tidx,
                                              double* sh) {
  const int R = P.R, M = P.M;
  const int r = tk.rb * 256 + tidx;
  const double* const pm = gptr(P.pm);
  const double* const aw = gptr(P.aw);
  const double* const Sd = gptr(P.Sd);
  double* const p = gptr(P.p);
  double d2 = 0.0;
  if (r < R) {
    // eight measures' loads in flight at a time; the sums keep the order m = 0, 1, ...
    constexpr int U = 8;
    double pr = 0.0;
    for (int m0 = 0; m0 < M; m0 += U) {
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = m0 + u < M ? pm[(size_t)(m0 + u) * R + r] : 0.0;
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (m0 + u < M) pr += aw[m0 + u] * v[u];
    }
    for (int m0 = 0; m0 < M; m0 += U) {
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = m0 + u < M ? pm[(size_t)(m0 + u) * R + r] : 0.0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (m0 + u < M) {
          const double e = pr - v[u];
          d2 += e * e / Sd[m0 + u];
        }
      }
    }
    if (save_prev) gptr(P.p_prev)[r] = p[r];
    p[r] = pr;
  }
  d2 = wave_sum(d2);
  if ((tidx & 63) == 0) sh[tidx >> 6] = d2;
  __syncthreads();
  if (tidx == 0) gptr(P.d2part)[tk.rb] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// Short columns, Steps 3 and 1 of one block of 256 rows, fused: both are
// row-parallel.  Row r's new marginals are
//   p^(m)_r = sum_s pi_hat_rs - S^m b^(m)_r,  b^(m)_r = t (p_r - p^(m)_r) / S^m
// (the pi_hat sum from the column kernel's fixed-point accumulator, which is
// cleared; t as the column kernel formed it; p and p^(m) of the iterate,
// each read by this thread alone before it overwrites them), then
// p_r = sum_m a_m p^(m)_r and the block's partial sum of
// sum_r sum_m (p_r - p^(m)_r)^2 / S^m.  Called by all 256 threads of a
// workgroup (tidx = thread index; sh: four doubles of LDS).
__device__ __forceinline__ void close_rows(const AvgTask& tk, const ProbAux& P, int save_prev, int tidx,
                                           double* sh) {
  const int R = uniform_i(P.R), M = uniform_i(P.M);
  const int r = tk.rb * 256 + tidx;
  const double t = uniform_d(*gptr(P.t));
  double* const pm = gptr(P.pm);
  unsigned long long* const acc = gptr(P.acc);
  const double* const aw = gptr(P.aw);
  const double* const Sd = gptr(P.Sd);
  const double* const fxinv = gptr(P.fxinv);
  double* const p = gptr(P.p);
  double d2 = 0.0;
  if (r < R) {
    const double pold = p[r];
    double pr = 0.0;
    constexpr int U = 8;  // eight measures' loads in flight; sums in the order m = 0, 1, ...
    for (int m0 = 0; m0 < M; m0 += U) {
      double old[U];
      unsigned long long ac[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const size_t o = (size_t)(m0 + u) * R + r;
        old[u] = m0 + u < M ? pm[o] : 0.0;
        ac[u] = m0 + u < M ? acc[o] : 0ull;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (m0 + u < M) {
          const int m = m0 + u;
          const size_t o = (size_t)m * R + r;
          const double Sm = Sd[m];
          const double b = t * (pold - old[u]) / Sm;
          const double v = (double)ac[u] * fxinv[m] - Sm * b;
          acc[o] = 0ull;
          if (save_prev) gptr(P.pm_prev)[o] = old[u];
          pm[o] = v;
          pr += aw[m] * v;
        }
      }
    }
    for (int m0 = 0; m0 < M; m0 += U) {
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = m0 + u < M ? pm[(size_t)(m0 + u) * R + r] : 0.0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (m0 + u < M) {
          const double e = pr - v[u];
          d2 += e * e / Sd[m0 + u];
        }
      }
    }
    if (save_prev) gptr(P.p_prev)[r] = pold;
    p[r] = pr;
  }
  d2 = wave_reduce<OpSum>(d2);
  if ((tidx & 63) == 0) sh[tidx >> 6] = d2;
  __syncthreads();
  if (tidx == 0) gptr(P.d2part)[tk.rb] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// One problem as the column kernel sees it (a batch holds many).
template <typename T>
struct ProbDev {
  T* theta;
  const T* cost;
  const T* q;
  const int32_t* cidx;
  unsigned long long* acc;  // M x R fixed-point sums of pi_hat (zero between iterations)
  const double* fx;         // M scales 2^E_m of the fixed-point sums
  int64_t ld, cost_ld;
  int32_t R, cost_mode;
  int32_t nb, warm;       // nb: d^2 partials; warm: use stored thresholds as starts
  int32_t relaxed, pad;   // relaxed: columns projected onto {u >= 0, sum u <= q_s}
  double rho, inv_rho, gamma;
  const double* pm;       // M x R marginals of the current plans
  const double* p;        // R, averaged marginal
  const double* d2part;   // nb partial sums of d^2
  double* lam;            // T thresholds of the last projection (NaN = none)
  double* t_out;          // 1
  const int64_t* col_off; // M+1
  const double* Sd;       // S^m as double
};

template <typename T>
struct ColArgs {
  const ProbDev<T>* probs;
  const int32_t* seg_p;   // problem of each segment
  const int32_t* seg_m;   // measure of each segment
  const int64_t* seg_j0;  // first column
  const int64_t* seg_j1;  // one past the last column
  const int32_t* seg_st;  // column stride between the segment's blocks
  const int32_t* wg_seg;  // segments of workgroup w: [wg_seg[w], wg_seg[w+1])
  double* diag;           // nwg x DIAG_STRIDE (single-problem plans)
  uint8_t* rec;           // null, or: per column j, the threads' active-set
                          // mask words at rec + j*rec_ld (single-problem plans)
  int64_t rec_ld;
  const int32_t* stop;    // null, or a flag: nonzero once a stopping test
                          // held, and then the launch does nothing
  int32_t nwg, xcd_remap;
  int32_t kb;             // columns a group takes at a time (a block): with
                          // several groups per workgroup the schedule's
                          // columns in flight (1, 2 or 4), with one group
                          // kOneGroupBlock; every instance walking the
                          // tables has KC dividing it
};

// The block of a workgroup that is one column group.  Its columns are
// consecutive whatever the block, and a block of 4 (every KC divides it)
// keeps the step arithmetic in compile-time constants.
constexpr int kOneGroupBlock = 4;

constexpr int DIAG_STRIDE = 8;  // W_hat, meas_resid, dtheta_inf, rounds, active, columns

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

// Active-set mask word of one thread (bit k = slot k): 8 or 16 bits.
template <int VPT> struct MaskWord { using type = uint16_t; };
template <> struct MaskWord<1> { using type = uint8_t; };
template <> struct MaskWord<2> { using type = uint8_t; };
template <> struct MaskWord<4> { using type = uint8_t; };
template <> struct MaskWord<8> { using type = uint8_t; };

template <int NT> struct GroupShape {
  // a 64-thread group is one wave: four of them share a workgroup;
  // larger groups are the whole workgroup
  static constexpr int NG = NT == 64 ? 4 : 1;
  static constexpr int WG = NT * NG;
};

// One threshold round for KC columns: per column, over the entries of w,
//   S = sum of w > lam (double), n = #{w > lam},
//   mnA = min of w > lam rounded down to float,
//   mxN = max of w <= lam rounded up to float,
//   wmx = max of w in double, on cold rounds (lam = NaN) only,
// reduced over the column group (NW waves) in a fixed order.  The float
// bounds are conservative (mnA <= true min, mxN >= true max), so a test
// passed on them holds for the exact values; they cost a third of a double
// reduction.
template <int NW, int KC>
struct Rounds {
  double* red_d;  // [2][KC][2][NW]
  float* red_f;   // [2][KC][2][NW]
  int* red_i;     // [2][KC][NW]
  int par;

  __device__ __forceinline__ void reduce(double (&S)[KC], float (&mnA)[KC], float (&mxN)[KC],
                                         double (&wmx)[KC], int (&n)[KC], const bool (&act)[KC],
                                         const bool (&cold)[KC], int wv, int lane) {
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      if (act[kc]) {
        if (n[kc] != 0) {  // wave-uniform: some lane of this wave is active
          S[kc] = wave_reduce<OpSum>(S[kc]);
          mnA[kc] = wave_reduce_f<OpMinF>(mnA[kc]);
        } else {
          S[kc] = 0.0;
          mnA[kc] = __builtin_huge_valf();
        }
        mxN[kc] = wave_reduce_f<OpMaxF>(mxN[kc]);
        if (cold[kc]) wmx[kc] = wave_reduce<OpMax>(wmx[kc]);
      }
    }
    if constexpr (NW > 1) {
      if (lane == 0) {
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
          red_d[((par * KC + kc) * 2 + 0) * NW + wv] = S[kc];
          red_d[((par * KC + kc) * 2 + 1) * NW + wv] = wmx[kc];
          red_f[((par * KC + kc) * 2 + 0) * NW + wv] = mnA[kc];
          red_f[((par * KC + kc) * 2 + 1) * NW + wv] = mxN[kc];
          red_i[(par * KC + kc) * NW + wv] = n[kc];
        }
      }
      __syncthreads();
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) {
        const double* d = red_d + ((par * KC + kc) * 2 + 0) * NW;
        const double* d1 = red_d + ((par * KC + kc) * 2 + 1) * NW;
        const float* f0 = red_f + ((par * KC + kc) * 2 + 0) * NW;
        const float* f1 = red_f + ((par * KC + kc) * 2 + 1) * NW;
        const int* ni = red_i + (par * KC + kc) * NW;
        double sum = d[0], mx = d1[0];
        float a = f0[0], b = f1[0];
        int nn = ni[0];
#pragma unroll
        for (int i = 1; i < NW; ++i) {
          sum += d[i];
          mx = fmax(mx, d1[i]);
          a = fminf(a, f0[i]);
          b = fmaxf(b, f1[i]);
          nn += ni[i];
        }
        S[kc] = uniform_d(sum);
        wmx[kc] = uniform_d(mx);
        mnA[kc] = uniform_f(a);
        mxN[kc] = uniform_f(b);
        n[kc] = __builtin_amdgcn_readfirstlane(nn);
      }
      par ^= 1;
    }
  }
};

// Column kernel.  Workgroup = NG groups of NT threads; a group advances KC
// columns of one segment at a time.  Thread tid of a group holds rows
// (c*NT + tid)*VEC + v (c < VPT/VEC, v < VEC) of each of its KC columns.
//
// Inactive entries.  An entry with w_r <= lambda has pi_hat_r = 0, so its
// update is theta'_r = -b_r whatever theta and c were: every column of a
// segment is the constant vector -b^(m) except at its active rows.  The
// kernel therefore keeps no per-entry state beyond the raw theta and c of
// the columns in flight: each column writes -b^(m) patched at its active
// rows, and the marginal's row sums are -S^m b^(m) plus the patches' values
// pi_hat (taken before the update is rounded to the storage type), which
// the active entries add to a fixed-point accumulator.
//
// Threshold of a column (tau = q_s > 0): Newton steps
//   lam' = (sum_{w > lam} w - tau) / #{w > lam}
// from the column's threshold of the previous iteration (warm start) or,
// without one, from w_max - tau (a lower bound, since one entry carries at
// most tau).  A step from any start lands at or below the root (the tangent
// of a convex decreasing function meets zero before it does); from there the
// steps increase monotonically and the active set shrinks.  The set A used
// for lam' is exact when it did not change (the level sets are nested, so
// equal counts mean equal sets) or when min_A w >= lam' >= max_{not A} w;
// then lam' is the root itself, so one round usually both moves and
// verifies.  Entries equal to lam' contribute 0 either way.
//
// Loads ahead.  Everything a column step needs (raw theta and c, q_s, the
// stored threshold, and for an indexed cost the cost column number one step
// earlier still) is requested PF steps before the step runs, so no load
// waits inside a step.  STREAM instances load and store theta with the
// non-temporal policy (plans larger than the Infinity Cache).
//
// Dynamic LDS: VPT*NT doubles of b^(m) (with one group per workgroup each
// thread reads and writes only its own slots), then NG*VPT*NT doubles of
// row sums of pi_hat, one block per group (own slots per thread).
// Waves per SIMD the register allocation must allow: five while a thread
// holds at most 16 bytes of a column step, four up to 32, else two.
// Without the bound the compiler spends registers freely and the smaller
// shapes lose a resident wave.
template <typename T, int VPT, int KC>
constexpr int col_waves() { return sizeof(T) * VPT * KC <= 16 ? 5 : (sizeof(T) * VPT * KC <= 32 ? 4 : 2); }

template <typename T, int NT, int VPT, int VEC, int KC, bool DIAG, bool STREAM = false>
__global__ void __launch_bounds__(GroupShape<NT>::WG, (col_waves<T, VPT, KC>()))
column_kernel(ColArgs<T> a) {
  constexpr int WG = GroupShape<NT>::WG;
  constexpr int NG = GroupShape<NT>::NG;  // independent column groups per workgroup
  constexpr int NW = NT / 64;             // waves per group
  constexpr int NCH = VPT / VEC;          // vector chunks per thread
  static_assert(VPT % VEC == 0, "VPT must be a multiple of VEC");
  static_assert(VPT <= 32, "the active mask is one 32-bit word");
  static_assert(NG == 1 || NW == 1, "multi-wave groups fill the workgroup");
  // column steps whose raw loads are in flight at once: two for float plans
  // with vector loads and at most 512 threads per group, where the extra
  // buffer still fits the register budget without spills (not with the
  // diagnostics' extra state, which would halve the occupancy)
  constexpr int PF = (sizeof(T) == 4 && KC == 1 && VEC > 1 && NT <= 512 && !DIAG) ? 2 : 1;

  __shared__ double red_d[NW > 1 ? 2 * KC * 2 * NW : 1];
  __shared__ float red_f[NW > 1 ? 2 * KC * 2 * NW : 1];
  __shared__ int red_i[NW > 1 ? 2 * KC * NW : 1];
  __shared__ double sh_diag[WG / 64][6];
  extern __shared__ double lds_dyn[];
  double* lds_b = lds_dyn;                // [VPT][NT]
  unsigned long long* lds_fix = reinterpret_cast<unsigned long long*>(lds_dyn + VPT * NT);  // [NG][VPT][NT]

  const int gtid = threadIdx.x;
  // the group index is wave-uniform (a group is one wave, or the whole
  // workgroup); saying so keeps all column bookkeeping in scalar registers
  const int g = NG == 1 ? 0 : __builtin_amdgcn_readfirstlane(gtid / NT);
  const int tid = gtid % NT;
  const int lane = gtid & 63;
  const int wv = NW == 1 ? 0 : __builtin_amdgcn_readfirstlane(tid >> 6);
  // this group's fixed-point row sums of pi_hat, own slots per thread
  unsigned long long* const fix = lds_fix + (size_t)g * VPT * NT;

  const int wg = logical_block(blockIdx.x, gridDim.x, a.xcd_remap);
  // The stop flag and this workgroup's segment range are requested together,
  // so the early exit adds no memory latency in front of the first segment.
  // Table entries are read through vector loads (the compiler cannot prove
  // them constant); readfirstlane makes them scalar again.
  const int stopv = a.stop != nullptr ? *gptr(a.stop) : 0;
  const int sb0 = a.wg_seg[wg], se0 = a.wg_seg[wg + 1];
  if (uniform_i(stopv) != 0) return;  // early exit: the run has stopped
  const int sb = uniform_i(sb0), se = uniform_i(se0);

  Rounds<NW, KC> rounds{red_d, red_f, red_i, 0};
  double dW = 0.0, dRes = 0.0, dTh = 0.0, dRounds = 0.0, dAct = 0.0, dCols = 0.0;
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
    const int64_t stride = uniform_i(a.seg_st[si]);  // columns from one block of the group to its next
    const double Sm = uniform_d(gptr(P.Sd)[m]);
    unsigned long long* const accm = gptr((unsigned long long*)uniform_l((int64_t)P.acc)) + (size_t)m * R;
    const double fxm = uniform_d(gptr(P.fx)[m]);
    const int64_t off_m = uniform_l(gptr(P.col_off)[m]);
    const double* __restrict__ pmm = gptr(P.pm) + (size_t)m * R;
    const double* __restrict__ pv = gptr(P.p);

    // Column steps of this group: blocks of kb columns taken in turn by the
    // NG groups (and, with a segment stride beyond NG*kb, by the other
    // workgroups of a team sweeping the same columns), each walked KC
    // columns at a time.  With kb = KC a group takes one step's columns and
    // the groups of a workgroup share a segment's columns to within one
    // step.  The raw loads of the next step are issued before the current
    // step's threshold rounds and stores, so their HBM latency overlaps that
    // work.
    const int kb = NG == 1 ? kOneGroupBlock : uniform_i(a.kb);
    const int sps = __builtin_ctz(kb / KC);  // log2 of the steps per block
    const int64_t gbase = j0 + (int64_t)g * kb;
    auto step_exists = [&](int64_t i) -> bool { return gbase + (i >> sps) * stride < j1; };
    auto step_col = [&](int64_t i, int kc, int64_t& j) -> bool {
      const int64_t base = gbase + (i >> sps) * stride;
      const int64_t bend = base + kb < j1 ? base + kb : j1;
      j = base + (i & ((1 << sps) - 1)) * KC + kc;
      return j < bend;
    };
    auto cost_col = [&](int64_t j) -> const T* {
      int64_t cc;
      if (cost_mode == MAM_COST_INDEXED) cc = uniform_i(cidx[j]);
      else if (cost_mode == MAM_COST_SHARED) cc = j - off_m;
      else cc = j;
      return cost + cc * cost_ld;
    };
    // raw theta and cost of the next PF steps, one buffer per step in flight,
    // with each column's weight q_s and stored threshold (the warm start).
    // Loads are unconditional: a column slot past the segment's end loads
    // the segment's first column and is ignored.  (Conditional loads into
    // the rotating buffers made the compiler copy whole buffers per step.)
    T rt[PF][KC][VPT], rc[PF][KC][VPT], rq[PF][KC];
    double rl[PF][KC];
    auto step_col_clamped = [&](int64_t i, int kc) -> int64_t {
      int64_t j;
      return step_col(i, kc, j) ? j : j0;
    };
    // an indexed cost's column numbers are read one issued step ahead, so
    // forming a cost address never waits on memory
    int32_t cnext[KC];
    auto load_index = [&](int64_t i) {
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) cnext[kc] = cidx[step_col_clamped(i, kc)];
    };
    if (cost_mode == MAM_COST_INDEXED) load_index(0);
    auto issue = [&](int64_t i, T (&bt)[KC][VPT], T (&bc)[KC][VPT], T (&bq)[KC], double (&bl)[KC]) {
      int32_t cthis[KC];
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) cthis[kc] = cnext[kc];
      if (cost_mode == MAM_COST_INDEXED) load_index(i + 1);
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) {
        const int64_t j = step_col_clamped(i, kc);
        bq[kc] = qv[j];
        bl[kc] = lamv[j];
        const T* __restrict__ thp = theta + j * ld;
        int64_t cc;
        if (cost_mode == MAM_COST_INDEXED) cc = uniform_i(cthis[kc]);
        else if (cost_mode == MAM_COST_SHARED) cc = j - off_m;
        else cc = j;
        const T* __restrict__ cp = cost + cc * cost_ld;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          // rows past R read the column's first vector (in bounds); their
          // b = -inf makes them inactive whatever they hold
          const int r0 = (c * NT + tid) * VEC < R ? (c * NT + tid) * VEC : 0;
          T tv[VEC], cv[VEC];
          if constexpr (STREAM) load_vec_nt<T, VEC>(thp + r0, tv);
          else load_vec<T, VEC>(thp + r0, tv);
          load_vec<T, VEC>(cp + r0, cv);
#pragma unroll
          for (int v = 0; v < VEC; ++v) {
            bt[kc][c * VEC + v] = tv[v];
            bc[kc][c * VEC + v] = cv[v];
          }
        }
      }
    };
    // the first raw loads overlap the set-up below
#pragma unroll
    for (int b = 0; b < PF; ++b) issue(b, rt[b], rc[b], rq[b], rl[b]);

    // t^k of this problem from its d^2 partials
    const double t = damping_t(gptr(P.d2part), uniform_i(P.nb), uniform_d(P.rho), uniform_d(P.gamma), lane);
    if (gtid == 0 && j0 == 0) gptr(P.t_out)[0] = t;

    // b^(m) = t (p - p^(m)) / S^m at this thread's rows, in LDS (a thread
    // holds the same rows in every column of the segment; with several
    // groups per workgroup, group 0 writes the rows every group reads, so
    // the previous segment's readers must be done first).  A row past R gets
    // b = -inf, which makes its w = -inf (never active, never the maximum)
    // without a select per entry.
    if constexpr (NG > 1) __syncthreads();
    if (g == 0) {
#pragma unroll
      for (int k = 0; k < VPT; ++k) {
        const int r = ((k / VEC) * NT + tid) * VEC + (k % VEC);
        lds_b[k * NT + tid] = (r < R) ? t * (pv[r] - pmm[r]) / Sm : -__builtin_huge_val();
      }
    }
    if constexpr (NG > 1) __syncthreads();  // group 0 wrote every group's b
#pragma unroll
    for (int k = 0; k < VPT; ++k) fix[k * NT + tid] = 0ull;
    T nb[VPT];  // -b^(m) rounded to the storage type: every inactive entry's new value
#pragma unroll
    for (int k = 0; k < VPT; ++k) nb[k] = (T)(-lds_b[k * NT + tid]);

    auto body = [&](int64_t step, T (&bt)[KC][VPT], T (&bc)[KC][VPT], T (&bq)[KC], double (&bl)[KC]) {
      // ---- reflect the step's columns: w = theta + 2b - c/rho (double) ----
      // (a column slot past the segment's end is computed too, on defined
      // values, and then ignored: no select per entry)
      double w[KC][VPT], wt[KC];  // wt: the thread's largest w of each column
      T told[DIAG ? KC : 1][DIAG ? VPT : 1];
      bool valid[KC];
      int64_t jj[KC];
      double b2[VPT];  // 2b of this thread's rows, all requested before the first use
#pragma unroll
      for (int k = 0; k < VPT; ++k) b2[k] = 2.0 * lds_b[k * NT + tid];
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) {
        valid[kc] = step_col(step, kc, jj[kc]);
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
          w[kc][k] = ((double)bt[kc][k] + b2[k]) - (double)bc[kc][k] * inv_rho;
          if constexpr (DIAG) told[kc][k] = bt[kc][k];
        }
        wt[kc] = w[kc][0];
#pragma unroll
        for (int k = 1; k < VPT; ++k) wt[kc] = max_arith(wt[kc], w[kc][k]);
      }
      // this step's q_s and stored threshold, taken before the buffer is refilled
      double qcol[KC], lcol[KC];
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) {
        qcol[kc] = (double)bq[kc];
        lcol[kc] = bl[kc];
      }
      // the next step's loads are issued at a raised wave priority, so the
      // co-resident waves' arithmetic does not delay their requests (FP32
      // plans; it measured slower in FP64)
      if constexpr (sizeof(T) == 4) __builtin_amdgcn_s_setprio(2);
      issue(step + PF, bt, bc, bq, bl);
      if constexpr (sizeof(T) == 4) __builtin_amdgcn_s_setprio(0);

      // ---- thresholds ----
      double tau[KC], lam[KC];
      bool act[KC];
      int mask[KC], nrounds[KC], nact[KC], nprev[KC];
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) {
        tau[kc] = valid[kc] ? uniform_d(qcol[kc]) : 0.0;
        act[kc] = valid[kc] && tau[kc] > 0.0;
        lam[kc] = (act[kc] && warm) ? uniform_d(lcol[kc]) : __builtin_nan("");
        if (!act[kc]) lam[kc] = __builtin_huge_val();
        mask[kc] = 0;
        nrounds[kc] = 0;
        nact[kc] = 0;
        nprev[kc] = -1;
      }
      for (int it = 0; it < R + 4; ++it) {
        bool any = false;
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) any |= act[kc];
        if (!any) break;
        double S[KC], wmx[KC];
        float mnA[KC], mxN[KC];
        int n[KC];
        bool cold[KC];
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
          S[kc] = 0.0;
          wmx[kc] = -__builtin_huge_val();
          mnA[kc] = __builtin_huge_valf();
          mxN[kc] = -__builtin_huge_valf();
          n[kc] = 0;
          cold[kc] = lam[kc] != lam[kc];
          if (act[kc]) {
            const double l = lam[kc];
            double lo = __builtin_huge_val(), hi = -__builtin_huge_val();
            int bits = 0;
            // Most waves of a column hold no active entry at all: one compare
            // of the thread's largest w settles that case for the whole wave.
            // Otherwise usually no lane of the wave holds an active entry in
            // slot k, and a uniform branch keeps that slot to one compare and
            // one max.
            if (__ballot(wt[kc] > l) == 0ull) {
              hi = wt[kc];
            } else {
#pragma unroll
              for (int k = 0; k < VPT; ++k) {
                const double x = w[kc][k];
                const unsigned long long bal = __ballot(x > l);
                if (bal == 0ull) {
                  hi = fmax(hi, x);
                } else {
                  const bool in = x > l;
                  n[kc] += __popcll(bal);
                  bits |= (int)in << k;
                  S[kc] += in ? x : 0.0;
                  lo = fmin(lo, in ? x : __builtin_huge_val());
                  hi = fmax(hi, in ? -__builtin_huge_val() : x);
                }
              }
            }
            mask[kc] = bits;
            mnA[kc] = float_down(lo);
            mxN[kc] = float_up(hi);
            wmx[kc] = hi;  // with lam = NaN nothing is active: hi = w_max
          }
        }
        rounds.reduce(S, mnA, mxN, wmx, n, act, cold, wv, lane);
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
          if (!act[kc]) continue;
          ++nrounds[kc];
          if (n[kc] == 0) {
            if (cold[kc]) {
              // start from the exact lower bound w_max - tau
              lam[kc] = wmx[kc] - tau[kc];
              nprev[kc] = 0x7fffffff;
            } else if (nprev[kc] < 0) {
              // the warm start lay above w_max: take a cold round
              lam[kc] = __builtin_nan("");
            } else {
              // w_max - tau rounded to w_max (tau below half an ulp of
              // w_max): nothing is active and the column is 0
              act[kc] = false;
              mask[kc] = 0;
            }
          } else {
            const double ln = (S[kc] - tau[kc]) / (double)n[kc];
            if (n[kc] == nprev[kc] || ((double)mnA[kc] >= ln && (double)mxN[kc] <= ln)) {
              act[kc] = false;  // mask[kc] is the exact active set
              nact[kc] = n[kc];
            }
            nprev[kc] = n[kc];
            lam[kc] = ln;
          }
        }
      }

      // ---- theta' = -b, patched at the active rows with max(w - lam, 0) - b ----
      // Only a wave holding an active entry looks at the mask bits; it also
      // adds the patches' pi_hat, before rounding, to the thread's row sums
      // (an inactive entry's stored -b enters nothing else: it is inactive
      // again or, if it becomes active, off by a relative 2^-24 of b, so the
      // marginals follow the double iteration).  With relaxed columns the
      // projection onto {u >= 0, sum u <= q_s} is max(w - max(lam, 0), 0):
      // the clamped column if it carries at most q_s (then the simplex
      // threshold is <= 0), else the simplex projection.  The stored warm
      // start stays the simplex threshold.
      double lout[KC];
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) lout[kc] = relaxed ? fmax(lam[kc], 0.0) : lam[kc];
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) {
        if (!valid[kc]) continue;
        const int64_t j = jj[kc];
        T* __restrict__ thp = theta + j * ld;
        double colsum = 0.0;
        const T* __restrict__ cp = cost;
        if constexpr (DIAG) cp = cost_col(j);
        T out[VPT];
#pragma unroll
        for (int k = 0; k < VPT; ++k) out[k] = nb[k];
        if (__ballot(mask[kc] != 0) != 0ull) {
#pragma unroll
          for (int k = 0; k < VPT; ++k) {
            if ((mask[kc] >> k) & 1) {
              const double ph = fmax(w[kc][k] - lout[kc], 0.0);
              out[k] = (T)(ph - lds_b[k * NT + tid]);
              fix[k * NT + tid] += to_fixed(ph, fxm);
              if constexpr (DIAG) {
                colsum += ph;
                dW += (double)cp[((k / VEC) * NT + tid) * VEC + (k % VEC)] * ph;
              }
            }
          }
        }
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          const int r0 = (c * NT + tid) * VEC;
          if (r0 < R) {
            if constexpr (DIAG) {
#pragma unroll
              for (int v = 0; v < VEC; ++v)
                if (r0 + v < R) dTh = fmax(dTh, fabs((double)out[c * VEC + v] - (double)told[kc][c * VEC + v]));
            }
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
        if (tid == 0) lamv[j] = lam[kc];
        if (a.rec) {
          // the exact active set, one bit per slot, for the reverse mode
          using W = typename MaskWord<VPT>::type;
          reinterpret_cast<W*>(a.rec + j * a.rec_ld)[tid] = (W)mask[kc];
        }
        if constexpr (DIAG) {
          colsum = wave_sum(colsum);
          if constexpr (NW > 1) {
            // reuse the round slots (parity keeps them apart from the last round)
            if (lane == 0) red_d[(rounds.par * KC * 2) * NW + wv] = colsum;
            __syncthreads();
            double cs = 0.0;
            for (int i = 0; i < NW; ++i) cs += red_d[(rounds.par * KC * 2) * NW + i];
            colsum = cs;
            rounds.par ^= 1;
          }
          dRes = fmax(dRes, relaxed ? fmax(colsum - tau[kc], 0.0) : fabs(colsum - tau[kc]));
          if (tid == 0) {
            dRounds += nrounds[kc];
            dAct += nact[kc];
            dCols += 1.0;
          }
        }
      }
    };
    // steps in turn, PF of them in flight: unrolled so every buffer index is static
    for (int64_t step = 0; step_exists(step); step += PF) {
      body(step, rt[0], rc[0], rq[0], rl[0]);
      if constexpr (PF > 1) {
        if (!step_exists(step + 1)) break;
        body(step + 1, rt[1], rc[1], rq[1], rl[1]);
      }
    }
    // the segment's fixed-point row sums of pi_hat into the accumulators:
    // one integer addition per row with mass
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
      const unsigned long long f = fix[k * NT + tid];
      if (f != 0ull) atomicAdd(accm + ((k / VEC) * NT + tid) * VEC + (k % VEC), f);
    }
  }

  if constexpr (DIAG) {
    // sums of W_hat, rounds, active entries, columns; maxima of residual and change
    const double s0 = wave_sum(dW), r1 = wave_max(dRes), r2 = wave_max(dTh);
    const double s3 = wave_sum(dRounds), s4 = wave_sum(dAct), s5 = wave_sum(dCols);
    if (lane == 0) {
      sh_diag[gtid >> 6][0] = s0;
      sh_diag[gtid >> 6][1] = r1;
      sh_diag[gtid >> 6][2] = r2;
      sh_diag[gtid >> 6][3] = s3;
      sh_diag[gtid >> 6][4] = s4;
      sh_diag[gtid >> 6][5] = s5;
    }
    __syncthreads();
    if (gtid == 0) {
      double S0 = 0.0, m1 = 0.0, m2 = 0.0, S3 = 0.0, S4 = 0.0, S5 = 0.0;
      for (int i = 0; i < WG / 64; ++i) {
        S0 += sh_diag[i][0];
        m1 = fmax(m1, sh_diag[i][1]);
        m2 = fmax(m2, sh_diag[i][2]);
        S3 += sh_diag[i][3];
        S4 += sh_diag[i][4];
        S5 += sh_diag[i][5];
      }
      double* o = a.diag + (size_t)wg * DIAG_STRIDE;
      o[0] = S0;
      o[1] = m1;
      o[2] = m2;
      o[3] = S3;
      o[4] = S4;
      o[5] = S5;
      o[6] = 0.0;
      o[7] = 0.0;
    }
  }

}

}  // namespace mam

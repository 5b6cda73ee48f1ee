// Column-kernel instance lookup.  The instances are compiled in separate
// translation units (one per element type and diagnostics mode) so the
// build runs in parallel.
#pragma once

#include "mam_kernels.hpp"

namespace mam {

template <typename T>
using ColFn = void (*)(ColArgs<T>);

// Returns the instance for (threads per column, values per thread, vector
// width, columns in flight, diagnostics) or nullptr if none exists.
// Instances: 64 threads with 1-16 values per thread, 128-1024 threads with
// 4-16; columns in flight 1, 2, 4 for vector loads without diagnostics,
// otherwise 1.
template <typename T, int KC>
ColFn<T> pick_column_kc(int nt, int vpt, int vec, int stream);
template <typename T>
ColFn<T> pick_column_diag(int nt, int vpt, int vec);

// Sub-wave instance (16 or 32 lanes per column, one column in flight, no
// diagnostics) or nullptr.
template <typename T>
ColFn<T> pick_subwave(int nt, int vpt, int vec, int stream);
extern template ColFn<float> pick_subwave<float>(int, int, int, int);
extern template ColFn<double> pick_subwave<double>(int, int, int, int);

template <typename T>
inline ColFn<T> pick_column(int nt, int vpt, int vec, int kc, int diag, int stream) {
  if (nt < 64) return (diag || kc != 1) ? nullptr : pick_subwave<T>(nt, vpt, vec, stream);
  if (diag) return pick_column_diag<T>(nt, vpt, vec);
  switch (kc) {
    case 1: return pick_column_kc<T, 1>(nt, vpt, vec, stream);
    case 2: return pick_column_kc<T, 2>(nt, vpt, vec, stream);
    case 4: return pick_column_kc<T, 4>(nt, vpt, vec, stream);
    default: return nullptr;
  }
}

// Long-column tile kernels for (values per thread, vector width, grid
// cost); null members if no instance exists.
template <typename T> struct LongArgs;
template <typename T>
struct LongFns {
  void (*scan)(LongArgs<T>) = nullptr;
  void (*thresh)(LongArgs<T>) = nullptr;
  void (*write)(LongArgs<T>) = nullptr;
  void (*rowsum)(LongArgs<T>, int) = nullptr;
  void (*materialize)(LongArgs<T>) = nullptr;  // sparse store write-back
  void (*scan_sparse)(LongArgs<T>) = nullptr;  // sparse-store scan
  void (*thresh_diag)(LongArgs<T>) = nullptr;  // with the iteration's diagnostics
  void (*write_diag)(LongArgs<T>) = nullptr;
};
template <typename T>
LongFns<T> pick_long(int vpt, int vec, bool grid);
extern template LongFns<float> pick_long<float>(int, int, bool);
extern template LongFns<double> pick_long<double>(int, int, bool);

// Reverse-mode column kernel for (mask bytes per lane, columns per wave at
// a time); nullptr if none exists.
struct AdjArgs;
using AdjFn = void (*)(AdjArgs);
AdjFn pick_adjoint(int lane_bytes, int kc);

extern template ColFn<float> pick_column_kc<float, 1>(int, int, int, int);
extern template ColFn<float> pick_column_kc<float, 2>(int, int, int, int);
extern template ColFn<float> pick_column_kc<float, 4>(int, int, int, int);
extern template ColFn<double> pick_column_kc<double, 1>(int, int, int, int);
extern template ColFn<double> pick_column_kc<double, 2>(int, int, int, int);
extern template ColFn<double> pick_column_kc<double, 4>(int, int, int, int);
extern template ColFn<float> pick_column_diag<float>(int, int, int);
extern template ColFn<double> pick_column_diag<double>(int, int, int);

}  // namespace mam

// Column-kernel instance lookup.  The instances are compiled in separate
// translation units (one per element type and diagnostics mode) so the
// build runs in parallel.
#pragma once

#include "mam_kernels.hpp"

namespace mam {

template <typename T>
using ColFn = void (*)(ColArgs<T>);

// Returns the instance for (threads per column, values per thread, vector
// width, diagnostics) or nullptr if none exists.
template <typename T, bool DIAG>
ColFn<T> pick_column_impl(int nt, int vpt, int vec);

template <typename T>
inline ColFn<T> pick_column(int nt, int vpt, int vec, int diag) {
  return diag ? pick_column_impl<T, true>(nt, vpt, vec) : pick_column_impl<T, false>(nt, vpt, vec);
}

extern template ColFn<float> pick_column_impl<float, false>(int, int, int);
extern template ColFn<float> pick_column_impl<float, true>(int, int, int);
extern template ColFn<double> pick_column_impl<double, false>(int, int, int);
extern template ColFn<double> pick_column_impl<double, true>(int, int, int);

}  // namespace mam

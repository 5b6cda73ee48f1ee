// Instances of the long-column tile kernels: row tiles of 256*VPT rows,
// VPT in {4, 8, 16}, vector loads of 16 bytes or single elements, the cost
// read or formed from a grid.
#include "mam_dispatch.hpp"
#include "mam_long.hpp"

namespace mam {

template <typename T, int VPT, bool GRID>
LongFns<T> pick_long_vec(int vec) {
  constexpr int VN = VecOf<T>::N;
  if (vec == VN)
    return {&long_scan_kernel<T, VPT, VN, GRID, false>, &long_threshold_kernel<T, VPT, VN, false>,
            &long_write_kernel<T, VPT, VN, false>, &long_rowsum_kernel<T>, &long_materialize_kernel<T, VPT, VN>,
            &long_scan_kernel<T, VPT, VN, GRID, true>, &long_threshold_kernel<T, VPT, VN, true>,
            &long_write_kernel<T, VPT, VN, true>};
  if (vec == 1)
    return {&long_scan_kernel<T, VPT, 1, GRID, false>, &long_threshold_kernel<T, VPT, 1, false>,
            &long_write_kernel<T, VPT, 1, false>, &long_rowsum_kernel<T>, &long_materialize_kernel<T, VPT, 1>,
            &long_scan_kernel<T, VPT, 1, GRID, true>, &long_threshold_kernel<T, VPT, 1, true>,
            &long_write_kernel<T, VPT, 1, true>};
  return {};
}

template <typename T, bool GRID>
LongFns<T> pick_long_grid(int vpt, int vec) {
  switch (vpt) {
    case 4: return pick_long_vec<T, 4, GRID>(vec);
    case 8: return pick_long_vec<T, 8, GRID>(vec);
    case 16: return pick_long_vec<T, 16, GRID>(vec);
    default: return {};
  }
}

template <typename T>
LongFns<T> pick_long(int vpt, int vec, bool grid) {
  return grid ? pick_long_grid<T, true>(vpt, vec) : pick_long_grid<T, false>(vpt, vec);
}

template LongFns<float> pick_long<float>(int, int, bool);
template LongFns<double> pick_long<double>(int, int, bool);

}  // namespace mam

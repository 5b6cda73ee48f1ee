// Instances of the long-column tile kernels: row tiles of 256*VPT rows,
// VPT in {4, 8, 16}, vector loads of 16 bytes or single elements.
#include "mam_dispatch.hpp"
#include "mam_long.hpp"

namespace mam {

template <typename T, int VPT>
LongFns<T> pick_long_vec(int vec) {
  constexpr int VN = VecOf<T>::N;
  if (vec == VN)
    return {&long_scan_kernel<T, VPT, VN>, &long_threshold_kernel<T, VPT, VN>, &long_write_kernel<T, VPT, VN>,
            &long_rowsum_kernel<T>};
  if (vec == 1)
    return {&long_scan_kernel<T, VPT, 1>, &long_threshold_kernel<T, VPT, 1>, &long_write_kernel<T, VPT, 1>,
            &long_rowsum_kernel<T>};
  return {};
}

template <typename T>
LongFns<T> pick_long(int vpt, int vec) {
  switch (vpt) {
    case 4: return pick_long_vec<T, 4>(vec);
    case 8: return pick_long_vec<T, 8>(vec);
    case 16: return pick_long_vec<T, 16>(vec);
    default: return {};
  }
}

template LongFns<float> pick_long<float>(int, int);
template LongFns<double> pick_long<double>(int, int);

}  // namespace mam

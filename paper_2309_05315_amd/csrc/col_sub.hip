// Instances of the sub-wave column kernel: 16 or 32 lanes per column, 1-16
// values per lane, vector loads of 16 bytes when a lane holds at least one
// vector, plain or streaming (non-temporal) plans.
#include "mam_dispatch.hpp"
#include "mam_subwave.hpp"

namespace mam {

template <typename T, int NT, int VPT>
ColFn<T> pick_sub_vec(int vec, int stream) {
  constexpr int VN = VecOf<T>::N;
  if constexpr (VPT >= VN) {
    if (vec == VN) return stream ? &subwave_kernel<T, NT, VPT, VN, true> : &subwave_kernel<T, NT, VPT, VN, false>;
  }
  if (vec == 1) return stream ? &subwave_kernel<T, NT, VPT, 1, true> : &subwave_kernel<T, NT, VPT, 1, false>;
  return nullptr;
}

template <typename T, int NT>
ColFn<T> pick_sub_vpt(int vpt, int vec, int stream) {
  switch (vpt) {
    case 1: return pick_sub_vec<T, NT, 1>(vec, stream);
    case 2: return pick_sub_vec<T, NT, 2>(vec, stream);
    case 4: return pick_sub_vec<T, NT, 4>(vec, stream);
    case 8: return pick_sub_vec<T, NT, 8>(vec, stream);
    case 16: return pick_sub_vec<T, NT, 16>(vec, stream);
    default: return nullptr;
  }
}

template <typename T>
ColFn<T> pick_subwave(int nt, int vpt, int vec, int stream) {
  if (nt == 16) return pick_sub_vpt<T, 16>(vpt, vec, stream);
  if (nt == 32) return pick_sub_vpt<T, 32>(vpt, vec, stream);
  return nullptr;
}

template ColFn<float> pick_subwave<float>(int, int, int, int);
template ColFn<double> pick_subwave<double>(int, int, int, int);

}  // namespace mam

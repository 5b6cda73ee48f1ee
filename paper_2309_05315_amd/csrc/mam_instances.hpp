// Instantiation of the column kernel over the supported shapes; included
// by one translation unit per (element type, columns in flight) pair, which
// defines MAM_INST_T and MAM_INST_KC first (MAM_INST_KC 0 = the
// diagnostics instances, one column in flight).
#pragma once

#include "mam_dispatch.hpp"

namespace mam {

template <typename T, int NT, int VPT, int KC, bool DIAG>
ColFn<T> pick_vec(int vec, int stream) {
  constexpr int VN = VecOf<T>::N;
  if constexpr (VPT >= VN) {
    // streaming (non-temporal) forms of the vector-load, one-column shapes
    if constexpr (KC == 1 && !DIAG) {
      if (vec == VN && stream) return &column_kernel<T, NT, VPT, VN, KC, DIAG, true>;
    }
    if (vec == VN) return &column_kernel<T, NT, VPT, VN, KC, DIAG>;
  }
  if constexpr (KC == 1) {
    if (vec == 1) return &column_kernel<T, NT, VPT, 1, 1, DIAG>;
  }
  return nullptr;
}

template <typename T, int NT, int KC, bool DIAG>
ColFn<T> pick_vpt(int vpt, int vec, int stream) {
  if constexpr (NT == 64) {
    switch (vpt) {
      case 1: return pick_vec<T, NT, 1, KC, DIAG>(vec, stream);
      case 2: return pick_vec<T, NT, 2, KC, DIAG>(vec, stream);
      default: break;
    }
  }
  switch (vpt) {
    case 4: return pick_vec<T, NT, 4, KC, DIAG>(vec, stream);
    case 8: return pick_vec<T, NT, 8, KC, DIAG>(vec, stream);
    case 16: return pick_vec<T, NT, 16, KC, DIAG>(vec, stream);
    default: return nullptr;
  }
}

template <typename T, int KC, bool DIAG>
ColFn<T> pick_nt(int nt, int vpt, int vec, int stream) {
  switch (nt) {
    case 64: return pick_vpt<T, 64, KC, DIAG>(vpt, vec, stream);
    case 128: return pick_vpt<T, 128, KC, DIAG>(vpt, vec, stream);
    case 256: return pick_vpt<T, 256, KC, DIAG>(vpt, vec, stream);
    case 512: return pick_vpt<T, 512, KC, DIAG>(vpt, vec, stream);
    case 1024: return pick_vpt<T, 1024, KC, DIAG>(vpt, vec, stream);
    default: return nullptr;
  }
}

#if MAM_INST_KC == 0
template <typename T>
ColFn<T> pick_column_diag(int nt, int vpt, int vec) {
  return pick_nt<T, 1, true>(nt, vpt, vec, 0);
}
template ColFn<MAM_INST_T> pick_column_diag<MAM_INST_T>(int, int, int);
#else
template <typename T, int KC>
ColFn<T> pick_column_kc(int nt, int vpt, int vec, int stream) {
  return pick_nt<T, KC, false>(nt, vpt, vec, stream);
}
template ColFn<MAM_INST_T> pick_column_kc<MAM_INST_T, MAM_INST_KC>(int, int, int, int);
#endif

}  // namespace mam

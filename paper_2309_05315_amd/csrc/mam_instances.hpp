// Instantiation of the column kernel over the supported shapes; included
// by one translation unit per (element type, diagnostics) pair, which
// defines MAM_INST_T and MAM_INST_DIAG first.
#pragma once

#include "mam_dispatch.hpp"

namespace mam {

template <typename T, int NT, int VPT, bool DIAG>
ColFn<T> pick_vec(int vec) {
  constexpr int VN = VecOf<T>::N;
  if constexpr (VPT >= VN) {
    if (vec == VN) return &column_kernel<T, NT, VPT, VN, DIAG>;
  }
  if (vec != 1) return nullptr;
  return &column_kernel<T, NT, VPT, 1, DIAG>;
}

template <typename T, int NT, bool DIAG>
ColFn<T> pick_vpt(int vpt, int vec) {
  switch (vpt) {
    case 1: return pick_vec<T, NT, 1, DIAG>(vec);
    case 2: return pick_vec<T, NT, 2, DIAG>(vec);
    case 4: return pick_vec<T, NT, 4, DIAG>(vec);
    case 8: return pick_vec<T, NT, 8, DIAG>(vec);
    case 16: return pick_vec<T, NT, 16, DIAG>(vec);
    default: return nullptr;
  }
}

template <typename T, bool DIAG>
ColFn<T> pick_column_impl(int nt, int vpt, int vec) {
  switch (nt) {
    case 64: return pick_vpt<T, 64, DIAG>(vpt, vec);
    case 128: return pick_vpt<T, 128, DIAG>(vpt, vec);
    case 256: return pick_vpt<T, 256, DIAG>(vpt, vec);
    case 512: return pick_vpt<T, 512, DIAG>(vpt, vec);
    case 1024: return pick_vpt<T, 1024, DIAG>(vpt, vec);
    default: return nullptr;
  }
}

template ColFn<MAM_INST_T> pick_column_impl<MAM_INST_T, MAM_INST_DIAG>(int, int, int);

}  // namespace mam

// Reverse-mode column kernel instances: the shapes of the forward column
// kernel (64 threads with 1-16 values per thread, 128-1024 threads with
// 4-16); the vector width is a run-time argument of the row mapping.
#include "mam_adjoint.hpp"
#include "mam_dispatch.hpp"

namespace mam {

template <int NT>
AdjFn pick_adjoint_vpt(int vpt) {
  if constexpr (NT == 64) {
    if (vpt == 1) return &adjoint_kernel<NT, 1>;
    if (vpt == 2) return &adjoint_kernel<NT, 2>;
  }
  switch (vpt) {
    case 4: return &adjoint_kernel<NT, 4>;
    case 8: return &adjoint_kernel<NT, 8>;
    case 16: return &adjoint_kernel<NT, 16>;
    default: return nullptr;
  }
}

AdjFn pick_adjoint(int nt, int vpt) {
  switch (nt) {
    case 64: return pick_adjoint_vpt<64>(vpt);
    case 128: return pick_adjoint_vpt<128>(vpt);
    case 256: return pick_adjoint_vpt<256>(vpt);
    case 512: return pick_adjoint_vpt<512>(vpt);
    case 1024: return pick_adjoint_vpt<1024>(vpt);
    default: return nullptr;
  }
}

}  // namespace mam

// Reverse-mode column kernel instances: every mask size the forward column
// kernel records (64-1024 threads per column, 8- or 16-bit mask words, so
// 1-32 mask bytes per lane), 1, 2 or 4 columns per wave at a time.
#include "mam_adjoint.hpp"
#include "mam_dispatch.hpp"

namespace mam {

template <int KC>
AdjFn pick_adjoint_lb(int lane_bytes) {
  switch (lane_bytes) {
    case 1: return &adjoint_kernel<1, KC>;
    case 2: return &adjoint_kernel<2, KC>;
    case 4: return &adjoint_kernel<4, KC>;
    case 8: return &adjoint_kernel<8, KC>;
    case 16: return &adjoint_kernel<16, KC>;
    case 32: return &adjoint_kernel<32, KC>;
    default: return nullptr;
  }
}

AdjFn pick_adjoint(int lane_bytes, int kc) {
  switch (kc) {
    case 1: return pick_adjoint_lb<1>(lane_bytes);
    case 2: return pick_adjoint_lb<2>(lane_bytes);
    case 4: return pick_adjoint_lb<4>(lane_bytes);
    default: return nullptr;
  }
}

}  // namespace mam

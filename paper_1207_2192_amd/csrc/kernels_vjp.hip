// Persistent-kernel instances of one mode (compiled as a unit of its own).
#include "llg_kernels.hpp"

namespace llg {
const void* persistent_kernel_vjp(int UG, int RSEL, int PMAX) {
    return persistent_instance<MODE_RK4_VJP>(UG, RSEL, PMAX);
}
}  // namespace llg

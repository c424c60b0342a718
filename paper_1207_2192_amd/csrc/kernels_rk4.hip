// Persistent-kernel instances of one mode (compiled as a unit of its own).
#include "llg_kernels.hpp"

namespace llg {
const void* persistent_kernel_rk4(int UG, int RSEL, int PMAX) {
    return persistent_instance<MODE_RK4>(UG, RSEL, PMAX);
}
}  // namespace llg

// Persistent-kernel instances of one mode with the observable series (compiled as a unit of its own).
#include "llg_kernels.hpp"

namespace llg {
const void* persistent_kernel_rk4_series(int UG, int RSEL, int PMAX) {
    return persistent_instance<MODE_RK4, true>(UG, RSEL, PMAX);
}
}  // namespace llg

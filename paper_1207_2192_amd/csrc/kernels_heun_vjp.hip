// Persistent-kernel instances of one mode (compiled as a unit of its own).
#include "llg_kernels.hpp"

namespace llg {
const void* persistent_kernel_heun_vjp(int UG, int RSEL, int PMAX) {
    return persistent_instance<MODE_HEUN_VJP>(UG, RSEL, PMAX);
}
}  // namespace llg

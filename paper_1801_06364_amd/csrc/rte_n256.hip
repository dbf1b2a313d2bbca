// Kernels of the P_N stepper specialised for a 256^3 grid (row + pencil
// passes: a 256 x 129 complex plane does not fit in LDS).
#include "rte_kernels.h"

namespace rte {
RTE_DEFINE_SIZE(256)
}  // namespace rte

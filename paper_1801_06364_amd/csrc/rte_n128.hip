// Kernels of the P_N stepper specialised for a 128^3 grid.
#include "rte_kernels.h"

namespace rte {
RTE_DEFINE_SIZE(128)
}  // namespace rte

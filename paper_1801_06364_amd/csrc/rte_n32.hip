// Kernels of the P_N stepper specialised for a 32^3 grid.
#include "rte_kernels.h"

namespace rte {
RTE_DEFINE_SIZE(32)
}  // namespace rte

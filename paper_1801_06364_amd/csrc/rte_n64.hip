// Kernels of the P_N stepper specialised for a 64^3 grid.
#include "rte_kernels.h"

namespace rte {
RTE_DEFINE_SIZE(64)
}  // namespace rte

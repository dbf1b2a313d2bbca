// Kernels of the P_N stepper specialised for a 48^3 grid.
#include "rte_kernels.h"

namespace rte {
RTE_DEFINE_SIZE(48)
}  // namespace rte

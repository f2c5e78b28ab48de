// k_f64_pass.hip -- FP64 column, row, propagator-table and adaptive-step kernels.
#include "kernel_list.h"

namespace opo {
OPO_PASS_KERNELS_F64(template)
} // namespace opo

// k_f32_pass.hip -- FP32 column, row, propagator-table and adaptive-step kernels.
#include "kernel_list.h"

namespace opo {
OPO_PASS_KERNELS_F32(template)
} // namespace opo

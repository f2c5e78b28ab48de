// k_f32_mixed3.hip -- FP32 mixed launches of three-wave instances.
#include "kernel_list.h"

namespace opo {
OPO_MIXED_KERNELS_F32_CR0(template, 3)
OPO_MIXED_KERNELS_F32_CR12(template, 3)
} // namespace opo

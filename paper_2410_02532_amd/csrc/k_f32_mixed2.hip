// k_f32_mixed2.hip -- FP32 mixed launches of two-wave instances.
#include "kernel_list.h"

namespace opo {
OPO_MIXED_KERNELS_F32_CR0(template, 2)
OPO_MIXED_KERNELS_F32_CR12(template, 2)
} // namespace opo

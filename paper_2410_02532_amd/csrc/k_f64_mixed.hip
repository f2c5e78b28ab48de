// k_f64_mixed.hip -- FP64 mixed launches.
#include "kernel_list.h"

namespace opo {
OPO_MIXED_KERNELS_F64(template, 2)
OPO_MIXED_KERNELS_F64(template, 3)
} // namespace opo

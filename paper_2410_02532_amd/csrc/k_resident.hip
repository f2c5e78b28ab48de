// k_resident.hip -- resident passes (one workgroup per instance for a whole pass).
#include "kernel_list.h"

namespace opo {
OPO_RESIDENT_KERNELS(template)
} // namespace opo

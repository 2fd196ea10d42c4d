// Kernel instantiations: rope_configs.
#include "cord_kernels_impl.h"

namespace cord {

const KernelCfg* rope_configs(int* count) {
    static const KernelCfg t[] = {
    CORD_CFG(kRope, 64, 1, 4),
    CORD_CFG(kRope, 64, 2, 4),
    CORD_CFG(kRope, 128, 1, 4),
    CORD_CFG(kRope, 64, 4, 4),
    CORD_CFG(kRope, 128, 2, 4),
    CORD_CFG(kRope, 256, 1, 4),
    };
    *count = (int)(sizeof(t) / sizeof(t[0]));
    return t;
}

}  // namespace cord

// Kernel instantiations: cloth_configs_a.
#include "cord_kernels_impl.h"

namespace cord {

const KernelCfg* cloth_configs_a(int* count) {
    static const KernelCfg t[] = {
    CORD_CFG(kCloth, 64, 1, 4),
    CORD_CFG(kCloth, 128, 1, 4),
    CORD_CFG(kCloth, 256, 1, 4),
    CORD_CFG(kCloth, 128, 2, 4),
    };
    *count = (int)(sizeof(t) / sizeof(t[0]));
    return t;
}

}  // namespace cord

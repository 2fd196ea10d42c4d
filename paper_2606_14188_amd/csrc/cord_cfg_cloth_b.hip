// Kernel instantiations: cloth_configs_b.
#include "cord_kernels_impl.h"

namespace cord {

const KernelCfg* cloth_configs_b(int* count) {
    static const KernelCfg t[] = {
    CORD_CFG(kCloth, 512, 1, 4),
    CORD_CFG(kCloth, 256, 2, 4),
    CORD_CFG(kCloth, 1024, 1, 4),
    CORD_CFG(kCloth, 512, 2, 4),
    };
    *count = (int)(sizeof(t) / sizeof(t[0]));
    return t;
}

}  // namespace cord

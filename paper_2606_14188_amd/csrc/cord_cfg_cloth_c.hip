// Kernel instantiations: cloth_configs_c (cloths of up to 48 x 48 nodes,
// three particles per thread; this configuration spills registers to
// scratch and trades speed for coverage).
#include "cord_kernels_impl.h"

namespace cord {

const KernelCfg* cloth_configs_c(int* count) {
    static const KernelCfg t[] = {
    CORD_CFG(kCloth, 768, 3, 4),
    };
    *count = (int)(sizeof(t) / sizeof(t[0]));
    return t;
}

}  // namespace cord

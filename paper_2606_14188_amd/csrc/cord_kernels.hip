// Configuration table over all size-class translation units, and the
// small utility kernels.
#include <hip/hip_runtime.h>

#include <vector>

#include "cord_kernels.h"

namespace cord {

const KernelCfg* rope_configs(int* count);
const KernelCfg* cloth_configs_a(int* count);
const KernelCfg* cloth_configs_b(int* count);
const KernelCfg* cloth_configs_c(int* count);

const KernelCfg* kernel_configs(int* count) {
    static const std::vector<KernelCfg> all = [] {
        std::vector<KernelCfg> v;
        for (auto f : {rope_configs, cloth_configs_a, cloth_configs_b, cloth_configs_c}) {
            int c = 0;
            const KernelCfg* t = f(&c);
            v.insert(v.end(), t, t + c);
        }
        return v;
    }();
    *count = (int)all.size();
    return all.data();
}

}  // namespace cord

namespace cord {

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + 255) / 256;
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)nb), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace cord

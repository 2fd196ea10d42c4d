// Kernel configuration table shared by the kernels and the host API.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "cord_internal.h"

namespace cord {

struct KernelCfg {
    int topo;      // kRope / kCloth
    int nt;        // threads per workgroup
    int ppt;       // particles per thread
    int nobs;      // obstacle slots
    size_t lds;    // dynamic LDS bytes
    hipError_t (*rollout)(const KArgs&, int nblk, hipStream_t);
    hipError_t (*backward)(const KArgs&, int nblk, hipStream_t);
    hipError_t (*linearize)(const KArgs&, int nblk, int tmax, hipStream_t);
    int (*blocks_per_cu)(int which);   // occupancy of the rollout (0) / backward (1) kernel
};

const KernelCfg* kernel_configs(int* count);

}  // namespace cord

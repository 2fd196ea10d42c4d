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

// Dense A_t (and B_t) of ropes by banded direct solves, for size classes up
// to 128 particles.  The scratch query returns the floats of the optional
// scratch table (a.kept, with a.kept_tg = *wg_per_cu workgroup slots per CU;
// any other work must leave it alone until the kernel ends), or 0 with
// *wg_per_cu = 0 for other classes or if the device's LDS is too small: the
// caller then uses the class's iterative linearize kernel.  With a.kept null
// the kernel keeps its vectors inside A.
size_t linearize_rope_direct_scratch(int nmax, int* wg_per_cu);
hipError_t linearize_rope_direct(int nmax, const KArgs& a, int nblk, int tmax, hipStream_t s);

}  // namespace cord

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
    // the same three kernels compiled with the friction cone (mu > 0)
    hipError_t (*rollout_f)(const KArgs&, int nblk, hipStream_t);
    hipError_t (*backward_f)(const KArgs&, int nblk, hipStream_t);
    hipError_t (*linearize_f)(const KArgs&, int nblk, int tmax, hipStream_t);
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

// Static device scratch of cord_rollout_backward_noalloc (64 MiB per GPU):
// the checkpoint offset table (int64 per instance, padded to 256 bytes)
// followed by the recomputed-segment workspace (K n_s floats per instance).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
// This GPU's address of that scratch (looked up once per device, with the
// device current).
hipError_t noalloc_scratch(int device, void** out);
// Conformal calibration: per-instance score |x_next - x_pred|_2 over the
// positions (both in the state layout), and the score of 1-based rank k
// (ties by index; +inf if k > n, NaN if n is 0) with its index.
hipError_t launch_cp_scores(const InstDev* inst, int B, const float* pred, const float* s_next, float* scores,
                            hipStream_t s);
hipError_t launch_cp_radius(const float* scores, int n, int k, float* radius, int32_t* rank, hipStream_t s);
// out[b] = sum_{b' < b} (ceil(T/K) + 1) n_s over the instance table.
hipError_t launch_ckpt_offsets(const InstDev* inst, int B, int K, int64_t* out, hipStream_t s);

}  // namespace cord

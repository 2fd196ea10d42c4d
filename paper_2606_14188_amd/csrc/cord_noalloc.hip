// Device scratch of the checkpointed adjoint for callers that cannot
// allocate (cord_rollout_backward_noalloc): a file-scope device array, one
// copy per GPU for the life of the process, holding the checkpoint offset
// table and the workspace of the recomputed segments.
#include <hip/hip_runtime.h>

#include <mutex>

#include "cord_internal.h"
#include "cord_kernels.h"

namespace cord {

static __device__ __align__(256) float scratch[kNoAllocScratchBytes / sizeof(float)];

namespace {
constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;
}  // namespace

// This GPU's copy of `scratch`, looked up once per device with that device
// current.  Host code passes this address to kernels; the array's own name
// is a host-side stand-in, not a device address.
hipError_t noalloc_scratch(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[device] = p;
    }
    *out = g_scratch[device];
    return hipSuccess;
}

// Checkpoint offsets for spacing K: out[b] = sum_{b' < b} (ceil(T/K) + 1) n_s.
// One workgroup of 256 threads: each sums a contiguous chunk of instances,
// thread 0 scans the 256 chunk sums, then each writes its chunk's offsets.
__global__ __launch_bounds__(256) void ckpt_offsets_kernel(const InstDev* inst, int B, int K, int64_t* out) {
    __shared__ int64_t part[256];
    const int tid = threadIdx.x;
    const int chunk = (B + 255) / 256;
    const int b0 = min(B, tid * chunk), b1 = min(B, b0 + chunk);
    int64_t sum = 0;
    for (int b = b0; b < b1; ++b) sum += (int64_t)((inst[b].T + K - 1) / K + 1) * inst[b].n_s;
    part[tid] = sum;
    __syncthreads();
    if (tid == 0) {
        int64_t run = 0;
        for (int i = 0; i < 256; ++i) {
            const int64_t v = part[i];
            part[i] = run;
            run += v;
        }
    }
    __syncthreads();
    int64_t o = part[tid];
    for (int b = b0; b < b1; ++b) {
        out[b] = o;
        o += (int64_t)((inst[b].T + K - 1) / K + 1) * inst[b].n_s;
    }
}

hipError_t launch_ckpt_offsets(const InstDev* inst, int B, int K, int64_t* out, hipStream_t s) {
    hipLaunchKernelGGL(ckpt_offsets_kernel, dim3(1), dim3(256), 0, s, inst, B, K, out);
    return hipGetLastError();
}

}  // namespace cord

// Conformal calibration of the one-step model error (Sec. 4.4): the
// nonconformity score of every calibration pair and the order statistic
// that is the radius r_CP.
#include <hip/hip_runtime.h>

#include <cmath>

#include "cord_internal.h"
#include "cord_kernels.h"

namespace cord {

// scores[b] = |x_next_b - x_pred_b|_2 over the 3n positions of instance b;
// one workgroup per instance, a wavefront reduction then one LDS exchange.
__global__ __launch_bounds__(256) void cp_score_kernel(const InstDev* inst, int B, const float* pred,
                                                       const float* s_next, float* scores) {
    const int b = blockIdx.x;
    if (b >= B) return;
    const InstDev& I = inst[b];
    const int m = 3 * I.n;
    const float* p = pred + I.s_off;
    const float* q = s_next + I.s_off;
    float acc = 0.f;
    for (int i = threadIdx.x; i < m; i += 256) {
        const float d = q[i] - p[i];
        acc += d * d;
    }
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    __shared__ float part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) scores[b] = sqrtf((part[0] + part[1]) + (part[2] + part[3]));
}

hipError_t launch_cp_scores(const InstDev* inst, int B, const float* pred, const float* s_next, float* scores,
                            hipStream_t s) {
    hipLaunchKernelGGL(cp_score_kernel, dim3(B), dim3(256), 0, s, inst, B, pred, s_next, scores);
    return hipGetLastError();
}

__global__ void cp_init_kernel(float* radius, int32_t* rank, float value) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *radius = value;
        if (rank) *rank = -1;
    }
}

// Sort key of a score: NaN orders after every number.
__device__ __forceinline__ float cp_key(float s) { return s == s ? s : INFINITY; }

// The score at 0-based position k0 of the ascending order, ties broken by
// index: thread i counts the scores below s_i, and the equal ones of lower
// index, over tiles of 256 scores staged in LDS; (score, index) is a total
// order, so exactly one thread finds the count k0 and writes its score and
// index.
__global__ __launch_bounds__(256) void cp_rank_kernel(const float* scores, int n, int k0, float* radius,
                                                      int32_t* rank) {
    __shared__ float tile[256];
    const int i = blockIdx.x * 256 + threadIdx.x;
    const float si = i < n ? cp_key(scores[i]) : 0.f;
    int below = 0;
    for (int t0 = 0; t0 < n; t0 += 256) {
        __syncthreads();
        const int j = t0 + threadIdx.x;
        tile[threadIdx.x] = j < n ? cp_key(scores[j]) : 0.f;
        __syncthreads();
        const int cnt = min(256, n - t0);
        for (int jj = 0; jj < cnt; ++jj) {
            const float sj = tile[jj];
            below += (sj < si || (sj == si && t0 + jj < i)) ? 1 : 0;
        }
    }
    if (i < n && below == k0) {
        *radius = scores[i];
        if (rank) *rank = i;
    }
}

hipError_t launch_cp_radius(const float* scores, int n, int k, float* radius, int32_t* rank, hipStream_t s) {
    // +inf when k exceeds n; NaN stays if no score can be selected
    hipLaunchKernelGGL(cp_init_kernel, dim3(1), dim3(64), 0, s, radius, rank, k > n ? INFINITY : NAN);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || k > n) return e;
    hipLaunchKernelGGL(cp_rank_kernel, dim3((n + 255) / 256), dim3(256), 0, s, scores, n, k - 1, radius, rank);
    return hipGetLastError();
}

}  // namespace cord

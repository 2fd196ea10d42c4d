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
// index.  (score, index) is a total order, so the position of score i is
// the number of scores below it plus the equal ones of lower index, and
// exactly one i has position k0.  A workgroup takes 16 candidates i and
// splits the n scores into 16 ranges: thread (r, c) counts candidate c
// against range r, the 16 partial counts of a candidate are summed in LDS,
// and the candidate whose count is k0 writes its score and index.  The
// counts are exact integers, so the split does not change the selection.
constexpr int kCpCand = 16;    // candidates per workgroup
constexpr int kCpRanges = 16;  // ranges of the scores per candidate
__global__ __launch_bounds__(kCpCand * kCpRanges) void cp_rank_kernel(const float* scores, int n, int k0,
                                                                      float* radius, int32_t* rank) {
    __shared__ int part[kCpRanges][kCpCand];
    const int c = threadIdx.x % kCpCand, r = threadIdx.x / kCpCand;
    const int i = blockIdx.x * kCpCand + c;
    const float si = i < n ? cp_key(scores[i]) : 0.f;
    const int len = (n + kCpRanges - 1) / kCpRanges;
    const int j0 = r * len, j1 = min(n, j0 + len);
    int below = 0;
    for (int j = j0; j < j1; ++j) {
        const float sj = cp_key(scores[j]);
        below += (sj < si || (sj == si && j < i)) ? 1 : 0;
    }
    part[r][c] = below;
    __syncthreads();
    if (r == 0 && i < n) {
        int tot = 0;
#pragma unroll
        for (int q = 0; q < kCpRanges; ++q) tot += part[q][c];
        if (tot == k0) {
            *radius = scores[i];
            if (rank) *rank = i;
        }
    }
}

hipError_t launch_cp_radius(const float* scores, int n, int k, float* radius, int32_t* rank, hipStream_t s) {
    // +inf when k exceeds n; NaN stays if no score can be selected
    hipLaunchKernelGGL(cp_init_kernel, dim3(1), dim3(64), 0, s, radius, rank, k > n ? INFINITY : NAN);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || k > n) return e;
    hipLaunchKernelGGL(cp_rank_kernel, dim3((n + kCpCand - 1) / kCpCand), dim3(kCpCand * kCpRanges), 0, s, scores,
                       n, k - 1, radius, rank);
    return hipGetLastError();
}

}  // namespace cord

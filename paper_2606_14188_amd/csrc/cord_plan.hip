// Small kernels of the planner: cost and terminal cotangent, projected
// gradient update, argmin over candidates, gather of the winner.
#include <hip/hip_runtime.h>

#include "cord_internal.h"

namespace cord {

// One workgroup per candidate c: J_c = |x_T[goal] - goal|^2 + reg sum u^2,
// and the cotangent of s_T (2 (x_T[goal] - goal) on the goal node, 0 else).
__global__ void plan_cost_kernel(const InstDev* inst, const float* traj, const float* u, int goal_node,
                                 float g0, float g1, float g2, float reg, float* cost, float* sT_bar) {
    const int c = blockIdx.x;
    const InstDev& I = inst[c];
    const int ns = I.n_s, nu = I.n_u, T = I.T;
    const float* xT = traj + I.traj_off + (int64_t)T * ns;
    const float d0 = xT[3 * goal_node] - g0, d1 = xT[3 * goal_node + 1] - g1, d2 = xT[3 * goal_node + 2] - g2;
    if (sT_bar) {
        for (int i = threadIdx.x; i < ns; i += blockDim.x) {
            float v = 0.f;
            if (i == 3 * goal_node) v = 2.f * d0;
            if (i == 3 * goal_node + 1) v = 2.f * d1;
            if (i == 3 * goal_node + 2) v = 2.f * d2;
            sT_bar[I.s_off + i] = v;
        }
    }
    // sum of squared controls: block reduction in a fixed order
    __shared__ float part[256];
    float acc = 0.f;
    const float* uc = u + I.u_off;
    for (int i = threadIdx.x; i < T * nu; i += blockDim.x) acc += uc[i] * uc[i];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) cost[c] = d0 * d0 + d1 * d1 + d2 * d2 + reg * part[0];
}

// u <- clip(u - step (u_bar + 2 reg u), -umax, umax)
__global__ void plan_update_kernel(float* u, const float* ubar, int64_t n, float step, float reg, float umax) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = ubar[i] + 2.f * reg * u[i];
    u[i] = fminf(fmaxf(u[i] - step * g, -umax), umax);
}

// Single workgroup: lowest cost, ties to the lowest index (NaN costs lose).
__global__ void plan_argmin_kernel(const float* cost, int n, int32_t* best, float* best_cost) {
    __shared__ float bv[256];
    __shared__ int bi[256];
    float v = 3.0e38f;
    int idx = n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const float c = cost[i];
        if (c < v) { v = c; idx = i; }
    }
    bv[threadIdx.x] = v;
    bi[threadIdx.x] = idx;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const float ov = bv[threadIdx.x + s];
            const int oi = bi[threadIdx.x + s];
            if (ov < bv[threadIdx.x] || (ov == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
                bv[threadIdx.x] = ov;
                bi[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *best = bi[0] < n ? bi[0] : 0;
        *best_cost = bv[0];
    }
}

// dst[i] = src[best * stride + i], i < len
__global__ void plan_gather_kernel(const float* src, int64_t stride, int64_t len, const int32_t* best, float* dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) dst[i] = src[(int64_t)(*best) * stride + i];
}

// worst status over candidates
__global__ void plan_status_kernel(const int32_t* st, int n, int32_t* out) {
    __shared__ int m[256];
    int v = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v = max(v, st[i]);
    m[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) m[threadIdx.x] = max(m[threadIdx.x], m[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = m[0];
}

hipError_t plan_cost(const InstDev* inst, int n_cand, const float* traj, const float* u, int goal_node,
                     const float goal[3], float reg, float* cost, float* sT_bar, hipStream_t s) {
    hipLaunchKernelGGL(plan_cost_kernel, dim3(n_cand), dim3(256), 0, s, inst, traj, u, goal_node, goal[0], goal[1],
                       goal[2], reg, cost, sT_bar);
    return hipGetLastError();
}

hipError_t plan_update(float* u, const float* ubar, int64_t n, float step, float reg, float umax, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(plan_update_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, u, ubar, n, step, reg,
                       umax);
    return hipGetLastError();
}

hipError_t plan_argmin(const float* cost, int n, int32_t* best, float* best_cost, hipStream_t s) {
    hipLaunchKernelGGL(plan_argmin_kernel, dim3(1), dim3(256), 0, s, cost, n, best, best_cost);
    return hipGetLastError();
}

hipError_t plan_gather(const float* src, int64_t stride, int64_t len, const int32_t* best, float* dst,
                       hipStream_t s) {
    if (len <= 0) return hipSuccess;
    hipLaunchKernelGGL(plan_gather_kernel, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s, src, stride, len,
                       best, dst);
    return hipGetLastError();
}

hipError_t plan_status(const int32_t* st, int n, int32_t* out, hipStream_t s) {
    hipLaunchKernelGGL(plan_status_kernel, dim3(1), dim3(256), 0, s, st, n, out);
    return hipGetLastError();
}

}  // namespace cord

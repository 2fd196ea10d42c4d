// Kernel templates (rollout, backward, linearize) and their launch wrappers;
// included by the per-size-class translation units.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/cord.h"
#include "cord_internal.h"
#include "cord_kernels.h"
#include "cord_solver.h"

namespace cord {

// Work distribution: with a.queue == null workgroup b handles ids[b]; with
// a work queue (persistent launch) every workgroup pulls the next id until
// the list is exhausted, so each one exits after a bounded number of items.
__device__ __forceinline__ int next_item(const KArgs& a, int prev, int* slot) {
    if (!a.queue) return prev < 0 ? (int)blockIdx.x : a.n_ids;
    __syncthreads();
    if (threadIdx.x == 0) *slot = atomicAdd(a.queue, 1);
    __syncthreads();
    return *slot;
}

template <int TOPO, int NT, int PPT, int NOBS, bool FRIC = false>
__global__ __launch_bounds__(NT) void rollout_kernel(KArgs a) {
    extern __shared__ float lds[];
    __shared__ int slot;
    for (int w = next_item(a, -1, &slot); w < a.n_ids; w = next_item(a, w, &slot)) {
        const int id = a.ids[w];
        const InstDev& I = a.inst[id];
        Solver<TOPO, NT, PPT, NOBS, true, FRIC> S;
        S.init(I, lds);
        S.load_state(a.s0 + I.s_off);
        const float kappa = a.use_kappa_bwd ? I.kappa_bwd : I.kappa_fwd;
        const int T = I.T, ns = I.n_s, K = a.ckpt_every;
        if (a.store == CORD_STORE_FULL) S.store_state(a.traj + I.traj_off);
        else if (a.store == CORD_STORE_CKPT) S.store_state(a.traj + a.ckpt_off[id]);
        const bool keep = a.aux_mode == 1 && I.kappa_fwd == I.kappa_bwd && a.store == CORD_STORE_FULL;
        for (int t = 0; t < T; ++t) {
            S.solve_step(a.u + I.u_off + (int64_t)t * I.n_u, kappa);
            if (keep) S.save_aux(a.aux + I.aux_off + (int64_t)t * kAuxFields * I.n);
            S.advance();
            if (a.store == CORD_STORE_FULL) {
                S.store_state(a.traj + I.traj_off + (int64_t)(t + 1) * ns);
            } else if (a.store == CORD_STORE_CKPT) {
                if ((t + 1) % K == 0 || t + 1 == T)
                    S.store_state(a.traj + a.ckpt_off[id] + (int64_t)((t + K) / K) * ns);
            } else if (t + 1 == T) {
                S.store_state(a.traj + I.s_off);
            }
        }
        if (a.final_out) S.store_state(a.final_out + I.s_off);
        if (threadIdx.x == 0) {
            if (a.status) a.status[id] = S.status;
            if (a.counters)
                for (int i = 0; i < 4; ++i) a.counters[4 * id + i] += S.cnt[i];
        }
    }
}

template <int PPT>
__device__ __forceinline__ void add_cot(float xb[PPT][3], float vb[PPT][3], const float* s, int n, int NT) {
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int p = (int)threadIdx.x + k * NT;
        if (p < n) {
#pragma unroll
            for (int c = 0; c < 3; ++c) { xb[k][c] += s[3 * p + c]; vb[k][c] += s[3 * n + 3 * p + c]; }
        }
    }
}

// Re-solve step t at kappa_bwd from the loaded state, apply its VJP, write
// u_bar[t] and add the state cotangent of traj_bar[t].
template <int TOPO, int NT, int PPT, int NOBS, bool FRIC>
__device__ __forceinline__ void adjoint_step(Solver<TOPO, NT, PPT, NOBS, true, FRIC>& S, const KArgs& a, const InstDev& I, int t,
                                             float xb[PPT][3], float vb[PPT][3], float ub[PPT][3]) {
    const int nu = I.n_u;
    if (a.aux_mode == 2 && I.kappa_fwd == I.kappa_bwd && a.store == CORD_STORE_FULL)
        S.restore_step(a.u + I.u_off + (int64_t)t * nu, a.aux + I.aux_off + (int64_t)t * kAuxFields * I.n);
    else
        S.solve_step(a.u + I.u_off + (int64_t)t * nu, I.kappa_bwd);
    float dxb[PPT][3];
    S.adjoint(xb, vb, ub, I.kappa_bwd, dxb);
#pragma unroll
    for (int k = 0; k < PPT; ++k)
        if (S.has_grip(k)) {
#pragma unroll
            for (int c = 0; c < 3; ++c) a.u_bar[I.u_off + (int64_t)t * nu + 3 * S.grip_index(k) + c] = ub[k][c];
        }
    if (a.traj_bar) {
        add_cot<PPT>(xb, vb, a.traj_bar + I.traj_off + (int64_t)t * I.n_s, I.n, NT);
        S.set_gcot(a.traj_bar + I.traj_off + (int64_t)t * I.n_s, true);
    }
}

template <int TOPO, int NT, int PPT, int NOBS, bool FRIC = false>
__global__ __launch_bounds__(NT) void backward_kernel(KArgs a) {
    extern __shared__ float lds[];
    __shared__ int slot;
    for (int w = next_item(a, -1, &slot); w < a.n_ids; w = next_item(a, w, &slot)) {
        const int id = a.ids[w];
        const InstDev& I = a.inst[id];
        Solver<TOPO, NT, PPT, NOBS, true, FRIC> S;
        S.init(I, lds);
        const int T = I.T, ns = I.n_s, nu = I.n_u, n = I.n, K = a.ckpt_every;
        const float kf = a.use_kappa_bwd ? I.kappa_bwd : I.kappa_fwd;
        float xb[PPT][3], vb[PPT][3], ub[PPT][3];
#pragma unroll
        for (int k = 0; k < PPT; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) { xb[k][c] = 0.f; vb[k][c] = 0.f; }
        if (a.traj_bar) add_cot<PPT>(xb, vb, a.traj_bar + I.traj_off + (int64_t)T * ns, n, NT);
        else if (a.sT_bar) add_cot<PPT>(xb, vb, a.sT_bar + I.s_off, n, NT);
        S.set_gcot(a.traj_bar ? a.traj_bar + I.traj_off + (int64_t)T * ns : (a.sT_bar ? a.sT_bar + I.s_off : nullptr),
                   false);

        if (a.store == CORD_STORE_FULL) {
            for (int t = T - 1; t >= 0; --t) {
                S.load_state(a.traj_in + I.traj_off + (int64_t)t * ns);
                adjoint_step<TOPO, NT, PPT, NOBS>(S, a, I, t, xb, vb, ub);
            }
        } else {
            // per-instance workspace: from the offset table, or K n_s floats
            // per instance in instance order when there is none
            float* ws = a.seg + (a.seg_off ? a.seg_off[id] : (int64_t)K * I.s_off);
            const int nseg = (T + K - 1) / K;
            for (int sg = nseg - 1; sg >= 0; --sg) {
                const int t0 = sg * K, t1 = min(T, t0 + K);
                // recompute the segment's states with the forward configuration
                S.load_state(a.traj_in + a.ckpt_off[id] + (int64_t)sg * ns);
                S.store_state(ws);
                for (int t = t0; t < t1 - 1; ++t) {
                    S.solve_step(a.u + I.u_off + (int64_t)t * nu, kf);
                    S.advance();
                    S.store_state(ws + (int64_t)(t + 1 - t0) * ns);
                }
                for (int t = t1 - 1; t >= t0; --t) {
                    S.load_state(ws + (int64_t)(t - t0) * ns);
                    adjoint_step<TOPO, NT, PPT, NOBS>(S, a, I, t, xb, vb, ub);
                }
            }
        }
        // s0_bar
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int p = (int)threadIdx.x + k * NT;
            if (p < n) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    a.s0_bar[I.s_off + 3 * p + c] = xb[k][c];
                    a.s0_bar[I.s_off + 3 * n + 3 * p + c] = vb[k][c];
                }
            }
        }
        S.get_gcot(a.s0_bar + I.s_off);
        if (threadIdx.x == 0) {
            if (a.status) a.status[id] = S.status;
            if (a.counters)
                for (int i = 0; i < 4; ++i) a.counters[4 * id + i] += S.cnt[i];
        }
    }
}

// One workgroup per (instance, step).  Dense rows of A_t/B_t come from one
// VJP per free DoF row (rows written coalesced); JVP tangents from the
// forward tangent map.
template <int TOPO, int NT, int PPT, int NOBS, bool FRIC = false>
__global__ __launch_bounds__(NT) void linearize_kernel(KArgs a) {
    extern __shared__ float lds[];
    const int id = a.ids[blockIdx.x];
    const InstDev& I = a.inst[id];
    const int t = blockIdx.y;
    if (t >= I.T) return;
    if (a.redo && !a.redo[I.t_off + t]) return;   // only the steps the direct kernel flagged
    Solver<TOPO, NT, PPT, NOBS, true, FRIC> S;
    S.init(I, lds);
    const int n = I.n, ns = I.n_s, nu = I.n_u;
    const float kb = I.kappa_bwd, dt = I.dt, idt = 1.0f / I.dt;
    S.load_state(a.traj_in + I.traj_off + (int64_t)t * ns);
    if (a.aux_mode == 2 && I.kappa_fwd == I.kappa_bwd)
        S.restore_step(a.u + I.u_off + (int64_t)t * nu, a.aux + I.aux_off + (int64_t)t * kAuxFields * n);
    else
        S.solve_step(a.u + I.u_off + (int64_t)t * nu, kb);

    if (a.A || a.Bm) {
        const int64_t aoff = a.lin_zero_off ? 0 : I.A_off, boff = a.lin_zero_off ? 0 : I.B_off;
        float* A = a.A ? a.A + aoff + (int64_t)t * ns * ns : nullptr;
        float* Bm = a.Bm ? a.Bm + boff + (int64_t)t * ns * nu : nullptr;
        float xb[PPT][3], vb[PPT][3], ub[PPT][3];
        for (int r = 0; r < 3 * n; ++r) {
            const int pr = r / 3, cr = r - 3 * pr;
            int gr = -1;
            for (int j = 0; j < I.n_grip; ++j)
                if (I.grip_node[j] == pr && !I.grip_mode) gr = j;
            float* Ax = A ? A + (int64_t)r * ns : nullptr;
            float* Av = A ? A + (int64_t)(3 * n + r) * ns : nullptr;
            if (gr >= 0) {
                // x+_j = x_j + dt u_g ; v+_j = u_g
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    const int p = (int)threadIdx.x + k * NT;
                    if (p >= n || !A) continue;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        Ax[3 * p + c] = (p == pr && c == cr) ? 1.f : 0.f;
                        Ax[3 * n + 3 * p + c] = 0.f;
                        Av[3 * p + c] = 0.f;
                        Av[3 * n + 3 * p + c] = 0.f;
                    }
                }
                if (Bm && (int)threadIdx.x < nu) {
                    const int col = threadIdx.x;
                    Bm[(int64_t)r * nu + col] = (col == 3 * gr + cr) ? dt : 0.f;
                    Bm[(int64_t)(3 * n + r) * nu + col] = (col == 3 * gr + cr) ? 1.f : 0.f;
                }
                continue;
            }
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int p = (int)threadIdx.x + k * NT;
#pragma unroll
                for (int c = 0; c < 3; ++c) { xb[k][c] = (p == pr && c == cr) ? 1.f : 0.f; vb[k][c] = 0.f; }
            }
            float dxb[PPT][3];
            S.set_gcot(nullptr, false);
            S.adjoint(xb, vb, ub, kb, dxb);
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int p = (int)threadIdx.x + k * NT;
                if (p >= n) continue;
                if (A) {
                    // row r of dv+/dx is (row r of dx+/dx - e_r)/dt = dxb/dt
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        Ax[3 * p + c] = xb[k][c];
                        Ax[3 * n + 3 * p + c] = vb[k][c];
                        Av[3 * p + c] = dxb[k][c] * idt;
                        Av[3 * n + 3 * p + c] = vb[k][c] * idt;
                    }
                }
                if (Bm && S.has_grip(k)) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        Bm[(int64_t)r * nu + 3 * S.grip_index(k) + c] = ub[k][c];
                        Bm[(int64_t)(3 * n + r) * nu + 3 * S.grip_index(k) + c] = ub[k][c] * idt;
                    }
                }
                // penalty grasp: columns of the gripper positions
                if (A && S.pen[k] >= 0) {
                    const float* G = S.pg(k);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        Ax[6 * n + 3 * S.pen[k] + c] = G[10 + c];
                        Av[6 * n + 3 * S.pen[k] + c] = G[10 + c] * idt;
                    }
                }
            }
        }
        if (I.grip_mode) {
            // rows of g+ = g + dt u
            for (int r = 6 * n; r < ns; ++r) {
                if (A)
                    for (int col = threadIdx.x; col < ns; col += NT) A[(int64_t)r * ns + col] = col == r ? 1.f : 0.f;
                if (Bm)
                    for (int col = threadIdx.x; col < nu; col += NT) Bm[(int64_t)r * nu + col] = col == r - 6 * n ? dt : 0.f;
            }
        }
    }

    if (a.jvp_out) {
        const int kt = a.jvp_k;
        float dx[PPT][3], dv[PPT][3], du[PPT][3], ox[PPT][3], ov[PPT][3];
        for (int i = 0; i < kt; ++i) {
            const int64_t sbase = (int64_t)kt * I.tns_off + ((int64_t)t * kt + i) * ns;
            const int64_t ubase = (int64_t)kt * I.u_off + ((int64_t)t * kt + i) * nu;
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int p = (int)threadIdx.x + k * NT;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    dx[k][c] = (a.jvp_ds && p < n) ? a.jvp_ds[sbase + 3 * p + c] : 0.f;
                    dv[k][c] = (a.jvp_ds && p < n) ? a.jvp_ds[sbase + 3 * n + 3 * p + c] : 0.f;
                    du[k][c] = (a.jvp_du && S.has_grip(k)) ? a.jvp_du[ubase + 3 * S.grip_index(k) + c] : 0.f;
                }
                if (S.pen[k] >= 0)
                    for (int c = 0; c < 3; ++c) S.pg(k)[13 + c] = a.jvp_ds ? a.jvp_ds[sbase + 6 * n + 3 * S.pen[k] + c] : 0.f;
            }
            S.tangent(dx, dv, du, ox, ov, kb);
#pragma unroll
            for (int k = 0; k < PPT; ++k)
                if (S.pen[k] >= 0)
                    for (int c = 0; c < 3; ++c) a.jvp_out[sbase + 6 * n + 3 * S.pen[k] + c] = S.pg(k)[13 + c];
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int p = (int)threadIdx.x + k * NT;
                if (p >= n) continue;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    a.jvp_out[sbase + 3 * p + c] = ox[k][c];
                    a.jvp_out[sbase + 3 * n + 3 * p + c] = ov[k][c];
                }
            }
        }
    }
    if (threadIdx.x == 0 && a.status) atomicMax(&a.status[id], S.status);
    if (threadIdx.x == 0 && a.counters)
        for (int i = 0; i < 4; ++i) atomicAdd(&a.counters[4 * id + i], S.cnt[i]);
}

// ----------------------------------------------------------------- launch table
template <int TOPO, int NT, int PPT, int NOBS>
struct Launch {
    static constexpr size_t kLds = sizeof(float) * lds_floats<NT, PPT>();
    static hipError_t rollout(const KArgs& a, int nblk, hipStream_t s) {
        hipLaunchKernelGGL((rollout_kernel<TOPO, NT, PPT, NOBS>), dim3(nblk), dim3(NT), kLds, s, a);
        return hipGetLastError();
    }
    static hipError_t backward(const KArgs& a, int nblk, hipStream_t s) {
        hipLaunchKernelGGL((backward_kernel<TOPO, NT, PPT, NOBS>), dim3(nblk), dim3(NT), kLds, s, a);
        return hipGetLastError();
    }
    static hipError_t linearize(const KArgs& a, int nblk, int tmax, hipStream_t s) {
        hipLaunchKernelGGL((linearize_kernel<TOPO, NT, PPT, NOBS>), dim3(nblk, tmax), dim3(NT), kLds, s, a);
        return hipGetLastError();
    }
    // the same kernels compiled with the friction cone (instances with mu > 0)
    static hipError_t rollout_f(const KArgs& a, int nblk, hipStream_t s) {
        hipLaunchKernelGGL((rollout_kernel<TOPO, NT, PPT, NOBS, true>), dim3(nblk), dim3(NT), kLds, s, a);
        return hipGetLastError();
    }
    static hipError_t backward_f(const KArgs& a, int nblk, hipStream_t s) {
        hipLaunchKernelGGL((backward_kernel<TOPO, NT, PPT, NOBS, true>), dim3(nblk), dim3(NT), kLds, s, a);
        return hipGetLastError();
    }
    static hipError_t linearize_f(const KArgs& a, int nblk, int tmax, hipStream_t s) {
        hipLaunchKernelGGL((linearize_kernel<TOPO, NT, PPT, NOBS, true>), dim3(nblk, tmax), dim3(NT), kLds, s, a);
        return hipGetLastError();
    }
    static int blocks_per_cu(int which) {
        int nb = 0;
        hipError_t e = which == 0
            ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, rollout_kernel<TOPO, NT, PPT, NOBS>, NT, kLds)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, backward_kernel<TOPO, NT, PPT, NOBS>, NT, kLds);
        return (e == hipSuccess && nb > 0) ? nb : 1;
    }
};

#define CORD_CFG(TOPO, NT, PPT, NOBS) \
    {TOPO, NT, PPT, NOBS, Launch<TOPO, NT, PPT, NOBS>::kLds, &Launch<TOPO, NT, PPT, NOBS>::rollout, \
     &Launch<TOPO, NT, PPT, NOBS>::backward, &Launch<TOPO, NT, PPT, NOBS>::linearize, \
     &Launch<TOPO, NT, PPT, NOBS>::blocks_per_cu, &Launch<TOPO, NT, PPT, NOBS>::rollout_f, \
     &Launch<TOPO, NT, PPT, NOBS>::backward_f, &Launch<TOPO, NT, PPT, NOBS>::linearize_f}

}  // namespace cord

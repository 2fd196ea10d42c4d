// Internal host/device structures of libcord (not part of the C ABI).
#pragma once
#include <stdint.h>

namespace cord {

constexpr int kRope = 0;
constexpr int kCloth = 1;

constexpr int kObsGround = 0;
constexpr int kObsSphere = 1;
constexpr int kObsBox = 2;

constexpr int kMaxObs = 4;      // obstacle slots held in registers per particle
constexpr int kMaxGrip = 4;

// Per-instance constants, uploaded once at create time.  Offsets are in
// floats into the concatenated batch buffers.
struct alignas(16) InstDev {
    int32_t kind, nx, ny, n;
    int32_t T, n_grip, n_obs, n_s;
    int32_t n_u, grip_mode, t_off, pad2;   // t_off: sum T (per-step flag tables)
    int32_t grip_node[kMaxGrip];
    int32_t obs_type[kMaxObs];
    float obs[kMaxObs][8];          // sphere: cx cy cz r; box: cx cy cz hx hy hz rho
    float h, mass, k_struct, k_shear;
    float k_bend, dt, gamma, kappa_fwd;
    float kappa_bwd, g0, g1, g2;
    float D_max, kappa_h, r_g, mu;   // mu: friction coefficient (0: frictionless)
    int64_t s_off;      // sum n_s
    int64_t u_off;      // sum T n_u
    int64_t traj_off;   // sum (T+1) n_s
    int64_t tns_off;    // sum T n_s   (JVP blocks are k * this)
    int64_t A_off;      // sum T n_s^2
    int64_t B_off;      // sum T n_s n_u
    int64_t aux_off;    // sum kAuxFields T n (step internals)
};

// Step internals kept per node and step: q* - x (3), the stage-2 correction
// (3), the contact multiplier and gap of each obstacle slot.
constexpr int kAuxFields = 6 + 2 * kMaxObs;

// Kernel arguments shared by the three kernels.
struct KArgs {
    const InstDev* inst;
    const int32_t* ids;        // instance ids handled by this launch
    int32_t n_ids;
    int32_t store;             // CORD_STORE_*
    int32_t ckpt_every;
    int32_t use_kappa_bwd;
    const int64_t* ckpt_off;   // per-instance checkpoint block offset (CKPT)
    const float* s0;
    const float* u;
    float* traj;               // rollout: output; backward/linearize: input
    float* final_out;          // rollout: optional copy of s_T
    const float* traj_in;
    const float* traj_bar;
    const float* sT_bar;
    float* s0_bar;
    float* u_bar;
    float* seg;                // backward: per-instance segment workspace
    const int64_t* seg_off;    // per-instance workspace offset (floats)
    float* A;
    float* Bm;
    int32_t jvp_k;
    const float* jvp_ds;
    const float* jvp_du;
    float* jvp_out;
    int32_t* status;
    uint32_t* counters;
    int32_t* queue;            // persistent launch: work-queue counter (zeroed before launch), or null
    int32_t lin_zero_off;      // linearize: write A/B at offset 0 (single-instance outputs)
    float* aux;                // step internals, or null
    int32_t aux_mode;          // 1: rollout writes them; 2: backward / linearize read them
    float* kept;               // direct rope linearization: scratch slots, or null
    int32_t kept_tg;           // workgroup slots per CU in that scratch table
    uint32_t* lin_stats;       // direct linearization counters: [0] scratch-slot overlaps, [1] steps redone
    int32_t* redo;             // per (instance, step) at t_off + t: the direct linearization sets 1 where a
                               // band factor met a non-positive pivot; the iterative linearize kernel run
                               // with this set does only those steps (null: every step)
};

}  // namespace cord

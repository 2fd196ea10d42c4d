// Device-side solver of one rope/cloth instance per workgroup (gfx950).
//
// One workgroup owns one instance for the whole horizon.  Thread t owns the
// particles p = t + k*NT (k < PPT).  Per-particle state (x, v, the stage-1
// increment d = q* - x, the stage-2 correction, contact multipliers, the
// per-spring Hessian data) lives in VGPRs across all time steps; the only
// vectors that neighbours read (x, d, the CG direction, the stage-2
// correction) are mirrored in LDS as structure-of-arrays, so neighbour reads
// of consecutive lanes hit consecutive banks.  HBM is touched only for
// controls, states/trajectories, cotangents and Jacobian blocks.
//
// The step follows Sec. 4.1 of the paper (two-stage solver, contact
// smoothing); the derivatives follow its "Differentiating Through
// Simulation" paragraph and eq. (diff-sim).  Design choices that differ from
// the paper's (dense GPU factorizations in JAX): every linear solve is a
// matrix-free block-Jacobi preconditioned conjugate gradient whose
// Hessian-vector product is a nearest-neighbour stencil evaluated from the
// LDS mirror; reductions are DPP wave reductions plus one LDS exchange.
#pragma once

#include <hip/hip_runtime.h>

#include "cord_internal.h"

namespace cord {

// ----------------------------------------------------------------- status
constexpr int kStOK = 0;
constexpr int kStNewton = 1;
constexpr int kStNotPD = 2;
constexpr int kStQP = 3;
constexpr int kStNonFinite = 4;

// ----------------------------------------------------------------- solver settings
constexpr int kNewtonMax = 40;
constexpr int kLineSearchMax = 30;
constexpr int kIpmMax = 60;
constexpr int kIpmFricMax = 150;        // friction cone: Newton steps over all relaxation levels
constexpr int kPcgMax = 300;
constexpr int kMinresMax = 600;
constexpr float kMinresAccept = 1e-4f;  // true relative residual accepted after the last MINRES pass
constexpr float kPcgTolInner = 1e-3f;   // relative residual (preconditioned norm), Newton / IPM
constexpr float kPcgTolAdj = 1e-6f;     // adjoint / tangent solves
constexpr float kTolForce = 1e-5f;      // x force scale (m|g| + 1e-3 m/dt^2 h)
constexpr float kTolGap = 2e-7f;        // x (h + |phi|)
constexpr float kTolCompl = 1e-5f;      // x kappa

// ----------------------------------------------------------------- reductions
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float rdlane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
// Butterfly inside rows of 16 (quad_perm, half-mirror, mirror), then the
// four row results via readlane.  Every lane gets the same bits: IEEE
// addition is commutative, so both partners of a swap compute equal sums.
__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_mov<0xB1>(v);
    v += dpp_mov<0x4E>(v);
    v += dpp_mov<0x141>(v);
    v += dpp_mov<0x140>(v);
    return (rdlane(v, 0) + rdlane(v, 16)) + (rdlane(v, 32) + rdlane(v, 48));
}
__device__ __forceinline__ float wave_max(float v) {
    v = fmaxf(v, dpp_mov<0xB1>(v));
    v = fmaxf(v, dpp_mov<0x4E>(v));
    v = fmaxf(v, dpp_mov<0x141>(v));
    v = fmaxf(v, dpp_mov<0x140>(v));
    return fmaxf(fmaxf(rdlane(v, 0), rdlane(v, 16)), fmaxf(rdlane(v, 32), rdlane(v, 48)));
}
__device__ __forceinline__ float wave_min(float v) {
    v = fminf(v, dpp_mov<0xB1>(v));
    v = fminf(v, dpp_mov<0x4E>(v));
    v = fminf(v, dpp_mov<0x141>(v));
    v = fminf(v, dpp_mov<0x140>(v));
    return fminf(fminf(rdlane(v, 0), rdlane(v, 16)), fminf(rdlane(v, 32), rdlane(v, 48)));
}

// NaN-propagating max inside a thread.  fmaxf drops NaNs, so before a wave
// reduction a non-finite value is mapped to the sentinel kBad (finite and
// larger than any real residual); a reduced value >= kBad means some lane
// held a NaN or Inf.
constexpr float kBad = 3.0e38f;
__device__ __forceinline__ float nmax(float a, float b) { return (a != a || b != b) ? __int_as_float(0x7fc00000) : fmaxf(a, b); }
__device__ __forceinline__ float finite_key(float a) { return (a == a && a < kBad) ? a : kBad; }

// ----------------------------------------------------------------- 3x3 symmetric helpers
// (a b c; b d e; c e f) stored as {a, b, c, d, e, f}
__device__ __forceinline__ void sym_inv(const float m[6], float o[6]) {
    const float a = m[0], b = m[1], c = m[2], d = m[3], e = m[4], f = m[5];
    const float c00 = d * f - e * e, c01 = c * e - b * f, c02 = b * e - c * d;
    const float c11 = a * f - c * c, c12 = b * c - a * e, c22 = a * d - b * b;
    const float det = a * c00 + b * c01 + c * c02;
    const float id = 1.0f / det;
    o[0] = c00 * id; o[1] = c01 * id; o[2] = c02 * id;
    o[3] = c11 * id; o[4] = c12 * id; o[5] = c22 * id;
}
// entry (r, c) of a symmetric 3x3 stored as {a, b, c, d, e, f}
__device__ __forceinline__ float sym_at(const float m[6], int r, int c) {
    const int i = r <= c ? r : c, j = r <= c ? c : r;
    return m[i == 0 ? j : i == 1 ? 2 + j : 5];
}
__device__ __forceinline__ void sym_to_full3(const float s[6], float m[3][3]) {
    m[0][0] = s[0]; m[0][1] = s[1]; m[0][2] = s[2];
    m[1][0] = s[1]; m[1][1] = s[3]; m[1][2] = s[4];
    m[2][0] = s[2]; m[2][1] = s[4]; m[2][2] = s[5];
}
// positive definite by Sylvester's criterion
__device__ __forceinline__ bool sym_pd(const float m[6]) {
    const float m2 = m[0] * m[3] - m[1] * m[1];
    const float m3 = m[0] * (m[3] * m[5] - m[4] * m[4]) - m[1] * (m[1] * m[5] - m[4] * m[2]) +
                     m[2] * (m[1] * m[4] - m[3] * m[2]);
    return m[0] > 0.f && m2 > 0.f && m3 > 0.f;
}
__device__ __forceinline__ void sym_mul(const float m[6], const float r[3], float o[3]) {
    o[0] = m[0] * r[0] + m[1] * r[1] + m[2] * r[2];
    o[1] = m[1] * r[0] + m[3] * r[1] + m[4] * r[2];
    o[2] = m[2] * r[0] + m[4] * r[1] + m[5] * r[2];
}
__device__ __forceinline__ void sym_add_outer(float m[6], float w, const float e[3]) {
    m[0] += w * e[0] * e[0]; m[1] += w * e[0] * e[1]; m[2] += w * e[0] * e[2];
    m[3] += w * e[1] * e[1]; m[4] += w * e[1] * e[2]; m[5] += w * e[2] * e[2];
}
__device__ __forceinline__ float dot3(const float a[3], const float b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// ----------------------------------------------------------------- obstacles
// Signed distance and its gradient (the contact normal).  Ground z = 0;
// sphere |y - c| - r; rounded box with b = |y - c| - (h - rho):
// |max(b,0)| - rho outside, max_i b_i - rho inside (ties -> lowest axis).
__device__ __forceinline__ void sdf_eval(int type, const float* ob, const float y[3], float& phi, float n[3]) {
    if (type == kObsGround) {
        phi = y[2]; n[0] = 0.f; n[1] = 0.f; n[2] = 1.f;
    } else if (type == kObsSphere) {
        float q[3] = {y[0] - ob[0], y[1] - ob[1], y[2] - ob[2]};
        float L = sqrtf(dot3(q, q));
        phi = L - ob[3];
        if (L > 0.f) { float il = 1.0f / L; n[0] = q[0] * il; n[1] = q[1] * il; n[2] = q[2] * il; }
        else { n[0] = 0.f; n[1] = 0.f; n[2] = 1.f; }
    } else {
        float s[3], b[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float q = y[c] - ob[c];
            s[c] = q >= 0.f ? 1.f : -1.f;
            b[c] = s[c] * q - (ob[3 + c] - ob[6]);
        }
        if (b[0] > 0.f || b[1] > 0.f || b[2] > 0.f) {
            float m[3] = {fmaxf(b[0], 0.f), fmaxf(b[1], 0.f), fmaxf(b[2], 0.f)};
            float L = sqrtf(dot3(m, m));
            float il = 1.0f / L;
            phi = L - ob[6];
#pragma unroll
            for (int c = 0; c < 3; ++c) n[c] = s[c] * m[c] * il;
        } else {
            // deepest face; ties go to the lowest axis (no dynamic indexing,
            // which would force the arrays out of registers)
            int k = 0;
            float bk = b[0];
            if (b[1] > bk) { k = 1; bk = b[1]; }
            if (b[2] > bk) { k = 2; bk = b[2]; }
            phi = bk - ob[6];
            n[0] = k == 0 ? s[0] : 0.f;
            n[1] = k == 1 ? s[1] : 0.f;
            n[2] = k == 2 ? s[2] : 0.f;
        }
    }
}

// Hessian of the signed distance (curvature of the contact normal).
__device__ __forceinline__ void sdf_hess(int type, const float* ob, const float y[3], float H[6]) {
#pragma unroll
    for (int i = 0; i < 6; ++i) H[i] = 0.f;
    if (type == kObsSphere) {
        float q[3] = {y[0] - ob[0], y[1] - ob[1], y[2] - ob[2]};
        float L = sqrtf(dot3(q, q));
        if (L > 0.f) {
            float il = 1.0f / L;
            float n[3] = {q[0] * il, q[1] * il, q[2] * il};
            H[0] = (1.f - n[0] * n[0]) * il; H[1] = -n[0] * n[1] * il; H[2] = -n[0] * n[2] * il;
            H[3] = (1.f - n[1] * n[1]) * il; H[4] = -n[1] * n[2] * il; H[5] = (1.f - n[2] * n[2]) * il;
        }
    } else if (type == kObsBox) {
        float s[3], b[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float q = y[c] - ob[c];
            s[c] = q >= 0.f ? 1.f : -1.f;
            b[c] = s[c] * q - (ob[3 + c] - ob[6]);
        }
        if (b[0] > 0.f || b[1] > 0.f || b[2] > 0.f) {
            float pm[3] = {b[0] > 0.f ? 1.f : 0.f, b[1] > 0.f ? 1.f : 0.f, b[2] > 0.f ? 1.f : 0.f};
            float m[3] = {fmaxf(b[0], 0.f), fmaxf(b[1], 0.f), fmaxf(b[2], 0.f)};
            float L = sqrtf(dot3(m, m));
            float il = 1.0f / L;
            float mh[3] = {m[0] * il, m[1] * il, m[2] * il};
            float ds[3] = {s[0] * pm[0], s[1] * pm[1], s[2] * pm[2]};
            H[0] = ds[0] * ds[0] * (pm[0] - mh[0] * mh[0]) * il;
            H[1] = ds[0] * ds[1] * (-mh[0] * mh[1]) * il;
            H[2] = ds[0] * ds[2] * (-mh[0] * mh[2]) * il;
            H[3] = ds[1] * ds[1] * (pm[1] - mh[1] * mh[1]) * il;
            H[4] = ds[1] * ds[2] * (-mh[1] * mh[2]) * il;
            H[5] = ds[2] * ds[2] * (pm[2] - mh[2] * mh[2]) * il;
        }
    }
}

// ----------------------------------------------------------------- topology
// Spring slots of a particle.  Rope: neighbours +1, -1.  Cloth (node
// (ix, iy) = iy*nx + ix): structural (+-1,0),(0,+-1); shear (+-1,+-1);
// bend (+-2,0),(0,+-2).
template <int TOPO> struct Topo;
template <> struct Topo<kRope> {
    static constexpr int NS = 2;
    __device__ static constexpr int dx(int s) { return s == 0 ? 1 : -1; }
    __device__ static constexpr int dy(int) { return 0; }
    __device__ static constexpr int type(int) { return 0; }
};
template <> struct Topo<kCloth> {
    static constexpr int NS = 12;
    __device__ static constexpr int dx(int s) {
        return s == 0 ? 1 : s == 1 ? -1 : s == 4 ? 1 : s == 5 ? -1 : s == 6 ? 1 : s == 7 ? -1 : s == 8 ? 2 : s == 9 ? -2 : 0;
    }
    __device__ static constexpr int dy(int s) {
        return s == 2 ? 1 : s == 3 ? -1 : s == 4 ? 1 : s == 5 ? -1 : s == 6 ? -1 : s == 7 ? 1 : s == 10 ? 2 : s == 11 ? -2 : 0;
    }
    __device__ static constexpr int type(int s) { return s < 4 ? 0 : s < 8 ? 1 : 2; }
};

// LDS floats used by one workgroup.
template <int NT, int PPT>
constexpr int lds_floats() { return 12 * NT * PPT + 64 + 16 * kMaxGrip; }

// ----------------------------------------------------------------- solver
// FALLBACK = false compiles the solves without MINRES and the hard-contact
// polish (for the direct rope linearization, whose band factorizations
// detect an indefinite dF/dq* themselves and hand such steps to the
// iterative kernel, which has both).
template <int TOPO, int NT, int PPT, int NOBS, bool FALLBACK = true, bool FRIC = false>
struct Solver {
    static constexpr int NM = NT * PPT;
    static constexpr int NS = Topo<TOPO>::NS;
    using TP = Topo<TOPO>;

    // LDS mirrors (SoA, component c at offset c*NM)
    float* X;    // positions at step start
    float* D;    // stage-1 increment d = q* - x
    float* V;    // exchange vector (CG direction, adjoints, tangents)
    float* DL;   // stage-2 correction / line-search step
    float* rb;   // reduction scratch (2 x 16)
    float* GR;   // penalty grasp, 16 floats per gripper (read and written only by
                 // the thread owning its node): g, g+, D, dD/dc, cotangent of g, tangent of g
    int rslot;

    // instance constants
    int n, nx, ny, ngrip, nobs;
    float h, mass, dt, gam, mdt2, kb, tolF, fscale;
    float g[3];
    float kS[3], rS[3];
    int otype[NOBS];
    float ob[NOBS][7];

    // particles
    int grip[PPT];          // -1 free, else gripper index; -2 inactive slot
    int pen[PPT];           // penalty grasp: gripper pulling this (free) particle, or -1
    int pmode;
    float Dmax, khal, rgrip;
    int px[PPT], py[PPT];   // grid coordinates (cloth)
    float x[PPT][3], v[PPT][3], d[PPT][3], dl[PPT][3], ug[PPT][3];
    float se[PPT][NS][3], sa[PPT][NS], sb[PPT][NS];
    float Bd[PPT][6], Mi[PPT][6];
    // rope, one particle per lane: rows of the inverse of the 6 x 6 block of
    // the particle pair (2q, 2q + 1) -- own columns (symmetric) and the
    // partner's columns (row-major)
    float Pd[PPT][6], Pc[PPT][9];
    float bw[PPT][3];       // rope: bending weights of the centres p-1, p, p+1 (zero if not a centre)
    float cn[PPT][NOBS][3], cphi[PPT][NOBS], clam[PPT][NOBS], cgap[PPT][NOBS];
    // friction (mu > 0; compiled only into the FRIC instantiation): the tangential
    // slack of each pair in its frame (n, t1, t2), and per particle the sum
    // of its pairs' stiffness blocks (the contact part of the stage-2 matrix)
    static constexpr int kFP = FRIC ? PPT : 1;
    static constexpr int kFO = FRIC ? NOBS : 1;
    float fmu;
    float cy1[kFP][kFO], cy2[kFP][kFO];
    float ck[kFP][6];

    int status;
    uint32_t cnt[4];   // Newton its, PCG its, interior-point its, steps
    float pcpd;        // 1 if every preconditioner block of this thread is positive definite

    __device__ __forceinline__ int pidx(int k) const { return (int)threadIdx.x + k * NT; }
    __device__ __forceinline__ bool active(int k) const { return grip[k] != -2; }
    __device__ __forceinline__ bool isfree(int k) const { return grip[k] == -1; }
    // particle k is moved by a gripper (either grasp mode) / that gripper's index
    __device__ __forceinline__ bool has_grip(int k) const { return grip[k] >= 0 || pen[k] >= 0; }
    __device__ __forceinline__ int grip_index(int k) const { return grip[k] >= 0 ? grip[k] : pen[k]; }
    __device__ __forceinline__ float* pg(int k) const { return GR + 16 * pen[k]; }

    __device__ __forceinline__ void init(const InstDev& I, float* lds) {
        X = lds; D = X + 3 * NM; V = D + 3 * NM; DL = V + 3 * NM; rb = DL + 3 * NM; GR = rb + 64; rslot = 0;
        pmode = I.grip_mode; Dmax = I.D_max; khal = I.kappa_h; rgrip = I.r_g;
        fmu = FRIC ? I.mu : 0.f;
        n = I.n; nx = I.nx; ny = I.ny; ngrip = I.n_grip; nobs = I.n_obs;
        h = I.h; mass = I.mass; dt = I.dt; gam = I.gamma; mdt2 = I.mass / (I.dt * I.dt);
        kb = (TOPO == kRope) ? I.k_bend : 0.f;
        g[0] = I.g0; g[1] = I.g1; g[2] = I.g2;
        kS[0] = I.k_struct; kS[1] = I.k_shear; kS[2] = I.k_bend;
        rS[0] = I.h; rS[1] = I.h * 1.41421356237309515f; rS[2] = 2.f * I.h;
        // force scale: the weight of a node plus the inertial force of a
        // 1e-3 h displacement in one step
        float gn = fmaxf(fabsf(g[0]), fmaxf(fabsf(g[1]), fabsf(g[2])));
        fscale = mass * gn + 1e-3f * mdt2 * h;
        tolF = kTolForce * fscale;
#pragma unroll
        for (int o = 0; o < NOBS; ++o) {
            otype[o] = I.obs_type[o];
#pragma unroll
            for (int c = 0; c < 7; ++c) ob[o][c] = I.obs[o][c];
        }
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            int p = pidx(k);
            int gk = (p < n) ? -1 : -2;
            for (int j = 0; j < I.n_grip; ++j)
                if (I.grip_node[j] == p) gk = j;
            // penalty grasp: the node stays free and its gripper is tracked in GR
            pen[k] = (pmode && gk >= 0) ? gk : -1;
            grip[k] = (pmode && gk >= 0) ? -1 : gk;
            if (pen[k] >= 0)
                for (int f = 0; f < 16; ++f) pg(k)[f] = 0.f;
            px[k] = (TOPO == kCloth) ? p % nx : p;
            py[k] = (TOPO == kCloth) ? p / nx : 0;
            // d/dx_p of the bending energy: the centres cc = p-1, p, p+1 that
            // lie in [1, n-2] carry the stencil (1, -2, 1), weighted 1, -2, 1
#pragma unroll
            for (int j = -1; j <= 1; ++j) {
                const int cc = p + j;
                bw[k][j + 1] = (TOPO == kRope && cc >= 1 && cc <= n - 2) ? ((j == 0) ? -2.f : 1.f) * kb : 0.f;
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) { x[k][c] = 0.f; v[k][c] = 0.f; d[k][c] = 0.f; dl[k][c] = 0.f; ug[k][c] = 0.f; }
        }
        status = kStOK;
        cnt[0] = cnt[1] = cnt[2] = cnt[3] = 0;
    }

    // Orders the LDS mirrors between lanes.  A single wavefront performs its
    // LDS reads and writes in issue order, so it needs only a compiler-level
    // fence (no s_barrier, no wait for outstanding LDS operations).
    __device__ __forceinline__ void sync() {
        if constexpr (NT == 64) {
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        } else {
            __syncthreads();
        }
    }

    // -------------------------------------------------- friction helpers
    __device__ __forceinline__ bool friction() const {
        if constexpr (FRIC) return fmu > 0.f;
        else return false;
    }
    __device__ __forceinline__ static constexpr int fk(int k) { return FRIC ? k : 0; }
    __device__ __forceinline__ static constexpr int fo(int o) { return FRIC ? o : 0; }
    // unit tangents completing n to an orthonormal frame (any choice: the
    // cone and its barrier are invariant under rotations about n)
    __device__ __forceinline__ static void tframe(const float n[3], float t1[3], float t2[3]) {
        const float a0 = fabsf(n[0]) < 0.9f ? 1.f : 0.f, a1 = 1.f - a0;   // a = e_x, or e_y
        float c[3] = {-n[2] * a1, n[2] * a0, n[0] * a1 - n[1] * a0};       // n x a
        const float il = 1.f / sqrtf(dot3(c, c));
#pragma unroll
        for (int i = 0; i < 3; ++i) t1[i] = c[i] * il;
        t2[0] = n[1] * t1[2] - n[2] * t1[1];
        t2[1] = n[2] * t1[0] - n[0] * t1[2];
        t2[2] = n[0] * t1[1] - n[1] * t1[0];
    }
    // the largest a > 0 with y + a dy inside the cone {y0 > mu |(y1, y2)|}
    // (y inside): the smallest positive root of Q(a) = y0(a)^2 - mu^2 |y_t(a)|^2
    // or of y0(a), whichever comes first
    __device__ __forceinline__ static float cone_step(float y0, float y1, float y2, float d0, float d1, float d2,
                                                      float m2) {
        float am = 1e30f;
        if (d0 < 0.f) am = -y0 / d0;
        const float A = d0 * d0 - m2 * (d1 * d1 + d2 * d2);
        const float B = 2.f * (y0 * d0 - m2 * (y1 * d1 + y2 * d2));
        const float C = y0 * y0 - m2 * (y1 * y1 + y2 * y2);
        const float disc = B * B - 4.f * A * C;
        if (disc >= 0.f) {
            const float q = -0.5f * (B + copysignf(sqrtf(disc), B));
            if (q != 0.f) {
                const float r1 = C / q;
                if (r1 > 0.f) am = fminf(am, r1);
            }
            if (A != 0.f) {
                const float r2 = q / A;
                if (r2 > 0.f) am = fminf(am, r2);
            }
        }
        return am;
    }
    // One pair with friction at the stage-2 correction D = dl[k]: u = d + D
    // (the node's displacement over the step), y_n = phi + n.D, tau = T u,
    // Q = y_n^2 - mu^2 |tau|^2, a = y_n n - mu^2 tau, w = kappa / Q; the
    // force is w a.  Returns false for an invalid pair.
    struct Pair {
        float n[3], H[6], u[3], tau[3], a[3], Hu[3], HD[3];
        float yn, nu, Q, w;
    };
    __device__ __forceinline__ void fric_pair(int k, int o, float kappa, const float yst[3], Pair& P) const {
        const float m2 = fmu * fmu;
#pragma unroll
        for (int c = 0; c < 3; ++c) { P.n[c] = cn[k][o][c]; P.u[c] = d[k][c] + dl[k][c]; }
        sdf_hess(otype[o], ob[o], yst, P.H);
        P.yn = cphi[k][o] + dot3(P.n, dl[k]);
        P.nu = dot3(P.n, P.u);
#pragma unroll
        for (int c = 0; c < 3; ++c) P.tau[c] = P.u[c] - P.nu * P.n[c];
        P.Q = P.yn * P.yn - m2 * dot3(P.tau, P.tau);
        P.w = kappa / P.Q;
#pragma unroll
        for (int c = 0; c < 3; ++c) P.a[c] = P.yn * P.n[c] - m2 * P.tau[c];
        sym_mul(P.H, P.u, P.Hu);
        sym_mul(P.H, dl[k], P.HD);
    }
    // ck[k] = sum of the pairs' blocks K_c = w (2 a a^T / Q - (1 + mu^2) n n^T + mu^2 I)
    // (minus the derivative of the force in D) at relaxation kappa
    __device__ __forceinline__ void fric_blocks(float kappa) {
        const float m2 = fmu * fmu;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
#pragma unroll
            for (int i = 0; i < 6; ++i) ck[fk(k)][i] = 0.f;
            if (!isfree(k)) continue;
            float yst[3] = {x[k][0] + d[k][0], x[k][1] + d[k][1], x[k][2] + d[k][2]};
#pragma unroll
            for (int o = 0; o < NOBS; ++o) {
                if (o >= nobs) continue;
                Pair P;
                fric_pair(k, o, kappa, yst, P);
                sym_add_outer(ck[fk(k)], 2.f * P.w / P.Q, P.a);
                sym_add_outer(ck[fk(k)], -P.w * (1.f + m2), P.n);
                ck[fk(k)][0] += P.w * m2;
                ck[fk(k)][3] += P.w * m2;
                ck[fk(k)][5] += P.w * m2;
            }
        }
    }
    // dlam/dq* of a pair applied to r (forward) or transposed (adjoint):
    //   Ly = w (A_y - a q_y^T / Q),
    //   A_y = n (n + H D)^T + y_n H + mu^2 ((n.u) H + n (H u)^T - T),
    //   q_y = 2 y_n (n + H D) + 2 mu^2 (n.u) H tau - 2 mu^2 tau;
    // dlam/dx of the pair's node: Lx = w (mu^2 T - 2 mu^2 a tau^T / Q).
    __device__ __forceinline__ void fric_ly(const Pair& P, const float r[3], bool transpose, float out[3]) const {
        const float m2 = fmu * fmu;
        float nH[3], Hr[3], Htau[3], qy[3], Tr[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) nH[c] = P.n[c] + P.HD[c];
        sym_mul(P.H, r, Hr);
        sym_mul(P.H, P.tau, Htau);
        const float nr = dot3(P.n, r);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            qy[c] = 2.f * P.yn * nH[c] + 2.f * m2 * P.nu * Htau[c] - 2.f * m2 * P.tau[c];
            Tr[c] = r[c] - nr * P.n[c];
        }
        if (!transpose) {
            const float s1 = dot3(nH, r), s2 = dot3(P.Hu, r), s3 = dot3(qy, r) / P.Q;
#pragma unroll
            for (int c = 0; c < 3; ++c)
                out[c] = P.w * (P.n[c] * s1 + P.yn * Hr[c] + m2 * (P.nu * Hr[c] + P.n[c] * s2 - Tr[c]) - P.a[c] * s3);
        } else {
            const float s3 = dot3(P.a, r) / P.Q;
#pragma unroll
            for (int c = 0; c < 3; ++c)
                out[c] = P.w * (nH[c] * nr + P.yn * Hr[c] + m2 * (P.nu * Hr[c] + P.Hu[c] * nr - Tr[c]) - qy[c] * s3);
        }
    }
    __device__ __forceinline__ void fric_lx(const Pair& P, const float r[3], bool transpose, float out[3]) const {
        const float m2 = fmu * fmu;
        const float nr = dot3(P.n, r);
        const float s = transpose ? dot3(P.a, r) / P.Q : dot3(P.tau, r) / P.Q;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float Tr = r[c] - nr * P.n[c];
            out[c] = P.w * m2 * (Tr - 2.f * (transpose ? P.tau[c] : P.a[c]) * s);
        }
    }

    // -------------------------------------------------- block reductions
    __device__ __forceinline__ float bsum(float v) {
        v = wave_sum(v);
        if constexpr (NT == 64) return v;
        float* b = rb + (rslot & 1) * 16; ++rslot;
        if ((threadIdx.x & 63) == 0) b[threadIdx.x >> 6] = v;
        sync();
        float r = b[0];
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) r += b[w];
        return r;
    }
    __device__ __forceinline__ float bmax(float v) {
        v = wave_max(v);
        if constexpr (NT == 64) return v;
        float* b = rb + (rslot & 1) * 16; ++rslot;
        if ((threadIdx.x & 63) == 0) b[threadIdx.x >> 6] = v;
        sync();
        float r = b[0];
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) r = fmaxf(r, b[w]);
        return r;
    }
    __device__ __forceinline__ float bmin(float v) {
        v = wave_min(v);
        if constexpr (NT == 64) return v;
        float* b = rb + (rslot & 1) * 16; ++rslot;
        if ((threadIdx.x & 63) == 0) b[threadIdx.x >> 6] = v;
        sync();
        float r = b[0];
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) r = fminf(r, b[w]);
        return r;
    }

    // -------------------------------------------------- LDS mirrors
    __device__ __forceinline__ void put(float* A, int k, const float val[3]) {
        int p = pidx(k);
        A[p] = val[0]; A[NM + p] = val[1]; A[2 * NM + p] = val[2];
    }
    __device__ __forceinline__ void get(const float* A, int q, float out[3]) const {
        out[0] = A[q]; out[1] = A[NM + q]; out[2] = A[2 * NM + q];
    }
    // Publish a per-particle vector (zero on gripped / inactive slots unless
    // keep_grip).  `presync` = false only where a block reduction (with its
    // barrier) already separates the last reads of A from this write.
    __device__ __forceinline__ void publish(float* A, const float val[PPT][3], bool keep_grip = false, bool presync = true) {
        if (presync || NT == 64) sync();
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            float z[3] = {0.f, 0.f, 0.f};
            put(A, k, (isfree(k) || (keep_grip && active(k))) ? val[k] : z);
        }
        sync();
    }

    // neighbour of owned particle k (index p) in spring slot s, or -1
    __device__ __forceinline__ int nbr(int k, int p, int s) const {
        if constexpr (TOPO == kRope) {
            int q = p + TP::dx(s);
            return (q >= 0 && q < n) ? q : -1;
        } else {
            int jx = px[k] + TP::dx(s), jy = py[k] + TP::dy(s);
            return (jx >= 0 && jx < nx && jy >= 0 && jy < ny) ? p + TP::dx(s) + TP::dy(s) * nx : -1;
        }
    }

    // -------------------------------------------------- state I/O
    __device__ __forceinline__ void load_state(const float* s) {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            int p = pidx(k);
            if (active(k)) {
#pragma unroll
                for (int c = 0; c < 3; ++c) { x[k][c] = s[3 * p + c]; v[k][c] = s[3 * n + 3 * p + c]; }
                if (pen[k] >= 0)
                    for (int c = 0; c < 3; ++c) pg(k)[c] = s[6 * n + 3 * pen[k] + c];
            }
        }
    }
    __device__ __forceinline__ void store_state(float* s) const {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            int p = pidx(k);
            if (active(k)) {
#pragma unroll
                for (int c = 0; c < 3; ++c) { s[3 * p + c] = x[k][c]; s[3 * n + 3 * p + c] = v[k][c]; }
                if (pen[k] >= 0)
                    for (int c = 0; c < 3; ++c) s[6 * n + 3 * pen[k] + c] = pg(k)[c];
            }
        }
    }

    // penalty grasp: cotangent of the gripper positions (GR[10..12])
    __device__ __forceinline__ void set_gcot(const float* s, bool add) {
#pragma unroll
        for (int k = 0; k < PPT; ++k)
            if (pen[k] >= 0)
                for (int c = 0; c < 3; ++c) pg(k)[10 + c] = (add ? pg(k)[10 + c] : 0.f) + (s ? s[6 * n + 3 * pen[k] + c] : 0.f);
    }
    __device__ __forceinline__ void get_gcot(float* s) const {
#pragma unroll
        for (int k = 0; k < PPT; ++k)
            if (pen[k] >= 0)
                for (int c = 0; c < 3; ++c) s[6 * n + 3 * pen[k] + c] = pg(k)[10 + c];
    }

    // -------------------------------------------------- stage-1 pieces
    // Gradient F of the incremental potential at y = x + d and the spring
    // Hessian data: K_s w = sa e (e.w) + sb w with sa = k(1 - f), sb = k f,
    // f = 1 - l0/L, clamped at 0 when `project`.  Also the diagonal 3x3 block
    // of the Hessian in Bd.  Gripped particles get F = 0 (the cache is still
    // filled: their rows are needed by the backward pass).
    __device__ __forceinline__ void grad_cache(bool project, float F[PPT][3]) {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int p = pidx(k);
#pragma unroll
            for (int c = 0; c < 3; ++c) F[k][c] = 0.f;
#pragma unroll
            for (int i = 0; i < 6; ++i) Bd[k][i] = 0.f;
            Bd[k][0] = Bd[k][3] = Bd[k][5] = mdt2;
#pragma unroll
            for (int s = 0; s < NS; ++s) { sa[k][s] = 0.f; sb[k][s] = 0.f; se[k][s][0] = se[k][s][1] = se[k][s][2] = 0.f; }
            if (!active(k)) continue;
            if (isfree(k)) {
                const float cv = dt * (1.f - gam);
#pragma unroll
                for (int c = 0; c < 3; ++c) F[k][c] = mdt2 * (d[k][c] - cv * v[k][c]) - mass * g[c];
                if (pen[k] >= 0) {
                    const float* G = pg(k);
                    for (int c = 0; c < 3; ++c) F[k][c] += G[6] * ((x[k][c] - G[3 + c]) + d[k][c]);
                    Bd[k][0] += G[6]; Bd[k][3] += G[6]; Bd[k][5] += G[6];
                }
            }
            // rope: X and D at p-2..p+2 read once (clamped indices; only the
            // neighbours that exist are used below)
            float x5[5][3], d5[5][3];
            if constexpr (TOPO == kRope) {
#pragma unroll
                for (int e = 0; e < 5; ++e) {
                    const int qe = min(max(p + e - 2, 0), n - 1);
                    get(X, qe, x5[e]);
                    get(D, qe, d5[e]);
                }
            }
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int q = nbr(k, p, s);
                if (q < 0) continue;
                const int ty = TP::type(s);
                const float kk = kS[ty], l0 = rS[ty];
                float e[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float xq = (TOPO == kRope) ? x5[2 + TP::dx(s)][c] : X[c * NM + q];
                    const float dq = (TOPO == kRope) ? d5[2 + TP::dx(s)][c] : D[c * NM + q];
                    e[c] = (xq - x[k][c]) + (dq - d[k][c]);
                }
                const float L = sqrtf(dot3(e, e));
                const float il = 1.0f / L;
                float eh[3] = {e[0] * il, e[1] * il, e[2] * il};
                const float f = 1.f - l0 * il;
                const float fr = isfree(k) ? kk * (L - l0) : 0.f;
#pragma unroll
                for (int c = 0; c < 3; ++c) F[k][c] -= fr * eh[c];
                const float fp = project ? fmaxf(f, 0.f) : f;
                sa[k][s] = kk * (1.f - fp);
                sb[k][s] = kk * fp;
#pragma unroll
                for (int c = 0; c < 3; ++c) se[k][s][c] = eh[c];
                sym_add_outer(Bd[k], sa[k][s], eh);
                Bd[k][0] += sb[k][s]; Bd[k][3] += sb[k][s]; Bd[k][5] += sb[k][s];
            }
            if constexpr (TOPO == kRope) {
                float wdiag = 0.f;
#pragma unroll
                for (int j = -1; j <= 1; ++j) {
                    const int cc = p + j;
                    if (cc < 1 || cc > n - 2) continue;
                    const float w = (j == 0) ? -2.f : 1.f;
                    wdiag += w * w;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const float kap = (x5[j + 1][c] - 2.f * x5[j + 2][c] + x5[j + 3][c]) +
                                          (d5[j + 1][c] - 2.f * d5[j + 2][c] + d5[j + 3][c]);
                        if (isfree(k)) F[k][c] += w * kb * kap;
                    }
                }
                Bd[k][0] += kb * wdiag; Bd[k][3] += kb * wdiag; Bd[k][5] += kb * wdiag;
            }
        }
    }

    // Hessian-vector product with the vector mirrored in V.  Rows of free
    // particles: (M/dt^2) w_p + sum_s K_s (w_p - w_q) + bending stencil
    // (+ contact weights if CONTACT).  With `grip_rows`, gripped particles get
    // their elastic row (no mass term), else 0.
    template <bool CONTACT>
    __device__ __forceinline__ void apply(float q[PPT][3], bool grip_rows = false, bool with_mass = true) {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int p = pidx(k);
#pragma unroll
            for (int c = 0; c < 3; ++c) q[k][c] = 0.f;
            if (!active(k)) continue;
            if (!isfree(k) && !grip_rows) continue;
            float wp[3];
            if constexpr (TOPO == kRope) {
                // V at p-2..p+2 (indices clamped into the rope: the springs
                // and bending weights of missing neighbours are zero), then
                // the springs to p+1 and p-1 and the curvature at the three
                // centres, without branches (same arithmetic as the
                // neighbour-by-neighbour form)
                float w5[5][3];
#pragma unroll
                for (int e = 0; e < 5; ++e) get(V, min(max(p + e - 2, 0), n - 1), w5[e]);
#pragma unroll
                for (int c = 0; c < 3; ++c) wp[c] = w5[2][c];
                if (isfree(k) && with_mass) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) q[k][c] = mdt2 * wp[c];
                }
                if (pen[k] >= 0) {
                    const float Dv = pg(k)[6];
#pragma unroll
                    for (int c = 0; c < 3; ++c) q[k][c] += Dv * wp[c];
                }
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const float* wq = w5[2 + TP::dx(s)];
                    float dv[3] = {wp[0] - wq[0], wp[1] - wq[1], wp[2] - wq[2]};
                    const float t = sa[k][s] * dot3(se[k][s], dv);
#pragma unroll
                    for (int c = 0; c < 3; ++c) q[k][c] += t * se[k][s][c] + sb[k][s] * dv[c];
                }
#pragma unroll
                for (int j = 0; j < 3; ++j)
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        q[k][c] += bw[k][j] * (w5[j][c] - 2.f * w5[j + 1][c] + w5[j + 2][c]);
            } else {
                get(V, p, wp);
                if (isfree(k) && with_mass) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) q[k][c] = mdt2 * wp[c];
                }
                if (pen[k] >= 0) {
                    const float Dv = pg(k)[6];
#pragma unroll
                    for (int c = 0; c < 3; ++c) q[k][c] += Dv * wp[c];
                }
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const int nq = nbr(k, p, s);
                    if (nq < 0) continue;
                    float wq[3];
                    get(V, nq, wq);
                    float dv[3] = {wp[0] - wq[0], wp[1] - wq[1], wp[2] - wq[2]};
                    const float t = sa[k][s] * dot3(se[k][s], dv);
#pragma unroll
                    for (int c = 0; c < 3; ++c) q[k][c] += t * se[k][s][c] + sb[k][s] * dv[c];
                }
            }
            if constexpr (CONTACT) {
                if (isfree(k)) {
                    bool fr = false;
                    if constexpr (FRIC) {
                        if (friction()) {
                            float t[3];
                            sym_mul(ck[fk(k)], wp, t);
#pragma unroll
                            for (int c = 0; c < 3; ++c) q[k][c] += t[c];
                            fr = true;
                        }
                    }
                    if (!fr) {
#pragma unroll
                        for (int o = 0; o < NOBS; ++o) {
                            if (o >= nobs) continue;
                            const float w = clam[k][o] / cgap[k][o] * dot3(cn[k][o], wp);
#pragma unroll
                            for (int c = 0; c < 3; ++c) q[k][c] += w * cn[k][o][c];
                        }
                    }
                }
            }
        }
    }

    // block-Jacobi preconditioner from Bd (+ contact weights); pcpd = 0 if
    // the Hessian block Bd of some particle of this thread is not positive
    // definite (Sylvester's criterion), which makes the preconditioned
    // residual norm meaningless.  The test is taken before the contact
    // weights are added: they only add positive semi-definite terms, and
    // the minors of a block with a weight many orders above the mass term
    // would be lost to cancellation.
    template <bool CONTACT>
    __device__ __forceinline__ void build_precond() {
        pcpd = 1.f;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            float m[6];
#pragma unroll
            for (int i = 0; i < 6; ++i) m[i] = Bd[k][i];
            if (isfree(k)) {
                const float m2 = m[0] * m[3] - m[1] * m[1];
                const float m3 = m[0] * (m[3] * m[5] - m[4] * m[4]) - m[1] * (m[1] * m[5] - m[4] * m[2]) +
                                 m[2] * (m[1] * m[4] - m[3] * m[2]);
                if (!(m[0] > 0.f && m2 > 0.f && m3 > 0.f)) pcpd = 0.f;
            }
            if constexpr (CONTACT) {
                bool fr = false;
                if constexpr (FRIC) {
                    if (friction()) {
#pragma unroll
                        for (int i = 0; i < 6; ++i) m[i] += ck[fk(k)][i];
                        fr = true;
                    }
                }
                if (!fr) {
#pragma unroll
                    for (int o = 0; o < NOBS; ++o)
                        if (o < nobs) sym_add_outer(m, clam[k][o] / cgap[k][o], cn[k][o]);
                }
            }
            if (isfree(k)) sym_inv(m, Mi[k]);
            else {
#pragma unroll
                for (int i = 0; i < 6; ++i) Mi[k][i] = 0.f;
            }
            if constexpr (kPairPrecond) {
#pragma unroll
                for (int i = 0; i < 6; ++i) mown[i] = m[i];
            }
        }
        if constexpr (kPairPrecond) pair_precond(mown);
    }

    // Ropes with one particle per lane precondition the conjugate gradients
    // with the inverse of the 6 x 6 diagonal block of each particle pair
    // (2q, 2q + 1), held by adjacent lanes, instead of each particle's 3 x 3
    // block: the pair's coupling (the spring between them and the bending
    // weight) is the chain's stiffest off-diagonal term.  Both lanes of a
    // pair form the same inverse from the same values (the even particle's
    // coupling block, exchanged by DPP), so the preconditioner is exactly
    // symmetric.  A pair with a particle that is not free, or whose block or
    // Schur complement is not positive definite, keeps the 3 x 3 blocks.
    static constexpr bool kPairPrecond = TOPO == kRope && PPT == 1;
    float mown[6];
    __device__ __forceinline__ void pair_precond(const float own[6]) {
        const int p = pidx(0);
        const bool even = (p & 1) == 0;
        // coupling of p and p + 1 as the even particle sees it:
        // -(sa e e^T + sb I) of the spring between them + the bending weight
        float c6[6];
        {
            const float cb = bw[0][1] - 2.f * bw[0][2];
            const float a = sa[0][0], b = sb[0][0];
            const float* e = se[0][0];
            c6[0] = cb - (a * e[0] * e[0] + b);
            c6[1] = -a * e[0] * e[1];
            c6[2] = -a * e[0] * e[2];
            c6[3] = cb - (a * e[1] * e[1] + b);
            c6[4] = -a * e[1] * e[2];
            c6[5] = cb - (a * e[2] * e[2] + b);
        }
        float A[6], B[6], C[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            const float op = dpp_mov<0xB1>(own[i]), cp = dpp_mov<0xB1>(c6[i]);
            A[i] = even ? own[i] : op;
            B[i] = even ? op : own[i];
            C[i] = even ? c6[i] : cp;
        }
        const float fp = dpp_mov<0xB1>(isfree(0) ? 1.f : 0.f);
        float Cf[3][3], Ai[6], X[3][3], S[6], Si[6];
        sym_to_full3(C, Cf);
        sym_inv(A, Ai);
        // X = A^{-1} C
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                X[r][c] = sym_at(Ai, r, 0) * Cf[0][c] + sym_at(Ai, r, 1) * Cf[1][c] + sym_at(Ai, r, 2) * Cf[2][c];
        // S = B - C^T X (upper triangle)
        {
            int q = 0;
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = r; c < 3; ++c, ++q)
                    S[q] = B[q] - (Cf[0][r] * X[0][c] + Cf[1][r] * X[1][c] + Cf[2][r] * X[2][c]);
        }
        const bool ok = isfree(0) && fp > 0.f && sym_pd(A) && sym_pd(S);
        sym_inv(S, Si);
        // P12 = -X S^{-1};  P11 = A^{-1} - P12 X^T;  P22 = S^{-1}
        float P12[3][3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                P12[r][c] = -(X[r][0] * sym_at(Si, 0, c) + X[r][1] * sym_at(Si, 1, c) + X[r][2] * sym_at(Si, 2, c));
        float P11[6];
        {
            int q = 0;
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = r; c < 3; ++c, ++q)
                    P11[q] = Ai[q] - (P12[r][0] * X[c][0] + P12[r][1] * X[c][1] + P12[r][2] * X[c][2]);
        }
#pragma unroll
        for (int i = 0; i < 6; ++i) Pd[0][i] = ok ? (even ? P11[i] : Si[i]) : Mi[0][i];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) Pc[0][3 * r + c] = ok ? (even ? P12[r][c] : P12[c][r]) : 0.f;
    }

    // z = M^{-1} r: the pair blocks on ropes with one particle per lane,
    // else the 3 x 3 blocks.  Every lane of the workgroup must execute it
    // (the partner's residual is read by DPP).
    __device__ __forceinline__ void precond(const float r[PPT][3], float z[PPT][3]) const {
        if constexpr (kPairPrecond) {
            const float q0 = dpp_mov<0xB1>(r[0][0]), q1 = dpp_mov<0xB1>(r[0][1]), q2 = dpp_mov<0xB1>(r[0][2]);
            sym_mul(Pd[0], r[0], z[0]);
#pragma unroll
            for (int c = 0; c < 3; ++c) z[0][c] += Pc[0][3 * c] * q0 + Pc[0][3 * c + 1] * q1 + Pc[0][3 * c + 2] * q2;
        } else {
#pragma unroll
            for (int k = 0; k < PPT; ++k) sym_mul(Mi[k], r[k], z[k]);
        }
    }

    // Preconditioned conjugate gradients on the free DoFs.  Returns false if
    // non-positive curvature was met (the iterate so far is kept).
    template <bool CONTACT>
    __device__ __forceinline__ bool pcg(const float b[PPT][3], float xs[PPT][3], float rtol) {
        float r[PPT][3], z[PPT][3], pp[PPT][3], q[PPT][3];
        float rz = 0.f;
#pragma unroll
        for (int k = 0; k < PPT; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) { xs[k][c] = 0.f; r[k][c] = isfree(k) ? b[k][c] : 0.f; }
        precond(r, z);
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
#pragma unroll
            for (int c = 0; c < 3; ++c) pp[k][c] = z[k][c];
            rz += dot3(r[k], z[k]);
        }
        rz = bsum(rz);
        const float rz0 = rz;
        if (!(rz0 > 0.f)) return rz0 == 0.f;
        bool ok = true;
        for (int it = 0; it < kPcgMax; ++it) {
            publish(V, pp, false, false);
            apply<CONTACT>(q);
            float pq = 0.f;
#pragma unroll
            for (int k = 0; k < PPT; ++k) pq += dot3(pp[k], q[k]);
            pq = bsum(pq);
            ++cnt[1];
            if (!(pq > 0.f)) { ok = false; break; }
            // step lengths from the hardware reciprocal (1 ulp): two
            // instructions instead of the ten of a correctly rounded
            // division on the iteration's dependent chain; r and xs take
            // the same alpha, so the recurrence stays consistent
            const float alpha = rz * __builtin_amdgcn_rcpf(pq);
            float rzn = 0.f;
#pragma unroll
            for (int k = 0; k < PPT; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) { xs[k][c] += alpha * pp[k][c]; r[k][c] -= alpha * q[k][c]; }
            precond(r, z);
#pragma unroll
            for (int k = 0; k < PPT; ++k) rzn += dot3(r[k], z[k]);
            rzn = bsum(rzn);
            if (!(rzn > rtol * rtol * rz0)) break;
            const float beta = rzn * __builtin_amdgcn_rcpf(rz);
            rz = rzn;
#pragma unroll
            for (int k = 0; k < PPT; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) pp[k][c] = z[k][c] + beta * pp[k][c];
        }
        return ok;
    }

    // Minimum residual method (Paige and Saunders, 1975) on the free DoFs:
    // the solver of the derivative and interior-point systems when conjugate
    // gradients cannot be used.  Compression makes the exact dF/dq*
    // indefinite at a stationary point of Psi that is not a minimum (a
    // straight compressed rope); the implicit derivative of eq. (diff-sim)
    // still exists there and this solves for it.  No preconditioner: the
    // block-Jacobi blocks need not be positive definite then.  Lanczos
    // vectors r1 (previous) and r2 (current, unnormalised), the two last
    // search directions wa, wb and the iterate stay in registers.  Each pass
    // runs until its recursive residual estimate is below rtol |b|; in FP32
    // the Lanczos vectors lose orthogonality, so the true residual b - A x
    // is then formed and the method restarts on it (iterative refinement,
    // at most three passes).  The true residual cannot go below about
    // eps cond(A) |b| (its own rounding), so the solve is accepted once it
    // is within rtol |b| or, after the last pass, within kMinresAccept |b|.
    template <bool CONTACT>
    __device__ __forceinline__ bool minres(const float b[PPT][3], float xs[PPT][3], float rtol) {
        float r1[PPT][3], r2[PPT][3], y[PPT][3], wa[PPT][3], wb[PPT][3];
        float bb = 0.f;
#pragma unroll
        for (int k = 0; k < PPT; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                xs[k][c] = 0.f;
                const float bk = isfree(k) ? b[k][c] : 0.f;
                bb += bk * bk;
            }
        const float bnorm = sqrtf(bsum(bb));
        if (!(bnorm > 0.f)) return bnorm == 0.f;
        for (int pass = 0; pass <= 3; ++pass) {
            // r1 = b - A xs
            if (pass > 0) {
                publish(V, xs, false, false);
                apply<CONTACT>(y);
            }
            float rr = 0.f;
#pragma unroll
            for (int k = 0; k < PPT; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    r1[k][c] = isfree(k) ? b[k][c] - (pass > 0 ? y[k][c] : 0.f) : 0.f;
                    r2[k][c] = r1[k][c];
                    wa[k][c] = 0.f;
                    wb[k][c] = 0.f;
                    rr += r1[k][c] * r1[k][c];
                }
            const float beta1 = sqrtf(bsum(rr));
            if (!(beta1 > rtol * bnorm)) return beta1 == beta1;
            if (pass == 3) return beta1 <= kMinresAccept * bnorm;
            float oldb = 0.f, beta = beta1, dbar = 0.f, epsln = 0.f, phibar = beta1, cs = -1.f, sn = 0.f;
            for (int it = 0; it < kMinresMax; ++it) {
                const float sc = 1.0f / beta;              // v = sc r2
#pragma unroll
                for (int k = 0; k < PPT; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c) y[k][c] = sc * r2[k][c];
                publish(V, y, false, false);
                apply<CONTACT>(y);
                ++cnt[1];
                float vy = 0.f;
#pragma unroll
                for (int k = 0; k < PPT; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        if (it > 0) y[k][c] -= (beta / oldb) * r1[k][c];
                        vy += sc * r2[k][c] * y[k][c];
                    }
                const float alfa = bsum(vy);
                float yy = 0.f;
#pragma unroll
                for (int k = 0; k < PPT; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        y[k][c] -= (alfa / beta) * r2[k][c];
                        yy += y[k][c] * y[k][c];
                    }
                oldb = beta;
                beta = sqrtf(bsum(yy));
                const float oldeps = epsln;
                const float delta = cs * dbar + sn * alfa;
                const float gbar = sn * dbar - cs * alfa;
                epsln = sn * beta;
                dbar = -cs * beta;
                const float gam = fmaxf(sqrtf(gbar * gbar + beta * beta), 1e-30f);
                cs = gbar / gam;
                sn = beta / gam;
                const float phi = cs * phibar;
                phibar = sn * phibar;
                const float ig = 1.0f / gam;
#pragma unroll
                for (int k = 0; k < PPT; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        // new direction from v (= sc r2, before r2 moves on)
                        const float wn = (sc * r2[k][c] - oldeps * wb[k][c] - delta * wa[k][c]) * ig;
                        wb[k][c] = wa[k][c];
                        wa[k][c] = wn;
                        xs[k][c] += phi * wn;
                        r1[k][c] = r2[k][c];
                        r2[k][c] = y[k][c];
                    }
                if (!(phibar > 0.5f * rtol * bnorm) || !(beta > 0.f)) break;
            }
        }
        return false;
    }

    // A derivative or interior-point solve: conjugate gradients, or MINRES if
    // they meet non-positive curvature or if some preconditioner block is
    // not positive definite (a compressed particle; the preconditioned
    // residual norm is then no norm).  Flags NOT_PD only if MINRES fails.
    template <bool CONTACT>
    __device__ __forceinline__ void solve(const float b[PPT][3], float xs[PPT][3], float rtol) {
        if constexpr (!FALLBACK) {
            if (!pcg<CONTACT>(b, xs, rtol)) status = max(status, kStNotPD);
        } else {
            if (bmin(pcpd) > 0.f && pcg<CONTACT>(b, xs, rtol)) return;
            if (!minres<CONTACT>(b, xs, rtol)) status = max(status, kStNotPD);
        }
    }

    // Psi(y + DL) - Psi(y) with DL mirrored in LDS, in cancellation-free form
    // (each spring counted half at each end, each bending triplet at its
    // centre, inertia and gravity at free particles).
    __device__ __forceinline__ float psi_diff() {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int p = pidx(k);
            if (!active(k)) continue;
            float sp[3];
            get(DL, p, sp);
            // rope: X, D and DL at p-1..p+1 read once (clamped indices; only
            // the neighbours that exist are used below)
            float x3[3][3], d3[3][3], l3[3][3];
            if constexpr (TOPO == kRope) {
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    const int qe = min(max(p + e - 1, 0), n - 1);
                    get(X, qe, x3[e]);
                    get(D, qe, d3[e]);
                    get(DL, qe, l3[e]);
                }
            }
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int q = nbr(k, p, s);
                if (q < 0) continue;
                const int ty = TP::type(s);
                float e0[3], de[3], e1[3], sm[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int eq = 1 + TP::dx(s);
                    const float xq = (TOPO == kRope) ? x3[eq][c] : X[c * NM + q];
                    const float dq = (TOPO == kRope) ? d3[eq][c] : D[c * NM + q];
                    const float lq = (TOPO == kRope) ? l3[eq][c] : DL[c * NM + q];
                    e0[c] = (xq - x[k][c]) + (dq - d[k][c]);
                    de[c] = lq - sp[c];
                    e1[c] = e0[c] + de[c];
                    sm[c] = e1[c] + e0[c];
                }
                const float L0 = sqrtf(dot3(e0, e0)), L1 = sqrtf(dot3(e1, e1));
                const float dL = dot3(de, sm) / (L1 + L0);
                acc += 0.25f * kS[ty] * dL * (L1 + L0 - 2.f * rS[ty]);
            }
            if constexpr (TOPO == kRope) {
                if (p >= 1 && p <= n - 2) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const float k0 = (x3[0][c] - 2.f * x3[1][c] + x3[2][c]) +
                                         (d3[0][c] - 2.f * d3[1][c] + d3[2][c]);
                        const float dk = l3[0][c] - 2.f * l3[1][c] + l3[2][c];
                        acc += 0.5f * kb * dk * (2.f * k0 + dk);
                    }
                }
            }
            if (isfree(k)) {
                const float cv = dt * (1.f - gam);
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    acc += 0.5f * mdt2 * sp[c] * (2.f * (d[k][c] - cv * v[k][c]) + sp[c]) - mass * g[c] * sp[c];
                if (pen[k] >= 0) {
                    const float* G = pg(k);
                    for (int c = 0; c < 3; ++c)
                        acc += 0.5f * G[6] * sp[c] * (2.f * ((x[k][c] - G[3 + c]) + d[k][c]) + sp[c]);
                }
            }
        }
        return bsum(acc);
    }

    // -------------------------------------------------- one step
    // Grippers and predictor; publishes x and d.
    __device__ __forceinline__ void begin_step(const float* ut) {
        sync();
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (!active(k)) continue;
            if (grip[k] >= 0) {
#pragma unroll
                for (int c = 0; c < 3; ++c) { ug[k][c] = ut[3 * grip[k] + c]; d[k][c] = dt * ug[k][c]; }
            } else {
                // Newton starts from the predictor plus the free-fall drop
                // dt^2 g (the root does not depend on the start)
                const float cv = dt * (1.f - gam);
#pragma unroll
                for (int c = 0; c < 3; ++c) d[k][c] = cv * v[k][c] + dt * dt * g[c];
                if (pen[k] >= 0) {
                    // g+ = g + dt u; activation from c = x_j - g (the state before the step)
                    float* G = pg(k);
                    float cc[3];
                    for (int c = 0; c < 3; ++c) {
                        G[3 + c] = G[c] + dt * ut[3 * pen[k] + c];
                        cc[c] = x[k][c] - G[c];
                    }
                    const float r = sqrtf(dot3(cc, cc));
                    float Dv, sd;
                    if (khal > 0.f) {
                        Dv = Dmax * expf(-r / khal);
                        sd = r > 0.f ? -Dv / (khal * r) : 0.f;
                    } else {
                        Dv = r <= rgrip ? Dmax : 0.f;
                        sd = 0.f;
                    }
                    G[6] = Dv;
                    for (int c = 0; c < 3; ++c) G[7 + c] = sd * cc[c];
                }
            }
            put(X, k, x[k]);
            put(D, k, d[k]);
        }
        sync();
    }

    // Stage 1: Newton on F(y) = 0 (minimising Psi), projected-Hessian
    // directions, Armijo backtracking on Psi.
    __device__ __forceinline__ void stage1() {
        float F[PPT][3], del[PPT][3];
        bool conv = false;
        float fmax = 0.f;
        for (int it = 0; it < kNewtonMax; ++it) {
            grad_cache(true, F);
            float lm = 0.f;
#pragma unroll
            for (int k = 0; k < PPT; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) lm = nmax(lm, fabsf(F[k][c]));
            fmax = bmax(finite_key(lm));
            if (fmax >= kBad) { status = max(status, kStNonFinite); return; }
            if (fmax <= tolF) { conv = true; break; }
            build_precond<false>();
            float rhs[PPT][3];
#pragma unroll
            for (int k = 0; k < PPT; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) rhs[k][c] = -F[k][c];
            pcg<false>(rhs, del, kPcgTolInner);
            ++cnt[0];
            float gtd = 0.f;
#pragma unroll
            for (int k = 0; k < PPT; ++k) gtd += dot3(F[k], del[k]);
            gtd = bsum(gtd);
            if (!(gtd < 0.f)) break;
            float alpha = 1.f;
            bool acc = false;
            float stp[PPT][3];
            for (int ls = 0; ls < kLineSearchMax; ++ls) {
#pragma unroll
                for (int k = 0; k < PPT; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c) stp[k][c] = alpha * del[k][c];
                publish(DL, stp);
                const float dpsi = psi_diff();
                if (dpsi <= 1e-4f * alpha * gtd) { acc = true; break; }
                alpha *= 0.5f;
            }
            if (!acc) break;
            float smax = 0.f;
            if constexpr (NT == 64) sync();
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                if (isfree(k)) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) { d[k][c] += stp[k][c]; smax = fmaxf(smax, fabsf(stp[k][c])); }
                    put(D, k, d[k]);
                }
            }
            sync();
            smax = bmax(finite_key(smax));
            if (smax <= 1e-7f * h) { conv = fmax <= 100.f * tolF; break; }
        }
        if (!conv) {
            grad_cache(true, F);
            float lm = 0.f;
#pragma unroll
            for (int k = 0; k < PPT; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) lm = nmax(lm, fabsf(F[k][c]));
            fmax = bmax(finite_key(lm));
            if (fmax >= kBad) status = max(status, kStNonFinite);
            else if (!(fmax <= 100.f * tolF)) status = max(status, kStNewton);
        }
    }

    // Contact pairs at y* = x + d for every (free particle, obstacle).
    __device__ __forceinline__ void eval_contacts() {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            float y[3] = {x[k][0] + d[k][0], x[k][1] + d[k][1], x[k][2] + d[k][2]};
#pragma unroll
            for (int o = 0; o < NOBS; ++o) {
                if (o < nobs && isfree(k)) sdf_eval(otype[o], ob[o], y, cphi[k][o], cn[k][o]);
                else { cphi[k][o] = 1.f; cn[k][o][0] = cn[k][o][1] = cn[k][o][2] = 0.f; }
            }
        }
    }

    // Stage 2 (eq. dynamics-second-stage with the smoothed complementarity):
    // P D = sum_c n_c lam_c, lam_c gap_c = mu, gap_c = phi_c + n_c . D_p,
    // solved by a primal-dual interior point from an infeasible start.
    // kappa > 0: mu = kappa.  kappa = 0: mu is driven towards 0 (hard contact).
    __device__ __forceinline__ void stage2(float kappa) {
        if constexpr (FRIC) {
            if (friction()) {
                stage2_friction(kappa);
                return;
            }
        }
        float F[PPT][3];
        grad_cache(false, F);      // exact Hessian data at y*
        eval_contacts();
        const bool hard = !(kappa > 0.f);
        // initial point: each pair as if alone with stiffness n^T P_pp n
        float mu = kappa;
        if (hard) {
            float acc = 0.f;
#pragma unroll
            for (int k = 0; k < PPT; ++k)
#pragma unroll
                for (int o = 0; o < NOBS; ++o)
                    if (o < nobs && isfree(k)) {
                        float t[3];
                        sym_mul(Bd[k], cn[k][o], t);
                        acc += dot3(cn[k][o], t) * cphi[k][o] * cphi[k][o];
                    }
            acc = bsum(acc);
            int np = 0;
            np = (n - ngrip) * nobs;
            mu = fmaxf(1e-2f * acc / fmaxf((float)np, 1.f), 1e-9f * fscale * h);
        }
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
#pragma unroll
            for (int c = 0; c < 3; ++c) dl[k][c] = 0.f;
#pragma unroll
            for (int o = 0; o < NOBS; ++o) {
                float t[3];
                sym_mul(Bd[k], cn[k][o], t);
                const float pi = fmaxf(dot3(cn[k][o], t), mdt2);
                const float ph = cphi[k][o];
                const float gp = 0.5f * (ph + sqrtf(ph * ph + 4.f * mu / pi));
                cgap[k][o] = (o < nobs && isfree(k)) ? gp : 1.f;
                clam[k][o] = (o < nobs && isfree(k)) ? mu / gp : 0.f;
            }
        }
        if (nobs == 0) return;
        const float mu_min = 1e-7f * fscale * h;
        bool conv = false;
        for (int it = 0; it < kIpmMax; ++it) {
            float rd[PPT][3];
            publish(V, dl);
            apply<false>(rd);
            float err = 0.f, comp = 0.f;
            float rp[PPT][NOBS], rc[PPT][NOBS];
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                // FP32 rounding floor of the force balance grows with the
                // forces acting on the particle
                float fm = fmaxf(fabsf(rd[k][0]), fmaxf(fabsf(rd[k][1]), fabsf(rd[k][2])));
#pragma unroll
                for (int o = 0; o < NOBS; ++o) {
                    rp[k][o] = 0.f; rc[k][o] = 0.f;
                    if (o < nobs && isfree(k)) {
#pragma unroll
                        for (int c = 0; c < 3; ++c) rd[k][c] -= cn[k][o][c] * clam[k][o];
                        fm += fabsf(clam[k][o]);
                        rp[k][o] = cgap[k][o] - cphi[k][o] - dot3(cn[k][o], dl[k]);
                        comp += clam[k][o] * cgap[k][o];
                        err = nmax(err, fabsf(rp[k][o]) / (kTolGap * (h + fabsf(cphi[k][o]))));
                    }
                }
                const float tolD = tolF + 5e-7f * fm;
                if (isfree(k))
#pragma unroll
                    for (int c = 0; c < 3; ++c) err = nmax(err, fabsf(rd[k][c]) / tolD);
            }
            float mtarget = mu;
            if (hard) {
                float cs = bsum(comp);
                mtarget = fmaxf(0.1f * cs / fmaxf((float)((n - ngrip) * nobs), 1.f), mu_min);
            }
#pragma unroll
            for (int k = 0; k < PPT; ++k)
#pragma unroll
                for (int o = 0; o < NOBS; ++o)
                    if (o < nobs && isfree(k)) {
                        rc[k][o] = clam[k][o] * cgap[k][o] - mtarget;
                        if (!hard) err = nmax(err, fabsf(rc[k][o]) / (kTolCompl * kappa));
                        else err = nmax(err, clam[k][o] * cgap[k][o] / (10.f * mu_min));
                    }
            err = bmax(finite_key(err));
            if (err >= kBad) { status = max(status, kStNonFinite); return; }
            if (err <= 1.f) { conv = true; break; }
            float rhs[PPT][3], dD[PPT][3];
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
#pragma unroll
                for (int c = 0; c < 3; ++c) rhs[k][c] = -rd[k][c];
#pragma unroll
                for (int o = 0; o < NOBS; ++o)
                    if (o < nobs && isfree(k)) {
                        const float w = (-rc[k][o] + clam[k][o] * rp[k][o]) / cgap[k][o];
#pragma unroll
                        for (int c = 0; c < 3; ++c) rhs[k][c] += w * cn[k][o][c];
                    }
            }
            build_precond<true>();
            solve<true>(rhs, dD, kPcgTolInner);
            ++cnt[2];
            float amax = 1.f / 0.995f;
            float dg[PPT][NOBS], dlm[PPT][NOBS];
#pragma unroll
            for (int k = 0; k < PPT; ++k)
#pragma unroll
                for (int o = 0; o < NOBS; ++o) {
                    dg[k][o] = 0.f; dlm[k][o] = 0.f;
                    if (o < nobs && isfree(k)) {
                        dg[k][o] = dot3(cn[k][o], dD[k]) - rp[k][o];
                        dlm[k][o] = (-rc[k][o] - clam[k][o] * dg[k][o]) / cgap[k][o];
                        if (dg[k][o] < 0.f) amax = fminf(amax, -cgap[k][o] / dg[k][o]);
                        if (dlm[k][o] < 0.f) amax = fminf(amax, -clam[k][o] / dlm[k][o]);
                    }
                }
            amax = bmin(amax);
            const float alpha = fminf(1.f, 0.995f * amax);
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
#pragma unroll
                for (int c = 0; c < 3; ++c) dl[k][c] += alpha * dD[k][c];
#pragma unroll
                for (int o = 0; o < NOBS; ++o)
                    if (o < nobs && isfree(k)) { cgap[k][o] += alpha * dg[k][o]; clam[k][o] += alpha * dlm[k][o]; }
            }
        }
        if (!conv) status = max(status, kStQP);
        else if constexpr (FALLBACK) {
            if (hard) hard_polish();
        }
    }

    // Stage 2 with the friction cone (eq. contact-constraint, Anitescu's
    // relaxation).  Per pair the constraint value y = [phi + n.D ; t1.(d + D) ;
    // t2.(d + D)] (normal row at y*, tangential rows the node's displacement
    // over the step) must lie in the dual cone {y0 >= mu |(y1, y2)|}.
    // Smoothed: the central-path point of min 1/2 D^T P D - kappa sum psi(y),
    // psi = 1/2 log(y0^2 - mu^2 (y1^2 + y2^2)), so lam = kappa grad psi lies in
    // the cone and y . lam = kappa.  Newton from an infeasible start on D and
    // the slack y (cgap, cy1, cy2) with lam = kappa grad psi(y): residuals
    // r_D = P D - sum J^T lam, r_p = y - J D - b; the step solves
    // (P + sum J^T Hb J) dD = -r_D + sum J^T Hb r_p (Hb = -kappa Hess psi, per
    // particle summed into ck), dy = J dD - r_p, and stays inside the cone.
    // Hard (kappa = 0): the relaxation is lowered tenfold after each
    // converged level down to 1e-7 fscale h.
    __device__ __forceinline__ void stage2_friction(float kappa) {
        float F[PPT][3];
        grad_cache(false, F);      // exact Hessian data at y*
        eval_contacts();
        const bool hard = !(kappa > 0.f);
        const float m2 = fmu * fmu;
        const float kmin = 1e-7f * fscale * h;
        float kk = kappa;
        if (hard) {
            float acc = 0.f;
#pragma unroll
            for (int k = 0; k < PPT; ++k)
#pragma unroll
                for (int o = 0; o < NOBS; ++o)
                    if (o < nobs && isfree(k)) {
                        float t[3];
                        sym_mul(Bd[k], cn[k][o], t);
                        acc += dot3(cn[k][o], t) * cphi[k][o] * cphi[k][o];
                    }
            acc = bsum(acc);
            kk = fmaxf(1e-2f * acc / fmaxf((float)((n - ngrip) * nobs), 1.f), kmin);
        }
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
#pragma unroll
            for (int c = 0; c < 3; ++c) dl[k][c] = 0.f;
#pragma unroll
            for (int o = 0; o < NOBS; ++o) {
                clam[k][o] = 0.f;
                cgap[k][o] = 1.f;
                cy1[fk(k)][fo(o)] = 0.f;
                cy2[fk(k)][fo(o)] = 0.f;
                if (o < nobs && isfree(k)) {
                    float t1[3], t2[3], t[3];
                    tframe(cn[k][o], t1, t2);
                    sym_mul(Bd[k], cn[k][o], t);
                    const float pi = fmaxf(dot3(cn[k][o], t), mdt2);
                    const float s1 = dot3(t1, d[k]), s2 = dot3(t2, d[k]);
                    cy1[fk(k)][fo(o)] = s1;
                    cy2[fk(k)][fo(o)] = s2;
                    cgap[k][o] = fmaxf(cphi[k][o], 0.f) + fmu * sqrtf(s1 * s1 + s2 * s2) + sqrtf(kk / pi);
                }
            }
        }
        if (nobs == 0) return;
        bool conv = false;
        for (int it = 0; it < kIpmFricMax; ++it) {
            float rd[PPT][3], rhs[PPT][3];
            float rp[PPT][NOBS][3];
            publish(V, dl);
            apply<false>(rd);
            float err = 0.f;
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                float fm = fmaxf(fabsf(rd[k][0]), fmaxf(fabsf(rd[k][1]), fabsf(rd[k][2])));
#pragma unroll
                for (int i = 0; i < 6; ++i) ck[fk(k)][i] = 0.f;
#pragma unroll
                for (int c = 0; c < 3; ++c) rhs[k][c] = 0.f;
#pragma unroll
                for (int o = 0; o < NOBS; ++o) {
                    rp[k][o][0] = rp[k][o][1] = rp[k][o][2] = 0.f;
                    if (!(o < nobs && isfree(k))) continue;
                    float t1[3], t2[3], u[3];
                    tframe(cn[k][o], t1, t2);
#pragma unroll
                    for (int c = 0; c < 3; ++c) u[c] = d[k][c] + dl[k][c];
                    const float y0 = cgap[k][o], y1 = cy1[fk(k)][fo(o)], y2 = cy2[fk(k)][fo(o)];
                    rp[k][o][0] = y0 - cphi[k][o] - dot3(cn[k][o], dl[k]);
                    rp[k][o][1] = y1 - dot3(t1, u);
                    rp[k][o][2] = y2 - dot3(t2, u);
                    const float iq = 1.f / (y0 * y0 - m2 * (y1 * y1 + y2 * y2));
                    const float g[3] = {y0 * iq, -m2 * y1 * iq, -m2 * y2 * iq};
                    // Hb = kappa (2 g g^T - diag(1, -mu^2, -mu^2) / Q), in the pair's frame
                    const float Hb[6] = {kk * (2.f * g[0] * g[0] - iq), kk * 2.f * g[0] * g[1], kk * 2.f * g[0] * g[2],
                                         kk * (2.f * g[1] * g[1] + m2 * iq), kk * 2.f * g[1] * g[2],
                                         kk * (2.f * g[2] * g[2] + m2 * iq)};
                    float hr[3];
                    sym_mul(Hb, rp[k][o], hr);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        rd[k][c] -= kk * (g[0] * cn[k][o][c] + g[1] * t1[c] + g[2] * t2[c]);
                        rhs[k][c] += hr[0] * cn[k][o][c] + hr[1] * t1[c] + hr[2] * t2[c];
                    }
                    // ck += R^T Hb R, R = rows (n, t1, t2)
                    const float* e[3] = {cn[k][o], t1, t2};
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        const float hii = Hb[i == 0 ? 0 : (i == 1 ? 3 : 5)];
                        sym_add_outer(ck[fk(k)], hii, e[i]);
                    }
                    // off-diagonal frame terms Hb_ij (e_i e_j^T + e_j e_i^T)
                    const int oi[3] = {0, 0, 1}, oj[3] = {1, 2, 2}, oh[3] = {1, 2, 4};
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        const float hv = Hb[oh[q]];
                        const float* a = e[oi[q]];
                        const float* b = e[oj[q]];
                        ck[fk(k)][0] += 2.f * hv * a[0] * b[0];
                        ck[fk(k)][1] += hv * (a[0] * b[1] + a[1] * b[0]);
                        ck[fk(k)][2] += hv * (a[0] * b[2] + a[2] * b[0]);
                        ck[fk(k)][3] += 2.f * hv * a[1] * b[1];
                        ck[fk(k)][4] += hv * (a[1] * b[2] + a[2] * b[1]);
                        ck[fk(k)][5] += 2.f * hv * a[2] * b[2];
                    }
                    fm += kk * fabsf(g[0]);
                    const float gt = kTolGap * (h + fabsf(cphi[k][o]));
                    err = nmax(err, fmaxf(fabsf(rp[k][o][0]), fmaxf(fabsf(rp[k][o][1]), fabsf(rp[k][o][2]))) / gt);
                }
                const float tolD = tolF + 5e-7f * fm;
                if (isfree(k))
#pragma unroll
                    for (int c = 0; c < 3; ++c) err = nmax(err, fabsf(rd[k][c]) / tolD);
            }
            err = bmax(finite_key(err));
            if (err >= kBad) { status = max(status, kStNonFinite); return; }
            if (err <= 1.f) {
                if (hard && kk > kmin) {
                    kk = fmaxf(0.1f * kk, kmin);
                    continue;
                }
                conv = true;
                break;
            }
#pragma unroll
            for (int k = 0; k < PPT; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) rhs[k][c] = isfree(k) ? rhs[k][c] - rd[k][c] : 0.f;
            float dD[PPT][3];
            build_precond<true>();
            solve<true>(rhs, dD, kPcgTolInner);
            ++cnt[2];
            float amax = 1.f / 0.995f;
            float dy[PPT][NOBS][3];
#pragma unroll
            for (int k = 0; k < PPT; ++k)
#pragma unroll
                for (int o = 0; o < NOBS; ++o) {
                    dy[k][o][0] = dy[k][o][1] = dy[k][o][2] = 0.f;
                    if (!(o < nobs && isfree(k))) continue;
                    float t1[3], t2[3];
                    tframe(cn[k][o], t1, t2);
                    dy[k][o][0] = dot3(cn[k][o], dD[k]) - rp[k][o][0];
                    dy[k][o][1] = dot3(t1, dD[k]) - rp[k][o][1];
                    dy[k][o][2] = dot3(t2, dD[k]) - rp[k][o][2];
                    amax = fminf(amax, cone_step(cgap[k][o], cy1[fk(k)][fo(o)], cy2[fk(k)][fo(o)], dy[k][o][0],
                                                 dy[k][o][1], dy[k][o][2], m2));
                }
            amax = bmin(amax);
            const float alpha = fminf(1.f, 0.995f * amax);
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
#pragma unroll
                for (int c = 0; c < 3; ++c) dl[k][c] += alpha * dD[k][c];
#pragma unroll
                for (int o = 0; o < NOBS; ++o)
                    if (o < nobs && isfree(k)) {
                        cgap[k][o] += alpha * dy[k][o][0];
                        cy1[fk(k)][fo(o)] += alpha * dy[k][o][1];
                        cy2[fk(k)][fo(o)] += alpha * dy[k][o][2];
                    }
            }
        }
        if (!conv) status = max(status, kStQP);
        // normal force of each pair (kept with the step internals)
#pragma unroll
        for (int k = 0; k < PPT; ++k)
#pragma unroll
            for (int o = 0; o < NOBS; ++o)
                if (o < nobs && isfree(k)) {
                    const float y0 = cgap[k][o], y1 = cy1[fk(k)][fo(o)], y2 = cy2[fk(k)][fo(o)];
                    clam[k][o] = kk * y0 / (y0 * y0 - m2 * (y1 * y1 + y2 * y2));
                }
    }

    // Hard contact: the interior point ends with a small positive lam * gap
    // on every pair.  Fix its active set {lam_c > pi_c gap_c} (pi_c =
    // n_c^T P_pp n_c) and solve min 1/2 D^T P D s.t. phi_c + n_c . D_p = 0
    // over it, so the complementarity of eq. (dynamics-second-stage) holds
    // exactly instead of to the interior point's floor.  Per particle the
    // active normals (one or two) give a shift s_p onto the constraints and
    // the projector Pi_p onto the complement of their span; the rest solves
    // Pi P Pi w = -Pi P (D + s) by projected conjugate gradients
    // (preconditioner Pi M^-1 Pi from the diagonal blocks of P).  The
    // multipliers follow from (P D)_p = sum_c lam_c n_c.  The interior
    // point's correction is kept if some particle has more than two active
    // pairs or two nearly parallel ones, or if the result has a negative
    // active multiplier or a penetrating inactive pair.
    __device__ __forceinline__ void hard_polish() {
        float pj[PPT][6], dn[PPT][3], n1[PPT][3], n2[PPT][3];
        int na[PPT];
        float c12[PPT];
        float bad = 0.f;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            na[k] = 0;
            c12[k] = 0.f;
            float g1 = 0.f, g2 = 0.f;
#pragma unroll
            for (int c = 0; c < 3; ++c) { n1[k][c] = 0.f; n2[k][c] = 0.f; }
#pragma unroll
            for (int o = 0; o < NOBS; ++o) {
                if (!(o < nobs && isfree(k))) continue;
                float t[3];
                sym_mul(Bd[k], cn[k][o], t);
                const float pi = dot3(cn[k][o], t);
                if (!(clam[k][o] > pi * cgap[k][o])) continue;
                const float gnow = cphi[k][o] + dot3(cn[k][o], dl[k]);
                if (na[k] == 0) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) n1[k][c] = cn[k][o][c];
                    g1 = gnow;
                } else if (na[k] == 1) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) n2[k][c] = cn[k][o][c];
                    g2 = gnow;
                }
                ++na[k];
            }
            float sh[3] = {0.f, 0.f, 0.f};
            pj[k][0] = 1.f; pj[k][1] = 0.f; pj[k][2] = 0.f; pj[k][3] = 1.f; pj[k][4] = 0.f; pj[k][5] = 1.f;
            if (!isfree(k)) {
#pragma unroll
                for (int i = 0; i < 6; ++i) pj[k][i] = 0.f;
            } else if (na[k] == 1) {
                sym_add_outer(pj[k], -1.f, n1[k]);
#pragma unroll
                for (int c = 0; c < 3; ++c) sh[c] = -g1 * n1[k][c];
            } else if (na[k] == 2) {
                const float cc = dot3(n1[k], n2[k]);
                const float det = 1.f - cc * cc;
                if (!(det > 1e-4f)) bad = 1.f;
                const float id = det > 1e-4f ? 1.0f / det : 0.f;
                const float a1 = (-g1 + cc * g2) * id, a2 = (-g2 + cc * g1) * id;
                float tx[3] = {n1[k][1] * n2[k][2] - n1[k][2] * n2[k][1], n1[k][2] * n2[k][0] - n1[k][0] * n2[k][2],
                               n1[k][0] * n2[k][1] - n1[k][1] * n2[k][0]};
                const float tl = sqrtf(dot3(tx, tx));
                const float it = tl > 0.f ? 1.0f / tl : 0.f;
#pragma unroll
                for (int c = 0; c < 3; ++c) { tx[c] *= it; sh[c] = a1 * n1[k][c] + a2 * n2[k][c]; }
#pragma unroll
                for (int i = 0; i < 6; ++i) pj[k][i] = 0.f;
                sym_add_outer(pj[k], 1.f, tx);
                c12[k] = cc;
            } else if (na[k] > 2) {
                bad = 1.f;
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) dn[k][c] = isfree(k) ? dl[k][c] + sh[c] : 0.f;
        }
        if (bmax(bad) > 0.f) return;
        build_precond<false>();
        if (!(bmin(pcpd) > 0.f)) return;   // P not positive definite: a nonconvex QP, keep the interior point
        // residual of the projected stationarity: r = -Pi P dn
        float r[PPT][3], z[PPT][3], pp[PPT][3], q[PPT][3], w[PPT][3], t3[3];
        publish(V, dn);
        apply<false>(q);
        float rz = 0.f;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            sym_mul(pj[k], q[k], t3);
#pragma unroll
            for (int c = 0; c < 3; ++c) { r[k][c] = -t3[c]; w[k][c] = 0.f; }
            sym_mul(Mi[k], r[k], t3);
            sym_mul(pj[k], t3, z[k]);
#pragma unroll
            for (int c = 0; c < 3; ++c) pp[k][c] = z[k][c];
            rz += dot3(r[k], z[k]);
        }
        rz = bsum(rz);
        const float rz0 = rz;
        if (rz0 > 0.f) {
            for (int it = 0; it < kPcgMax; ++it) {
                publish(V, pp, false, false);
                apply<false>(q);
                float pq = 0.f;
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    sym_mul(pj[k], q[k], t3);
#pragma unroll
                    for (int c = 0; c < 3; ++c) q[k][c] = t3[c];
                    pq += dot3(pp[k], q[k]);
                }
                pq = bsum(pq);
                ++cnt[1];
                if (!(pq > 0.f)) return;
                const float alpha = rz / pq;
                float rzn = 0.f;
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) { w[k][c] += alpha * pp[k][c]; r[k][c] -= alpha * q[k][c]; }
                    sym_mul(Mi[k], r[k], t3);
                    sym_mul(pj[k], t3, z[k]);
                    rzn += dot3(r[k], z[k]);
                }
                rzn = bsum(rzn);
                if (!(rzn > kPcgTolAdj * kPcgTolAdj * rz0)) break;
                const float beta = rzn / rz;
                rz = rzn;
#pragma unroll
                for (int k = 0; k < PPT; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c) pp[k][c] = z[k][c] + beta * pp[k][c];
            }
        }
#pragma unroll
        for (int k = 0; k < PPT; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) dn[k][c] += w[k][c];
        // multipliers of the active pairs and the gaps of the others
        publish(V, dn);
        apply<false>(q);
        const float ltol = -1e-5f * fscale;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (!isfree(k)) continue;
            const float a1 = dot3(n1[k], q[k]), a2 = dot3(n2[k], q[k]);
            float l1 = a1, l2 = 0.f;
            if (na[k] == 2) {
                const float cc = c12[k], id = 1.0f / (1.f - cc * cc);
                l1 = (a1 - cc * a2) * id;
                l2 = (a2 - cc * a1) * id;
            }
            if (na[k] >= 1 && !(l1 >= ltol)) bad = 1.f;
            if (na[k] == 2 && !(l2 >= ltol)) bad = 1.f;
#pragma unroll
            for (int o = 0; o < NOBS; ++o) {
                if (!(o < nobs)) continue;
                float t[3];
                sym_mul(Bd[k], cn[k][o], t);
                if (clam[k][o] > dot3(cn[k][o], t) * cgap[k][o]) continue;
                const float gp = cphi[k][o] + dot3(cn[k][o], dn[k]);
                if (!(gp >= -10.f * kTolGap * (h + fabsf(cphi[k][o])))) bad = 1.f;
            }
        }
        if (bmax(bad) > 0.f) return;
#pragma unroll
        for (int k = 0; k < PPT; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) dl[k][c] = dn[k][c];
    }

    // -------------------------------------------------- step internals
    // Field-major per step: a[f * n + p], f < kAuxFields: q* - x (0..2), the
    // stage-2 correction (3..5), contact multipliers (6..), gaps (6 + kMaxObs..).
    __device__ __forceinline__ void save_aux(float* a) const {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int p = pidx(k);
            if (!active(k)) continue;
#pragma unroll
            for (int c = 0; c < 3; ++c) { a[c * n + p] = d[k][c]; a[(3 + c) * n + p] = dl[k][c]; }
#pragma unroll
            for (int o = 0; o < NOBS; ++o) {
                a[(6 + o) * n + p] = clam[k][o];
                a[(6 + kMaxObs + o) * n + p] = cgap[k][o];
            }
        }
    }
    // The state of a solved step from its saved internals: the same
    // registers and LDS mirrors solve_step leaves (same inputs, same
    // arithmetic for the spring and contact data), without solving.
    __device__ __forceinline__ void restore_step(const float* ut, const float* a) {
        begin_step(ut);                    // grippers, predictor, penalty data; publishes X
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int p = pidx(k);
            if (!isfree(k)) continue;
#pragma unroll
            for (int c = 0; c < 3; ++c) d[k][c] = a[c * n + p];
            put(D, k, d[k]);
        }
        sync();
        float F[PPT][3];
        grad_cache(false, F);              // exact Hessian data at y*
        eval_contacts();
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int p = pidx(k);
#pragma unroll
            for (int c = 0; c < 3; ++c) dl[k][c] = isfree(k) ? a[(3 + c) * n + p] : 0.f;
#pragma unroll
            for (int o = 0; o < NOBS; ++o) {
                const bool valid = o < nobs && isfree(k);
                clam[k][o] = valid ? a[(6 + o) * n + p] : 0.f;
                cgap[k][o] = valid ? a[(6 + kMaxObs + o) * n + p] : 1.f;
            }
        }
        publish(DL, dl);
        ++cnt[3];
    }

    // Full step at relaxation kappa: stages 1 and 2 (state not advanced).
    __device__ __forceinline__ void solve_step(const float* ut, float kappa) {
        begin_step(ut);
        stage1();
        stage2(kappa);
        publish(DL, dl);   // stage-2 correction mirrored for the derivatives
        ++cnt[3];
    }

    // x <- x+, v <- v+  (free: x + (d + D), (d + D)/dt; gripped: x + dt u, u)
    __device__ __forceinline__ void advance() {
        const float idt = 1.0f / dt;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (!active(k)) continue;
            if (isfree(k)) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float inc = d[k][c] + dl[k][c];
                    x[k][c] = x[k][c] + inc;
                    v[k][c] = inc * idt;
                }
                if (pen[k] >= 0)
                    for (int c = 0; c < 3; ++c) pg(k)[c] = pg(k)[3 + c];
            } else {
#pragma unroll
                for (int c = 0; c < 3; ++c) { x[k][c] = x[k][c] + dt * ug[k][c]; v[k][c] = ug[k][c]; }
            }
        }
    }

    // -------------------------------------------------- derivatives
    // (W w)_p = sum_s W_s (w_p - w_q), W_s = k l0/L^3 [(e.De) I + De e^T +
    // e De^T - 3 (e.De) e_hat e_hat^T], De = D_q - D_p (third derivative of
    // the spring energy contracted with the stage-2 correction).  The vector
    // w is mirrored in V, the correction in DL, y* = X + D.
    __device__ __forceinline__ void apply_third(float q[PPT][3], bool grip_rows) {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int p = pidx(k);
#pragma unroll
            for (int c = 0; c < 3; ++c) q[k][c] = 0.f;
            if (!active(k) || (!isfree(k) && !grip_rows)) continue;
            float wp[3], Dp[3];
            get(V, p, wp);
            get(DL, p, Dp);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int nq = nbr(k, p, s);
                if (nq < 0) continue;
                const int ty = TP::type(s);
                float e[3], De[3], we[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    e[c] = (X[c * NM + nq] - x[k][c]) + (D[c * NM + nq] - d[k][c]);
                    De[c] = DL[c * NM + nq] - Dp[c];
                    we[c] = wp[c] - V[c * NM + nq];
                }
                const float L2 = dot3(e, e);
                const float L = sqrtf(L2);
                const float il = 1.0f / L;
                const float cw = kS[ty] * rS[ty] * il * il * il;
                const float eD = dot3(e, De), ew = dot3(e, we), Dw = dot3(De, we);
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    q[k][c] += cw * (eD * we[c] + De[c] * ew + e[c] * Dw - 3.f * eD * ew * e[c] / L2);
            }
        }
    }

    // VJP of one solved step (eq. diff-sim).  In: xb, vb = cotangents of
    // (x+, v+).  Out: xb, vb = cotangents of (x, v); ubk = cotangent of the
    // gripper velocity (gripped particles only); dxb = change of xb.
    //
    // With qb = xb + vb/dt, z = K^{-1} qb and mu = P^{-1} (P - W + C - R)^T z
    // the update is xb <- (M/dt^2) mu - vb/dt, vb <- dt (1-gamma) (M/dt^2) mu.
    // Both terms of the first carry vb/dt, which grows along the horizon, so
    // it is evaluated through the increment delta = (M/dt^2) mu - qb:
    //   P delta = (M/dt^2)(C - W - R^T - N^T Lam N) z - K_el qb
    // (K_el = P - M/dt^2, the elastic part), xb <- xb + delta,
    // vb <- dt (1-gamma)(qb + delta): no cancellation of large terms.
    __device__ __forceinline__ void adjoint(float xb[PPT][3], float vb[PPT][3], float ubk[PPT][3], float kappa,
                                            float dxb[PPT][3]) {
        const float idt = 1.0f / dt;
        float qb[PPT][3], z[PPT][3], e1[PPT][3], del[PPT][3], mu[PPT][3], t1[PPT][3], t2[PPT][3];
        float bb[PPT][3];
#pragma unroll
        for (int k = 0; k < PPT; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                qb[k][c] = isfree(k) ? xb[k][c] + vb[k][c] * idt : 0.f;
                bb[k][c] = (active(k) && !isfree(k)) ? xb[k][c] : 0.f;
            }
        // stage 2: z = K^{-1} qb, K = P + N^T Lam N (with friction P + sum K_c)
        if constexpr (FRIC) {
            if (friction()) fric_blocks(kappa);
        }
        build_precond<true>();
        solve<true>(qb, z, kPcgTolAdj);
        // friction: the step depends on x directly through the tangential
        // displacement; its cotangent Lx^T z joins xb below
        float xadd[PPT][3];
#pragma unroll
        for (int k = 0; k < PPT; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) xadd[k][c] = 0.f;
        // e1 = (C - W - R^T - N^T Lam N) z ; gripped rows: bb -= (W z)_g
        publish(V, z);
        apply_third(t2, true);
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
#pragma unroll
            for (int c = 0; c < 3; ++c) e1[k][c] = 0.f;
            if (!active(k)) continue;
            if (!isfree(k)) {
#pragma unroll
                for (int c = 0; c < 3; ++c) bb[k][c] -= t2[k][c];
                continue;
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) e1[k][c] = -t2[k][c];
            float yst[3] = {x[k][0] + d[k][0], x[k][1] + d[k][1], x[k][2] + d[k][2]};
            if constexpr (FRIC) {
                if (friction()) {
                    // e1 gains sum_c Ly_c^T z, xb gains sum_c Lx_c^T z
#pragma unroll
                    for (int o = 0; o < NOBS; ++o) {
                        if (o >= nobs) continue;
                        Pair P;
                        fric_pair(k, o, kappa, yst, P);
                        float t[3];
                        fric_ly(P, z[k], true, t);
#pragma unroll
                        for (int c = 0; c < 3; ++c) e1[k][c] += t[c];
                        fric_lx(P, z[k], true, t);
#pragma unroll
                        for (int c = 0; c < 3; ++c) xadd[k][c] += t[c];
                    }
                    continue;
                }
            }
#pragma unroll
            for (int o = 0; o < NOBS; ++o) {
                if (o >= nobs) continue;
                float Hc[6], cz[3], hd[3];
                sdf_hess(otype[o], ob[o], yst, Hc);
                sym_mul(Hc, z[k], cz);
                sym_mul(Hc, dl[k], hd);
                const float w = kappa > 0.f ? clam[k][o] / cgap[k][o] : 0.f;
                const float nz = dot3(cn[k][o], z[k]);
#pragma unroll
                for (int c = 0; c < 3; ++c) e1[k][c] += clam[k][o] * cz[c] - w * nz * (hd[c] + cn[k][o][c]);
            }
        }
        // rhs = (M/dt^2) e1 - K_el qb
        publish(V, qb);
        apply<false>(t1, false, false);
        float rhs[PPT][3];
#pragma unroll
        for (int k = 0; k < PPT; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) rhs[k][c] = isfree(k) ? mdt2 * e1[k][c] - t1[k][c] : 0.f;
        build_precond<false>();
        solve<false>(rhs, del, kPcgTolAdj);
        const float imdt2 = 1.0f / mdt2;
#pragma unroll
        for (int k = 0; k < PPT; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) mu[k][c] = isfree(k) ? (qb[k][c] + del[k][c]) * imdt2 : 0.f;
        publish(V, mu);
        apply<false>(t1, true);    // gripped rows: (H_gf mu)
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (!active(k)) {
#pragma unroll
                for (int c = 0; c < 3; ++c) { dxb[k][c] = 0.f; ubk[k][c] = 0.f; }
                continue;
            }
            if (isfree(k)) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    dxb[k][c] = del[k][c] + xadd[k][c];
                    vb[k][c] = dt * (1.f - gam) * (qb[k][c] + del[k][c]);
                    xb[k][c] += del[k][c] + xadd[k][c];
                    ubk[k][c] = 0.f;
                }
                if (pen[k] >= 0) {
                    // penalty grasp: D enters F (D (y - g+)) and P (D I); its
                    // activation depends on c = x_j - g.  With z = K^{-1} qb
                    // and mu = H^{-1}(...): Dbar = -z.Delta_j - mu.(y_j - g+),
                    // g+bar = D mu + gbar, xbar_j += Dbar dD/dc,
                    // gbar = g+bar - Dbar dD/dc, ubar = dt g+bar.
                    float* G = pg(k);
                    float Dbar = -dot3(z[k], dl[k]);
#pragma unroll
                    for (int c = 0; c < 3; ++c) Dbar -= mu[k][c] * ((x[k][c] - G[3 + c]) + d[k][c]);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const float gpb = G[6] * mu[k][c] + G[10 + c];
                        xb[k][c] += Dbar * G[7 + c];
                        dxb[k][c] += Dbar * G[7 + c];
                        G[10 + c] = gpb - Dbar * G[7 + c];
                        ubk[k][c] = dt * gpb;
                    }
                }
            } else {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float tot = bb[k][c] - t1[k][c];
                    ubk[k][c] = dt * tot + vb[k][c];
                    dxb[k][c] = tot - xb[k][c];
                    xb[k][c] = tot;
                    vb[k][c] = 0.f;
                }
            }
        }
    }

    // JVP of one solved step: (dx, dv, du) -> (dx+, dv+).  du is this
    // particle's gripper tangent (gripped particles only).  Written through
    // increments so that dv+ never forms (dx+ - dx)/dt:
    //   dxhat = dx + dt (1-gamma) dv,  db = dx_g + dt du,
    //   H eps = -(K_el dxhat + H_fg db),            dy = dxhat + eps,
    //   K eta = (C - W - R - N^T Lam N) dy - W_fg db,  dx+ = dy + eta,
    //   dv+ = (1-gamma) dv + (eps + eta)/dt.
    __device__ __forceinline__ void tangent(const float dx[PPT][3], const float dv[PPT][3], const float du[PPT][3],
                                            float ox[PPT][3], float ov[PPT][3], float kappa) {
        const float idt = 1.0f / dt;
        float db[PPT][3], xh[PPT][3], r1[PPT][3], eps[PPT][3], dy[PPT][3], t1[PPT][3], t2[PPT][3];
#pragma unroll
        for (int k = 0; k < PPT; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const bool g = active(k) && !isfree(k);
                db[k][c] = g ? dx[k][c] + dt * du[k][c] : 0.f;
                xh[k][c] = isfree(k) ? dx[k][c] + dt * (1.f - gam) * dv[k][c] : 0.f;
            }
        float full[PPT][3];
#pragma unroll
        for (int k = 0; k < PPT; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) full[k][c] = isfree(k) ? xh[k][c] : db[k][c];
        publish(V, full, true);
        apply<false>(t1, false, false);   // K_el dxhat + H_fg db (free rows)
#pragma unroll
        for (int k = 0; k < PPT; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) r1[k][c] = isfree(k) ? -t1[k][c] : 0.f;
        // penalty grasp (tangent of g in GR[13..15]): dF gains
        // dD (y - g+) - D dg+ with dD = dD/dc . (dx - dg), dg+ = dg + dt du
        float pdk[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            pdk[k] = 0.f;
            if (pen[k] < 0) continue;
            const float* G = pg(k);
#pragma unroll
            for (int c = 0; c < 3; ++c) pdk[k] += G[7 + c] * (dx[k][c] - G[13 + c]);
#pragma unroll
            for (int c = 0; c < 3; ++c)
                r1[k][c] -= pdk[k] * ((x[k][c] - G[3 + c]) + d[k][c]) - G[6] * (G[13 + c] + dt * du[k][c]);
        }
        build_precond<false>();
        solve<false>(r1, eps, kPcgTolAdj);
#pragma unroll
        for (int k = 0; k < PPT; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                dy[k][c] = isfree(k) ? xh[k][c] + eps[k][c] : 0.f;
                full[k][c] = isfree(k) ? dy[k][c] : db[k][c];
            }
        publish(V, full, true);
        apply_third(t2, false);           // W_ff dy + W_fg db
        float r2[PPT][3];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
#pragma unroll
            for (int c = 0; c < 3; ++c) r2[k][c] = isfree(k) ? -t2[k][c] : 0.f;
            if (!isfree(k)) continue;
            float yst[3] = {x[k][0] + d[k][0], x[k][1] + d[k][1], x[k][2] + d[k][2]};
            if constexpr (FRIC) {
                if (friction()) {
                    // r2 gains sum_c (Ly_c dy + Lx_c dx)
#pragma unroll
                    for (int o = 0; o < NOBS; ++o) {
                        if (o >= nobs) continue;
                        Pair P;
                        fric_pair(k, o, kappa, yst, P);
                        float t[3], dxk[3] = {dx[k][0], dx[k][1], dx[k][2]};
                        fric_ly(P, dy[k], false, t);
#pragma unroll
                        for (int c = 0; c < 3; ++c) r2[k][c] += t[c];
                        fric_lx(P, dxk, false, t);
#pragma unroll
                        for (int c = 0; c < 3; ++c) r2[k][c] += t[c];
                    }
                    continue;
                }
            }
#pragma unroll
            for (int o = 0; o < NOBS; ++o) {
                if (o >= nobs) continue;
                float Hc[6], cy[3], hd[3];
                sdf_hess(otype[o], ob[o], yst, Hc);
                sym_mul(Hc, dy[k], cy);
                sym_mul(Hc, dl[k], hd);
                const float w = kappa > 0.f ? clam[k][o] / cgap[k][o] : 0.f;
                const float s2 = w * (dot3(hd, dy[k]) + dot3(cn[k][o], dy[k]));
#pragma unroll
                for (int c = 0; c < 3; ++c) r2[k][c] += clam[k][o] * cy[c] - s2 * cn[k][o][c];
            }
        }
        // penalty grasp: P gains D I, so the stage-2 right-hand side gains -dD Delta_j
#pragma unroll
        for (int k = 0; k < PPT; ++k)
            if (pen[k] >= 0)
#pragma unroll
                for (int c = 0; c < 3; ++c) r2[k][c] -= pdk[k] * dl[k][c];
        float eta[PPT][3];
        if constexpr (FRIC) {
            if (friction()) fric_blocks(kappa);
        }
        build_precond<true>();
        solve<true>(r2, eta, kPcgTolAdj);
#pragma unroll
        for (int k = 0; k < PPT; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (isfree(k)) {
                    ox[k][c] = dy[k][c] + eta[k][c];
                    ov[k][c] = (1.f - gam) * dv[k][c] + (eps[k][c] + eta[k][c]) * idt;
                } else if (active(k)) { ox[k][c] = db[k][c]; ov[k][c] = du[k][c]; }
                else { ox[k][c] = 0.f; ov[k][c] = 0.f; }
            }
        // tangent of g+ replaces that of g
#pragma unroll
        for (int k = 0; k < PPT; ++k)
            if (pen[k] >= 0)
#pragma unroll
                for (int c = 0; c < 3; ++c) pg(k)[13 + c] += dt * du[k][c];
    }
};

}  // namespace cord

// Dense per-step linearization of ropes by banded direct solves.
//
// For a rope every operator of the step derivative (the stage-1 Hessian H,
// the stage-2 matrix K = H + N^T Lam N and J = H - W + C - R of eq.
// (diff-sim)) couples a particle only with its neighbours up to distance 2
// (stretch springs at distance 1, the bending stencil at distance 2).  The
// bending coupling of particles two apart, k_b I, is diagonal, so in the 3n
// scalar unknowns (xyz of particle p at 3p..3p+2) H and K are band matrices
// of half-bandwidth 6 (a full 3x3 block two particles away would make it
// 8), and so are their band Cholesky factors; G = C - R - W couples
// neighbouring particles only (9 scalar taps per row).  So one
// workgroup per (instance, step) restores (or solves again) the step,
// assembles the bands in LDS, factors H_ff = L L^T and K_ff = U U^T (U upper
// triangular: the Cholesky factor of the index-reversed matrix) with one
// wavefront each, and then every lane solves for one column j of the step
// map on its own.
//
// Column j is the response E = dx+ - z to the unit predictor tangent z = e_j
// (z is dxhat on free particles and the gripper displacement db on gripped
// ones).  With the increments of the tangent map
//     eps = -H_ff^{-1} (H_el z)_f,   E = K_ff^{-1} (J_ff eps + Qhat z),
//     Qhat = (J - K)_ff on free columns, -W_fg on gripped columns,
// so E never forms dx+ - z by cancellation.  Since H_ff eps = -(H_el z)_f,
// the stage-2 right-hand side needs only G = C - R - W (J = H + G), whose
// half-bandwidth is 5 (springs reach one particle):
//     r = G dy - (H_el z)_f - [j free] (N^T Lam N) z,   dy = z + eps.
// Three sweeps over the rows:
//   1 (ascending)  w1 = L^{-1} r1         (r1 = -(H_el z)_f is local to j)
//   2 (descending) eps = L^{-T} w1, r (lagging 5 rows), w2 = U^{-1} r
//                  (U is upper triangular: also descending)
//   3 (ascending)  E = U^{-T} w2, written out as the A_t (and B_t) columns.
// Choosing U U^T for K makes its first triangular solve run in the same
// direction as the second solve with L, so one vector per column (w1, then
// w2 in its place) is all that must be kept between sweeps.  It is kept in a
// scratch slot owned by the workgroup's hardware slot (XCD, shader engine,
// CU, workgroup slot on the CU; [wavefront][row][lane], each wavefront's rows
// one contiguous stream): workgroups resident at the same time never share a
// slot, a slot is reused only on one XCD (one L2), and the kept data of all
// resident workgroups is a small working set rewritten in place.  Without
// scratch (or on a device whose hardware slot falls outside the table) the
// vector is kept in the column's own slot of the dv+/dv block of A_t, which
// sweep 3 overwrites last.  The band factors, J and the right-hand-side
// stencils sit in LDS and are read at wave-uniform addresses (broadcast).
//
// Outputs for column j (dx+ rows first, then dv+ rows; d_ij = [i == j]):
//   A[i][j] = d_ij + E_i,  A[3n+i][j] = E_i / dt,
//   j free:    A[i][3n+j] = dt(1-gamma)(d_ij + E_i), A[3n+i][3n+j] = (1-gamma)(d_ij + E_i)
//   j gripped: A[.][3n+j] = 0, B[i][g] = dt (d_ij + E_i), B[3n+i][g] = d_ij + E_i.
#pragma once
#include "cord_solver.h"

namespace cord {

constexpr int kBand = 6;   // half-bandwidth of H, K and of their factors in scalar unknowns
constexpr int kTri = kBand * (kBand + 1) / 2;   // entries of the trailing window of a factorization step
constexpr int kGB = 5;     // half-bandwidth of G = C - R - W
constexpr int kBlk1 = 24;  // rows per unrolled block of sweep 1
constexpr int kBlk2 = 24;  // rows per unrolled block of sweeps 2 and 3 (they load)
constexpr int kWin = 12;   // slots of the rolling windows of the recurrences
constexpr int kPf = 23;    // rows of prefetch distance for the kept vector
constexpr int kPfR = 24;   // slots of the prefetch ring
// A row's window slot is its position in the block mod kWin (mod kPfR for
// the prefetch ring), a constant of the unrolled body; the windows hold the
// last kBand values (L and U solves) and the last 11 (eps for the G product).
static_assert(kWin > 2 * kGB && kWin > kBand && kBlk1 % kWin == 0 && kBlk2 % kWin == 0,
              "windows must divide the blocks");
static_assert(kPf < kPfR && kBlk2 % kPfR == 0 && kBlk1 >= 2 * kBand && kBlk2 >= 2 * kBand,
              "prefetch ring must divide the blocks");

// LDS carve-up (floats) for up to 3*NMAX rows.  HB and NL are written only
// after the assembly has read the solver's LDS mirrors, so they reuse the
// solver's region (SA floats at the start of the workgroup's LDS); the
// other bands follow it.
template <int NMAX>
struct LinLds {
    static constexpr int N3 = 3 * NMAX;
    // inside the solver's region
    static constexpr int HB = 0;                  // H_el(i, i-m), m = 0..kBand [i][9] (H - M/dt^2 on free rows)
    static constexpr int NL = HB + N3 * 9;        // (w n n^T) row i, same-particle columns [i][3]
    static constexpr int SA = NL + N3 * 3;
    // after the solver's region
    static constexpr int LC = 0;                  // L(k+m, k), m = 1..kBand   [k][8]
    static constexpr int LI = LC + N3 * 8;        // 1 / L(k, k)
    static constexpr int UW = LI + N3;            // U(i-m, i) at [N-1-i][m-1]
    static constexpr int UD = UW + N3 * 8;        // 1 / U(i, i) at [N-1-i]
    static constexpr int UR = UD + N3;            // U(i, i+m), m = 1..kBand   [i][8]
    static constexpr int GB = UR + N3 * 8;        // G(i, i-5+q), q = 0..10 [i][12]
    static constexpr int RF = GB + N3 * 12;       // 1 if row i is free
    static constexpr int TOTAL = RF + N3;
    // B_t staging after sweep 2, over UR, GB and RF: 3 kMaxGrip columns and
    // a sink of 2 N3 floats for the lanes of free particles
    static_assert((3 * kMaxGrip + 2) * N3 <= TOTAL - UR, "B_t staging must fit in UR..RF");
};

// Raw buffer resource over one allocation (gfx9 descriptor: 32-bit data
// format, no stride).  Loads whose lane offset lies past `bytes` return zero
// without a memory access; the scalar offset is not range-checked, so the
// callers keep it inside the allocation.
struct BufRes {
    __amdgpu_buffer_rsrc_t r;
    __device__ BufRes(const float* base, uint32_t bytes)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), 0, (int)bytes, 0x00020000)) {}
    __device__ float ld(uint32_t voff, uint32_t soff) const {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
    }
    __device__ void st(float v, uint32_t voff, uint32_t soff) const {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, (int)soff, 0);
    }
    // non-temporal store (output written once and not read back here)
    __device__ void st_nt(float v, uint32_t voff, uint32_t soff) const {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, (int)soff, 2);
    }
};

// A wave-uniform row index copied into a VGPR.  LDS reads at "array + f(row)
// + constant" then keep one vector base per array and put the constant in
// the instruction's offset field; a base in a scalar register is instead
// rebuilt and copied to a VGPR for every read.
__device__ __forceinline__ int vrow(int x) {
    int r;
    asm("v_mov_b32 %0, %1" : "=v"(r) : "s"(x));
    return r;
}

__device__ __forceinline__ void sym_to_full(const float s[6], float m[3][3]) {
    m[0][0] = s[0]; m[0][1] = s[1]; m[0][2] = s[2];
    m[1][0] = s[1]; m[1][1] = s[3]; m[1][2] = s[4];
    m[2][0] = s[2]; m[2][1] = s[4]; m[2][2] = s[5];
}

// Banded Cholesky (half-bandwidth kBand) by one wavefront, in place:
// C[k][m-1] = A(k+m, k) -> L(k+m, k),  Dg[k] = A(k, k) -> 1 / L(k, k).
// Right-looking; at step k every lane has one job and writes one value:
// lanes 0..kTri-1 apply the rank-1 update to one of the kTri entries of
// the trailing kBand x kBand window, the next kBand lanes scale one entry
// of column k, the next one stores the pivot's inverse square root, the
// others write to their own
// slot of `sink` (64 floats of LDS not in use during the factorization).
// All LDS reads of a step (at addresses inside the workgroup's LDS for
// every lane) are issued before its write, and the entries a step writes
// are not read again within it, so a step costs one LDS round trip; steps
// depend on each other only through LDS, whose reads and writes a
// wavefront performs in program order.  The pivot's inverse square root is
// the hardware approximation (within 1 ulp).  Rows past N act as identity
// rows.  Returns false if a pivot was not positive (it is then replaced by
// 1 so that the sweeps stay finite).
__device__ __forceinline__ bool band_cholesky(float* C, float* Dg, int N, float* sink) {
    const int lane = (int)threadIdx.x & 63;
    // lanes 0..kTri-1 -> (a, b), 1 <= a <= b <= kBand, column-major over b
    int ua = 1, ub = 1;
    if (lane < kTri) {
        int idx = lane, b = 1;
        while (b <= kBand && idx >= b) { idx -= b; ++b; }
        ub = b;
        ua = idx + 1;
    }
    const bool upd = lane < kTri;
    const bool scl = lane >= kTri && lane < kTri + kBand;
    const bool piv = lane == kTri + kBand;
    const int sm = scl ? lane - kTri + 1 : 0;   // column entry m of a scaling lane
    // per-lane offsets relative to step k (floats): reads xa, xb from column
    // k, t from the update target; the write goes to w (stride ws) or sink
    const int ra = upd ? ua - 1 : (scl ? sm - 1 : 0);
    const int rb = upd ? ub - 1 : ra;
    float* const tgt0 = (ua == ub) ? Dg + ua : C + ua * 8 + (ub - ua) - 1;
    const int tstride = (ua == ub) ? 1 : 8;
    float* const t0 = upd ? tgt0 : Dg;
    const int ts = upd ? tstride : 1;
    float* const w0 = upd ? tgt0 : (scl ? C + sm - 1 : Dg);
    const int ws = upd ? tstride : (scl ? 8 : 1);
    const int lim = upd ? ub : (scl ? sm : 0);   // the write is real while k + lim < N
    float* const sk = sink + lane;
    const float fu = upd ? 1.f : 0.f, fs = scl ? 1.f : 0.f, fp = piv ? 1.f : 0.f;
    bool ok = true;
    for (int k = 0; k < N; ++k) {
        float d = Dg[k];
        const float xa = C[k * 8 + ra], xb = C[k * 8 + rb];
        const float tv = t0[k * ts];
        __builtin_amdgcn_wave_barrier();
        ok = ok && (d > 0.f);
        d = d > 0.f ? d : 1.f;
        const float is = __builtin_amdgcn_rsqf(d);
        const bool live = (upd || scl || piv) && (k + lim < N || scl);
        // every lane evaluates all three values and keeps its own with 0/1
        // weights (finite operands: no branch, the kept value is exact)
        const float pa = xa * is;
        const float vu = tv - pa * (xb * is);
        const float vs = (k + sm < N) ? pa : 0.f;
        const float val = fu * vu + (fs * vs + fp * is);
        *(live ? w0 + k * ws : sk) = val;
        __builtin_amdgcn_wave_barrier();
    }
    return ok;
}

// Floats of scratch per workgroup: one vector of 3 NMAX rows per lane.
template <int NT, int NMAX>
constexpr size_t kept_slot_floats() { return (size_t)NT * 3 * NMAX; }

// Scratch slots: XCDs x shader engines x CU ids x workgroup slots per CU.
constexpr int kSlotXcc = 8, kSlotSe = 4, kSlotCu = 16;
__host__ __device__ constexpr int kept_slots(int wg_per_cu) { return kSlotXcc * kSlotSe * kSlotCu * wg_per_cu; }
// After the slots: two guard words per slot (workgroups using it now,
// workgroups that have started on it), zero when the table is allocated.
__host__ __device__ constexpr size_t kept_guard_floats(int wg_per_cu) { return 2 * (size_t)kept_slots(wg_per_cu); }

// This workgroup's scratch slot from the hardware registers (wave-uniform),
// or -1 if a field lies outside the table.  HW_ID: CU_ID bits 8-11, SH_ID
// bit 12 (must be 0: it is not part of the key), SE_ID bits 13-15, TG_ID
// (workgroup slot on the CU) bits 16-19.  Whether two resident workgroups
// ever share a slot is not left to this mapping alone: the guard words
// detect any overlap in time (see lin_direct_item).
__device__ __forceinline__ int hw_slot(int wg_per_cu) {
    unsigned hw, xcc;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_HW_ID)" : "=s"(hw));
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
    const int cu = (hw >> 8) & 15, sh = (hw >> 12) & 1, se = (hw >> 13) & 7, tg = (hw >> 16) & 15, x = xcc & 15;
    if (x >= kSlotXcc || se >= kSlotSe || tg >= wg_per_cu || sh != 0) return -1;
    return ((x * kSlotSe + se) * kSlotCu + cu) * wg_per_cu + tg;
}

// One item: the A_t (and B_t) of instance `id` at step t.
template <int NT, int NMAX, int NOBS>
__device__ __forceinline__ void lin_direct_item(const KArgs& a, const int id, const int t) {
    static_assert(NT % 64 == 0 && NT >= 3 * NMAX && NT >= 128, "one lane per column, two factor waves");
    using LL = LinLds<NMAX>;
    extern __shared__ float lds[];
    const InstDev& I = a.inst[id];
    if (t >= I.T) return;
    Solver<kRope, NT, 1, NOBS, false> S;
    S.init(I, lds);
    const int n = I.n, ns = I.n_s, nu = I.n_u, N = 3 * n;
    const float kap = I.kappa_bwd, dt = I.dt, idt = 1.0f / I.dt, gam = I.gamma, mdt2 = S.mdt2;
    S.load_state(a.traj_in + I.traj_off + (int64_t)t * ns);
    if (a.aux_mode == 2 && I.kappa_fwd == I.kappa_bwd)
        S.restore_step(a.u + I.u_off + (int64_t)t * nu, a.aux + I.aux_off + (int64_t)t * kAuxFields * n);
    else
        S.solve_step(a.u + I.u_off + (int64_t)t * nu, kap);

    float* B = lds + lds_floats<NT, 1>();
    float* LC = B + LL::LC;
    float* LI = B + LL::LI;
    float* UW = B + LL::UW;
    float* UD = B + LL::UD;
    static_assert(LL::SA <= lds_floats<NT, 1>(), "HB and NL must fit in the solver's LDS");
    float* HB = lds + LL::HB;
    float* UR = B + LL::UR;
    float* GB = B + LL::GB;
    float* NL = lds + LL::NL;
    float* RF = B + LL::RF;

    // ---------------------------------------------------------- assembly
    // Thread p < n writes rows 3p..3p+2 of every band.  Blocks of particle p
    // (3x3): spring blocks K_s = sa e e^T + sb I (slot 0: p+1, slot 1: p-1),
    // bending couplings kb * (stencil^T stencil), third-derivative blocks W_s,
    // contact C_p, R_p = w n (H_phi D)^T and N^T Lam N (free particles).
    {
        const int p = threadIdx.x;
        const bool live = p < n;
        const bool fr = live && S.isfree(0);
        float Ks[2][6], Ws[2][6];
        float Cp[3][3], Rp[3][3], NLq[6], NLk[6];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int e = 0; e < 6; ++e) { Ks[s][e] = 0.f; Ws[s][e] = 0.f; }
#pragma unroll
        for (int e = 0; e < 6; ++e) { NLq[e] = 0.f; NLk[e] = 0.f; }
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) { Cp[r][c] = 0.f; Rp[r][c] = 0.f; }
        if (live) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int q = S.nbr(0, p, s);
                if (q < 0) continue;
                sym_add_outer(Ks[s], S.sa[0][s], S.se[0][s]);
                Ks[s][0] += S.sb[0][s]; Ks[s][3] += S.sb[0][s]; Ks[s][5] += S.sb[0][s];
                // W_s = cw (eD I + De e^T + e De^T - 3 eD e e^T / L^2)
                float e[3], De[3], Dp[3];
                S.get(S.DL, p, Dp);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    e[c] = (S.X[c * NT + q] - S.x[0][c]) + (S.D[c * NT + q] - S.d[0][c]);
                    De[c] = S.DL[c * NT + q] - Dp[c];
                }
                const float L2 = dot3(e, e);
                const float il = 1.0f / sqrtf(L2);
                const float cw = S.kS[0] * S.rS[0] * il * il * il;
                const float eD = dot3(e, De);
                float m[3][3];
#pragma unroll
                for (int r = 0; r < 3; ++r)
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        m[r][c] = cw * ((r == c ? eD : 0.f) + De[r] * e[c] + e[r] * De[c] - 3.f * eD * e[r] * e[c] / L2);
                Ws[s][0] = m[0][0]; Ws[s][1] = m[0][1]; Ws[s][2] = m[0][2];
                Ws[s][3] = m[1][1]; Ws[s][4] = m[1][2]; Ws[s][5] = m[2][2];
            }
            if (fr) {
                const float yst[3] = {S.x[0][0] + S.d[0][0], S.x[0][1] + S.d[0][1], S.x[0][2] + S.d[0][2]};
#pragma unroll
                for (int o = 0; o < NOBS; ++o) {
                    if (o >= S.nobs) continue;
                    float Hc[6], hd[3], Hm[3][3];
                    sdf_hess(S.otype[o], S.ob[o], yst, Hc);
                    sym_mul(Hc, S.dl[0], hd);
                    sym_to_full(Hc, Hm);
                    const float lam = S.clam[0][o], gap = S.cgap[0][o];
                    const float wk = lam / gap;
                    const float w = kap > 0.f ? wk : 0.f;
                    const float* nn = S.cn[0][o];
#pragma unroll
                    for (int r = 0; r < 3; ++r)
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            Cp[r][c] += lam * Hm[r][c];
                            Rp[r][c] += w * nn[r] * hd[c];
                        }
                    sym_add_outer(NLq, w, nn);
                    sym_add_outer(NLk, wk, nn);
                }
            }
        }
        // the solver's LDS mirrors are read for the last time above; HB and
        // NL are written over them below
        __syncthreads();
        // bending: particle c in [1, n-2] carries the stencil (1, -2, 1)
        const float kb = S.kb;
        auto inR = [&](int c) { return (c >= 1 && c <= n - 2) ? 1.f : 0.f; };
        const float bd0 = kb * (inR(p - 1) + 4.f * inR(p) + inR(p + 1));
        const float bm1 = -2.f * kb * (inR(p - 1) + inR(p));     // (p, p-1)
        const float bp1 = -2.f * kb * (inR(p) + inR(p + 1));     // (p, p+1)
        const float bm2 = kb * inR(p - 1);                        // (p, p-2)
        const float bp2 = kb * inR(p + 1);                        // (p, p+2)
        // H block (p, p+dq)[r][c], dq in -2..2
        auto Hblk = [&](int dq, int r, int c) -> float {
            const float I3 = (r == c) ? 1.f : 0.f;
            float ks[3][3];
            if (dq == 0) {
                float v = (fr ? mdt2 : 0.f) * I3 + bd0 * I3;
                sym_to_full(Ks[0], ks); v += ks[r][c];
                sym_to_full(Ks[1], ks); v += ks[r][c];
                return v;
            }
            if (dq == 1) { sym_to_full(Ks[0], ks); return -ks[r][c] + bp1 * I3; }
            if (dq == -1) { sym_to_full(Ks[1], ks); return -ks[r][c] + bm1 * I3; }
            if (dq == 2) return bp2 * I3;
            return bm2 * I3;
        };
        auto Wblk = [&](int dq, int r, int c) -> float {
            float ws[3][3];
            if (dq == 0) {
                float v = 0.f;
                sym_to_full(Ws[0], ws); v += ws[r][c];
                sym_to_full(Ws[1], ws); v += ws[r][c];
                return v;
            }
            if (dq == 1) { sym_to_full(Ws[0], ws); return -ws[r][c]; }
            if (dq == -1) { sym_to_full(Ws[1], ws); return -ws[r][c]; }
            return 0.f;
        };
        if (live) {
            int gq[kMaxGrip];
#pragma unroll
            for (int g = 0; g < kMaxGrip; ++g) gq[g] = g < I.n_grip ? I.grip_node[g] : -1;
            auto is_free = [&](int q) {
                bool f = true;
#pragma unroll
                for (int g = 0; g < kMaxGrip; ++g) f = f && (gq[g] != q);
                return f;
            };
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const int i = 3 * p + r;
                RF[i] = fr ? 1.f : 0.f;
                {
                    float nq[3][3];
                    sym_to_full(NLq, nq);
#pragma unroll
                    for (int c = 0; c < 3; ++c) NL[i * 3 + c] = nq[r][c];
                }
                float nk[3][3];
                sym_to_full(NLk, nk);
                // lower band of H (full coupling), of H_ff and (reversed) K_ff
#pragma unroll
                for (int m = 0; m <= kBand; ++m) {
                    const int k = i - m;
                    // column k = 3(p + dq) + c with dq, c fixed by r and m
                    const int off = r - m;
                    const int dq = off >= 0 ? off / 3 : -((2 - off) / 3);
                    const int c = off - 3 * dq;
                    float hv = 0.f, hf = 0.f, kf = 0.f;
                    if (k >= 0) {
                        hv = Hblk(dq, r, c);
                        const bool cf = is_free(p + dq);
                        if (fr && cf) {
                            hf = hv;
                            kf = hv + (dq == 0 ? nk[r][c] : 0.f);
                        } else {
                            hf = (m == 0) ? 1.f : 0.f;
                            kf = hf;
                        }
                    }
                    HB[i * 9 + m] = hv - ((m == 0 && fr) ? mdt2 : 0.f);   // H_el
                    if (m == 0) {
                        LI[i] = hf;
                        UD[N - 1 - i] = kf;
                    } else {
                        if (k >= 0) LC[k * 8 + m - 1] = hf;
                        UW[(N - 1 - i) * 8 + m - 1] = kf;
                    }
                }
                // G row (free rows; zero on gripped rows)
#pragma unroll
                for (int qq = 0; qq < 12; ++qq) {
                    const int k = i - kGB + qq;
                    const int off = r - kGB + qq;
                    const int dq = off >= 0 ? off / 3 : -((2 - off) / 3);
                    const int c = off - 3 * dq;
                    float gv = 0.f;
                    if (qq <= 2 * kGB && fr && k >= 0 && k < N)
                        gv = -Wblk(dq, r, c) + (dq == 0 ? Cp[r][c] - Rp[r][c] : 0.f);
                    GB[i * 12 + qq] = gv;
                }
            }
        }
        // entries that reach past the last row: L(k+m, k) with k+m >= N and
        // U(i-m, i) with i-m < 0 are zero
        if (live) {
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const int k = 3 * p + r;
#pragma unroll
                for (int m = 1; m <= kBand; ++m) {
                    if (k + m >= N) LC[k * 8 + m - 1] = 0.f;
                    if (k - m < 0) UW[(N - 1 - k) * 8 + m - 1] = 0.f;
                }
            }
        }
    }
    // flag: this step goes to the iterative kernel.  It lives in the
    // solver's reduction slots (not in use any more; HB and NL end below
    // them): a static __shared__ variable would shift the dynamic LDS base
    // off the 16-byte alignment of the band rows' 128-bit reads.
    volatile int* const redone = reinterpret_cast<volatile int*>(S.rb) + 48;
    static_assert(LL::SA <= 12 * NT, "the reduction slots must lie above HB and NL");
    if (threadIdx.x == 0) *redone = 0;
    __syncthreads();
    // ---------------------------------------------------------- factorizations
    {
        // wavefront 0 factors H_ff, wavefront 1 the reversed K_ff
        const int wv = threadIdx.x >> 6;
        bool ok = true;
        // UR is written only after both factorizations: its first 128
        // floats are the two wavefronts' sinks
        if (wv == 0) ok = band_cholesky(LC, LI, N, UR);
        else if (wv == 1) ok = band_cholesky(UW, UD, N, UR + 64);
        // a non-positive pivot: dF/dq* (or K) is not positive definite here
        // (e.g. a compressed rope); the step is done again by the iterative
        // kernel when the caller keeps per-step flags, else reported
        if (!ok && (threadIdx.x & 63) == 0) {
            if (a.redo) {
                a.redo[I.t_off + t] = 1;
                *redone = 1;
            } else if (a.status) {
                atomicMax(&a.status[id], kStNotPD);
            }
        }
    }
    __syncthreads();
    if (*redone) {         // the whole workgroup: the iterative kernel writes this step
        if (threadIdx.x == 0 && a.lin_stats) atomicAdd(a.lin_stats + 1, 1u);
        return;
    }
    // row layout of U for the descending solve: UR[i][m-1] = U(i, i+m)
    for (int i = threadIdx.x; i < N; i += NT)
#pragma unroll
        for (int m = 1; m <= kBand; ++m) UR[i * 8 + m - 1] = i + m < N ? UW[(N - 1 - i - m) * 8 + m - 1] : 0.f;
    __syncthreads();

    // ---------------------------------------------------------- column sweeps
    // Global accesses of the sweeps are raw buffer instructions over this
    // step's A_t and the kept vector's storage: a loop-invariant lane offset
    // (VGPR) plus a wave-uniform row offset in bytes (SGPR).  LDS reads of a
    // block of rows go through one base address per array and constant
    // offsets.
    const int j = threadIdx.x;
    const bool jok = j < N;
    if (a.A) {
        const int64_t aoff = a.lin_zero_off ? 0 : I.A_off, boff = a.lin_zero_off ? 0 : I.B_off;
        float* At = a.A + aoff + (int64_t)t * ns * ns;
        float* Bt = a.Bm ? a.Bm + boff + (int64_t)t * ns * nu : nullptr;
        const BufRes rA(At, (uint32_t)ns * (uint32_t)ns * 4u);
        const uint32_t rs = (uint32_t)ns * 4u;                  // bytes per row of A_t
        const uint32_t vJ = 4u * (uint32_t)j, vJN = 4u * (uint32_t)(N + j);
        const uint32_t vNJ = (uint32_t)N * rs + vJ, vK = (uint32_t)N * rs + vJN;
        const int pj = j / 3, cj = j - 3 * pj;
        const bool fj = jok && RF[jok ? j : 0] != 0.f;
        // first row that can be nonzero in w1 for any column of this
        // wavefront (wave-uniform: kept in a scalar register)
        const int i0 = __builtin_amdgcn_readfirstlane(max(0, (int)(threadIdx.x & ~63) - kBand));
        // rows that can carry a column-local right-hand-side term for some
        // column of this wavefront: |row - j| <= kBand for j in j0..j0+63
        const int jl0 = i0, jl1 = __builtin_amdgcn_readfirstlane((int)(threadIdx.x & ~63) + 63 + kBand);
        // kept vector of this lane: row r at byte rS-base + vS + r krow;
        // wbase + (r - i0) krow + wl addresses row r >= i0 for a window
        const int wf = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
        const int slot = a.kept ? hw_slot(a.kept_tg) : -1;
        // guard of the slot: thread 0 marks it busy and counts a start; a
        // workgroup that finds it busy leaves it alone and hands its step to
        // the iterative kernel (the one using it detects the overlap at its
        // end, from the start count, and does the same)
        uint32_t* const guard = slot >= 0 ? reinterpret_cast<uint32_t*>(
            a.kept + (size_t)kept_slots(a.kept_tg) * kept_slot_floats<NT, NMAX>()) + 2 * slot : nullptr;
        uint32_t my_start = 0;
        if (guard) {
            if (threadIdx.x == 0) {
                const uint32_t busy = atomicAdd(guard, 1u);
                my_start = atomicAdd(guard + 1, 1u);
                *redone = busy != 0u ? 1 : 0;
            }
            __syncthreads();
            if (*redone) {
                if (threadIdx.x == 0) {
                    atomicSub(guard, 1u);
                    if (a.redo) a.redo[I.t_off + t] = 1;
                    if (a.lin_stats) { atomicAdd(a.lin_stats, 1u); atomicAdd(a.lin_stats + 1, 1u); }
                }
                return;
            }
        }
        const float* kbase;
        uint32_t kbytes, vS, krow, wl;
        const float* wbase;
        if (slot >= 0) {   // scratch [wavefront][row][lane], 256 bytes a row
            kbase = a.kept + (size_t)slot * kept_slot_floats<NT, NMAX>();
            kbytes = (uint32_t)(NT * LL::N3 * 4);
            vS = (uint32_t)(wf * LL::N3) * 256u + 4u * (threadIdx.x & 63);
            krow = 256u;
            wl = 4u * (threadIdx.x & 63);
            wbase = kbase + (wf * LL::N3 + i0) * 64;
        } else {           // column j of the dv+/dv block of A_t
            kbase = At;
            kbytes = (uint32_t)ns * (uint32_t)ns * 4u;
            vS = vK;
            krow = rs;
            wl = 4u * (uint32_t)j;
            wbase = At + (int64_t)(N + i0) * ns + N;
        }
        const BufRes rS(kbase, kbytes);

        // Each sweep runs in blocks of rows whose body is unrolled, so the
        // window slot of a row is a constant and the rolling windows stay in
        // registers.  Blocks that cannot reach
        // past either end of the matrix run a body without any condition
        // (one basic block, so its LDS reads can be issued ahead of the
        // arithmetic); the first and last blocks run the guarded body.  Sums
        // are taken from the oldest window entry to the newest, so each
        // recurrence waits on one multiply-add per row.  Band entries outside
        // the band are read at clamped (valid) indices and zeroed by selects.

        // sweep 1: w1 = L^{-1} r1 for rows i0..N-1 (rows above i0 are zero
        // for every column of this wavefront and are not stored)
        if (jok) {
            float w[kWin];
#pragma unroll
            for (int u = 0; u < kWin; ++u) w[u] = 0.f;
            for (int tb = 0; i0 + tb < N; tb += kBlk1) {
                const int r0 = i0 + tb;                         // row of u = 0
                const float* LCb = lds + vrow((int)(LC - lds) + (r0 - kBand) * 8);   // L(i, i-m) at LCb[(u+kBand-m)*8 + m-1]
                const float* LIb = lds + vrow((int)(LI - lds) + r0);
                const float* RFb = lds + vrow((int)(RF - lds) + r0);
                const int db = r0 - j;
                auto row = [&](const int u, const bool guard, const bool loc) {
                    const int i = r0 + u;
                    if (guard && i >= N) return;
                    float acc = 0.f;
                    if (loc) {
                        // -(H_el z)_f: H_el(max(i,j), min(i,j)) inside the band
                        const int dd = db + u;
                        const int ddc = min(max(dd, -kBand), kBand);
                        const int hidx = 9 * j - ddc + (dd >= 0 ? 9 * dd + 2 * ddc : 0);
                        const float h = HB[hidx];
                        const float rfi = RFb[u];
                        acc = (dd == ddc) ? -rfi * h : 0.f;
                    }
#pragma unroll
                    for (int m = kBand; m >= 1; --m)
                        if (!guard || i - m >= i0) acc -= LCb[(u + kBand - m) * 8 + m - 1] * w[(u - m + kWin) % kWin];
                    const float wi = acc * LIb[u];
                    w[u % kWin] = wi;
                    rS.st(wi, vS, (uint32_t)(r0 + u) * krow);
                };
                if (tb > 0 && r0 + kBlk1 <= N) {
                    if (r0 <= jl1) {
#pragma unroll
                        for (int u = 0; u < kBlk1; ++u) row(u, false, true);
                    } else {   // no column of this wavefront reaches these rows
#pragma unroll
                        for (int u = 0; u < kBlk1; ++u) row(u, false, false);
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < kBlk1; ++u) row(u, true, true);
                }
            }
        }
        // sweep 2 (descending, position s = N-1-i): eps, r (kGB rows behind), w2
        if (jok) {
            // loads of w1 through a window that starts at row i0: rows above
            // it fall outside the window (the lane offset wraps past its
            // size) and read as zero without touching memory
            const BufRes rK(wbase, (uint32_t)(N - i0) * krow);
            const uint32_t vW = wl;
            float e[kWin], w2[kWin], pf[kPfR];
#pragma unroll
            for (int u = 0; u < kWin; ++u) { e[u] = 0.f; w2[u] = 0.f; }
#pragma unroll
            for (int u = 0; u < kPfR; ++u) pf[u] = 0.f;
#pragma unroll
            for (int u = 0; u < kPf; ++u) pf[u] = rK.ld(vW + (uint32_t)(N - 1 - u - i0) * krow, 0);
            for (int sb = 0; sb < N + kGB; sb += kBlk2) {
                // row of position sb+u is i = ib + v, v = kBlk2-1-u
                const int ib = N - kBlk2 - sb;
                const int mb = ib + kGB;                        // mrow = mb + v
                const float* LCb = lds + vrow((int)(LC - lds) + ib * 8);
                const float* LIb = lds + vrow((int)(LI - lds) + ib);
                const float* GBb = lds + vrow((int)(GB - lds) + mb * 12);
                const float* URb = lds + vrow((int)(UR - lds) + mb * 8);
                const float* RFb = lds + vrow((int)(RF - lds) + mb);
                const float* NLb = NL + mb * 3 + cj;
                const float* UDb = lds + vrow((int)(UD - lds) + sb - kGB);   // UD[N-1-mrow] = UDb[u]
                const int qb = j - mb;                          // dq = j - mrow = qb - v
                const uint32_t vpf = vW + (uint32_t)(ib - kPf - i0) * krow;   // row i-kPf = ib-kPf+v
                auto row = [&](const int u, const bool guard, const bool loc) {
                    const int v = kBlk2 - 1 - u;
                    const int sp = sb + u;
                    const int i = ib + v;
                    if (guard && sp >= N + kGB) return;
                    // kept w1 kPf rows ahead
                    pf[(u + kPf) % kPfR] = rK.ld(vpf + (uint32_t)v * krow, 0);
                    float ei = 0.f;
                    if (!guard || i >= 0) {
                        const float4 l0 = *reinterpret_cast<const float4*>(LCb + v * 8);
                        const float4 l1 = *reinterpret_cast<const float4*>(LCb + v * 8 + 4);
                        const float lc[8] = {l0.x, l0.y, l0.z, l0.w, l1.x, l1.y, l1.z, l1.w};
                        float acc = pf[u % kPfR];
#pragma unroll
                        for (int m = kBand; m >= 1; --m) acc -= lc[m - 1] * e[(u - m + kWin) % kWin];
                        ei = acc * LIb[v];
                    }
                    e[u % kWin] = ei;
                    if (guard && i + kGB >= N) { w2[u % kWin] = 0.f; return; }
                    // column-local part: G(m, j) - H_el(m, j) - [same particle] NLN(m, j)
                    // (a same-particle column of a free row is free)
                    float r = 0.f;
                    if (loc) {
                        const int dq = qb - v;
                        const int dqc = min(max(dq, -kBand), kBand), dgc = min(max(dq, -kGB), kGB);
                        const int hidx = 9 * j + dqc - (dq <= 0 ? 9 * dq + 2 * dqc : 0);
                        const float hv = HB[hidx];
                        const float gv = GBb[v * 12 + kGB + dgc];
                        const float nl = NLb[v * 3];
                        const bool same = (uint32_t)(cj - dq) <= 2u;
                        r = ((dq == dgc) ? gv : 0.f) - (same ? nl : 0.f) - ((dq == dqc) ? hv : 0.f);
                    }
                    // G(m, m-5..m+5) eps; e[(u - qq)] holds eps_{mrow - 5 + qq}.
                    // Row mrow = 3p + rc couples with particles p-1, p, p+1
                    // only: taps qq = 2-rc .. 10-rc (the others are zero).
                    // ib is a multiple of 3, so rc = (kGB + v) mod 3 is a
                    // constant of the unrolled body.
                    const int rc = (kGB + v) % 3;
                    const float4 g0 = *reinterpret_cast<const float4*>(GBb + v * 12);
                    const float4 g1 = *reinterpret_cast<const float4*>(GBb + v * 12 + 4);
                    const float4 g2 = *reinterpret_cast<const float4*>(GBb + v * 12 + 8);
                    const float gr[12] = {g0.x, g0.y, g0.z, g0.w, g1.x, g1.y, g1.z, g1.w, g2.x, g2.y, g2.z, g2.w};
#pragma unroll
                    for (int qq = 2 * kGB; qq >= 0; --qq)
                        if (qq >= 2 - rc && qq <= 2 * kGB - rc) r += gr[qq] * e[(u - qq + kWin) % kWin];
                    if (loc) r *= RFb[v];   // (G rows of gripped particles are zero)
                    const float4 q0 = *reinterpret_cast<const float4*>(URb + v * 8);
                    const float4 q1 = *reinterpret_cast<const float4*>(URb + v * 8 + 4);
                    const float ur[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
                    float pre = 0.f;
#pragma unroll
                    for (int q = kBand; q >= 2; --q) pre += ur[q - 1] * w2[(u - q + kWin) % kWin];
                    const float acc = (r - pre) - ur[0] * w2[(u - 1 + kWin) % kWin];
                    const float wv = acc * UDb[u];
                    w2[u % kWin] = wv;
                    rS.st(wv, vS, (uint32_t)(mb + v) * krow);
                };
                if (sb >= kGB && sb + kBlk2 <= N) {
                    if (mb + kBlk2 - 1 >= jl0 && mb <= jl1) {
#pragma unroll
                        for (int u = 0; u < kBlk2; ++u) row(u, false, true);
                    } else {   // no column of this wavefront reaches these rows
#pragma unroll
                        for (int u = 0; u < kBlk2; ++u) row(u, false, false);
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < kBlk2; ++u) row(u, true, true);
                }
            }
        }
        // UR, GB and RF are not read again: B_t columns are staged there
        __syncthreads();
        float* BS = B + LL::UR;                         // [3 kMaxGrip][N3]: column 3g+c of B_t
        float* BD = BS + 3 * kMaxGrip * LL::N3;         // per-lane sink for columns that are not gripped
        // sweep 3 (ascending): E = U^{-T} w2 and the outputs
        if (jok) {
            int gj = -1;
            for (int g = 0; g < I.n_grip; ++g)
                if (I.grip_node[g] == pj) gj = g;
            float* const bsl = gj >= 0 ? BS + (3 * gj + cj) * LL::N3 : BD + j;
            float E[kWin], pf[kPfR];
#pragma unroll
            for (int u = 0; u < kWin; ++u) E[u] = 0.f;
#pragma unroll
            for (int u = 0; u < kPfR; ++u) pf[u] = 0.f;
#pragma unroll
            for (int u = 0; u < kPf; ++u) pf[u] = rS.ld(vS, (uint32_t)min(u, N - 1) * krow);
            const float c1 = dt * (1.f - gam), omg = 1.f - gam;
            const float cv = fj ? c1 : 0.f, vv = fj ? omg : 0.f;
            for (int tb = 0; tb < N; tb += kBlk2) {
                // U(i-q, i) at UWb[(kBlk2-1-u)*8 + q-1], 1/U(i,i) at UDb[kBlk2-1-u]
                const float* UWb = lds + vrow((int)(UW - lds) + (N - kBlk2 - tb) * 8);
                const float* UDb = lds + vrow((int)(UD - lds) + N - kBlk2 - tb);
                float* const bsb = bsl + tb;
                const uint32_t so = (uint32_t)tb * rs;
                auto row = [&](const int u, const bool guard) {
                    const int i = tb + u;
                    if (guard && i >= N) return;
                    pf[(u + kPf) % kPfR] = rS.ld(vS, (uint32_t)(guard ? min(i + kPf, N - 1) : i + kPf) * krow);
                    const float4 c0 = *reinterpret_cast<const float4*>(UWb + (kBlk2 - 1 - u) * 8);
                    const float4 c1v = *reinterpret_cast<const float4*>(UWb + (kBlk2 - 1 - u) * 8 + 4);
                    const float uc[8] = {c0.x, c0.y, c0.z, c0.w, c1v.x, c1v.y, c1v.z, c1v.w};
                    float acc = pf[u % kPfR];
#pragma unroll
                    for (int q = kBand; q >= 1; --q) acc -= uc[q - 1] * E[(u - q + kWin) % kWin];
                    const float Ei = acc * UDb[kBlk2 - 1 - u];
                    E[u % kWin] = Ei;
                    const float dx = (i == j ? 1.f : 0.f) + Ei;
                    const uint32_t sr = so + (uint32_t)u * rs;
                    rA.st_nt(dx, vJ, sr);
                    rA.st_nt(Ei * idt, vNJ, sr);
                    rA.st_nt(cv * dx, vJN, sr);
                    rA.st_nt(vv * dx, vK, sr);
                    bsb[u] = dx;
                };
                if (tb + kBlk2 + kPf <= N) {
#pragma unroll
                    for (int u = 0; u < kBlk2; ++u) row(u, false);
                } else {
#pragma unroll
                    for (int u = 0; u < kBlk2; ++u) row(u, true);
                }
            }
        }
        // end of the slot's use: another workgroup that started on it since
        // (or was on it at the start) may have overwritten the kept vectors,
        // so the step is handed to the iterative kernel, which runs after
        // this launch and rewrites all of A_t and B_t for it
        if (guard) {
            __syncthreads();
            if (threadIdx.x == 0) {
                const uint32_t starts = atomicAdd(guard + 1, 0u);
                const uint32_t busy = atomicSub(guard, 1u);
                if (starts != my_start + 1u || busy != 1u) {
                    if (a.redo) a.redo[I.t_off + t] = 1;
                    if (a.lin_stats) { atomicAdd(a.lin_stats, 1u); atomicAdd(a.lin_stats + 1, 1u); }
                    if (!a.redo && a.status) atomicMax(&a.status[id], kStNotPD);
                }
            }
        }
        // B_t: j gripped (node of gripper g, coordinate c) gives column 3g+c,
        // B[i][3g+c] = dt (d_ij + E_i), B[3n+i][3g+c] = d_ij + E_i
        if (Bt) {
            __syncthreads();
            for (int idx = threadIdx.x; idx < N * nu; idx += NT) {
                const int i = idx / nu, s = idx - i * nu;
                const float v = BS[s * LL::N3 + i];
                __builtin_nontemporal_store(dt * v, Bt + (int64_t)i * nu + s);
                __builtin_nontemporal_store(v, Bt + (int64_t)(N + i) * nu + s);
            }
        }
    }
    // a step done again by the iterative kernel reports that kernel's status
    if (threadIdx.x == 0 && a.status) atomicMax(&a.status[id], S.status);
    if (threadIdx.x == 0 && a.counters)
        for (int i = 0; i < 4; ++i) atomicAdd(&a.counters[4 * id + i], S.cnt[i]);
}

// Grid (blocks of a.ids, steps): one workgroup per (instance, step).
template <int NT, int NMAX, int NOBS>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void linearize_direct_kernel(KArgs a) {
    lin_direct_item<NT, NMAX, NOBS>(a, a.ids[blockIdx.x], (int)blockIdx.y);
}

template <int NT, int NMAX, int NOBS>
struct LinDirect {
    static constexpr size_t kLds = sizeof(float) * (lds_floats<NT, 1>() + LinLds<NMAX>::TOTAL);
    static constexpr size_t kSlot = kept_slot_floats<NT, NMAX>();
    static int resident_per_cu() {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, linearize_direct_kernel<NT, NMAX, NOBS>, NT, kLds) !=
            hipSuccess)
            nb = 0;
        return nb;
    }
    static hipError_t launch(const KArgs& a, int nblk, int tmax, hipStream_t s) {
        hipLaunchKernelGGL((linearize_direct_kernel<NT, NMAX, NOBS>), dim3(nblk, tmax), dim3(NT), kLds, s, a);
        return hipGetLastError();
    }
};

}  // namespace cord

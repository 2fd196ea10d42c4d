// Output-feedback SLS, stage 3 (Sec. 4.2): the Kalman recursion (eq.
// kalman_recursions) serially or as the associative scan of eqs.
// combination_rules / initialization, the observer propagations (eq.
// backward_propagations), the assembly of the closed-loop responses and the
// tube widths of the tightening constraints (eq. of_optimization).
//
// C = I (the perception returns the full state, Sec. 4.4), so p = n.  Per
// instance b and step j: A_j, E_j, F_j are n x n row-major, blocks of
// (B, N, n, n) arrays; the horizon operators are dense row-major matrices of
// (N+1) block rows (block (k, j) at rows k r, columns j c).
//
// Building blocks, all workgroup-wide (256 threads, 4 wavefronts):
//   wg_gemm   C = alpha op(A) op(B) + add1 + add2 + diag I, 64 x 64 output
//             tiles, K in chunks of 32 staged through LDS, each wavefront a
//             32 x 32 quarter on v_mfma_f32_16x16x4f32 (FP32 in, FP32 acc);
//   wg_solve  Gauss-Jordan with partial pivoting on [M | R] (n x (n + m)),
//             in LDS when it fits, else in a global workspace.
// The operands are small (n ~ 10^2): each matrix op of a step or of a scan
// combination is one workgroup's job, and the parallelism is across
// instances, steps and scan elements.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <new>
#include <vector>

#include "../../include/cord.h"
#include "cord_host.h"

namespace cord {
namespace sls {

constexpr int kThreads = 256;
constexpr int kTile = 64;                 // output tile edge
constexpr int kChunk = 32;                // K chunk
constexpr int kPadA = kChunk + 1;         // As[64][33]
constexpr int kPadB = kTile + 1;          // Bs[32][65]
constexpr int kGemmLds = kTile * kPadA + kChunk * kPadB + 2 * kThreads;   // + reduction scratch
constexpr size_t kMaxLdsBytes = 150 * 1024;

typedef float f4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- workgroup GEMM
// C[r][c] = alpha sum_k op(A)[r][k] op(B)[k][c] + add1[r][c] + add2[r][c] + (r == c ? diag : 0)
// for r < M, c < N.  op(X)[r][c] = tX ? X[c ldx + r] : X[r ldx + c].  Pointers
// may point to global memory or LDS; C must not overlap A or B (add1/add2 may
// be C itself).  Ends with a barrier: C is visible to the whole workgroup.
__device__ __forceinline__ void wg_gemm(float* C, int ldc, const float* A, int lda, bool tA, const float* B, int ldb, bool tB,
                        int M, int N, int K, float alpha, const float* add1, int ld1, const float* add2, int ld2,
                        float diag, float* lds) {
    float* As = lds;
    float* Bs = lds + kTile * kPadA;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
    const int l16 = lane & 15, lk = lane >> 4;
    // operand elements per thread and chunk: loaded into registers one
    // chunk ahead, so the loads of chunk k+1 are in flight during the
    // products of chunk k
    constexpr int kPer = kTile * kChunk / kThreads;
    float va[kPer], vb[kPer];
    // element q of this thread: op(A) row ra0 + q dra, column ca0 + q dca
    // (inside the chunk), and likewise for op(B)
    const int ra0 = tA ? (tid & 63) : (tid >> 5), ca0 = tA ? (tid >> 6) : (tid & 31);
    const int dra = tA ? 0 : kThreads / kChunk, dca = tA ? kThreads / kTile : 0;
    const int rb0 = tB ? (tid & 31) : (tid >> 6), cb0 = tB ? (tid >> 5) : (tid & 63);
    const int drb = tB ? 0 : kThreads / kTile, dcb = tB ? kThreads / kChunk : 0;
    auto load = [&](int tm, int tn, int k0) {
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int gr = tm + ra0 + q * dra, gc = k0 + ca0 + q * dca;
            const size_t off = tA ? (size_t)gc * lda + gr : (size_t)gr * lda + gc;
            va[q] = (gr < M && gc < K) ? A[off] : 0.f;
        }
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int gr = k0 + rb0 + q * drb, gc = tn + cb0 + q * dcb;
            const size_t off = tB ? (size_t)gc * ldb + gr : (size_t)gr * ldb + gc;
            vb[q] = (gr < K && gc < N) ? B[off] : 0.f;
        }
    };
    load(0, 0, 0);
    for (int tm = 0; tm < M; tm += kTile)
        for (int tn = 0; tn < N; tn += kTile) {
            f4 acc[2][2];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
            for (int k0 = 0; k0 < K; k0 += kChunk) {
#pragma unroll
                for (int q = 0; q < kPer; ++q) {
                    As[(ra0 + q * dra) * kPadA + ca0 + q * dca] = va[q];
                    Bs[(rb0 + q * drb) * kPadB + cb0 + q * dcb] = vb[q];
                }
                __syncthreads();
                // the next chunk of this tile, else the first chunk of the next
                // tile (past the last tile every element is out of range)
                {
                    int nm = tm, nn_ = tn, nk = k0 + kChunk;
                    if (nk >= K) {
                        nk = 0;
                        nn_ = tn + kTile;
                        if (nn_ >= N) { nn_ = 0; nm = tm + kTile; }
                    }
                    load(nm, nn_, nk);
                }
#pragma unroll
                for (int kk = 0; kk < kChunk; kk += 4) {
                    const int kr = kk + lk;
                    const float a0 = As[(wm + l16) * kPadA + kr];
                    const float a1 = As[(wm + 16 + l16) * kPadA + kr];
                    const float b0 = Bs[kr * kPadB + wn + l16];
                    const float b1 = Bs[kr * kPadB + wn + 16 + l16];
                    acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
                    acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
                    acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
                    acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
                }
                __syncthreads();
            }
            // accumulator v of lane l: row 4 (l / 16) + v, column l % 16 of its
            // 16 x 16 block.  The addends of a block are read before any of
            // its elements of C is written (each element is read and written
            // by its own thread, so C may be add1 or add2).
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int r0 = tm + wm + 16 * i + 4 * lk, c = tn + wn + 16 * j + l16;
                    float ad1[4], ad2[4];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const bool in = r0 + v < M && c < N;
                        ad1[v] = (add1 && in) ? add1[(size_t)(r0 + v) * ld1 + c] : 0.f;
                        ad2[v] = (add2 && in) ? add2[(size_t)(r0 + v) * ld2 + c] : 0.f;
                    }
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int r = r0 + v;
                        if (r < M && c < N) {
                            float x = alpha * acc[i][j][v];
                            if (add1) x += ad1[v];
                            if (add2) x += ad2[v];
                            if (r == c) x += diag;
                            C[(size_t)r * ldc + c] = x;
                        }
                    }
                }
        }
    __syncthreads();
}

// Element-wise pass over `total` elements by the workgroup: st(e, ld(e)).
// Four elements per thread are loaded before any is stored, so the loads
// are in flight together (stores through a pointer that may alias the
// sources would otherwise order each load after the previous store).  An
// element is loaded and stored by the same thread, so dst may alias src
// element for element.  No barrier.
template <class Ld, class St>
__device__ __forceinline__ void wg_map(int total, Ld ld, St st) {
    for (int e0 = threadIdx.x; e0 < total; e0 += 4 * kThreads) {
        float v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = e0 + q * kThreads;
            v[q] = e < total ? ld(e) : 0.f;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = e0 + q * kThreads;
            if (e < total) st(e, v[q]);
        }
    }
}

// dst[r][c] = alpha src[r][c] (+ beta I), workgroup-wide, ends with a barrier.
__device__ __forceinline__ void wg_copy(float* dst, int ldd, const float* src, int lds_, int M, int N, float alpha, float diag) {
    wg_map(
        M * N,
        [&](int e) {
            const int r = e / N, c = e - r * N;
            return src[(size_t)r * lds_ + c];
        },
        [&](int e, float v) {
            const int r = e / N, c = e - r * N;
            dst[(size_t)r * ldd + c] = alpha * v + (r == c ? diag : 0.f);
        });
    __syncthreads();
}

// dst = src^T (n x n), workgroup-wide, ends with a barrier.
__device__ __forceinline__ void wg_transpose(float* dst, const float* src, int n) {
    wg_map(
        n * n,
        [&](int e) {
            const int r = e / n, c = e - r * n;
            return src[(size_t)c * n + r];
        },
        [&](int e, float v) { dst[e] = v; });
    __syncthreads();
}

__device__ __forceinline__ void wg_zero(float* dst, int ldd, int M, int N) {
    for (int e = threadIdx.x; e < M * N; e += kThreads) {
        const int r = e / N, c = e - r * N;
        dst[(size_t)r * ldd + c] = 0.f;
    }
    __syncthreads();
}

__device__ __forceinline__ void wg_ident(float* dst, int ldd, int n) {
    for (int e = threadIdx.x; e < n * n; e += kThreads) {
        const int r = e / n, c = e - r * n;
        dst[(size_t)r * ldd + c] = r == c ? 1.f : 0.f;
    }
    __syncthreads();
}

// ---------------------------------------------------------------- workgroup solve
// A lane's value from the lane that the DPP control CTRL names (all rows and
// banks enabled).
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}

// Gauss-Jordan with partial pivoting on G = [M | R] (n rows, ld = n + m):
// on return G[:, n : n + m] = M^{-1} R.  Returns false if a pivot is zero or
// not finite.  `red` is 2 * kThreads floats of LDS.  Per column: the first
// wavefront finds the pivot with DPP and lane reads (no barrier inside),
// then one barrier each after the search, the row swap and the
// elimination.
__device__ __forceinline__ bool wg_solve(float* G, int ld, int n, int m, float* red) {
    const int tid = threadIdx.x;
    const int W = n + m;
    int* pidx = reinterpret_cast<int*>(red);
    bool ok = true;
    for (int k = 0; k < n; ++k) {
        if (tid < 64) {
            // the largest |G[i][k]| for i >= k, lowest row on ties, as the
            // largest key (bits of |v|, ~i) (the bits of a non-negative
            // float order like its value; a NaN counts as 0).  Maximum
            // inside rows of 16 lanes by DPP, then across the four rows.
            uint32_t hi = 0u, lo = 0u;
            for (int i = k + tid; i < n; i += 64) {
                const float a = fabsf(G[i * ld + k]);
                const uint32_t h = a == a ? __float_as_uint(a) : 0u, l = ~(uint32_t)i;
                if (h > hi || (h == hi && l > lo)) { hi = h; lo = l; }
            }
            auto take = [&](uint32_t oh, uint32_t ol) {
                if (oh > hi || (oh == hi && ol > lo)) { hi = oh; lo = ol; }
            };
            take(dpp_u32<0xB1>(hi), dpp_u32<0xB1>(lo));     // quad_perm [1,0,3,2]
            take(dpp_u32<0x4E>(hi), dpp_u32<0x4E>(lo));     // quad_perm [2,3,0,1]
            take(dpp_u32<0x141>(hi), dpp_u32<0x141>(lo));   // row_half_mirror
            take(dpp_u32<0x140>(hi), dpp_u32<0x140>(lo));   // row_mirror
#pragma unroll
            for (int r = 16; r < 64; r += 16)
                take((uint32_t)__builtin_amdgcn_readlane((int)hi, r), (uint32_t)__builtin_amdgcn_readlane((int)lo, r));
            hi = (uint32_t)__builtin_amdgcn_readlane((int)hi, 0);
            lo = (uint32_t)__builtin_amdgcn_readlane((int)lo, 0);
            if (tid == 0) {
                const int bi = (int)~lo;
                pidx[0] = bi;
                red[1] = G[bi * ld + k];
            }
        }
        __syncthreads();
        const int p = pidx[0];
        const float pv = red[1];
        if (!(fabsf(pv) > 0.f) || !isfinite(pv)) ok = false;
        const float inv = 1.f / pv;
        // swap rows k and p and scale the new row k (columns k .. W-1)
        for (int c = k + tid; c < W; c += kThreads) {
            const float a = G[k * ld + c];
            const float b = G[p * ld + c];
            G[p * ld + c] = a;
            G[k * ld + c] = b * inv;
        }
        __syncthreads();
        // eliminate column k from every other row (columns k+1 .. W-1) in
        // blocks of four rows: the flat index e = b wc + (c - k - 1) over
        // row blocks b advances by kThreads per pass, and a pass issues all
        // its reads (the pivot row's entry, the four multipliers in column
        // k and the four entries) before its writes.  Column k and the
        // pivot row are not written here, and each entry is read and
        // written by one thread.
        const int wc = W - k - 1;
        if (wc > 0) {
            const int nb = (n + 3) / 4;
            int b = tid / wc, c = tid - b * wc;
            const int db = kThreads / wc, dc = kThreads - db * wc;
            for (; b < nb;) {
                const int col = k + 1 + c;
                const float pk = G[k * ld + col];
                float mv[4], gv[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = 4 * b + q;
                    const bool on = i < n && i != k;
                    mv[q] = on ? G[i * ld + k] : 0.f;
                    gv[q] = on ? G[i * ld + col] : 0.f;
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = 4 * b + q;
                    if (i < n && i != k) G[i * ld + col] = gv[q] - mv[q] * pk;
                }
                b += db;
                c += dc;
                if (c >= wc) { c -= wc; ++b; }
            }
        }
        __syncthreads();
    }
    return ok;
}

// ---------------------------------------------------------------- arguments
struct Args {
    int B, N, n, m;            // instances, horizon, state size, input size
    const float* A;            // (B, N, n, n)
    const float* E;            // (B, N, n, n)
    const float* F;            // (B, N, n, n)
    const float* Xi;           // (B, n, n)
    float* Qw;                 // (B, N, n, n): E E^T
    float* Rv;                 // (B, N, n, n): F F^T
    float* el[2];              // scan elements (B, N+1, 3, n, n): At, Dt, P
    float* Pi;                 // (B, N+1, n, n)
    float* L;                  // (B, N, n, n)
    float* ws;                 // per-workgroup workspace
    size_t ws_stride;          // floats per workgroup slot
    int32_t* status;           // (B): CORD_ST_NOT_PD if a pivot vanished
    int g_in_lds;              // the solve matrix lives in LDS
};

__device__ __forceinline__ size_t nn(const Args& a) { return (size_t)a.n * a.n; }
__device__ __forceinline__ void flag(const Args& a, int b, bool ok) {
    if (!ok && threadIdx.x == 0) atomicMax(a.status + b, (int)CORD_ST_NOT_PD);
}
// The solve matrix G of a workgroup lives in LDS after the GEMM region when
// it fits, else in the workgroup's global slot.  The kernels run their body
// once for each case (`with_g`), so that in the LDS case every access to G
// is an LDS instruction (a pointer that may be either would make them all
// generic ones, slower and with 64-bit addressing).
template <class Body>
__device__ __forceinline__ void with_g(const Args& a, float* lds, float* slot, Body body) {
    if (a.g_in_lds) body(lds + kGemmLds);
    else body(slot);
}

// ---------------------------------------------------------------- kernels
// grid (N, B): Qw_j = E_j E_j^T, Rv_j = F_j F_j^T; with `scan`, the scan
// elements (eq. initialization): e_0 = (0, 0, Xi Xi^T) and
// e_{j+1} = (A_j^T, (F_j F_j^T)^{-1}, E_j E_j^T) (C = I).
__global__ __launch_bounds__(kThreads) void prep_kernel(Args a, int scan) {
    extern __shared__ float lds[];
    const int j = blockIdx.x, b = blockIdx.y;
    const int n = a.n;
    const size_t o = ((size_t)b * a.N + j) * nn(a);
    float* slot = a.ws + ((size_t)b * a.N + j) * a.ws_stride;
    wg_gemm(a.Qw + o, n, a.E + o, n, false, a.E + o, n, true, n, n, n, 1.f, nullptr, 0, nullptr, 0, 0.f, lds);
    wg_gemm(a.Rv + o, n, a.F + o, n, false, a.F + o, n, true, n, n, n, 1.f, nullptr, 0, nullptr, 0, 0.f, lds);
    if (!scan) return;
    float* e = a.el[0] + ((size_t)b * (a.N + 1) + j + 1) * 3 * nn(a);
    wg_transpose(e, a.A + o, n);
    // Dt = (F F^T)^{-1}: solve [F F^T | I]
    with_g(a, lds, slot, [&](float* G) {
        wg_copy(G, 2 * n, a.Rv + o, n, n, n, 1.f, 0.f);
        for (int x = threadIdx.x; x < n * n; x += kThreads) {
            const int r = x / n, c = x - r * n;
            G[r * 2 * n + n + c] = r == c ? 1.f : 0.f;
        }
        __syncthreads();
        flag(a, b, wg_solve(G, 2 * n, n, n, lds + kGemmLds - 2 * kThreads));
        wg_copy(e + nn(a), n, G + n, 2 * n, n, n, 1.f, 0.f);
    });
    wg_copy(e + 2 * nn(a), n, a.Qw + o, n, n, n, 1.f, 0.f);
    if (j == 0) {
        float* e0 = a.el[0] + (size_t)b * (a.N + 1) * 3 * nn(a);
        wg_zero(e0, n, 2 * n, n);
        wg_gemm(e0 + 2 * nn(a), n, a.Xi + (size_t)b * nn(a), n, false, a.Xi + (size_t)b * nn(a), n, true, n, n, n,
                1.f, nullptr, 0, nullptr, 0, 0.f, lds);
    }
}

// One Kalman step (eq. kalman_recursions, C = I) in the calling workgroup:
// X = Pi A^T, [Rv + Pi | X] -> Y = (Rv + Pi)^{-1} X, L = -Y,
// Pi' = Qw + A X - X^T Y.  `X` is n x n of the workgroup's slot, G the
// solve matrix (n x 2n).
__device__ __forceinline__ bool kalman_step(const Args& a, const float* A, const float* Qw, const float* Rv,
                                            const float* Pi, float* L, float* Pn, float* X, float* G, float* lds) {
    const int n = a.n;
    wg_gemm(X, n, Pi, n, false, A, n, true, n, n, n, 1.f, nullptr, 0, nullptr, 0, 0.f, lds);
    wg_map(
        n * n, [&](int x) { return Rv[x] + Pi[x]; },
        [&](int x, float v) {
            const int r = x / n, c = x - r * n;
            G[(size_t)r * 2 * n + c] = v;
        });
    wg_map(
        n * n, [&](int x) { return X[x]; },
        [&](int x, float v) {
            const int r = x / n, c = x - r * n;
            G[(size_t)r * 2 * n + n + c] = v;
        });
    __syncthreads();
    const bool ok = wg_solve(G, 2 * n, n, n, lds + kGemmLds - 2 * kThreads);
    if (L) wg_copy(L, n, G + n, 2 * n, n, n, -1.f, 0.f);
    if (Pn) {
        wg_gemm(Pn, n, A, n, false, X, n, false, n, n, n, 1.f, Qw, n, nullptr, 0, 0.f, lds);
        wg_gemm(Pn, n, X, n, true, G + n, 2 * n, false, n, n, n, -1.f, Pn, n, nullptr, 0, 0.f, lds);
    }
    return ok;
}

// One Kalman step in the form of the scan's elements, free of cancellation:
// with Dinv = (F F^T)^{-1}, W = (I + Dinv Pi)^{-1} A^T,
//   Pi' = E E^T + W^T (Pi A^T),   L = W - A^T.
// (Pi' = E E^T + A (Pi^{-1} + Dinv)^{-1} A^T adds a positive semidefinite
// term; the printed form A Pi A^T + A Pi L subtracts two nearly equal
// matrices when the measurements are accurate (F F^T << Pi), which FP32
// cannot resolve.  L = -(F F^T + Pi)^{-1} Pi A^T = W - A^T since
// (I + Dinv Pi)^{-1} = (F F^T + Pi)^{-1} F F^T.)
__device__ __forceinline__ bool kalman_step_stable(const Args& a, const float* A, const float* Qw, const float* Dinv,
                                                   const float* Pi, float* L, float* Pn, float* X, float* G,
                                                   float* lds) {
    const int n = a.n;
    wg_gemm(G, 2 * n, Dinv, n, false, Pi, n, false, n, n, n, 1.f, nullptr, 0, nullptr, 0, 1.f, lds);
    wg_map(
        n * n,
        [&](int x) {
            const int r = x / n, c = x - r * n;
            return A[(size_t)c * n + r];
        },
        [&](int x, float v) {
            const int r = x / n, c = x - r * n;
            G[(size_t)r * 2 * n + n + c] = v;
        });
    __syncthreads();
    const bool ok = wg_solve(G, 2 * n, n, n, lds + kGemmLds - 2 * kThreads);
    wg_map(
        n * n,
        [&](int x) {
            const int r = x / n, c = x - r * n;
            return G[(size_t)r * 2 * n + n + c] - A[(size_t)c * n + r];
        },
        [&](int x, float v) { L[x] = v; });
    wg_gemm(X, n, Pi, n, false, A, n, true, n, n, n, 1.f, nullptr, 0, nullptr, 0, 0.f, lds);
    wg_gemm(Pn, n, G + n, 2 * n, true, X, n, false, n, n, n, 1.f, Qw, n, nullptr, 0, 0.f, lds);
    return ok;
}

// grid (B): the recursion run serially over the horizon, one workgroup per
// instance (the scan's step elements give Dinv).
__global__ __launch_bounds__(kThreads) void kalman_serial_kernel(Args a) {
    extern __shared__ float lds[];
    const int b = blockIdx.x, n = a.n;
    float* slot = a.ws + (size_t)b * a.ws_stride;
    float* Pi = a.Pi + (size_t)b * (a.N + 1) * nn(a);
    const float* el = a.el[0] + (size_t)b * (a.N + 1) * 3 * nn(a);
    wg_gemm(Pi, n, a.Xi + (size_t)b * nn(a), n, false, a.Xi + (size_t)b * nn(a), n, true, n, n, n, 1.f, nullptr, 0,
            nullptr, 0, 0.f, lds);
    bool ok = true;
    with_g(a, lds, slot + nn(a), [&](float* G) {
        for (int j = 0; j < a.N; ++j) {
            const size_t o = ((size_t)b * a.N + j) * nn(a);
            const float* Dinv = el + (size_t)(j + 1) * 3 * nn(a) + nn(a);
            ok &= kalman_step_stable(a, a.A + o, a.Qw + o, Dinv, Pi + j * nn(a), a.L + o, Pi + (j + 1) * nn(a), slot,
                                     G, lds);
        }
    });
    flag(a, b, ok);
}

// grid (N, B): L_{j+1} from Pi_j for every step at once (after the scan).
__global__ __launch_bounds__(kThreads) void gains_kernel(Args a) {
    extern __shared__ float lds[];
    const int j = blockIdx.x, b = blockIdx.y;
    const size_t o = ((size_t)b * a.N + j) * nn(a);
    float* slot = a.ws + ((size_t)b * a.N + j) * a.ws_stride;
    const float* Pi = a.Pi + ((size_t)b * (a.N + 1) + j) * nn(a);
    with_g(a, lds, slot + nn(a), [&](float* G) {
        flag(a, b, kalman_step(a, a.A + o, nullptr, a.Rv + o, Pi, a.L + o, nullptr, slot, G, lds));
    });
}

// grid (N+1, B): one round of the inclusive Hillis-Steele scan with offset
// `off`, from el[src] to el[1 - src].  Element i < off is a finished prefix
// (copied); for off <= i < 2 off the left operand is a finished prefix, whose
// At and Dt are zero, so only P is formed; otherwise the full combination
// (eq. combination_rules) of a = e_{i-off} (applied first) and b = e_i:
//   [I + Dt_b P_a | At_b | Dt_b At_a^T] -> W1 | W2
//   At = At_a W1,  Dt = At_a W2 + Dt_a,  P = W1^T (P_a At_b) + P_b.
// On the last round P goes to Pi.
__global__ __launch_bounds__(kThreads) void scan_round_kernel(Args a, int src, int off, int last) {
    extern __shared__ float lds[];
    const int i = blockIdx.x, b = blockIdx.y, n = a.n;
    const size_t esz = 3 * nn(a);
    const float* S = a.el[src] + (size_t)b * (a.N + 1) * esz;
    float* D = a.el[1 - src] + (size_t)b * (a.N + 1) * esz;
    float* Pout = last ? a.Pi + ((size_t)b * (a.N + 1) + i) * nn(a) : D + i * esz + 2 * nn(a);
    if (i < off) {
        wg_copy(Pout, n, S + i * esz + 2 * nn(a), n, n, n, 1.f, 0.f);
        return;
    }
    const float* Aa = S + (i - off) * esz;
    const float* Da = Aa + nn(a);
    const float* Pa = Aa + 2 * nn(a);
    const float* Ab = S + i * esz;
    const float* Db = Ab + nn(a);
    const float* Pb = Ab + 2 * nn(a);
    float* slot = a.ws + ((size_t)b * (a.N + 1) + i) * a.ws_stride;
    float* T2 = slot;
    const bool full = i >= 2 * off;
    const int m = full ? 2 * n : n;
    const int ld = n + m;
    with_g(a, lds, slot + nn(a), [&](float* G) {
        wg_gemm(G, ld, Db, n, false, Pa, n, false, n, n, n, 1.f, nullptr, 0, nullptr, 0, 1.f, lds);
        wg_copy(G + n, ld, Ab, n, n, n, 1.f, 0.f);
        if (full) wg_gemm(G + 2 * n, ld, Db, n, false, Aa, n, true, n, n, n, 1.f, nullptr, 0, nullptr, 0, 0.f, lds);
        flag(a, b, wg_solve(G, ld, n, m, lds + kGemmLds - 2 * kThreads));
        wg_gemm(T2, n, Pa, n, false, Ab, n, false, n, n, n, 1.f, nullptr, 0, nullptr, 0, 0.f, lds);
        wg_gemm(Pout, n, G + n, ld, true, T2, n, false, n, n, n, 1.f, Pb, n, nullptr, 0, 0.f, lds);
        if (full && !last) {
            float* Ao = D + i * esz;
            wg_gemm(Ao, n, Aa, n, false, G + n, ld, false, n, n, n, 1.f, nullptr, 0, nullptr, 0, 0.f, lds);
            wg_gemm(Ao + nn(a), n, Aa, n, false, G + 2 * n, ld, false, n, n, n, 1.f, Da, n, nullptr, 0, 0.f, lds);
        }
    });
}

// ---------------------------------------------------------------- transitions
struct TArgs {
    int B, N, n, r2;           // r2: rows (right mode) or rows of the left factor (left mode)
    const float* A;            // (B, N, n, n)
    const float* X;            // L (B, N, n, n) for the observer, K (B, N+1, m, n) for state feedback
    const float* Bm;           // (B, N, n, m) for state feedback, else null
    float* Ahat;               // (B, N, n, n) workspace
    float* T;                  // (B, D, D), D = (N+1) n: the transition products
    float* Y;                  // second product, dense (B, (N+1) r2, D) or (B, D, (N+1) n)
    int left;                  // 0: Y_{k,j} = T_{k,j} X_{j-1}^T (observer), 1: Y_{k,j} = K_k T_{k,j}
    int m;                     // input size (state feedback)
};

// grid (N, B): Ahat_j = A_j + L_{j+1}^T (observer, C = I) or A_j + B_j K_j.
__global__ __launch_bounds__(kThreads) void ahat_kernel(TArgs t) {
    extern __shared__ float lds[];
    const int j = blockIdx.x, b = blockIdx.y, n = t.n;
    const size_t o = ((size_t)b * t.N + j) * n * n;
    if (!t.left) {
        wg_map(
            n * n,
            [&](int e) {
                const int r = e / n, c = e - r * n;
                return t.A[o + e] + t.X[o + (size_t)c * n + r];
            },
            [&](int e, float v) { t.Ahat[o + e] = v; });
    } else {
        const float* K = t.X + ((size_t)b * (t.N + 1) + j) * t.m * n;
        wg_gemm(t.Ahat + o, n, t.Bm + ((size_t)b * t.N + j) * n * t.m, t.m, false, K, n, false, n, n, t.m, 1.f,
                t.A + o, n, nullptr, 0, 0.f, lds);
    }
}

__device__ __forceinline__ size_t tdim(const TArgs& t) { return (size_t)(t.N + 1) * t.n; }

// the second product of block (k, j) of T, once T_{k,j} is written
__device__ void second_product(const TArgs& t, int b, int k, int j, float* lds) {
    const int n = t.n;
    const size_t D = tdim(t);
    const float* Tk = t.T + (size_t)b * D * D + (size_t)k * n * D + (size_t)j * n;
    if (!t.left) {
        float* Yk = t.Y + (size_t)b * D * D + (size_t)k * n * D + (size_t)j * n;
        if (j == 0) wg_zero(Yk, (int)D, n, n);
        else
            wg_gemm(Yk, (int)D, Tk, (int)D, false, t.X + ((size_t)b * t.N + j - 1) * n * n, n, true, n, n, n, 1.f,
                    nullptr, 0, nullptr, 0, 0.f, lds);
    } else {
        const int m = t.m;
        float* Yk = t.Y + (size_t)b * (t.N + 1) * m * D + (size_t)k * m * D + (size_t)j * n;
        wg_gemm(Yk, (int)D, t.X + ((size_t)b * (t.N + 1) + k) * m * n, n, false, Tk, (int)D, false, m, n, n, 1.f,
                nullptr, 0, nullptr, 0, 0.f, lds);
    }
}

// grid (N+1, B): block row k of T: zeros right of the diagonal, T_{k,k} = I,
// T_{k,k-1} = Ahat_{k-1}; the second products of those blocks, and zeros in
// the second operator right of the diagonal.
__global__ __launch_bounds__(kThreads) void trans_init_kernel(TArgs t) {
    extern __shared__ float lds[];
    const int k = blockIdx.x, b = blockIdx.y, n = t.n;
    const size_t D = tdim(t);
    float* row = t.T + (size_t)b * D * D + (size_t)k * n * D;
    const int c0 = (k + 1) * n;
    if ((size_t)c0 < D) wg_zero(row + c0, (int)D, n, (int)(D - c0));
    wg_ident(row + (size_t)k * n, (int)D, n);
    if (k >= 1) wg_copy(row + (size_t)(k - 1) * n, (int)D, t.Ahat + ((size_t)b * t.N + k - 1) * n * n, n, n, n, 1.f, 0.f);
    const int rr = t.left ? t.m : n;
    float* yrow = t.Y + (size_t)b * (t.N + 1) * rr * D + (size_t)k * rr * D;
    if ((size_t)c0 < D) wg_zero(yrow + c0, (int)D, rr, (int)(D - c0));
    second_product(t, b, k, k, lds);
    if (k >= 1) second_product(t, b, k, k - 1, lds);
}

// grid (N+1, ndiag, B): T_{j+d, j} = T_{j+d, j+e} T_{j+e, j} for d = d0 + blockIdx.y,
// e = d - split (split = d0 for the first launch of a doubling round, whose
// only diagonal is d0 = 2^r with e = 2^{r-1}).
__global__ __launch_bounds__(kThreads) void trans_round_kernel(TArgs t, int d0, int split) {
    extern __shared__ float lds[];
    const int j = blockIdx.x, d = d0 + blockIdx.y, b = blockIdx.z, n = t.n;
    if (j + d > t.N) return;
    const int e = d - split;
    const size_t D = tdim(t);
    float* Tb = t.T + (size_t)b * D * D;
    const int k = j + d, mid = j + e;
    wg_gemm(Tb + (size_t)k * n * D + (size_t)j * n, (int)D, Tb + (size_t)k * n * D + (size_t)mid * n, (int)D, false,
            Tb + (size_t)mid * n * D + (size_t)j * n, (int)D, false, n, n, n, 1.f, nullptr, 0, nullptr, 0, 0.f, lds);
    second_product(t, b, k, j, lds);
}

// ---------------------------------------------------------------- assembly
// grid (N+1, column tiles of 64, B): block row i of M X = X - Z A X,
// (M X)_i = X_i - A_{i-1} X_{i-1}, for the dense block-lower X ((N+1) n x cols).
__global__ __launch_bounds__(kThreads) void shift_kernel(int N, int n, int cols, const float* A, const float* X,
                                                         float* out) {
    extern __shared__ float lds[];
    const int i = blockIdx.x, c0 = blockIdx.y * kTile, b = blockIdx.z;
    const size_t D = (size_t)(N + 1) * n;
    const int cw = std::min(kTile, cols - c0);
    const float* Xb = X + (size_t)b * D * cols;
    float* Ob = out + (size_t)b * D * cols + (size_t)i * n * cols + c0;
    if (i == 0) {
        wg_copy(Ob, cols, Xb + c0, cols, n, cw, 1.f, 0.f);
        return;
    }
    // columns beyond the diagonal block of row i are zero in both terms
    const int w = std::min<int>(cols, (i + 1) * n) - c0;
    if (w <= 0) {
        wg_zero(Ob, cols, n, cw);
        return;
    }
    const int ww = std::min(w, cw);
    wg_gemm(Ob, cols, A + ((size_t)b * N + i - 1) * n * n, n, false, Xb + (size_t)(i - 1) * n * cols + c0, cols,
            false, n, ww, n, -1.f, Xb + (size_t)i * n * cols + c0, cols, nullptr, 0, 0.f, lds);
    if (ww < cw) wg_zero(Ob + ww, cols, n, cw - ww);
}

// One output tile per workgroup of C = alpha A B + add1 + add2 with A
// (rows x K) block-lower in blocks of ra rows by n columns and B (K x cols)
// block-lower in n x n blocks: A[r][k] = 0 beyond block k/n > r/ra, B[k][c] =
// 0 for k/n < c/n.  grid (tiles_c, tiles_r, batch).
__global__ __launch_bounds__(kThreads) void tri_gemm_kernel(int rows, int cols, int K, int ra, int n, float alpha,
                                                            const float* A, const float* Bm, const float* add1,
                                                            const float* add2, float* C) {
    extern __shared__ float lds[];
    const int tn = blockIdx.x * kTile, tm = blockIdx.y * kTile, b = blockIdx.z;
    const size_t sa = (size_t)rows * K, sb = (size_t)K * cols, sc = (size_t)rows * cols;
    const int r1 = std::min(rows, tm + kTile);
    const int k0 = (tn / n) * n;
    const int k1 = std::min(K, ((r1 - 1) / ra + 1) * n);
    const int M = r1 - tm, N = std::min(cols, tn + kTile) - tn;
    float* Cb = C + b * sc + (size_t)tm * cols + tn;
    const float* a1 = add1 ? add1 + b * sc + (size_t)tm * cols + tn : nullptr;
    const float* a2 = add2 ? add2 + b * sc + (size_t)tm * cols + tn : nullptr;
    if (k1 <= k0) {
        for (int e = threadIdx.x; e < M * N; e += kThreads) {
            const int r = e / N, c = e - r * N;
            float x = 0.f;
            if (a1) x += a1[(size_t)r * cols + c];
            if (a2) x += a2[(size_t)r * cols + c];
            Cb[(size_t)r * cols + c] = x;
        }
        return;
    }
    wg_gemm(Cb, cols, A + b * sa + (size_t)tm * K + k0, K, false, Bm + b * sb + (size_t)k0 * cols + tn, cols, false, M,
            N, k1 - k0, alpha, a1, cols, a2, cols, 0.f, lds);
}

// The same product with 128 x 128 output tiles for the large assembly
// operators: each wavefront a 64 x 64 quarter (4 x 4 blocks of
// v_mfma_f32_16x16x4f32, 64 accumulators), K in chunks of 16 staged through
// two LDS buffers (the next chunk is loaded into registers while the
// current one is multiplied), rows read as float2 (every row and tile
// offset is even).  grid (tiles_c, tiles_r, batch).
constexpr int kBT = 128, kBK = 16;
constexpr int kBPadA = kBK + 1, kBPadB = kBT + 1;
constexpr int kBBuf = kBT * kBPadA + kBK * kBPadB;
constexpr int kBigLds = 2 * kBBuf;

__global__ __launch_bounds__(kThreads) void tri_gemm128_kernel(int rows, int cols, int K, int ra, int n, float alpha,
                                                               const float* A, const float* Bm, const float* add1,
                                                               const float* add2, float* C) {
    extern __shared__ float lds[];
    const int tn = blockIdx.x * kBT, tm = blockIdx.y * kBT, b = blockIdx.z;
    const size_t sa = (size_t)rows * K, sb = (size_t)K * cols, sc = (size_t)rows * cols;
    const int r1 = min(rows, tm + kBT);
    const int c1 = min(cols, tn + kBT);
    const int k0 = (tn / n) * n;
    const int k1 = min(K, ((r1 - 1) / ra + 1) * n);
    const float* Ab = A + b * sa;
    const float* Bb = Bm + b * sb;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = (w & 1) * 64, wn = (w >> 1) * 64;
    const int l16 = lane & 15, lk = lane >> 4;
    f4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    // per thread: A rows ar, k columns ac..ac+7; B row br, columns bc..bc+7
    const int ar = tid >> 1, ac = (tid & 1) * 8;
    const int br = tid >> 4, bc = (tid & 15) * 8;
    float ra_[8], rb_[8];
    // A chunk that ends inside [k0, k1) needs no column test, and a thread
    // whose A row and B columns are inside the tile needs no row or column
    // test: those loads are unconditional (one branch per chunk); the last
    // chunk and the edge threads take the element-wise tests.
    const bool a_in = tm + ar < r1, b_in = tn + bc + 8 <= c1;
    auto load = [&](int kc) {
        const int gr = tm + ar;
        const int gkb = kc + br;
        if (kc + kBK <= k1 && a_in && b_in) {
            const float* pa = Ab + (size_t)gr * K + kc + ac;
            const float* pb = Bb + (size_t)gkb * cols + tn + bc;
#pragma unroll
            for (int q = 0; q < 8; q += 2) {
                const float2 va = *reinterpret_cast<const float2*>(pa + q);
                const float2 vb = *reinterpret_cast<const float2*>(pb + q);
                ra_[q] = va.x;
                ra_[q + 1] = va.y;
                rb_[q] = vb.x;
                rb_[q + 1] = vb.y;
            }
            return;
        }
#pragma unroll
        for (int q = 0; q < 8; q += 2) {
            const int gk = kc + ac + q;
            float2 v = make_float2(0.f, 0.f);
            if (gr < r1 && gk + 1 < k1) v = *reinterpret_cast<const float2*>(Ab + (size_t)gr * K + gk);
            else if (gr < r1 && gk < k1) v.x = Ab[(size_t)gr * K + gk];
            ra_[q] = v.x;
            ra_[q + 1] = v.y;
        }
#pragma unroll
        for (int q = 0; q < 8; q += 2) {
            const int gc = tn + bc + q;
            float2 v = make_float2(0.f, 0.f);
            if (gkb < k1 && gc + 1 < c1) v = *reinterpret_cast<const float2*>(Bb + (size_t)gkb * cols + gc);
            else if (gkb < k1 && gc < c1) v.x = Bb[(size_t)gkb * cols + gc];
            rb_[q] = v.x;
            rb_[q + 1] = v.y;
        }
    };
    auto store = [&](int buf) {
        float* As = lds + buf * kBBuf;
        float* Bs = As + kBT * kBPadA;
#pragma unroll
        for (int q = 0; q < 8; ++q) As[ar * kBPadA + ac + q] = ra_[q];
#pragma unroll
        for (int q = 0; q < 8; ++q) Bs[br * kBPadB + bc + q] = rb_[q];
    };
    if (k1 > k0) {
        load(k0);
        store(0);
        __syncthreads();
        int buf = 0;
        for (int kc = k0; kc < k1; kc += kBK) {
            const bool more = kc + kBK < k1;
            if (more) load(kc + kBK);
            const float* As = lds + buf * kBBuf;
            const float* Bs = As + kBT * kBPadA;
#pragma unroll
            for (int kk = 0; kk < kBK; kk += 4) {
                const int kr = kk + lk;
                float a[4], bv[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) a[i] = As[(wm + 16 * i + l16) * kBPadA + kr];
#pragma unroll
                for (int j = 0; j < 4; ++j) bv[j] = Bs[kr * kBPadB + wn + 16 * j + l16];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], bv[j], acc[i][j], 0, 0, 0);
            }
            if (more) store(buf ^ 1);
            __syncthreads();
            buf ^= 1;
        }
    }
    float* Cb = C + b * sc;
    const float* a1 = add1 ? add1 + b * sc : nullptr;
    const float* a2 = add2 ? add2 + b * sc : nullptr;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = tm + wm + 16 * i + 4 * lk + v;
                const int c = tn + wn + 16 * j + l16;
                if (r < r1 && c < c1) {
                    float x = alpha * acc[i][j][v];
                    if (a1) x += a1[(size_t)r * cols + c];
                    if (a2) x += a2[(size_t)r * cols + c];
                    Cb[(size_t)r * cols + c] = x;
                }
            }
}

// ---------------------------------------------------------------- tubes
// grid (N, N+1, B), workgroup (j, k) with j < k: the row norms of
// Pw_{k,j+1} E_j and of Pe_{k,j+1} F_j for the dense Pw, Pe ((N+1) rr x D),
// their sum per row to part[b][k][j][:].  The products go through LDS in
// 64 x 64 pieces; a thread owns one row of a 64-row piece and accumulates
// its squares over the column pieces.
__global__ __launch_bounds__(kThreads) void tube_part_kernel(int N, int n, int rr, const float* Pw, const float* Pe,
                                                             const float* E, const float* F, float* part) {
    extern __shared__ float lds[];
    const int j = blockIdx.x, k = blockIdx.y, b = blockIdx.z;
    if (j >= k) return;
    const size_t D = (size_t)(N + 1) * n;
    float* Pt = lds + kGemmLds;
    float* out = part + (((size_t)b * (N + 1) + k) * N + j) * rr;
    const int tid = threadIdx.x;
    for (int r0 = 0; r0 < rr; r0 += kTile) {
        const int rows = std::min(kTile, rr - r0);
        float norm = 0.f;
        for (int s = 0; s < 2; ++s) {
            const float* Ph = (s ? Pe : Pw) + (size_t)b * (N + 1) * rr * D + ((size_t)k * rr + r0) * D +
                              (size_t)(j + 1) * n;
            const float* S = (s ? F : E) + ((size_t)b * N + j) * n * n;
            float sq = 0.f;
            for (int c0 = 0; c0 < n; c0 += kTile) {
                const int cols = std::min(kTile, n - c0);
                wg_gemm(Pt, kTile, Ph, (int)D, false, S + c0, n, false, rows, cols, n, 1.f, nullptr, 0, nullptr, 0,
                        0.f, lds);
                if (tid < rows)
                    for (int c = 0; c < cols; ++c) sq += Pt[tid * kTile + c] * Pt[tid * kTile + c];
                __syncthreads();
            }
            norm += sqrtf(sq);
        }
        if (tid < rows) out[r0 + tid] = norm;
    }
}

// grid (N+1, B): tau[b][k][r] = sum_{j<k} part[b][k][j][r], in increasing j.
__global__ __launch_bounds__(kThreads) void tube_sum_kernel(int N, int rr, const float* part, float* tau) {
    const int k = blockIdx.x, b = blockIdx.y;
    const float* p = part + ((size_t)b * (N + 1) + k) * N * rr;
    for (int r = threadIdx.x; r < rr; r += kThreads) {
        float acc = 0.f;
        for (int j = 0; j < k; ++j) acc += p[(size_t)j * rr + r];
        tau[((size_t)b * (N + 1) + k) * rr + r] = acc;
    }
}

}  // namespace sls
}  // namespace cord

// ================================================================ C ABI
using namespace cord::sls;

struct cord_sls {
    int B, N, n, m;
    int device;
    float* Qw = nullptr;
    float* Rv = nullptr;
    float* el[2] = {nullptr, nullptr};
    float* ws = nullptr;
    size_t ws_stride = 0;
    size_t ws_slots = 0;
    float* Ahat = nullptr;
    float* MX = nullptr;       // M Phihat^x
    float* MY = nullptr;       // M Phihat^y
    float* tube_part = nullptr; // (B, N+1, N, max(n, m)) row norms per (k, j)
};

namespace {

int sls_fail(int code, const char* msg) { return cord::set_error(code, msg); }

#define SLS_HIP(call)                                                                  \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            char b_[256];                                                              \
            snprintf(b_, sizeof(b_), "%s: %s", #call, hipGetErrorString(e_));          \
            return cord::set_error(CORD_EHIP, b_);                                     \
        }                                                                              \
    } while (0)

size_t solve_floats(int n, int m) { return (size_t)n * (n + m); }
bool solve_in_lds(int n, int m) { return sizeof(float) * (kGemmLds + solve_floats(n, m)) <= kMaxLdsBytes; }
size_t lds_bytes(int n, int m, bool in_lds) {
    return sizeof(float) * (kGemmLds + (in_lds ? solve_floats(n, m) : 0));
}

Args base_args(cord_sls* s, bool in_lds) {
    Args a{};
    a.B = s->B;
    a.N = s->N;
    a.n = s->n;
    a.m = s->m;
    a.Qw = s->Qw;
    a.Rv = s->Rv;
    a.el[0] = s->el[0];
    a.el[1] = s->el[1];
    a.ws = s->ws;
    a.ws_stride = s->ws_stride;
    a.g_in_lds = in_lds ? 1 : 0;
    return a;
}

}  // namespace

extern "C" {

int cord_sls_create(int32_t batch, int32_t horizon, int32_t n, int32_t n_u, cord_sls** out) {
    if (!out || batch < 1 || horizon < 1 || n < 1 || n_u < 0) return sls_fail(CORD_EINVAL, "cord_sls_create: bad arguments");
    if (n > 1024) return sls_fail(CORD_EUNSUPPORTED, "cord_sls_create: state size above 1024");
    const size_t D = (size_t)(horizon + 1) * n;
    if ((double)batch * D * D * 4.0 > 64.0 * (1ull << 30))
        return sls_fail(CORD_ETOOBIG, "cord_sls_create: one horizon operator exceeds 64 GiB");
    cord_sls* s = new (std::nothrow) cord_sls();
    if (!s) return sls_fail(CORD_ENOMEM, "host allocation");
    s->B = batch;
    s->N = horizon;
    s->n = n;
    s->m = n_u;
    (void)hipGetDevice(&s->device);
    const size_t nn = (size_t)n * n;
    const size_t steps = (size_t)batch * horizon;
    const size_t elems = (size_t)batch * (horizon + 1);
    // a slot holds X / T2 (n^2) and the solve matrix when it is not in LDS (3 n^2)
    s->ws_stride = (nn + (solve_in_lds(n, 2 * n) ? 0 : 3 * nn) + 63) / 64 * 64;
    s->ws_slots = elems;
    bool ok = hipMalloc(&s->Qw, 4 * steps * nn) == hipSuccess && hipMalloc(&s->Rv, 4 * steps * nn) == hipSuccess &&
              hipMalloc(&s->el[0], 4 * elems * 3 * nn) == hipSuccess &&
              hipMalloc(&s->el[1], 4 * elems * 3 * nn) == hipSuccess &&
              hipMalloc(&s->ws, 4 * s->ws_slots * s->ws_stride) == hipSuccess &&
              hipMalloc(&s->Ahat, 4 * steps * nn) == hipSuccess &&
              hipMalloc(&s->MX, 4 * (size_t)batch * D * D) == hipSuccess &&
              hipMalloc(&s->MY, 4 * (size_t)batch * D * D) == hipSuccess &&
              hipMalloc(&s->tube_part, 4 * elems * horizon * (size_t)std::max(n, n_u)) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        cord_sls_destroy(s);
        return sls_fail(CORD_ENOMEM, "cord_sls_create: device workspace");
    }
    *out = s;
    return CORD_OK;
}

int cord_sls_destroy(cord_sls* s) {
    if (!s) return CORD_OK;
    for (float* p : {s->Qw, s->Rv, s->el[0], s->el[1], s->ws, s->Ahat, s->MX, s->MY, s->tube_part})
        if (p) (void)hipFree(p);
    delete s;
    return CORD_OK;
}

int cord_sls_kalman(cord_sls* s, const float* A, const float* E, const float* F, const float* Xi, int32_t mode,
                    float* Pi, float* L, int32_t* status, void* stream) {
    if (!s || !A || !E || !F || !Xi || !Pi || !L || !status || (mode != CORD_SLS_SERIAL && mode != CORD_SLS_SCAN))
        return sls_fail(CORD_EINVAL, "cord_sls_kalman: bad arguments");
    hipStream_t st = (hipStream_t)stream;
    const bool scan = mode == CORD_SLS_SCAN;
    const int n = s->n;
    // the widest solve: [M | R] with m = 2n in the scan, m = n otherwise
    const bool in_lds = solve_in_lds(n, scan ? 2 * n : n);
    const size_t lb = lds_bytes(n, scan ? 2 * n : n, in_lds);
    Args a = base_args(s, in_lds);
    a.A = A;
    a.E = E;
    a.F = F;
    a.Xi = Xi;
    a.Pi = Pi;
    a.L = L;
    a.status = status;
    SLS_HIP(cord::launch_fill_i32(status, s->B, CORD_ST_OK, st));
    // both modes use the step elements (the serial step takes Dinv from them)
    hipLaunchKernelGGL(prep_kernel, dim3(s->N, s->B), dim3(kThreads), lb, st, a, 1);
    SLS_HIP(hipGetLastError());
    if (!scan) {
        hipLaunchKernelGGL(kalman_serial_kernel, dim3(s->B), dim3(kThreads), lb, st, a);
        SLS_HIP(hipGetLastError());
        return CORD_OK;
    }
    int src = 0;
    for (int off = 1; off < s->N + 1; off *= 2) {
        const int last = 2 * off >= s->N + 1;
        hipLaunchKernelGGL(scan_round_kernel, dim3(s->N + 1, s->B), dim3(kThreads), lb, st, a, src, off, last);
        SLS_HIP(hipGetLastError());
        src = 1 - src;
    }
    hipLaunchKernelGGL(gains_kernel, dim3(s->N, s->B), dim3(kThreads), lb, st, a);
    SLS_HIP(hipGetLastError());
    return CORD_OK;
}

static int run_transitions(cord_sls* s, TArgs& t, hipStream_t st) {
    const size_t lb = sizeof(float) * kGemmLds;
    hipLaunchKernelGGL(ahat_kernel, dim3(s->N, s->B), dim3(kThreads), lb, st, t);
    SLS_HIP(hipGetLastError());
    hipLaunchKernelGGL(trans_init_kernel, dim3(s->N + 1, s->B), dim3(kThreads), lb, st, t);
    SLS_HIP(hipGetLastError());
    // diagonals 2^r from two of 2^{r-1}, then 2^r + e from 2^r and e < 2^r
    for (int p = 1; p <= s->N; p *= 2) {
        if (p >= 2) {
            hipLaunchKernelGGL(trans_round_kernel, dim3(s->N + 1, 1, s->B), dim3(kThreads), lb, st, t, p, p / 2);
            SLS_HIP(hipGetLastError());
        }
        const int d0 = p + 1, d1 = std::min(2 * p - 1, s->N);
        if (d0 <= d1) {
            hipLaunchKernelGGL(trans_round_kernel, dim3(s->N + 1, d1 - d0 + 1, s->B), dim3(kThreads), lb, st, t, d0,
                               p);
            SLS_HIP(hipGetLastError());
        }
    }
    return CORD_OK;
}

int cord_sls_observer(cord_sls* s, const float* A, const float* L, float* Phx, float* Phy, void* stream) {
    if (!s || !A || !L || !Phx || !Phy) return sls_fail(CORD_EINVAL, "cord_sls_observer: bad arguments");
    TArgs t{};
    t.B = s->B;
    t.N = s->N;
    t.n = s->n;
    t.A = A;
    t.X = L;
    t.Ahat = s->Ahat;
    t.T = Phx;
    t.Y = Phy;
    t.left = 0;
    return run_transitions(s, t, (hipStream_t)stream);
}

int cord_sls_state_feedback(cord_sls* s, const float* A, const float* Bm, const float* K, float* Pbx, float* Pbu,
                            void* stream) {
    if (!s || !A || !Bm || !K || !Pbx || !Pbu || s->m < 1)
        return sls_fail(CORD_EINVAL, "cord_sls_state_feedback: bad arguments");
    TArgs t{};
    t.B = s->B;
    t.N = s->N;
    t.n = s->n;
    t.A = A;
    t.X = K;
    t.Bm = Bm;
    t.Ahat = s->Ahat;
    t.T = Pbx;
    t.Y = Pbu;
    t.left = 1;
    t.m = s->m;
    return run_transitions(s, t, (hipStream_t)stream);
}

int cord_sls_assemble(cord_sls* s, const float* A, const float* Pbx, const float* Pbu, const float* Phx,
                      const float* Phy, float* Pxw, float* Puw, float* Pxe, float* Pue, void* stream) {
    if (!s || !A || !Pbx || !Pbu || !Phx || !Phy || !Pxw || !Puw || !Pxe || !Pue || s->m < 1)
        return sls_fail(CORD_EINVAL, "cord_sls_assemble: bad arguments");
    hipStream_t st = (hipStream_t)stream;
    const int n = s->n, m = s->m;
    const int D = (s->N + 1) * n, Du = (s->N + 1) * m;
    const size_t lb = sizeof(float) * kGemmLds;
    const dim3 gs(s->N + 1, (D + kTile - 1) / kTile, s->B);
    hipLaunchKernelGGL(shift_kernel, gs, dim3(kThreads), lb, st, s->N, n, D, A, Phx, s->MX);
    SLS_HIP(hipGetLastError());
    hipLaunchKernelGGL(shift_kernel, gs, dim3(kThreads), lb, st, s->N, n, D, A, Phy, s->MY);
    SLS_HIP(hipGetLastError());
    // even row lengths and block offsets let the big-tile kernel read float2;
    // otherwise the 64 x 64 kernel
    const bool big = (D % 2 == 0) && (n % 2 == 0);
    const int T = big ? kBT : kTile;
    const size_t lbig = big ? sizeof(float) * kBigLds : lb;
    auto tri = big ? tri_gemm128_kernel : tri_gemm_kernel;
    const dim3 gx((D + T - 1) / T, (D + T - 1) / T, s->B);
    const dim3 gu((D + T - 1) / T, (Du + T - 1) / T, s->B);
    // Phi^xw = Phibar^x + Phihat^x - Phibar^x M Phihat^x
    hipLaunchKernelGGL(tri, gx, dim3(kThreads), lbig, st, D, D, D, n, n, -1.f, Pbx, s->MX, Pbx, Phx, Pxw);
    SLS_HIP(hipGetLastError());
    // Phi^uw = Phibar^u - Phibar^u M Phihat^x
    hipLaunchKernelGGL(tri, gu, dim3(kThreads), lbig, st, Du, D, D, m, n, -1.f, Pbu, s->MX, Pbu,
                       (const float*)nullptr, Puw);
    SLS_HIP(hipGetLastError());
    // Phi^xe = Phihat^y - Phibar^x M Phihat^y
    hipLaunchKernelGGL(tri, gx, dim3(kThreads), lbig, st, D, D, D, n, n, -1.f, Pbx, s->MY, Phy,
                       (const float*)nullptr, Pxe);
    SLS_HIP(hipGetLastError());
    // Phi^ue = -Phibar^u M Phihat^y
    hipLaunchKernelGGL(tri, gu, dim3(kThreads), lbig, st, Du, D, D, m, n, -1.f, Pbu, s->MY,
                       (const float*)nullptr, (const float*)nullptr, Pue);
    SLS_HIP(hipGetLastError());
    return CORD_OK;
}

int cord_sls_tubes(cord_sls* s, const float* Pxw, const float* Pxe, const float* Puw, const float* Pue, const float* E,
                   const float* F, float* tau_x, float* tau_u, void* stream) {
    if (!s || !Pxw || !Pxe || !E || !F || !tau_x || ((Puw || Pue || tau_u) && !(Puw && Pue && tau_u && s->m >= 1)))
        return sls_fail(CORD_EINVAL, "cord_sls_tubes: bad arguments");
    hipStream_t st = (hipStream_t)stream;
    const size_t lb = sizeof(float) * (kGemmLds + kTile * kTile);
    for (int pass = 0; pass < (tau_u ? 2 : 1); ++pass) {
        const int rr = pass ? s->m : s->n;
        const float* Pw = pass ? Puw : Pxw;
        const float* Pe = pass ? Pue : Pxe;
        hipLaunchKernelGGL(tube_part_kernel, dim3(s->N, s->N + 1, s->B), dim3(kThreads), lb, st, s->N, s->n, rr, Pw,
                           Pe, E, F, s->tube_part);
        SLS_HIP(hipGetLastError());
        hipLaunchKernelGGL(tube_sum_kernel, dim3(s->N + 1, s->B), dim3(kThreads), 0, st, s->N, rr, s->tube_part,
                           pass ? tau_u : tau_x);
        SLS_HIP(hipGetLastError());
    }
    return CORD_OK;
}

}  // extern "C"

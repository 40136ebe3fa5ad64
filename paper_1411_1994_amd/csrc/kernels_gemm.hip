// MFMA contraction kernels (gfx950): the dense steps of the RHOSVD and Tucker evaluation.
//
//  * k_gemm: strided GEMM C = alpha A B + beta C on v_mfma_f64_16x16x4 (FP64),
//    v_mfma_f32_16x16x4 (FP32) or split-BF16x3 on v_mfma_f32_16x16x32_bf16 (x = hi + lo,
//    hi*hi + hi*lo + lo*hi).  The FP32 and BF16x3 variants accumulate in FP32 inside each
//    k-tile (16 or 32 terms) and add the tile's partial sums into FP64 registers, so the
//    accumulation error stays near 2^-24 sqrt(16) instead of growing like 2^-24 sqrt(K).  Used for the side-matrix column Grams,
//    the projections Z^T A (Appendix theorem (c)) and the mode products of eq.
//    Tucker_singePot.
//  * k_core: the RHOSVD core mu = sum_nu xi_nu y1_nu (x) y2_nu (x) y3_nu (eq. C-core) as a GEMM
//    whose left operand, the Khatri-Rao product of the mode-1 and mode-2 projections, is formed
//    on the fly from LDS so it never touches HBM.
//  * k_cp_norm2: ||A||_F^2 of the canonical sum from the column Grams (used by the truncation
//    rule).
//
// MFMA operand layout (16x16xK, wave64): lane l supplies A[row l%16][k-group l/16] and
// B[k-group l/16][col l%16]; the 16x16 result sits in lane l, register v at column l%16 and
// row 4*(l/16)+v for the FP32-output instructions but row l/16+4*v for the FP64 one.
// Tiles: 64x64 per workgroup (4 waves in 2x2, each 32x32 = 2x2 MFMA blocks).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lsum_internal.h"

namespace lsum {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

template <int P> struct GT;
template <> struct GT<GEMM_F64> { using T = double; using Acc = d4; static constexpr int BK = 16; };
template <> struct GT<GEMM_F32> { using T = float; using Acc = f4; static constexpr int BK = 16; };
template <> struct GT<GEMM_BF16X3> { using T = float; using Acc = f4; static constexpr int BK = 32; };

constexpr int BM = 64, BN = 64;

// row of the 16x16 MFMA result held by lane `lane`, accumulator register v
template <int P>
__device__ __forceinline__ int acc_row(int lane, int v) {
    if constexpr (P == GEMM_F64) return (lane >> 4) + 4 * v;
    else return 4 * (lane >> 4) + v;
}

// FP64 partial sums of the FP32-accumulating variants
struct Acc64 {
    double v[2][2][4];
};

template <int P>
__device__ __forceinline__ void flush(typename GT<P>::Acc (&acc)[2][2], Acc64& a64) {
    if constexpr (P != GEMM_F64) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
#pragma unroll
                for (int v = 0; v < 4; ++v) a64.v[i][j][v] += (double)acc[i][j][v];
                acc[i][j] = typename GT<P>::Acc{0, 0, 0, 0};
            }
    }
}

template <int P>
__device__ __forceinline__ double result(const typename GT<P>::Acc (&acc)[2][2], const Acc64& a64, int i,
                                         int j, int v) {
    if constexpr (P == GEMM_F64) return acc[i][j][v];
    else return a64.v[i][j][v];
}

// One k-chunk of MFMAs over the LDS tiles As[k][m], Bs[k][n] for this wave's 32x32 block.
template <int P>
__device__ __forceinline__ void mfma_chunk(const typename GT<P>::T (*As)[BM + 1],
                                           const typename GT<P>::T (*Bs)[BN + 1], int wm, int wn,
                                           int lane, typename GT<P>::Acc (&acc)[2][2]) {
    constexpr int BK = GT<P>::BK;
    const int r = lane & 15, kg = lane >> 4;
    if constexpr (P == GEMM_F64) {
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            double a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[kk + kg][wm + i * 16 + r];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[kk + kg][wn + j * 16 + r];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    } else if constexpr (P == GEMM_F32) {
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            float a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[kk + kg][wm + i * 16 + r];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[kk + kg][wn + j * 16 + r];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    } else {
        bf8 ahi[2], alo[2], bhi[2], blo[2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float x = As[kg * 8 + e][wm + i * 16 + r];
                const __bf16 hx = (__bf16)x;
                ahi[i][e] = hx;
                alo[i][e] = (__bf16)(x - (float)hx);
            }
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float x = Bs[kg * 8 + e][wn + j * 16 + r];
                const __bf16 hx = (__bf16)x;
                bhi[j][e] = hx;
                blo[j][e] = (__bf16)(x - (float)hx);
            }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[i], bhi[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[i], blo[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[i], bhi[j], acc[i][j], 0, 0, 0);
            }
    }
}

template <int P>
__global__ void __launch_bounds__(256) k_gemm(GemmArgs g) {
    using T = typename GT<P>::T;
    using Acc = typename GT<P>::Acc;
    constexpr int BK = GT<P>::BK;
    __shared__ T As[BK][BM + 1];
    __shared__ T Bs[BK][BN + 1];
    const long bz = blockIdx.z;
    const T* __restrict__ A = (const T*)g.A + bz * g.bA;
    const T* __restrict__ B = (const T*)g.B + bz * g.bB;
    T* __restrict__ C = (T*)g.C + bz * g.bC;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    Acc acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = Acc{0, 0, 0, 0};
    Acc64 a64{};
    const bool a_kfast = (g.sak == 1);
    const bool b_nfast = (g.sbn == 1);
    for (int k0 = 0; k0 < g.k; k0 += BK) {
        for (int e = tid; e < BM * BK; e += 256) {
            int mm, kk;
            if (a_kfast) { kk = e % BK; mm = e / BK; } else { mm = e % BM; kk = e / BM; }
            const int gm = m0 + mm, gk = k0 + kk;
            As[kk][mm] = (gm < g.m && gk < g.k) ? A[(long)gm * g.sam + (long)gk * g.sak] : T(0);
        }
        for (int e = tid; e < BN * BK; e += 256) {
            int nn, kk;
            if (b_nfast) { nn = e % BN; kk = e / BN; } else { kk = e % BK; nn = e / BK; }
            const int gn = n0 + nn, gk = k0 + kk;
            Bs[kk][nn] = (gn < g.n && gk < g.k) ? B[(long)gk * g.sbk + (long)gn * g.sbn] : T(0);
        }
        __syncthreads();
        mfma_chunk<P>(As, Bs, wm, wn, lane, acc);
        flush<P>(acc, a64);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm + i * 16 + acc_row<P>(lane, v);
                const int col = n0 + wn + j * 16 + (lane & 15);
                if (row < g.m && col < g.n) {
                    T* c = C + (long)row * g.scm + (long)col * g.scn;
                    const double val = g.alpha * result<P>(acc, a64, i, j, v);
                    *c = (T)((g.beta != 0.0) ? val + g.beta * (double)*c : val);
                }
            }
}

// --------------------------------------------------------------------------------------------
// Core contraction (eq. C-core) as a GEMM with rows m = (a, b) and columns c, reduced over the
// canonical terms nu.  A workgroup owns a 128 x 64 tile: 8 values of a times 16 of b, and 64
// of c.  Per chunk of CK terms it stages rows of the term-major operands, forms the Khatri-Rao
// tile K[nu][(a,b)] = x1[a] x2[b] in LDS (so the r1*r2 x K operand never exists in HBM), and
// each wave multiplies its 32 rows by the 64 columns:
//   FP32:   v_mfma_f32_32x32x2f32, FP32 sums within the chunk, FP64 across chunks;
//   BF16X3: v_mfma_f32_32x32x16_bf16 on hi*hi + hi*lo + lo*hi of the split operands;
//   FP64:   v_mfma_f64_16x16x4f64 throughout.
// The next chunk's rows are loaded into registers while the current one is multiplied.
// --------------------------------------------------------------------------------------------
constexpr int CTA = 8, CTB = 16, CBM = CTA * CTB, CBN = 64;

template <int P> struct CoreCfg;
template <> struct CoreCfg<GEMM_F32> { using T = float; static constexpr int CK = 64; };
template <> struct CoreCfg<GEMM_BF16X3> { using T = float; static constexpr int CK = 64; };
template <> struct CoreCfg<GEMM_F64> { using T = double; static constexpr int CK = 32; };

typedef float f16v __attribute__((ext_vector_type(16)));

// row of the 32x32 FP32-output MFMA result held by lane `lane`, register v (column lane % 32)
__device__ __forceinline__ int row32(int lane, int v) { return (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3); }

template <int P>
__global__ void __launch_bounds__(256) k_core(CoreArgs g, int kchunk, typename CoreCfg<P>::T* work) {
    using T = typename CoreCfg<P>::T;
    constexpr int CK = CoreCfg<P>::CK;
    constexpr bool BF = (P == GEMM_BF16X3);
    constexpr int KPAD = BF ? 8 : 4;
    // staged projections; K tile [k][m] (FP32/FP64) or split bf16 [m][k] (BF16X3); B likewise
    __shared__ T Y1s[CK][CTA];
    __shared__ T Y2s[CK][CTB];
    __shared__ __attribute__((aligned(16))) T Bs[BF ? 1 : CK][BF ? 1 : CBN + 4];
    __shared__ __attribute__((aligned(16))) T Ks[BF ? 1 : CK][BF ? 1 : CBM + 4];
    __shared__ __attribute__((aligned(16))) __bf16 Khi[BF ? CBM : 1][BF ? CK + KPAD : 1];
    __shared__ __attribute__((aligned(16))) __bf16 Klo[BF ? CBM : 1][BF ? CK + KPAD : 1];
    __shared__ __attribute__((aligned(16))) __bf16 Bhi[BF ? CBN : 1][BF ? CK + KPAD : 1];
    __shared__ __attribute__((aligned(16))) __bf16 Blo[BF ? CBN : 1][BF ? CK + KPAD : 1];
    const int nb2 = (g.r2 + CTB - 1) / CTB;
    const int a0 = (blockIdx.y / nb2) * CTA, b0 = (blockIdx.y % nb2) * CTB, c0 = blockIdx.x * CBN;
    const int kbeg = blockIdx.z * kchunk;
    const int kend = min(g.K, kbeg + kchunk);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wm = wave * 32;

    // register prefetch of one chunk: X3 rows (CK x 64, read as 16-byte vectors: the rows are
    // 16-byte aligned since ldx is a multiple of 4) and the CK x 24 values of X1, X2
    constexpr int VW = 16 / (int)sizeof(T);
    using TV = T __attribute__((ext_vector_type(VW)));
    constexpr int NB = CK * CBN / (256 * VW);                // Y3 vectors per thread
    constexpr int NXY = (CK * (CTA + CTB) + 255) / 256;      // Y1/Y2 values per thread
    TV pb[NB];
    T pxy[NXY];
    const T* __restrict__ X1 = (const T*)g.X1;
    const T* __restrict__ X2 = (const T*)g.X2;
    const T* __restrict__ X3 = (const T*)g.X3;
    auto fetch = [&](int k0) {
#pragma unroll
        for (int t = 0; t < NB; ++t) {
            const int e = tid + 256 * t;
            const int kk = e / (CBN / VW), cc = (e % (CBN / VW)) * VW;
            const int nu = k0 + kk, c = c0 + cc;
            TV v = {};
            if (nu < kend) {
                const T* row = X3 + (long)nu * g.ldx3;
                if (c + VW <= g.r3) {
                    v = *(const TV*)(row + c);
                } else {
#pragma unroll
                    for (int u = 0; u < VW; ++u)
                        if (c + u < g.r3) v[u] = row[c + u];
                }
            }
            pb[t] = v;
        }
#pragma unroll
        for (int t = 0; t < NXY; ++t) {
            const int e = tid + 256 * t;
            T v = T(0);
            if (e < CK * (CTA + CTB)) {
                const int kk = e / (CTA + CTB), cc = e % (CTA + CTB);
                const int nu = k0 + kk;
                if (nu < kend) {
                    if (cc < CTA) {
                        if (a0 + cc < g.r1) v = X1[(long)nu * g.ldx1 + a0 + cc];
                    } else if (b0 + cc - CTA < g.r2) {
                        v = X2[(long)nu * g.ldx2 + b0 + cc - CTA];
                    }
                }
            }
            pxy[t] = v;
        }
    };

    // accumulators
    f16v acc[2];            // FP32 / BF16X3: 32 x 64 per wave as two 32x32 blocks
    double acc64[2][16];    // their FP64 sums across chunks
    d4 accd[2][4];          // FP64: 2 x 4 blocks of 16x16
    if constexpr (P == GEMM_F64) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) accd[i][j] = d4{0, 0, 0, 0};
    } else {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            acc[j] = f16v{};
#pragma unroll
            for (int v = 0; v < 16; ++v) acc64[j][v] = 0.0;
        }
    }

    fetch(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += CK) {
        // registers -> LDS
#pragma unroll
        for (int t = 0; t < NB; ++t) {
            const int e = tid + 256 * t;
            const int kk = e / (CBN / VW), cc = (e % (CBN / VW)) * VW;
#pragma unroll
            for (int u = 0; u < VW; ++u) {
                if constexpr (BF) {
                    const float x = pb[t][u];
                    const __bf16 hx = (__bf16)x;
                    Bhi[cc + u][kk] = hx;
                    Blo[cc + u][kk] = (__bf16)(x - (float)hx);
                } else {
                    Bs[kk][cc + u] = pb[t][u];
                }
            }
        }
#pragma unroll
        for (int t = 0; t < NXY; ++t) {
            const int e = tid + 256 * t;
            if (e < CK * (CTA + CTB)) {
                const int kk = e / (CTA + CTB), cc = e % (CTA + CTB);
                if (cc < CTA) Y1s[kk][cc] = pxy[t];
                else Y2s[kk][cc - CTA] = pxy[t];
            }
        }
        __syncthreads();
        if (k0 + CK < kend) fetch(k0 + CK);
        // Khatri-Rao tile
        for (int e = tid; e < CK * CBM; e += 256) {
            if constexpr (BF) {
                const int m = e / CK, kk = e % CK;
                const float x = Y1s[kk][m / CTB] * Y2s[kk][m % CTB];
                const __bf16 hx = (__bf16)x;
                Khi[m][kk] = hx;
                Klo[m][kk] = (__bf16)(x - (float)hx);
            } else {
                const int kk = e / CBM, m = e % CBM;
                Ks[kk][m] = Y1s[kk][m / CTB] * Y2s[kk][m % CTB];
            }
        }
        __syncthreads();
        if constexpr (P == GEMM_F32) {
#pragma unroll
            for (int kk = 0; kk < CK; kk += 2) {
                const float a = Ks[kk + (lane >> 5)][wm + (lane & 31)];
                float b[2];
#pragma unroll
                for (int j = 0; j < 2; ++j) b[j] = Bs[kk + (lane >> 5)][j * 32 + (lane & 31)];
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b[j], acc[j], 0, 0, 0);
            }
        } else if constexpr (BF) {
#pragma unroll
            for (int kk = 0; kk < CK; kk += 16) {
                const int ko = kk + 8 * (lane >> 5);
                const bf8 ah = *(const bf8*)&Khi[wm + (lane & 31)][ko];
                const bf8 al = *(const bf8*)&Klo[wm + (lane & 31)][ko];
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const bf8 bh = *(const bf8*)&Bhi[j * 32 + (lane & 31)][ko];
                    const bf8 bl = *(const bf8*)&Blo[j * 32 + (lane & 31)][ko];
                    acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[j], 0, 0, 0);
                    acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[j], 0, 0, 0);
                    acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[j], 0, 0, 0);
                }
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < CK; kk += 4) {
                double a[2], b[4];
#pragma unroll
                for (int i = 0; i < 2; ++i) a[i] = Ks[kk + (lane >> 4)][wm + 16 * i + (lane & 15)];
#pragma unroll
                for (int j = 0; j < 4; ++j) b[j] = Bs[kk + (lane >> 4)][16 * j + (lane & 15)];
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        accd[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], accd[i][j], 0, 0, 0);
            }
        }
        if constexpr (P != GEMM_F64) {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
#pragma unroll
                for (int v = 0; v < 16; ++v) acc64[j][v] += (double)acc[j][v];
                acc[j] = f16v{};
            }
        }
        __syncthreads();
    }
    const long plane = (long)g.r1 * g.r2 * g.r3;
    T* out = (gridDim.z > 1) ? work + (long)blockIdx.z * plane : (T*)g.core;
    if constexpr (P == GEMM_F64) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int m = wm + 16 * i + (lane >> 4) + 4 * v;
                    const int a = a0 + m / CTB, b = b0 + m % CTB, c = c0 + 16 * j + (lane & 15);
                    if (a < g.r1 && b < g.r2 && c < g.r3) out[((long)a * g.r2 + b) * g.r3 + c] = accd[i][j][v];
                }
    } else {
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int m = wm + row32(lane, v);
                const int a = a0 + m / CTB, b = b0 + m % CTB, c = c0 + 32 * j + (lane & 31);
                if (a < g.r1 && b < g.r2 && c < g.r3) out[((long)a * g.r2 + b) * g.r3 + c] = (float)acc64[j][v];
            }
    }
}

// Term-major operands of the core: one 64-lane row copy per term.
template <typename T>
__global__ void __launch_bounds__(256) k_gather_terms(int K, int r, const T* __restrict__ Yt, long ldy,
                                                      const int32_t* __restrict__ idx,
                                                      const double* __restrict__ sc, T* __restrict__ X,
                                                      long ldx) {
    const int nu = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (nu >= K) return;
    const T* src = Yt + (long)idx[nu] * ldy;
    T* dst = X + (long)nu * ldx;
    const T s = sc ? (T)sc[nu] : T(1);
    for (int a = threadIdx.x & 63; a < ldx; a += 64) dst[a] = a < r ? s * src[a] : T(0);
}

template <typename T>
__global__ void __launch_bounds__(256) k_reduce_split(long n, int k_split, const T* __restrict__ work,
                                                      T* __restrict__ out) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int z = 0; z < k_split; ++z) s += (double)work[(long)z * n + i];
    out[i] = (T)s;
}

// ||A||^2 = sum_{g,g'} s_g s_g' sum_{q,q'} prod_l C_l[s_l(g)R+q, s_l(g')R+q'] (unnormalised
// columns, so xi_nu = scale_g).  One workgroup per g; partial[g] written, summed on the host.
__global__ void __launch_bounds__(256) k_cp_norm2(int R, int n_groups, const int32_t* __restrict__ s1,
                                                  const int32_t* __restrict__ s2,
                                                  const int32_t* __restrict__ s3,
                                                  const double* __restrict__ scale,
                                                  const double* __restrict__ C1,
                                                  const double* __restrict__ C2,
                                                  const double* __restrict__ C3, int D1, int D2,
                                                  int D3, double* __restrict__ partial) {
    __shared__ double red[256];
    const int g = blockIdx.x;
    const long r1 = (long)s1[g] * R, r2 = (long)s2[g] * R, r3 = (long)s3[g] * R;
    double acc = 0.0;
    for (int gp = 0; gp < n_groups; ++gp) {
        const long c1 = (long)s1[gp] * R, c2 = (long)s2[gp] * R, c3 = (long)s3[gp] * R;
        double sub = 0.0;
        for (int e = threadIdx.x; e < R * R; e += 256) {
            const int q = e / R, qp = e % R;
            sub += C1[(r1 + q) * D1 + c1 + qp] * C2[(r2 + q) * D2 + c2 + qp] * C3[(r3 + q) * D3 + c3 + qp];
        }
        acc += scale[gp] * sub;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[g] = scale[g] * red[0];
}

inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

void launch_gemm(hipStream_t st, GemmPrec prec, const GemmArgs& a) {
    if (a.m <= 0 || a.n <= 0 || a.batch <= 0) return;
    dim3 grid(cdiv(a.n, BN), cdiv(a.m, BM), a.batch);
    switch (prec) {
        case GEMM_F64: hipLaunchKernelGGL(k_gemm<GEMM_F64>, grid, dim3(256), 0, st, a); break;
        case GEMM_F32: hipLaunchKernelGGL(k_gemm<GEMM_F32>, grid, dim3(256), 0, st, a); break;
        case GEMM_BF16X3: hipLaunchKernelGGL(k_gemm<GEMM_BF16X3>, grid, dim3(256), 0, st, a); break;
    }
}

void launch_core(hipStream_t st, GemmPrec prec, const CoreArgs& a, int k_split, void* work) {
    if (a.r1 <= 0 || a.r2 <= 0 || a.r3 <= 0) return;
    const int ck = prec == GEMM_F64 ? CoreCfg<GEMM_F64>::CK : CoreCfg<GEMM_F32>::CK;
    k_split = std::max(1, k_split);
    const int kchunk = (int)(((long)(a.K + k_split - 1) / k_split + ck - 1) / ck * ck);
    dim3 grid(cdiv(a.r3, CBN), cdiv(a.r1, CTA) * cdiv(a.r2, CTB), k_split);
    const long plane = (long)a.r1 * a.r2 * a.r3;
    switch (prec) {
        case GEMM_F64:
            hipLaunchKernelGGL(k_core<GEMM_F64>, grid, dim3(256), 0, st, a, kchunk, (double*)work);
            if (k_split > 1)
                hipLaunchKernelGGL(k_reduce_split<double>, dim3(cdiv(plane, 256)), dim3(256), 0, st,
                                   plane, k_split, (const double*)work, (double*)a.core);
            break;
        case GEMM_F32:
            hipLaunchKernelGGL(k_core<GEMM_F32>, grid, dim3(256), 0, st, a, kchunk, (float*)work);
            if (k_split > 1)
                hipLaunchKernelGGL(k_reduce_split<float>, dim3(cdiv(plane, 256)), dim3(256), 0, st,
                                   plane, k_split, (const float*)work, (float*)a.core);
            break;
        case GEMM_BF16X3:
            hipLaunchKernelGGL(k_core<GEMM_BF16X3>, grid, dim3(256), 0, st, a, kchunk, (float*)work);
            if (k_split > 1)
                hipLaunchKernelGGL(k_reduce_split<float>, dim3(cdiv(plane, 256)), dim3(256), 0, st,
                                   plane, k_split, (const float*)work, (float*)a.core);
            break;
    }
}

void launch_gather_terms(hipStream_t st, int elem, int K, int r, const void* Yt, long ldy,
                         const int32_t* idx, const double* sc, void* X, long ldx) {
    if (K <= 0) return;
    if (elem == 8)
        hipLaunchKernelGGL(k_gather_terms<double>, dim3(cdiv(K, 4)), dim3(256), 0, st, K, r, (const double*)Yt,
                           ldy, idx, sc, (double*)X, ldx);
    else
        hipLaunchKernelGGL(k_gather_terms<float>, dim3(cdiv(K, 4)), dim3(256), 0, st, K, r, (const float*)Yt,
                           ldy, idx, sc, (float*)X, ldx);
}

void launch_cp_norm2(hipStream_t st, int R, int n_groups, const int32_t* src1, const int32_t* src2,
                     const int32_t* src3, const double* scale, const double* C1, const double* C2,
                     const double* C3, int D1, int D2, int D3, double* partial, int n_partial) {
    (void)n_partial;
    if (n_groups <= 0) return;
    hipLaunchKernelGGL(k_cp_norm2, dim3(n_groups), dim3(256), 0, st, R, n_groups, src1, src2, src3,
                       scale, C1, C2, C3, D1, D2, D3, partial);
}

}  // namespace lsum

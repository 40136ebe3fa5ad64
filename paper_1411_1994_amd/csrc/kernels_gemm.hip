// MFMA contraction kernels (gfx950): the dense steps of the RHOSVD and Tucker evaluation.
//
//  * k_gemm: strided GEMM C = alpha A B + beta C (column Grams, the projections of Appendix
//    theorem (c), the mode products of eq. Tucker_singePot, Tucker values at points);
//  * k_core: the RHOSVD core mu = sum_nu xi_nu y1_nu (x) y2_nu (x) y3_nu (eq. C-core) as a GEMM
//    whose left operand, the Khatri-Rao product of the mode-1 and mode-2 projections, is formed
//    on the fly in LDS so it never touches HBM;
//  * k_core_groups: the same sum with the terms that share a mode-3 column added first (the
//    mode-3 contraction is then a k_gemm over the distinct columns);
//  * k_cp_norm2: ||A||_F^2 of the canonical sum from the column Grams (truncation rule).
//
// Both GEMM-shaped kernels use 128 x 64 workgroup tiles with 32 rows per wave:
// v_mfma_f32_32x32x2f32 (FP32), v_mfma_f32_32x32x16_bf16 three times (split BF16x3: x = hi +
// lo, hi*hi + hi*lo + lo*hi) or v_mfma_f64_16x16x4f64 (FP64).  FP32 and BF16x3 partial sums are
// added into FP64 registers every chunk of 32 (GEMM) or 64 (core) terms, so the summation error stays near the
// operand rounding instead of growing with the contraction length.
//
// MFMA lane layouts: 16x16x4 (f64) takes A[row lane%16][k lane/16], B[k lane/16][col lane%16]
// and leaves row lane/16 + 4v, column lane%16 in register v.  32x32x2 (f32) takes A[row
// lane%32][k lane/32] and leaves row 8(v/4) + 4(lane/32) + v%4, column lane%32 in register v;
// 32x32x16 (bf16) takes 8 consecutive k per lane, k = 8(lane/32) + e, with the same output
// layout.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lsum_internal.h"

namespace lsum {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// --------------------------------------------------------------------------------------------
// General strided GEMM, C = alpha A B + beta C, on a 128 x 64 workgroup tile: wave w owns rows
// 32w..32w+31 and the 64 columns, multiplied in chunks of GK terms staged in LDS.
//   FP32:   v_mfma_f32_32x32x2f32, FP32 sums within the chunk, FP64 across chunks;
//   BF16X3: v_mfma_f32_32x32x16_bf16 on hi*hi + hi*lo + lo*hi (operands split when staged);
//   FP64:   v_mfma_f64_16x16x4f64 throughout.
// Operands are read with the element strides given (threads walk the unit-stride direction when
// there is one, so loads coalesce), and the next chunk is fetched into registers while the
// current one is multiplied.
// --------------------------------------------------------------------------------------------
constexpr int GBM = 128, GBN = 64;
template <int P> struct GemmCfg;
template <> struct GemmCfg<GEMM_F32> { using T = float; static constexpr int GK = 32; };
template <> struct GemmCfg<GEMM_BF16X3> { using T = float; static constexpr int GK = 32; };
template <> struct GemmCfg<GEMM_F64> { using T = double; static constexpr int GK = 16; };

typedef float f16v_g __attribute__((ext_vector_type(16)));

__device__ __forceinline__ int row32g(int lane, int v) { return (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3); }

template <int P>
__global__ void __launch_bounds__(256) k_gemm(GemmArgs g) {
    using T = typename GemmCfg<P>::T;
    constexpr int GK = GemmCfg<P>::GK;
    constexpr bool BF = (P == GEMM_BF16X3);
    constexpr int KPAD = 8;
    __shared__ __attribute__((aligned(16))) T As[BF ? 1 : GK][BF ? 1 : GBM + 4];
    __shared__ __attribute__((aligned(16))) T Bs[BF ? 1 : GK][BF ? 1 : GBN + 4];
    __shared__ __attribute__((aligned(16))) __bf16 Ahi[BF ? GBM : 1][BF ? GK + KPAD : 1];
    __shared__ __attribute__((aligned(16))) __bf16 Alo[BF ? GBM : 1][BF ? GK + KPAD : 1];
    __shared__ __attribute__((aligned(16))) __bf16 Bhi[BF ? GBN : 1][BF ? GK + KPAD : 1];
    __shared__ __attribute__((aligned(16))) __bf16 Blo[BF ? GBN : 1][BF ? GK + KPAD : 1];
    const long bz = blockIdx.z;
    const T* __restrict__ A = (const T*)g.A + bz * g.bA;
    const T* __restrict__ B = (const T*)g.B + bz * g.bB;
    T* __restrict__ C = (T*)g.C + bz * g.bC;
    const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wm = wave * 32;
    const bool a_kfast = (g.sak == 1);
    const bool b_nfast = (g.sbn == 1);
    constexpr int NA = GBM * GK / 256, NB = GBN * GK / 256;   // staged elements per thread
    // Each thread keeps one position along the unit-stride direction and steps along the other:
    // element t of A is (mA + t * dmA, kA + t * dkA), of B (kB + t * dkB, nB + t * dnB).
    const int mA = a_kfast ? tid / GK : tid % GBM, kA = a_kfast ? tid % GK : tid / GBM;
    const int dmA = a_kfast ? 256 / GK : 0, dkA = a_kfast ? 0 : 256 / GBM;
    const int nB = b_nfast ? tid % GBN : tid / GK, kB = b_nfast ? tid / GBN : tid % GK;
    const int dnB = b_nfast ? 0 : 256 / GK, dkB = b_nfast ? 256 / GBN : 0;
    const long stepA = (long)dmA * g.sam + (long)dkA * g.sak;
    const long stepB = (long)dkB * g.sbk + (long)dnB * g.sbn;
    T pa[NA], pb[NB];
    // Loads are unconditional, so no lane overwrites a register that a load is still filling and
    // the next chunk stays in flight while the current one is multiplied: an element outside the
    // operand reads the operand's first element instead (rows and columns past m, n only reach
    // outputs that are never stored; terms past k are zeroed when staged).
    auto fetch = [&](int k0) {
        const T* a = A + (long)(m0 + mA) * g.sam + (long)(k0 + kA) * g.sak;
        const bool a_in = m0 + GBM <= g.m && k0 + GK <= g.k;
#pragma unroll
        for (int t = 0; t < NA; ++t) {
            const bool ok = a_in || (m0 + mA + t * dmA < g.m && k0 + kA + t * dkA < g.k);
            pa[t] = *(ok ? a + t * stepA : A);
        }
        const T* b = B + (long)(k0 + kB) * g.sbk + (long)(n0 + nB) * g.sbn;
        const bool b_in = n0 + GBN <= g.n && k0 + GK <= g.k;
#pragma unroll
        for (int t = 0; t < NB; ++t) {
            const bool ok = b_in || (n0 + nB + t * dnB < g.n && k0 + kB + t * dkB < g.k);
            pb[t] = *(ok ? b + t * stepB : B);
        }
    };
    f16v_g acc[2];
    double acc64[2][16];
    d4 accd[2][4];
    if constexpr (P == GEMM_F64) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) accd[i][j] = d4{0, 0, 0, 0};
    } else {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            acc[j] = f16v_g{};
#pragma unroll
            for (int v = 0; v < 16; ++v) acc64[j][v] = 0.0;
        }
    }
    if (g.k > 0) fetch(0);   // k = 0: only the beta C epilogue
    for (int k0 = 0; k0 < g.k; k0 += GK) {
#pragma unroll
        for (int t = 0; t < NA; ++t) {
            const int mm = mA + t * dmA, kk = kA + t * dkA;
            const T xa = k0 + kk < g.k ? pa[t] : T(0);
            if constexpr (BF) {
                const float x = xa;
                const __bf16 hx = (__bf16)x;
                Ahi[mm][kk] = hx;
                Alo[mm][kk] = (__bf16)(x - (float)hx);
            } else {
                As[kk][mm] = xa;
            }
        }
#pragma unroll
        for (int t = 0; t < NB; ++t) {
            const int nn = nB + t * dnB, kk = kB + t * dkB;
            const T xb = k0 + kk < g.k ? pb[t] : T(0);
            if constexpr (BF) {
                const float x = xb;
                const __bf16 hx = (__bf16)x;
                Bhi[nn][kk] = hx;
                Blo[nn][kk] = (__bf16)(x - (float)hx);
            } else {
                Bs[kk][nn] = xb;
            }
        }
        __syncthreads();
        if (k0 + GK < g.k) fetch(k0 + GK);
        if constexpr (P == GEMM_F32) {
#pragma unroll
            for (int kk = 0; kk < GK; kk += 2) {
                const float a = As[kk + (lane >> 5)][wm + (lane & 31)];
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, Bs[kk + (lane >> 5)][32 * j + (lane & 31)], acc[j],
                                                                  0, 0, 0);
            }
        } else if constexpr (BF) {
#pragma unroll
            for (int kk = 0; kk < GK; kk += 16) {
                const int ko = kk + 8 * (lane >> 5);
                const bf8 ah = *(const bf8*)&Ahi[wm + (lane & 31)][ko];
                const bf8 al = *(const bf8*)&Alo[wm + (lane & 31)][ko];
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const bf8 bh = *(const bf8*)&Bhi[32 * j + (lane & 31)][ko];
                    const bf8 bl = *(const bf8*)&Blo[32 * j + (lane & 31)][ko];
                    acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[j], 0, 0, 0);
                    acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[j], 0, 0, 0);
                    acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[j], 0, 0, 0);
                }
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < GK; kk += 4) {
                double a[2], b[4];
#pragma unroll
                for (int i = 0; i < 2; ++i) a[i] = As[kk + (lane >> 4)][wm + 16 * i + (lane & 15)];
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
                acc[j] = f16v_g{};
            }
        }
        __syncthreads();
    }
    auto store = [&](int row, int col, double val) {
        if (row < g.m && col < g.n) {
            T* c = C + (long)row * g.scm + (long)col * g.scn;
            const double v = g.alpha * val;
            *c = (T)((g.beta != 0.0) ? v + g.beta * (double)*c : v);
        }
    };
    if constexpr (P == GEMM_F64) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    store(m0 + wm + 16 * i + (lane >> 4) + 4 * v, n0 + 16 * j + (lane & 15), accd[i][j][v]);
    } else {
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v)
                store(m0 + wm + row32g(lane, v), n0 + 32 * j + (lane & 31), acc64[j][v]);
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

    // register prefetch of one chunk: X3 rows (CK x 64, read as 16-byte vectors) and the CK x 24
    // values of X1, X2.  Every load is unconditional from a clamped address inside the operands
    // (rows past the chunk repeat its last row; columns past r3 stay in the row: ldx3 is a
    // multiple of 4 and its padding is zero), so no lane overwrites a register a load is still
    // filling and the loads stay in flight across the multiplication of the current chunk.
    // Rows past the chunk are zeroed when staged in LDS; out-of-range a, b, c only reach outputs
    // that are never stored.
    constexpr int VW = 16 / (int)sizeof(T);
    using TV = T __attribute__((ext_vector_type(VW)));
    constexpr int NB = CK * CBN / (256 * VW);                // Y3 vectors per thread
    constexpr int NXY = CK * (CTA + CTB) / 256;              // Y1/Y2 values per thread
    static_assert(CK * (CTA + CTB) % 256 == 0 && CK * CBN % (256 * VW) == 0, "chunk must tile the workgroup");
    TV pb[NB];
    T pxy[NXY];
    const T* __restrict__ X1 = (const T*)g.X1;
    const T* __restrict__ X2 = (const T*)g.X2;
    const T* __restrict__ X3 = (const T*)g.X3;
    const int ld1 = (int)g.ldx1, ld2 = (int)g.ldx2, ld3 = (int)g.ldx3;
    auto fetch = [&](int k0) {
#pragma unroll
        for (int t = 0; t < NB; ++t) {
            const int e = tid + 256 * t;
            const int kk = e / (CBN / VW), cc = (e % (CBN / VW)) * VW;
            const int nu = min(k0 + kk, kend - 1), c = min(c0 + cc, ld3 - VW);
            pb[t] = *(const TV*)(X3 + (size_t)nu * ld3 + c);
        }
#pragma unroll
        for (int t = 0; t < NXY; ++t) {
            const int e = tid + 256 * t;
            const int kk = e / (CTA + CTB), cc = e % (CTA + CTB);
            const int nu = min(k0 + kk, kend - 1);
            const T* src = cc < CTA ? X1 + (size_t)nu * ld1 + min(a0 + cc, g.r1 - 1)
                                    : X2 + (size_t)nu * ld2 + min(b0 + cc - CTA, g.r2 - 1);
            pxy[t] = *src;
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

    if (kbeg < kend) fetch(kbeg);   // an empty split chunk stores zeros
    for (int k0 = kbeg; k0 < kend; k0 += CK) {
        // registers -> LDS
#pragma unroll
        for (int t = 0; t < NB; ++t) {
            const int e = tid + 256 * t;
            const int kk = e / (CBN / VW), cc = (e % (CBN / VW)) * VW;
            const bool live = k0 + kk < kend;
#pragma unroll
            for (int u = 0; u < VW; ++u) {
                if constexpr (BF) {
                    const float x = live ? pb[t][u] : 0.0f;
                    const __bf16 hx = (__bf16)x;
                    Bhi[cc + u][kk] = hx;
                    Blo[cc + u][kk] = (__bf16)(x - (float)hx);
                } else {
                    Bs[kk][cc + u] = live ? pb[t][u] : T(0);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < NXY; ++t) {
            const int e = tid + 256 * t;
            const int kk = e / (CTA + CTB), cc = e % (CTA + CTB);
            const T v = k0 + kk < kend ? pxy[t] : T(0);
            if (cc < CTA) Y1s[kk][cc] = v;
            else Y2s[kk][cc - CTA] = v;
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

// Grouped core terms: the canonical terms that share a mode-3 column j are summed before the
// mode-3 contraction, T[j][a][b] = sum_{nu in j} s_nu Y1[i1(nu), a] Y2[i2(nu), b], so that the
// core becomes mu = T x_3 Y3 (a plain GEMM over the D3 columns instead of the K terms).  A
// workgroup owns a 64 x 64 tile of (a, b) for one j; the terms of j are staged through LDS 32 at
// a time (the scale folded into the mode-1 row) and summed in FP64 in term order.
constexpr int CG_T = 32;
template <typename T>
__global__ void __launch_bounds__(256) k_core_groups(int r1, int r2, int a_begin, int a_count, int j0,
                                                     const int32_t* __restrict__ off,
                                                     const int32_t* __restrict__ i1, const int32_t* __restrict__ i2,
                                                     const double* __restrict__ sc, const T* __restrict__ Y1,
                                                     long ldy1, const T* __restrict__ Y2, long ldy2,
                                                     T* __restrict__ out) {
    __shared__ double s1[CG_T][64];
    __shared__ double s2[CG_T][64];
    const int a_end = min(r1, a_begin + a_count);
    const int a0 = a_begin + blockIdx.y * 64, b0 = blockIdx.x * 64, jl = blockIdx.z, j = j0 + jl;
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    const int t0 = off[j], t1 = off[j + 1];
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[i][k] = 0.0;
    for (int tb = t0; tb < t1; tb += CG_T) {
        const int nt = min(CG_T, t1 - tb);
        for (int e = tid; e < CG_T * 64; e += 256) {
            const int t = e >> 6, c = e & 63;
            double v1 = 0.0, v2 = 0.0;
            if (t < nt) {
                const int a = a0 + c, b = b0 + c;
                if (a < a_end) v1 = sc[tb + t] * (double)Y1[(long)i1[tb + t] * ldy1 + a];
                if (b < r2) v2 = (double)Y2[(long)i2[tb + t] * ldy2 + b];
            }
            s1[t][c] = v1;
            s2[t][c] = v2;
        }
        __syncthreads();
        for (int t = 0; t < nt; ++t) {
            double x[4], y[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                x[i] = s1[t][ty * 4 + i];
                y[i] = s2[t][tx * 4 + i];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int k = 0; k < 4; ++k) acc[i][k] = fma(x[i], y[k], acc[i][k]);
        }
        __syncthreads();
    }
    T* o = out + (long)jl * a_count * r2;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int a = a0 + ty * 4 + i;
        if (a >= a_end) continue;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int b = b0 + tx * 4 + k;
            if (b < r2) o[(long)(a - a_begin) * r2 + b] = (T)acc[i][k];
        }
    }
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

// Row-wise Khatri-Rao product of two term-major operands: KR[nu, i * rb + j] = Xa[nu, i] Xb[nu, j]
// (Xa K x ra, Xb K x rb, row-major, KR K x (ra rb)).
__global__ void __launch_bounds__(256) k_khatri_rao(long total, int ra, int rb, const double* __restrict__ Xa,
                                                    const double* __restrict__ Xb, double* __restrict__ KR) {
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= total) return;
    const long w = (long)ra * rb;
    const long nu = e / w;
    const int ij = (int)(e - nu * w);
    const int i = ij / rb, j = ij - i * rb;
    KR[e] = Xa[nu * ra + i] * Xb[nu * rb + j];
}

// Galerkin functional (eq. nuc_pot): H[k * nb + m, x] = G[k, x] G[m, x], the 1D Hadamard products
// of every pair of basis vectors of one mode (G nb x n, row-major).
__global__ void __launch_bounds__(256) k_hadamard_pairs(int nb, int n, const double* __restrict__ G,
                                                        double* __restrict__ H) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int pr = blockIdx.y;
    if (x >= n) return;
    const int k = pr / nb, m = pr - k * nb;
    H[(long)pr * n + x] = G[(long)k * n + x] * G[(long)m * n + x];
}

// v[p] = scale * sum_{a,b} X[p, a r2 + b] Y1[p, a] Y2[p, b]: the last two mode contractions of the
// Tucker core with the pairs' projections; one wavefront per pair, fixed summation order.
__global__ void __launch_bounds__(256) k_galerkin_finish(int P, int r1, int r2, const double* __restrict__ X,
                                                         const double* __restrict__ Y1,
                                                         const double* __restrict__ Y2, double scale,
                                                         double* __restrict__ v) {
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (p >= P) return;
    const double* x = X + (long)p * r1 * r2;
    double acc = 0.0;
    for (int e = lane; e < r1 * r2; e += 64) {
        const int a = e / r2, b = e - a * r2;
        acc += x[e] * Y1[(long)p * r1 + a] * Y2[(long)p * r2 + b];
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) v[p] = scale * acc;
}

// A[i * ld + off + i] = 1 for i < n: the identity block of an augmented matrix.
// UT[i * ldt + q] = U[q * ldu + i] (q < R, i < N), through a 32 x 32 LDS tile.
__global__ void __launch_bounds__(256) k_transpose_ld(int R, int N, const double* __restrict__ U, int ldu,
                                                      double* __restrict__ UT, long ldt) {
    __shared__ double tile[32][33];
    const int i0 = blockIdx.x * 32, q0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int k = ty; k < 32; k += 8) {
        const int q = q0 + k, i = i0 + tx;
        tile[k][tx] = (q < R && i < N) ? U[(size_t)q * ldu + i] : 0.0;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int i = i0 + k, q = q0 + tx;
        if (i < N && q < R) UT[(size_t)i * ldt + q] = tile[tx][k];
    }
}

__global__ void __launch_bounds__(256) k_unit_diag(int n, long ld, long off, double* __restrict__ A) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) A[(long)i * ld + off + i] = 1.0;
}

// C = alpha * sum_z work_z + beta * C for an m x n output with strides (scm, scn): the partial
// products of a GEMM whose reduction was split into slices, summed in slice order.
__global__ void __launch_bounds__(256) k_sum_split(int m, int n, int split, const double* __restrict__ work,
                                                   double alpha, double beta, double* __restrict__ C, long scm,
                                                   long scn) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    const long mn = (long)m * n;
    if (i >= mn) return;
    double s = 0.0;
    for (int z = 0; z < split; ++z) s += work[(long)z * mn + i];
    double* c = C + (i / n) * scm + (i % n) * scn;
    *c = (beta != 0.0) ? alpha * s + beta * *c : alpha * s;
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
    if (blas_gemm(st, prec, a)) return;
    dim3 grid(cdiv(a.n, GBN), cdiv(a.m, GBM), a.batch);
    switch (prec) {
        case GEMM_F64: hipLaunchKernelGGL(k_gemm<GEMM_F64>, grid, dim3(256), 0, st, a); break;
        case GEMM_F32: hipLaunchKernelGGL(k_gemm<GEMM_F32>, grid, dim3(256), 0, st, a); break;
        case GEMM_BF16X3: hipLaunchKernelGGL(k_gemm<GEMM_BF16X3>, grid, dim3(256), 0, st, a); break;
    }
}

int gemm_split_slices(const GemmArgs& a, int split) {
    constexpr int GKf = GemmCfg<GEMM_F64>::GK;
    const long kslice = ((long)(a.k + split - 1) / split + GKf - 1) / GKf * GKf;
    return (int)((a.k + kslice - 1) / kslice);
}

void launch_khatri_rao(hipStream_t st, int K, int ra, int rb, const double* Xa, const double* Xb, double* KR) {
    const long total = (long)K * ra * rb;
    if (total <= 0) return;
    hipLaunchKernelGGL(k_khatri_rao, dim3(cdiv(total, 256)), dim3(256), 0, st, total, ra, rb, Xa, Xb, KR);
}

void launch_hadamard_pairs(hipStream_t st, int nb, int n, const double* G, double* H) {
    if (nb <= 0 || n <= 0) return;
    hipLaunchKernelGGL(k_hadamard_pairs, dim3(cdiv(n, 256), (unsigned)nb * nb), dim3(256), 0, st, nb, n, G, H);
}

void launch_galerkin_finish(hipStream_t st, int P, int r1, int r2, const double* X, const double* Y1,
                            const double* Y2, double scale, double* v) {
    if (P <= 0) return;
    hipLaunchKernelGGL(k_galerkin_finish, dim3(cdiv(P, 4)), dim3(256), 0, st, P, r1, r2, X, Y1, Y2, scale, v);
}

void launch_transpose_ld(hipStream_t st, int R, int N, const double* U, int ldu, double* UT, long ldt) {
    if (R <= 0 || N <= 0) return;
    hipLaunchKernelGGL(k_transpose_ld, dim3(cdiv(N, 32), cdiv(R, 32)), dim3(256), 0, st, R, N, U, ldu, UT, ldt);
}

void launch_unit_diag(hipStream_t st, int n, long ld, long off, double* A) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_unit_diag, dim3(cdiv(n, 256)), dim3(256), 0, st, n, ld, off, A);
}

void launch_gemm_split_f64(hipStream_t st, const GemmArgs& a, int split, double* work) {
    if (a.m <= 0 || a.n <= 0 || a.batch != 1) return;
    constexpr int GKf = GemmCfg<GEMM_F64>::GK;
    const long kslice = ((long)(a.k + split - 1) / split + GKf - 1) / GKf * GKf;
    const int slices = (int)((a.k + kslice - 1) / kslice);
    const int full = (int)(a.k / kslice);                 // slices of kslice terms; the rest is shorter
    const long mn = (long)a.m * a.n;
    GemmArgs b = a;
    b.C = work;
    b.scm = a.n;
    b.scn = 1;
    b.alpha = 1.0;
    b.beta = 0.0;
    b.bA = kslice * a.sak;
    b.bB = kslice * a.sbk;
    b.bC = mn;
    if (full > 0) {
        b.k = (int)kslice;
        b.batch = full;
        hipLaunchKernelGGL(k_gemm<GEMM_F64>, dim3(cdiv(a.n, GBN), cdiv(a.m, GBM), full), dim3(256), 0, st, b);
    }
    if (full < slices) {
        GemmArgs r = b;
        r.k = (int)(a.k - (long)full * kslice);
        r.batch = 1;
        r.A = (const double*)a.A + (long)full * kslice * a.sak;
        r.B = (const double*)a.B + (long)full * kslice * a.sbk;
        r.C = work + (long)full * mn;
        hipLaunchKernelGGL(k_gemm<GEMM_F64>, dim3(cdiv(a.n, GBN), cdiv(a.m, GBM), 1), dim3(256), 0, st, r);
    }
    hipLaunchKernelGGL(k_sum_split, dim3(cdiv(mn, 256)), dim3(256), 0, st, a.m, a.n, slices, work, a.alpha,
                       a.beta, (double*)a.C, a.scm, a.scn);
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

void launch_core_groups(hipStream_t st, int elem, int r1, int r2, int a_begin, int a_count, int j0, int nj,
                        const int32_t* off, const int32_t* i1, const int32_t* i2, const double* sc, const void* Y1,
                        long ldy1, const void* Y2, long ldy2, void* out) {
    if (nj <= 0 || r1 <= 0 || r2 <= 0 || a_count <= 0 || a_begin < 0 || a_begin >= r1) return;
    const dim3 grid(cdiv(r2, 64), cdiv(std::min(a_count, r1 - a_begin), 64), nj);
    if (elem == 8)
        hipLaunchKernelGGL(k_core_groups<double>, grid, dim3(256), 0, st, r1, r2, a_begin, a_count, j0, off, i1, i2,
                           sc, (const double*)Y1, ldy1, (const double*)Y2, ldy2, (double*)out);
    else
        hipLaunchKernelGGL(k_core_groups<float>, grid, dim3(256), 0, st, r1, r2, a_begin, a_count, j0, off, i1, i2,
                           sc, (const float*)Y1, ldy1, (const float*)Y2, ldy2, (float*)out);
}

// The canonical sum at probe cells, in FP64 (the discrete tensor before truncation):
// out[p] = sum_g scale[g] sum_k prod_l C_l[(src_l[g] R + k) * N_l + cell_l(p)], one workgroup per
// cell, the terms strided over its threads and summed by a fixed tree (deterministic).
__global__ void __launch_bounds__(256) k_probe_canonical(int R, int n_groups, const int32_t* __restrict__ s1,
                                                         const int32_t* __restrict__ s2,
                                                         const int32_t* __restrict__ s3,
                                                         const double* __restrict__ scale,
                                                         const double* __restrict__ C1, const double* __restrict__ C2,
                                                         const double* __restrict__ C3, int N1, int N2, int N3,
                                                         const int32_t* __restrict__ cells, double* __restrict__ out) {
    __shared__ double red[256];
    const int p = blockIdx.x, tid = threadIdx.x;
    const int i1 = cells[3 * p], i2 = cells[3 * p + 1], i3 = cells[3 * p + 2];
    const long K = (long)n_groups * R;
    double v = 0.0;
    for (long nu = tid; nu < K; nu += 256) {
        const int g = (int)(nu / R), k = (int)(nu % R);
        v += scale[g] * C1[(size_t)(s1[g] * R + k) * N1 + i1] * C2[(size_t)(s2[g] * R + k) * N2 + i2] *
             C3[(size_t)(s3[g] * R + k) * N3 + i3];
    }
    red[tid] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) out[p] = red[0];
}

void launch_probe_canonical(hipStream_t st, int n_cells, int R, int n_groups, const int32_t* s1, const int32_t* s2,
                            const int32_t* s3, const double* scale, const double* C1, const double* C2,
                            const double* C3, int N1, int N2, int N3, const int32_t* cells, double* out) {
    if (n_cells <= 0) return;
    hipLaunchKernelGGL(k_probe_canonical, dim3(n_cells), dim3(256), 0, st, R, n_groups, s1, s2, s3, scale, C1, C2,
                       C3, N1, N2, N3, cells, out);
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

// One-sided block-Jacobi SVD (FP64) of a side matrix, for the truncated SVD of Def. def:RHOSVD.
//
// The D columns of the side matrix are the rows of X (length N).  A sweep visits every pair of
// 8-column blocks once (circle-method round robin, nblk-1 rounds of nblk/2 disjoint pairs); for
// each pair one workgroup
//   1. forms the 16x16 Gram of the 16 columns on v_mfma_f64_16x16x4 (K = N split over 4 waves),
//   2. diagonalises it with cyclic two-sided Jacobi in one wavefront (LDS-resident), which is
//      accurate relative to each column's own norm once the columns are nearly orthogonal,
//   3. rotates the 16 columns in place, X <- Q^T X, again on MFMA.
// Columns are never squared against each other globally, so singular values are resolved far
// below sqrt(eps_mach) * sigma_max -- the RHOSVD threshold at eps = 1e-6 sits near 1e-8 sigma_1.
// Between sweeps the columns are re-sorted by norm so that blocks hold similar magnitudes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>

#include "lsum_internal.h"

namespace lsum {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void pair_of(int n, int round, int i, int* a, int* b) {
    if (i == 0) {
        *a = n - 1;
        *b = round;
    } else {
        *a = (round + i) % (n - 1);
        *b = (round - i + n - 1) % (n - 1);
    }
}

__global__ void __launch_bounds__(256) k_jacobi_round(double* __restrict__ X, int ldx, int N, int nblk,
                                                      int round, double floor2,
                                                      unsigned long long* __restrict__ stat) {
    __shared__ double Gp[4][16][17];
    __shared__ double G[16][17];
    __shared__ double Q[16][17];
    __shared__ double cs[8][2];
    __shared__ double sweep_off;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    int I, J;
    pair_of(nblk, round, blockIdx.x, &I, &J);
    const int r = lane & 15, kg = lane >> 4;
    const int my_row = (r < 8) ? I * 8 + r : J * 8 + (r - 8);
    const double* __restrict__ xr = X + (size_t)my_row * ldx;

    // 1. Gram of the 16 columns: G = Xp Xp^T, K = N split over the 4 waves
    {
        const int nsteps = ldx / 4;                        // MFMA k-steps of 4 columns
        const int kq = (nsteps + 3) / 4;                   // per wave
        const int kb = wave * kq, ke = min(kb + kq, nsteps);
        d4 acc = {0, 0, 0, 0};
        for (int ks = kb; ks < ke; ++ks) {
            const double x = xr[ks * 4 + kg];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, x, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) Gp[wave][kg + 4 * v][r] = acc[v];   // FP64 MFMA result layout
    }
    __syncthreads();
    {
        const int a = tid >> 4, b = tid & 15;
        G[a][b] = ((Gp[0][a][b] + Gp[1][a][b]) + Gp[2][a][b]) + Gp[3][a][b];
        Q[a][b] = (a == b) ? 1.0 : 0.0;
    }
    __syncthreads();

    // 2. cyclic Jacobi on G (wave 0 only; LDS ops of one wave execute in order)
    if (wave == 0) {
        // coupling measure before rotation (for the sweep's convergence test)
        double off = 0.0;
        for (int e = lane; e < 256; e += 64) {
            const int a = e >> 4, b = e & 15;
            if (a < b) {
                const double gaa = G[a][a], gbb = G[b][b];
                if (gaa > floor2 && gbb > floor2) off = fmax(off, fabs(G[a][b]) / sqrt(gaa * gbb));
            }
        }
        for (int m = 32; m > 0; m >>= 1) off = fmax(off, __shfl_xor(off, m));
        if (lane == 0) sweep_off = off;
        for (int sw = 0; sw < 12; ++sw) {
            double mx = 0.0;
            for (int step = 0; step < 15; ++step) {
                // rotation parameters of the 8 disjoint pairs of this step
                if (lane < 8) {
                    int p, q;
                    if (lane == 0) { p = 15; q = step; }
                    else { p = (step + lane) % 15; q = (step - lane + 15) % 15; }
                    const double a = G[p][p], d = G[q][q], b = G[p][q];
                    double c = 1.0, s = 0.0;
                    if (a > floor2 && d > floor2) {
                        const double rel = fabs(b) / sqrt(a * d);
                        mx = fmax(mx, rel);
                        if (rel > 1e-16) {
                            const double th = (d - a) / (2.0 * b);
                            const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                            c = 1.0 / sqrt(t * t + 1.0);
                            s = t * c;
                        }
                    } else if (b != 0.0 && (a > floor2 || d > floor2)) {
                        const double th = (d - a) / (2.0 * b);
                        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        s = t * c;
                    }
                    cs[lane][0] = c;
                    cs[lane][1] = s;
                }
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                // rows: G <- J^T G  (2 tasks per lane: pair i = task/16, column k = task%16)
                for (int task = lane; task < 128; task += 64) {
                    const int i = task >> 4, k = task & 15;
                    int p, q;
                    if (i == 0) { p = 15; q = step; }
                    else { p = (step + i) % 15; q = (step - i + 15) % 15; }
                    const double c = cs[i][0], s = cs[i][1];
                    const double gp = G[p][k], gq = G[q][k];
                    G[p][k] = c * gp - s * gq;
                    G[q][k] = s * gp + c * gq;
                }
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                // columns: G <- G J, Q <- Q J
                for (int task = lane; task < 128; task += 64) {
                    const int i = task >> 4, k = task & 15;
                    int p, q;
                    if (i == 0) { p = 15; q = step; }
                    else { p = (step + i) % 15; q = (step - i + 15) % 15; }
                    const double c = cs[i][0], s = cs[i][1];
                    const double gp = G[k][p], gq = G[k][q];
                    G[k][p] = c * gp - s * gq;
                    G[k][q] = s * gp + c * gq;
                    const double qp = Q[k][p], qq = Q[k][q];
                    Q[k][p] = c * qp - s * qq;
                    Q[k][q] = s * qp + c * qq;
                }
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            }
            for (int m = 32; m > 0; m >>= 1) mx = fmax(mx, __shfl_xor(mx, m));
            if (mx <= 1e-15) break;
        }
    }
    __syncthreads();
    if (tid == 0) {
        const double off = sweep_off;
        unsigned long long bits;
        std::memcpy(&bits, &off, sizeof(bits));
        atomicMax(stat, bits);   // non-negative doubles order like their bit patterns
    }

    // 3. X_pair <- Q^T X_pair, 16-column tiles of N spread over the 4 waves
    const int ntile = ldx / 16 + ((ldx % 16) ? 1 : 0);
    for (int tl = wave; tl < ntile; tl += 4) {
        const int n0 = tl * 16;
        const int col = n0 + r;
        d4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int k0 = 0; k0 < 16; k0 += 4) {
            const int k = k0 + kg;
            const double a = Q[k][r];                        // (Q^T)[r][k]
            const int src_row = (k < 8) ? I * 8 + k : J * 8 + (k - 8);
            const double b = (col < ldx) ? X[(size_t)src_row * ldx + col] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
        // every lane has read its inputs for this tile before any lane writes (same wave)
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int orow = kg + 4 * v;                     // FP64 MFMA result layout
            const int dst_row = (orow < 8) ? I * 8 + orow : J * 8 + (orow - 8);
            if (col < ldx) X[(size_t)dst_row * ldx + col] = acc[v];
        }
    }
}

__global__ void __launch_bounds__(256) k_copy_rows_in(int D, int N, const double* __restrict__ A, int lda,
                                                      double* __restrict__ X, int ldx) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int row = blockIdx.y;
    if (i >= ldx) return;
    X[(size_t)row * ldx + i] = (row < D && i < N) ? A[(size_t)row * lda + i] : 0.0;
}

__global__ void __launch_bounds__(256) k_permute_rows(int ldx, const int32_t* __restrict__ perm,
                                                      const double* __restrict__ X,
                                                      double* __restrict__ Y, int ldy, int ncopy) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int row = blockIdx.y;
    if (i >= ncopy) return;
    Y[(size_t)row * ldy + i] = X[(size_t)perm[row] * ldx + i];
}

__global__ void __launch_bounds__(256) k_norms(int ldx, const double* __restrict__ X, double* __restrict__ nrm) {
    __shared__ double red[256];
    const double* x = X + (size_t)blockIdx.x * ldx;
    double acc = 0.0;
    for (int i = threadIdx.x; i < ldx; i += 256) acc += x[i] * x[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) nrm[blockIdx.x] = red[0];
}

inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

struct JacobiLayout {
    int Dp, ldx;
    size_t x_bytes, off_x2, off_nrm, off_perm, off_stat, total;
};

JacobiLayout layout(int D, int N) {
    JacobiLayout L{};
    L.Dp = std::max(16, (D + 15) / 16 * 16);
    L.ldx = (N + 15) / 16 * 16;
    L.x_bytes = (size_t)L.Dp * L.ldx * sizeof(double);
    L.off_x2 = L.x_bytes;
    L.off_nrm = 2 * L.x_bytes;
    L.off_perm = L.off_nrm + (size_t)L.Dp * sizeof(double);
    L.off_stat = (L.off_perm + (size_t)L.Dp * sizeof(int32_t) + 255) / 256 * 256;
    L.total = L.off_stat + 256;
    return L;
}

}  // namespace

size_t jacobi_work_bytes(int D, int N) { return layout(D, N).total; }

// Sorted norms: sigma2[j] for rows j of X, descending; perm[a] = row of the a-th largest.
static int sorted_norms(hipStream_t st, const JacobiLayout& L, double* X, char* base,
                        std::vector<double>& sig2, std::vector<int32_t>& perm) {
    double* nrm = (double*)(base + L.off_nrm);
    hipLaunchKernelGGL(k_norms, dim3(L.Dp), dim3(256), 0, st, L.ldx, X, nrm);
    sig2.resize(L.Dp);
    LSUM_HIP(hipMemcpyAsync(sig2.data(), nrm, L.Dp * sizeof(double), hipMemcpyDeviceToHost, st));
    LSUM_HIP(hipStreamSynchronize(st));
    perm.resize(L.Dp);
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return sig2[a] > sig2[b]; });
    return LSUM_OK;
}

int jacobi_svd(hipStream_t st, int D, int N, double* A, int lda, double tol, int max_sweeps,
               std::vector<double>& sigma, std::vector<int32_t>& order, int* sweeps_out,
               double* work_dev, size_t work_bytes) {
    if (D <= 0 || N <= 0) return fail(LSUM_E_INVALID, "empty side matrix");
    const JacobiLayout L = layout(D, N);
    if (work_bytes < L.total) return fail(LSUM_E_INVALID, "Jacobi workspace too small");
    char* base = (char*)work_dev;
    double* X = (double*)base;
    double* X2 = (double*)(base + L.off_x2);
    int32_t* perm_dev = (int32_t*)(base + L.off_perm);
    unsigned long long* stat = (unsigned long long*)(base + L.off_stat);
    const int nblk = L.Dp / 8;
    hipLaunchKernelGGL(k_copy_rows_in, dim3(cdiv(L.ldx, 256), L.Dp), dim3(256), 0, st, D, N, A, lda,
                       X, L.ldx);
    std::vector<double> sig2;
    std::vector<int32_t> perm;
    int rc = sorted_norms(st, L, X, base, sig2, perm);
    if (rc) return rc;
    const double total = std::accumulate(sig2.begin(), sig2.end(), 0.0);
    // columns whose squared norm is below this are exact zeros for every purpose downstream
    const double floor2 = std::max(total * 1e-60, 1e-300);
    int sweeps = 0;
    bool converged = false;
    for (; sweeps < max_sweeps && !converged; ++sweeps) {
        // sort the columns by norm so that blocks hold similar magnitudes
        LSUM_HIP(hipMemcpyAsync(perm_dev, perm.data(), L.Dp * sizeof(int32_t), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_permute_rows, dim3(cdiv(L.ldx, 256), L.Dp), dim3(256), 0, st, L.ldx,
                           perm_dev, X, X2, L.ldx, L.ldx);
        std::swap(X, X2);
        LSUM_HIP(hipMemsetAsync(stat, 0, sizeof(unsigned long long), st));
        for (int round = 0; round < nblk - 1; ++round)
            hipLaunchKernelGGL(k_jacobi_round, dim3(nblk / 2), dim3(256), 0, st, X, L.ldx, N, nblk,
                               round, floor2, stat);
        unsigned long long bits = 0;
        LSUM_HIP(hipMemcpyAsync(&bits, stat, sizeof(bits), hipMemcpyDeviceToHost, st));
        rc = sorted_norms(st, L, X, base, sig2, perm);   // synchronises
        if (rc) return rc;
        double off;
        std::memcpy(&off, &bits, sizeof(off));
        if (off <= tol) converged = true;
    }
    LSUM_HIP(hipGetLastError());
    // write back the D largest columns in descending order
    LSUM_HIP(hipMemcpyAsync(perm_dev, perm.data(), L.Dp * sizeof(int32_t), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_permute_rows, dim3(cdiv(N, 256), D), dim3(256), 0, st, L.ldx, perm_dev, X, A,
                       lda, N);
    LSUM_HIP(hipStreamSynchronize(st));
    sigma.resize(D);
    order.resize(D);
    for (int a = 0; a < D; ++a) {
        sigma[a] = std::sqrt(std::max(sig2[perm[a]], 0.0));
        order[a] = a;
    }
    *sweeps_out = sweeps;
    if (!converged) return fail(LSUM_E_NOCONV, "Jacobi SVD did not converge");
    return LSUM_OK;
}

}  // namespace lsum

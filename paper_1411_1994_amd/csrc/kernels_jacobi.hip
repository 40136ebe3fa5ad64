// One-sided block-Jacobi SVD (FP64) of a side matrix, for the truncated SVD of Def. def:RHOSVD.
//
// The D columns of the side matrix are the rows of X (length N).  A sweep visits every pair of
// column blocks once (circle-method round robin: nblk-1 rounds of nblk/2 disjoint pairs); blocks
// hold 8, 16 or 32 columns (the wider ones below: pair problems of 32 or 64 columns, half or a
// quarter of the rounds).  One round of 8-column blocks is three wide launches:
//   1. k_pair_gram:   16x16 Gram partials of every pair's 16 columns over chunks of 256 cells,
//                     on v_mfma_f64_16x16x4 (grid: chunks x pairs);
//   2. k_pair_eig:    per pair, the chunk partials are summed in a fixed order (256 threads), the
//                     coupling max |g_ij| / sqrt(g_ii g_jj) is measured and, unless the pair is
//                     already orthogonal, one or two sweeps of cyclic two-sided Jacobi on the Gram
//                     run in one wavefront (one when a round holds many pairs);
//   3. k_pair_rotate: X_pair <- Q^T X_pair over the same chunks, again on MFMA.
// Columns are never squared against each other globally, so singular values keep an absolute
// accuracy of a few eps * sigma_max -- the RHOSVD threshold at eps = 1e-6 sits near 1e-8 sigma_1,
// far below what a Gram-matrix eigensolver can resolve.  Pairs in which one column is below the
// caller's irrelevance floor are left alone: such a column cannot change the certified tail.
// Between sweeps the columns are re-sorted by norm so that blocks hold similar magnitudes, and
// once a sweep's couplings are small the rows' full Gram checks whether the next sweep would
// only confirm convergence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>

#include "lsum_internal.h"

namespace lsum {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int CW = 256;   // cells per chunk

__device__ __forceinline__ void pair_of(int n, int round, int i, int* a, int* b) {
    if (i == 0) {
        *a = n - 1;
        *b = round;
    } else {
        *a = (round + i) % (n - 1);
        *b = (round - i + n - 1) % (n - 1);
    }
}

__device__ __forceinline__ int pair_row(int I, int J, int k) { return k < 8 ? I * 8 + k : J * 8 + (k - 8); }

// 1. Gram partials: part[(pair * nchunk + chunk) * 256 + a*16 + b]
__global__ void __launch_bounds__(256) k_pair_gram(double* const* __restrict__ xp, int ldx, int n_gram, int nblk,
                                                   int round, int nchunk, double* __restrict__ part) {
    __shared__ double Gp[4][16][17];
    const double* __restrict__ X = xp[0];
    const int chunk = blockIdx.x, pair = blockIdx.y;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int r = lane & 15, kg = lane >> 4;
    int I, J;
    pair_of(nblk, round, pair, &I, &J);
    const double* __restrict__ xr = X + (size_t)pair_row(I, J, r) * ldx;
    const int c0 = chunk * CW + wave * (CW / 4);
    double x[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int c = c0 + 4 * s + kg;
        x[s] = c < n_gram ? xr[c] : 0.0;
    }
    d4 acc = {0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < 16; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x[s], x[s], acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) Gp[wave][kg + 4 * v][r] = acc[v];   // FP64 MFMA result layout
    __syncthreads();
    const int a = tid >> 4, b = tid & 15;
    part[((size_t)pair * nchunk + chunk) * 256 + a * 16 + b] =
        ((Gp[0][a][b] + Gp[1][a][b]) + Gp[2][a][b]) + Gp[3][a][b];
}

// 2. per-pair eigen-decomposition of the 16x16 Gram (one wavefront)
// A coupling g_ab is worth a rotation when both columns are relevant (norm^2 > irr2).
__device__ __forceinline__ bool coupled(double gaa, double gbb, double gab, double irr2) {
    return gaa > irr2 && gbb > irr2 && gab != 0.0;
}

// Round-robin pairing of the 16 columns for the 15 steps of an inner sweep: step t pairs
// (15, t) and ((t + i) % 15, (t - i + 15) % 15) for i = 1..7.  Computed in registers (a table in
// memory would cost a load round trip per step).
__device__ __forceinline__ int inner_p(int t, int i) { return i == 0 ? 15 : (t + i >= 15 ? t + i - 15 : t + i); }
__device__ __forceinline__ int inner_q(int t, int i) { return i == 0 ? t : (t - i < 0 ? t - i + 15 : t - i); }

// The rotation (c, s) that annihilates the coupling b of two columns with squared norms a and d,
// and the squared relative coupling b^2 / (a d) it removes (0 for a pair that is left alone).
__device__ __forceinline__ void rotation(double a, double d, double b, double irr2, double* c, double* s,
                                         double* rel2, double skip2 = 1e-32) {
    // computed without branches (every lane of the wavefront takes the same path) and selected
    // at the end: a pair left alone gets (1, 0)
    const bool cpl = coupled(a, d, b, irr2);
    // the coupling only steers decisions: an approximate reciprocal suffices
    const double r2 = (b * b) * __builtin_amdgcn_rcp(a * d);
    const bool go = cpl && r2 > skip2;
    // tan of the angle that annihilates b: t = 2b / (z + sign(z) sqrt(z^2 + 4 b^2)), z = d - a (the
    // smaller root, |t| <= 1).  t may be approximate (the rotation is then slightly short of
    // optimal but still orthogonal); c = (1 + t^2)^(-1/2) is refined to full precision so that
    // c^2 + s^2 = 1 to rounding.
    const double z = d - a;
    const double x = z * z + 4.0 * b * b;
    const double r = x * __builtin_amdgcn_rsq(x);
    const double t = 2.0 * b * __builtin_amdgcn_rcp(z >= 0.0 ? z + r : z - r);
    const double u = 1.0 + t * t;
    double y = __builtin_amdgcn_rsq(u);
    y = y * (1.5 - 0.5 * u * y * y);
    y = y * (1.5 - 0.5 * u * y * y);
    *c = go ? y : 1.0;
    *s = go ? t * y : 0.0;
    *rel2 = cpl ? r2 : 0.0;
}

constexpr int EIG_LOADS = 16;   // chunk partials in flight per thread

// The 16 x 16 pair problem in LDS, solved by the 64 lanes of one wavefront (lane = its index):
// the pair's coupling is recorded (stat[0]; stat[4]: the largest coupling among columns whose
// squared norms both exceed keep2) and, unless the pair is already orthogonal to tol, G and Q
// (entering as the identity) are updated by cyclic two-sided Jacobi.  Returns whether the pair
// is to be rotated.
__device__ __forceinline__ bool solve_pair(int lane, double (*G)[17], double (*Q)[17], double tol, double irr2, double keep2,
                           int max_inner, unsigned long long* __restrict__ stat) {
    // coupling of relevant pairs (both squared norms above the irrelevance floor)
    double off = 0.0, offk = 0.0;
    for (int e = lane; e < 256; e += 64) {
        const int a = e >> 4, b = e & 15;
        if (a < b) {
            const double gaa = G[a][a], gbb = G[b][b];
            if (coupled(gaa, gbb, G[a][b], irr2)) {
                // decisions only: the approximate reciprocal square root suffices
                const double cab = fabs(G[a][b]) * __builtin_amdgcn_rsq(gaa * gbb);
                off = fmax(off, cab);
                if (gaa > keep2 && gbb > keep2) offk = fmax(offk, cab);
            }
        }
    }
    for (int m = 32; m > 0; m >>= 1) {
        off = fmax(off, __shfl_xor(off, m));
        offk = fmax(offk, __shfl_xor(offk, m));
    }
    if (lane == 0) {
        unsigned long long bits;
        std::memcpy(&bits, &off, sizeof(bits));
        atomicMax(stat, bits);   // non-negative doubles order like their bit patterns
        std::memcpy(&bits, &offk, sizeof(bits));
        atomicMax(stat + 4, bits);
    }
    if (!(off > tol)) return false;
    // Each step applies 8 disjoint rotations at once: G <- J^T G J, Q <- Q J.  With the step's
    // pairing, index i of pair (p, q) maps to alpha_i row_i + beta_i row_partner, (alpha, beta) =
    // (c, -s) for p and (c, s) for q; lane (bi, bj) owns the 2x2 blocks {p_bi, q_bi} x {p_bj, q_bj}
    // of G and of Q, so it writes only its own entries.  It computes the rotations of pairs bi and
    // bj itself from the step's entering G (the same values on every lane that needs them): all
    // reads of a step precede its writes in the wavefront's program order.
    const int bi = lane >> 3, bj = lane & 7;
    double prev = 2.0;
    int nsw = 0;
    for (int sw = 0; sw < max_inner; ++sw) {
        nsw = sw + 1;
        double mx = 0.0;
        for (int step = 0; step < 15; ++step) {
            const int pi = inner_p(step, bi), qi = inner_q(step, bi);
            const int pj = inner_p(step, bj), qj = inner_q(step, bj);
            // every read of the step first (one LDS round trip), then the rotations
            const double gpp_i = G[pi][pi], gqq_i = G[qi][qi], gpq_i = G[pi][qi];
            const double gpp_j = G[pj][pj], gqq_j = G[qj][qj], gpq_j = G[pj][qj];
            // G block [pi qi] x [pj qj]
            const double g00 = G[pi][pj], g01 = G[pi][qj], g10 = G[qi][pj], g11 = G[qi][qj];
            const double q00 = Q[pi][pj], q01 = Q[pi][qj], q10 = Q[qi][pj], q11 = Q[qi][qj];
            double ci, si, cj, sj, ri, rj;
            rotation(gpp_i, gqq_i, gpq_i, irr2, &ci, &si, &ri);
            rotation(gpp_j, gqq_j, gpq_j, irr2, &cj, &sj, &rj);
            mx = fmax(mx, ri);
            // rows: J^T
            const double h00 = ci * g00 - si * g10, h01 = ci * g01 - si * g11;
            const double h10 = si * g00 + ci * g10, h11 = si * g01 + ci * g11;
            // columns: J
            G[pi][pj] = cj * h00 - sj * h01;
            G[pi][qj] = sj * h00 + cj * h01;
            G[qi][pj] = cj * h10 - sj * h11;
            G[qi][qj] = sj * h10 + cj * h11;
            // Q rows {pi, qi} (any row partition), columns {pj, qj}
            Q[pi][pj] = cj * q00 - sj * q01;
            Q[pi][qj] = sj * q00 + cj * q01;
            Q[qi][pj] = cj * q10 - sj * q11;
            Q[qi][qj] = sj * q10 + cj * q11;
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
        for (int m = 32; m > 0; m >>= 1) mx = fmax(mx, __shfl_xor(mx, m));
        mx = sqrt(mx);
        if (mx <= 1e-16) break;   // nothing above the noise was rotated in this sweep
        // cyclic Jacobi converges quadratically; a sweep that no longer reduces the largest
        // relative coupling is rotating rounding noise of the small columns (entries of G carry
        // errors of order eps * max_k g_kk after the first rotations), which later rounds of the
        // outer sweep resolve against columns of their own size
        if (sw >= 2 && mx > 0.9 * prev) break;
        prev = mx;
    }
    if (lane == 0) {   // inner sweep statistics: total, maximum, solved pairs
        atomicAdd(stat + 1, (unsigned long long)nsw);
        atomicMax(stat + 2, (unsigned long long)nsw);
        atomicAdd(stat + 3, 1ull);
    }
    return true;
}

// 256 threads sum the chunk partials (one Gram entry each); one wavefront then solves.
__global__ void __launch_bounds__(256) k_pair_eig(int nchunk, const double* __restrict__ part, double tol,
                                                  double irr2, const double* __restrict__ keep2p, int max_inner,
                                                  double* __restrict__ Qout,
                                                  int* __restrict__ active, unsigned long long* __restrict__ stat) {
    __shared__ double G[16][17];
    __shared__ double Q[16][17];
    const int pair = blockIdx.x, tid = threadIdx.x;
    const double keep2 = *keep2p;
    {
        // entry tid over the chunks in chunk order; the loads of a group are issued together so
        // that the sum waits on one memory latency per EIG_LOADS chunks (indices past the last
        // chunk repeat it and add 0)
        const double* __restrict__ pp = part + (size_t)pair * nchunk * 256 + tid;
        double s = 0.0;
        for (int c = 0; c < nchunk; c += EIG_LOADS) {
            double v[EIG_LOADS];
#pragma unroll
            for (int k = 0; k < EIG_LOADS; ++k) v[k] = pp[(size_t)min(c + k, nchunk - 1) * 256];
#pragma unroll
            for (int k = 0; k < EIG_LOADS; ++k) s += c + k < nchunk ? v[k] : 0.0;
        }
        G[tid >> 4][tid & 15] = s;
        Q[tid >> 4][tid & 15] = ((tid >> 4) == (tid & 15)) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (tid >= 64) return;   // the solve uses wavefront barriers only
    const bool act = solve_pair(tid, G, Q, tol, irr2, keep2, max_inner, stat);
    if (tid == 0) active[pair] = act ? 1 : 0;
    if (!act) return;
    for (int e = tid; e < 256; e += 64) Qout[(size_t)pair * 256 + e] = Q[e >> 4][e & 15];
}

// 3. rotation of the pair's 16 columns over one chunk: X_pair <- Q^T X_pair
__global__ void __launch_bounds__(256) k_pair_rotate(double* const* __restrict__ xp, int ldx, int nblk, int round,
                                                     const double* __restrict__ Qin,
                                                     const int* __restrict__ active) {
    const int chunk = blockIdx.x, pair = blockIdx.y;
    if (!active[pair]) return;
    double* __restrict__ X = xp[0];
    __shared__ double Q[16][17];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int r = lane & 15, kg = lane >> 4;
    Q[tid >> 4][tid & 15] = Qin[(size_t)pair * 256 + tid];
    __syncthreads();
    int I, J;
    pair_of(nblk, round, pair, &I, &J);
    const int c0 = chunk * CW + wave * (CW / 4);    // 64 cells = 4 tiles of 16 per wave
    double b[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int k0 = 0; k0 < 4; ++k0) {
            const int col = c0 + 16 * t + r;
            b[t][k0] = col < ldx ? X[(size_t)pair_row(I, J, 4 * k0 + kg) * ldx + col] : 0.0;
        }
    d4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        acc[t] = d4{0, 0, 0, 0};
#pragma unroll
        for (int k0 = 0; k0 < 4; ++k0)
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(Q[4 * k0 + kg][r], b[t][k0], acc[t], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int col = c0 + 16 * t + r;
        if (col < ldx) {
#pragma unroll
            for (int v = 0; v < 4; ++v)
                X[(size_t)pair_row(I, J, kg + 4 * v) * ldx + col] = acc[t][v];   // FP64 MFMA result layout
        }
    }
}

// ---- 16-column blocks: pairs of 32 rows, half the rounds per sweep --------------------------
// The same three launches per round on blocks of 16 columns: the 32 x 32 pair Gram (three
// 16 x 16 MFMA tiles per chunk, the fourth its transpose), the 32 x 32 pair solve by four
// waves, and the rotation of the pair's 32 rows.  A sweep has nblk - 1 rounds for nblk
// blocks, so doubling the block halves the rounds (and the launches) per sweep.

__device__ __forceinline__ int pair_row32(int I, int J, int k) { return k < 16 ? I * 16 + k : J * 16 + (k - 16); }

// 1. Gram partials: part[(pair * nchunk + chunk) * 1024 + a*32 + b]
__global__ void __launch_bounds__(256) k_pair_gram32(double* const* __restrict__ xp, int ldx, int n_gram, int nblk,
                                                     int round, int nchunk, double* __restrict__ part) {
    __shared__ double Gp[4][32][33];
    const double* __restrict__ X = xp[0];
    const int chunk = blockIdx.x, pair = blockIdx.y;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int r = lane & 15, kg = lane >> 4;
    int I, J;
    pair_of(nblk, round, pair, &I, &J);
    const double* __restrict__ x0r = X + (size_t)pair_row32(I, J, r) * ldx;
    const double* __restrict__ x1r = X + (size_t)pair_row32(I, J, 16 + r) * ldx;
    const int c0 = chunk * CW + wave * (CW / 4);
    double x0[16], x1[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int c = c0 + 4 * s + kg;
        x0[s] = c < n_gram ? x0r[c] : 0.0;
        x1[s] = c < n_gram ? x1r[c] : 0.0;
    }
    d4 a00 = {0, 0, 0, 0}, a01 = {0, 0, 0, 0}, a11 = {0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        a00 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0[s], x0[s], a00, 0, 0, 0);
        a01 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0[s], x1[s], a01, 0, 0, 0);
        a11 = __builtin_amdgcn_mfma_f64_16x16x4f64(x1[s], x1[s], a11, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {   // FP64 MFMA result layout: row kg + 4v, column r
        Gp[wave][kg + 4 * v][r] = a00[v];
        Gp[wave][kg + 4 * v][16 + r] = a01[v];
        Gp[wave][16 + r][kg + 4 * v] = a01[v];
        Gp[wave][16 + kg + 4 * v][16 + r] = a11[v];
    }
    __syncthreads();
    for (int e = tid; e < 1024; e += 256) {
        const int a = e >> 5, b = e & 31;
        part[((size_t)pair * nchunk + chunk) * 1024 + e] = ((Gp[0][a][b] + Gp[1][a][b]) + Gp[2][a][b]) + Gp[3][a][b];
    }
}

// Round-robin pairing of 32 columns for the 31 steps of an inner sweep: step t pairs (31, t)
// and ((t + i) % 31, (t - i + 31) % 31) for i = 1..15.
__device__ __forceinline__ int inner_p32(int t, int i) { return i == 0 ? 31 : (t + i >= 31 ? t + i - 31 : t + i); }
__device__ __forceinline__ int inner_q32(int t, int i) { return i == 0 ? t : (t - i < 0 ? t - i + 31 : t - i); }

// The 32 x 32 pair problem solved by the 256 threads of a workgroup: as solve_pair, with thread
// (bi, bj) = (tid / 16, tid % 16) owning the 2 x 2 blocks {p_bi, q_bi} x {p_bj, q_bj} of G and
// of Q in each step.  G alternates between two LDS copies (a step reads one and writes the
// other), so one barrier per step orders its reads before the next step's writes; Q is updated
// in place (a thread reads and writes only its own entries of it).  Returns whether the pair is
// to be rotated (the same value on every thread) and leaves the final G in G[cur].
// Each lane computes one rotation, that of pair bj (lanes 0..15 of every wavefront hold the 16
// rotations of the step); the rotation of pair bi is read from lane bi of the same wavefront
// (bi = 4 wave + lane / 16 < 16, and lane bi has bj = bi).  Rotations whose squared relative
// coupling is at most skip2 are not applied, and a step with none to apply is skipped whole:
// every wavefront computes the same 16 rotations from the same entries, so all of them take the
// same decision and the barrier stays uniform.
__device__ bool solve_pair32(int tid, double (*G)[32][33], double (*Q)[33], int* cur_out, double tol, double irr2,
                             double keep2, double skip2, int max_inner, unsigned long long* __restrict__ stat,
                             double* red) {
    const int lane = tid & 63, wave = tid >> 6;
    double off = 0.0, offk = 0.0;
    for (int e = tid; e < 1024; e += 256) {
        const int a = e >> 5, b = e & 31;
        if (a < b) {
            const double gaa = G[0][a][a], gbb = G[0][b][b], gab = G[0][a][b];
            if (coupled(gaa, gbb, gab, irr2)) {
                const double cab = fabs(gab) * __builtin_amdgcn_rsq(gaa * gbb);
                off = fmax(off, cab);
                if (gaa > keep2 && gbb > keep2) offk = fmax(offk, cab);
            }
        }
    }
    for (int m = 32; m > 0; m >>= 1) {
        off = fmax(off, __shfl_xor(off, m));
        offk = fmax(offk, __shfl_xor(offk, m));
    }
    if (lane == 0) {
        red[wave] = off;
        red[4 + wave] = offk;
    }
    __syncthreads();
    off = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    offk = fmax(fmax(red[4], red[5]), fmax(red[6], red[7]));
    if (tid == 0) {
        unsigned long long bits;
        std::memcpy(&bits, &off, sizeof(bits));
        atomicMax(stat, bits);   // non-negative doubles order like their bit patterns
        std::memcpy(&bits, &offk, sizeof(bits));
        atomicMax(stat + 4, bits);
    }
    *cur_out = 0;
    if (!(off > tol)) return false;
    const int bi = tid >> 4, bj = tid & 15;
    int cur = 0;
    double prev = 2.0;
    int nsw = 0, nrun = 0;
    for (int sw = 0; sw < max_inner; ++sw) {
        nsw = sw + 1;
        double mx = 0.0;
        for (int step = 0; step < 31; ++step) {
            const int pj = inner_p32(step, bj), qj = inner_q32(step, bj);
            const double (*Gc)[33] = G[cur];
            double cj, sj, rj;
            rotation(Gc[pj][pj], Gc[qj][qj], Gc[pj][qj], irr2, &cj, &sj, &rj, skip2);
            mx = fmax(mx, rj);
            if (__ballot(sj != 0.0) == 0ull) continue;   // no rotation of this step is applied
            ++nrun;
            const int pi = inner_p32(step, bi), qi = inner_q32(step, bi);
            double (*Gn)[33] = G[cur ^ 1];
            const double g00 = Gc[pi][pj], g01 = Gc[pi][qj], g10 = Gc[qi][pj], g11 = Gc[qi][qj];
            const double q00 = Q[pi][pj], q01 = Q[pi][qj], q10 = Q[qi][pj], q11 = Q[qi][qj];
            const double ci = __shfl(cj, bi), si = __shfl(sj, bi);
            const double h00 = ci * g00 - si * g10, h01 = ci * g01 - si * g11;
            const double h10 = si * g00 + ci * g10, h11 = si * g01 + ci * g11;
            Gn[pi][pj] = cj * h00 - sj * h01;
            Gn[pi][qj] = sj * h00 + cj * h01;
            Gn[qi][pj] = cj * h10 - sj * h11;
            Gn[qi][qj] = sj * h10 + cj * h11;
            Q[pi][pj] = cj * q00 - sj * q01;
            Q[pi][qj] = sj * q00 + cj * q01;
            Q[qi][pj] = cj * q10 - sj * q11;
            Q[qi][qj] = sj * q10 + cj * q11;
            __syncthreads();
            cur ^= 1;
        }
        for (int m = 32; m > 0; m >>= 1) mx = fmax(mx, __shfl_xor(mx, m));
        if (lane == 0) red[wave] = mx;
        __syncthreads();
        mx = sqrt(fmax(fmax(red[0], red[1]), fmax(red[2], red[3])));
        __syncthreads();   // red is reused
        if (mx <= 1e-16) break;
        if (sw >= 2 && mx > 0.9 * prev) break;
        prev = mx;
    }
    if (tid == 0) {   // inner sweep statistics: total, maximum, solved pairs; steps applied, steps visited
        atomicAdd(stat + 1, (unsigned long long)nsw);
        atomicMax(stat + 2, (unsigned long long)nsw);
        atomicAdd(stat + 3, 1ull);
        atomicAdd(stat + 5, (unsigned long long)nrun);
        atomicAdd(stat + 6, (unsigned long long)(31 * nsw));
    }
    *cur_out = cur;
    return true;
}

// 2. per pair: the chunk partials summed in chunk order (four entries per thread), then solved
__global__ void __launch_bounds__(256) k_pair_eig32(int nchunk, const double* __restrict__ part, double tol,
                                                    double irr2, double skip2, const double* __restrict__ keep2p,
                                                    int max_inner,
                                                    double* __restrict__ Qout, int* __restrict__ active,
                                                    unsigned long long* __restrict__ stat) {
    __shared__ double G[2][32][33];
    __shared__ double Q[32][33];
    __shared__ double red[8];
    // the pair solve is the latency chain of a round: its waves issue first on a shared SIMD
    __builtin_amdgcn_s_setprio(3);
    const int pair = blockIdx.x, tid = threadIdx.x;
    for (int u = 0; u < 4; ++u) {
        const int e = tid + 256 * u;
        const double* pp = part + (size_t)pair * nchunk * 1024 + e;
        double s = 0.0;
        for (int c = 0; c < nchunk; c += EIG_LOADS) {
            double v[EIG_LOADS];
#pragma unroll
            for (int k = 0; k < EIG_LOADS; ++k) v[k] = pp[(size_t)min(c + k, nchunk - 1) * 1024];
#pragma unroll
            for (int k = 0; k < EIG_LOADS; ++k) s += c + k < nchunk ? v[k] : 0.0;
        }
        G[0][e >> 5][e & 31] = s;
        Q[e >> 5][e & 31] = ((e >> 5) == (e & 31)) ? 1.0 : 0.0;
    }
    __syncthreads();
    int cur = 0;
    const bool act = solve_pair32(tid, G, Q, &cur, tol, irr2, *keep2p, skip2, max_inner, stat, red);
    if (tid == 0) active[pair] = act ? 1 : 0;
    if (!act) return;
    for (int e = tid; e < 1024; e += 256) Qout[(size_t)pair * 1024 + e] = Q[e >> 5][e & 31];
}

// 3. X_pair <- Q^T X_pair over one chunk of CWR32 cells: each wave a quarter of it x 32 rows
#ifndef LSUM_ROT32_CHUNK
#define LSUM_ROT32_CHUNK 128
#endif
constexpr int CWR32 = LSUM_ROT32_CHUNK;
__global__ void __launch_bounds__(256) k_pair_rotate32(double* const* __restrict__ xp, int ldx, int nblk, int round,
                                                       const double* __restrict__ Qin,
                                                       const int* __restrict__ active) {
    const int chunk = blockIdx.x, pair = blockIdx.y;
    if (!active[pair]) return;
    double* __restrict__ X = xp[0];
    __shared__ double Q[32][33];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int r = lane & 15, kg = lane >> 4;
    for (int e = tid; e < 1024; e += 256) Q[e >> 5][e & 31] = Qin[(size_t)pair * 1024 + e];
    __syncthreads();
    int I, J;
    pair_of(nblk, round, pair, &I, &J);
    constexpr int NT = CWR32 / 64;   // tiles of 16 cells per wave
    const int c0 = chunk * CWR32 + wave * (CWR32 / 4);
    double b[NT][8];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int k0 = 0; k0 < 8; ++k0) {
            const int col = c0 + 16 * t + r;
            b[t][k0] = col < ldx ? X[(size_t)pair_row32(I, J, 4 * k0 + kg) * ldx + col] : 0.0;
        }
    d4 acc[NT][2];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            acc[t][rt] = d4{0, 0, 0, 0};
#pragma unroll
            for (int k0 = 0; k0 < 8; ++k0)
                acc[t][rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(Q[4 * k0 + kg][16 * rt + r], b[t][k0], acc[t][rt],
                                                                   0, 0, 0);
        }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int col = c0 + 16 * t + r;
        if (col < ldx) {
#pragma unroll
            for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    X[(size_t)pair_row32(I, J, 16 * rt + kg + 4 * v) * ldx + col] = acc[t][rt][v];
        }
    }
}

// ---- 32-column blocks: pairs of 64 rows, a quarter of the rounds of 8-column blocks ----------
// The three launches of a round on blocks of 32 columns: the 64 x 64 pair Gram (ten 16 x 16
// MFMA tiles per chunk, the other six their transposes), the 64 x 64 pair solve by eight waves,
// and the rotation of the pair's 64 rows.  Every round still reads and writes each row once, so
// halving the rounds of a sweep halves the bytes a sweep moves.

__device__ __forceinline__ int pair_row64(int I, int J, int k) { return k < 32 ? I * 32 + k : J * 32 + (k - 32); }

// 1. Gram partials: part[(pair * nchunk + chunk) * 4096 + a*64 + b].  Each wave multiplies its
// quarter of the chunk for all ten tiles (row tiles ti <= tj); the quarters are then added in
// wave order ((w0 + w1) + w2) + w3 one tile at a time through LDS.
__global__ void __launch_bounds__(256) k_pair_gram64(double* const* __restrict__ xp, int ldx, int n_gram, int nblk,
                                                     int round, int nchunk, double* __restrict__ part) {
    __shared__ double Gp[4][16][17];
    const double* __restrict__ X = xp[0];
    const int chunk = blockIdx.x, pair = blockIdx.y;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int r = lane & 15, kg = lane >> 4;
    int I, J;
    pair_of(nblk, round, pair, &I, &J);
    const int c0 = chunk * CW + wave * (CW / 4);
    double x[4][16];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const double* __restrict__ xr = X + (size_t)pair_row64(I, J, 16 * t + r) * ldx;
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const int c = c0 + 4 * s + kg;
            x[t][s] = c < n_gram ? xr[c] : 0.0;
        }
    }
    d4 acc[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) acc[k] = d4{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        int k = 0;
#pragma unroll
        for (int ti = 0; ti < 4; ++ti)
#pragma unroll
            for (int tj = ti; tj < 4; ++tj, ++k)
                acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[ti][s], x[tj][s], acc[k], 0, 0, 0);
    }
    double* __restrict__ out = part + ((size_t)pair * nchunk + chunk) * 4096;
    int k = 0;
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
        for (int tj = ti; tj < 4; ++tj, ++k) {
#pragma unroll
            for (int v = 0; v < 4; ++v) Gp[wave][kg + 4 * v][r] = acc[k][v];   // FP64 MFMA result layout
            __syncthreads();
            {
                const int a = tid >> 4, b = tid & 15;
                const double g = ((Gp[0][a][b] + Gp[1][a][b]) + Gp[2][a][b]) + Gp[3][a][b];
                out[(16 * ti + a) * 64 + 16 * tj + b] = g;
                if (ti != tj) out[(16 * tj + b) * 64 + 16 * ti + a] = g;
            }
            __syncthreads();
        }
}

// Round-robin pairing of 64 columns for the 63 steps of an inner sweep: step t pairs (63, t)
// and ((t + i) % 63, (t - i + 63) % 63) for i = 1..31.
__device__ __forceinline__ int inner_p64(int t, int i) { return i == 0 ? 63 : (t + i >= 63 ? t + i - 63 : t + i); }
__device__ __forceinline__ int inner_q64(int t, int i) { return i == 0 ? t : (t - i < 0 ? t - i + 63 : t - i); }

#ifndef LSUM_EIG64_THREADS
#define LSUM_EIG64_THREADS 512
#endif
constexpr int E64T = LSUM_EIG64_THREADS;   // threads of the 64 x 64 pair solve (256, 512 or 1024)
constexpr int E64W = E64T / 64;            // its waves

// The 64 x 64 pair problem solved by the E64T threads of a workgroup, as solve_pair32 with
// 32 x 32 blocks of 2 x 2: with 512 threads, thread (i0, j) = (tid / 32, tid % 32) owns the
// blocks {p_bi, q_bi} x {p_j, q_j} for bi in {i0, i0 + 16} of G and of Q; with 256 threads,
// thread (i0, j0) = (tid / 16, tid % 16) owns those for bi in {i0, i0 + 16}, bj in {j0, j0 + 16}.
// Each lane computes the rotations of its pairs bj; those of i0 and i0 + 16 are read from lanes
// i0 and i0 + 16 of the same wavefront (which hold pairs i0 and i0 + 16).  Rotations whose
// squared relative coupling is at most skip2 are not applied, and a step with none left is
// skipped whole (every wavefront computes the same 32 rotations from the same entries).
__device__ bool solve_pair64(int tid, double (*G)[64][65], double (*Q)[65], int* cur_out, double tol, double irr2,
                             double keep2, double skip2, int max_inner, unsigned long long* __restrict__ stat,
                             double* red) {
    constexpr int NJ = E64T >= 512 ? 1 : 2;     // block columns per thread
    constexpr int NI = E64T == 1024 ? 1 : 2;    // block rows per thread
    const int lane = tid & 63, wave = tid >> 6;
    double off = 0.0, offk = 0.0;
    for (int e = tid; e < 4096; e += E64T) {
        const int a = e >> 6, b = e & 63;
        if (a < b) {
            const double gaa = G[0][a][a], gbb = G[0][b][b], gab = G[0][a][b];
            if (coupled(gaa, gbb, gab, irr2)) {
                const double cab = fabs(gab) * __builtin_amdgcn_rsq(gaa * gbb);
                off = fmax(off, cab);
                if (gaa > keep2 && gbb > keep2) offk = fmax(offk, cab);
            }
        }
    }
    for (int m = 32; m > 0; m >>= 1) {
        off = fmax(off, __shfl_xor(off, m));
        offk = fmax(offk, __shfl_xor(offk, m));
    }
    if (lane == 0) {
        red[wave] = off;
        red[16 + wave] = offk;
    }
    __syncthreads();
    off = 0.0;
    offk = 0.0;
    for (int w = 0; w < E64W; ++w) {
        off = fmax(off, red[w]);
        offk = fmax(offk, red[16 + w]);
    }
    if (tid == 0) {
        unsigned long long bits;
        std::memcpy(&bits, &off, sizeof(bits));
        atomicMax(stat, bits);   // non-negative doubles order like their bit patterns
        std::memcpy(&bits, &offk, sizeof(bits));
        atomicMax(stat + 4, bits);
    }
    *cur_out = 0;
    __syncthreads();   // red is reused below
    if (!(off > tol)) return false;
    const int i0 = NJ == 1 ? tid >> 5 : tid >> 4;
    const int j0 = NJ == 1 ? tid & 31 : tid & 15;
    int cur = 0;
    double prev = 2.0;
    int nsw = 0, nrun = 0;
    for (int sw = 0; sw < max_inner; ++sw) {
        nsw = sw + 1;
        double mx = 0.0;
        for (int step = 0; step < 63; ++step) {
            const double (*Gc)[65] = G[cur];
            int pj[NJ], qj[NJ];
            double cj[NJ], sj[NJ];
            bool any = false;
#pragma unroll
            for (int h = 0; h < NJ; ++h) {
                pj[h] = inner_p64(step, j0 + 16 * h);
                qj[h] = inner_q64(step, j0 + 16 * h);
                double rj;
                rotation(Gc[pj[h]][pj[h]], Gc[qj[h]][qj[h]], Gc[pj[h]][qj[h]], irr2, &cj[h], &sj[h], &rj, skip2);
                mx = fmax(mx, rj);
                any = any || sj[h] != 0.0;
            }
            if (__ballot(any) == 0ull) continue;   // no rotation of this step is applied
            ++nrun;
            double (*Gn)[65] = G[cur ^ 1];
#pragma unroll
            for (int hi = 0; hi < NI; ++hi) {
                const int bi = i0 + 16 * hi;
                const int pi = inner_p64(step, bi), qi = inner_q64(step, bi);
                // pair bi's rotation, from the lane that computed it: with one block column per
                // thread lane bi holds pair bi; with two, lane i0 holds pairs i0 and i0 + 16
                const double ci = NJ == 1 ? __shfl(cj[0], bi) : __shfl(cj[hi], i0);
                const double si = NJ == 1 ? __shfl(sj[0], bi) : __shfl(sj[hi], i0);
#pragma unroll
                for (int h = 0; h < NJ; ++h) {
                    const double g00 = Gc[pi][pj[h]], g01 = Gc[pi][qj[h]], g10 = Gc[qi][pj[h]], g11 = Gc[qi][qj[h]];
                    const double q00 = Q[pi][pj[h]], q01 = Q[pi][qj[h]], q10 = Q[qi][pj[h]], q11 = Q[qi][qj[h]];
                    const double c = cj[h], s = sj[h];
                    const double h00 = ci * g00 - si * g10, h01 = ci * g01 - si * g11;
                    const double h10 = si * g00 + ci * g10, h11 = si * g01 + ci * g11;
                    Gn[pi][pj[h]] = c * h00 - s * h01;
                    Gn[pi][qj[h]] = s * h00 + c * h01;
                    Gn[qi][pj[h]] = c * h10 - s * h11;
                    Gn[qi][qj[h]] = s * h10 + c * h11;
                    Q[pi][pj[h]] = c * q00 - s * q01;
                    Q[pi][qj[h]] = s * q00 + c * q01;
                    Q[qi][pj[h]] = c * q10 - s * q11;
                    Q[qi][qj[h]] = s * q10 + c * q11;
                }
            }
            __syncthreads();
            cur ^= 1;
        }
        for (int m = 32; m > 0; m >>= 1) mx = fmax(mx, __shfl_xor(mx, m));
        if (lane == 0) red[wave] = mx;
        __syncthreads();
        mx = 0.0;
        for (int w = 0; w < E64W; ++w) mx = fmax(mx, red[w]);
        mx = sqrt(mx);
        __syncthreads();   // red is reused
        if (mx <= 1e-16) break;
        if (sw >= 2 && mx > 0.9 * prev) break;
        prev = mx;
    }
    if (tid == 0) {   // inner sweep statistics: total, maximum, solved pairs; steps applied, steps visited
        atomicAdd(stat + 1, (unsigned long long)nsw);
        atomicMax(stat + 2, (unsigned long long)nsw);
        atomicAdd(stat + 3, 1ull);
        atomicAdd(stat + 5, (unsigned long long)nrun);
        atomicAdd(stat + 6, (unsigned long long)(63 * nsw));
    }
    *cur_out = cur;
    return true;
}

// 2. per pair: the chunk partials summed in chunk order (4096 / E64T entries per thread, four
// chunks of them in flight at a time), then solved
__global__ void __launch_bounds__(E64T) k_pair_eig64(int nchunk, const double* __restrict__ part, double tol,
                                                     double irr2, double skip2, const double* __restrict__ keep2p,
                                                     int max_inner, double* __restrict__ Qout,
                                                     int* __restrict__ active, unsigned long long* __restrict__ stat) {
    constexpr int NE = 4096 / E64T;
    __shared__ double G[2][64][65];
    __shared__ double Q[64][65];
    __shared__ double red[32];
    // the pair solve is the latency chain of a round: its waves issue first on a shared SIMD
    __builtin_amdgcn_s_setprio(3);
    const int pair = blockIdx.x, tid = threadIdx.x;
    const double* pp = part + (size_t)pair * nchunk * 4096 + tid;
    double s[NE];
#pragma unroll
    for (int u = 0; u < NE; ++u) s[u] = 0.0;
    for (int c = 0; c < nchunk; c += 4) {
        double v[4][NE];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int u = 0; u < NE; ++u) v[k][u] = pp[(size_t)min(c + k, nchunk - 1) * 4096 + E64T * u];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int u = 0; u < NE; ++u) s[u] += c + k < nchunk ? v[k][u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < NE; ++u) {
        const int e = tid + E64T * u;
        G[0][e >> 6][e & 63] = s[u];
        Q[e >> 6][e & 63] = ((e >> 6) == (e & 63)) ? 1.0 : 0.0;
    }
    __syncthreads();
    int cur = 0;
    const bool act = solve_pair64(tid, G, Q, &cur, tol, irr2, *keep2p, skip2, max_inner, stat, red);
    if (tid == 0) active[pair] = act ? 1 : 0;
    if (!act) return;
    for (int e = tid; e < 4096; e += E64T) Qout[(size_t)pair * 4096 + e] = Q[e >> 6][e & 63];
}

// 3. X_pair <- Q^T X_pair over one chunk of CWR64 cells: each wave 32 cells (2 tiles of 16) x 64
// rows (chunks of 128 cells: twice the work-groups of 256-cell chunks, one pass per wave)
#ifndef LSUM_ROT64_CHUNK
#define LSUM_ROT64_CHUNK 128
#endif
constexpr int CWR64 = LSUM_ROT64_CHUNK;
__global__ void __launch_bounds__(256) k_pair_rotate64(double* const* __restrict__ xp, int ldx, int nblk, int round,
                                                       const double* __restrict__ Qin,
                                                       const int* __restrict__ active) {
    const int chunk = blockIdx.x, pair = blockIdx.y;
    if (!active[pair]) return;
    double* __restrict__ X = xp[0];
    __shared__ double Q[64][65];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int r = lane & 15, kg = lane >> 4;
    for (int e = tid; e < 4096; e += 256) Q[e >> 6][e & 63] = Qin[(size_t)pair * 4096 + e];
    __syncthreads();
    int I, J;
    pair_of(nblk, round, pair, &I, &J);
#pragma unroll 1
    for (int half = 0; half < CWR64 / 128; ++half) {
        const int c0 = chunk * CWR64 + wave * (CWR64 / 4) + 32 * half;
        double b[2][16];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int k0 = 0; k0 < 16; ++k0) {
                const int col = c0 + 16 * t + r;
                b[t][k0] = col < ldx ? X[(size_t)pair_row64(I, J, 4 * k0 + kg) * ldx + col] : 0.0;
            }
        d4 acc[2][4];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
                acc[t][rt] = d4{0, 0, 0, 0};
#pragma unroll
                for (int k0 = 0; k0 < 16; ++k0)
                    acc[t][rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(Q[4 * k0 + kg][16 * rt + r], b[t][k0],
                                                                       acc[t][rt], 0, 0, 0);
            }
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int col = c0 + 16 * t + r;
            if (col < ldx) {
#pragma unroll
                for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        X[(size_t)pair_row64(I, J, 16 * rt + kg + 4 * v) * ldx + col] = acc[t][rt][v];
            }
        }
    }
}

// A whole sweep in one launch: workgroup p owns pair slot p of every round of the round robin.
// A round on blocks (I, J) starts once both blocks have finished the previous round (their
// version counters, set with release order after the rows are written; read with acquire
// order), so no launch boundary separates the rounds.  Per pair the steps are those of the
// three-kernel round, in the same arithmetic order: the 16 x 16 Gram over chunks of CW cells
// (per chunk the four waves' MFMA partials ((w0 + w1) + w2) + w3, the chunks summed in order),
// the pair solve, and the rotation of the pair's rows chunk by chunk.  Every wait is bounded by
// tick_limit ticks of the constant-rate wall clock: a group that runs out raises the abort
// flag, and every group leaves at its next wait once the flag is up.  A group rotates only
// pairs it has started, so an aborted sweep leaves the rows an orthogonal transform of the
// input.
// A pair group of WAVES waves takes WAVES / 4 chunks of CW cells at a time (16 waves: one group
// fills a compute unit and has four chunks in flight; 4 waves: four groups share a compute unit,
// which is easier to place next to other work).  Both add the chunk partials in chunk order.
template <int WAVES>
__global__ void __launch_bounds__(WAVES * 64) k_jacobi_sweep(double* const* __restrict__ xp, int ldx, int n_gram,
                                                      int nblk, int nchunk, int nchunk_all, double tol, double irr2,
                                                      const double* __restrict__ keep2p, int max_inner,
                                                      unsigned long long* __restrict__ stat, int* __restrict__ ver,
                                                      int* __restrict__ abort_flag, long long tick_limit) {
    constexpr int CPS = WAVES / 4;   // chunks per step
    __shared__ double Gp[WAVES][16][17];
    __shared__ double G[16][17];
    __shared__ double Q[16][17];
    __shared__ int sh_go, sh_act;
    const int p = blockIdx.x;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int r = lane & 15, kg = lane >> 4;
    const int ga = (tid >> 4) & 15, gb = tid & 15;
    const int sub = wave >> 2, quarter = wave & 3;   // chunk within a step, quarter of it
    double* X = xp[0];   // not restrict: other groups write its rows between the rounds
    const double keep2 = *keep2p;
    const long long t0 = (long long)wall_clock64();
    for (int round = 0; round < nblk - 1; ++round) {
        int I, J;
        pair_of(nblk, round, p, &I, &J);
        if (tid == 0) {
            int go = 1;
            for (;;) {
                // relaxed polling; one acquire fence once both counters are there
                const int vi = __hip_atomic_load(ver + I, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const int vj = __hip_atomic_load(ver + J, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (vi >= round && vj >= round) {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    break;
                }
                if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                    go = 0;
                    break;
                }
                if ((long long)wall_clock64() - t0 > tick_limit) {
                    __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    go = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            sh_go = go;
        }
        __syncthreads();
        if (!sh_go) return;   // the same value on every thread
        // the rows other groups wrote: thread 0's acquire fence above invalidated this compute
        // unit's caches; the barrier orders every wave's loads after it
        // 1. the pair's Gram: wave (sub, quarter) takes quarter `quarter` of chunk step + sub
        const double* xr = X + (size_t)pair_row(I, J, r) * ldx;
        double gsum = 0.0;
        for (int step = 0; step < nchunk; step += CPS) {
            const int c0 = (step + sub) * CW + quarter * (CW / 4);
            double x[16];
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) {
                const int c = c0 + 4 * s2 + kg;
                x[s2] = c < n_gram ? xr[c] : 0.0;
            }
            d4 acc = {0, 0, 0, 0};
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x[s2], x[s2], acc, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 4; ++v) Gp[wave][kg + 4 * v][r] = acc[v];
            __syncthreads();
            if (tid < 256)
                for (int cc = 0; cc < CPS && step + cc < nchunk; ++cc)
                    gsum += ((Gp[4 * cc][ga][gb] + Gp[4 * cc + 1][ga][gb]) + Gp[4 * cc + 2][ga][gb]) +
                            Gp[4 * cc + 3][ga][gb];
            __syncthreads();
        }
        if (tid < 256) {
            G[ga][gb] = gsum;
            Q[ga][gb] = ga == gb ? 1.0 : 0.0;
        }
        __syncthreads();
        // 2. the pair solve (one wavefront)
        if (tid < 64) {
            const bool act = solve_pair(tid, G, Q, tol, irr2, keep2, max_inner, stat);
            if (tid == 0) sh_act = act ? 1 : 0;
        }
        __syncthreads();
        // 3. X_pair <- Q^T X_pair, four chunks at a time (each wave owns 64 cells of one)
        if (sh_act) {
            for (int step = 0; step < nchunk_all; step += CPS) {
                const int c0 = (step + sub) * CW + quarter * (CW / 4);
                double b[4][4];
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int k0 = 0; k0 < 4; ++k0) {
                        const int col = c0 + 16 * t + r;
                        b[t][k0] = col < ldx ? X[(size_t)pair_row(I, J, 4 * k0 + kg) * ldx + col] : 0.0;
                    }
                d4 acc[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    acc[t] = d4{0, 0, 0, 0};
#pragma unroll
                    for (int k0 = 0; k0 < 4; ++k0)
                        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(Q[4 * k0 + kg][r], b[t][k0], acc[t], 0, 0, 0);
                }
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int col = c0 + 16 * t + r;
                    if (col < ldx) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) X[(size_t)pair_row(I, J, kg + 4 * v) * ldx + col] = acc[t][v];
                    }
                }
            }
        }
        // 4. publish: every wave's row stores complete (workgroup-scope release), then one
        // agent-scope release by thread 0 makes them visible before the blocks' versions move on
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        if (tid == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_store(ver + I, round + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(ver + J, round + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Sweep prologue and epilogue on the current / other buffer pair xp = {current, other}: rows of
// the current buffer permuted into the other; then the pair swapped and the sweep statistics
// cleared (one thread; a kernel, not a memset, so that a captured sweep holds no memset node);
// after the rounds, the squared norms of the current rows.
__global__ void __launch_bounds__(256) k_permute_xp(int ldx, const int32_t* __restrict__ perm,
                                                    double* const* __restrict__ xp) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int row = blockIdx.y;
    if (i >= ldx) return;
    const double* __restrict__ X = xp[0];
    double* __restrict__ Y = xp[1];
    Y[(size_t)row * ldx + i] = X[(size_t)perm[row] * ldx + i];
}

__global__ void k_swap_clear(double** __restrict__ xp, unsigned long long* __restrict__ stat, int* __restrict__ ver,
                             int n_ver) {
    if (blockIdx.x != 0) return;
    if (threadIdx.x == 0) {
        double* t = xp[0];
        xp[0] = xp[1];
        xp[1] = t;
        for (int k = 0; k < 7; ++k) stat[k] = 0ull;
    }
    for (int k = threadIdx.x; k <= n_ver; k += blockDim.x) ver[k] = 0;   // versions, then the abort flag
}

// The largest relative coupling |g_ab| / sqrt(g_aa g_bb) over the pairs a < b of the n x n Gram G
// (row stride ldg) whose squared norms both exceed irr2 (out[0]), and over those whose squared
// norms both exceed keep2 (out[1]), as the bit patterns of non-negative doubles (out zeroed
// before).  The same test as the pair solves' coupling pass, on all pairs at once.
__global__ void __launch_bounds__(256) k_gram_coupling(int n, const double* __restrict__ G, long ldg, double irr2,
                                                       double keep2, unsigned long long* __restrict__ out) {
    __shared__ double red[2][4];
    const int b = blockIdx.x * 256 + threadIdx.x, a = blockIdx.y;
    double off = 0.0, offk = 0.0;
    if (a < b && b < n) {
        const double gaa = G[(size_t)a * ldg + a], gbb = G[(size_t)b * ldg + b], gab = G[(size_t)a * ldg + b];
        if (coupled(gaa, gbb, gab, irr2)) {
            const double cab = fabs(gab) / sqrt(gaa * gbb);
            off = cab;
            if (gaa > keep2 && gbb > keep2) offk = cab;
        }
    }
    for (int m = 32; m > 0; m >>= 1) {
        off = fmax(off, __shfl_xor(off, m));
        offk = fmax(offk, __shfl_xor(offk, m));
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wave] = off;
        red[1][wave] = offk;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        off = fmax(fmax(red[0][0], red[0][1]), fmax(red[0][2], red[0][3]));
        offk = fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3]));
        unsigned long long bits;
        std::memcpy(&bits, &off, sizeof(bits));
        atomicMax(out, bits);
        std::memcpy(&bits, &offk, sizeof(bits));
        atomicMax(out + 1, bits);
    }
}

__global__ void k_zero_u64(unsigned long long* __restrict__ p, int n) {
    for (int k = threadIdx.x; k < n; k += blockDim.x) p[k] = 0ull;
}

__global__ void __launch_bounds__(256) k_norms_xp(int ldx, int n_gram, double* const* __restrict__ xp,
                                                  double* __restrict__ nrm) {
    __shared__ double red[256];
    const double* x = xp[0] + (size_t)blockIdx.x * ldx;
    double acc = 0.0;
    for (int i = threadIdx.x; i < n_gram; i += 256) acc += x[i] * x[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) nrm[blockIdx.x] = red[0];
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

__global__ void __launch_bounds__(256) k_norms(int ldx, int n_gram, const double* __restrict__ X,
                                               double* __restrict__ nrm) {
    __shared__ double red[256];
    const double* x = X + (size_t)blockIdx.x * ldx;
    double acc = 0.0;
    for (int i = threadIdx.x; i < n_gram; i += 256) acc += x[i] * x[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) nrm[blockIdx.x] = red[0];
}

// Random signs for the range sketch: out[i] = +-1 from the SplitMix64 output function of
// seed + (i + 1) * golden-ratio increment (Steele, Lea, Flood 2014).
__global__ void __launch_bounds__(256) k_random_signs(long n, unsigned long long seed, double* __restrict__ out) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    unsigned long long z = seed + (unsigned long long)(i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    out[i] = (z & 1ull) ? 1.0 : -1.0;
}

// Rank-revealing Cholesky of a Gram matrix, in one workgroup (the orthonormalisation of a block
// of sketch rows: Y_p = R^T Q_b with Q_b orthonormal, Q_b = R^{-T} Y_p).  Right-looking: at step
// j the largest diagonal entry not yet pivoted (ties: the lowest index; without `pivot`, index j)
// is the j-th pivot p, R's row j is A's row p times 1 / sqrt(A_pp) (0 at earlier pivots), and
// A loses the outer product of that row.  A (n <= PC_MAXN) is held in registers, a 4 x 4 tile
// per thread, and updated whole (rows and columns of earlier pivots then only change by rounding
// and are never read again), so a step is two barriers and sixteen fused multiply-adds per
// thread.  The factorisation stops at the first pivot <= tau2 times the first.  Out: R^T in
// pivot order (Rt[jj][k] = R[k][pivot jj], k <= jj < keep), the pivot order (the unpivoted
// indices follow in increasing order) and keep.
#ifndef LSUM_PCHOL_THREADS
#define LSUM_PCHOL_THREADS 1024
#endif
constexpr int PC_THREADS = LSUM_PCHOL_THREADS;          // 1024 (tiles of 4 x 4) or 256 (8 x 8)
constexpr int PC_MAXN = 128;
constexpr int PC_SIDE = PC_THREADS == 1024 ? 32 : 16;    // threads per side of the tile grid
constexpr int PC_TT = PC_MAXN / PC_SIDE;                 // tile edge

__global__ void __launch_bounds__(PC_THREADS) k_pchol(int n, const double* __restrict__ A, double tau2, int pivot,
                                                      double* __restrict__ Rt, int* __restrict__ perm_out,
                                                      int* __restrict__ keep_dev) {
    __shared__ double Rr[PC_MAXN][PC_MAXN + 1];   // R's row j by original index
    __shared__ double diag[PC_MAXN];
    __shared__ double row[PC_MAXN];
    __shared__ int piv[PC_MAXN];
    __shared__ int done[PC_MAXN];
    const int tid = threadIdx.x, lane = tid & 63;
    const int i0 = (tid / PC_SIDE) * PC_TT, k0 = (tid % PC_SIDE) * PC_TT;   // this thread's tile
    double a[PC_TT][PC_TT];
#pragma unroll
    for (int u = 0; u < PC_TT; ++u)
#pragma unroll
        for (int v = 0; v < PC_TT; ++v)
            a[u][v] = (i0 + u < n && k0 + v < n) ? A[(size_t)(i0 + u) * n + k0 + v] : 0.0;
    if (tid < PC_MAXN) done[tid] = tid < n ? 0 : 1;
    if (i0 == k0)
#pragma unroll
        for (int u = 0; u < PC_TT; ++u) diag[i0 + u] = a[u][u];
    __syncthreads();
    double d0 = 0.0;
    int keep = n;
    for (int j = 0; j < n; ++j) {
        // the pivot, found by every wave alike from the same diagonal: the largest of the keys
        // (positive entry's bits with the low 7 bits replaced by 127 - index; 0 for entries
        // already pivoted or not positive), so values equal to within 2^-45 relative tie and
        // the lowest index wins
        int p = j;
        if (pivot) {
            unsigned long long key = 0;
            for (int i = lane; i < PC_MAXN; i += 64) {
                const double v = diag[i];
                unsigned long long bits;
                __builtin_memcpy(&bits, &v, sizeof(bits));
                const unsigned long long ki =
                    (!done[i] && v > 0.0) ? ((bits & ~0x7Full) | (unsigned long long)(PC_MAXN - 1 - i)) : 0ull;
                key = ki > key ? ki : key;
            }
            for (int off = 32; off > 0; off >>= 1) {
                const unsigned long long o = __shfl_xor(key, off);
                key = o > key ? o : key;
            }
            p = key ? PC_MAXN - 1 - (int)(key & 0x7F) : PC_MAXN;
        }
        const double d = p < n ? diag[p] : 0.0;   // no candidate left: stop
        if (j == 0) d0 = d;
        if (!(d > 0.0) || !(d > tau2 * d0)) {   // the same value on every thread: a uniform exit
            keep = j;
            break;
        }
        const double rjj = sqrt(d);
        if (i0 == p - p % PC_TT) {   // the threads holding row p
            const int u = p % PC_TT;
            const double inv = 1.0 / rjj;
#pragma unroll
            for (int v = 0; v < PC_TT; ++v) {
                const int k = k0 + v;
                double av = a[0][v];   // a[u][v] by selects (a dynamic index would send a to scratch)
#pragma unroll
                for (int uu = 1; uu < PC_TT; ++uu) av = uu == u ? a[uu][v] : av;
                row[k] = k == p ? rjj : (done[k] ? 0.0 : av * inv);
            }
        }
        __syncthreads();   // row j of R is complete; every wave has read diag and done
        if (tid == 0) {
            done[p] = 1;
            piv[j] = p;
        }
        if (tid < PC_MAXN) Rr[j][tid] = row[tid];
        double ri[PC_TT], rk[PC_TT];
#pragma unroll
        for (int u = 0; u < PC_TT; ++u) ri[u] = row[i0 + u];
#pragma unroll
        for (int v = 0; v < PC_TT; ++v) rk[v] = row[k0 + v];
#pragma unroll
        for (int u = 0; u < PC_TT; ++u)
#pragma unroll
            for (int v = 0; v < PC_TT; ++v) a[u][v] -= ri[u] * rk[v];
        if (i0 == k0)
#pragma unroll
            for (int u = 0; u < PC_TT; ++u) diag[i0 + u] = a[u][u];
        __syncthreads();   // diag and done for the next step; row free again
    }
    __syncthreads();
    for (int e = tid; e < keep * keep; e += PC_THREADS) {
        const int jj = e / keep, k = e % keep;
        if (k <= jj) Rt[(size_t)jj * n + k] = Rr[k][piv[jj]];
    }
    if (tid == 0) {
        for (int j = 0; j < keep; ++j) perm_out[j] = piv[j];
        int pos = keep;
        for (int i = 0; i < n; ++i)
            if (!done[i]) perm_out[pos++] = i;
        *keep_dev = keep;
    }
}

// Forward substitution R^T Q = Y_p for the kept rows (the rows of Y in pivot order): Q[i][c] =
// (Y[perm[i]][c] - sum_{k<i} R[k][i] Q[k][c]) / R[i][i], each column c by its own lane of the
// first wave.  The workgroup first loads R^T's lower triangle (packed by rows) and its 64
// columns of Y_p into LDS.  Rows are then solved 16 at a time: all earlier rows are subtracted
// from the 16 right-hand sides at once (16 independent sums, so the LDS reads overlap), then the
// 16 x 16 triangle is solved in registers.
constexpr int TS_MAXK = 128;
constexpr int TS_COLS = 64;
constexpr int TS_BLK = 16;

__device__ __forceinline__ int tri(int i) { return i * (i + 1) / 2; }

__global__ void __launch_bounds__(256) k_trsm_rows(int keep, int ncol, int n, const double* __restrict__ Rt,
                                                   const int* __restrict__ perm, const double* __restrict__ Y,
                                                   long ldy, double* __restrict__ out, long ldo) {
    __shared__ double rl[TS_MAXK * (TS_MAXK + 1) / 2];
    __shared__ double q[TS_MAXK][TS_COLS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col = blockIdx.x * TS_COLS + lane;
    // R^T's lower triangle: eight loads in flight per thread (indices past the end repeat the
    // last entry and are not stored)
    const int kk = keep * keep;
    for (int e0 = tid; e0 < kk; e0 += 256 * 8) {
        double v[8];
        int dst[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = min(e0 + 256 * u, kk - 1);
            const int i = e / keep, k = e - i * keep;
            v[u] = Rt[(size_t)i * n + k];
            dst[u] = (e0 + 256 * u < kk && k <= i) ? tri(i) + k : -1;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (dst[u] >= 0) rl[dst[u]] = v[u];
    }
    // the right-hand sides: eight rows per wave in flight (indices past keep repeat the last row
    // and are not stored)
    for (int i0 = wave; i0 < keep; i0 += 32) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = min(i0 + 4 * u, keep - 1);
            v[u] = col < ncol ? Y[(size_t)perm[i] * ldy + col] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (i0 + 4 * u < keep) q[i0 + 4 * u][lane] = v[u];
    }
    __syncthreads();
    if (wave == 0) {
        for (int b0 = 0; b0 < keep; b0 += TS_BLK) {
            // a block's rows past keep (indices below TS_MAXK, inside both LDS arrays) are
            // computed from unset entries and discarded: no branch separates the 16 sums
            double x[TS_BLK];
            const double* rrow[TS_BLK];
#pragma unroll
            for (int r = 0; r < TS_BLK; ++r) {
                x[r] = q[b0 + r][lane];
                rrow[r] = rl + tri(b0 + r);
            }
            for (int k = 0; k < b0; ++k) {
                const double qk = q[k][lane];
#pragma unroll
                for (int r = 0; r < TS_BLK; ++r) x[r] -= rrow[r][k] * qk;
            }
#pragma unroll
            for (int r = 0; r < TS_BLK; ++r) {
#pragma unroll
                for (int rr = 0; rr < r; ++rr) x[r] -= rrow[r][b0 + rr] * x[rr];
                x[r] /= rrow[r][b0 + r];
            }
#pragma unroll
            for (int r = 0; r < TS_BLK; ++r)
                if (b0 + r < keep) q[b0 + r][lane] = x[r];
        }
    }
    __syncthreads();
    for (int i = wave; i < keep; i += 4)
        if (col < ncol) out[(size_t)i * ldo + col] = q[i][lane];
}

inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

struct JacobiLayout {
    int Dp, ldx, nblk, npair, nchunk;   // nchunk: Gram chunks (over the first n_gram entries)
    int nchunk_all;                      // rotation chunks (whole rows)
    size_t off_x2, off_nrm, off_perm, off_stat, off_part, off_q, off_act, off_ptr, off_ver, total;
};

// bw: columns per block (8, 16 for pairs of 32 rows, 32 for pairs of 64); rows are padded to whole
// block pairs
JacobiLayout layout(int D, int N, int n_gram, int bw = 8) {
    JacobiLayout L{};
    L.Dp = std::max(2 * bw, (D + 2 * bw - 1) / (2 * bw) * (2 * bw));
    L.ldx = (N + 15) / 16 * 16;
    L.nblk = L.Dp / bw;
    L.npair = L.nblk / 2;
    L.nchunk = (n_gram + CW - 1) / CW;
    L.nchunk_all = (L.ldx + CW - 1) / CW;
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t xb = al((size_t)L.Dp * L.ldx * sizeof(double));
    L.off_x2 = xb;
    L.off_nrm = 2 * xb;
    L.off_perm = al(L.off_nrm + (size_t)L.Dp * sizeof(double));
    L.off_stat = al(L.off_perm + (size_t)L.Dp * sizeof(int32_t));
    L.off_part = al(L.off_stat + 64);
    const size_t pe = (size_t)4 * bw * bw;   // entries of a pair's Gram
    L.off_q = al(L.off_part + (size_t)L.npair * L.nchunk * pe * sizeof(double));
    L.off_act = al(L.off_q + (size_t)L.npair * pe * sizeof(double));
    L.off_ptr = al(L.off_act + (size_t)L.npair * sizeof(int));   // {current, other} buffer, keep2
    L.off_ver = al(L.off_ptr + 3 * sizeof(double));               // block versions, abort flag
    L.total = al(L.off_ver + (size_t)(L.nblk + 1) * sizeof(int));
    return L;
}

}  // namespace

size_t jacobi_work_bytes(int D, int N) {
    return std::max(std::max(layout(D, N, N, 8).total, layout(D, N, N, 16).total), layout(D, N, N, 32).total);
}

void launch_pchol(hipStream_t st, int n, const double* A, double tau2, int pivot, double* Rt, int* perm, int* keep_dev) {
    hipLaunchKernelGGL(k_pchol, dim3(1), dim3(PC_THREADS), 0, st, n, A, tau2, pivot, Rt, perm, keep_dev);
}

void launch_trsm_rows(hipStream_t st, int keep, int ncol, int n, const double* Rt, const int* perm, const double* Y,
                      long ldy, double* out, long ldo) {
    if (keep <= 0 || ncol <= 0 || keep > TS_MAXK) return;   // callers pass at most TS_MAXK rows
    hipLaunchKernelGGL(k_trsm_rows, dim3(cdiv(ncol, TS_COLS)), dim3(256), 0, st, keep, ncol, n, Rt, perm, Y, ldy, out,
                       ldo);
}

void launch_random_signs(hipStream_t st, long n, unsigned long long seed, double* out) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_random_signs, dim3(cdiv(n, 256)), dim3(256), 0, st, n, seed, out);
}

// Persistent sweep capacity of the device in units of a quarter compute unit (the CU count x 4),
// and what one group of each persistent variant takes (4 / groups that fit in a compute unit:
// 4 units for the 16-wave group, 1 for the 4-wave one), per device; 0 if unknown.
struct PersistentCap {
    int units = 0;
    int per_group[3] = {0, 0, 0};   // indexed by the persistent variant (1: 16 waves, 2: 4 waves)
};

static PersistentCap persistent_capacity() {
    static std::mutex mu;
    static std::vector<PersistentCap> cap;
    static std::vector<int> known;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PersistentCap{};
    std::lock_guard<std::mutex> lk(mu);
    if ((int)cap.size() <= dev) {
        cap.resize(dev + 1);
        known.resize(dev + 1, 0);
    }
    if (!known[dev]) {
        PersistentCap c;
        int b16 = 0, b4 = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b16, k_jacobi_sweep<16>, 16 * 64, 0) == hipSuccess &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&b4, k_jacobi_sweep<4>, 4 * 64, 0) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && b16 > 0 &&
            b4 > 0) {
            c.units = 4 * cus;
            c.per_group[1] = (4 + b16 - 1) / b16;
            c.per_group[2] = (4 + b4 - 1) / b4;
        } else {
            (void)hipGetLastError();
        }
        cap[dev] = c;
        known[dev] = 1;
    }
    return cap[dev];
}

// Reserves n persistent groups within 3/4 of the capacity; released on destruction.
struct GroupTokens {
    std::atomic<int>* use = nullptr;
    int n = 0;
    bool take(std::atomic<int>* u, int want, int budget) {
        if (!u) return true;
        int cur = u->load();
        do {
            if (cur + want > budget) return false;
        } while (!u->compare_exchange_weak(cur, cur + want));
        use = u;
        n = want;
        return true;
    }
    ~GroupTokens() {
        if (use) use->fetch_sub(n);
    }
};

// The permutation sorting squared row norms in descending order.
static void sort_norms(const std::vector<double>& sig2, std::vector<int32_t>& perm) {
    perm.resize(sig2.size());
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return sig2[a] > sig2[b]; });
}

namespace {

// Executable graphs of the sweep for one call, keyed by the number of column blocks (which only
// changes when columns drop below the irrelevance floor); destroyed with the call.
struct SweepGraphs {
    std::vector<std::pair<int, hipGraphExec_t>> execs;
    ~SweepGraphs() {
        for (auto& e : execs) (void)hipGraphExecDestroy(e.second);
    }
    hipGraphExec_t find(int nblk) const {
        for (auto& e : execs)
            if (e.first == nblk) return e.second;
        return nullptr;
    }
};

}  // namespace

int jacobi_svd(hipStream_t st, int D, int N, double* A, int lda, double tol, double irrelevant, int max_sweeps,
               std::vector<double>& sigma, int* sweeps_out, double* work_dev, size_t work_bytes, int n_gram,
               double stop_tail2, JacobiRun* run) {
    JacobiRun defaults;
    if (!run) run = &defaults;
    int graphs = run->graphs;
    int persistent = run->persistent;
    if (n_gram <= 0 || n_gram > N) n_gram = N;
    if (D <= 0 || N <= 0) return fail(LSUM_E_INVALID, "empty side matrix");
    // 16- and 32-column blocks (pairs of 32 or 64 rows) halve or quarter the rounds per sweep;
    // they run round by round (the persistent ways are written for 8-column blocks).  By size
    // (block 0): a sweep reads and writes every row once per round, so 32-column blocks halve the
    // bytes a sweep moves, which pays when several SVDs share the device; alone the 64 x 64 pair
    // solve's latency makes them a few percent slower on large side matrices and 10-30 % slower
    // on small ones, which keep 16-column blocks (served mix: 512 rows and up on 32-column blocks
    // 22.8-22.9 -> 24.1 sums/s, its requests one at a time 690 -> 733 ms of SVD).
    constexpr int kWideRows = 512;
    const int bw = run->block == 0 ? (D >= kWideRows ? 32 : 16) : (run->block == 32 ? 32 : (run->block == 16 ? 16 : 8));
    if (bw != 8) persistent = 0;
    const JacobiLayout L = layout(D, N, n_gram, bw);
    if (work_bytes < L.total) return fail(LSUM_E_INVALID, "Jacobi workspace too small");
    char* base = (char*)work_dev;
    double* X = (double*)base;
    double* X2 = (double*)(base + L.off_x2);
    double* nrm = (double*)(base + L.off_nrm);
    int32_t* perm_dev = (int32_t*)(base + L.off_perm);
    unsigned long long* stat = (unsigned long long*)(base + L.off_stat);
    double* part = (double*)(base + L.off_part);
    double* Qd = (double*)(base + L.off_q);
    int* act = (int*)(base + L.off_act);
    double** xp_dev = (double**)(base + L.off_ptr);
    double* keep2_dev = (double*)(base + L.off_ptr + 2 * sizeof(double*));
    int* ver = (int*)(base + L.off_ver);
    // the bound on a persistent sweep's waits, in ticks of the constant-rate wall clock (kHz)
    // (persistent sweeps may also be chosen later by the autotuner, so it is set up front; without
    // a clock rate no sweep runs persistently)
    long long tick_limit = 0;
    bool clock_ok = true;
    {
        int dev = 0, khz = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) {
            (void)hipGetLastError();
            persistent = 0;
            clock_ok = false;
        }
        tick_limit = (long long)(run->wait_us * 1e-3 * khz);
    }
    // host values read by asynchronous copies: they live until the call returns, and every sweep
    // synchronises before they change
    double* xp_host[2] = {X, X2};
    double keep2 = 0.0;
    LSUM_HIP(hipMemcpyAsync(xp_dev, xp_host, sizeof(xp_host), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_copy_rows_in, dim3(cdiv(L.ldx, 256), L.Dp), dim3(256), 0, st, D, N, A, lda, X, L.ldx);
    hipLaunchKernelGGL(k_norms, dim3(L.Dp), dim3(256), 0, st, L.ldx, n_gram, X, nrm);
    std::vector<double> sig2(L.Dp);
    std::vector<int32_t> perm;
    LSUM_HIP(hipMemcpyAsync(sig2.data(), nrm, L.Dp * sizeof(double), hipMemcpyDeviceToHost, st));
    LSUM_HIP(hipStreamSynchronize(st));
    sort_norms(sig2, perm);
    // columns this small cannot move the certified tail; below 1e-15 sigma_max they are rounding
    const double smax2 = sig2[perm[0]];
    const double irr2 = std::max(irrelevant * irrelevant, 1e-30 * smax2);
    const bool trace = std::getenv("LSUM_JACOBI_TRACE") != nullptr;
    // squared relative coupling at or below which the 32-column pair solve applies no rotation
    const double skip2 = std::max(1e-32, run->skip_rel * run->skip_rel * tol * tol);
    // One sweep: permute the rows (largest first) into the other buffer and make it current, then
    // nblk - 1 rounds of (pair Grams, pair solves, rotations), then the new row norms.  Every
    // sweep with the same nblk issues the same launches; the buffers and keep2 are read from
    // device memory, so one captured graph replays any such sweep.
    auto enqueue_sweep = [&](int nblk) {
        const int npair = nblk / 2;
        // inner cyclic sweeps per visit of a pair.  Two keep the outer sweep count of inner
        // solves run to convergence at a quarter of the inner work (measured on the defected 48^3
        // and step-lattice side matrices).  With many pairs per round the round time is the pair
        // solve's latency, and one inner sweep is faster overall even though it costs about one
        // more outer sweep (cfg3 side matrices: SVD 147 -> 134 ms); with few pairs and long rows
        // the Gram and rotation passes dominate a round, and the second inner sweep pays for
        // itself (few tens of columns of 5633-34305 cells: 30-50 % slower with one).
        const int max_inner = npair >= (bw == 32 ? 8 : 16) ? 1 : 2;
        hipLaunchKernelGGL(k_permute_xp, dim3(cdiv(L.ldx, 256), L.Dp), dim3(256), 0, st, L.ldx, perm_dev, xp_dev);
        hipLaunchKernelGGL(k_swap_clear, dim3(1), dim3(64), 0, st, xp_dev, stat, ver, nblk);
        if (persistent) {
            if (persistent == 2)
                hipLaunchKernelGGL(k_jacobi_sweep<4>, dim3(npair), dim3(4 * 64), 0, st, xp_dev, L.ldx, n_gram, nblk,
                                   L.nchunk, L.nchunk_all, tol, irr2, keep2_dev, max_inner, stat, ver, ver + nblk,
                                   tick_limit);
            else
                hipLaunchKernelGGL(k_jacobi_sweep<16>, dim3(npair), dim3(16 * 64), 0, st, xp_dev, L.ldx, n_gram, nblk,
                                   L.nchunk, L.nchunk_all, tol, irr2, keep2_dev, max_inner, stat, ver, ver + nblk,
                                   tick_limit);
            hipLaunchKernelGGL(k_norms_xp, dim3(L.Dp), dim3(256), 0, st, L.ldx, n_gram, xp_dev, nrm);
            return;
        }
        for (int round = 0; round < nblk - 1; ++round) {
            if (bw == 32) {
                hipLaunchKernelGGL(k_pair_gram64, dim3(L.nchunk, npair), dim3(256), 0, st, xp_dev, L.ldx, n_gram,
                                   nblk, round, L.nchunk, part);
                hipLaunchKernelGGL(k_pair_eig64, dim3(npair), dim3(E64T), 0, st, L.nchunk, part, tol, irr2, skip2,
                                   keep2_dev, max_inner, Qd, act, stat);
                hipLaunchKernelGGL(k_pair_rotate64, dim3(cdiv(L.ldx, CWR64), npair), dim3(256), 0, st, xp_dev, L.ldx,
                                   nblk, round, Qd, act);
                continue;
            }
            if (bw == 16) {
                hipLaunchKernelGGL(k_pair_gram32, dim3(L.nchunk, npair), dim3(256), 0, st, xp_dev, L.ldx, n_gram,
                                   nblk, round, L.nchunk, part);
                hipLaunchKernelGGL(k_pair_eig32, dim3(npair), dim3(256), 0, st, L.nchunk, part, tol, irr2, skip2,
                                   keep2_dev, max_inner, Qd, act, stat);
                hipLaunchKernelGGL(k_pair_rotate32, dim3(cdiv(L.ldx, CWR32), npair), dim3(256), 0, st, xp_dev, L.ldx,
                                   nblk, round, Qd, act);
                continue;
            }
            hipLaunchKernelGGL(k_pair_gram, dim3(L.nchunk, npair), dim3(256), 0, st, xp_dev, L.ldx, n_gram, nblk,
                               round, L.nchunk, part);
            hipLaunchKernelGGL(k_pair_eig, dim3(npair), dim3(256), 0, st, L.nchunk, part, tol, irr2, keep2_dev,
                               max_inner, Qd, act, stat);
            hipLaunchKernelGGL(k_pair_rotate, dim3(L.nchunk_all, npair), dim3(256), 0, st, xp_dev, L.ldx, nblk,
                               round, Qd, act);
        }
        hipLaunchKernelGGL(k_norms_xp, dim3(L.Dp), dim3(256), 0, st, L.ldx, n_gram, xp_dev, nrm);
    };
    SweepGraphs cache;
    int sweeps = 0, cur = 0;
    bool converged = false;
    // rank stop: the certified rank of the current rows, and the squared norm above which rows
    // count as kept (the rank plus a margin of max(16, r/8) rows; 0: every row)
    int r_prev = -1;
    // the autotuner's shape bucket: rows, row length and Gram length, each rounded up to a power
    // of two; its decision (once made) sets how the sweeps are launched
    auto pow2 = [](long x) {
        long b = 1;
        while (b < x) b <<= 1;
        return b;
    };
    const std::string tune_key = "jacobi/" + std::to_string(pow2(L.Dp)) + "/" + std::to_string(pow2(L.ldx)) + "/" +
                                 std::to_string(pow2(n_gram)) + (bw == 16 ? "/b16" : (bw == 32 ? "/b32" : ""));
    int tune_key_choice = run->tuner ? run->tuner->get(tune_key) : -2;
    if (tune_key_choice >= 0) {
        persistent = bw != 8 ? 0 : (tune_key_choice == 2 ? 1 : (tune_key_choice == 3 ? 2 : 0));
        graphs = tune_key_choice == 1;
    }
    const PersistentCap pcap = persistent_capacity();
    for (; sweeps < max_sweeps && !converged; ++sweeps) {
        bool was_persistent = false, used_graph = false;
        // only columns above the floor take part (sorted first); the rest are never rotated
        int d_act = 0;
        while (d_act < L.Dp && sig2[perm[d_act]] > irr2) ++d_act;
        const int nblk = std::max(2, (d_act + 2 * bw - 1) / (2 * bw) * 2);
        LSUM_HIP(hipMemcpyAsync(perm_dev, perm.data(), L.Dp * sizeof(int32_t), hipMemcpyHostToDevice, st));
        LSUM_HIP(hipMemcpyAsync(keep2_dev, &keep2, sizeof(double), hipMemcpyHostToDevice, st));
        // persistent groups reserved against 3/4 of the device (per variant: its share of a CU)
        auto take_tokens = [&](GroupTokens& t) -> bool {
            if (pcap.units <= 0 || persistent < 1 || persistent > 2) return false;
            return t.take(run->wg_in_use, (nblk / 2) * pcap.per_group[persistent], pcap.units * 3 / 4);
        };
        // the sweep's graph for this block count, captured on first use (nullptr if refused)
        auto graph_for = [&](int nb) -> hipGraphExec_t {
            hipGraphExec_t gx = cache.find(nb);
            if (gx) return gx;
            hipGraph_t g = nullptr;
            const int keep_persistent = persistent;
            persistent = 0;
            bool ok = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess;
            if (ok) {
                enqueue_sweep(nb);
                ok = hipStreamEndCapture(st, &g) == hipSuccess && g != nullptr;
            }
            persistent = keep_persistent;
            if (ok) ok = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0) == hipSuccess;
            if (g) (void)hipGraphDestroy(g);
            if (!ok) {
                (void)hipGetLastError();
                return nullptr;
            }
            cache.execs.push_back({nb, gx});
            return gx;
        };
        // autotuning (first sweep of a shape bucket not yet decided): the sweep runs once in each
        // way -- persistent, from a graph, round by round -- from the same rows X (a sweep reads X
        // and writes only the other buffer), each timed; all three give the same rows bit for bit,
        // and the last one's stand as this sweep's result
        if (sweeps == 0 && tune_key_choice == -1) {
            // variants: 0 round by round, 1 graph, 2 persistent 16-wave groups, 3 persistent 4-wave
            std::vector<double> ms(4, -1.0);
            hipEvent_t e0 = nullptr, e1 = nullptr;
            LSUM_HIP(hipEventCreate(&e0));
            LSUM_HIP(hipEventCreate(&e1));
            for (int m : {3, 2, 1, 0}) {
                if (m >= 2 && (!clock_ok || bw != 8)) continue;
                LSUM_HIP(hipMemcpyAsync(xp_dev, xp_host, sizeof(xp_host), hipMemcpyHostToDevice, st));
                persistent = m == 2 ? 1 : (m == 3 ? 2 : 0);
                GroupTokens tk;
                bool ok = true;
                if (persistent && !take_tokens(tk)) {
                    persistent = 0;
                    ok = false;
                }
                hipGraphExec_t gx = m == 1 ? graph_for(nblk) : nullptr;
                if (m == 1 && !gx) ok = false;
                LSUM_HIP(hipEventRecord(e0, st));
                if (gx) {
                    LSUM_HIP(hipGraphLaunch(gx, st));
                } else {
                    enqueue_sweep(nblk);
                }
                LSUM_HIP(hipEventRecord(e1, st));
                int ab = 0;
                if (persistent) LSUM_HIP(hipMemcpyAsync(&ab, ver + nblk, sizeof(int), hipMemcpyDeviceToHost, st));
                LSUM_HIP(hipStreamSynchronize(st));
                float t = 0.f;
                if (ok && !ab && hipEventElapsedTime(&t, e0, e1) == hipSuccess) ms[m] = t;
                (void)hipGetLastError();
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            const int ch = run->tuner->put(tune_key, ms);
            persistent = bw != 8 ? 0 : (ch == 2 ? 1 : (ch == 3 ? 2 : 0));
            graphs = ch == 1;
            tune_key_choice = ch;
            run->tuned = 1;
        } else {
            // a persistent sweep needs all its groups resident at once: it runs only while the
            // groups of the persistent sweeps in flight stay within 3/4 of the device; else round
            // by round
            GroupTokens tokens;
            const int persistent_mode = persistent;
            if (persistent && !take_tokens(tokens)) persistent = 0;
            hipGraphExec_t ge = graphs && !persistent ? graph_for(nblk) : nullptr;
            if (graphs && !persistent && !ge) graphs = 0;   // capture refused: launch directly
            if (ge) {
                LSUM_HIP(hipGraphLaunch(ge, st));
                used_graph = true;
            } else {
                enqueue_sweep(nblk);
            }
            was_persistent = persistent != 0;
            if (!was_persistent) persistent = persistent_mode;   // no tokens this sweep: try again next sweep
        }
        // the buffers before this sweep: it read the current one and wrote only the other
        double* before[2] = {cur ? X2 : X, cur ? X : X2};
        cur ^= 1;
        // FP64 MFMA work of the sweep: every pair visit forms a 2bw x 2bw Gram over n_gram entries
        // and (when active) rotates 2bw rows of ldx entries; counted for every visit
        run->flops += (double)(nblk / 2) * (nblk - 1) * 8.0 * bw * bw * ((double)n_gram + L.ldx);
        unsigned long long st4[7] = {0, 0, 0, 0, 0, 0, 0};
        int aborted = 0;
        LSUM_HIP(hipMemcpyAsync(st4, stat, sizeof(st4), hipMemcpyDeviceToHost, st));
        if (was_persistent) LSUM_HIP(hipMemcpyAsync(&aborted, ver + nblk, sizeof(int), hipMemcpyDeviceToHost, st));
        LSUM_HIP(hipMemcpyAsync(sig2.data(), nrm, L.Dp * sizeof(double), hipMemcpyDeviceToHost, st));
        LSUM_HIP(hipStreamSynchronize(st));
        LSUM_HIP(hipGetLastError());
        if (was_persistent) {
            ++run->persistent_sweeps;
            if (aborted) {
                // some groups were not resident together (or the wait bound is tiny), so the
                // sweep visited only part of the pairs.  It read the rows before it and wrote only
                // the other buffer: it runs again, round by round, from those rows, which gives the
                // rows an uninterrupted sweep gives; the remaining sweeps launch round by round
                ++run->aborted;
                persistent = 0;
                was_persistent = false;
                if (trace) std::fprintf(stderr, "jacobi D=%d N=%d sweep %d: persistent sweep aborted, run again\n", D, N, sweeps);
                LSUM_HIP(hipMemcpyAsync(xp_dev, before, sizeof(before), hipMemcpyHostToDevice, st));
                enqueue_sweep(nblk);
                LSUM_HIP(hipMemcpyAsync(st4, stat, sizeof(st4), hipMemcpyDeviceToHost, st));
                LSUM_HIP(hipMemcpyAsync(sig2.data(), nrm, L.Dp * sizeof(double), hipMemcpyDeviceToHost, st));
                LSUM_HIP(hipStreamSynchronize(st));
                LSUM_HIP(hipGetLastError());
            }
        }
        sort_norms(sig2, perm);
        double off, offk;
        std::memcpy(&off, &st4[0], sizeof(off));
        std::memcpy(&offk, &st4[4], sizeof(offk));
        if (off <= tol) converged = true;
        int r_now = -1;
        if (stop_tail2 > 0.0 && !converged) {
            // The rows stay an orthogonal transform of the input, so for any r the projection on
            // the span of the r largest rows leaves at most the energy of the other rows: that
            // tail is certified in every sweep, and the sweeps that follow only tighten it.  Stop
            // once the smallest certified r is the same as after the previous sweep and the rows
            // that were kept in this sweep (r + margin) were orthogonal to tol when visited: the
            // kept rows then normalise to an orthonormal basis, and the remaining sweeps would only
            // rotate rows of the tail against each other and against the basis.
            double t = 0.0;
            r_now = L.Dp;
            for (int k = L.Dp - 1; k >= 0; --k) {
                t += sig2[perm[k]];
                if (t > stop_tail2) break;
                r_now = k;
            }
            if (r_now == r_prev && offk <= tol) converged = true;
            r_prev = r_now;
            const int m = r_now + std::max(16, r_now / 8);
            keep2 = m < L.Dp ? sig2[perm[m]] : 0.0;
        }
        // A sweep whose pairs were already close to orthogonal when visited (quadratic
        // convergence: couplings of 1e-4 .. 1e-8 measured to leave 1e-11 .. 1e-13) usually
        // leaves every coupling below tol; the sweep that would find that out rotates nothing but
        // still forms every pair's Gram.  The rows' full Gram (one FP64 GEMM into the buffer the
        // next sweep writes) checks all couplings at once instead.
        double off_after = -1.0;
        if (!converged && off <= 1e-4 && L.Dp <= L.ldx) {
            double* Xc = cur ? X2 : X;
            double* Gs = cur ? X : X2;   // free until the next sweep permutes into it
            GemmArgs g{};
            g.m = L.Dp; g.n = L.Dp; g.k = n_gram;
            g.A = Xc; g.sam = L.ldx; g.sak = 1;
            g.B = Xc; g.sbk = 1; g.sbn = L.ldx;
            g.C = Gs; g.scm = L.Dp; g.scn = 1;
            g.alpha = 1.0; g.beta = 0.0; g.batch = 1;
            unsigned long long* cbits = (unsigned long long*)part;
            hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, cbits, 2);
            launch_gemm(st, GEMM_F64, g);
            hipLaunchKernelGGL(k_gram_coupling, dim3(cdiv(L.Dp, 256), L.Dp), dim3(256), 0, st, L.Dp, Gs, (long)L.Dp,
                               irr2, keep2, cbits);
            unsigned long long cb[2] = {0, 0};
            LSUM_HIP(hipMemcpyAsync(cb, cbits, sizeof(cb), hipMemcpyDeviceToHost, st));
            LSUM_HIP(hipStreamSynchronize(st));
            LSUM_HIP(hipGetLastError());
            std::memcpy(&off_after, &cb[0], sizeof(off_after));
            if (off_after <= tol) converged = true;
        }
        if (trace)
            std::fprintf(stderr, "jacobi D=%d N=%d sweep %d active %d max coupling %.3e (after the sweep %.3e) kept %.3e rank %d inner sweeps %.2f avg %llu max over %llu pairs, steps applied %llu of %llu%s\n",
                         D, N, sweeps, d_act, off, off_after, offk, r_now, st4[3] ? (double)st4[1] / (double)st4[3] : 0.0, st4[2],
                         st4[3], st4[5], st4[6], was_persistent ? " (persistent)" : (used_graph ? " (graph)" : ""));
    }
    // write back the D largest columns in descending order
    double* Xcur = cur ? X2 : X;
    LSUM_HIP(hipMemcpyAsync(perm_dev, perm.data(), L.Dp * sizeof(int32_t), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_permute_rows, dim3(cdiv(N, 256), D), dim3(256), 0, st, L.ldx, perm_dev, Xcur, A, lda, N);
    LSUM_HIP(hipGetLastError());
    LSUM_HIP(hipStreamSynchronize(st));
    sigma.resize(D);
    for (int a = 0; a < D; ++a) sigma[a] = std::sqrt(std::max(sig2[perm[a]], 0.0));
    *sweeps_out = sweeps;
    if (!converged) return fail(LSUM_E_NOCONV, "Jacobi SVD did not converge");
    return LSUM_OK;
}

}  // namespace lsum

// Pipeline stages of the lattice-sum library, run by the request workers on a slot's stream:
//   reference vectors (Sec. 2.1, 3.1) -> assembled shift-sums for a whole batch of requests in
//   one launch (Thm thm:sumCaseE (A)) -> point-major copies of the factors -> for a reduction
//   request: side-matrix columns, ||A|| and ||xi||, the certified truncation threshold, the
//   Jacobi SVD, Tucker factors, projections, the core (Def. def:RHOSVD, Appendix theorem) and
//   an optional tile (eq. Tucker_singePot) -> sampling at the request's points.
#include "lsum_runtime.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>

namespace lsum {

// cells at which every Tucker result is compared with its untruncated canonical sum, on this
// many mode-3 planes
constexpr int kProbeCells = 32;
constexpr int kProbePlanes = 4;

static GemmPrec gemm_prec(int precision) {
    return precision == LSUM_FP64 ? GEMM_F64 : (precision == LSUM_FP32 ? GEMM_F32 : GEMM_BF16X3);
}

// Truncated SVD of one weighted side matrix W (D rows of length N; Def. def:RHOSVD).  The
// result is a list of singular values and rows holding the matching left singular vectors,
// such that for every r, ||A - Z_r Z_r^T A||_F^2 <= res2 + sum_{a >= r} sigma_a^2.
//  * direct: one-sided Jacobi on W itself (res2 = 0; rows = rotated W, sigma-scaled) when
//    D <= N, else on the N rows of [W^T | I] (the identity block accumulates the rotation and
//    holds the unit vectors);
//  * range basis, for min(D, N) >= range_min: an orthonormal basis Q of k <= min(D, N) rows
//    grown in blocks of random-sign sketches of the residual, B = Q W^T, and the residual
//    E = W - B^T Q computed explicitly (res2 = ||E||_F^2, which must stay below (thr/10)^2, else
//    the direct solve runs); then Jacobi on the k rows [B | I] with the Gram taken over B only
//    (the identity part accumulates the rotation V), and the vectors V Q are orthonormal, so
//    ||A - Z_r Z_r^T A||^2 = res2 + sum_{a >= r} sigma_a^2 exactly.
// A GEMM launch that splits a long FP64 reduction over many workgroups when the output has few
// tiles (Grams of a few tens of columns over N_l cells, projections onto a few tens of vectors):
// one tile would otherwise walk all N_l terms alone.  Synchronous when split (the workspace goes
// back to the pool).
int gemm_auto(Context* c, hipStream_t st, GemmPrec prec, const GemmArgs& a) {
    const long tiles = (long)((a.n + 63) / 64) * ((a.m + 127) / 128) * a.batch;
    if (blas_gemm(st, prec, a)) return LSUM_OK;
    if (prec != GEMM_F64 || a.batch != 1 || tiles >= 64 || a.k < 2048) {
        launch_gemm(st, prec, a);
        return LSUM_OK;
    }
    const int split = (int)std::max<long>(2, std::min<long>(std::min<long>(512 / tiles, a.k / 128), 512));
    const int slices = gemm_split_slices(a, split);
    DevBuf work;
    int rc = work.get(c->pool, (size_t)slices * a.m * a.n * 8);
    if (rc) return rc;
    launch_gemm_split_f64(st, a, split, work.as<double>());
    LSUM_HIP(hipStreamSynchronize(st));
    return LSUM_OK;
}

struct ModeSVD {
    std::vector<double> sigma;   // descending
    double res2 = 0.0;
    DevBuf rows;
    long ld = 0, off = 0;        // row stride, offset of the vector part
    bool unit = false;           // vector rows are unit (range path) or sigma-scaled (direct)
    int k = 0, sweeps = 0;
    double flops = 0.0;          // FP64 MFMA work: range-basis GEMMs, Jacobi Grams and rotations
    int persistent = 0, aborted = 0;   // Jacobi sweeps launched persistently / aborted
    int tuned = 0;                     // the autotuner timed the ways of launching a sweep
};

// C (m x n) = alpha * X Y + beta * C over row-major operands; tX / tY: use the transpose.
static void gemm_rm(hipStream_t st, int m, int n, int k, const double* X, long ldx, bool tX, const double* Y,
                    long ldy, bool tY, double* C, long ldc, double alpha, double beta) {
    GemmArgs a{};
    a.m = m; a.n = n; a.k = k;
    a.A = X; a.sam = tX ? 1 : ldx; a.sak = tX ? ldx : 1;
    a.B = Y; a.sbk = tY ? 1 : ldy; a.sbn = tY ? ldy : 1;
    a.C = C; a.scm = ldc; a.scn = 1;
    a.alpha = alpha; a.beta = beta; a.batch = 1;
    launch_gemm(st, GEMM_F64, a);
}

// Squared Frobenius norm of a rows x n row-major matrix (synchronises st).
static int frob2(Context* c, hipStream_t st, int rows, int n, const double* X, double* out) {
    DevBuf nrm;
    int rc = nrm.get(c->pool, (size_t)rows * 8);
    if (rc) return rc;
    launch_row_norms(st, rows, n, X, n, nrm.as<double>());
    std::vector<double> en(rows);
    LSUM_HIP(hipMemcpyAsync(en.data(), nrm.p, (size_t)rows * 8, hipMemcpyDeviceToHost, st));
    LSUM_HIP(hipStreamSynchronize(st));
    double s = 0.0;
    for (double v : en) s += v * v;
    *out = s;
    return LSUM_OK;
}

// G (m x m) = X X^T for the m rows of X (length n, stride ldx); split over n when G has few tiles.
static int gram_rows(Context* c, hipStream_t st, int m, int n, const double* X, long ldx, double* G) {
    GemmArgs a{};
    a.m = m; a.n = m; a.k = n;
    a.A = X; a.sam = ldx; a.sak = 1;
    a.B = X; a.sbk = 1; a.sbn = ldx;
    a.C = G; a.scm = m; a.scn = 1;
    a.alpha = 1.0; a.beta = 0.0; a.batch = 1;
    return gemm_auto(c, st, GEMM_F64, a);
}

// Orthonormal rows spanning the significant rows of Y (m x n, stride n; m <= 128): the
// rank-revealing Cholesky of Y Y^T keeps pivots above tau2 times the first (rows above
// sqrt(tau2) in norm), and out (keep x n) = R^{-T} Y_p by forward substitution.  Returns keep
// (0: nothing above the threshold).  Without `pivot` the rows are taken in their order (for
// rows that are already orthonormal to a few digits, whose Gram is near the identity).
static int chol_rows(Context* c, hipStream_t st, int m, int n, const double* Y, double tau2, double* small,
                     double* out, int* keep, int pivot = 1) {
    if (m > 128) return fail(LSUM_E_INVALID, "chol_rows: more than 128 rows");
    double* G = small;
    double* Rt = small + (size_t)m * m;
    int* perm = (int*)(Rt + (size_t)m * m);
    int* kd = perm + m;
    int rc;
    if ((rc = gram_rows(c, st, m, n, Y, n, G))) return rc;
    launch_pchol(st, m, G, tau2, pivot, Rt, perm, kd);
    LSUM_HIP(hipGetLastError());
    LSUM_HIP(hipMemcpyAsync(keep, kd, sizeof(int), hipMemcpyDeviceToHost, st));
    LSUM_HIP(hipStreamSynchronize(st));
    launch_trsm_rows(st, *keep, n, m, Rt, perm, Y, n, out, n);
    LSUM_HIP(hipGetLastError());
    return LSUM_OK;
}

// Range basis grown in blocks (a blocked form of the adaptive randomized range finder): each
// block sketches the current residual E (Y = Omega^T E, random signs) and is orthogonalised
// twice against the basis so far.  Its significant rows (down to 1e-6 of the largest in norm)
// are made orthonormal by the rank-revealing Cholesky of their Gram, once more orthogonalised
// against the basis and orthonormalised by a second Cholesky pass (CholeskyQR2: orthonormal to
// rounding); E then loses the block's directions.  The growth stops once ||E||_F <= thr / 10 or
// the basis would exceed k_max rows.  B = Q W^T and E = W - B^T Q are then recomputed from W.
// Jacobi on the rows [B | I] (Gram over B) finds the orthogonal V whose rows V B are orthogonal
// (their norms the singular values), the identity block accumulating V; the singular vectors
// are then the rows of V Q, one product at the end instead of rotating Q's N entries per row in
// every round (rows of D + k entries instead of D + N).
static int range_svd(Context* c, hipStream_t st, int D, int N, const double* W, int k_block, int k_max,
                     double thr, double irrelevant, ModeSVD& out, bool* enough) {
    int rc;
    *enough = false;
    if (k_block < 16 || k_max < k_block) return LSUM_OK;
    DevBuf Qall, E, Om, Yt, Y2, P, small;
    if ((rc = Qall.get(c->pool, (size_t)k_max * N * 8))) return rc;
    if ((rc = E.get(c->pool, (size_t)D * N * 8))) return rc;
    if ((rc = Om.get(c->pool, (size_t)D * k_block * 8))) return rc;
    if ((rc = Yt.get(c->pool, (size_t)k_block * N * 8))) return rc;
    if ((rc = Y2.get(c->pool, (size_t)k_block * N * 8))) return rc;
    if ((rc = P.get(c->pool, (size_t)std::max(D, k_block) * k_max * 8))) return rc;
    if ((rc = small.get(c->pool, (size_t)3 * k_block * k_block * 8 + 256))) return rc;
    LSUM_HIP(hipMemcpyAsync(E.p, W, (size_t)D * N * 8, hipMemcpyDeviceToDevice, st));
    double* Q = Qall.as<double>();
    int kq = 0, blocks = 0;
    double res2 = 0.0;
    for (;;) {
        const int kb = std::min(k_block, k_max - kq);
        if (kb < 16) return LSUM_OK;   // the basis would grow past k_max
        launch_random_signs(st, (long)D * kb, 0x5eed1411ull + 7919ull * (unsigned long long)blocks + (unsigned long long)kb,
                            Om.as<double>());
        // Yt (kb x N) = Omega^T E
        gemm_rm(st, kb, N, D, Om.as<double>(), kb, true, E.as<double>(), N, false, Yt.as<double>(), N, 1.0, 0.0);
        out.flops += 2.0 * kb * (double)N * D + 8.0 * kb * (double)kq * N * (kq > 0) + 2.0 * kb * (double)kb * N;
        for (int pass = 0; kq > 0 && pass < 2; ++pass) {
            // Yt -= (Yt Q^T) Q
            gemm_rm(st, kb, kq, N, Yt.as<double>(), N, false, Q, N, true, P.as<double>(), kq, 1.0, 0.0);
            gemm_rm(st, kb, N, kq, P.as<double>(), kq, false, Q, N, false, Yt.as<double>(), N, -1.0, 1.0);
        }
        int keep = 0;
        if ((rc = chol_rows(c, st, kb, N, Yt.as<double>(), 1e-12, small.as<double>(), Y2.as<double>(), &keep)))
            return rc;
        if (keep == 0) return LSUM_OK;
        if (kq > 0) {
            gemm_rm(st, keep, kq, N, Y2.as<double>(), N, false, Q, N, true, P.as<double>(), kq, 1.0, 0.0);
            gemm_rm(st, keep, N, kq, P.as<double>(), kq, false, Q, N, false, Y2.as<double>(), N, -1.0, 1.0);
        }
        double* Qb = Q + (size_t)kq * N;
        int keep2 = 0;
        // the second pass factors a Gram within rounding of the identity: no pivots needed
        if ((rc = chol_rows(c, st, keep, N, Y2.as<double>(), 1e-12, small.as<double>(), Qb, &keep2, 0))) return rc;
        if (keep2 == 0) return LSUM_OK;
        keep = keep2;
        out.flops += 2.0 * keep * (double)kb * N + 4.0 * keep * (double)kq * N + 4.0 * keep * (double)keep * N +
                     4.0 * D * (double)keep * N;
        // E -= (E Qb^T) Qb
        gemm_rm(st, D, keep, N, E.as<double>(), N, false, Qb, N, true, P.as<double>(), keep, 1.0, 0.0);
        gemm_rm(st, D, N, keep, P.as<double>(), keep, false, Qb, N, false, E.as<double>(), N, -1.0, 1.0);
        kq += keep;
        ++blocks;
        if ((rc = frob2(c, st, D, N, E.as<double>(), &res2))) return rc;   // synchronises
        if (std::getenv("LSUM_JACOBI_TRACE"))
            std::fprintf(stderr, "range D=%d N=%d block %d kept %d of %d basis %d of %d residual/thr %.3e\n", D, N,
                         blocks, keep, kb, kq, k_max, std::sqrt(res2) / thr);
        if (std::sqrt(res2) <= 0.1 * thr) break;
    }
    Om.reset();
    Yt.reset();
    Y2.reset();
    P.reset();
    small.reset();
    // AUG rows [B_a | I_a]: B (kq x D) = Q W^T; the exact residual E = W - B^T Q
    const long ld = (long)D + kq;
    DevBuf AUG;
    if ((rc = AUG.get(c->pool, (size_t)kq * ld * 8))) return rc;
    LSUM_HIP(hipMemsetAsync(AUG.p, 0, (size_t)kq * ld * 8, st));
    gemm_rm(st, kq, D, N, Q, N, false, W, N, true, AUG.as<double>(), ld, 1.0, 0.0);
    launch_unit_diag(st, kq, ld, D, AUG.as<double>());
    LSUM_HIP(hipMemcpyAsync(E.p, W, (size_t)D * N * 8, hipMemcpyDeviceToDevice, st));
    gemm_rm(st, D, N, kq, AUG.as<double>(), ld, true, Q, N, false, E.as<double>(), N, -1.0, 1.0);
    out.flops += 4.0 * kq * (double)D * N;
    if ((rc = frob2(c, st, D, N, E.as<double>(), &res2))) return rc;
    if (!(std::sqrt(res2) <= 0.1 * thr)) return LSUM_OK;   // basis too small
    E.reset();
    DevBuf work;
    const size_t wb2 = jacobi_work_bytes(kq, (int)ld);
    if ((rc = work.get(c->pool, wb2))) return rc;
    // the accumulated rows of V stay orthonormal in any sweep, so the rank stop needs no extra
    // step here
    JacobiRun jr = jacobi_run(c);
    rc = jacobi_svd(st, kq, (int)ld, AUG.as<double>(), (int)ld, 1e-12, irrelevant, c->jacobi_max_sweeps.load(),
                    out.sigma, &out.sweeps,
                    work.as<double>(), wb2, D, c->jacobi_rank_stop ? thr * thr - res2 : 0.0, &jr);
    out.flops += jr.flops;
    out.persistent += jr.persistent_sweeps;
    out.aborted += jr.aborted;
    out.tuned |= jr.tuned;
    if (rc) return rc;
    work.reset();
    // the singular vectors: rows of V Q (kq x N), in the sorted order of the rows
    DevBuf Z;
    if ((rc = Z.get(c->pool, (size_t)kq * N * 8))) return rc;
    gemm_rm(st, kq, N, kq, AUG.as<double>() + D, ld, false, Q, N, false, Z.as<double>(), N, 1.0, 0.0);
    out.flops += 2.0 * kq * (double)kq * N;
    LSUM_HIP(hipGetLastError());
    // AUG and Q return to the pool (which hands memory on at once) when this returns
    LSUM_HIP(hipStreamSynchronize(st));
    out.res2 = res2;
    out.rows = std::move(Z);
    out.ld = N;
    out.off = 0;
    out.unit = true;
    out.k = kq;
    *enough = true;
    return LSUM_OK;
}

static int mode_svd(Context* c, hipStream_t st, int D, int N, DevBuf& W, double thr, double irrelevant,
                    ModeSVD& out, bool allow_range = true) {
    int rc;
    const int mn = std::min(D, N);
    const int range_min = allow_range ? c->range_min : 0;
    if (range_min > 0 && mn >= range_min) {
        // a basis grown in blocks of 128 vectors (the Gram of a block is factored in LDS) up to
        // min(D, N): the residual E takes the directions below thr / 10, which the direct solve
        // would otherwise drain row by row over many sweeps
        const int k_max = mn;
        const int k_block = std::min(128, k_max);
        bool enough = false;
        if ((rc = range_svd(c, st, D, N, W.as<double>(), k_block, k_max, thr, irrelevant, out, &enough))) return rc;
        if (enough) return LSUM_OK;
    }
    if (N < D) {
        // more columns than cells: Jacobi on the N rows of [W^T | I] with the Gram over W^T's D
        // entries.  The identity block accumulates the orthogonal V; for any V the rows W v_a of
        // the W^T part satisfy ||W - W Z_r^T Z_r||^2 = sum_{a >= r} ||W v_a||^2 with Z_r the first
        // r rows of V^T, so the certificate is that of the direct solve, and the unit rows of the
        // identity block are the vectors.  N rows instead of D: no D - N null-space rows to drain.
        const long ld = (long)D + N;
        DevBuf AUG;
        if ((rc = AUG.get(c->pool, (size_t)N * ld * 8))) return rc;
        LSUM_HIP(hipMemsetAsync(AUG.p, 0, (size_t)N * ld * 8, st));
        launch_transpose_ld(st, D, N, W.as<double>(), N, AUG.as<double>(), ld);
        launch_unit_diag(st, N, ld, D, AUG.as<double>());
        LSUM_HIP(hipGetLastError());
        DevBuf work;
        const size_t wb = jacobi_work_bytes(N, (int)ld);
        if ((rc = work.get(c->pool, wb))) return rc;
        // no irrelevance floor here: a row is a cell, and a cell of small norm still carries small
        // components of the leading vectors, which a row left unrotated would drop
        JacobiRun jr = jacobi_run(c);
        rc = jacobi_svd(st, N, (int)ld, AUG.as<double>(), (int)ld, 1e-12, 0.0, c->jacobi_max_sweeps.load(),
                        out.sigma, &out.sweeps, work.as<double>(), wb, D, c->jacobi_rank_stop ? thr * thr : 0.0, &jr);
        out.flops += jr.flops;
        out.persistent += jr.persistent_sweeps;
        out.aborted += jr.aborted;
        out.tuned |= jr.tuned;
        if (rc) return rc;
        out.res2 = 0.0;
        out.rows = std::move(AUG);
        out.ld = ld;
        out.off = D;
        out.unit = true;
        out.k = 0;
        return LSUM_OK;
    }
    DevBuf work;
    const size_t wb = jacobi_work_bytes(D, N);
    if ((rc = work.get(c->pool, wb))) return rc;
    JacobiRun jr = jacobi_run(c);
    rc = jacobi_svd(st, D, N, W.as<double>(), N, 1e-12, irrelevant, c->jacobi_max_sweeps.load(), out.sigma,
                    &out.sweeps, work.as<double>(),
                    wb, 0, c->jacobi_rank_stop ? thr * thr : 0.0, &jr);
    out.flops += jr.flops;
    out.persistent += jr.persistent_sweeps;
    out.aborted += jr.aborted;
    out.tuned |= jr.tuned;
    if (rc) return rc;
    out.res2 = 0.0;
    out.rows = std::move(W);
    out.ld = N;
    out.off = 0;
    out.unit = false;
    out.k = 0;
    return LSUM_OK;
}

// Optional tile of a Tucker result: V = mu x_3 Z3 x_2 Z2 x_1 Z1 restricted to [lo, lo+T), in the
// request's precision (eq. Tucker_singePot).
static int make_tile(Request* q, hipStream_t st, StageTimer& tm) {
    Context* c = q->ctx;
    const Plan& P = q->plan();
    const GemmPrec prec = gemm_prec(P.precision);
    const size_t es = (prec == GEMM_F64) ? 8 : 4;
    int rc;
    tm.begin("tile", (double)P.tile_T[0] * P.tile_T[1] * P.tile_T[2] * (P.precision == LSUM_FP64 ? 8 : 4), 2.0 * ((double)q->r[0] * q->r[1] * q->r[2] * P.tile_T[2] + (double)q->r[0] * q->r[1] * P.tile_T[1] * P.tile_T[2] + (double)q->r[0] * P.tile_T[0] * P.tile_T[1] * P.tile_T[2]));
    const int r1 = q->r[0], r2 = q->r[1], r3 = q->r[2];
    const int T1 = P.tile_T[0], T2 = P.tile_T[1], T3 = P.tile_T[2];
    const void* Zp[3];
    DevBuf Zf[3];
    for (int l = 0; l < 3; ++l) {
        Zp[l] = q->Z[l].p;
        if (prec != GEMM_F64) {
            if ((rc = Zf[l].get(c->pool, (size_t)q->r[l] * P.N[l] * 4))) return rc;
            launch_f64_to_f32(st, (long)q->r[l] * P.N[l], q->Z[l].as<double>(), Zf[l].as<float>());
            Zp[l] = Zf[l].p;
        }
    }
    DevBuf X1, X2;
    if ((rc = X1.get(c->pool, (size_t)r1 * r2 * T3 * es))) return rc;
    if ((rc = X2.get(c->pool, (size_t)r1 * T2 * T3 * es))) return rc;
    if ((rc = q->tile.get(c->pool, (size_t)T1 * T2 * T3 * es))) return rc;
    const long e = (long)es;
    GemmArgs a{};
    // X1[(a,b), n] = sum_c mu[(a,b), c] Z3[c, lo3 + n]
    a.m = r1 * r2; a.n = T3; a.k = r3;
    a.A = q->core.p; a.sam = r3; a.sak = 1;
    a.B = (const char*)Zp[2] + (long)P.tile_lo[2] * e; a.sbk = P.N[2]; a.sbn = 1;
    a.C = X1.p; a.scm = T3; a.scn = 1;
    a.alpha = 1.0; a.beta = 0.0; a.batch = 1;
    launch_gemm(st, prec, a);
    // X2[a][m, n] = sum_b Z2[b, lo2 + m] X1[(a,b), n]
    a = GemmArgs{};
    a.m = T2; a.n = T3; a.k = r2;
    a.A = (const char*)Zp[1] + (long)P.tile_lo[1] * e; a.sam = 1; a.sak = P.N[1];
    a.B = X1.p; a.sbk = T3; a.sbn = 1;
    a.C = X2.p; a.scm = T3; a.scn = 1;
    a.alpha = 1.0; a.beta = 0.0; a.batch = r1; a.bA = 0; a.bB = (long)r2 * T3; a.bC = (long)T2 * T3;
    launch_gemm(st, prec, a);
    // V[m, (n2,n3)] = sum_a Z1[a, lo1 + m] X2[a, (n2,n3)]
    a = GemmArgs{};
    a.m = T1; a.n = T2 * T3; a.k = r1;
    a.A = (const char*)Zp[0] + (long)P.tile_lo[0] * e; a.sam = 1; a.sak = P.N[0];
    a.B = X2.p; a.sbk = (long)T2 * T3; a.sbn = 1;
    a.C = q->tile.p; a.scm = (long)T2 * T3; a.scn = 1;
    a.alpha = 1.0; a.beta = 0.0; a.batch = 1;
    launch_gemm(st, prec, a);
    LSUM_HIP(hipGetLastError());
    LSUM_HIP(hipStreamSynchronize(st));
    tm.end();
    q->bytes["tile"] = (double)T1 * T2 * T3 * es;
    return LSUM_OK;
}

// The leading r singular vectors of an SVD as factor rows (r x N): rotated rows / sigma, or the
// unit rows of the range path.
static int rows_to_factor(Context* c, hipStream_t st, ModeSVD& ms, int r, int N, DevBuf& Z) {
    int rc;
    std::vector<double> inv(r);
    std::vector<int32_t> ord(r);
    for (int a = 0; a < r; ++a) { inv[a] = ms.unit ? 1.0 : 1.0 / ms.sigma[a]; ord[a] = a; }
    DevBuf od, iv;
    if ((rc = od.get(c->pool, r * 4))) return rc;
    if ((rc = iv.get(c->pool, r * 8))) return rc;
    if ((rc = Z.get(c->pool, (size_t)r * N * 8))) return rc;
    LSUM_HIP(hipMemcpyAsync(od.p, ord.data(), r * 4, hipMemcpyHostToDevice, st));
    LSUM_HIP(hipMemcpyAsync(iv.p, inv.data(), r * 8, hipMemcpyHostToDevice, st));
    launch_gather_scale_rows(st, r, N, ms.rows.as<double>() + ms.off, (int)ms.ld, od.as<int32_t>(), iv.as<double>(),
                             Z.as<double>(), N);
    LSUM_HIP(hipStreamSynchronize(st));
    ms.rows.reset();
    return LSUM_OK;
}

// ALS sweeps (Thm thm:C2Tucker (b)) from the current factors q->Z: per mode l, with a, b the
// other modes, the rows of M_l^T = sum_nu (x_a,nu (x) x_b,nu) t_l,nu^T (r_a r_b x N_l), where
// t_l,nu is term nu's side column (times xi_nu for mode 0) and x_m,nu = Z_m t_m,nu its
// projection; the leading r_l left singular vectors of M_l replace Z_l.  ||core|| after a mode is
// the root of the sum of M_l's r_l largest sigma^2, recorded after each sweep.
static int run_als(Request* q, hipStream_t st, DevBuf cols[3], StageTimer& tm) {
    Context* c = q->ctx;
    const Plan& P = q->plan();
    int rc;
    const int* r = q->r;
    for (int l = 0; l < 3; ++l) {
        const int a = (l + 1) % 3, b = (l + 2) % 3;
        if ((long)r[a] * r[b] > 4096 || r[l] > r[a] * r[b]) {
            q->als_skipped = 1;
            return LSUM_OK;
        }
    }
    tm.begin("als");
    const long K = (long)P.n_groups * P.R;
    std::vector<int32_t> idx(3 * (size_t)K);
    std::vector<double> scv(K);
    for (int g = 0; g < P.n_groups; ++g)
        for (int k = 0; k < P.R; ++k) {
            const long nu = (long)g * P.R + k;
            for (int l = 0; l < 3; ++l) idx[(size_t)l * K + nu] = P.g_src[l][g] * P.R + k;
            scv[nu] = P.g_scale[g];
        }
    DevBuf idx_d, sc_d, T[3];
    if ((rc = idx_d.get(c->pool, idx.size() * 4)) || (rc = sc_d.get(c->pool, K * 8))) return rc;
    LSUM_HIP(hipMemcpyAsync(idx_d.p, idx.data(), idx.size() * 4, hipMemcpyHostToDevice, st));
    LSUM_HIP(hipMemcpyAsync(sc_d.p, scv.data(), K * 8, hipMemcpyHostToDevice, st));
    for (int l = 0; l < 3; ++l) {
        const int N = P.N[l];
        if ((rc = T[l].get(c->pool, (size_t)K * N * 8))) return rc;
        launch_gather_terms(st, 8, (int)K, N, cols[l].p, N, idx_d.as<int32_t>() + (size_t)l * K,
                            l == 0 ? sc_d.as<double>() : nullptr, T[l].p, N);
    }
    DevBuf X[3], KR, Mr;
    int rmax2 = 0;
    for (int l = 0; l < 3; ++l) rmax2 = std::max(rmax2, r[(l + 1) % 3] * r[(l + 2) % 3]);
    for (int l = 0; l < 3; ++l)
        if ((rc = X[l].get(c->pool, (size_t)K * r[l] * 8))) return rc;
    if ((rc = KR.get(c->pool, (size_t)K * rmax2 * 8))) return rc;
    auto project = [&](int m) -> int {          // X_m (K x r_m) = T_m Z_m^T
        GemmArgs g{};
        g.m = (int)K; g.n = r[m]; g.k = P.N[m];
        g.A = T[m].p; g.sam = P.N[m]; g.sak = 1;
        g.B = q->Z[m].p; g.sbk = 1; g.sbn = P.N[m];
        g.C = X[m].p; g.scm = r[m]; g.scn = 1;
        g.alpha = 1.0; g.beta = 0.0; g.batch = 1;
        return gemm_auto(c, st, GEMM_F64, g);
    };
    for (int l = 0; l < 3; ++l)
        if ((rc = project(l))) return rc;
    for (int s = 0; s < P.als_sweeps; ++s) {
        double cn = 0.0;
        for (int l = 0; l < 3; ++l) {
            const int a = (l + 1) % 3, b = (l + 2) % 3, N = P.N[l], D = r[a] * r[b];
            launch_khatri_rao(st, (int)K, r[a], r[b], X[a].as<double>(), X[b].as<double>(), KR.as<double>());
            ModeSVD ms;
            if (N < D) {
                // Jacobi on the N rows of [M_l | I] with the Gram over M_l's columns: the rotated
                // identity block holds M_l's left singular vectors (unit rows)
                const long ld = (long)D + N;
                if ((rc = Mr.get(c->pool, (size_t)N * ld * 8))) return rc;
                LSUM_HIP(hipMemsetAsync(Mr.p, 0, (size_t)N * ld * 8, st));
                GemmArgs g{};
                g.m = N; g.n = D; g.k = (int)K;
                g.A = T[l].p; g.sam = 1; g.sak = N;
                g.B = KR.p; g.sbk = D; g.sbn = 1;
                g.C = Mr.p; g.scm = ld; g.scn = 1;
                g.alpha = 1.0; g.beta = 0.0; g.batch = 1;
                if ((rc = gemm_auto(c, st, GEMM_F64, g))) return rc;
                launch_unit_diag(st, N, ld, D, Mr.as<double>());
                DevBuf work;
                const size_t wb = jacobi_work_bytes(N, (int)ld);
                if ((rc = work.get(c->pool, wb))) return rc;
                JacobiRun jr = jacobi_run(c);
                rc = jacobi_svd(st, N, (int)ld, Mr.as<double>(), (int)ld, 1e-12, 0.0, 40, ms.sigma, &ms.sweeps,
                                work.as<double>(), wb, D, 0.0, &jr);
                if (rc) return rc;
                ms.rows = std::move(Mr);
                ms.ld = ld;
                ms.off = D;
                ms.unit = true;
            } else {
                if ((rc = Mr.get(c->pool, (size_t)D * N * 8))) return rc;
                GemmArgs g{};
                g.m = D; g.n = N; g.k = (int)K;
                g.A = KR.p; g.sam = 1; g.sak = D;
                g.B = T[l].p; g.sbk = N; g.sbn = 1;
                g.C = Mr.p; g.scm = N; g.scn = 1;
                g.alpha = 1.0; g.beta = 0.0; g.batch = 1;
                if ((rc = gemm_auto(c, st, GEMM_F64, g))) return rc;
                LSUM_HIP(hipStreamSynchronize(st));
                if ((rc = mode_svd(c, st, D, N, Mr, 0.0, 0.0, ms, false))) return rc;
            }
            LSUM_HIP(hipStreamSynchronize(st));
            double lead = 0.0;
            for (int k = 0; k < r[l] && k < (int)ms.sigma.size(); ++k) lead += ms.sigma[k] * ms.sigma[k];
            cn = std::sqrt(lead);
            if ((rc = rows_to_factor(c, st, ms, r[l], N, q->Z[l]))) return rc;
            if ((rc = project(l))) return rc;
        }
        q->als_core_norm.push_back(cn);
    }
    LSUM_HIP(hipStreamSynchronize(st));
    tm.end();
    return LSUM_OK;
}

// RHOSVD of one request whose canonical factors are computed (q->U, q->ref ready on st).
static int run_tucker(Request* q, hipStream_t st, const hipStream_t* aux, StageTimer& tm) {
    Context* c = q->ctx;
    const Plan& P = q->plan();
    int rc;
    const double* G = q->rows();
    // (4) side matrices per mode: lattice sources and defect windows (unnormalised)
    DevBuf cols[3], W[3], nrm[3], C[3];
    std::vector<double> nrm_h[3];
    const GemmPrec prec = gemm_prec(P.precision);
    tm.begin("columns", (double)(P.D[0] * (size_t)P.N[0] + P.D[1] * (size_t)P.N[1] + P.D[2] * (size_t)P.N[2]) * 8);
    for (int l = 0; l < 3; ++l) {
        const int D = P.D[l], N = P.N[l];
        if ((rc = cols[l].get(c->pool, (size_t)D * N * 8))) return rc;
        if ((rc = nrm[l].get(c->pool, (size_t)D * 8))) return rc;
        std::vector<const double*> latp(P.n_lat[l]);
        for (int s = 0; s < P.n_lat[l]; ++s) latp[s] = q->U[P.lat_block[l][s]].as<double>() + q->U_axis_off[l];
        DevBuf lp, wc;
        if ((rc = lp.get(c->pool, std::max<size_t>(1, latp.size()) * sizeof(void*)))) return rc;
        std::vector<int32_t> wo(P.win_cell[l].size());
        for (size_t w = 0; w < wo.size(); ++w) wo[w] = (int32_t)win_off(P, P.win_cls[l][w], P.win_cell[l][w]);
        if ((rc = wc.get(c->pool, std::max<size_t>(1, wo.size()) * 4))) return rc;
        LSUM_HIP(hipMemcpyAsync(lp.p, latp.data(), latp.size() * sizeof(void*), hipMemcpyHostToDevice, st));
        if (!wo.empty()) LSUM_HIP(hipMemcpyAsync(wc.p, wo.data(), wo.size() * 4, hipMemcpyHostToDevice, st));
        launch_gather_columns(st, P.R, P.n_lat[l], lp.as<const double*>(), P.N[l], P.n_win[l],
                              wc.as<int32_t>(), G, P.ldg, N, cols[l].as<double>(), N);
        launch_row_norms(st, D, N, cols[l].as<double>(), N, nrm[l].as<double>());
        nrm_h[l].resize(D);
        LSUM_HIP(hipMemcpyAsync(nrm_h[l].data(), nrm[l].p, D * 8, hipMemcpyDeviceToHost, st));
        LSUM_HIP(hipStreamSynchronize(st));   // lp, wc released after the kernels ran
    }
    tm.end();
    for (int l = 0; l < 3; ++l)
        for (double v : nrm_h[l])
            if (!(v > 0.0)) return fail(LSUM_E_INVALID, "a side-matrix column vanishes on the grid");

    // (5) ||A|| from the column Grams, ||xi|| from the norms, truncation (host FP64)
    tm.begin("norm", 0, 2.0 * ((double)P.D[0] * P.D[0] * P.N[0] + (double)P.D[1] * P.D[1] * P.N[1] + (double)P.D[2] * P.D[2] * P.N[2]));
    for (int l = 0; l < 3; ++l) {
        const int D = P.D[l], N = P.N[l];
        if ((rc = C[l].get(c->pool, (size_t)D * D * 8))) return rc;
        GemmArgs a{};
        a.m = D; a.n = D; a.k = N;
        a.A = cols[l].p; a.sam = N; a.sak = 1;
        a.B = cols[l].p; a.sbk = 1; a.sbn = N;
        a.C = C[l].p; a.scm = D; a.scn = 1;
        a.alpha = 1.0; a.beta = 0.0; a.batch = 1;
        if ((rc = gemm_auto(c, st, GEMM_F64, a))) return rc;
    }
    DevBuf src_d, scale_d, part_d;
    const int ng = P.n_groups;
    std::vector<int32_t> srcs(3 * (size_t)ng);
    for (int l = 0; l < 3; ++l) std::copy(P.g_src[l].begin(), P.g_src[l].end(), srcs.begin() + (size_t)l * ng);
    if ((rc = src_d.get(c->pool, srcs.size() * 4))) return rc;
    if ((rc = scale_d.get(c->pool, ng * 8))) return rc;
    if ((rc = part_d.get(c->pool, ng * 8))) return rc;
    LSUM_HIP(hipMemcpyAsync(src_d.p, srcs.data(), srcs.size() * 4, hipMemcpyHostToDevice, st));
    LSUM_HIP(hipMemcpyAsync(scale_d.p, P.g_scale.data(), ng * 8, hipMemcpyHostToDevice, st));
    const int32_t* s1 = src_d.as<int32_t>();
    const int32_t* s2 = s1 + ng;
    const int32_t* s3 = s2 + ng;
    launch_cp_norm2(st, P.R, ng, s1, s2, s3, scale_d.as<double>(), C[0].as<double>(), C[1].as<double>(),
                    C[2].as<double>(), P.D[0], P.D[1], P.D[2], part_d.as<double>(), ng);
    std::vector<double> part(ng);
    LSUM_HIP(hipMemcpyAsync(part.data(), part_d.p, ng * 8, hipMemcpyDeviceToHost, st));
    LSUM_HIP(hipStreamSynchronize(st));
    tm.end();
    for (int l = 0; l < 3; ++l) C[l].reset();
    double nA2 = 0.0;
    for (double v : part) nA2 += v;
    q->norm_A = std::sqrt(std::max(nA2, 0.0));
    double nxi2 = 0.0;
    for (int g = 0; g < ng; ++g)
        for (int k = 0; k < P.R; ++k) {
            double xi = P.g_scale[g];
            for (int l = 0; l < 3; ++l) xi *= nrm_h[l][(size_t)P.g_src[l][g] * P.R + k];
            nxi2 += xi * xi;
        }
    q->norm_xi = std::sqrt(nxi2);
    const double thr = P.eps * q->norm_A / (3.0 * q->norm_xi);
    // columns with norm below 1% of thr / sqrt(D) cannot change whether a tail passes thr
    const double irrelevant = 1e-2 * thr / std::sqrt((double)std::max(P.D[0], std::max(P.D[1], P.D[2])));
    // weighted, normalised side matrices: row j = col_j / |col_j| * sqrt(multiplicity)
    tm.begin("svd");
    ModeSVD ms[3];
    // the three modes are independent: with auxiliary streams they run concurrently (the block
    // Jacobi launches are far too small to fill the chip on their own)
    auto svd_one = [&](int l, hipStream_t s) -> int {
        int rc1;
        const int D = P.D[l], N = P.N[l];
        std::vector<double> sc(D);
        for (int j = 0; j < D; ++j) sc[j] = std::sqrt((double)P.src_mult[l][j / P.R]) / nrm_h[l][j];
        DevBuf scd;
        if ((rc1 = scd.get(c->pool, D * 8))) return rc1;
        if ((rc1 = W[l].get(c->pool, (size_t)D * N * 8))) return rc1;
        LSUM_HIP(hipMemcpyAsync(scd.p, sc.data(), D * 8, hipMemcpyHostToDevice, s));
        launch_scale_rows(s, D, N, cols[l].as<double>(), N, scd.as<double>(), W[l].as<double>(), N);
        if ((rc1 = mode_svd(c, s, D, N, W[l], thr, irrelevant, ms[l]))) return rc1;
        LSUM_HIP(hipStreamSynchronize(s));
        W[l].reset();
        return LSUM_OK;
    };
    int mrc[3] = {LSUM_OK, LSUM_OK, LSUM_OK};
    if (aux) {
        std::thread th[3];
        for (int l = 0; l < 3; ++l)
            th[l] = std::thread([&, l] {
                (void)hipSetDevice(c->device);
                FailStream fs(aux[l]);
                mrc[l] = svd_one(l, aux[l]);
            });
        for (auto& t : th) t.join();
    } else {
        for (int l = 0; l < 3; ++l) mrc[l] = svd_one(l, st);
    }
    double svd_flops = 0.0;
    for (int l = 0; l < 3; ++l) {
        if (mrc[l]) return fail(mrc[l], "SVD of mode " + std::to_string(l) + " failed");
        q->sigma[l] = ms[l].sigma;
        q->sweeps[l] = ms[l].sweeps;
        q->range_k[l] = ms[l].k;
        q->range_res[l] = std::sqrt(ms[l].res2);
        svd_flops += ms[l].flops;
        q->jacobi_persistent[l] = ms[l].persistent;
        q->jacobi_aborted[l] = ms[l].aborted;
        q->jacobi_tuned[l] = ms[l].tuned;
    }
    tm.work(0, svd_flops);
    tm.end();

    // certified truncation: tail(r)^2 = res2 + sum_{a >= r} sigma_a^2 <= thr^2
    q->bound = 0.0;
    for (int l = 0; l < 3; ++l) {
        const auto& sg = q->sigma[l];
        const int n = (int)sg.size();
        std::vector<double> tail(n + 1, 0.0);
        tail[n] = ms[l].res2;
        for (int k = n - 1; k >= 0; --k) tail[k] = tail[k + 1] + sg[k] * sg[k];
        int r = n;
        for (int k = 1; k <= n; ++k)
            if (std::sqrt(tail[k]) <= thr) { r = k; break; }
        r = std::min(r, P.N[l]);
        q->r[l] = r;
        q->tails[l] = std::sqrt(tail[r]);
        q->bound += q->tails[l];
    }
    q->bound *= q->norm_xi;

    // Tucker factors: the leading r singular vectors (rotated rows / sigma, or unit rows)
    for (int l = 0; l < 3; ++l) {
        const int r = q->r[l], N = P.N[l];
        std::vector<double> inv(r);
        std::vector<int32_t> ord(r);
        for (int a = 0; a < r; ++a) { inv[a] = ms[l].unit ? 1.0 : 1.0 / q->sigma[l][a]; ord[a] = a; }
        DevBuf od, iv;
        if ((rc = od.get(c->pool, r * 4))) return rc;
        if ((rc = iv.get(c->pool, r * 8))) return rc;
        if ((rc = q->Z[l].get(c->pool, (size_t)r * N * 8))) return rc;
        LSUM_HIP(hipMemcpyAsync(od.p, ord.data(), r * 4, hipMemcpyHostToDevice, st));
        LSUM_HIP(hipMemcpyAsync(iv.p, inv.data(), r * 8, hipMemcpyHostToDevice, st));
        launch_gather_scale_rows(st, r, N, ms[l].rows.as<double>() + ms[l].off, (int)ms[l].ld, od.as<int32_t>(),
                                 iv.as<double>(), q->Z[l].as<double>(), N);
        LSUM_HIP(hipStreamSynchronize(st));
        ms[l].rows.reset();
    }

    // (5b) optional ALS sweeps from the RHOSVD factors
    if (P.als_sweeps > 0 && (rc = run_als(q, st, cols, tm))) return rc;

    // (6) projections, stored transposed: Yt_l = cols_l Z_l^T (D_l x r_l, row stride ldy_l), in the
    // problem's precision
    const size_t es = (prec == GEMM_F64) ? 8 : 4;
    DevBuf Y[3];
    long ldy[3];
    tm.begin("projection", 0, 2.0 * ((double)q->r[0] * P.N[0] * P.D[0] + (double)q->r[1] * P.N[1] * P.D[1] + (double)q->r[2] * P.N[2] * P.D[2]));
    for (int l = 0; l < 3; ++l) {
        const int r = q->r[l], D = P.D[l], N = P.N[l];
        ldy[l] = (r + 3) / 4 * 4;
        if ((rc = Y[l].get(c->pool, (size_t)D * ldy[l] * es))) return rc;
        const void* Zp = q->Z[l].p;
        const void* Cp = cols[l].p;
        DevBuf Zf, Cf;
        if (prec != GEMM_F64) {
            if ((rc = Zf.get(c->pool, (size_t)r * N * 4))) return rc;
            if ((rc = Cf.get(c->pool, (size_t)D * N * 4))) return rc;
            launch_f64_to_f32(st, (long)r * N, q->Z[l].as<double>(), Zf.as<float>());
            launch_f64_to_f32(st, (long)D * N, cols[l].as<double>(), Cf.as<float>());
            Zp = Zf.p;
            Cp = Cf.p;
        }
        GemmArgs a{};
        a.m = D; a.n = r; a.k = N;
        a.A = Cp; a.sam = N; a.sak = 1;
        a.B = Zp; a.sbk = 1; a.sbn = N;
        a.C = Y[l].p; a.scm = ldy[l]; a.scn = 1;
        a.alpha = 1.0; a.beta = 0.0; a.batch = 1;
        if ((rc = gemm_auto(c, st, prec, a))) return rc;
        LSUM_HIP(hipStreamSynchronize(st));
    }
    tm.end();
    // the columns stay until the result's error has been probed against them (step 9)

    // (7) core mu = sum_nu xi_nu y1 (x) y2 (x) y3 (eq. C-core), unnormalised columns: xi = scale;
    // term tables nu = g R + q -> projection rows src_l(g) R + q and the group scale.  When the
    // terms share the columns of a mode m (defects on common lattice planes: D_m <= K / 2), the
    // terms of each such column j are summed first over the other two modes (u, v),
    // T[j] = sum_{nu: src_m = j} xi y_u (x) y_v, and the core is the product of T with Y_m over
    // the D_m columns: 2 r_u r_v (K + D_m r_m) flops instead of 2 r1 r2 r3 K.  The mode with the
    // fewest flops is taken (mode 2 only when it saves at least 5 %: its product is a batch of
    // r1 GEMMs rather than one).
    const long K = (long)ng * P.R;
    const int r1 = q->r[0], r2 = q->r[1], r3 = q->r[2];
    int gm = -1;
    double gflops = 2.0 * r1 * (double)r2 * r3 * (double)K;
    {
        double best[3];
        for (int m = 0; m < 3; ++m) {
            const double ru = q->r[m == 0 ? 1 : 0], rv = q->r[m == 2 ? 1 : 2];
            best[m] = 2L * P.D[m] <= K ? 2.0 * ru * rv * ((double)K + (double)P.D[m] * q->r[m]) : -1.0;
        }
        for (int m : {2, 0})
            if (best[m] >= 0 && (gm < 0 || best[m] < gflops)) { gm = m; gflops = best[m]; }
        if (best[1] >= 0 && (gm < 0 ? best[1] < gflops : best[1] < 0.95 * gflops)) { gm = 1; gflops = best[1]; }
    }
    q->core_mode = gm;
    tm.begin("core", 0, gflops);
    if (gm >= 0) {
        // the grouping mode m and the two others u < v
        const int m = gm, u = m == 0 ? 1 : 0, v = m == 2 ? 1 : 2;
        const int Dm = P.D[m], ru = q->r[u], rv = q->r[v];
        std::vector<int32_t> off(Dm + 1, 0), iu(K), iv(K);
        std::vector<double> scv(K);
        for (int g = 0; g < ng; ++g)
            for (int k = 0; k < P.R; ++k) ++off[P.g_src[m][g] * P.R + k + 1];
        for (int j = 0; j < Dm; ++j) off[j + 1] += off[j];
        std::vector<int32_t> pos(off.begin(), off.end() - 1);
        for (int g = 0; g < ng; ++g)
            for (int k = 0; k < P.R; ++k) {
                const int t = pos[P.g_src[m][g] * P.R + k]++;
                iu[t] = P.g_src[u][g] * P.R + k;
                iv[t] = P.g_src[v][g] * P.R + k;
                scv[t] = P.g_scale[g];
            }
        DevBuf off_d, iu_d, iv_d, sc_d;
        if ((rc = off_d.get(c->pool, off.size() * 4)) || (rc = iu_d.get(c->pool, (size_t)K * 4)) ||
            (rc = iv_d.get(c->pool, (size_t)K * 4)) || (rc = sc_d.get(c->pool, (size_t)K * 8)))
            return rc;
        LSUM_HIP(hipMemcpyAsync(off_d.p, off.data(), off.size() * 4, hipMemcpyHostToDevice, st));
        LSUM_HIP(hipMemcpyAsync(iu_d.p, iu.data(), (size_t)K * 4, hipMemcpyHostToDevice, st));
        LSUM_HIP(hipMemcpyAsync(iv_d.p, iv.data(), (size_t)K * 4, hipMemcpyHostToDevice, st));
        LSUM_HIP(hipMemcpyAsync(sc_d.p, scv.data(), (size_t)K * 8, hipMemcpyHostToDevice, st));
        const long plane = (long)r1 * r2 * r3;
        if ((rc = q->core.get(c->pool, (size_t)plane * es))) return rc;
        // T in chunks of mode-u rows x (at most 2 GiB each, every column j up to the launch
        // limit), laid out T[j][x - x0][y]: each chunk's product runs over all D_m columns and
        // writes its part of the core once (chunks of columns instead re-read and re-wrote the
        // whole core for every chunk)
        const long per_x = (long)rv * Dm * (long)es;
        const int x_chunk = (int)std::max<long>(1, std::min<long>((long)ru, (2L << 30) / per_x));
        const int j_chunk = std::min(Dm, 65535);
        DevBuf Tb;
        if ((rc = Tb.get(c->pool, (size_t)x_chunk * rv * (size_t)j_chunk * es))) return rc;
        for (int x0 = 0; x0 < ru; x0 += x_chunk) {
            const int nx = std::min(x_chunk, ru - x0);
            for (int j0 = 0; j0 < Dm; j0 += j_chunk) {
                const int nj = std::min(j_chunk, Dm - j0);
                launch_core_groups(st, (int)es, ru, rv, x0, nx, j0, nj, off_d.as<int32_t>(), iu_d.as<int32_t>(),
                                   iv_d.as<int32_t>(), sc_d.as<double>(), Y[u].p, ldy[u], Y[v].p, ldy[v], Tb.p);
                const char* Ym = (const char*)Y[m].p + (size_t)j0 * ldy[m] * es;   // Y_m[j][idx_m]
                GemmArgs a{};
                a.alpha = 1.0; a.beta = j0 == 0 ? 0.0 : 1.0; a.batch = 1;
                if (m == 2) {
                    // core[(x, y)][c] = sum_j T[j][(x, y)] Y3[j][c]: rows x0.. of the core
                    a.m = nx * r2; a.n = r3; a.k = nj;
                    a.A = Tb.p; a.sam = 1; a.sak = (long)nx * r2;
                    a.B = Ym; a.sbk = ldy[2]; a.sbn = 1;
                    a.C = (char*)q->core.p + (size_t)x0 * r2 * r3 * es; a.scm = r3; a.scn = 1;
                } else if (m == 0) {
                    // core[a][(x, y)] = sum_j Y1[j][a] T[j][(x, y)]: columns x0 r3.. of every row a
                    a.m = r1; a.n = nx * r3; a.k = nj;
                    a.A = Ym; a.sam = 1; a.sak = ldy[0];
                    a.B = Tb.p; a.sbk = (long)nx * r3; a.sbn = 1;
                    a.C = (char*)q->core.p + (size_t)x0 * r3 * es; a.scm = (long)r2 * r3; a.scn = 1;
                } else {
                    // core[x][b][y] = sum_j Y2[j][b] T[j][x][y]: one product per x (Y2 shared)
                    a.m = r2; a.n = r3; a.k = nj;
                    a.A = Ym; a.sam = 1; a.sak = ldy[1]; a.bA = 0;
                    a.B = Tb.p; a.sbk = (long)nx * r3; a.sbn = 1; a.bB = r3;
                    a.C = (char*)q->core.p + (size_t)x0 * r2 * r3 * es; a.scm = r3; a.scn = 1;
                    a.bC = (long)r2 * r3;
                    a.batch = nx;
                }
                launch_gemm(st, prec, a);
            }
        }
        LSUM_HIP(hipGetLastError());
        LSUM_HIP(hipStreamSynchronize(st));
        q->bytes["core"] = (double)plane * es;
    } else {
        std::vector<int32_t> idx(3 * (size_t)K);
        std::vector<double> scv(K);
        for (int g = 0; g < ng; ++g)
            for (int k = 0; k < P.R; ++k) {
                const long nu = (long)g * P.R + k;
                for (int l = 0; l < 3; ++l) idx[(size_t)l * K + nu] = P.g_src[l][g] * P.R + k;
                scv[nu] = P.g_scale[g];
            }
        DevBuf idx_d, sc_d;
        if ((rc = idx_d.get(c->pool, idx.size() * 4))) return rc;
        if ((rc = sc_d.get(c->pool, K * 8))) return rc;
        LSUM_HIP(hipMemcpyAsync(idx_d.p, idx.data(), idx.size() * 4, hipMemcpyHostToDevice, st));
        LSUM_HIP(hipMemcpyAsync(sc_d.p, scv.data(), K * 8, hipMemcpyHostToDevice, st));
        // term-major operands X_l (K x ldy_l), the group scale folded into mode 1
        DevBuf X[3];
        for (int l = 0; l < 3; ++l) {
            if ((rc = X[l].get(c->pool, (size_t)K * ldy[l] * es))) return rc;
            launch_gather_terms(st, (int)es, (int)K, q->r[l], Y[l].p, ldy[l], idx_d.as<int32_t>() + (size_t)l * K,
                                l == 0 ? sc_d.as<double>() : nullptr, X[l].p, ldy[l]);
        }
        const long plane = (long)q->r[0] * q->r[1] * q->r[2];
        if ((rc = q->core.get(c->pool, (size_t)plane * es))) return rc;
        CoreArgs ca{};
        ca.r1 = q->r[0]; ca.r2 = q->r[1]; ca.r3 = q->r[2]; ca.K = (int)K;
        ca.X1 = X[0].p; ca.X2 = X[1].p; ca.X3 = X[2].p;
        ca.ldx1 = ldy[0]; ca.ldx2 = ldy[1]; ca.ldx3 = ldy[2];
        ca.core = q->core.p;
        // enough workgroups for the chip: split the terms when the output has few tiles
        const long tiles = (long)((ca.r3 + 63) / 64) * ((ca.r1 + 7) / 8) * ((ca.r2 + 15) / 16);
        int ks = 1;
        while (tiles * ks < 2048 && ks < 64 && K / (ks * 2) >= 512) ks *= 2;
        DevBuf work;
        if (ks > 1 && (rc = work.get(c->pool, (size_t)plane * ks * es))) return rc;
        launch_core(st, prec, ca, ks, work.p);
        LSUM_HIP(hipGetLastError());
        LSUM_HIP(hipStreamSynchronize(st));
        q->bytes["core"] = (double)plane * es;
    }
    tm.end();

    // (8) optional tile
    if (P.has_tile() && (rc = make_tile(q, st, tm))) return rc;
    LSUM_HIP(hipStreamSynchronize(st));

    // (9) the result's own error: its values at kProbeCells seeded cells, evaluated like any
    // sample (in the request's precision), against the untruncated canonical sum in FP64.  The
    // cells lie on kProbePlanes mode-3 planes (random along the other two axes), so that the
    // evaluation forms only that many mode-3 products of the core.
    {
        const int np = kProbeCells;
        std::vector<int32_t> cells(3 * (size_t)np);
        std::vector<double> xyz(3 * (size_t)np);
        uint64_t state = 0x1411199400000000ull ^ ((uint64_t)P.N[0] << 40) ^ ((uint64_t)P.N[1] << 20) ^ (uint64_t)P.N[2];
        auto next = [&state](int n) {
            // SplitMix64 (Steele, Lea, Flood 2014) of a counter
            uint64_t z = (state += 0x9E3779B97F4A7C15ull);
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            z ^= z >> 31;
            return (int)(z % (uint64_t)n);
        };
        int planes[kProbePlanes];
        for (int k = 0; k < kProbePlanes; ++k) planes[k] = next(P.N[2]);
        for (int p = 0; p < np; ++p)
            for (int l = 0; l < 3; ++l) {
                const int i = l == 2 ? planes[p % kProbePlanes] : next(P.N[l]);
                cells[3 * p + l] = i;
                xyz[3 * p + l] = (i - (P.N[l] - 1) / 2) * P.h;
            }
        if (!cols[0].p || !cols[1].p || !cols[2].p || !src_d.p || !scale_d.p)
            return fail(LSUM_E_STATE, "probe: the side-matrix columns or term tables were released");
        DevBuf cd, xd, vt, vc;
        if ((rc = cd.get(c->pool, cells.size() * 4)) || (rc = xd.get(c->pool, xyz.size() * 8)) ||
            (rc = vt.get(c->pool, (size_t)np * 8)) || (rc = vc.get(c->pool, (size_t)np * 8)))
            return rc;
        LSUM_HIP(hipMemcpyAsync(cd.p, cells.data(), cells.size() * 4, hipMemcpyHostToDevice, st));
        LSUM_HIP(hipMemcpyAsync(xd.p, xyz.data(), xyz.size() * 8, hipMemcpyHostToDevice, st));
        tm.begin("probe");
        launch_probe_canonical(st, np, P.R, ng, s1, s2, s3, scale_d.as<double>(), cols[0].as<double>(),
                               cols[1].as<double>(), cols[2].as<double>(), P.N[0], P.N[1], P.N[2],
                               cd.as<int32_t>(), vc.as<double>());
        double fl = 0.0;
        if ((rc = sample_points(q, st, np, xd.as<double>(), vt.as<double>(), nullptr, &fl))) return rc;
        tm.work(0, fl);
        tm.end();
        std::vector<double> a(np), b(np);
        LSUM_HIP(hipMemcpyAsync(a.data(), vt.p, (size_t)np * 8, hipMemcpyDeviceToHost, st));
        LSUM_HIP(hipMemcpyAsync(b.data(), vc.p, (size_t)np * 8, hipMemcpyDeviceToHost, st));
        LSUM_HIP(hipStreamSynchronize(st));
        double dmax = 0.0, vmax = 0.0;
        for (int p = 0; p < np; ++p) {
            dmax = std::max(dmax, std::fabs(a[p] - b[p]));
            vmax = std::max(vmax, std::fabs(b[p]));
        }
        q->probe_err = vmax > 0.0 ? dmax / vmax : dmax;
        q->n_probe = np;
        q->probe_cells = cells;
    }
    for (int l = 0; l < 3; ++l) cols[l].reset();
    return LSUM_OK;
}

// Orthonormal rows Q (D x N) spanning the rows of F by CholeskyQR2: twice G = F F^T (MFMA GEMM),
// G = L L^T (host), F <- L^-1 F.  *ok is false (and Q unset) when a Cholesky pivot ratio falls
// below 1e-7 (F too close to rank deficient for this route).
static int chol_qr2(Context* c, hipStream_t st, int D, int N, const double* F, DevBuf& Q, bool* ok) {
    int rc;
    *ok = false;
    DevBuf Gd, Ld, Q1;
    if ((rc = Gd.get(c->pool, (size_t)D * D * 8)) || (rc = Ld.get(c->pool, (size_t)D * D * 8))) return rc;
    if ((rc = Q1.get(c->pool, (size_t)D * N * 8))) return rc;
    const double* src = F;
    std::vector<double> G((size_t)D * D), Li((size_t)D * D);
    for (int pass = 0; pass < 2; ++pass) {
        GemmArgs a{};
        a.m = D; a.n = D; a.k = N;
        a.A = src; a.sam = N; a.sak = 1;
        a.B = src; a.sbk = 1; a.sbn = N;
        a.C = Gd.p; a.scm = D; a.scn = 1;
        a.alpha = 1.0; a.beta = 0.0; a.batch = 1;
        if ((rc = gemm_auto(c, st, GEMM_F64, a))) return rc;
        LSUM_HIP(hipMemcpyAsync(G.data(), Gd.p, G.size() * 8, hipMemcpyDeviceToHost, st));
        LSUM_HIP(hipStreamSynchronize(st));
        // Cholesky in place (lower), then the inverse of L by forward substitution
        double dmax = 0.0, dmin = INFINITY;
        for (int j = 0; j < D; ++j) {
            double d = G[(size_t)j * D + j];
            for (int k = 0; k < j; ++k) d -= G[(size_t)j * D + k] * G[(size_t)j * D + k];
            if (!(d > 0.0)) return LSUM_OK;
            d = std::sqrt(d);
            G[(size_t)j * D + j] = d;
            dmax = std::max(dmax, d);
            dmin = std::min(dmin, d);
            for (int i = j + 1; i < D; ++i) {
                double v = G[(size_t)i * D + j];
                for (int k = 0; k < j; ++k) v -= G[(size_t)i * D + k] * G[(size_t)j * D + k];
                G[(size_t)i * D + j] = v / d;
            }
        }
        if (dmin < 1e-7 * dmax) return LSUM_OK;
        std::fill(Li.begin(), Li.end(), 0.0);
        for (int j = 0; j < D; ++j) {
            Li[(size_t)j * D + j] = 1.0 / G[(size_t)j * D + j];
            for (int i = j + 1; i < D; ++i) {
                double v = 0.0;
                for (int k = j; k < i; ++k) v -= G[(size_t)i * D + k] * Li[(size_t)k * D + j];
                Li[(size_t)i * D + j] = v / G[(size_t)i * D + i];
            }
        }
        LSUM_HIP(hipMemcpyAsync(Ld.p, Li.data(), Li.size() * 8, hipMemcpyHostToDevice, st));
        DevBuf& dst = pass == 0 ? Q1 : Q;
        if (pass == 1 && (rc = Q.get(c->pool, (size_t)D * N * 8))) return rc;
        a = GemmArgs{};
        a.m = D; a.n = N; a.k = D;
        a.A = Ld.p; a.sam = D; a.sak = 1;
        a.B = src; a.sbk = N; a.sbn = 1;
        a.C = dst.p; a.scm = N; a.scn = 1;
        a.alpha = 1.0; a.beta = 0.0; a.batch = 1;
        launch_gemm(st, GEMM_F64, a);
        LSUM_HIP(hipStreamSynchronize(st));   // Ld is rewritten by the next pass
        src = Q1.as<double>();
    }
    *ok = true;
    return LSUM_OK;
}

// mu (k1 x k2 x k3) += scale * B x_1 C1 x_2 C2 x_3 C3 for B (s1 x s2 x s3, last index fastest):
// mu[a,e,f] += scale sum_{i,j,k} B[i,j,k] C1[a, o1 + i] C2[e, o2 + j] C3[f, o3 + k], C_l row-major
// with row stride ld_l (host FP64; the sizes are a few tens per mode).
static void add_mode_products(const double* B, int s1, int s2, int s3, const double* C1, int ld1, int o1,
                              const double* C2, int ld2, int o2, const double* C3, int ld3, int o3, int k1, int k2,
                              int k3, double scale, double* mu) {
    std::vector<double> X((size_t)k1 * s2 * s3, 0.0), Y((size_t)k1 * k2 * s3, 0.0);
    for (int a = 0; a < k1; ++a)
        for (int i = 0; i < s1; ++i) {
            const double cf = C1[(size_t)a * ld1 + o1 + i];
            const double* Bi = B + (size_t)i * s2 * s3;
            double* Xa = &X[(size_t)a * s2 * s3];
            for (int jk = 0; jk < s2 * s3; ++jk) Xa[jk] += cf * Bi[jk];
        }
    for (int a = 0; a < k1; ++a)
        for (int e = 0; e < k2; ++e)
            for (int j = 0; j < s2; ++j) {
                const double cf = C2[(size_t)e * ld2 + o2 + j];
                const double* Xj = &X[((size_t)a * s2 + j) * s3];
                double* Ye = &Y[((size_t)a * k2 + e) * s3];
                for (int k = 0; k < s3; ++k) Ye[k] += cf * Xj[k];
            }
    for (size_t ae = 0; ae < (size_t)k1 * k2; ++ae)
        for (int f = 0; f < k3; ++f) {
            const double* c3 = C3 + (size_t)f * ld3 + o3;
            const double* Ya = &Y[ae * s3];
            double acc = 0.0;
            for (int k = 0; k < s3; ++k) acc += c3[k] * Ya[k];
            mu[ae * k3 + f] += scale * acc;
        }
}

// Orthonormal rows Q (k x N) spanning the D rows of F: CholeskyQR2 (k = D), or, when the rows are
// close to dependent, the SVD with every direction above 1e-13 of ||F|| kept.
static int orthonormal_rows(Context* c, hipStream_t st, int D, int N, const double* F, DevBuf& Q, int* k) {
    int rc;
    bool ok = false;
    if ((rc = chol_qr2(c, st, D, N, F, Q, &ok))) return rc;
    if (ok) {
        *k = D;
        return LSUM_OK;
    }
    DevBuf W, nrm;
    if ((rc = W.get(c->pool, (size_t)D * N * 8)) || (rc = nrm.get(c->pool, (size_t)D * 8))) return rc;
    LSUM_HIP(hipMemcpyAsync(W.p, F, (size_t)D * N * 8, hipMemcpyDeviceToDevice, st));
    launch_row_norms(st, D, N, F, N, nrm.as<double>());
    std::vector<double> nh(D);
    LSUM_HIP(hipMemcpyAsync(nh.data(), nrm.p, D * 8, hipMemcpyDeviceToHost, st));
    LSUM_HIP(hipStreamSynchronize(st));
    double f2 = 0.0;
    for (double v : nh) f2 += v * v;
    const double thr = 1e-13 * std::sqrt(f2);
    ModeSVD ms;
    if ((rc = mode_svd(c, st, D, N, W, thr, 1e-2 * thr / std::sqrt((double)D), ms))) return rc;
    LSUM_HIP(hipStreamSynchronize(st));
    const int n = (int)ms.sigma.size();
    std::vector<double> tail(n + 1, 0.0);
    tail[n] = ms.res2;
    for (int j = n - 1; j >= 0; --j) tail[j] = tail[j + 1] + ms.sigma[j] * ms.sigma[j];
    int r = n;
    for (int j = 1; j <= n; ++j)
        if (std::sqrt(tail[j]) <= thr) { r = j; break; }
    r = std::max(1, std::min(r, N));
    *k = r;
    return rows_to_factor(c, st, ms, r, N, Q);
}

// ------------------------------------------------------------------------------------------
// Tucker-reference sum (Thm thm:sumCaseE (B)): the rank-r Tucker form of the reference, its
// vectors assembled over the lattice, orthonormalised per mode
// ------------------------------------------------------------------------------------------
static int run_tucker_ref(Request* q, hipStream_t st, const hipStream_t* aux, StageTimer& tm) {
    Context* c = q->ctx;
    const Plan& P = q->plan();
    const int nb = (int)P.blocks.size();
    int rc;
    // (1)-(2) the reference's Tucker form (cached per kernel, quadrature, grid and eps): RHOSVD at
    // eps of one unit charge in the centre cell of the doubled box (2 N_ref - 1 cells per axis,
    // cell m at displacement (m - (N_ref - 1)) h), with this plan's kernel, step and scale; its
    // vectors kept as zero-padded rows of ldg (>= 2 N_ref) for the shift-sum
    auto make = [&](RefEntry& e) -> int {
        Request rq;
        rq.ctx = c;
        lsum_problem rp{};
        rp.kernel = P.kernel;
        rp.kernel.h_u = P.h_u;
        rp.kernel.s = P.s;
        const int Nd = 2 * P.N_ref - 1;
        rp.N[0] = rp.N[1] = rp.N[2] = Nd;
        rp.h = P.h;
        lsum_block one{};
        for (int l = 0; l < 3; ++l) one.L[l] = 1, one.b[l] = 1.0, one.center[l] = 0.0;
        one.charge = 1.0;
        rp.n_blocks = 1;
        rp.blocks = &one;
        rp.eps = P.eps;
        rp.precision = LSUM_FP64;
        rp.als_sweeps = P.als_sweeps;
        auto rplan = std::make_shared<Plan>();
        int rc1 = make_plan(rp, *rplan);
        if (rc1) return rc1;
        rq.plan_sp = rplan;
        std::vector<Request*> rb{&rq};
        rc1 = run_batch(rb, st, aux);
        drop_reference(&rq);
        if (rc1) return rc1;
        if (rq.status.load() < 0) return rq.status.load();
        const size_t tab = (size_t)P.R * P.ldg;
        LSUM_HIP(hipMemsetAsync(e.G.p, 0, 3 * tab * 8, st));
        for (int l = 0; l < 3; ++l) {
            e.r[l] = rq.r[l];
            LSUM_HIP(hipMemcpy2DAsync(e.G.as<double>() + l * tab, (size_t)P.ldg * 8, rq.Z[l].p, (size_t)Nd * 8,
                                      (size_t)Nd * 8, rq.r[l], hipMemcpyDeviceToDevice, st));
        }
        e.core.resize((size_t)rq.r[0] * rq.r[1] * rq.r[2]);
        LSUM_HIP(hipMemcpyAsync(e.core.data(), rq.core.p, e.core.size() * 8, hipMemcpyDeviceToHost, st));
        LSUM_HIP(hipStreamSynchronize(st));
        e.norm_A = rq.norm_A;
        e.norm_xi = rq.norm_xi;
        e.bound = rq.bound;
        return LSUM_OK;
    };
    std::shared_ptr<RefEntry> tr;
    if ((rc = get_tucker_ref(c, P, st, make, tr))) return rc;
    struct Unuse {
        std::shared_ptr<RefEntry>& e;
        ~Unuse() { e->users.fetch_sub(1); }
    } unuse{tr};
    const int rr[3] = {tr->r[0], tr->r[1], tr->r[2]};
    q->norm_A = tr->norm_A;               // of the reference tensor: the certified bound is the reference's
    q->norm_xi = tr->norm_xi;
    q->bound = tr->bound;
    tm.begin("assemble");
    const double* Zr[3];
    for (int l = 0; l < 3; ++l) Zr[l] = tr->G.as<double>() + (size_t)l * P.R * P.ldg;
    // (3) assembled Tucker vectors: per block and axis the shift-sum of the r_l reference rows
    // over the block's sites (combs through window sums of those rows), stacked block after block
    // as the rows of F_l ((nb r_l) x N_l)
    DevBuf F[3];
    for (int l = 0; l < 3; ++l)
        if ((rc = F[l].get(c->pool, (size_t)nb * rr[l] * P.N[l] * 8))) return rc;
    std::map<std::tuple<int, int, int>, DevBuf> wins;   // (axis, stride, n) -> window sums
    auto windows = [&](int l, int S, int n, const double** out) -> int {
        auto key = std::make_tuple(l, S, n);
        auto it = wins.find(key);
        if (it == wins.end()) {
            DevBuf w;
            int rc1 = w.get(c->pool, (size_t)rr[l] * P.ldg * 8);
            if (rc1) return rc1;
            launch_window_sums(st, rr[l], Zr[l], P.ldg, S, n, w.as<double>());
            it = wins.emplace(key, std::move(w)).first;
        }
        *out = it->second.as<double>();
        return LSUM_OK;
    };
    std::vector<ShiftJob> jobs;
    std::vector<int2> terms_h, tv;
    std::vector<size_t> term_off;
    int maxN = 0, maxR = 0;
    for (int b = 0; b < nb; ++b)
        for (int l = 0; l < 3; ++l) {
            const auto& sites = P.offs[l][b];
            int stride = 0, n_tab[2] = {0, 0};
            bool two = false;
            shift_terms(sites.data(), (int)sites.size(), P.N_ref, P.N[l], P.ldg, tv, &stride, n_tab, &two);
            ShiftJob j{};
            j.T0 = Zr[l];
            if (stride > 0) {
                if ((rc = windows(l, stride, n_tab[0], &j.T0))) return rc;
                if (two && (rc = windows(l, stride, n_tab[1], &j.T1))) return rc;
            }
            term_off.push_back(terms_h.size());
            terms_h.insert(terms_h.end(), tv.begin(), tv.end());
            j.n_terms = (int)tv.size();
            j.U = F[l].as<double>() + (size_t)b * rr[l] * P.N[l];
            j.ldu = P.N[l];
            j.N_axis = P.N[l];
            j.ldg = P.ldg;
            j.R = rr[l];
            jobs.push_back(j);
            maxN = std::max(maxN, P.N[l]);
            maxR = std::max(maxR, rr[l]);
        }
    DevBuf terms_d, jobs_d;
    if ((rc = terms_d.get(c->pool, std::max<size_t>(1, terms_h.size()) * sizeof(int2)))) return rc;
    if ((rc = jobs_d.get(c->pool, jobs.size() * sizeof(ShiftJob)))) return rc;
    for (size_t k = 0; k < jobs.size(); ++k) jobs[k].terms = terms_d.as<int2>() + term_off[k];
    LSUM_HIP(hipMemcpyAsync(terms_d.p, terms_h.data(), terms_h.size() * sizeof(int2), hipMemcpyHostToDevice, st));
    LSUM_HIP(hipMemcpyAsync(jobs_d.p, jobs.data(), jobs.size() * sizeof(ShiftJob), hipMemcpyHostToDevice, st));
    launch_shift_sum(st, jobs_d.as<ShiftJob>(), (int)jobs.size(), maxN, maxR);
    LSUM_HIP(hipGetLastError());
    LSUM_HIP(hipStreamSynchronize(st));   // the job tables and window sums are released below
    tm.end();

    // (4) per block and mode an orthonormal basis Q_b,l of the assembled vectors (the Gram-Schmidt
    // step after Thm thm:sumCaseE), and the block's core B_b = charge_b B x_l C_b,l with
    // C_b,l = Q_b,l F_b,l^T (its triangular factor)
    tm.begin("svd");
    const double* Bref = tr->core.data();
    std::vector<DevBuf> Qb((size_t)nb * 3);
    std::vector<int> kb((size_t)nb * 3);
    std::vector<std::vector<double>> Bb(nb);
    int kbl[3] = {0, 0, 0};          // stacked rows per mode
    for (int b = 0; b < nb; ++b) {
        std::vector<double> Cb[3];
        for (int l = 0; l < 3; ++l) {
            const int N = P.N[l];
            const double* Fb = F[l].as<double>() + (size_t)b * rr[l] * N;
            int k = 0;
            if ((rc = orthonormal_rows(c, st, rr[l], N, Fb, Qb[b * 3 + l], &k))) return rc;
            kb[b * 3 + l] = k;
            kbl[l] += k;
            DevBuf Cd;
            if ((rc = Cd.get(c->pool, (size_t)k * rr[l] * 8))) return rc;
            GemmArgs a{};
            a.m = k; a.n = rr[l]; a.k = N;
            a.A = Qb[b * 3 + l].p; a.sam = N; a.sak = 1;
            a.B = Fb; a.sbk = 1; a.sbn = N;
            a.C = Cd.p; a.scm = rr[l]; a.scn = 1;
            a.alpha = 1.0; a.beta = 0.0; a.batch = 1;
            if ((rc = gemm_auto(c, st, GEMM_F64, a))) return rc;
            Cb[l].resize((size_t)k * rr[l]);
            LSUM_HIP(hipMemcpyAsync(Cb[l].data(), Cd.p, Cb[l].size() * 8, hipMemcpyDeviceToHost, st));
            LSUM_HIP(hipStreamSynchronize(st));
        }
        const int k1 = kb[b * 3], k2 = kb[b * 3 + 1], k3 = kb[b * 3 + 2];
        Bb[b].assign((size_t)k1 * k2 * k3, 0.0);
        add_mode_products(Bref, rr[0], rr[1], rr[2], Cb[0].data(), rr[0], 0, Cb[1].data(), rr[1], 0, Cb[2].data(),
                          rr[2], 0, k1, k2, k3, P.blocks[b].charge, Bb[b].data());
    }
    std::vector<double> mu;
    if (nb == 1) {
        for (int l = 0; l < 3; ++l) {
            q->r[l] = kb[l];
            q->Z[l] = std::move(Qb[l]);
            q->sigma[l].clear();
            q->tails[l] = 0.0;
        }
        mu = std::move(Bb[0]);
        double n2 = 0.0;
        for (double v : mu) n2 += v * v;
        q->norm_A = std::sqrt(n2);
        q->norm_xi = q->norm_A;
        q->bound = 0.0;
        tm.end();
    } else {
        // (5) several blocks: the generalised RHOSVD of their Tucker sum (Thm thm:TSum2Tucker).
        // Stacked side rows per mode (eq. SideMTuckS), their Gram, ||U||^2 = sum_{b,b'} <T_b, T_b'>
        // from the cross Grams, |B|^2 = sum_b ||B_b||^2, per mode the smallest rank whose tail is
        // <= eps ||U|| / (3 |B|), and the core by projection: mu = sum_b B_b x_l (Z_l Q_b,l^T)
        DevBuf S[3];
        std::vector<int> off((size_t)nb * 3);
        std::vector<double> G[3];
        for (int l = 0; l < 3; ++l) {
            const int N = P.N[l], K = kbl[l];
            if ((rc = S[l].get(c->pool, (size_t)K * N * 8))) return rc;
            int o = 0;
            for (int b = 0; b < nb; ++b) {
                off[b * 3 + l] = o;
                LSUM_HIP(hipMemcpyAsync(S[l].as<double>() + (size_t)o * N, Qb[b * 3 + l].p,
                                        (size_t)kb[b * 3 + l] * N * 8, hipMemcpyDeviceToDevice, st));
                o += kb[b * 3 + l];
            }
            DevBuf Gd;
            if ((rc = Gd.get(c->pool, (size_t)K * K * 8))) return rc;
            GemmArgs a{};
            a.m = K; a.n = K; a.k = N;
            a.A = S[l].p; a.sam = N; a.sak = 1;
            a.B = S[l].p; a.sbk = 1; a.sbn = N;
            a.C = Gd.p; a.scm = K; a.scn = 1;
            a.alpha = 1.0; a.beta = 0.0; a.batch = 1;
            if ((rc = gemm_auto(c, st, GEMM_F64, a))) return rc;
            G[l].resize((size_t)K * K);
            LSUM_HIP(hipMemcpyAsync(G[l].data(), Gd.p, G[l].size() * 8, hipMemcpyDeviceToHost, st));
            LSUM_HIP(hipStreamSynchronize(st));
        }
        double n2 = 0.0, bh2 = 0.0;
        for (int b = 0; b < nb; ++b) {
            for (double v : Bb[b]) bh2 += v * v;
            for (int e = 0; e < nb; ++e) {
                // <T_b, T_e> = sum B_b[i,j,k] B_e[i',j',k'] G1[i,i'] G2[j,j'] G3[k,k']: B_e x_l (G_l blocks)
                const int i1 = kb[b * 3], i2 = kb[b * 3 + 1], i3 = kb[b * 3 + 2];
                std::vector<double> T((size_t)i1 * i2 * i3, 0.0);
                add_mode_products(Bb[e].data(), kb[e * 3], kb[e * 3 + 1], kb[e * 3 + 2],
                                  G[0].data() + (size_t)off[b * 3] * kbl[0], kbl[0], off[e * 3],
                                  G[1].data() + (size_t)off[b * 3 + 1] * kbl[1], kbl[1], off[e * 3 + 1],
                                  G[2].data() + (size_t)off[b * 3 + 2] * kbl[2], kbl[2], off[e * 3 + 2], i1, i2, i3,
                                  1.0, T.data());
                for (size_t x = 0; x < T.size(); ++x) n2 += Bb[b][x] * T[x];
            }
        }
        const double normU = std::sqrt(std::max(n2, 0.0)), Bhat = std::sqrt(bh2);
        const double thr = P.eps * normU / (3.0 * Bhat);
        q->norm_A = normU;
        q->norm_xi = Bhat;
        q->bound = 0.0;
        std::vector<double> Cp[3];
        for (int l = 0; l < 3; ++l) {
            const int N = P.N[l], K = kbl[l];
            DevBuf W;
            if ((rc = W.get(c->pool, (size_t)K * N * 8))) return rc;
            LSUM_HIP(hipMemcpyAsync(W.p, S[l].p, (size_t)K * N * 8, hipMemcpyDeviceToDevice, st));
            ModeSVD ms;
            if ((rc = mode_svd(c, st, K, N, W, thr, 1e-2 * thr / std::sqrt((double)K), ms))) return rc;
            LSUM_HIP(hipStreamSynchronize(st));
            const auto& sg = ms.sigma;
            const int n = (int)sg.size();
            std::vector<double> tail(n + 1, 0.0);
            tail[n] = ms.res2;
            for (int k = n - 1; k >= 0; --k) tail[k] = tail[k + 1] + sg[k] * sg[k];
            int r = n;
            for (int k = 1; k <= n; ++k)
                if (std::sqrt(tail[k]) <= thr) { r = k; break; }
            r = std::max(1, std::min(r, N));
            q->r[l] = r;
            q->sigma[l] = sg;
            q->sweeps[l] = ms.sweeps;
            q->tails[l] = std::sqrt(tail[r]);
            q->bound += q->tails[l];
            if ((rc = rows_to_factor(c, st, ms, r, N, q->Z[l]))) return rc;
            DevBuf Cd;
            if ((rc = Cd.get(c->pool, (size_t)r * K * 8))) return rc;
            GemmArgs a{};
            a.m = r; a.n = K; a.k = N;
            a.A = q->Z[l].p; a.sam = N; a.sak = 1;
            a.B = S[l].p; a.sbk = 1; a.sbn = N;
            a.C = Cd.p; a.scm = K; a.scn = 1;
            a.alpha = 1.0; a.beta = 0.0; a.batch = 1;
            if ((rc = gemm_auto(c, st, GEMM_F64, a))) return rc;
            Cp[l].resize((size_t)r * K);
            LSUM_HIP(hipMemcpyAsync(Cp[l].data(), Cd.p, Cp[l].size() * 8, hipMemcpyDeviceToHost, st));
            LSUM_HIP(hipStreamSynchronize(st));
        }
        q->bound *= Bhat;
        tm.end();
        tm.begin("core");
        mu.assign((size_t)q->r[0] * q->r[1] * q->r[2], 0.0);
        for (int b = 0; b < nb; ++b)
            add_mode_products(Bb[b].data(), kb[b * 3], kb[b * 3 + 1], kb[b * 3 + 2], Cp[0].data(), kbl[0],
                              off[b * 3], Cp[1].data(), kbl[1], off[b * 3 + 1], Cp[2].data(), kbl[2], off[b * 3 + 2],
                              q->r[0], q->r[1], q->r[2], 1.0, mu.data());
        tm.end();
    }
    if ((rc = q->core.get(c->pool, mu.size() * 8))) return rc;
    LSUM_HIP(hipMemcpyAsync(q->core.p, mu.data(), mu.size() * 8, hipMemcpyHostToDevice, st));
    LSUM_HIP(hipStreamSynchronize(st));
    q->bytes["core"] = (double)mu.size() * 8;
    if (P.has_tile() && (rc = make_tile(q, st, tm))) return rc;
    return LSUM_OK;
}

// ------------------------------------------------------------------------------------------
// sampling: canonical factors (point-major rows, plus defect windows from the reference), or
// the Tucker tensor (mode-3 contraction as a GEMM per chunk of points, then modes 1 and 2)
// ------------------------------------------------------------------------------------------
// Canonical requests of a batch: one launch per factor row width (usually one), then each
// request's defect windows.  Timing: start on the first launch, stop on the last.
int sample_canonical(Context* c, hipStream_t st, const std::vector<CanonSample>& items, const KTime* kt) {
    std::vector<std::vector<size_t>> by_ldt;
    std::vector<int> ldts;   // one group per (row stride, FP32 rows); FP32 groups as -ldt
    size_t n_blk = 0, n_win = 0;
    for (size_t k = 0; k < items.size(); ++k) {
        const Plan& P = items[k].q->plan();
        if (items[k].n <= 0) continue;
        const int key = P.rows_f32() ? -P.ldt : P.ldt;
        auto it = std::find(ldts.begin(), ldts.end(), key);
        if (it == ldts.end()) {
            ldts.push_back(key);
            by_ldt.emplace_back();
            it = ldts.end() - 1;
        }
        by_ldt[it - ldts.begin()].push_back(k);
        n_blk += P.blocks.size();
        n_win += P.defects.empty() ? 0 : 1;
    }
    if (ldts.empty()) return LSUM_OK;
    std::vector<SampleBlock> blk_h;
    std::vector<SampleJob> jobs_h;
    blk_h.reserve(n_blk);
    jobs_h.reserve(items.size());
    DevBuf blk_d, jobs_d;
    int rc;
    if ((rc = blk_d.get(c->pool, std::max<size_t>(1, n_blk) * sizeof(SampleBlock)))) return rc;
    if ((rc = jobs_d.get(c->pool, items.size() * sizeof(SampleJob)))) return rc;
    std::vector<int> first_job, n_jobs, n_wg;
    for (size_t g = 0; g < by_ldt.size(); ++g) {
        const auto& grp = by_ldt[g];
        const int ppw = sample_points_per_wg(ldts[g] < 0);
        first_job.push_back((int)jobs_h.size());
        int wg = 0;
        for (size_t k : grp) {
            const CanonSample& it = items[k];
            const Request* q = it.q;
            const Plan& P = q->plan();
            SampleJob j{};
            j.xyz = it.xyz;
            j.out = it.out;
            j.blk = blk_d.as<SampleBlock>() + blk_h.size();
            j.h = P.h;
            j.n_blocks = (int)P.blocks.size();
            j.n_pts = it.n;
            j.wg0 = wg;
            j.N0 = P.N[0];
            j.N1 = P.N[1];
            j.N2 = P.N[2];
            j.off1 = (int)q->UT_axis_off[1];
            j.off2 = (int)q->UT_axis_off[2];
            j.f32 = P.rows_f32() ? 1 : 0;
            for (size_t b = 0; b < P.blocks.size(); ++b) blk_h.push_back(SampleBlock{q->UT[b].p, P.blocks[b].charge});
            jobs_h.push_back(j);
            wg += (it.n + ppw - 1) / ppw;
        }
        n_jobs.push_back((int)grp.size());
        n_wg.push_back(wg);
    }
    LSUM_HIP(hipMemcpyAsync(blk_d.p, blk_h.data(), blk_h.size() * sizeof(SampleBlock), hipMemcpyHostToDevice, st));
    LSUM_HIP(hipMemcpyAsync(jobs_d.p, jobs_h.data(), jobs_h.size() * sizeof(SampleJob), hipMemcpyHostToDevice, st));
    size_t wins_left = n_win;
    for (size_t g = 0; g < ldts.size(); ++g) {
        KTime k;
        if (kt && g == 0) k.start = kt->start;
        if (kt && g + 1 == ldts.size() && wins_left == 0) k.stop = kt->stop;
        launch_sample_batch(st, std::abs(ldts[g]), ldts[g] < 0, jobs_d.as<SampleJob>() + first_job[g], n_jobs[g],
                            n_wg[g], &k);
    }
    for (const auto& it : items) {
        const Request* q = it.q;
        const Plan& P = q->plan();
        if (it.n <= 0 || P.defects.empty()) continue;
        KTime k;
        if (kt && --wins_left == 0) k.stop = kt->stop;
        launch_sample_windows(st, P.R, q->rows(), P.ldg, (int)P.defects.size(),
                              q->def_offs.as<int32_t>(), q->def_scale.as<double>(), P.N[0], P.N[1], P.N[2],
                              P.h, it.n, it.xyz, it.out, &k);
    }
    LSUM_HIP(hipGetLastError());
    // the job and block arrays go back to the pool, whose next user may run on another stream
    LSUM_HIP(hipStreamSynchronize(st));
    return LSUM_OK;
}

int sample_points(Request* q, hipStream_t st, int n, const double* xyz_d, double* out_d, const KTime* kt,
                  double* flops) {
    Context* c = q->ctx;
    const Plan& P = q->plan();
    int rc;
    if (n <= 0) return LSUM_OK;
    if (!P.tucker()) return sample_canonical(c, st, {CanonSample{q, n, xyz_d, out_d}}, kt);
    const int r1 = q->r[0], r2 = q->r[1], r3 = q->r[2];
    const size_t ncore = (size_t)r1 * r2 * r3;
    // the mode-3 contraction runs in the request's precision on the core as stored (FP32
    // elements unless FP64, with FP64 sums across chunks); the finishing sums are FP64
    (void)ncore;
    DevBuf Z3f, idx, W, Z3s, i3c;
    const GemmPrec gp = gemm_prec(P.precision);
    const size_t we = P.precision == LSUM_FP64 ? 8 : 4;
    const void* Z3p = q->Z[2].p;
    if (we == 4) {
        if ((rc = Z3f.get(c->pool, (size_t)r3 * P.N[2] * 4))) return rc;
        launch_f64_to_f32(st, (long)r3 * P.N[2], q->Z[2].as<double>(), Z3f.as<float>());
        Z3p = Z3f.p;
    }
    if ((rc = idx.get(c->pool, (size_t)n * 12))) return rc;
    launch_snap_points(st, n, xyz_d, P.N[0], P.N[1], P.N[2], P.h, idx.as<int32_t>());
    std::vector<int32_t> idx_h((size_t)3 * n);
    LSUM_HIP(hipMemcpyAsync(idx_h.data(), idx.p, (size_t)n * 12, hipMemcpyDeviceToHost, st));
    LSUM_HIP(hipStreamSynchronize(st));
    // The mode-3 contraction W[u][(a,b)] = sum_c mu[(a,b)][c] Z3[c, u] dominates (r1 r2 r3 per
    // row): it is formed once per distinct mode-3 cell u of the points, in chunks of cells, and
    // each point then reads its cell's row.  Points are taken in order of their mode-3 cell.
    std::vector<int32_t> order;
    order.reserve(n);
    for (int p = 0; p < n; ++p)
        if (idx_h[(size_t)2 * n + p] >= 0) order.push_back(p);
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        return idx_h[(size_t)2 * n + x] < idx_h[(size_t)2 * n + y];
    });
    std::vector<int32_t> cells;   // distinct mode-3 cells in increasing order
    std::vector<int32_t> slot(order.size());
    for (size_t t = 0; t < order.size(); ++t) {
        const int32_t u = idx_h[(size_t)2 * n + order[t]];
        if (cells.empty() || cells.back() != u) cells.push_back(u);
        slot[t] = (int32_t)cells.size() - 1;
    }
    const size_t per = std::max<size_t>(1, (size_t)r1 * r2);
    int chunk = (int)std::max<size_t>(1, std::min<size_t>(cells.size(), ((size_t)1 << 28) / per));
    chunk = std::min(chunk, 4096);
    if ((rc = W.get(c->pool, per * chunk * we))) return rc;
    if ((rc = Z3s.get(c->pool, (size_t)r3 * chunk * we))) return rc;
    if ((rc = i3c.get(c->pool, (size_t)chunk * 4))) return rc;
    DevBuf lists;
    if ((rc = lists.get(c->pool, std::max<size_t>(1, order.size()) * 16))) return rc;
    std::vector<int32_t> lh(4 * std::max<size_t>(1, order.size()));
    size_t t0 = 0;
    for (size_t u0 = 0; u0 < cells.size(); u0 += chunk) {
        const int Un = (int)std::min<size_t>(chunk, cells.size() - u0);
        size_t t1 = t0;
        while (t1 < order.size() && slot[t1] < (int32_t)(u0 + Un)) ++t1;
        const int Pn = (int)(t1 - t0);
        // per point of the chunk: i1, i2, row of W, output index
        int32_t* i1h = lh.data();
        int32_t* i2h = i1h + Pn;
        int32_t* wrh = i2h + Pn;
        int32_t* ooh = wrh + Pn;
        for (int k = 0; k < Pn; ++k) {
            const int32_t p = order[t0 + k];
            i1h[k] = idx_h[p];
            i2h[k] = idx_h[(size_t)n + p];
            wrh[k] = slot[t0 + k] - (int32_t)u0;
            ooh[k] = p;
        }
        LSUM_HIP(hipMemcpyAsync(i3c.p, cells.data() + u0, (size_t)Un * 4, hipMemcpyHostToDevice, st));
        LSUM_HIP(hipMemcpyAsync(lists.p, lh.data(), (size_t)Pn * 16, hipMemcpyHostToDevice, st));
        launch_select_cols(st, r3, Un, Z3p, P.N[2], i3c.as<int32_t>(), Z3s.p, (int)we);
        // W[u][(a,b)] = sum_c Z3s[c][u] mu[(a,b)][c]: row-major per cell, so each row is contiguous
        GemmArgs a{};
        a.m = Un; a.n = r1 * r2; a.k = r3;
        a.A = Z3s.p; a.sam = 1; a.sak = Un;
        a.B = q->core.p; a.sbk = 1; a.sbn = r3;
        a.C = W.p; a.scm = (long)r1 * r2; a.scn = 1;
        a.alpha = 1.0; a.beta = 0.0; a.batch = 1;
        launch_gemm(st, gp, a);
        if (flops) *flops += 2.0 * Un * (double)r1 * r2 * r3 + 2.0 * (double)r1 * r2 * Pn;
        const int32_t* ld = lists.as<int32_t>();
        launch_tucker_finish(st, r1, r2, Pn, W.p, (int)we, q->Z[0].as<double>(), P.N[0], q->Z[1].as<double>(),
                             P.N[1], ld, ld + Pn, ld + 2 * Pn, ld + 3 * Pn, out_d);
        LSUM_HIP(hipStreamSynchronize(st));   // i3c and the lists are rewritten by the next chunk
        t0 = t1;
    }
    if (order.size() < (size_t)n) {
        // points outside the grid along axis 3 (axes 1 and 2 are marked by the finishing kernel)
        std::vector<double> o(n);
        LSUM_HIP(hipMemcpyAsync(o.data(), out_d, (size_t)n * 8, hipMemcpyDeviceToHost, st));
        LSUM_HIP(hipStreamSynchronize(st));
        for (int p = 0; p < n; ++p)
            if (idx_h[(size_t)2 * n + p] < 0) o[p] = std::nan("");
        LSUM_HIP(hipMemcpyAsync(out_d, o.data(), (size_t)n * 8, hipMemcpyHostToDevice, st));
        LSUM_HIP(hipStreamSynchronize(st));
    }
    LSUM_HIP(hipGetLastError());
    return LSUM_OK;
}

// ------------------------------------------------------------------------------------------
// exact sites off their cell centres: the request's own row tables
// ------------------------------------------------------------------------------------------
// The terms of every (block, axis) job of an off-grid request, keyed by block * 3 + axis.  Per
// sub-cell class the job's sites of that class are summed from the class's rows (directly, or
// through the window sums of their combs, as on grid).  All tables are R x ldg with stride
// R * ldg in q->tabs (the class rows first, then each (class, stride, n) window table), and a
// term's offset carries its table's element offset, so every job reads T0 = q->tabs (from the
// context's row cache, built on st on a miss).
static int offgrid_terms(Context* c, Request* q, hipStream_t st, std::map<int, std::vector<int2>>& out,
                         double* table_bytes) {
    const Plan& P = q->plan();
    const int nb = (int)P.blocks.size();
    const int C = (int)P.cls_f.size();
    const int64_t tab = (int64_t)P.R * P.ldg;
    std::map<std::tuple<int, int, int>, int> wins;   // (class, stride, n) -> table
    std::vector<std::tuple<int, int, int>> win_list;
    auto table_of = [&](int cl, int S, int n) {
        auto it = wins.emplace(std::make_tuple(cl, S, n), C + (int)win_list.size());
        if (it.second) win_list.push_back(std::make_tuple(cl, S, n));
        return it.first->second;
    };
    std::vector<int32_t> cs;
    std::vector<int2> tv;
    for (int b = 0; b < nb; ++b)
        for (int l = 0; l < 3; ++l) {
            if (q->axis_src[l] != l) continue;
            const auto& sites = P.offs[l][b];
            const auto& cls = P.cls[l][b];
            std::vector<int2>& terms = out[b * 3 + l];
            for (int cl = 0; cl < C; ++cl) {
                cs.clear();
                for (size_t k = 0; k < sites.size(); ++k)
                    if (cls[k] == cl) cs.push_back(sites[k]);
                if (cs.empty()) continue;
                int stride = 0, n_tab[2] = {0, 0};
                bool two = false;
                shift_terms(cs.data(), (int)cs.size(), P.N_ref, P.N[l], P.ldg, tv, &stride, n_tab, &two);
                for (const int2& t : tv) {
                    const int table = stride == 0 ? cl : table_of(cl, stride, n_tab[t.y & 1]);
                    terms.push_back(make_int2((int)(t.x + table * tab), t.y & 2));   // keeps the sign
                }
            }
        }
    const int n_tab = C + (int)win_list.size();
    if ((double)n_tab * (double)tab + P.ldg >= 2147483647.0)
        return fail(LSUM_E_INVALID, "too many sub-cell offset tables");
    int rc = get_tables(c, P, win_list, st, q->tabs);
    if (rc) return rc;
    *table_bytes = (double)n_tab * P.R * (2 * P.N_ref - 1) * 8;
    return LSUM_OK;
}

// One Tucker-reference request: the sum, then its completion sampling; stage times as for a batch.
static int run_tucker_ref_batch(Request* q, hipStream_t st, const hipStream_t* aux) {
    Context* c = q->ctx;
    StageTimer tm(st);
    int rc = run_tucker_ref(q, st, aux, tm);
    if (rc) {
        (void)hipStreamSynchronize(st);
        (void)hipGetLastError();
        q->status.store(rc);
    } else if (q->n_points > 0) {
        const int n = q->n_points;
        const double* xyz_d = q->points;
        double* out_d = q->values;
        DevBuf xd, od;
        if (!q->points_on_device) {
            if ((rc = xd.get(c->pool, (size_t)n * 24)) || (rc = od.get(c->pool, (size_t)n * 8))) {
                q->status.store(rc);
                return LSUM_OK;
            }
            LSUM_HIP(hipMemcpyAsync(xd.p, q->points, (size_t)n * 24, hipMemcpyHostToDevice, st));
            xyz_d = xd.as<double>();
            out_d = od.as<double>();
        }
        double fl = 0.0;
        tm.begin("sample", (double)n * 32, 0);
        rc = sample_points(q, st, n, xyz_d, out_d, nullptr, &fl);
        if (fl > 0.0) tm.work(0, fl);   // a Tucker result: a contraction in the request's precision
        tm.end();
        if (rc) q->status.store(rc);
        else if (!q->points_on_device)
            LSUM_HIP(hipMemcpyAsync(q->values, out_d, (size_t)n * 8, hipMemcpyDeviceToHost, st));
    }
    LSUM_HIP(hipStreamSynchronize(st));
    std::map<std::string, double> t;
    tm.collect(t, c);
    q->t_ms = std::make_shared<const std::map<std::string, double>>(std::move(t));
    return LSUM_OK;
}

// ------------------------------------------------------------------------------------------
// a batch of requests (several canonical ones, or one reduction request)
// ------------------------------------------------------------------------------------------
int run_batch(std::vector<Request*>& reqs, hipStream_t st, const hipStream_t* aux) {
    Context* c = reqs[0]->ctx;
    StageTimer tm(st);
    int rc;
    if (reqs.size() == 1 && reqs[0]->plan().tucker_ref()) return run_tucker_ref_batch(reqs[0], st, aux);
    // (1)-(2) quadrature is in the plan; reference vectors from the cache
    for (auto* q : reqs)
        if ((rc = get_reference(c, q->plan(), st, q->ref))) return rc;

    // (3) assembled shift-sums of every block and axis of every request: one launch.  Canonical
    // requests keep point-major factors (for sampling), reduction requests vector-major ones
    // (side-matrix columns).
    std::vector<int2> terms_h;
    std::vector<ShiftJob> jobs;
    std::vector<size_t> term_off;
    int maxN = 0, maxR = 0;
    double out_bytes = 0, loads = 0, ref_extra = 0;
    std::vector<const RefEntry*> distinct;
    std::vector<int2> tv;
    for (auto* q : reqs) {
        const Plan& P = q->plan();
        const int nb = (int)P.blocks.size();
        const bool vector_major = P.tucker();
        // Axes with the same cell count and the same snapped sites in every block (a cubic lattice
        // on a cubic grid) have identical factors: they are summed and stored once and shared.
        size_t uN = 0, uoff = 0, utoff = 0;
        for (int l = 0; l < 3; ++l) {
            int src = l;
            for (int k = 0; k < l && src == l; ++k) {
                if (q->axis_src[k] != k || P.N[k] != P.N[l]) continue;
                bool same = true;
                for (int b = 0; b < nb && same; ++b)
                    same = P.offs[k][b] == P.offs[l][b] && (!P.off_grid() || P.cls[k][b] == P.cls[l][b]);
                if (same) src = k;
            }
            q->axis_src[l] = src;
            if (src == l) {
                q->U_axis_off[l] = uoff;
                q->UT_axis_off[l] = utoff;
                uoff += (size_t)P.R * P.N[l];
                utoff += (size_t)P.ldt * P.N[l];
                uN += P.N[l];
            } else {
                q->U_axis_off[l] = q->U_axis_off[src];
                q->UT_axis_off[l] = q->UT_axis_off[src];
            }
        }
        q->U.resize(nb);
        q->UT.resize(nb);
        std::map<int, std::vector<int2>> og;
        if (P.off_grid()) {
            double tb = 0;
            if ((rc = offgrid_terms(c, q, st, og, &tb))) return rc;
            ref_extra += tb;
        }
        for (int b = 0; b < nb; ++b) {
            DevBuf& out = vector_major ? q->U[b] : q->UT[b];
            if ((rc = out.get(c->pool, vector_major ? (size_t)P.R * uN * 8 : (size_t)P.ldt * uN * P.row_elem()))) return rc;
            for (int l = 0; l < 3; ++l) {
                if (q->axis_src[l] != l) continue;
                const auto& sites = P.offs[l][b];
                int stride = 0, n_tab[2] = {0, 0};
                bool two = false;
                ShiftJob j{};
                if (P.off_grid()) {
                    tv = og[b * 3 + l];
                    j.T0 = q->tabs->G.as<double>();
                } else {
                    shift_terms(sites.data(), (int)sites.size(), P.N_ref, P.N[l], P.ldg, tv, &stride, n_tab, &two);
                    j.T0 = q->ref->G.as<double>();
                }
                if (stride > 0) {
                    const double* w = nullptr;
                    if ((rc = get_windows(c, *q->ref, stride, n_tab[0], st, &w))) return rc;
                    j.T0 = w;
                    if (two) {
                        if ((rc = get_windows(c, *q->ref, stride, n_tab[1], st, &w))) return rc;
                        j.T1 = w;
                    }
                }
                term_off.push_back(terms_h.size());
                terms_h.insert(terms_h.end(), tv.begin(), tv.end());
                j.n_terms = (int)tv.size();
                j.U = vector_major ? q->U[b].as<double>() + q->U_axis_off[l] : nullptr;
                j.ldu = P.N[l];
                if (!vector_major && P.rows_f32()) j.UT32 = q->UT[b].as<float>() + q->UT_axis_off[l];
                else if (!vector_major) j.UT = q->UT[b].as<double>() + q->UT_axis_off[l];
                j.ldt = P.ldt;
                j.N_axis = P.N[l];
                j.ldg = P.ldg;
                j.R = P.R;
                jobs.push_back(j);
                maxN = std::max(maxN, P.N[l]);
                maxR = std::max(maxR, P.R);
                loads += (double)P.R * P.N[l] * tv.size();
            }
            // algorithmic: the R values per distinct cell, no padding
            out_bytes += (double)P.R * uN * (vector_major ? 8 : P.row_elem());
        }
        if (std::find(distinct.begin(), distinct.end(), q->ref.get()) == distinct.end()) distinct.push_back(q->ref.get());
        q->canonical_bytes = (double)nb * P.R * uN * (vector_major ? 8 : P.row_elem());
    }
    double ref_bytes = ref_extra;
    for (auto* e : distinct) ref_bytes += (double)e->R * (2 * e->N_ref - 1) * 8;
    DevBuf terms_d, jobs_d;
    if ((rc = terms_d.get(c->pool, std::max<size_t>(1, terms_h.size()) * sizeof(int2)))) return rc;
    if ((rc = jobs_d.get(c->pool, jobs.size() * sizeof(ShiftJob)))) return rc;
    for (size_t k = 0; k < jobs.size(); ++k) jobs[k].terms = terms_d.as<int2>() + term_off[k];
    if (!terms_h.empty())
        LSUM_HIP(hipMemcpyAsync(terms_d.p, terms_h.data(), terms_h.size() * sizeof(int2), hipMemcpyHostToDevice, st));
    LSUM_HIP(hipMemcpyAsync(jobs_d.p, jobs.data(), jobs.size() * sizeof(ShiftJob), hipMemcpyHostToDevice, st));
    // algorithmic traffic: every distinct reference read once, every factor written once
    const KTime kt = tm.kernels("shift_sum", ref_bytes + out_bytes, loads);
    launch_shift_sum(st, jobs_d.as<ShiftJob>(), (int)jobs.size(), maxN, maxR, &kt, &c->tuner);
    LSUM_HIP(hipGetLastError());

    // defect tables (canonical sampling evaluates defect windows from the reference rows)
    for (auto* q : reqs) {
        const Plan& P = q->plan();
        const int nd = (int)P.defects.size();
        if (nd == 0) continue;
        std::vector<int32_t> offs(3 * (size_t)nd);
        std::vector<double> sc(nd);
        for (int s = 0; s < nd; ++s) {
            const auto& d = P.defects[s];
            for (int l = 0; l < 3; ++l)
                offs[3 * s + l] = (int32_t)win_off(P, P.site_cls(l, d.block, d.site[l]), P.offs[l][d.block][d.site[l]]);
            sc[s] = d.dZ;
        }
        if ((rc = q->def_offs.get(c->pool, offs.size() * 4))) return rc;
        if ((rc = q->def_scale.get(c->pool, nd * 8))) return rc;
        LSUM_HIP(hipMemcpyAsync(q->def_offs.p, offs.data(), offs.size() * 4, hipMemcpyHostToDevice, st));
        LSUM_HIP(hipMemcpyAsync(q->def_scale.p, sc.data(), nd * 8, hipMemcpyHostToDevice, st));
    }

    // (4)-(8) reduction requests
    for (auto* q : reqs) {
        if (!q->plan().tucker()) continue;
        rc = run_tucker(q, st, aux, tm);
        if (rc) {
            (void)hipStreamSynchronize(st);
            (void)hipGetLastError();
            q->status.store(rc);
        }
    }

    // completion sampling at the request's points: the canonical requests of the batch in one
    // launch, reduction requests one by one
    std::vector<DevBuf> staged;
    staged.reserve(2 * reqs.size());
    std::vector<CanonSample> canon;
    std::vector<Request*> canon_q;
    double canon_bytes = 0;
    for (auto* q : reqs) {
        if (q->n_points <= 0 || q->status.load() < 0) continue;
        const int n = q->n_points;
        const double* xyz_d = q->points;
        double* out_d = q->values;
        if (!q->points_on_device) {
            DevBuf xd, od;
            if ((rc = xd.get(c->pool, (size_t)n * 24)) || (rc = od.get(c->pool, (size_t)n * 8))) {
                q->status.store(rc);
                continue;
            }
            LSUM_HIP(hipMemcpyAsync(xd.p, q->points, (size_t)n * 24, hipMemcpyHostToDevice, st));
            xyz_d = xd.as<double>();
            out_d = od.as<double>();
            staged.push_back(std::move(xd));
            staged.push_back(std::move(od));
        }
        const Plan& P = q->plan();
        // factors read once (R values per distinct cell) + points in + values out
        double uN = 0;
        for (int l = 0; l < 3; ++l)
            if (q->axis_src[l] == l) uN += P.N[l];
        const double fb = (double)P.blocks.size() * P.R * uN * P.row_elem();
        if (P.tucker()) {
            double fl = 0.0;
            tm.begin("sample", (double)n * 32, 0);
            rc = sample_points(q, st, n, xyz_d, out_d, nullptr, &fl);
            if (fl > 0.0) tm.work(0, fl);   // a contraction in the request's precision
            tm.end();
            if (rc) {
                q->status.store(rc);
                continue;
            }
            if (!q->points_on_device)
                LSUM_HIP(hipMemcpyAsync(q->values, out_d, (size_t)n * 8, hipMemcpyDeviceToHost, st));
        } else {
            canon.push_back(CanonSample{q, n, xyz_d, out_d});
            canon_q.push_back(q);
            canon_bytes += (double)n * 32 + fb;
        }
    }
    if (!canon.empty()) {
        const KTime kt = tm.kernels("sample", canon_bytes, 0);
        rc = sample_canonical(c, st, canon, &kt);
        for (size_t k = 0; k < canon.size(); ++k) {
            Request* q = canon_q[k];
            if (rc) q->status.store(rc);
            else if (!q->points_on_device)
                LSUM_HIP(hipMemcpyAsync(q->values, canon[k].out, (size_t)canon[k].n * 8, hipMemcpyDeviceToHost, st));
        }
    }
    LSUM_HIP(hipStreamSynchronize(st));
    std::map<std::string, double> t;
    tm.collect(t, c);
    auto shared_t = std::make_shared<const std::map<std::string, double>>(std::move(t));
    for (auto* q : reqs) q->t_ms = shared_t;
    return LSUM_OK;
}

}  // namespace lsum

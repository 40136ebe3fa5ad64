// Internal declarations shared by the host driver and the HIP kernels of the lattice-sum
// library.  Not part of the public ABI (see include/lsum.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <atomic>
#include <map>
#include <mutex>
#include <vector>

#include "lsum.h"

namespace lsum {

// ------------------------------------------------------------------------------------------
// error handling
// ------------------------------------------------------------------------------------------
void set_error(const std::string& msg);
// Records the message and returns code.  When the calling thread has a FailStream, fail() first
// waits for that stream (errors are raised where they are detected, so queued kernels finish
// before the caller's device buffers unwind into the shared pool).
int fail(int code, const std::string& msg);
// The calling thread's last error message.
const char* last_error();
// Scope in which fail() on this thread waits for `st` (restores the previous stream on exit).
class FailStream {
  public:
    explicit FailStream(hipStream_t st);
    ~FailStream();
    FailStream(const FailStream&) = delete;
    FailStream& operator=(const FailStream&) = delete;

  private:
    hipStream_t prev_;
};

#define LSUM_HIP(call)                                                                      \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return ::lsum::fail(LSUM_E_DEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------------------------------------
// host-side steps (FP64 / integer)
// ------------------------------------------------------------------------------------------
void default_quadrature(int kind, const int N[3], double h, double* h_u, double* s);
// Laplace-Gauss density a(t) of the kernel (Sec. 2.2).
double laplace_density(int kind, double param, double t);
// The folded rule before dropping: t[k] = sinh(k h_u)/s, w[k], k = 0..M (no validation).
void sinc_rule(int kind, double param, int M, double h_u, double s, double* t, double* w);
// Returns LSUM_OK or an error; t/w receive R <= M+1 nodes.
int sinc_nodes(int kind, double param, int M, double h_u, double s, std::vector<double>& t,
               std::vector<double>& w);
int snap_coord(double x, double h, int N, int32_t* idx);
// Sinc error control: scans M = M_lo..M_hi for the first max-norm relative error <= eps (see
// lsum_sinc_error.cpp); LSUM_E_NOCONV with the best M when none (eps < 0: always LSUM_OK).
int sinc_error_scan(const lsum_kernel& k, const int N[3], double h, double eps, int M_lo, int M_hi, int* M_out,
                    double* err_out);
// Coordinate of site k of axis l: the block's explicit list, or (k - (L-1)/2) b + center.
double site_x(const lsum_block& blk, int l, int k);
int block_offsets(const lsum_block& blk, const int N[3], double h, std::vector<int32_t> offs[3]);
// SVD of a small dense m x n matrix M (row-major) by one-sided Jacobi rotations (host FP64):
// M = sum_e S[e] u_e v_e^T, k = min(m, n) terms by decreasing S, u_e = Ul[e*m .. e*m+m),
// v_e = Vr[e*n .. e*n+n).
void small_svd(const double* M, int m, int n, std::vector<double>& Ul, std::vector<double>& S,
               std::vector<double>& Vr);
// Sub-cell offsets of a block's sites (exact sites): f = x/h - j for the snapped cell j.
void block_subcell(const lsum_block& blk, double h, std::vector<double> f[3]);

// ------------------------------------------------------------------------------------------
// plan of one problem: bookkeeping shared by every stage
// ------------------------------------------------------------------------------------------
struct Plan {
    // problem (deep copy)
    lsum_kernel kernel{};
    int N[3]{};
    double h = 0;
    std::vector<lsum_block> blocks;
    std::vector<lsum_defect> defects;
    double eps = 0;
    int precision = LSUM_FP64;
    int tile_lo[3]{}, tile_T[3]{};

    // quadrature
    double h_u = 0, s = 0;
    std::vector<double> t, w;
    int R = 0;
    int N_ref = 0;   // max N
    int ldg = 0;     // reference row stride
    int ldt = 0;     // point-major factor row stride: R rounded up to 16 (64- or 128-byte rows)

    // per block, per axis snapped cell indices
    std::vector<std::vector<int32_t>> offs[3];   // offs[axis][block]
    // exact sites: a site at (j + f) h along an axis sits in cell j with sub-cell offset f.  The
    // distinct offsets are the classes (class 0 is f = 0); cls[axis][block][site] is the class
    // of each site, empty unless some site is off its cell centre (then every class has its own
    // reference rows, class c at element c * R * ldg of the request's row tables).
    int exact_sites = 0;
    std::vector<double> cls_f{0.0};
    std::vector<std::vector<int32_t>> cls[3];
    bool off_grid() const { return cls_f.size() > 1; }
    int site_cls(int l, int b, int k) const { return off_grid() ? cls[l][b][k] : 0; }

    // Side-matrix columns per mode, grouped in "sources" of R columns (one per node q):
    // sources [0, n_lat[l]) are distinct lattice offset lists, the rest distinct defect cells.
    int n_lat[3]{}, n_win[3]{};
    std::vector<int32_t> lat_block[3];   // representative block of each lattice source
    std::vector<int32_t> win_cell[3];    // cell index of each window source
    std::vector<int32_t> win_cls[3];     // class of each window source
    // term groups: blocks first, then defects; scale = block charge or dZ
    int n_groups = 0;
    std::vector<double> g_scale;
    std::vector<int32_t> g_src[3];       // source index of each group per mode
    std::vector<int32_t> src_mult[3];    // multiplicity of each source (groups using it)
    int D[3]{};                          // R * (n_lat + n_win)

    int method = LSUM_SUM_CANONICAL;
    int als_sweeps = 0;
    bool tucker() const { return eps > 0; }
    bool tucker_ref() const { return tucker() && method == LSUM_SUM_TUCKER_REF; }
    // canonical output with FP32 precision keeps its point-major factors in FP32 (sampling
    // multiplies and sums them in FP64); everything else is FP64
    bool rows_f32() const { return !tucker() && precision != LSUM_FP64; }
    size_t row_elem() const { return rows_f32() ? 4 : 8; }
    bool has_tile() const { return tile_T[0] > 0 && tile_T[1] > 0 && tile_T[2] > 0; }
    size_t planned_bytes() const;        // HBM footprint estimate of the request
};

// Validates the problem and fills the plan (host only).  Returns LSUM_OK or an error.
int make_plan(const lsum_problem& p, Plan& plan);
// Element offset of the window of a charge in cell `cell` of class `cls` into the row tables
// (the reference rows when on grid): entry i of the window is rows[q * ldg + i + win_off].
inline int64_t win_off(const Plan& P, int cls, int cell) {
    return (int64_t)cls * P.R * P.ldg + (P.N_ref - 1 - cell);
}

// ------------------------------------------------------------------------------------------
// kernel launchers (defined in the .hip files); all asynchronous on `st`
// ------------------------------------------------------------------------------------------
// shift: the charge's offset from its cell centre (exact sites), 0 on the centre.
void launch_collocate(hipStream_t st, int R, const double* t_dev, const double* w13_dev, int N_ref,
                      double h, double* G, int ldg, double shift = 0.0);
// Optional kernel-bound timing: both events are recorded by the dispatch of the kernel itself
// (hipExtLaunchKernel), so their difference is the kernel's own execution time.
// ------------------------------------------------------------------------------------------
// autotuner: launch variants that add the same terms in the same order (so every variant gives
// the same results bit for bit) are timed on the first launch of a shape bucket, and the
// fastest is kept, per context and optionally in a file shared between processes
// ------------------------------------------------------------------------------------------
class Tuner {
  public:
    // the variant chosen for key, or -1 (none yet, or tuning off: -2)
    int get(const std::string& key);
    // records the timings (ms, < 0: variant not measured) and keeps the fastest; returns it
    int put(const std::string& key, const std::vector<double>& ms);
    void set_device_tag(const std::string& tag) { tag_ = tag; }
    void enable(bool on) { on_.store(on ? 1 : 0); }
    bool enabled() const { return on_.load() != 0; }
    // decisions of earlier runs (same device tag) from `path`, which new ones are appended to
    int use_file(const std::string& path);
    std::string json();

  private:
    struct Entry {
        int choice;
        std::vector<double> ms;
    };
    std::mutex mu_;
    std::string tag_, path_;
    std::map<std::string, Entry> dec_;
    std::atomic<int> on_{1};
};

struct KTime {
    hipEvent_t start = nullptr, stop = nullptr;
};

// Shift-sum for a batch of (axis, block) jobs; see kernels_lattice.hip.  Each job is a list of
// terms (off, tab): out[q, i] = sum_t s_t T_(tab & 1)[q * ldg + i + off] for i < N_axis, q < R,
// with s_t = -1 when bit 1 of tab is set and +1 otherwise.  With the reference rows as T0 and
// off = N_ref - 1 - c_k per site this is the direct sum over the sites; an axis whose sites form
// interleaved uniform combs uses windowed strided sums of the reference rows
// (launch_window_sums) and one term per comb, and one whose sites form runs of one stride uses
// differences of strided prefix or suffix sums, two terms per run.
struct ShiftJob {
    const double* T0;      // rows of length >= ldg, R of them
    const double* T1;      // second table (combs one site shorter, or the suffix sums) or nullptr
    const int2* terms;     // n_terms pairs (off, tab)
    double* U;             // vector-major output (R x ldu) or nullptr
    double* UT;            // point-major output (N_axis x ldt, zero padded beyond R) or nullptr
    float* UT32;           // the same, rounded to FP32, or nullptr
    int n_terms;
    int N_axis;
    int ldg;
    int R;
    int ldu;
    int ldt;
};
// max_N, max_R: largest N_axis and R of the jobs; kt: optional kernel-bound timing.  Every row read must
// extend one entry past the last cell window (ldg >= 2 * N_ref - 1 and ldg >= 2).
void launch_shift_sum(hipStream_t st, const ShiftJob* jobs_dev, int n_jobs, int max_N, int max_R,
                      const KTime* kt = nullptr, Tuner* tuner = nullptr);
// Q[q, x] = sum_{m=0}^{n-1} G[q, x - m S] over the terms with x - m S >= 0, for x < ldg; with
// n = kPrefixSums every m >= 0 (the strided prefix sum), with n = kSuffixSums the strided
// suffix sum Q[q, x] = sum_{m >= 0, x + m S < ldg} G[q, x + m S].  The prefix and suffix sums are
// compensated (each within a few units of roundoff of the exact sum of |G| along the chain).
constexpr int kPrefixSums = -1;
constexpr int kSuffixSums = -2;
void launch_window_sums(hipStream_t st, int R, const double* G, int ldg, int stride, int n, double* Q);
// The static scratch array of the allocation-free shift-sum (scratch_noalloc.hip): its size, and
// its address on `device` (taken once per device with hipGetSymbolAddress; `device` current).
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
int noalloc_scratch(int device, void** ptr);
// Host: the smallest period p <= max_p with c[k+p] - c[k] constant (its stride), or 0.
int comb_period(const int32_t* c, int n, int max_p, int* stride);
// Host: the terms of one axis of N_axis cells (sites c[0..n) in [0, N_axis), rows of ldg >=
// max(2, 2 N_ref - 1) entries), the form with the fewest terms of:
// * runs of one stride S (sites a, a + S, ..., a + (n_r - 1) S): each two terms on the strided
//   prefix sums (table 0, n_tab[0] = kPrefixSums) or suffix sums (table 1, kSuffixSums) of the
//   rows, bit 1 of tab marking the subtracted one (a run that fits neither is split in two);
// * when the ascending sites are `period` interleaved combs of uniform stride, comb j (sites
//   c[j], c[j] + S, ...) with n_j = ceil((n - j) / period) sites: one term (N_ref - 1 - c[j], tab),
//   tab 0 for n_j == n_tab[0] and 1 for n_tab[1] = n_tab[0] - 1 (window sums of that length);
// * otherwise one term (N_ref - 1 - c[k], 0) per site on the reference rows, *stride = 0.
// *stride is the tables' stride and *two_tables tells whether table 1 is used.  Every term's
// reads i + off lie in [0, ldg) for i < max(N_axis, 2).
void shift_terms(const int32_t* c, int n, int N_ref, int N_axis, int ldg, std::vector<int2>& terms, int* stride,
                 int n_tab[2], bool* two_tables);
// Canonical sum at points from n_fac factor sets given vector-major (the sample stage of the
// C ABI): out[p] = sum_f lam[f] sum_q prod_l U_f,l[q, i_l(p)], NaN outside the grid.
void launch_sample_cp(hipStream_t st, int n_fac, int R, const double* U, int ldu,
                      const double* lam_dev, int N0, int N1, int N2, double h, int n_pts,
                      const double* xyz, double* out);
// R x N (stride ldu) -> N x R
void launch_transpose(hipStream_t st, int R, int N, const double* U, int ldu, double* UT);
void launch_transpose(hipStream_t st, int R, int N, const float* U, int ldu, double* UT);
// UT[i * ldt + q] = U[q * ldu + i] for q < R, i < N
void launch_transpose_ld(hipStream_t st, int R, int N, const double* U, int ldu, double* UT, long ldt);
// One block of a canonical request in a batched sampling launch: its factor base (axis 0 rows;
// axes 1 and 2 at the job's offsets) and its charge.
struct SampleBlock {
    const void* T;            // double, or float for a job with f32 set
    double lam;
};
// One canonical request in a batched sampling launch: n_pts points (x, y, z interleaved) whose
// values are written to out (NaN for a point outside the grid); work-groups wg0 .. wg0 +
// ceil(n_pts / 32) - 1 serve it, in increasing wg0 over the job array.
struct SampleJob {
    const double* xyz;
    double* out;
    const SampleBlock* blk;   // n_blocks entries, device
    double h;
    int n_blocks, n_pts, wg0;
    int N0, N1, N2;
    int off1, off2;           // axis offsets (elements) of axes 1 and 2 from each block's base
    int f32;                  // factors stored as FP32
};
// Point-major canonical evaluation of a batch of requests whose rows are ldt apart (zero
// padded) and all FP64 or all FP32 (f32); n_wg = total work-groups of the job array (device),
// sample_points_per_wg(f32) points each.
int sample_points_per_wg(bool f32);
void launch_sample_batch(hipStream_t st, int ldt, bool f32, const SampleJob* jobs_dev, int n_jobs, int n_wg,
                         const KTime* kt = nullptr);
// Defect windows evaluated straight from the reference rows, added to out.
// def_offs: per defect and axis the window offset (win_off) into the rows G.
void launch_sample_windows(hipStream_t st, int R, const double* G, int ldg,
                           int n_def, const int32_t* def_offs, const double* def_scale,
                           int N0, int N1, int N2, double h, int n_pts, const double* xyz,
                           double* out, const KTime* kt = nullptr);
// Side-matrix columns of one mode: rows [src*R + q] of cols (D x ldc); win_offs: the window
// offset (win_off) of each window source into the rows G.
void launch_gather_columns(hipStream_t st, int R, int n_lat, const double* const* lat_U_dev,
                           int ldu, int n_win, const int32_t* win_offs_dev, const double* G,
                           int ldg, int N_axis, double* cols, int ldc);
void launch_row_norms(hipStream_t st, int rows, int n, const double* X, int ldx, double* nrm);
// Y[j, :] = X[j, :] * scale[j]
void launch_scale_rows(hipStream_t st, int rows, int n, const double* X, int ldx,
                       const double* scale, double* Y, int ldy);

// General strided GEMM on MFMA: C(m,n) = alpha * sum_k A(m,k) B(k,n) + beta * C(m,n),
// A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn], C(m,n) = C[m*scm + n*scn].
// Batched over `batch` with element offsets bA, bB, bC between batches.
struct GemmArgs {
    int m, n, k;
    const void* A; long sam, sak;
    const void* B; long sbk, sbn;
    void* C; long scm, scn;
    double alpha, beta;
    int batch; long bA, bB, bC;
};
enum GemmPrec { GEMM_F64 = 0, GEMM_F32 = 1, GEMM_BF16X3 = 2 };
void launch_gemm(hipStream_t st, GemmPrec prec, const GemmArgs& a);
// Plain FP64 products (unit-stride operands, at least 2^24 multiply-adds in all; a batch at
// fixed strides) through the ROCm BLAS library's DGEMM (strided batched for a batch), on st;
// false (nothing launched) for anything else (FP32 and split-BF16x3 included).  Process-wide
// switch: set_gemm_library.
bool blas_gemm(hipStream_t st, GemmPrec prec, const GemmArgs& a);
void set_gemm_library(bool on);
bool gemm_library();
// FP64 GEMM (batch 1) with the reduction split into about `split` slices of a multiple of the
// staging depth: the slices' products go to work (gemm_split_slices(a, split) x m x n doubles),
// then C = alpha * (their sum in slice order) + beta * C.
// KR[nu, i * rb + j] = Xa[nu, i] Xb[nu, j] (row-major, K rows): the ALS mode operand.
void launch_khatri_rao(hipStream_t st, int K, int ra, int rb, const double* Xa, const double* Xb, double* KR);
// Galerkin functional: H[k nb + m, :] = G[k, :] G[m, :] (nb^2 rows of n), and
// v[p] = scale sum_{a,b} X[p, a r2 + b] Y1[p, a] Y2[p, b].
void launch_hadamard_pairs(hipStream_t st, int nb, int n, const double* G, double* H);
void launch_galerkin_finish(hipStream_t st, int P, int r1, int r2, const double* X, const double* Y1,
                            const double* Y2, double scale, double* v);
// A[i * ld + off + i] = 1 for i < n (the rest untouched).
void launch_unit_diag(hipStream_t st, int n, long ld, long off, double* A);
int gemm_split_slices(const GemmArgs& a, int split);
void launch_gemm_split_f64(hipStream_t st, const GemmArgs& a, int split, double* work);

// Core contraction (eq. C-core): mu[a,b,c] = sum_nu X1[nu, a] X2[nu, b] X3[nu, c] over the K
// canonical terms nu = g*R + q.  X_l (K x ldx_l, row-major, FP64 or FP32 by precision) are the
// term-major operands made by launch_gather_terms: row nu of X_l is row src_l(g)*R + q of the
// transposed projection of mode l (times scale_g for mode 1).  ldx_l must be multiples of 4.
struct CoreArgs {
    int r1, r2, r3, K;
    const void* X1; const void* X2; const void* X3;
    long ldx1, ldx2, ldx3;
    void* core;                                       // r1*r2*r3, last index fastest
};
// X[nu, a] = (sc ? sc[nu] : 1) * Yt[idx[nu], a] for a < r, zero for r <= a < ldx; elem 4 or 8 bytes
void launch_gather_terms(hipStream_t st, int elem, int K, int r, const void* Yt, long ldy,
                         const int32_t* idx, const double* sc, void* X, long ldx);
void launch_core(hipStream_t st, GemmPrec prec, const CoreArgs& a, int k_split, void* work);
// T[jl][a - a_begin][b] = sum_{t in [off[j], off[j+1])} sc[t] Y1[i1[t], a] Y2[i2[t], b] for
// j = j0 + jl, jl < nj, a_begin <= a < min(r1, a_begin + a_count), b < r2 (FP64 sums, stored as
// elem 4 or 8 bytes like Y1, Y2; column jl of the chunk is a_count * r2 entries).
void launch_core_groups(hipStream_t st, int elem, int r1, int r2, int a_begin, int a_count, int j0, int nj,
                        const int32_t* off, const int32_t* i1, const int32_t* i2, const double* sc, const void* Y1,
                        long ldy1, const void* Y2, long ldy2, void* out);
// ||A||^2 from the three unnormalised column Grams (D x D) and the group table.
// The canonical sum (groups of R terms: sources src_l[g] in the unnormalised columns C_l, D_l x N_l,
// weights scale[g]) at n_cells cells (cells[3p + l]), in FP64: out[p].
void launch_probe_canonical(hipStream_t st, int n_cells, int R, int n_groups, const int32_t* s1, const int32_t* s2,
                            const int32_t* s3, const double* scale, const double* C1, const double* C2,
                            const double* C3, int N1, int N2, int N3, const int32_t* cells, double* out);
void launch_cp_norm2(hipStream_t st, int R, int n_groups, const int32_t* src1, const int32_t* src2,
                     const int32_t* src3, const double* scale, const double* C1, const double* C2,
                     const double* C3, int D1, int D2, int D3, double* partial, int n_partial);

// One-sided block-Jacobi SVD of the D rows of A (length N): rows are rotated in place and
// written back sorted by descending norm (sigma).  Pairs involving a row whose norm is below
// `irrelevant` are not rotated (such rows cannot move a certified tail).  With n_gram < N only
// the first n_gram entries of each row define the Gram matrix, the norms and the convergence;
// the remaining entries are companion data rotated along (they receive the same orthogonal
// transformation).  With stop_tail2 > 0 the sweeps also end once the smallest r whose tail
// (sum of the squared norms of rows r, r+1, ...) is at most stop_tail2 repeats between two
// sweeps and the r largest rows (plus a margin) are orthogonal to tol; the norms of the tail
// rows are then bounds, not singular values (their squared sum bounds the true tail from above).
// How the sweeps are launched, and what a call reports back.  persistent: each sweep is one
// launch of one workgroup per pair slot, rounds ordered by per-block version counters (waits
// bounded by wait_us; a sweep whose groups were not all resident aborts and the remaining sweeps
// launch round by round); otherwise, with graphs, the round-by-round launches of a sweep are
// captured once per block count in a HIP graph and replayed; otherwise launched one by one.
// Every way adds the same terms in the same order (the same results bit for bit).
struct JacobiRun {
    int graphs = 0;
    int block = 8;                 // columns per block: 8, 16 or 32 (pairs of 32 or 64 rows, round by
                                   // round); 0: 32 for side matrices of at least 512 rows, else 16
                                   // (contexts default to 0; this struct's default serves direct callers)
    int persistent = 0;            // 1: 16-wave pair groups, 2: 4-wave pair groups
    // 16-column blocks: rotations whose relative coupling is at most skip_rel * tol are not
    // applied in the pair solve (0: every rotation above the rounding floor)
    double skip_rel = 0.0;
    double wait_us = 2e4;
    // workgroups of persistent sweeps running on the device (shared by every SVD of a context):
    // a sweep runs persistently only while the total stays within 3/4 of what the device holds
    // at once, else round by round (nullptr: no accounting)
    std::atomic<int>* wg_in_use = nullptr;
    Tuner* tuner = nullptr;        // decides the launch way per shape bucket (nullptr: as above)
    int tuned = 0;                 // out: 1 if this call timed the three ways
    double flops = 0.0;            // out: FP64 MFMA work of the pair Grams and rotations (added)
    int persistent_sweeps = 0;     // out: sweeps launched persistently (added)
    int aborted = 0;               // out: persistent sweeps that aborted (added)
};
int jacobi_svd(hipStream_t st, int D, int N, double* A, int lda, double tol, double irrelevant,
               int max_sweeps, std::vector<double>& sigma, int* sweeps_out, double* work_dev,
               size_t work_bytes, int n_gram = 0, double stop_tail2 = 0.0, JacobiRun* run = nullptr);
size_t jacobi_work_bytes(int D, int N);
// out[i] = +-1, i < n, a deterministic function of (seed, i)
void launch_random_signs(hipStream_t st, long n, unsigned long long seed, double* out);
// Rank-revealing Cholesky of a symmetric positive semi-definite n x n matrix A (row-major,
// n <= 128): with `pivot`, the largest remaining diagonal is taken first, and the
// factorisation stops at the first step whose pivot is <= tau2 times the first one (or not
// positive).  Out: keep (the steps done, *keep_dev), the pivot order perm[n], and R^T in pivot
// order, Rt[j*n + k] = R[k][j] for k <= j < keep, with (P A P^T)[0:keep, 0:keep] = R^T R.  One
// workgroup.
void launch_pchol(hipStream_t st, int n, const double* A, double tau2, int pivot, double* Rt, int* perm, int* keep_dev);
// out (keep x ncol, stride ldo) = R^{-T} Y_p, Y_p the rows perm[0..keep) of Y (stride ldy):
// orthonormal rows when A was their Gram.  keep <= 128.
void launch_trsm_rows(hipStream_t st, int keep, int ncol, int n, const double* Rt, const int* perm, const double* Y,
                      long ldy, double* out, long ldo);

// type conversions
void launch_f64_to_f32(hipStream_t st, long n, const double* x, float* y);
void launch_f32_to_f64(hipStream_t st, long n, const float* x, double* y);
// Z rows a = X[order[a]] / sigma[a]
void launch_gather_scale_rows(hipStream_t st, int r, int n, const double* X, int ldx,
                              const int32_t* order_dev, const double* inv_sigma_dev, double* Z,
                              int ldz);
// Rows of a factor selected by index lists: out[a * nsel + p] = Z[a * ldz + idx[p]]
void launch_select_cols(hipStream_t st, int rows, int nsel, const void* Z, long ldz,
                        const int32_t* idx, void* out, int elem_size);
// Tucker values of P points from W (rows r1*r2, layout [row][a*r2+b], elements of w_elem bytes)
// and Z1, Z2 rows: point t reads row wrow[t] and writes out[oidx[t]] (identity where the list is
// null); FP64 sums
void launch_tucker_finish(hipStream_t st, int r1, int r2, int P, const void* W, int w_elem, const double* Z1,
                          int ld1, const double* Z2, int ld2, const int32_t* i1, const int32_t* i2,
                          const int32_t* wrow, const int32_t* oidx, double* out);
void launch_snap_points(hipStream_t st, int n, const double* xyz, int N0, int N1, int N2, double h,
                        int32_t* idx /* 3 x n */);

}  // namespace lsum

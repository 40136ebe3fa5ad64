/*
 * lsum.h -- C ABI of the MI355X (gfx950) grid-based lattice-sum library.
 *
 * The library computes the projected potential of charges on 3D lattices (with vacancies,
 * impurities and unions of rectangular blocks) as a low-rank tensor on a fine N1 x N2 x N3
 * grid, following V. Khoromskaia, B. N. Khoromskij, "Tucker tensor method for fast
 * grid-based summation of long-range potentials on 3D lattices with defects"
 * (arXiv:1411.1994):
 *
 *   1. sinc-quadrature nodes/weights of the kernel's Laplace-Gauss transform (Sec. 2.1-2.2),
 *   2. reference canonical vectors by cell-average collocation on the doubled box (Sec. 3.1),
 *   3. assembled 1D shift-sums over the lattice (Thm thm:sumCaseE (A), eq. EwaldTensorGl),
 *   4. defects and blocks as algebraic sums of canonical tensors (Sec. 4.1-4.2),
 *   5. RHOSVD eps-rank reduction to Tucker format (Def. def:RHOSVD, Appendix theorem),
 *   6. Tucker/canonical evaluation on grid tiles and at points (eq. Tucker_singePot).
 *
 * Conventions used by every call:
 *   - Grid: N[l] odd cells per axis l, one mesh size h; cell i of axis l is centred at
 *     (i - (N[l]-1)/2) h.  Cell values are cell averages of the potential.
 *   - Reference vectors: R rows of length 2*N_ref-1 (row stride ldg); entry m of row q is
 *     w_q^(1/3) times the cell average of exp(-t_q^2 x^2) over the cell at displacement
 *     (m - (N_ref-1)) h.  An axis with N[l] <= N_ref uses the same rows.
 *   - Lattice block: L[3] sites per axis, spacing b[3], geometric centre center[3], every
 *     site carrying charge `charge`; site k of axis l sits at (k-(L-1)/2) b + center and is
 *     snapped to the cell j + (N-1)/2, j = sign(x/h) floor(|x/h| + 1/2) (halves away from
 *     zero).  A snapped site outside [0, N-1] is an error (LSUM_E_OUT_OF_BOX).
 *   - Canonical factor matrices are stored vector-major: R rows of N[l] doubles (row q is
 *     the q-th canonical vector of axis l).  Tucker factors Z_l are stored the same way:
 *     r_l rows of N[l] doubles (row a is the a-th orthonormal Tucker vector).  The Tucker
 *     core is r1 x r2 x r3 with the last index fastest.
 *   - Errors: every call returns LSUM_OK (0) or a negative LSUM_E_* code; lsum_last_error()
 *     returns a message for the calling thread.  No C++ exception crosses this boundary.
 *   - Pointers named *_dev are device (HBM) pointers on the context's device, allocated and
 *     owned by the caller unless stated otherwise; all other pointers are host pointers.
 *     `stream` is a hipStream_t passed as void* (NULL: the context's own stream).  Calls
 *     taking a stream are asynchronous with respect to the host unless stated otherwise.
 */
#ifndef LSUM_H
#define LSUM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------------------ */
#define LSUM_OK 0
#define LSUM_E_INVALID (-1)    /* bad argument: even N, M < 1, unknown kernel, bad eps, ...   */
#define LSUM_E_OUT_OF_BOX (-2) /* a snapped site or point lies outside the grid               */
#define LSUM_E_DUP_DEFECT (-3) /* two defects at the same site                                */
#define LSUM_E_NOMEM (-4)      /* the job can never fit the context's HBM budget              */
#define LSUM_E_BUSY (-5)       /* non-blocking submit on a full queue                         */
#define LSUM_E_CANCELLED (-6)  /* the request was cancelled before it ran                     */
#define LSUM_E_DEVICE (-7)     /* a HIP runtime error                                         */
#define LSUM_E_TIMEOUT (-8)    /* lsum_wait ran out of time (the request keeps running)       */
#define LSUM_E_STATE (-9)      /* result not available in this state / format                 */
#define LSUM_E_NOCONV (-10)    /* an iteration or search did not reach its target (Jacobi SVD
                                  sweeps, lsum_choose_M)                                       */

/* ---- problem description ---------------------------------------------------------------- */
enum { LSUM_NEWTON = 0, LSUM_YUKAWA = 1, LSUM_SLATER = 2 };
enum { LSUM_FP64 = 0, LSUM_FP32 = 1, LSUM_BF16X3 = 2 };
enum { LSUM_SUM_CANONICAL = 0, LSUM_SUM_TUCKER_REF = 1 };

/* Kernel p(r): Newton 1/r, Yukawa exp(-param r)/r, Slater exp(-param r) (Sec. 2.2).
 * Quadrature: u_k = k h_u, t_k = sinh(u_k)/s, k = 0..M (trapezoid rule of eq. hM after the
 * substitution t = sinh(u)/s, folded onto k >= 0).  h_u <= 0 or s <= 0 select defaults:
 * s = h sqrt(sum_l (N_l-1)^2) / 4, h_u = 0.30 (Slater) or 0.35 (Newton, Yukawa). */
typedef struct {
    int kind;
    double param;
    int M;
    double h_u;
    double s;
} lsum_kernel;

typedef struct {
    int L[3];
    double b[3];
    double center[3];
    double charge;   /* charge of every site; -1 describes a tensor sub-lattice of vacancies */
    const double* x[3];   /* optional: the L[l] site coordinates of axis l (a non-equidistant
                             tensor lattice, e.g. clusters on a coarse lattice, Sec. 4.4 case (D));
                             NULL: (k - (L-1)/2) b[l] + center[l].  Read while the request is
                             submitted (or by lsum_block_offsets); caller-owned              */
} lsum_block;

/* A change dZ of the charge at site `site` (indices 0..L-1 per axis) of block `block`:
 * dZ = -charge is a vacancy, dZ = Z - charge an impurity of charge Z (Sec. 4.1). */
typedef struct {
    int block;
    int site[3];
    double dZ;
} lsum_defect;

typedef struct {
    lsum_kernel kernel;
    int N[3];                 /* odd cell counts                                               */
    double h;                 /* mesh size                                                     */
    int n_blocks;
    const lsum_block* blocks;
    int n_defects;
    const lsum_defect* defects;
    double eps;               /* > 0: RHOSVD to a Tucker tensor with relative Frobenius error
                                 <= eps (certified); <= 0: canonical output, no reduction     */
    int precision;            /* arithmetic of projection, core and tile (LSUM_FP64/FP32/BF16X3);
                                 for canonical output (eps <= 0) FP32/BF16X3 keep the factors
                                 that sampling reads rounded to FP32 (products and sums FP64);
                                 quadrature, collocation, shift-sums, SVD and truncation are
                                 always FP64                                                   */
    int tile_lo[3];           /* optional reconstruction tile: cells [lo, lo+T) per axis      */
    int tile_T[3];            /* T = 0: no tile                                                */
    int n_points;             /* optional: potential sampled at these points on completion    */
    const double* points;     /* 3 * n_points coordinates (x, y, z interleaved); caller-owned,
                                 must stay valid until the request finishes                   */
    double* values;           /* n_points results, written before the request finishes        */
    int points_on_device;     /* 1: points/values are device pointers on the context's device */
    int exact_sites;          /* 0: every site (and defect) is snapped to the centre of its cell
                                 (Sec. 3.2, error O(h)).  1: sites keep their exact positions:
                                 along each axis a site at (j + f) h, |f| <= 1/2, takes reference
                                 rows collocated at the sub-cell offset f (Galerkin entries of the
                                 shifted charge), and sites with the same f share them, so a
                                 lattice with b/h = p/q needs at most q row sets per axis.
                                 Offsets within 2^-30 of each other share the rows of the smallest
                                 (|f| <= 2^-30: the cell centre), which absorbs the rounding of
                                 x/h; a problem whose row sets exceed 2^30 doubles is rejected
                                 (LSUM_E_INVALID)                                               */
    int method;               /* with eps > 0: LSUM_SUM_CANONICAL (0) assembles the canonical sum
                                 and reduces it by RHOSVD (Sec. 4); LSUM_SUM_TUCKER_REF (1) takes
                                 the rank-r Tucker form of the reference (RHOSVD of one charge on
                                 the doubled box at eps) and assembles its vectors over the lattice
                                 (Thm thm:sumCaseE (B)), then orthonormalises them per mode: one
                                 block keeps the reference's ranks for every L; a union of blocks
                                 (e.g. vacancy or impurity sub-lattices as blocks of charge -1 or
                                 Z - 1) is reduced by the generalised RHOSVD of Thm
                                 thm:TSum2Tucker at eps (lsum_info: norm_A = ||U|| of the sum,
                                 bound = its certified truncation bound, 0 for one block).  Needs
                                 eps > 0, FP64, no defects and exact_sites = 0 (LSUM_E_INVALID
                                 otherwise)                                                     */
    int als_sweeps;           /* 0..64: ALS sweeps after the RHOSVD (Thm thm:C2Tucker (b)): per
                                 mode the leading r_l left singular vectors of the sum projected
                                 onto the other modes' factors; the ranks stay, ||core|| only
                                 grows and the certified bound still holds.  Applied when every
                                 r_a r_b <= 4096 and r_l <= r_a r_b (otherwise skipped, reported
                                 in lsum_get_stats).  With LSUM_SUM_TUCKER_REF it refines the
                                 reference's Tucker form (the paper's C2T).                    */
} lsum_problem;

/* ---- host-side steps (FP64 / integer, no device work) ----------------------------------- */

/* Sinc quadrature of the kernel's Laplace-Gauss transform (Sec. 2.1 eqs. laplace, hM,
 * sinc_Newt; Sec. 2.2 eqs. LalpNewt, LalpYukawa with exponent param^2/(4 t^2), LalpSlater).
 * Writes up to `cap` nodes t[] and weights w[] (nodes with w < 1e-18 max w are dropped) and
 * the rank R = number written.  Needs N and h only for the default (h_u, s). */
int lsum_nodes(const lsum_kernel* k, const int N[3], double h, double* t, double* w, int cap,
               int* R);

/* Parallelogram-type lattice (Sec. 4.4 case (B)): the sites of `base` with coordinate
 * `shear_axis` moved by (k - (L-1)/2) * shear, k the site index along `along_axis` (the two axes
 * differ).  Written as the base->L[along_axis] rectangular blocks of one site along that axis
 * (out[0..*n), cap at least that many), whose sum the canonical route assembles with its
 * shared axes once.  base->x[shear_axis] must be NULL.  Host only. */
int lsum_shear_blocks(const lsum_block* base, int shear_axis, int along_axis, double shear, int cap,
                      lsum_block* out, int* n);

/* Lattice with the tensor structure in one axis only (Sec. 4.4 case (C)): the sites of `base`
 * along `axis` (its L, b, center or explicit coordinates), repeated at each of the n points of
 * the plane of the two other axes (pts: n pairs in increasing axis order).  Written as n blocks
 * of one site in those two axes (out[0..n), cap at least n), which the canonical route sums with
 * the column axis once; the rank grows with n, as the paper notes.  Host only. */
int lsum_column_blocks(const lsum_block* base, int axis, int n, const double* pts, int cap,
                       lsum_block* out);

/* Snapped cell indices of a block's sites (windowing offsets of Sec. 3.1 eq. sub_tens for the
 * centred lattice of Sec. 3.2): offs[0..L0-1] axis 0, then L1 for axis 1, then L2 for axis 2.
 * Bit-exact IEEE FP64 arithmetic: x = (k - (L-1)/2) * b + center; u = x / h. */
int lsum_block_offsets(const lsum_block* blk, const int N[3], double h, int32_t* offs);

/* Error control of the sinc rule (Sec. 2.1, the max-norm bound after eq. sinc_general).
 * P is the Galerkin tensor (cell averages) of one unit charge on the doubled reference box that
 * shift-and-windowing reads: displacements (i, j, k) h with |i| <= N_1 - 1, |j| <= N_2 - 1,
 * |k| <= N_3 - 1.  P_R is the rule of `k` (its M, h_u, s; defaults as for lsum_nodes).
 * *err = max |P - P_R| / max |P|, the maxima taken over probe cells: every displacement with
 * all |components| <= 4, and log-spaced cells (ratio 3/2) out to the box corner along six
 * directions (entries depend only on the sorted |components|).  The exact entries are
 * integrated on the host in FP64 to far below rounding.  Host only; a few ms for N ~ 4097. */
int lsum_sinc_error(const lsum_kernel* k, const int N[3], double h, double* err);

/* The smallest M in [1, M_max] (M_max <= 4096) whose rule (the kernel's h_u and s; k->M is
 * ignored) has lsum_sinc_error <= eps: *M and its *err.  When none does, returns LSUM_E_NOCONV
 * with the M of the smallest error in *M and that error in *err: the step h_u, not M, then
 * limits the accuracy (a smaller h_u lowers that floor). */
int lsum_choose_M(const lsum_kernel* k, const int N[3], double h, double eps, int M_max, int* M,
                  double* err);

/* ---- context ----------------------------------------------------------------------------- */
typedef struct lsum_ctx_s* lsum_ctx;
typedef struct lsum_req_s* lsum_req;

/* Create a context on HIP device `device` with `hbm_budget_bytes` of HBM for request data
 * (0: 80% of the device's free memory) and `n_slots` concurrent request slots (each slot a
 * HIP stream and a worker thread; 0: 4).  The context owns its streams, caches and workers. */
int lsum_create(lsum_ctx* ctx, int device, size_t hbm_budget_bytes, int n_slots);
/* Stops the workers (queued requests finish as LSUM_E_CANCELLED); device memory is freed when
 * the last unreleased request of the context is released. */
int lsum_destroy(lsum_ctx ctx);
const char* lsum_last_error(void);

/* Options: LSUM_OPT_MAX_BATCH (default 32): consecutive canonical requests (eps <= 0) a slot
 * fuses into one batch whose shift-sums run as one launch (1: no batching).
 * LSUM_OPT_REF_CACHE_BYTES (default 4 GiB): HBM kept for reference vectors shared by requests
 * with the same kernel, quadrature and grid (0: every request recomputes its own).
 * LSUM_OPT_RANGE_MIN (default 64): side matrices with min(D, N) at least this large are
 * compressed to a randomized range basis, grown in blocks of 128 vectors up to min(D, N),
 * before the Jacobi SVD (the residual outside the basis is computed exactly and enters the
 * certified tail; the directions below a tenth of the threshold then never reach the Jacobi
 * sweeps); 0 disables the compression.
 * LSUM_OPT_JACOBI_STOP (default 1): the Jacobi SVD of a side matrix (Def. def:RHOSVD) ends as
 * soon as the certified truncation rank is the same after two sweeps and the rows kept for it
 * are orthogonal; the reported sigma beyond that rank are then row norms whose squared sum
 * bounds the true tail from above (the error bound of Thm thm:C2Tucker (d) still holds).  0: sweep to
 * full convergence, every sigma a singular value to the Jacobi tolerance. */
#define LSUM_OPT_MAX_BATCH 1
#define LSUM_OPT_REF_CACHE_BYTES 2
#define LSUM_OPT_RANGE_MIN 3
#define LSUM_OPT_JACOBI_STOP 4
/* LSUM_OPT_JACOBI_MAX_SWEEPS (default 40, 1..1000): sweeps a side-matrix SVD may take; a request
 * whose SVD has not converged by then fails with LSUM_E_NOCONV (a bound on its latency).  Read
 * when a request's SVD starts. */
#define LSUM_OPT_JACOBI_MAX_SWEEPS 5
/* How the sweeps of a Jacobi SVD are launched; for a given block width (LSUM_OPT_JACOBI_BLOCK
 * below) every way gives the same results bit for bit.
 * Default: round by round (three launches per round of disjoint column-block pairs).
 * LSUM_OPT_JACOBI_PERSISTENT (default 0; 1: groups of 16 waves, 2: groups of 4 waves): a sweep
 * is one launch with one workgroup per pair of column blocks, its rounds ordered by per-block
 * completion counters in device memory; it runs persistently while the persistent workgroups
 * in flight fit 3/4 of the device, else round by round.  Each wait is bounded by
 * LSUM_OPT_JACOBI_WAIT_US (default 20000 microseconds, 0..1e8):
 * when the workgroups are not all resident at once the sweep aborts; it read the rows before it
 * and wrote only a second buffer, so it runs again round by round from those rows (the result
 * is unchanged; lsum_get_stats counts such sweeps in "jacobi_aborted"), and the rest of that
 * SVD launches round by round.
 * LSUM_OPT_GRAPHS (default 0; applies when not persistent): the round-by-round launches of a
 * sweep are captured once per block count in a HIP graph and replayed. */
#define LSUM_OPT_GRAPHS 6
#define LSUM_OPT_JACOBI_PERSISTENT 7
#define LSUM_OPT_JACOBI_WAIT_US 8
/* LSUM_OPT_AUTOTUNE (default 1): launch variants that add the same terms in the same order (the
 * four ways of launching a Jacobi sweep above; the shift-sum's 16- or 48-node workgroup tiles)
 * are timed on the first launch of each shape bucket and the fastest is used from then on; the
 * choice never changes a result.  With it, the sweep ways chosen override the two options
 * above.  0: the options and fixed thresholds decide. */
#define LSUM_OPT_AUTOTUNE 9
/* LSUM_OPT_GEMM_LIBRARY (default 1; applies to the whole process, not only this context): plain
 * FP64 products with unit-stride operands and at least 2^24 multiply-adds (the range basis,
 * the singular vectors, FP64 projections and core GEMMs, lsum_contract) run on the ROCm BLAS
 * library's DGEMM with atomics disabled (results independent of concurrent work); 0: every
 * product on this library's own MFMA kernels.  FP32 products always run on the library's own
 * kernel (FP32 partial sums of 32 terms added in FP64). */
#define LSUM_OPT_GEMM_LIBRARY 11
/* LSUM_OPT_JACOBI_BLOCK (default 0; or 8, 16, 32): columns per Jacobi block.  Blocks of 16 (pair
 * problems of 32 columns, solved by four waves) halve the rounds of a sweep, blocks of 32 (pair
 * problems of 64 columns, eight waves) halve them again and with them the bytes a sweep moves;
 * such sweeps run round by round (directly or from graphs).  0: 32 for side matrices of at least
 * 512 rows (the columns the SVD rotates), 16 below (a function of the size alone, never of
 * the load).  The persistent ways (LSUM_OPT_JACOBI_PERSISTENT) need blocks of 8.  Every width
 * gives an SVD to the same tolerance and the same certificate, not the same bits. */
#define LSUM_OPT_JACOBI_BLOCK 12
/* LSUM_OPT_JACOBI_SKIP (default 1; or 0): with 16-column blocks, the pair solve leaves out
 * rotations whose relative coupling |g_ab| / sqrt(g_aa g_bb) is at most a tenth of the sweep
 * tolerance, and a step of the pair's cyclic sweep with no rotation left is skipped; 0: every
 * rotation above the rounding floor (1e-16) is applied.  The sweeps end on the same
 * convergence test either way. */
#define LSUM_OPT_JACOBI_SKIP 13
int lsum_set_option(lsum_ctx ctx, int key, double value);
/* The autotuner's decisions of earlier runs on a device of the same architecture and compute
 * unit count are read from the text file at `path` (if it exists), and new ones are appended to
 * it ("<device> <bucket> <choice> <ms per variant ...>" per line). */
int lsum_tune_file(lsum_ctx ctx, const char* path);
/* JSON of the autotuner's decisions: {"device", "file", "enabled", "decisions": {bucket:
 * {"choice", "ms": [per variant, -1 if not measured]}}}; returns the full length (copy into
 * buf of len bytes, truncated, NUL-terminated). */
int lsum_get_tuning(lsum_ctx ctx, char* buf, size_t len);
/* Per stage (collocate, shift_sum, transpose, columns, norm, svd, projection, core, tile,
 * sample): summed event-timed GPU milliseconds, number of timed launches, and the algorithmic
 * bytes and flops those launches had to move or compute, as JSON; returns the needed length. */
int lsum_get_profile(lsum_ctx ctx, char* buf, size_t len);
int lsum_reset_profile(lsum_ctx ctx);

/* ---- device steps of the path (each one kernel family, on `stream`) --------------------- */

/* Reference vectors (Sec. 2.1 b(t_k); Sec. 3.1 eq. master_pot): G_dev[q*ldg + m],
 * q < R, m < 2*N_ref-1, from host nodes t[R], weights w[R].  ldg >= 2*N_ref-1. */
int lsum_collocate(lsum_ctx ctx, void* stream, int R, const double* t, const double* w,
                   int N_ref, double h, double* G_dev, int ldg);

/* Assembled 1D sums (Thm thm:sumCaseE (A)): U_dev[q*ldu + i] = sum_k G[q*ldg + i - c_k +
 * N_ref - 1] for i < N_axis, over the n_sites host cell indices c_k (0 <= c_k < N_axis <=
 * N_ref), in any order; ldg >= max(2, 2*N_ref-1).  FP64.  The form with the fewest terms is
 * taken: when the sites form p interleaved uniform combs (c_{k+p} - c_k constant), each comb is
 * summed first (as a windowed strided sum of the row) and the p comb sums are added in order;
 * when they split into fewer runs of one stride S than that (at least 6 sites, no period of 8
 * or less), each run is the difference of two compensated strided prefix (or suffix) sums of the
 * row, whose error is a few units of roundoff of the row's sum |G| rather than of the value;
 * otherwise the sites are added in order k = 0..n-1.  Errors: LSUM_E_INVALID for bad sizes or
 * null pointers, LSUM_E_OUT_OF_BOX for a site outside [0, N_axis).  Synchronous. */
int lsum_shift_sum(lsum_ctx ctx, void* stream, int R, const double* G_dev, int ldg, int N_ref,
                   int N_axis, int n_sites, const int32_t* sites, double* U_dev, int ldu);

/* Allocation-free variant of lsum_shift_sum, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, result (bitwise) and errors; the job descriptor, term list and window tables live
 * in a static device array of 64 MiB per device (held until the process ends) instead of pool
 * memory, so the call makes no allocation.  LSUM_E_NOMEM when the call needs more scratch than
 * that: 256 B + 8 B per term + up to two R x ldg FP64 tables (window, prefix or suffix sums).  Every call on a device
 * shares that device's array: calls that overlap on one device race.  Synchronous. */
int lsum_shift_sum_noalloc(lsum_ctx ctx, void* stream, int R, const double* G_dev, int ldg,
                           int N_ref, int N_axis, int n_sites, const int32_t* sites,
                           double* U_dev, int ldu);

/* Potential of a canonical sum at points (eq. CP_form evaluated pointwise):
 * out_dev[p] = sum_f lam_f sum_q prod_l U_f,l[q, i_l(p)] over n_fac factor sets, where
 * i_l(p) snaps xyz_dev[3p+l]; U_dev holds n_fac sets of 3 axis blocks, each R x ldu
 * (set f, axis l at offset (3f+l)*R*ldu).  Points outside the grid yield NaN. */
int lsum_sample_canonical(lsum_ctx ctx, void* stream, int n_fac, int R, const double* U_dev,
                          int ldu, const double* lam, const int N[3], double h, int n_pts,
                          const double* xyz_dev, double* out_dev);

/* Truncated SVD of a side matrix (Def. def:RHOSVD): the D columns a_j (row j of A_dev, length
 * N, stride lda) are rotated in place by a one-sided block-Jacobi SVD in FP64 until every
 * pair of columns whose norms both exceed `irrelevant` has relative coupling
 * |a_i.a_j|/(|a_i||a_j|) <= tol (irrelevant <= 0: 1e-15 of the largest column norm).  On return
 * the rows of A_dev hold the rotated columns sorted by descending norm and sigma[0..D-1] (host)
 * their norms; the leading rows divided by sigma are left singular vectors, and for every r the
 * residual of projecting A onto the first r of them is at most (sum_{k>=r} sigma_k^2)^(1/2).
 * Synchronous.  Returns LSUM_E_NOCONV after `max_sweeps` sweeps without convergence (results
 * are still written). */
int lsum_jacobi_svd(lsum_ctx ctx, void* stream, int D, int N, double* A_dev, int lda,
                    double tol, double irrelevant, int max_sweeps, double* sigma, int* sweeps);

/* Dense contraction used by the projections Z^T A (Appendix theorem (c)) and the mode
 * products of the Tucker reconstruction (eq. Tucker_singePot): C(m,n) = alpha * sum_k A(m,k)
 * B(k,n) + beta * C(m,n) with A(m,k) = A_dev[m*sam + k*sak], B(k,n) = B_dev[k*sbk + n*sbn],
 * C(m,n) = C_dev[m*scm + n*scn] (element strides).  prec: LSUM_FP64 (double operands, FP64
 * MFMA), LSUM_FP32 (float operands, FP32 MFMA) or LSUM_BF16X3 (float operands split into two
 * bfloat16 parts, three BF16 MFMA products, FP32 accumulation).  Large unit-stride FP64
 * products go to the ROCm BLAS library (LSUM_OPT_GEMM_LIBRARY).  Synchronous. */
int lsum_contract(lsum_ctx ctx, void* stream, int prec, int m, int n, int k, const void* A_dev,
                  long sam, long sak, const void* B_dev, long sbk, long sbn, void* C_dev, long scm,
                  long scn, double alpha, double beta);

/* ---- requests (the whole path for one problem) ------------------------------------------ */

/* Validate and enqueue a problem; the caller's arrays are deep-copied, so they may be freed on
 * return.  Non-blocking: LSUM_E_BUSY if `nonblocking` and the queue is full.  The request is
 * admitted when its planned HBM footprint fits the free budget (LSUM_E_NOMEM if it can never
 * fit).  Requests run concurrently on the context's slots. */
int lsum_submit(lsum_ctx ctx, const lsum_problem* p, int nonblocking, lsum_req* req);
/* Submit n problems p[0..n-1] at once (req[i] receives request i).  All are validated first
 * (on any error none is queued and the error of the first bad problem is returned); they enter
 * the queue together, so a slot can fuse consecutive canonical ones into one batch of up to
 * LSUM_OPT_MAX_BATCH requests (one shift-sum launch). */
int lsum_submit_many(lsum_ctx ctx, int n, const lsum_problem* p, int nonblocking, lsum_req* req);
/* Wait up to timeout_ms (< 0: forever); returns the request's final status or LSUM_E_TIMEOUT. */
int lsum_wait(lsum_req req, int timeout_ms);
/* Cancel a request that has not started (LSUM_E_STATE once it runs). */
int lsum_cancel(lsum_req req);

typedef struct {
    int status;        /* LSUM_OK, a negative error, or 1 while queued/running               */
    int R;             /* quadrature rank                                                    */
    int n_terms;       /* canonical terms R * (n_blocks + n_defects)                         */
    int is_tucker;     /* 1 if reduced to Tucker format                                      */
    int r[3];          /* Tucker ranks                                                       */
    int D[3];          /* distinct side-matrix columns per mode                              */
    double norm_A;     /* Frobenius norm of the canonical tensor                             */
    double norm_xi;    /* ||xi||                                                             */
    double bound;      /* ||xi|| sum_l tail_l: certified bound on ||A - A0||_F              */
    double rel_bound;  /* bound / norm_A                                                     */
    double t_queue_ms, t_run_ms;  /* enqueue->start, start->finish                            */
    /* The result's own error (Tucker results; -1 for canonical ones, which are the canonical sum
     * itself): at n_probe seeded cells, max |V(cell) - A(cell)| / max |A(cell)|, V the result
     * evaluated as any sample (in the request's precision) and A the untruncated canonical sum
     * in FP64 -- the discrete tensor the direct sum over the charges gives.  It holds the
     * truncation error (certified in Frobenius norm by `bound`) and the rounding of the FP32 /
     * split-BF16x3 contractions together. */
    double probe_err;
    int n_probe;
} lsum_info;
int lsum_get_info(lsum_req req, lsum_info* info);

/* Canonical factors of block `block` (eq. CP_form; Thm thm:sumCaseE (A)): the block's part of the
 * sum is weight * sum_q U0[q, :] (x) U1[q, :] (x) U2[q, :].  U_l (vector-major, R rows of N[l]
 * each; host, or device if on_device; NULL skips an axis) carry the node weights as w_q^(1/3)
 * per axis; *weight (host; NULL skips it) receives the block's charge.  Factors kept in FP32
 * (canonical output at FP32/BF16X3 precision) are returned widened to double. */
int lsum_get_canonical(lsum_req req, int block, double* U0, double* U1, double* U2, double* weight,
                       int on_device);
/* Galerkin matrix of a finished Tucker result in a separable basis (eq. nuc_pot): basis function
 * k is g_k(x) = g_k^(1)(x_1) g_k^(2)(x_2) g_k^(3)(x_3), given by its values at the cell centres,
 * G_l (nb x N_l, row k = g_k^(l), row-major).  V[k * nb + m] = h^3 sum_i T_i g_k(x_i) g_m(x_i),
 * the midpoint rule for the integral of v g_k g_m, computed from 1D Hadamard products and the
 * Tucker factors and core (MFMA products).  nb <= 255; G and V in host memory, or device memory
 * if on_device.  Synchronous. */
int lsum_galerkin(lsum_req req, int nb, const double* G0, const double* G1, const double* G2,
                  double* V, int on_device);

/* Canonical form of a finished Tucker result (the canonical -> Tucker -> canonical rank
 * reduction of Sec. 4.2): each mode-3 slice of the core by its SVD, mu[:, :, k] = sum_i s_i
 * u_i v_i^T, gives orthogonal rank-1 terms s_i (Z_1 u_i) (x) (Z_2 v_i) (x) z_3,k, so the rank is
 * at most r_3 min(r_1, r_2); the smallest s are dropped while their (sum s^2)^(1/2) stays
 * <= eps ||core||, which is then the Frobenius error (*err).  *R receives the rank; with xi ==
 * NULL nothing else is written (a size query).  Otherwise xi (R weights, decreasing) and U_l
 * (vector-major, R rows of N_l, unit rows; NULL skips a mode) are written to host memory, or
 * device memory if on_device; cap < R is LSUM_E_INVALID.  Needs r_1, r_2 <= 128 (the slices are
 * decomposed on the host).  Synchronous. */
int lsum_tucker_to_canonical(lsum_req req, double eps, int cap, int* R, double* xi, double* U0,
                             double* U1, double* U2, double* err, int on_device);
/* Tucker factors Z_l (r_l rows of N[l]) and core (r1*r2*r3, last index fastest), FP64. */
int lsum_get_tucker(lsum_req req, double* Z0, double* Z1, double* Z2, double* core, int on_device);
/* Singular values of the three side matrices, descending: min(D[l], N[l]) values (or the size of
 * the range basis, when one is used) are written into buffers of D[l] entries; the entries
 * after them are left as they are (the side matrix has no further nonzero values above the
 * basis residual, which the certified bound carries). */
int lsum_get_sigma(lsum_req req, double* s0, double* s1, double* s2);
/* Potential at n points xyz[3n]: the canonical sum with all defects, or the Tucker tensor.
 * Synchronous. */
int lsum_sample(lsum_req req, int n, const double* xyz, double* out, int on_device);
/* The reconstructed tile (T0*T1*T2 values, last index fastest) as float (precision FP32 or
 * BF16X3) or double (FP64); `elem_size` must match (4 or 8). */
int lsum_get_tile(lsum_req req, void* out, int elem_size, int on_device);
/* JSON with ranks, sigma tails, bound, stage times (ms) and bytes; returns the needed length. */
int lsum_get_stats(lsum_req req, char* buf, size_t len);
/* Free the request's device results and the handle. */
int lsum_release(lsum_req req);
/* Finish n requests in order: wait for each (no time limit), write its final status to
 * status[i] and, if info is not null, its lsum_info to info[i], then release it.  One call for
 * a client that harvests a batch of requests at once; the handles are invalid afterwards.
 * Returns LSUM_E_INVALID for a null request array or a null entry (nothing is released then). */
int lsum_finish_many(int n, lsum_req* req, int* status, lsum_info* info);

#ifdef __cplusplus
}
#endif
#endif /* LSUM_H */

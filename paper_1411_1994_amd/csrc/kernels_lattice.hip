// HIP kernels (gfx950) for the lattice stages: cell-average collocation of the quadrature
// Gaussians, assembled 1D shift-sums, side-matrix column gathering, and point evaluation.
// All arithmetic is FP64.  These stages stream memory (no dense contraction), so they use
// plain coalesced loads/stores and leave MFMA to the contraction kernels.
#include <hip/hip_runtime.h>

#include <string>
#include <vector>
#include <hip/hip_ext.h>

#include "lsum_internal.h"

namespace lsum {

namespace {

constexpr double kSqrtPi = 1.7724538509055160273;

// Pointers read from job descriptors are generic; casting them to the global (1) or constant (4)
// address space lets the compiler use global_load / s_load instead of flat accesses, whose
// shared counters force a full wait after every batch of loads.
#define LSUM_GLOBAL __attribute__((address_space(1)))
#define LSUM_CONST __attribute__((address_space(4)))

// --------------------------------------------------------------------------------------------
// Reference vectors (Sec. 2.1 b(t_k), Sec. 3.1 eq. master_pot): one thread per entry.
// Entry m of row q: w_q^(1/3) * (1/h) int over the cell at displacement d = (m-(N_ref-1)) h -
// shift of exp(-t_q^2 x^2) dx = w_q^(1/3) sqrt(pi)/(2 t h) [erf(t(|d|+h/2)) - erf(t(|d|-h/2))],
// with the complementary form when both ends are in the tail.  `shift` is the charge's offset
// from its cell centre (0 for a charge on the centre).  Padding entries are zero.
// --------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_collocate(int R, const double* __restrict__ t,
                                                   const double* __restrict__ w13, int N_ref,
                                                   double h, double shift, double* __restrict__ G,
                                                   int ldg) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    const int q = blockIdx.y;
    if (m >= ldg || q >= R) return;
    double v = 0.0;
    if (m < 2 * N_ref - 1) {
        const double d = fabs((double)(m - (N_ref - 1)) * h - shift);
        const double tq = t[q];
        double b = 1.0;
        if (tq > 0.0) {
            const double lo = tq * (d - 0.5 * h);
            const double hi = tq * (d + 0.5 * h);
            const double diff = lo > 1.0 ? erfc(lo) - erfc(hi) : erf(hi) - erf(lo);
            b = kSqrtPi / (2.0 * tq * h) * diff;
        }
        v = w13[q] * b;
    }
    G[(size_t)q * ldg + m] = v;
}

// --------------------------------------------------------------------------------------------
// Assembled 1D sums (Thm thm:sumCaseE (A)) for a batch of jobs: out[q, i] = sum_t
// +-T_tab(t)[q * ldg + i + off_t], summed in term order (bit 0 of tab picks the table, bit 1 the
// sign).  One workgroup per (64-cell tile, job).
// Each lane owns a pair of adjacent cells and loads both with one 16-byte access (the unit that
// bounds this kernel is the vector-memory path, not HBM: five 8-byte loads per output for the
// period-5 combs of a 64-site axis); the two halves of a wavefront serve two node slots, so the
// 8 slots of the workgroup take nodes s, s + 8, ..., s + 40 of each block of 48 nodes, and the
// loads of two terms for all six nodes are in flight together.  Vector-major rows are stored
// from the lanes; point-major rows (FP64, or rounded to FP32) go through an LDS tile so the 64
// rows of a tile (padded with zeros to ldt) leave as contiguous memory.  Stores are
// non-temporal so they do not evict the tables from L2.
// --------------------------------------------------------------------------------------------
typedef double dpair __attribute__((ext_vector_type(2), aligned(8)));

// A register budget for 6 waves per SIMD (the limit the LDS tile sets anyway): more waves in
// flight hide more of the gather latency (1024 jobs: 11 % faster than the compiler's own budget,
// which leaves 5).
// The grid is one-dimensional, tx x ny x nz work-groups (cell tile, job, node block) numbered so
// that consecutive numbers stay on one XCD (the hardware deals work-groups round-robin over the
// 8 XCDs): a job's tiles are then contiguous on one XCD and its table rows are fetched into that
// XCD's L2 only, where the terms of all its tiles re-read them.
template <int NU>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 8))) k_shift_sum(const ShiftJob* __restrict__ jobs,
                                                                                              int tx, int ny, int nz) {
    constexpr int QB = 8 * NU, TU = 2;
    __shared__ double tile[64][QB + 1];
    const int per_xcd = (int)(gridDim.x / 8);
    const int v = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
    if (v >= tx * ny * nz) return;
    const int bx = v % tx, by = (v / tx) % ny, bz = v / (tx * ny);
    const ShiftJob& jb = jobs[by];
    const int N = jb.N_axis;
    const int i0 = bx * 64;
    if (i0 >= N) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int pr = lane & 31;
    const int slot = 2 * wave + (lane >> 5);
    const int c0 = i0 + 2 * pr;
    // the pair loaded is (cc, cc + 1) with cc + 1 < max(N, 2) so that every load stays inside the
    // rows; a lane whose first cell is the last one (odd tail) takes it as the second of its pair
    const int cc = max(0, min(c0, N - 2));
    const bool shifted = cc != c0;
    const LSUM_CONST int* __restrict__ terms = (const LSUM_CONST int*)jb.terms;   // (off, tab) pairs
    const int nt = jb.n_terms;
    const size_t ldg = (size_t)jb.ldg;
    const LSUM_GLOBAL double* __restrict__ T0 = (const LSUM_GLOBAL double*)jb.T0 + cc;
    const LSUM_GLOBAL double* __restrict__ T1 = (const LSUM_GLOBAL double*)(jb.T1 ? jb.T1 : jb.T0) + cc;
    LSUM_GLOBAL double* __restrict__ U = (LSUM_GLOBAL double*)jb.U;
    LSUM_GLOBAL double* __restrict__ UT = (LSUM_GLOBAL double*)jb.UT;
    LSUM_GLOBAL float* __restrict__ UT32 = (LSUM_GLOBAL float*)jb.UT32;
    const bool rows = UT || UT32;
    for (int q0 = bz * QB; q0 < jb.R; q0 += nz * QB) {
        const int qn = min(QB, jb.R - q0);
        size_t qo[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u) qo[u] = (size_t)(q0 + min(slot + 8 * u, qn - 1)) * ldg;
        dpair acc[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u) acc[u] = dpair{0.0, 0.0};
        for (int t = 0; t < nt; t += TU) {
            dpair v[TU][NU];
            double sg[TU];
#pragma unroll
            for (int e = 0; e < TU; ++e) {
                const int te = min(t + e, nt - 1);
                const int tab = terms[2 * te + 1];
                const LSUM_GLOBAL double* r = ((tab & 1) ? T1 : T0) + terms[2 * te];
                sg[e] = (tab & 2) ? -1.0 : 1.0;
#pragma unroll
                for (int u = 0; u < NU; ++u) v[e][u] = *(const LSUM_GLOBAL dpair*)(r + qo[u]);
            }
            // a sign of +-1 scales exactly: acc + sg v rounds as acc +- v
#pragma unroll
            for (int e = 0; e < TU; ++e)
                if (t + e < nt)
#pragma unroll
                    for (int u = 0; u < NU; ++u) acc[u] += sg[e] * v[e][u];
        }
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int kk = slot + 8 * u;
            if (kk >= qn) continue;
            const double a = shifted ? acc[u].y : acc[u].x;
            if (U) {
                LSUM_GLOBAL double* row = U + (size_t)(q0 + kk) * jb.ldu;
                if (c0 < N) __builtin_nontemporal_store(a, row + c0);
                if (!shifted && c0 + 1 < N) __builtin_nontemporal_store(acc[u].y, row + c0 + 1);
            }
            if (rows) {
                tile[2 * pr][kk] = a;
                tile[2 * pr + 1][kk] = acc[u].y;
            }
        }
        if (rows) {
            __syncthreads();
            const int nr = min(64, N - i0);
            const int width = min(QB, jb.ldt - q0);   // includes the zero padding after R
            // (row, column) of the tile flattened over the workgroup, QB columns per row
            for (int e = threadIdx.x; e < nr * QB; e += 256) {
                const int rr = e / QB, cl = e - rr * QB;
                if (cl >= width) continue;
                const double v = cl < qn ? tile[rr][cl] : 0.0;
                const size_t o = (size_t)(i0 + rr) * jb.ldt + q0 + cl;
                if (UT) __builtin_nontemporal_store(v, &UT[o]);
                else __builtin_nontemporal_store((float)v, &UT32[o]);
            }
            __syncthreads();
        }
    }
}

// Windowed strided sums of the reference rows: Q[q, x] = sum_{m=0}^{n-1} G[q, x - m S] (terms
// with x - m S < 0 are absent).  A comb of n sites c, c + S, ..., c + (n-1) S adds
// Q[q, i + N_ref - 1 - c] to cell i.  n = kPrefixSums sums the whole chain below x and
// n = kSuffixSums the chain above it (x + m S < ldg); those two are compensated sums
// (Neumaier's variant of Kahan summation), since a run of sites is read as the difference of
// two of them.
__global__ void __launch_bounds__(256) k_window_sums(int ldg, const double* __restrict__ G, int S, int n,
                                                     double* __restrict__ Q) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= ldg) return;
    const double* g = G + (size_t)blockIdx.y * ldg;
    double acc = 0.0;
    if (n > 0) {
        for (int m = 0, y = x; m < n && y >= 0; ++m, y -= S) acc += g[y];
    } else {
        const int step = n == kSuffixSums ? S : -S;
        double comp = 0.0;
        for (int y = x; y >= 0 && y < ldg; y += step) {
            const double v = g[y], s = acc + v;
            comp += fabs(acc) >= fabs(v) ? (acc - s) + v : (v - s) + acc;
            acc = s;
        }
        acc += comp;
    }
    Q[(size_t)blockIdx.y * ldg + x] = acc;
}

__device__ __forceinline__ int snap_dev(double x, double h, int N) {
    const double u = x / h;
    double j = floor(fabs(u) + 0.5);
    if (u < 0.0) j = -j;
    const double i = j + (double)((N - 1) / 2);
    return (i >= 0.0 && i <= (double)(N - 1)) ? (int)i : -1;
}

// Canonical sum at points: out[p] = sum_f lam_f sum_q prod_l U[f][l][q, i_l(p)].
__global__ void __launch_bounds__(256) k_sample_cp(int n_fac, int R, const double* __restrict__ U,
                                                   int ldu, const double* __restrict__ lam, int N0,
                                                   int N1, int N2, double h, int n_pts,
                                                   const double* __restrict__ xyz,
                                                   double* __restrict__ out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_pts) return;
    const int i0 = snap_dev(xyz[3 * (size_t)p + 0], h, N0);
    const int i1 = snap_dev(xyz[3 * (size_t)p + 1], h, N1);
    const int i2 = snap_dev(xyz[3 * (size_t)p + 2], h, N2);
    if (i0 < 0 || i1 < 0 || i2 < 0) {
        out[p] = __builtin_nan("");
        return;
    }
    const size_t axis = (size_t)R * ldu;
    double total = 0.0;
    for (int f = 0; f < n_fac; ++f) {
        const double* u0 = U + (3 * (size_t)f + 0) * axis + i0;
        const double* u1 = U + (3 * (size_t)f + 1) * axis + i1;
        const double* u2 = U + (3 * (size_t)f + 2) * axis + i2;
        double acc = 0.0;
        for (int q = 0; q < R; ++q)
            acc += u0[(size_t)q * ldu] * u1[(size_t)q * ldu] * u2[(size_t)q * ldu];
        total += lam[f] * acc;
    }
    out[p] = total;
}

// Vector-major R x N rows -> point-major N x R rows, through a 32 x 32 LDS tile.
template <typename T>
__global__ void __launch_bounds__(256) k_transpose(int R, int N, const T* __restrict__ U, int ldu,
                                                   double* __restrict__ UT) {
    __shared__ double tile[32][33];
    const int i0 = blockIdx.x * 32, q0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int k = ty; k < 32; k += 8) {
        const int q = q0 + k, i = i0 + tx;
        tile[k][tx] = (q < R && i < N) ? (double)U[(size_t)q * ldu + i] : 0.0;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int i = i0 + k, q = q0 + tx;
        if (i < N && q < R) UT[(size_t)i * R + q] = tile[tx][k];
    }
}

// Canonical sums at points from point-major factors, for a batch of requests in one launch.
// Row i of axis l holds the values of cell i for every node, rows ldt apart, zero padded, ldt a
// multiple of 16 elements.  A point's row is read in 16-byte pieces by LP lanes (8 for FP64
// rows, 4 for FP32 rows; NQ = ldt / 16 pieces per lane and row), so one wave instruction moves
// 64 full 16-byte lanes; products and sums are formed in FP64, reduced over the LP lanes, and
// the blocks' charges applied in block order: out[p] = sum_b lam_b sum_q prod_l T_bl[i_l(p)][q].
// Work-groups are numbered so that consecutive numbers stay on one XCD (the hardware deals
// work-groups round-robin over the 8 XCDs): each request's work-groups are contiguous in that
// numbering, so its factor rows are fetched into one or two XCD L2 caches instead of all eight.
typedef float fquad __attribute__((ext_vector_type(4)));
template <typename T> struct RowPiece;
template <> struct RowPiece<double> {
    using V = dpair;
    static constexpr int E = 2;
    __device__ static double dot3(V x, V y, V z) {
        return x.x * y.x * z.x + x.y * y.y * z.y;
    }
};
template <> struct RowPiece<float> {
    using V = fquad;
    static constexpr int E = 4;
    __device__ static double dot3(V x, V y, V z) {
        double a = (double)x.x * (double)y.x * (double)z.x;
        a += (double)x.y * (double)y.y * (double)z.y;
        a += (double)x.z * (double)y.z * (double)z.z;
        a += (double)x.w * (double)y.w * (double)z.w;
        return a;
    }
};

template <int NQ, typename T>
__global__ void __launch_bounds__(256) k_sample_batch(int ldt, const SampleJob* __restrict__ jobs_in,
                                                      int n_jobs, int n_wg) {
    using RP = RowPiece<T>;
    using V = typename RP::V;
    constexpr int LP = 16 / RP::E, PPW = 256 / LP;
    const int per_xcd = gridDim.x / 8;
    const int w = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
    if (w >= n_wg) return;
    const LSUM_CONST SampleJob* jobs = (const LSUM_CONST SampleJob*)jobs_in;
    int lo = 0, hi = n_jobs - 1;   // last job whose first work-group is <= w
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].wg0 <= w) lo = mid;
        else hi = mid - 1;
    }
    const LSUM_CONST SampleJob& jb = jobs[lo];
    const int lp = threadIdx.x % LP;
    const int p = (w - jb.wg0) * PPW + (int)(threadIdx.x / LP);
    const bool live = p < jb.n_pts;
    const LSUM_GLOBAL double* xyz = (const LSUM_GLOBAL double*)jb.xyz + 3 * (size_t)(live ? p : 0);
    const double h = jb.h;
    const int i0 = snap_dev(xyz[0], h, jb.N0), i1 = snap_dev(xyz[1], h, jb.N1), i2 = snap_dev(xyz[2], h, jb.N2);
    const bool in = live && i0 >= 0 && i1 >= 0 && i2 >= 0;
    const size_t r0 = (size_t)(in ? i0 : 0) * ldt + RP::E * lp;
    const size_t r1 = (size_t)(in ? i1 : 0) * ldt + RP::E * lp + jb.off1;
    const size_t r2 = (size_t)(in ? i2 : 0) * ldt + RP::E * lp + jb.off2;
    const LSUM_CONST SampleBlock* blk = (const LSUM_CONST SampleBlock*)jb.blk;
    double total = 0.0;
    for (int b = 0; b < jb.n_blocks; ++b) {
        const LSUM_GLOBAL T* tb = (const LSUM_GLOBAL T*)blk[b].T;
        double acc = 0.0;
        if (NQ > 0) {
            V x[NQ > 0 ? NQ : 1], y[NQ > 0 ? NQ : 1], z[NQ > 0 ? NQ : 1];
#pragma unroll
            for (int k = 0; k < (NQ > 0 ? NQ : 1); ++k) {
                x[k] = *(const LSUM_GLOBAL V*)(tb + r0 + 16 * k);
                y[k] = *(const LSUM_GLOBAL V*)(tb + r1 + 16 * k);
                z[k] = *(const LSUM_GLOBAL V*)(tb + r2 + 16 * k);
            }
#pragma unroll
            for (int k = 0; k < (NQ > 0 ? NQ : 1); ++k) acc += RP::dot3(x[k], y[k], z[k]);
        } else {
            for (int k = 0; k < ldt / 16; ++k)
                acc += RP::dot3(*(const LSUM_GLOBAL V*)(tb + r0 + 16 * k), *(const LSUM_GLOBAL V*)(tb + r1 + 16 * k),
                                *(const LSUM_GLOBAL V*)(tb + r2 + 16 * k));
        }
        for (int m = LP / 2; m > 0; m >>= 1) acc += __shfl_xor(acc, m, LP);
        total += blk[b].lam * acc;
    }
    if (lp == 0 && live) ((LSUM_GLOBAL double*)jb.out)[p] = in ? total : __builtin_nan("");
}

// Defect terms straight from the reference rows: out[p] += sum_s dZ_s sum_q prod_l
// G[q, i_l(p) + off_s,l] (the windowed reference tensor of Sec. 3.1 per defect; off = N_ref - 1
// - c for a defect in cell c, plus the offset of its row table when sites are off grid).
__global__ void __launch_bounds__(256) k_sample_windows(int R, const double* __restrict__ G, int ldg,
                                                        int n_def,
                                                        const int32_t* __restrict__ offs,
                                                        const double* __restrict__ scale, int N0,
                                                        int N1, int N2, double h, int n_pts,
                                                        const double* __restrict__ xyz,
                                                        double* __restrict__ out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_pts) return;
    const int i0 = snap_dev(xyz[3 * (size_t)p + 0], h, N0);
    const int i1 = snap_dev(xyz[3 * (size_t)p + 1], h, N1);
    const int i2 = snap_dev(xyz[3 * (size_t)p + 2], h, N2);
    if (i0 < 0 || i1 < 0 || i2 < 0) return;
    double total = 0.0;
    for (int s = 0; s < n_def; ++s) {
        const int m0 = i0 + offs[3 * s + 0];
        const int m1 = i1 + offs[3 * s + 1];
        const int m2 = i2 + offs[3 * s + 2];
        double acc = 0.0;
        for (int q = 0; q < R; ++q) {
            const double* g = G + (size_t)q * ldg;
            acc += g[m0] * g[m1] * g[m2];
        }
        total += scale[s] * acc;
    }
    out[p] += total;
}

// Side-matrix columns of one mode (Sec. 4.2 side matrices; rows = columns of the paper's A):
// row src*R + q is the lattice sum of source src (src < n_lat) or the window of reference
// row q of the source's defect: entry i is G[q * ldg + i + win_offs[src - n_lat]].
__global__ void __launch_bounds__(256) k_gather_columns(int R, int n_lat,
                                                        const double* const* __restrict__ lat_U,
                                                        int ldu, const int32_t* __restrict__ win_offs,
                                                        const double* __restrict__ G, int ldg,
                                                        int N_axis,
                                                        double* __restrict__ cols, int ldc) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int row = blockIdx.y;
    if (i >= ldc) return;
    const int src = row / R, q = row % R;
    double v = 0.0;
    if (i < N_axis) {
        if (src < n_lat) {
            v = lat_U[src][(size_t)q * ldu + i];
        } else {
            v = G[(size_t)q * ldg + (i + win_offs[src - n_lat])];
        }
    }
    cols[(size_t)row * ldc + i] = v;
}

// Euclidean norm of each row, one workgroup per row, fixed reduction order.
__global__ void __launch_bounds__(256) k_row_norms(int n, const double* __restrict__ X, int ldx,
                                                   double* __restrict__ nrm) {
    __shared__ double red[256];
    const double* x = X + (size_t)blockIdx.x * ldx;
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += x[i] * x[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) nrm[blockIdx.x] = sqrt(red[0]);
}

__global__ void __launch_bounds__(256) k_scale_rows(int n, const double* __restrict__ X, int ldx,
                                                    const double* __restrict__ scale,
                                                    double* __restrict__ Y, int ldy) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int row = blockIdx.y;
    if (i >= n) return;
    Y[(size_t)row * ldy + i] = X[(size_t)row * ldx + i] * scale[row];
}

__global__ void __launch_bounds__(256) k_gather_scale_rows(int n, const double* __restrict__ X,
                                                           int ldx, const int32_t* __restrict__ order,
                                                           const double* __restrict__ inv_sigma,
                                                           double* __restrict__ Z, int ldz) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int a = blockIdx.y;
    if (i >= ldz) return;
    Z[(size_t)a * ldz + i] = i < n ? X[(size_t)order[a] * ldx + i] * inv_sigma[a] : 0.0;
}

__global__ void __launch_bounds__(256) k_f64_to_f32(long n, const double* __restrict__ x,
                                                    float* __restrict__ y) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] = (float)x[i];
}

__global__ void __launch_bounds__(256) k_f32_to_f64(long n, const float* __restrict__ x,
                                                    double* __restrict__ y) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] = (double)x[i];
}

template <typename T>
__global__ void __launch_bounds__(256) k_select_cols(int nsel, const T* __restrict__ Z, long ldz,
                                                     const int32_t* __restrict__ idx,
                                                     T* __restrict__ out) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    const int a = blockIdx.y;
    if (p >= nsel) return;
    out[(size_t)a * nsel + p] = Z[(size_t)a * ldz + idx[p]];
}

__global__ void __launch_bounds__(256) k_snap_points(int n, const double* __restrict__ xyz, int N0,
                                                     int N1, int N2, double h,
                                                     int32_t* __restrict__ idx) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    idx[p] = snap_dev(xyz[3 * (size_t)p + 0], h, N0);
    idx[n + p] = snap_dev(xyz[3 * (size_t)p + 1], h, N1);
    idx[2 * (size_t)n + p] = snap_dev(xyz[3 * (size_t)p + 2], h, N2);
}

// Tucker value at points after the mode-3 contraction: row w(t) of W (layout [row][a*r2+b]) holds
// sum_c mu[a,b,c] Z3[c, i3] for point t's mode-3 cell, and out[o(t)] = sum_a Z1[a, i1(t)] sum_b
// W[w(t)][a*r2+b] Z2[b, i2(t)] (w, o: identity when null).  One workgroup per point: the point's
// Z2 column is staged in LDS, each wave takes a subset of the a rows and reads them contiguously
// (lanes over b), and the waves' totals are summed in a fixed order.  (Without LDS staging, for
// r2 beyond the dynamic LDS limit, Z2 is read directly.)
template <bool STAGE, typename TW>
__global__ void __launch_bounds__(256) k_tucker_finish(int r1, int r2, int P,
                                                       const TW* __restrict__ W,
                                                       const double* __restrict__ Z1, int ld1,
                                                       const double* __restrict__ Z2, int ld2,
                                                       const int32_t* __restrict__ i1,
                                                       const int32_t* __restrict__ i2,
                                                       const int32_t* __restrict__ wrow,
                                                       const int32_t* __restrict__ oidx,
                                                       double* __restrict__ out) {
    extern __shared__ double z2s[];           // r2 values
    __shared__ double part[4];
    const int t = blockIdx.x;
    const int c1 = i1[t], c2 = i2[t];
    const int p = oidx ? oidx[t] : t;
    if (c1 < 0 || c2 < 0) {                   // uniform per workgroup
        if (threadIdx.x == 0) out[p] = __builtin_nan("");
        return;
    }
    if (STAGE) {
        for (int b = threadIdx.x; b < r2; b += 256) z2s[b] = Z2[(size_t)b * ld2 + c2];
        __syncthreads();
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const TW* w = W + (size_t)(wrow ? wrow[t] : t) * r1 * r2;
    double total = 0.0;
    for (int a = wave; a < r1; a += 4) {
        double acc = 0.0;
        for (int b = lane; b < r2; b += 64)
            acc += (double)w[(size_t)a * r2 + b] * (STAGE ? z2s[b] : Z2[(size_t)b * ld2 + c2]);
        for (int m = 32; m > 0; m >>= 1) acc += __shfl_xor(acc, m, 64);
        total += acc * Z1[(size_t)a * ld1 + c1];
    }
    if (lane == 0) part[wave] = total;
    __syncthreads();
    if (threadIdx.x == 0) out[p] = (part[0] + part[1]) + (part[2] + part[3]);
}

inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

void launch_collocate(hipStream_t st, int R, const double* t_dev, const double* w13_dev, int N_ref,
                      double h, double* G, int ldg, double shift) {
    dim3 grid(cdiv(ldg, 256), R);
    hipLaunchKernelGGL(k_collocate, grid, dim3(256), 0, st, R, t_dev, w13_dev, N_ref, h, shift, G, ldg);
}

// Workgroup tile of the shift-sum: 64 cells x 16 nodes (the nodes split over the grid's z
// dimension, NU = 2) or 64 cells x 48 nodes (NU = 6).  Both add the same terms in the same order.
static void launch_shift_variant(hipStream_t st, int variant, const ShiftJob* jobs_dev, int n_jobs, int max_N,
                                 int max_R, hipEvent_t a, hipEvent_t b) {
    const int tx = cdiv(max_N, 64);
    const int nz = variant == 0 ? cdiv(max_R, 16) : 1;
    const long total = (long)tx * n_jobs * nz;
    const dim3 grid((unsigned)((total + 7) / 8 * 8));   // a multiple of the 8 XCDs
    if (variant == 0) {
        hipExtLaunchKernelGGL(k_shift_sum<2>, grid, dim3(256), 0, st, a, b, 0, jobs_dev, tx, n_jobs, nz);
    } else {
        hipExtLaunchKernelGGL(k_shift_sum<6>, grid, dim3(256), 0, st, a, b, 0, jobs_dev, tx, n_jobs, nz);
    }
}

void launch_shift_sum(hipStream_t st, const ShiftJob* jobs_dev, int n_jobs, int max_N, int max_R,
                      const KTime* kt, Tuner* tuner) {
    if (n_jobs <= 0 || max_N <= 0) return;
    const int tiles = cdiv(max_N, 64) * n_jobs;
    hipEvent_t a = kt ? kt->start : nullptr, b = kt ? kt->stop : nullptr;
    // without a decision: a small batch splits the nodes over the grid's z dimension so that the
    // chip has enough workgroups to cover the L2 latency; a large one takes 48 nodes per group
    int variant = (tiles < 1024 && max_R > 16) ? 0 : 1;
    if (tuner && max_R > 16) {
        int b2 = 1;
        while (b2 < tiles) b2 <<= 1;
        const std::string key = "shift_sum/tiles" + std::to_string(b2) + "/R" + std::to_string(max_R <= 32 ? 32 : 64);
        const int ch = tuner->get(key);
        if (ch >= 0) {
            variant = ch;
        } else if (ch == -1) {
            // time both tiles (each writes the same values) and keep the faster
            std::vector<double> ms(2, -1.0);
            hipEvent_t e[4] = {};
            bool ok = true;
            for (auto& ev : e) ok = ok && hipEventCreate(&ev) == hipSuccess;
            if (ok) {
                launch_shift_variant(st, 0, jobs_dev, n_jobs, max_N, max_R, e[0], e[1]);
                launch_shift_variant(st, 1, jobs_dev, n_jobs, max_N, max_R, e[2], e[3]);
                float t0 = 0.f, t1 = 0.f;
                if (hipEventSynchronize(e[3]) == hipSuccess && hipEventElapsedTime(&t0, e[0], e[1]) == hipSuccess &&
                    hipEventElapsedTime(&t1, e[2], e[3]) == hipSuccess) {
                    ms[0] = t0;
                    ms[1] = t1;
                }
            }
            (void)hipGetLastError();
            for (auto& ev : e)
                if (ev) (void)hipEventDestroy(ev);
            const int best = tuner->put(key, ms);
            if (best >= 0) variant = best;
        }
    }
    launch_shift_variant(st, variant, jobs_dev, n_jobs, max_N, max_R, a, b);
}

void launch_window_sums(hipStream_t st, int R, const double* G, int ldg, int stride, int n, double* Q) {
    if (R <= 0 || ldg <= 0) return;
    hipLaunchKernelGGL(k_window_sums, dim3(cdiv(ldg, 256), R), dim3(256), 0, st, ldg, G, stride, n, Q);
}

void launch_sample_cp(hipStream_t st, int n_fac, int R, const double* U, int ldu,
                      const double* lam_dev, int N0, int N1, int N2, double h, int n_pts,
                      const double* xyz, double* out) {
    if (n_pts <= 0) return;
    hipLaunchKernelGGL(k_sample_cp, dim3(cdiv(n_pts, 256)), dim3(256), 0, st, n_fac, R, U, ldu,
                       lam_dev, N0, N1, N2, h, n_pts, xyz, out);
}

void launch_transpose(hipStream_t st, int R, int N, const double* U, int ldu, double* UT) {
    if (R <= 0 || N <= 0) return;
    hipLaunchKernelGGL(k_transpose<double>, dim3(cdiv(N, 32), cdiv(R, 32)), dim3(256), 0, st, R, N, U, ldu, UT);
}

void launch_transpose(hipStream_t st, int R, int N, const float* U, int ldu, double* UT) {
    if (R <= 0 || N <= 0) return;
    hipLaunchKernelGGL(k_transpose<float>, dim3(cdiv(N, 32), cdiv(R, 32)), dim3(256), 0, st, R, N, U, ldu, UT);
}

int sample_points_per_wg(bool f32) { return f32 ? 64 : 32; }

void launch_sample_batch(hipStream_t st, int ldt, bool f32, const SampleJob* jobs, int n_jobs, int n_wg,
                         const KTime* kt) {
    if (n_jobs <= 0 || n_wg <= 0) return;
    const dim3 grid(cdiv(n_wg, 8) * 8), blk(256);
    hipEvent_t a = kt ? kt->start : nullptr, b = kt ? kt->stop : nullptr;
#define LSUM_SAMPLE_BATCH(NQ, T) \
    hipExtLaunchKernelGGL((k_sample_batch<NQ, T>), grid, blk, 0, st, a, b, 0, ldt, jobs, n_jobs, n_wg)
#define LSUM_SAMPLE_BATCH_LDT(T)              \
    switch (ldt) {                            \
        case 16: LSUM_SAMPLE_BATCH(1, T); break; \
        case 32: LSUM_SAMPLE_BATCH(2, T); break; \
        case 48: LSUM_SAMPLE_BATCH(3, T); break; \
        case 64: LSUM_SAMPLE_BATCH(4, T); break; \
        default: LSUM_SAMPLE_BATCH(0, T);     \
    }
    if (f32) {
        LSUM_SAMPLE_BATCH_LDT(float)
    } else {
        LSUM_SAMPLE_BATCH_LDT(double)
    }
#undef LSUM_SAMPLE_BATCH_LDT
#undef LSUM_SAMPLE_BATCH
}

void launch_sample_windows(hipStream_t st, int R, const double* G, int ldg, int n_def,
                           const int32_t* def_offs, const double* def_scale, int N0, int N1,
                           int N2, double h, int n_pts, const double* xyz, double* out, const KTime* kt) {
    if (n_pts <= 0 || n_def <= 0) return;
    hipExtLaunchKernelGGL(k_sample_windows, dim3(cdiv(n_pts, 256)), dim3(256), 0, st, kt ? kt->start : nullptr,
                          kt ? kt->stop : nullptr, 0, R, G, ldg, n_def, def_offs, def_scale, N0, N1,
                          N2, h, n_pts, xyz, out);
}

void launch_gather_columns(hipStream_t st, int R, int n_lat, const double* const* lat_U_dev, int ldu,
                           int n_win, const int32_t* win_offs_dev, const double* G, int ldg,
                           int N_axis, double* cols, int ldc) {
    const int rows = R * (n_lat + n_win);
    if (rows <= 0) return;
    dim3 grid(cdiv(ldc, 256), rows);
    hipLaunchKernelGGL(k_gather_columns, grid, dim3(256), 0, st, R, n_lat, lat_U_dev, ldu,
                       win_offs_dev, G, ldg, N_axis, cols, ldc);
}

void launch_row_norms(hipStream_t st, int rows, int n, const double* X, int ldx, double* nrm) {
    if (rows <= 0) return;
    hipLaunchKernelGGL(k_row_norms, dim3(rows), dim3(256), 0, st, n, X, ldx, nrm);
}

void launch_scale_rows(hipStream_t st, int rows, int n, const double* X, int ldx, const double* scale,
                       double* Y, int ldy) {
    if (rows <= 0) return;
    hipLaunchKernelGGL(k_scale_rows, dim3(cdiv(n, 256), rows), dim3(256), 0, st, n, X, ldx, scale, Y,
                       ldy);
}

void launch_gather_scale_rows(hipStream_t st, int r, int n, const double* X, int ldx,
                              const int32_t* order_dev, const double* inv_sigma_dev, double* Z,
                              int ldz) {
    if (r <= 0) return;
    hipLaunchKernelGGL(k_gather_scale_rows, dim3(cdiv(ldz, 256), r), dim3(256), 0, st, n, X, ldx,
                       order_dev, inv_sigma_dev, Z, ldz);
}

void launch_f64_to_f32(hipStream_t st, long n, const double* x, float* y) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_f64_to_f32, dim3(cdiv(n, 256)), dim3(256), 0, st, n, x, y);
}

void launch_f32_to_f64(hipStream_t st, long n, const float* x, double* y) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_f32_to_f64, dim3(cdiv(n, 256)), dim3(256), 0, st, n, x, y);
}

void launch_select_cols(hipStream_t st, int rows, int nsel, const void* Z, long ldz,
                        const int32_t* idx, void* out, int elem_size) {
    if (rows <= 0 || nsel <= 0) return;
    dim3 grid(cdiv(nsel, 256), rows);
    if (elem_size == 8)
        hipLaunchKernelGGL(k_select_cols<double>, grid, dim3(256), 0, st, nsel,
                           (const double*)Z, ldz, idx, (double*)out);
    else
        hipLaunchKernelGGL(k_select_cols<float>, grid, dim3(256), 0, st, nsel, (const float*)Z,
                           ldz, idx, (float*)out);
}

void launch_tucker_finish(hipStream_t st, int r1, int r2, int P, const void* W, int w_elem, const double* Z1,
                          int ld1, const double* Z2, int ld2, const int32_t* i1, const int32_t* i2,
                          const int32_t* wrow, const int32_t* oidx, double* out) {
    if (P <= 0) return;
    const size_t lds = r2 <= 8192 ? (size_t)r2 * sizeof(double) : 0;
    if (w_elem == 8) {
        if (lds)
            hipLaunchKernelGGL((k_tucker_finish<true, double>), dim3(P), dim3(256), lds, st, r1, r2, P,
                               (const double*)W, Z1, ld1, Z2, ld2, i1, i2, wrow, oidx, out);
        else
            hipLaunchKernelGGL((k_tucker_finish<false, double>), dim3(P), dim3(256), 0, st, r1, r2, P,
                               (const double*)W, Z1, ld1, Z2, ld2, i1, i2, wrow, oidx, out);
    } else {
        if (lds)
            hipLaunchKernelGGL((k_tucker_finish<true, float>), dim3(P), dim3(256), lds, st, r1, r2, P,
                               (const float*)W, Z1, ld1, Z2, ld2, i1, i2, wrow, oidx, out);
        else
            hipLaunchKernelGGL((k_tucker_finish<false, float>), dim3(P), dim3(256), 0, st, r1, r2, P,
                               (const float*)W, Z1, ld1, Z2, ld2, i1, i2, wrow, oidx, out);
    }
}

void launch_snap_points(hipStream_t st, int n, const double* xyz, int N0, int N1, int N2, double h,
                        int32_t* idx) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_snap_points, dim3(cdiv(n, 256)), dim3(256), 0, st, n, xyz, N0, N1, N2, h,
                       idx);
}

}  // namespace lsum

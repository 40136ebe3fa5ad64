// Plain FP64 GEMMs through rocBLAS.  The range basis (sketches, re-orthogonalisation, B = Q W^T,
// the residual), the vectors V Q, the FP64 projections and the grouped core's second step are
// plain dense products with unit-stride operands; on MI355X the library's DGEMM runs them at
// 69-76 TFLOP/s where the library's own 128 x 64 tile (k_gemm<F64>) reaches 45-47 (large shapes)
// and 4-23 (the range basis's skinny ones).  FP32 products stay on k_gemm<F32>: the library's
// SGEMM is faster (122-129 TFLOP/s against 72 on the core's shapes) but adds in FP32 throughout,
// and on the defected 48^3 lattice at eps 1e-6 its core left values 1.7e-6 off the direct sum
// where k_gemm<F32> (FP32 partial sums of 32 terms added in FP64) stays within 1e-6.  Fused and
// mixed-precision contractions stay on the hand-written kernels.  Handles are pooled per device and bound to the caller's stream per
// call; atomics are disabled on every handle, so a product never depends on what else runs.
#include <rocblas/rocblas.h>

#include <atomic>
#include <mutex>
#include <vector>

#include "lsum_internal.h"

namespace lsum {

namespace {

std::atomic<int> g_enabled{1};
std::mutex g_mu;
std::vector<std::pair<int, rocblas_handle>> g_free;   // (device, handle) ready for use

rocblas_handle acquire(int dev) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (size_t i = 0; i < g_free.size(); ++i)
            if (g_free[i].first == dev) {
                rocblas_handle h = g_free[i].second;
                g_free.erase(g_free.begin() + (long)i);
                return h;
            }
    }
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) return nullptr;
    if (rocblas_set_atomics_mode(h, rocblas_atomics_not_allowed) != rocblas_status_success ||
        rocblas_set_pointer_mode(h, rocblas_pointer_mode_host) != rocblas_status_success) {
        rocblas_destroy_handle(h);
        return nullptr;
    }
    return h;
}

void release(int dev, rocblas_handle h) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_free.push_back({dev, h});
}

}  // namespace

void set_gemm_library(bool on) { g_enabled.store(on ? 1 : 0); }
bool gemm_library() { return g_enabled.load() != 0; }

// C (m x n, row stride scm, unit column stride) = alpha A B + beta C (per batch entry, at the
// element strides bA, bB, bC).  In column-major terms
// that is C^T = B^T A^T: a row-major operand is its transpose stored column-major, a
// column-major one is used transposed.  Returns false (nothing launched) when the layout or
// size is not one this path takes, so the caller's kernel runs instead.
bool blas_gemm(hipStream_t st, GemmPrec prec, const GemmArgs& a) {
    if (prec != GEMM_F64) return false;
    if (!gemm_library() || a.batch < 1 || a.scn != 1) return false;
    if ((double)a.m * a.n * std::max(a.k, 1) * a.batch < (double)(1 << 24)) return false;
    rocblas_operation opA, opB;
    long lda, ldb;
    if (a.sak == 1 && a.sam >= a.k && a.sam > 0) {
        opA = rocblas_operation_none;   // A^T column-major (k x m)
        lda = a.sam;
    } else if (a.sam == 1 && a.sak >= a.m) {
        opA = rocblas_operation_transpose;   // A column-major (m x k)
        lda = a.sak;
    } else {
        return false;
    }
    if (a.sbn == 1 && a.sbk >= a.n && a.sbk > 0) {
        opB = rocblas_operation_none;   // B^T column-major (n x k)
        ldb = a.sbk;
    } else if (a.sbk == 1 && a.sbn >= a.k) {
        opB = rocblas_operation_transpose;   // B column-major (k x n)
        ldb = a.sbn;
    } else {
        return false;
    }
    if (a.scm < a.n || lda > 0x7fffffff || ldb > 0x7fffffff || a.scm > 0x7fffffff) return false;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    rocblas_handle h = acquire(dev);
    if (!h) return false;
    bool ok = rocblas_set_stream(h, st) == rocblas_status_success;
    const double alpha = a.alpha, beta = a.beta;
    if (ok && a.batch > 1) {
        // a batch of products at fixed element strides (a stride may be 0: a shared operand)
        ok = rocblas_dgemm_strided_batched(h, opB, opA, a.n, a.m, a.k, &alpha, (const double*)a.B, (rocblas_int)ldb,
                                           a.bB, (const double*)a.A, (rocblas_int)lda, a.bA, &beta, (double*)a.C,
                                           (rocblas_int)a.scm, a.bC, a.batch) == rocblas_status_success;
    } else if (ok) {
        ok = rocblas_dgemm(h, opB, opA, a.n, a.m, a.k, &alpha, (const double*)a.B, (rocblas_int)ldb,
                           (const double*)a.A, (rocblas_int)lda, &beta, (double*)a.C, (rocblas_int)a.scm) ==
             rocblas_status_success;
    }
    release(dev, h);
    return ok;
}

}  // namespace lsum

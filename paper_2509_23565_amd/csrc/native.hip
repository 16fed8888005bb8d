// Native FP64 trailing updates for the comparison runs: the same blocked
// factorizations (panel, interchanges, triangular solve) with the Schur
// update C <- C - A B done by rocBLAS dgemm (LU) or the lower-triangle
// C <- C - A A^T by rocBLAS dsyrk (Cholesky) instead of the emulated GEMM
// (the performance section compares the LU with FP64 updates against the
// LU with emulated ones, over the blocking factor).
#include "common.h"

#include <rocblas/rocblas.h>


namespace emu {

// The calling thread's rocBLAS handle on the current device (kept in its
// thread context, created on first use, destroyed by emu_finalize).
static int handle(hipStream_t stream, rocblas_handle *out) {
    Device *dev;
    hipStream_t st;
    EMU_TRY(current(&dev, &st));
    ThreadCtx *c = thread_ctx(dev);
    rocblas_handle h = static_cast<rocblas_handle>(c->blas);
    if (!h) {
        if (rocblas_create_handle(&h) != rocblas_status_success) {
            set_error("rocblas_create_handle failed");
            return EMU_ERR_HIP;
        }
        c->blas = h;
    }
    if (rocblas_set_stream(h, stream) != rocblas_status_success) {
        set_error("rocblas_set_stream failed");
        return EMU_ERR_HIP;
    }
    *out = h;
    return 0;
}

int native_syrk_update(int m, int k, const double *A, long long lda, double *C, long long ldc,
                       hipStream_t stream) {
    if (m <= 0 || k <= 0) return 0;
    rocblas_handle h;
    EMU_TRY(handle(stream, &h));
    const double alpha = -1.0, beta = 1.0;
    const rocblas_status st = rocblas_dsyrk(h, rocblas_fill_lower, rocblas_operation_none, m, k,
                                            &alpha, A, (rocblas_int)lda, &beta, C,
                                            (rocblas_int)ldc);
    if (st != rocblas_status_success) {
        set_error("rocblas_dsyrk failed (status %d)", (int)st);
        return EMU_ERR_HIP;
    }
    return 0;
}

int native_update(int m, int n, int k, const double *A, long long lda, const double *B,
                  long long ldb, double *C, long long ldc, hipStream_t stream) {
    if (m <= 0 || n <= 0 || k <= 0) return 0;
    rocblas_handle h;
    EMU_TRY(handle(stream, &h));
    const double alpha = -1.0, beta = 1.0;
    const rocblas_status st =
        rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, m, n, k, &alpha, A,
                      (rocblas_int)lda, B, (rocblas_int)ldb, &beta, C, (rocblas_int)ldc);
    if (st != rocblas_status_success) {
        set_error("rocblas_dgemm failed (status %d)", (int)st);
        return EMU_ERR_HIP;
    }
    return 0;
}

void native_release(ThreadCtx *c) {
    if (c->blas) (void)rocblas_destroy_handle(static_cast<rocblas_handle>(c->blas));
    c->blas = nullptr;
}

}  // namespace emu

// Inverse of the dense SPD coarse matrix A_0 (Section 3.2: exact coarse
// solve, here by a precomputed inverse applied as a GEMV) by blocked
// Gauss-Jordan elimination without pivoting.  With K the current block of
// b pivots, D = A[K,K], P = A[:,K], R = A[K,:]:
//   A <- A - (P D^-1) R,  A[K,:] <- D^-1 R,  A[:,K] <- -P D^-1,  A[K,K] <- D^-1,
// which is the in-place Gauss-Jordan step for a block of pivots.  D^-1 comes
// from the scalar Gauss-Jordan of one workgroup; the three products are
// float64 GEMMs (rocBLAS).  2 n^3 flops in rank-b updates instead of n
// passes of rank-1 updates over the whole matrix.
#include <rocblas/rocblas.h>

#include <algorithm>

#include "lor_internal.h"

namespace lor {

namespace {

// row-major C (m x n) = alpha op(A) op(B) + beta C through the column-major
// library call on the transposed problem.
rocblas_status gemm_rm(rocblas_handle h, int m, int n, int k, double alpha, const double *A,
                       int lda, const double *B, int ldb, double beta, double *C, int ldc) {
  return rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, n, m, k, &alpha, B, ldb,
                       A, lda, &beta, C, ldc);
}

}  // namespace

int coarse_inverse(int n, double *A, hipStream_t st) {
  if (n <= 0) return LOR_OK;
  constexpr int kB = 128;
  double *P = nullptr, *R = nullptr, *PD = nullptr, *Dinv = nullptr;
  int *bad = nullptr;
  rocblas_handle rb = nullptr;
  int rc = LOR_OK;
  const int b0 = std::min(kB, n);
  auto done = [&](int code) {
    if (rb) (void)rocblas_destroy_handle(rb);
    (void)hipFree(P);
    (void)hipFree(R);
    (void)hipFree(PD);
    (void)hipFree(Dinv);
    (void)hipFree(bad);
    return code;
  };
  if (hipMalloc(&P, size_t(n) * b0 * 8) != hipSuccess || hipMalloc(&R, size_t(n) * b0 * 8) != hipSuccess ||
      hipMalloc(&PD, size_t(n) * b0 * 8) != hipSuccess ||
      hipMalloc(&Dinv, size_t(b0) * b0 * 8) != hipSuccess || hipMalloc(&bad, sizeof(int)) != hipSuccess)
    return done(LOR_EHIP);
  if (hipMemsetAsync(bad, 0, sizeof(int), st) != hipSuccess) return done(LOR_EHIP);
  if (rocblas_create_handle(&rb) != rocblas_status_success ||
      rocblas_set_stream(rb, st) != rocblas_status_success)
    return done(LOR_EHIP);
  for (int kb = 0; kb < n; kb += kB) {
    const int bk = std::min(kB, n - kb);
    // P = A[:, K] (n x bk), R = A[K, :] (bk x n), D^-1 from A[K, K]
    if (launch_copy_block(A + kb, n, P, bk, n, bk, 1.0, st) != hipSuccess ||
        launch_copy_block(A + size_t(kb) * n, n, R, n, bk, n, 1.0, st) != hipSuccess ||
        launch_small_inverse(A + size_t(kb) * n + kb, n, Dinv, bk, bad, st) != hipSuccess)
      return done(LOR_EHIP);
    if (gemm_rm(rb, n, bk, bk, 1.0, P, bk, Dinv, bk, 0.0, PD, bk) != rocblas_status_success ||
        gemm_rm(rb, n, n, bk, -1.0, PD, bk, R, n, 1.0, A, n) != rocblas_status_success ||
        gemm_rm(rb, bk, n, bk, 1.0, Dinv, bk, R, n, 0.0, A + size_t(kb) * n, n) !=
            rocblas_status_success)
      return done(LOR_EHIP);
    if (launch_copy_block(PD, bk, A + kb, n, n, bk, -1.0, st) != hipSuccess ||
        launch_copy_block(Dinv, bk, A + size_t(kb) * n + kb, n, bk, bk, 1.0, st) != hipSuccess)
      return done(LOR_EHIP);
  }
  int hb = 0;
  if (hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return done(LOR_EHIP);
  rc = hb ? LOR_EPIVOT : LOR_OK;
  return done(rc);
}

}  // namespace lor

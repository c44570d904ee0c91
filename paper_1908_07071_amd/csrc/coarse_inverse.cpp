// Inverse of the dense SPD coarse matrix A_0 (Section 3.2: exact coarse
// solve, here by a precomputed inverse applied as a GEMV) by blocked
// Gauss-Jordan elimination without pivoting.  With K the current block of
// b pivots, D = A[K,K], P = A[:,K], R = A[K,:]:
//   A <- A - (P D^-1) R,  A[K,:] <- D^-1 R,  A[:,K] <- -P D^-1,  A[K,K] <- D^-1,
// which is the in-place Gauss-Jordan step for a block of pivots.  D^-1 comes
// from the scalar Gauss-Jordan of one workgroup; the three products run on
// the float64 matrix cores (k_dgemm.hip).  2 n^3 flops in rank-b updates
// instead of n passes of rank-1 updates over the whole matrix.
#include <algorithm>

#include "lor.h"
#include "lor_internal.h"

namespace lor {

int coarse_inverse(int n, double *A, hipStream_t st) {
  if (n <= 0) return LOR_OK;
  constexpr int kB = 128;
  double *P = nullptr, *R = nullptr, *PD = nullptr, *Dinv = nullptr;
  int *bad = nullptr;
  int rc = LOR_OK;
  const int b0 = std::min(kB, n);
  auto done = [&](int code) {
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
  for (int kb = 0; kb < n; kb += kB) {
    const int bk = std::min(kB, n - kb);
    // P = A[:, K] (n x bk), R = A[K, :] (bk x n), D^-1 from A[K, K]
    if (launch_copy_block(A + kb, n, P, bk, n, bk, 1.0, st) != hipSuccess ||
        launch_copy_block(A + size_t(kb) * n, n, R, n, bk, n, 1.0, st) != hipSuccess ||
        launch_small_inverse(A + size_t(kb) * n + kb, n, Dinv, bk, bad, st) != hipSuccess)
      return done(LOR_EHIP);
    if (launch_dgemm(n, bk, bk, 1.0, P, bk, Dinv, bk, 0.0, PD, bk, st) != hipSuccess ||
        launch_dgemm(n, n, bk, -1.0, PD, bk, R, n, 1.0, A, n, st) != hipSuccess ||
        launch_dgemm(bk, n, bk, 1.0, Dinv, bk, R, n, 0.0, A + size_t(kb) * n, n, st) != hipSuccess)
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

extern "C" int lor_f64_gemm(int m, int n, int k, double alpha, const double *A, int64_t lda,
                            const double *B, int64_t ldb, double beta, double *C, int64_t ldc,
                            void *stream) {
  if (m < 0 || n < 0 || k < 0 || lda < k || ldb < n || ldc < n) return LOR_EINVAL;
  if (m > 0 && n > 0 && (!C || (k > 0 && (!A || !B)))) return LOR_EINVAL;
  if (lor::launch_dgemm(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                        static_cast<hipStream_t>(stream)) != hipSuccess)
    return LOR_EHIP;
  return LOR_OK;
}

// Float64 matrix product on the matrix cores, for the blocked Gauss-Jordan
// inverse of the coarse matrix (Section 3.2: exact coarse solve): the rank-b
// updates of its steps are dense contractions.
//
// C = alpha A B + beta C, row major: A(i,k) = A[i lda + k], B(k,j) = B[k ldb + j],
// C(i,j) = C[i ldc + j]; any m, n, k.  A workgroup of four wavefronts owns a
// 64 x 64 tile of C, each wavefront a 32 x 32 quarter as 2 x 2 blocks of
// v_mfma_f64_16x16x4f64.  K advances in chunks of 16 staged in LDS (rows
// padded against bank conflicts); tiles past the edges are zero filled, and
// with beta == 0 C is written without being read.
#include <hip/hip_runtime.h>

#include "lor_internal.h"

namespace lor {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 64;   // C tile per workgroup (m and n)
constexpr int kKc = 16;     // K chunk staged in LDS
constexpr int kApad = kKc + 1;
constexpr int kBpad = kTile + 1;

__global__ __launch_bounds__(256) void k_dgemm(int m, int n, int k, double alpha,
                                               const double *__restrict__ A, int64_t lda,
                                               const double *__restrict__ B, int64_t ldb, double beta,
                                               double *__restrict__ C, int64_t ldc) {
  __shared__ double As[kTile][kApad];
  __shared__ double Bs[kKc][kBpad];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i0 = blockIdx.y * kTile, j0 = blockIdx.x * kTile;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  // v_mfma_f64_16x16x4f64: lane l supplies A(l % 16, l / 16) and B(l / 16,
  // l % 16) of the 16 x 4 and 4 x 16 operands and holds D(l / 16 + 4 t,
  // l % 16), t = 0..3, of the 16 x 16 result (measured on gfx950)
  const int r16 = lane & 15, q4 = lane >> 4;
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < k; k0 += kKc) {
    // stage A(i0.., k0..) 64 x 16 and B(k0.., j0..) 16 x 64: four values per thread
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = tid + 256 * t;
      const int ar = e / kKc, ac = e % kKc;
      const int gi = i0 + ar, gk = k0 + ac;
      As[ar][ac] = (gi < m && gk < k) ? A[int64_t(gi) * lda + gk] : 0.0;
      const int br = e / kTile, bc = e % kTile;
      const int gk2 = k0 + br, gj = j0 + bc;
      Bs[br][bc] = (gk2 < k && gj < n) ? B[int64_t(gk2) * ldb + gj] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kKc; kk += 4) {
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[wi + 16 * a + r16][kk + q4];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Bs[kk + q4][wj + 16 * b + r16];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int gi = i0 + wi + 16 * a + q4 + 4 * t, gj = j0 + wj + 16 * b + r16;
        if (gi < m && gj < n) {
          double *c = C + int64_t(gi) * ldc + gj;
          const double v = alpha * acc[a][b][t];
          *c = beta == 0.0 ? v : v + beta * *c;
        }
      }
}

}  // namespace

hipError_t launch_dgemm(int m, int n, int k, double alpha, const double *A, int64_t lda,
                        const double *B, int64_t ldb, double beta, double *C, int64_t ldc,
                        hipStream_t st) {
  if (m < 0 || n < 0 || k < 0 || lda < k || ldb < n || ldc < n) return hipErrorInvalidValue;
  if (m == 0 || n == 0) return hipSuccess;
  const int64_t gy = (int64_t(m) + kTile - 1) / kTile;
  if (gy > 65535) return hipErrorInvalidValue;  // grid y limit
  const dim3 grid((n + kTile - 1) / kTile, unsigned(gy));
  k_dgemm<<<grid, 256, 0, st>>>(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
  return hipGetLastError();
}

}  // namespace lor

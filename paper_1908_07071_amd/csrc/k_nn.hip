// Kernels of the learned patch correction: gather of the normalised patch
// residuals into the (2p-1)^3 patch grid, im2col / col2im of 3x3x3
// convolutions on that grid, a BF16 MFMA GEMM with float accumulation, the
// bias / ReLU epilogue, the masked squared-error loss, Adam on float32 master
// weights, and the scatter of the network's patch corrections.
//
// Layouts: activations [rows][channels] with row = n G^3 + q (q = gx + G (gy +
// G gz)); im2col matrices [rows][Kp] with column k Cin + c (k = (dx+1) +
// 3 (dy+1) + 9 (dz+1)); weights [Kp][Np] (zero padded to multiples of 16).
#include <hip/hip_runtime.h>

#include "lor_internal.h"

namespace lor {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 rounded to nearest, ties to even (NaN stays NaN)
__device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return uint16_t((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

inline int grid_for(int64_t n, int bs) {
  int64_t g = (n + bs - 1) / bs;
  return int(g > 65536 ? 65536 : (g < 1 ? 1 : g));
}

// C (+)= A B with A(i,k) = A[i ai + k ak], B(k,j) = B[k bk + j bj] (bf16) and
// C float32 [M][ldc]; M, N, K multiples of 16.  One wavefront per 16 x 16
// tile of C.  v_mfma_f32_16x16x16bf16: lane l supplies A[l%16][4(l/16)+t] and
// B[4(l/16)+t][l%16] (t = 0..3) and receives C[4(l/16)+t][l%16].
// AK1: ak == 1 and ai a multiple of 4 (one 8-byte load per lane and step).
template <bool AK1, bool ACC>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const uint16_t *__restrict__ A,
                                              int64_t ai, int64_t ak,
                                              const uint16_t *__restrict__ B, int64_t bk,
                                              int64_t bj, float *__restrict__ C, int64_t ldc) {
  const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  const int tn = N >> 4;
  const int64_t tiles = int64_t(M >> 4) * tn;
  if (wave >= tiles) return;
  const int64_t ti = wave / tn;
  const int tj = int(wave % tn);
  const int r = lane & 15, kq = (lane >> 4) << 2;
  const uint16_t *Ap = A + (ti * 16 + r) * ai + int64_t(kq) * ak;
  const uint16_t *Bp = B + int64_t(kq) * bk + int64_t(tj * 16 + r) * bj;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 16) {
    bf16x4 a, b;
    if (AK1) {
      a = *reinterpret_cast<const bf16x4 *>(Ap + k0);
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t) a[t] = short(Ap[int64_t(k0 + t) * ak]);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) b[t] = short(Bp[int64_t(k0 + t) * bk]);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    float *c = C + (ti * 16 + kq + t) * ldc + tj * 16 + r;
    *c = ACC ? *c + acc[t] : acc[t];
  }
}

// cols[row][k Cin + c] = act[row + off(k)][c] (zero outside the grid, in
// padding rows and in padding columns).
__global__ void k_im2col(const uint16_t *__restrict__ act, int64_t rows, int G, int cin, int Kp,
                         int64_t npad, uint16_t *__restrict__ cols, const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;
  const int G3 = G * G * G;
  const int64_t tot = npad * Kp;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < tot;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t row = t / Kp;
    const int col = int(t % Kp);
    uint16_t v = 0;
    if (row < rows && col < 27 * cin) {
      const int q = int(row % G3);
      const int64_t base = row - q;
      const int k = col / cin, c = col % cin;
      const int gx = q % G + k % 3 - 1, gy = (q / G) % G + (k / 3) % 3 - 1, gz = q / (G * G) + k / 9 - 1;
      if (gx >= 0 && gx < G && gy >= 0 && gy < G && gz >= 0 && gz < G)
        v = act[(base + gx + G * (gy + G * gz)) * cin + c];
    }
    cols[t] = v;
  }
}

// dz[row][c] = (zprev[row][c] > 0) sum_k dcols[row - off(k)][k Cin + c]
// (rows outside the grid skipped): the input gradient of a convolution
// followed by the ReLU derivative of the previous layer.  Also the bf16 copy.
__global__ void k_col2im_relu(const float *__restrict__ dcols, int64_t rows, int64_t npad, int G,
                              int cin, int Kp, const float *__restrict__ zprev, int ldzp,
                              float *__restrict__ dz, uint16_t *__restrict__ dz16) {
  const int G3 = G * G * G;
  const int64_t tot = npad * cin;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < tot;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t row = t / cin;
    const int c = int(t % cin);
    if (row >= rows) {  // padding rows take part in the next GEMM's K sum
      dz[t] = 0.f;
      dz16[t] = 0;
      continue;
    }
    const int q = int(row % G3);
    const int64_t base = row - q;
    float acc = 0.f;
    for (int k = 0; k < 27; ++k) {
      const int gx = q % G - (k % 3 - 1), gy = (q / G) % G - ((k / 3) % 3 - 1),
                gz = q / (G * G) - (k / 9 - 1);
      if (gx >= 0 && gx < G && gy >= 0 && gy < G && gz >= 0 && gz < G)
        acc += dcols[(base + gx + G * (gy + G * gz)) * Kp + k * cin + c];
    }
    const float d = zprev[row * ldzp + c] > 0.f ? acc : 0.f;
    dz[row * cin + c] = d;
    dz16[row * cin + c] = f2bf(d);
  }
}

// z[row][o] += bias[o]; hidden layers: a[row][o] = bf16(max(z, 0)).
__global__ void k_bias_relu(float *__restrict__ z, int64_t rows, int cout, int Np,
                            const float *__restrict__ bias, uint16_t *__restrict__ a,
                            const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;
  const int64_t tot = rows * cout;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < tot;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t row = t / cout;
    const int o = int(t % cout);
    const float v = z[row * Np + o] + bias[o];
    z[row * Np + o] = v;
    if (a) a[row * cout + o] = f2bf(v > 0.f ? v : 0.f);
  }
}

// network input: a0[row] = bf16(X[row][0..1])
__global__ void k_input_bf16(const float *__restrict__ X, int64_t rows, int64_t npad,
                             uint16_t *__restrict__ a0, const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < npad * 2;
       t += int64_t(gridDim.x) * blockDim.x)
    a0[t] = t < rows * 2 ? f2bf(X[t]) : uint16_t(0);
}

// output: y[row] = (z[row][0]) mask[row] (the bias is already in z)
__global__ void k_output(const float *__restrict__ z, int Np, const float *__restrict__ X,
                         int64_t rows, float *__restrict__ y, const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < rows;
       t += int64_t(gridDim.x) * blockDim.x)
    y[t] = z[t * Np] * X[2 * t + 1];
}

// loss partials: sum of ((y - T) mask)^2 per block; dz of the output layer:
// column 0 = 2 (y - T) mask / m (m = *msum, the number of masked points),
// other columns 0.
__global__ __launch_bounds__(256) void k_loss(const float *__restrict__ y, const float *__restrict__ T,
                                              const float *__restrict__ X, int64_t rows,
                                              int64_t npad, int Np, const double *__restrict__ msum,
                                              float *__restrict__ dz, uint16_t *__restrict__ dz16,
                                              double *__restrict__ part) {
  __shared__ double red[256];
  const double inv_m = 1.0 / *msum;
  double acc = 0.0;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < npad;
       t += int64_t(gridDim.x) * blockDim.x) {
    float g = 0.f;
    if (t < rows) {
      const float mk = X[2 * t + 1];
      const float d = (y[t] - T[t]) * mk;
      acc += double(d) * d;
      g = float(2.0 * double(d) * inv_m) * mk;
    }
    for (int o = 0; o < Np; ++o) {
      dz[t * Np + o] = o == 0 ? g : 0.f;
      dz16[t * Np + o] = o == 0 ? f2bf(g) : uint16_t(0);
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (int(threadIdx.x) < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// per-block partial sums of strided float columns (mask count, bias grads):
// column col0 + blockIdx.y into part[blockIdx.y * kPartStride + blockIdx.x]
__global__ __launch_bounds__(256) void k_colsum(const float *__restrict__ a, int64_t rows, int ld,
                                                int col0, double *__restrict__ part) {
  __shared__ double red[256];
  const int col = col0 + int(blockIdx.y);
  part += size_t(blockIdx.y) * kPartStride;
  double acc = 0.0;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < rows;
       t += int64_t(gridDim.x) * blockDim.x)
    acc += a[t * ld + col];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (int(threadIdx.x) < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Totals of per-block partials, summed in block order in double (one thread
// per column): dsum[c] and, where given, fsum[c] = float(dsum[c]).
__global__ void k_sum_partials(const double *__restrict__ part, int nblk, int ncols,
                               double *__restrict__ dsum, float *__restrict__ fsum) {
  const int c = int(blockIdx.x * blockDim.x + threadIdx.x);
  if (c >= ncols) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[size_t(c) * kPartStride + b];
  if (dsum) dsum[c] = s;
  if (fsum) fsum[c] = float(s);
}

// Adam: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, w -= lr c1 m / (sqrt(c2 v) + eps)
// with the bias corrections c1 = 1/(1-b1^t), c2 = 1/(1-b2^t).
__global__ void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * c1 * mi / (sqrtf(c2 * vi) + eps);
  }
}

// bf16 weights [Kp][Np] (zero padded) and float bias [Np] of one layer from
// the flat float32 parameters (W [K27][cout] row-major, then bias).
__global__ void k_pack(const float *__restrict__ wl, int K27, int cout, int Kp, int Np,
                       uint16_t *__restrict__ Wb, float *__restrict__ bias) {
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < int64_t(Kp) * Np;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int k = int(t / Np), o = int(t % Np);
    Wb[t] = (k < K27 && o < cout) ? f2bf(wl[int64_t(k) * cout + o]) : uint16_t(0);
    if (k == 0) bias[o] = o < cout ? wl[int64_t(K27) * cout + o] : 0.f;
  }
}

// flat gradient of one layer from dW [Kp][Np] and the bias partial sums
__global__ void k_grad_gather(const float *__restrict__ dW, int K27, int cout, int Np,
                              float *__restrict__ g) {
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < int64_t(K27) * cout;
       t += int64_t(gridDim.x) * blockDim.x)
    g[t] = dW[(t / cout) * Np + t % cout];
}

// Network inputs of patches [first, first + count): one block per patch.
// Grid point g_d maps to level-0 node v_d p - p + 1 + g_d; the node is a
// patch unknown iff it is an interior grid node.  X[j][q] = (r / ||r_j||,
// mask); scale[j] = ||r_j||_2 (1 if zero).
__global__ __launch_bounds__(256) void k_nn_gather(MeshDims md, int first, const double *__restrict__ r,
                                                   float *__restrict__ X, double *__restrict__ scale,
                                                   const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;
  __shared__ double red[256];
  const int p = md.p, G = 2 * p - 1, G3 = G * G * G;
  const int j = first + int(blockIdx.x);
  const int nv0 = md.n[0] + 1, nv1 = md.n[1] + 1;
  const int v[3] = {j % nv0, (j / nv0) % nv1, j / (nv0 * nv1)};
  auto lidx = [&](int q) -> int64_t {
    const int g[3] = {q % G, (q / G) % G, q / (G * G)};
    int64_t li = 0, stride = 1;
    for (int d = 0; d < 3; ++d) {
      const int node = v[d] * p - p + 1 + g[d];
      if (node < 1 || node > md.ng[d] - 2) return -1;
      li += int64_t(node - 1) * stride;
      stride *= md.nu[d];
    }
    return li;
  };
  double acc = 0.0;
  for (int q = threadIdx.x; q < G3; q += blockDim.x) {
    const int64_t li = lidx(q);
    if (li >= 0) acc += r[li] * r[li];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (int(threadIdx.x) < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  const double nrm = sqrt(red[0]);
  const double s = nrm > 0.0 ? nrm : 1.0;
  if (threadIdx.x == 0) scale[blockIdx.x] = s;
  float *Xj = X + int64_t(blockIdx.x) * G3 * 2;
  for (int q = threadIdx.x; q < G3; q += blockDim.x) {
    const int64_t li = lidx(q);
    Xj[2 * q] = li >= 0 ? float(r[li] / s) : 0.f;
    Xj[2 * q + 1] = li >= 0 ? 1.f : 0.f;
  }
}

// z[unknown of patch j at q] += scale[j] y[j][q]
__global__ __launch_bounds__(256) void k_nn_scatter(MeshDims md, int first,
                                                    const float *__restrict__ y,
                                                    const double *__restrict__ scale,
                                                    double *__restrict__ z, const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;
  const int p = md.p, G = 2 * p - 1, G3 = G * G * G;
  const int j = first + int(blockIdx.x);
  const int nv0 = md.n[0] + 1, nv1 = md.n[1] + 1;
  const int v[3] = {j % nv0, (j / nv0) % nv1, j / (nv0 * nv1)};
  const double s = scale[blockIdx.x];
  for (int q = threadIdx.x; q < G3; q += blockDim.x) {
    const int g[3] = {q % G, (q / G) % G, q / (G * G)};
    int64_t li = 0, stride = 1;
    bool ok = true;
    for (int d = 0; d < 3; ++d) {
      const int node = v[d] * p - p + 1 + g[d];
      if (node < 1 || node > md.ng[d] - 2) ok = false;
      li += int64_t(node - 1) * stride;
      stride *= md.nu[d];
    }
    if (ok) unsafeAtomicAdd(z + li, s * double(y[int64_t(blockIdx.x) * G3 + q]));
  }
}

__global__ void k_fill_f32(float *x, int64_t n, float v) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    x[i] = v;
}

}  // namespace

hipError_t nn_gemm(int M, int N, int K, const uint16_t *A, int64_t ai, int64_t ak,
                   const uint16_t *B, int64_t bk, int64_t bj, float *C, int64_t ldc, bool acc,
                   hipStream_t st) {
  if (M % 16 || N % 16 || K % 16 || M <= 0 || N <= 0 || K <= 0) return hipErrorInvalidValue;
  const int64_t waves = int64_t(M / 16) * (N / 16);
  const int64_t blocks = (waves + 3) / 4;
  if (blocks > (int64_t(1) << 31) - 1) return hipErrorInvalidValue;
  const bool ak1 = ak == 1 && ai % 4 == 0;
  if (ak1 && acc)
    k_gemm<true, true><<<int(blocks), 256, 0, st>>>(M, N, K, A, ai, ak, B, bk, bj, C, ldc);
  else if (ak1)
    k_gemm<true, false><<<int(blocks), 256, 0, st>>>(M, N, K, A, ai, ak, B, bk, bj, C, ldc);
  else if (acc)
    k_gemm<false, true><<<int(blocks), 256, 0, st>>>(M, N, K, A, ai, ak, B, bk, bj, C, ldc);
  else
    k_gemm<false, false><<<int(blocks), 256, 0, st>>>(M, N, K, A, ai, ak, B, bk, bj, C, ldc);
  return hipGetLastError();
}

hipError_t nn_im2col(const uint16_t *act, int64_t rows, int G, int cin, int Kp, int64_t npad,
                     uint16_t *cols, const double *flag, hipStream_t st) {
  k_im2col<<<grid_for(npad * Kp, 256), 256, 0, st>>>(act, rows, G, cin, Kp, npad, cols, flag);
  return hipGetLastError();
}

hipError_t nn_col2im_relu(const float *dcols, int64_t rows, int64_t npad, int G, int cin, int Kp,
                          const float *zprev, int ldzp, float *dz, uint16_t *dz16, hipStream_t st) {
  k_col2im_relu<<<grid_for(npad * cin, 256), 256, 0, st>>>(dcols, rows, npad, G, cin, Kp, zprev,
                                                          ldzp, dz, dz16);
  return hipGetLastError();
}

hipError_t nn_bias_relu(float *z, int64_t rows, int cout, int Np, const float *bias, uint16_t *a,
                        const double *flag, hipStream_t st) {
  k_bias_relu<<<grid_for(rows * cout, 256), 256, 0, st>>>(z, rows, cout, Np, bias, a, flag);
  return hipGetLastError();
}

hipError_t nn_input(const float *X, int64_t rows, int64_t npad, uint16_t *a0, const double *flag,
                    hipStream_t st) {
  k_input_bf16<<<grid_for(npad * 2, 256), 256, 0, st>>>(X, rows, npad, a0, flag);
  return hipGetLastError();
}

hipError_t nn_output(const float *z, int Np, const float *X, int64_t rows, float *y,
                     const double *flag, hipStream_t st) {
  k_output<<<grid_for(rows, 256), 256, 0, st>>>(z, Np, X, rows, y, flag);
  return hipGetLastError();
}

int nn_red_blocks(int64_t n) { return std::min<int64_t>(kPartStride, std::max<int64_t>(1, (n + 255) / 256)); }

hipError_t nn_loss(const float *y, const float *T, const float *X, int64_t rows, int64_t npad,
                   int Np, const double *msum, float *dz, uint16_t *dz16, double *part, hipStream_t st) {
  k_loss<<<nn_red_blocks(npad), 256, 0, st>>>(y, T, X, rows, npad, Np, msum, dz, dz16, part);
  return hipGetLastError();
}

hipError_t nn_colsum(const float *a, int64_t rows, int ld, int col0, int ncols, double *part,
                     hipStream_t st) {
  if (ncols < 1) return hipErrorInvalidValue;
  k_colsum<<<dim3(nn_red_blocks(rows), ncols), 256, 0, st>>>(a, rows, ld, col0, part);
  return hipGetLastError();
}

hipError_t nn_sum_partials(const double *part, int nblk, int ncols, double *dsum, float *fsum,
                           hipStream_t st) {
  if (nblk < 1 || nblk > kPartStride || ncols < 1) return hipErrorInvalidValue;
  k_sum_partials<<<(ncols + 63) / 64, 64, 0, st>>>(part, nblk, ncols, dsum, fsum);
  return hipGetLastError();
}

hipError_t nn_adam(float *w, float *m, float *v, const float *g, int64_t n, float lr, float b1,
                   float b2, float eps, float c1, float c2, hipStream_t st) {
  k_adam<<<grid_for(n, 256), 256, 0, st>>>(w, m, v, g, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t nn_pack(const float *wl, int K27, int cout, int Kp, int Np, uint16_t *Wb, float *bias,
                   hipStream_t st) {
  k_pack<<<grid_for(int64_t(Kp) * Np, 256), 256, 0, st>>>(wl, K27, cout, Kp, Np, Wb, bias);
  return hipGetLastError();
}

hipError_t nn_grad_gather(const float *dW, int K27, int cout, int Np, float *g, hipStream_t st) {
  k_grad_gather<<<grid_for(int64_t(K27) * cout, 256), 256, 0, st>>>(dW, K27, cout, Np, g);
  return hipGetLastError();
}

hipError_t nn_gather(const MeshDims &md, int first, int count, const double *r, float *X,
                     double *scale, const double *flag, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  k_nn_gather<<<count, 256, 0, st>>>(md, first, r, X, scale, flag);
  return hipGetLastError();
}

hipError_t nn_scatter(const MeshDims &md, int first, int count, const float *y,
                      const double *scale, double *z, const double *flag, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  k_nn_scatter<<<count, 256, 0, st>>>(md, first, y, scale, z, flag);
  return hipGetLastError();
}

hipError_t nn_fill(float *x, int64_t n, float v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_fill_f32<<<grid_for(n, 256), 256, 0, st>>>(x, n, v);
  return hipGetLastError();
}

}  // namespace lor

// Fused vector kernels and deterministic reductions for preconditioned /
// flexible conjugate gradients (the Krylov driver of Section 4).
//
// Reductions are two-stage: every block writes one partial sum (grid-stride
// loop, LDS tree), and a one-block finalize kernel adds the partials in a
// fixed order and derives the CG scalars on the device, so the host never
// waits for alpha or beta.  Every kernel of an iteration returns immediately
// once the device-side "done" flag is set, which lets the host enqueue
// iterations ahead of the convergence check.
#include <hip/hip_runtime.h>

#include <cmath>

#include "lor_internal.h"

namespace lor {

namespace {

__device__ inline double block_sum(double v) {
  __shared__ double red[256];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  return red[0];
}

__global__ __launch_bounds__(256) void k_dot(const double *__restrict__ a,
                                             const double *__restrict__ b, int64_t n,
                                             double *__restrict__ partials, const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;
  double acc = 0.0;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    acc += a[i] * b[i];
  const double s = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// partials of a.b and a.c in one pass over a (flexible CG: z.r and z.rold);
// each partial adds its terms in the order k_dot does
__global__ __launch_bounds__(256) void k_dot2(const double *__restrict__ a,
                                              const double *__restrict__ b,
                                              const double *__restrict__ c, int64_t n,
                                              double *__restrict__ pb, double *__restrict__ pc,
                                              const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;
  __shared__ double rb[256], rc[256];
  double ab = 0.0, ac = 0.0;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const double ai = a[i];
    ab += ai * b[i];
    ac += ai * c[i];
  }
  rb[threadIdx.x] = ab;
  rc[threadIdx.x] = ac;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      rb[threadIdx.x] += rb[threadIdx.x + h];
      rc[threadIdx.x] += rc[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pb[blockIdx.x] = rb[0];
    pc[blockIdx.x] = rc[0];
  }
}

// x += alpha p ; r -= alpha q ; (optionally rold = r before) ; partial ||r||^2
__global__ __launch_bounds__(256) void k_cg_update(double *__restrict__ x, double *__restrict__ r,
                                                   double *__restrict__ rold,
                                                   const double *__restrict__ p,
                                                   const double *__restrict__ q, int64_t n,
                                                   const double *scal, double *partials) {
  if (scal[S_DONE] != 0.0) return;
  const double alpha = scal[S_ALPHA];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    x[i] += alpha * p[i];
    const double ri = r[i];
    if (rold) rold[i] = ri;
    const double rn = ri - alpha * q[i];
    r[i] = rn;
    acc += rn * rn;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// p = z + beta p ; q = 0 (q is accumulated with atomics by the operator)
__global__ __launch_bounds__(256) void k_p_update(double *__restrict__ p, double *__restrict__ q,
                                                  const double *__restrict__ z, int64_t n,
                                                  const double *scal) {
  if (scal[S_DONE] != 0.0) return;
  const double beta = scal[S_BETA];
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    p[i] = z[i] + beta * p[i];
    if (q) q[i] = 0.0;  // only when the operator accumulates into q
  }
}

// partial sums of (b - y)^2; with res != nullptr also res = b - y (res may
// be y itself: every element is read before it is written by the same lane)
__global__ __launch_bounds__(256) void k_sub_dot(const double *__restrict__ b, const double *y,
                                                 int64_t n, double *__restrict__ partials,
                                                 double *res) {
  double acc = 0.0;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const double d = b[i] - y[i];
    if (res) res[i] = d;
    acc += d * d;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void k_copy(double *__restrict__ d, const double *__restrict__ s, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    d[i] = s[i];
}

// The iteration count lives on the device (S_ITERS, incremented with each
// recursive residual), so that a captured chunk of iterations can be replayed;
// the solve also stops when S_ITERS reaches S_MAXIT.
__global__ __launch_bounds__(1024) void k_finalize(double *scal, const double *__restrict__ partials,
                                                   int count, int which,
                                                   const double *__restrict__ partials2) {
  if (which != FIN_BB && which != FIN_RRTRUE && scal[S_DONE] != 0.0) return;
  __shared__ double red[1024];
  __shared__ double red2[1024];
  double acc = 0.0, acc2 = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) {
    acc += partials[i];
    if (partials2) acc2 += partials2[i];
  }
  red[threadIdx.x] = acc;
  red2[threadIdx.x] = acc2;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      red[threadIdx.x] += red[threadIdx.x + h];
      red2[threadIdx.x] += red2[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double s = red[0], s2 = red2[0];
  switch (which) {
    case FIN_BB:
      scal[S_BB] = s;
      scal[S_RR] = s;
      scal[S_DONE] = s == 0.0 ? 1.0 : 0.0;
      scal[S_ITERS] = 0.0;
      scal[S_FAIL] = 0.0;
      if (!isfinite(s)) {
        scal[S_FAIL] = 2.0;
        scal[S_DONE] = 1.0;
      }
      break;
    case FIN_PQ:
      scal[S_PQ] = s;
      if (!(s > 0.0)) {
        scal[S_FAIL] = 1.0;
        scal[S_DONE] = 1.0;
      } else {
        scal[S_ALPHA] = scal[S_RHO] / s;
      }
      break;
    case FIN_RR:
      scal[S_RR] = s;
      scal[S_ITERS] += 1.0;
      if (s <= scal[S_TOL2] * scal[S_BB] || scal[S_ITERS] >= scal[S_MAXIT]) scal[S_DONE] = 1.0;
      if (!isfinite(s)) {
        scal[S_FAIL] = 2.0;
        scal[S_DONE] = 1.0;
      }
      break;
    case FIN_RHO:   // s = r.z; before the first iteration: the initial rho
    case FIN_FCG: { // s = r.z, s2 = z.rold
      if (!(s > 0.0)) {
        scal[S_FAIL] = 1.0;
        scal[S_DONE] = 1.0;
        break;
      }
      if (scal[S_ITERS] > 0.0) {
        const double num = which == FIN_FCG ? s - s2 : s;
        scal[S_BETA] = num / scal[S_RHO];
      }
      scal[S_RHO] = s;
      break;
    }
    case FIN_RRTRUE:
      scal[S_RRTRUE] = s;
      break;
  }
}

inline int grid_for(int64_t n, int bs) {
  int64_t g = (n + bs - 1) / bs;
  return int(g > kRedBlocks ? kRedBlocks : (g < 1 ? 1 : g));
}

}  // namespace

int red_blocks(int64_t n) { return grid_for(n, 256); }

hipError_t launch_dot_partials(const double *a, const double *b, int64_t n, double *partials,
                               const double *flag, hipStream_t st) {
  k_dot<<<grid_for(n, 256), 256, 0, st>>>(a, b, n, partials, flag);
  return hipGetLastError();
}

hipError_t launch_dot2_partials(const double *a, const double *b, const double *c, int64_t n,
                                double *pb, double *pc, const double *flag, hipStream_t st) {
  k_dot2<<<grid_for(n, 256), 256, 0, st>>>(a, b, c, n, pb, pc, flag);
  return hipGetLastError();
}

hipError_t launch_finalize(double *scal, const double *partials, int count, int which,
                           const double *partials2, hipStream_t st) {
  k_finalize<<<1, 1024, 0, st>>>(scal, partials, count, which, partials2);
  return hipGetLastError();
}

hipError_t launch_cg_update(double *x, double *r, double *rold, const double *p, const double *q,
                            int64_t n, const double *scal, double *partials, hipStream_t st) {
  k_cg_update<<<grid_for(n, 256), 256, 0, st>>>(x, r, rold, p, q, n, scal, partials);
  return hipGetLastError();
}

hipError_t launch_p_update(double *p, double *q, const double *z, int64_t n, const double *scal,
                           hipStream_t st) {
  k_p_update<<<grid_for(n, 256), 256, 0, st>>>(p, q, z, n, scal);
  return hipGetLastError();
}

hipError_t launch_sub_dot(const double *b, const double *y, int64_t n, double *partials,
                          hipStream_t st, double *res) {
  k_sub_dot<<<grid_for(n, 256), 256, 0, st>>>(b, y, n, partials, res);
  return hipGetLastError();
}

hipError_t launch_copy(double *dst, const double *src, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_copy<<<grid_for(n, 256), 256, 0, st>>>(dst, src, n);
  return hipGetLastError();
}

}  // namespace lor

// Matrix-free high-order CG operator y = K_p x by sum factorization
// (Section 2: O(p^{d+1}) operations per element instead of O(p^{2d})), and the
// collocated right-hand side b = M_p f (eq. system).
//
// 3D kernel layout: one element per group of Q^2 threads (Q = p+1), thread
// (a,b) owns the GLL column (a,b,0..p) in registers.  The xi_3 contractions
// run in registers, the xi_1/xi_2 contractions through LDS.  Geometric factors
// G = w|J| J^-1 J^-T are streamed (6 per node, SoA so that a column slice is
// one coalesced load).  Shared GLL nodes are accumulated with hardware FP64
// atomics; element-interior nodes are owned by one element and stored
// directly.  The element energy x_e . (K_e x_e) is reduced per block so that
// CG gets p^T K p without another pass over the vectors.
#include <hip/hip_runtime.h>

#include "lor_internal.h"

namespace lor {

namespace {

// Map block index -> element tile so that each XCD (blocks are dealt to the 8
// XCDs round robin) works on one contiguous range of elements, which keeps
// neighbouring elements' shared nodes in the same L2.
__device__ inline int xcd_tile(int bid, int nb) {
  const int per = nb / 8, rem = nb % 8;
  const int x = bid % 8, c = bid / 8;
  return x < rem ? x * (per + 1) + c : rem * (per + 1) + (x - rem) * per + c;
}

template <int Q>
__global__ __launch_bounds__(256) void k_apply_cg3(MeshDims md, const double *__restrict__ G,
                                                   const double *__restrict__ Dg,
                                                   const double *__restrict__ x,
                                                   double *__restrict__ y,
                                                   double *__restrict__ partials,
                                                   const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;
  constexpr int Q2 = Q * Q, Q3 = Q2 * Q, EPB = 256 / Q2;
  __shared__ double sD[Q2];
  __shared__ double s0[EPB][Q3];
  __shared__ double s1[EPB][Q3];
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int le = tid / Q2, t = tid % Q2, a = t % Q, b = t / Q;
  if (tid < Q2) sD[tid] = Dg[tid];
  const int64_t nel = int64_t(md.n[0]) * md.n[1] * md.n[2];
  const int64_t e = int64_t(xcd_tile(blockIdx.x, gridDim.x)) * EPB + le;
  const bool active = le < EPB && e < nel;
  const int p = Q - 1;
  int ex = 0, ey = 0, ez = 0;
  if (active) {
    ex = int(e % md.n[0]);
    ey = int((e / md.n[0]) % md.n[1]);
    ez = int(e / (int64_t(md.n[0]) * md.n[1]));
  }
  const int gx = ex * p + a, gy = ey * p + b;
  const bool dir = md.dirichlet;
  const int ox = dir ? 1 : 0;
  bool inxy = true;
  if (dir) inxy = gx > 0 && gx < md.ng[0] - 1 && gy > 0 && gy < md.ng[1] - 1;
  int64_t base = (int64_t(gx - ox) + int64_t(md.nu[0]) * (gy - ox));
  const int64_t sz = int64_t(md.nu[0]) * md.nu[1];
  double u[Q];
#pragma unroll
  for (int c = 0; c < Q; ++c) {
    const int gz = ez * p + c;
    const bool in = active && inxy && (!dir || (gz > 0 && gz < md.ng[2] - 1));
    u[c] = in ? x[base + sz * (gz - ox)] : 0.0;
  }
  __syncthreads();
  double uz[Q];
#pragma unroll
  for (int c = 0; c < Q; ++c) {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < Q; ++k) acc += sD[c * Q + k] * u[k];
    uz[c] = acc;
    if (le < EPB) s0[le][a + Q * (b + Q * c)] = u[c];
  }
  __syncthreads();
  double fz[Q];
  const double *Ge = G + (active ? e : 0) * 6 * Q3;
  double fx[Q], fy[Q];
#pragma unroll
  for (int c = 0; c < Q; ++c) {
    double ux = 0.0, uy = 0.0;
    if (le < EPB) {
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        ux += sD[a * Q + k] * s0[le][k + Q * (b + Q * c)];
        uy += sD[b * Q + k] * s0[le][a + Q * (k + Q * c)];
      }
    }
    const int q = a + Q * (b + Q * c);
    double g00 = 0, g01 = 0, g02 = 0, g11 = 0, g12 = 0, g22 = 0;
    if (active) {
      g00 = Ge[0 * Q3 + q];
      g01 = Ge[1 * Q3 + q];
      g02 = Ge[2 * Q3 + q];
      g11 = Ge[3 * Q3 + q];
      g12 = Ge[4 * Q3 + q];
      g22 = Ge[5 * Q3 + q];
    }
    fx[c] = g00 * ux + g01 * uy + g02 * uz[c];
    fy[c] = g01 * ux + g11 * uy + g12 * uz[c];
    fz[c] = g02 * ux + g12 * uy + g22 * uz[c];
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < Q; ++c) {
    if (le < EPB) {
      s0[le][a + Q * (b + Q * c)] = fx[c];
      s1[le][a + Q * (b + Q * c)] = fy[c];
    }
  }
  __syncthreads();
  double dotp = 0.0;
#pragma unroll
  for (int c = 0; c < Q; ++c) {
    double acc = 0.0;
    if (le < EPB) {
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        acc += sD[k * Q + a] * s0[le][k + Q * (b + Q * c)];
        acc += sD[k * Q + b] * s1[le][a + Q * (k + Q * c)];
        acc += sD[k * Q + c] * fz[k];
      }
    }
    dotp += u[c] * acc;
    const int gz = ez * p + c;
    const bool in = active && inxy && (!dir || (gz > 0 && gz < md.ng[2] - 1));
    if (in) {
      double *dst = y + base + sz * (gz - ox);
      const bool interior = a > 0 && a < p && b > 0 && b < p && c > 0 && c < p;
      if (interior)
        *dst = acc;
      else
        unsafeAtomicAdd(dst, acc);
    }
  }
  if (partials) {
    red[tid] = dotp;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (tid < h) red[tid] += red[tid + h];
      __syncthreads();
    }
    if (tid == 0) partials[blockIdx.x] = red[0];
  }
}

// 2D: one thread per element node, Q^2 threads per element.
template <int Q>
__global__ __launch_bounds__(256) void k_apply_cg2(MeshDims md, const double *__restrict__ G,
                                                   const double *__restrict__ Dg,
                                                   const double *__restrict__ x,
                                                   double *__restrict__ y,
                                                   double *__restrict__ partials,
                                                   const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;
  constexpr int Q2 = Q * Q, EPB = 256 / Q2;
  __shared__ double sD[Q2];
  __shared__ double su[EPB][Q2], sa[EPB][Q2], sb[EPB][Q2];
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int le = tid / Q2, t = tid % Q2, a = t % Q, b = t / Q;
  if (tid < Q2) sD[tid] = Dg[tid];
  const int64_t nel = int64_t(md.n[0]) * md.n[1];
  const int64_t e = int64_t(blockIdx.x) * EPB + le;
  const bool active = le < EPB && e < nel;
  const int p = Q - 1;
  const int ex = active ? int(e % md.n[0]) : 0, ey = active ? int(e / md.n[0]) : 0;
  const int gx = ex * p + a, gy = ey * p + b;
  const bool dir = md.dirichlet;
  const int ox = dir ? 1 : 0;
  bool in = active;
  if (dir) in = in && gx > 0 && gx < md.ng[0] - 1 && gy > 0 && gy < md.ng[1] - 1;
  const int64_t li = int64_t(gx - ox) + int64_t(md.nu[0]) * (gy - ox);
  const double u = in ? x[li] : 0.0;
  if (le < EPB) su[le][t] = u;
  __syncthreads();
  double ua = 0, ub = 0;
  if (le < EPB)
    for (int k = 0; k < Q; ++k) {
      ua += sD[a * Q + k] * su[le][k + Q * b];
      ub += sD[b * Q + k] * su[le][a + Q * k];
    }
  double g00 = 0, g01 = 0, g11 = 0;
  if (active) {
    const double *Ge = G + e * 3 * Q2;
    g00 = Ge[t];
    g01 = Ge[Q2 + t];
    g11 = Ge[2 * Q2 + t];
  }
  __syncthreads();
  if (le < EPB) {
    sa[le][t] = g00 * ua + g01 * ub;
    sb[le][t] = g01 * ua + g11 * ub;
  }
  __syncthreads();
  double acc = 0;
  if (le < EPB)
    for (int k = 0; k < Q; ++k) {
      acc += sD[k * Q + a] * sa[le][k + Q * b];
      acc += sD[k * Q + b] * sb[le][a + Q * k];
    }
  if (in) {
    const bool interior = a > 0 && a < p && b > 0 && b < p;
    if (interior)
      y[li] = acc;
    else
      unsafeAtomicAdd(y + li, acc);
  }
  if (partials) {
    red[tid] = u * acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (tid < h) red[tid] += red[tid + h];
      __syncthreads();
    }
    if (tid == 0) partials[blockIdx.x] = red[0];
  }
}

// b_i = sum over the elements containing node i (fixed order) of w|J| f_i.
template <int DIM>
__global__ void k_rhs_cg(MeshDims md, const double *__restrict__ wdet,
                         const double *__restrict__ f, double *__restrict__ b) {
  const int Q = md.p + 1;
  const int nq = DIM == 3 ? Q * Q * Q : Q * Q;
  const int ox = md.dirichlet ? 1 : 0;
  const int64_t N = int64_t(md.nu[0]) * md.nu[1] * (DIM == 3 ? md.nu[2] : 1);
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < N;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int g[3] = {int(i % md.nu[0]) + ox, int((i / md.nu[0]) % md.nu[1]) + ox,
                      DIM == 3 ? int(i / (int64_t(md.nu[0]) * md.nu[1])) + ox : 0};
    double acc = 0.0;
    for (int c = 0; c < (1 << DIM); ++c) {
      int e[3], l[3];
      bool ok = true;
      for (int d = 0; d < DIM; ++d) {
        const int bit = (c >> d) & 1;
        // candidate elements: g/p (local g%p) and, on an interface, g/p - 1
        if (bit == 0) {
          e[d] = g[d] / md.p;
          l[d] = g[d] - e[d] * md.p;
          if (e[d] >= md.n[d]) ok = false;
        } else {
          if (g[d] % md.p != 0 || g[d] == 0) ok = false;
          e[d] = g[d] / md.p - 1;
          l[d] = md.p;
        }
      }
      if (!ok) continue;
      int64_t ei = e[0] + int64_t(md.n[0]) * (e[1] + (DIM == 3 ? int64_t(md.n[1]) * e[2] : 0));
      int q = l[0] + Q * (l[1] + (DIM == 3 ? Q * l[2] : 0));
      acc += wdet[ei * nq + q];
    }
    b[i] = acc * f[i];
  }
}

inline int grid_for(int64_t n, int bs) {
  int64_t g = (n + bs - 1) / bs;
  return int(g > 65536 ? 65536 : (g < 1 ? 1 : g));
}

template <int Q>
hipError_t apply_q(const MeshDims &md, const double *G, const double *D, const double *x,
                   double *y, double *partials, const double *flag, hipStream_t st) {
  constexpr int Q2 = Q * Q;
  constexpr int EPB = 256 / Q2;
  if (md.dim == 3) {
    const int64_t nel = int64_t(md.n[0]) * md.n[1] * md.n[2];
    const int nb = int((nel + EPB - 1) / EPB);
    k_apply_cg3<Q><<<nb, 256, 0, st>>>(md, G, D, x, y, partials, flag);
  } else {
    const int64_t nel = int64_t(md.n[0]) * md.n[1];
    const int nb = int((nel + EPB - 1) / EPB);
    k_apply_cg2<Q><<<nb, 256, 0, st>>>(md, G, D, x, y, partials, flag);
  }
  return hipGetLastError();
}

}  // namespace

int apply_cg_blocks(const MeshDims &md) {
  const int Q = md.p + 1;
  const int EPB = 256 / (Q * Q);
  const int64_t nel = int64_t(md.n[0]) * md.n[1] * (md.dim == 3 ? md.n[2] : 1);
  return int((nel + EPB - 1) / EPB);
}

hipError_t launch_apply_cg(const MeshDims &md, const double *G, const double *D, const double *x,
                           double *y, double *partials, const double *flag, hipStream_t st) {
  switch (md.p + 1) {
    case 2: return apply_q<2>(md, G, D, x, y, partials, flag, st);
    case 3: return apply_q<3>(md, G, D, x, y, partials, flag, st);
    case 4: return apply_q<4>(md, G, D, x, y, partials, flag, st);
    case 5: return apply_q<5>(md, G, D, x, y, partials, flag, st);
    case 6: return apply_q<6>(md, G, D, x, y, partials, flag, st);
    case 7: return apply_q<7>(md, G, D, x, y, partials, flag, st);
    case 8: return apply_q<8>(md, G, D, x, y, partials, flag, st);
    case 9: return apply_q<9>(md, G, D, x, y, partials, flag, st);
    case 10: return apply_q<10>(md, G, D, x, y, partials, flag, st);
    case 11: return apply_q<11>(md, G, D, x, y, partials, flag, st);
    case 12: return apply_q<12>(md, G, D, x, y, partials, flag, st);
    case 13: return apply_q<13>(md, G, D, x, y, partials, flag, st);
    case 14: return apply_q<14>(md, G, D, x, y, partials, flag, st);
    case 15: return apply_q<15>(md, G, D, x, y, partials, flag, st);
    case 16: return apply_q<16>(md, G, D, x, y, partials, flag, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rhs_cg(const MeshDims &md, const double *wdet, const double *f, double *b,
                         hipStream_t st) {
  const int64_t N = int64_t(md.nu[0]) * md.nu[1] * (md.dim == 3 ? md.nu[2] : 1);
  if (md.dim == 3)
    k_rhs_cg<3><<<grid_for(N, 256), 256, 0, st>>>(md, wdet, f, b);
  else
    k_rhs_cg<2><<<grid_for(N, 256), 256, 0, st>>>(md, wdet, f, b);
  return hipGetLastError();
}

}  // namespace lor

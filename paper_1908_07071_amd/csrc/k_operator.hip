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

// Face records of the DG face kernel: per (face, side) 4 x QF values
// (V, C a_0, C a_1, C a_2), SoA.  Faces of direction s are a structured grid
// n + e_s after those of the lower directions; the element is side 1 of the
// face at its xi_s = 0 end and side 0 at its xi_s = 1 end.
struct FaceRef {
  int64_t f0, f1;  // faces at xi_s = 0 and xi_s = p
};

__device__ inline void elem_faces(const MeshDims &md, int ex, int ey, int ez, FaceRef fr[3]) {
  const int64_t n0 = md.n[0], n1 = md.n[1], n2 = md.n[2];
  const int64_t off1 = (n0 + 1) * n1 * n2, off2 = off1 + n0 * (n1 + 1) * n2;
  fr[0].f0 = ex + (n0 + 1) * (ey + n1 * int64_t(ez));
  fr[0].f1 = fr[0].f0 + 1;
  fr[1].f0 = off1 + ex + n0 * (ey + (n1 + 1) * int64_t(ez));
  fr[1].f1 = fr[1].f0 + n0;
  fr[2].f0 = off2 + ex + n0 * (ey + n1 * int64_t(ez));
  fr[2].f1 = fr[2].f0 + n0 * n1;
}

template <int QF>
__device__ inline void add_face(const double *__restrict__ fo, int64_t face, int side, int q,
                                double &v, double &g0, double &g1, double &g2) {
  const double *r = fo + (face * 2 + side) * 4 * QF;
  v += r[q];
  g0 += r[QF + q];
  g1 += r[2 * QF + q];
  g2 += r[3 * QF + q];
}

// DG == true: the same volume term on the E-vector (element-owned rows, plain
// stores) plus the face records of the IP / BR2 face kernel: flux terms added
// to the reference flux at face nodes before the transposed contractions,
// value terms added to the result.
template <int Q, bool DG>
__global__ __launch_bounds__(256) void k_apply_cg3(MeshDims md, const double *__restrict__ G,
                                                   const double *__restrict__ Dg,
                                                   const double *__restrict__ x,
                                                   double *__restrict__ y,
                                                   double *__restrict__ partials,
                                                   const double *flag,
                                                   const double *__restrict__ fo) {
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
  const int64_t ebase = (active ? e : 0) * Q3 + a + Q * b;
#pragma unroll
  for (int c = 0; c < Q; ++c) {
    if (DG) {
      u[c] = active ? x[ebase + Q2 * c] : 0.0;
    } else {
      const int gz = ez * p + c;
      const bool in = active && inxy && (!dir || (gz > 0 && gz < md.ng[2] - 1));
      u[c] = in ? x[base + sz * (gz - ox)] : 0.0;
    }
  }
  FaceRef fr[3];
  if (DG) elem_faces(md, ex, ey, ez, fr);
  double vt[DG ? Q : 1];
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
    if (DG) {
      double v = 0.0, h0 = 0.0, h1 = 0.0, h2 = 0.0;
      if (active) {
        if (a == 0) add_face<Q2>(fo, fr[0].f0, 1, b + Q * c, v, h0, h1, h2);
        if (a == p) add_face<Q2>(fo, fr[0].f1, 0, b + Q * c, v, h0, h1, h2);
        if (b == 0) add_face<Q2>(fo, fr[1].f0, 1, a + Q * c, v, h0, h1, h2);
        if (b == p) add_face<Q2>(fo, fr[1].f1, 0, a + Q * c, v, h0, h1, h2);
        if (c == 0) add_face<Q2>(fo, fr[2].f0, 1, a + Q * b, v, h0, h1, h2);
        if (c == p) add_face<Q2>(fo, fr[2].f1, 0, a + Q * b, v, h0, h1, h2);
      }
      fx[c] += h0;
      fy[c] += h1;
      fz[c] += h2;
      vt[DG ? c : 0] = v;
    }
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
    if (DG) {
      acc += vt[DG ? c : 0];
      dotp += u[c] * acc;
      if (active) y[ebase + Q2 * c] = acc;
      continue;
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
template <int Q, bool DG>
__global__ __launch_bounds__(256) void k_apply_cg2(MeshDims md, const double *__restrict__ G,
                                                   const double *__restrict__ Dg,
                                                   const double *__restrict__ x,
                                                   double *__restrict__ y,
                                                   double *__restrict__ partials,
                                                   const double *flag,
                                                   const double *__restrict__ fo) {
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
  const int64_t li = DG ? (active ? e : 0) * Q2 + t : int64_t(gx - ox) + int64_t(md.nu[0]) * (gy - ox);
  if (DG) in = active;
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
  double v = 0.0, h0 = 0.0, h1 = 0.0;
  if (DG && active) {
    const int64_t n0 = md.n[0], n1 = md.n[1], off1 = (n0 + 1) * n1;
    const int64_t fx0 = ex + (n0 + 1) * ey, fy0 = off1 + ex + n0 * ey;
    double h2 = 0.0;
    if (a == 0) add_face<Q>(fo, fx0, 1, b, v, h0, h1, h2);
    if (a == p) add_face<Q>(fo, fx0 + 1, 0, b, v, h0, h1, h2);
    if (b == 0) add_face<Q>(fo, fy0, 1, a, v, h0, h1, h2);
    if (b == p) add_face<Q>(fo, fy0 + n0, 0, a, v, h0, h1, h2);
  }
  if (le < EPB) {
    sa[le][t] = g00 * ua + g01 * ub + h0;
    sb[le][t] = g01 * ua + g11 * ub + h1;
  }
  __syncthreads();
  double acc = 0;
  if (le < EPB)
    for (int k = 0; k < Q; ++k) {
      acc += sD[k * Q + a] * sa[le][k + Q * b];
      acc += sD[k * Q + b] * sb[le][a + Q * k];
    }
  if (DG) {
    acc += v;
    if (in) y[li] = acc;
  } else if (in) {
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
                   double *y, double *partials, const double *flag, const double *fo,
                   hipStream_t st) {
  constexpr int Q2 = Q * Q;
  constexpr int EPB = 256 / Q2;
  const int64_t nel = int64_t(md.n[0]) * md.n[1] * (md.dim == 3 ? md.n[2] : 1);
  const int nb = int((nel + EPB - 1) / EPB);
  if (md.dim == 3) {
    if (fo)
      k_apply_cg3<Q, true><<<nb, 256, 0, st>>>(md, G, D, x, y, partials, flag, fo);
    else
      k_apply_cg3<Q, false><<<nb, 256, 0, st>>>(md, G, D, x, y, partials, flag, nullptr);
  } else {
    if (fo)
      k_apply_cg2<Q, true><<<nb, 256, 0, st>>>(md, G, D, x, y, partials, flag, fo);
    else
      k_apply_cg2<Q, false><<<nb, 256, 0, st>>>(md, G, D, x, y, partials, flag, nullptr);
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
                           double *y, double *partials, const double *flag, hipStream_t st,
                           const double *fo) {
  switch (md.p + 1) {
    case 2: return apply_q<2>(md, G, D, x, y, partials, flag, fo, st);
    case 3: return apply_q<3>(md, G, D, x, y, partials, flag, fo, st);
    case 4: return apply_q<4>(md, G, D, x, y, partials, flag, fo, st);
    case 5: return apply_q<5>(md, G, D, x, y, partials, flag, fo, st);
    case 6: return apply_q<6>(md, G, D, x, y, partials, flag, fo, st);
    case 7: return apply_q<7>(md, G, D, x, y, partials, flag, fo, st);
    case 8: return apply_q<8>(md, G, D, x, y, partials, flag, fo, st);
    case 9: return apply_q<9>(md, G, D, x, y, partials, flag, fo, st);
    case 10: return apply_q<10>(md, G, D, x, y, partials, flag, fo, st);
    case 11: return apply_q<11>(md, G, D, x, y, partials, flag, fo, st);
    case 12: return apply_q<12>(md, G, D, x, y, partials, flag, fo, st);
    case 13: return apply_q<13>(md, G, D, x, y, partials, flag, fo, st);
    case 14: return apply_q<14>(md, G, D, x, y, partials, flag, fo, st);
    case 15: return apply_q<15>(md, G, D, x, y, partials, flag, fo, st);
    case 16: return apply_q<16>(md, G, D, x, y, partials, flag, fo, st);
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

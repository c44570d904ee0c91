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

#include <cstdint>

#include "lor_internal.h"

namespace lor {

namespace {

// Workgroup barrier for LDS data only.  __syncthreads() is a release /
// acquire fence at workgroup scope, which makes every wavefront wait for all
// of its outstanding global loads as well; the element-loop kernel keeps the
// next element's loads in flight across its barriers, so it waits for its
// LDS operations only.  (The memory clobber keeps the compiler from moving
// LDS accesses across the barrier.)
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

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
__global__ __launch_bounds__(256) void k_apply_cg3(MeshDims md, const double *G,
                                                   const double *__restrict__ Dg,
                                                   const double *__restrict__ x,
                                                   double *__restrict__ y,
                                                   double *__restrict__ partials,
                                                   const double *flag,
                                                   const double *__restrict__ fo) {
  if (flag && flag[S_DONE] != 0.0) return;
  constexpr int Q2 = Q * Q, Q3 = Q2 * Q, EPB = 256 / Q2;
  __shared__ double sD[Q2];            // D[i][k] = l_k'(x_i)
  __shared__ double sDT[Q2];           // transposed
  __shared__ double su[EPB][Q3];       // element values, staged once
  __shared__ double sf[2][2][EPB][Q2]; // per z-plane fluxes fx, fy (double buffered)
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int le = tid / Q2, t = tid % Q2, a = t % Q, b = t / Q;
  const int lq = le < EPB ? le : 0;  // threads past the last element slot idle
  if (tid < Q2) {
    sD[tid] = Dg[tid];
    sDT[(tid % Q) * Q + tid / Q] = Dg[tid];
  }
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
  const int64_t base = (int64_t(gx - ox) + int64_t(md.nu[0]) * (gy - ox));
  const int64_t sz = int64_t(md.nu[0]) * md.nu[1];
  const int64_t ebase = (active ? e : 0) * Q3 + a + Q * b;
  // gather the column (a, b, 0..p) into LDS
#pragma unroll
  for (int c = 0; c < Q; ++c) {
    double u;
    if (DG) {
      u = active ? x[ebase + Q2 * c] : 0.0;
    } else {
      const int gz = ez * p + c;
      const bool in = active && inxy && (!dir || (gz > 0 && gz < md.ng[2] - 1));
      u = in ? x[base + sz * (gz - ox)] : 0.0;
    }
    if (le < EPB) su[le][a + Q * (b + Q * c)] = u;
  }
  FaceRef fr[3];
  if (DG) elem_faces(md, ex, ey, ez, fr);
  const double *Ge = G + (active ? e : 0) * 6 * Q3 + a + Q * b;
  double gn[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) gn[i] = active ? Ge[i * Q3] : 0.0;
  double acc[Q];
#pragma unroll
  for (int c = 0; c < Q; ++c) acc[c] = 0.0;
  __syncthreads();
  const double *U = su[lq];
  const double *Da = sD + a * Q, *Db = sD + b * Q, *DaT = sDT + a * Q, *DbT = sDT + b * Q;
  // One z-plane per iteration (a real loop: per-plane state only): reference
  // gradient, pointwise G, the transposed xi_1 / xi_2 contractions through a
  // plane buffer, and the transposed xi_3 contraction into the column
  // accumulator.  G of the next plane is loaded one iteration ahead.
#pragma unroll 1
  for (int c = 0; c < Q; ++c) {
    // keep the loop-invariant D rows in LDS instead of 4Q registers
    asm volatile("" ::: "memory");
    const double g00 = gn[0], g01 = gn[1], g02 = gn[2], g11 = gn[3], g12 = gn[4], g22 = gn[5];
    if (c + 1 < Q) {
#pragma unroll
      for (int i = 0; i < 6; ++i) gn[i] = active ? Ge[i * Q3 + Q2 * (c + 1)] : 0.0;
    }
    const double *Dc = Dg + c * Q;  // wave-uniform row
    // the scheduling fences keep each contraction's LDS reads next to their
    // FMAs, so that a plane needs few registers and many waves fit a SIMD
    double ux = 0.0, uy = 0.0, uz = 0.0;
#pragma unroll
    for (int k = 0; k < Q; ++k) ux += Da[k] * U[k + Q * (b + Q * c)];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < Q; ++k) uy += Db[k] * U[a + Q * (k + Q * c)];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < Q; ++k) uz += Dc[k] * U[a + Q * (b + Q * k)];
    __builtin_amdgcn_sched_barrier(0);
    double fx = g00 * ux + g01 * uy + g02 * uz;
    double fy = g01 * ux + g11 * uy + g12 * uz;
    double fz = g02 * ux + g12 * uy + g22 * uz;
    double own = 0.0;  // contributions to node (a, b, c) itself
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
      fx += h0;
      fy += h1;
      fz += h2;
      own = v;
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) acc[k] += Dc[k] * fz;
    if (le < EPB) {
      sf[c & 1][0][le][t] = fx;
      sf[c & 1][1][le][t] = fy;
    }
    __syncthreads();
    const double *FX = sf[c & 1][0][lq], *FY = sf[c & 1][1][lq];
#pragma unroll
    for (int k = 0; k < Q; ++k) own += DaT[k] * FX[k + Q * b];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < Q; ++k) own += DbT[k] * FY[a + Q * k];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < Q; ++k) acc[k] += k == c ? own : 0.0;
  }
  double dotp = 0.0;
#pragma unroll
  for (int c = 0; c < Q; ++c) {
    if (le < EPB) dotp += su[le][a + Q * (b + Q * c)] * acc[c];
    if (DG) {
      if (active) y[ebase + Q2 * c] = acc[c];
      continue;
    }
    const int gz = ez * p + c;
    const bool in = active && inxy && (!dir || (gz > 0 && gz < md.ng[2] - 1));
    if (in) {
      double *dst = y + base + sz * (gz - ox);
      const bool interior = a > 0 && a < p && b > 0 && b < p && c > 0 && c < p;
      if (interior)
        *dst = acc[c];
      else
        unsafeAtomicAdd(dst, acc[c]);
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

// 3D, 5 <= Q <= 8: one element per block of Q wavefronts; wavefront c owns
// the GLL plane (., ., c) with one node per lane.  The plane index is uniform
// in a wavefront, so the xi_3 derivative entries D[c][k] and D[k][c] are
// scalar operands; the rows D[a][.], D[b][.] stay in registers and the
// transposed rows are read from LDS, which keeps the kernel at about 70
// registers so that four elements per CU have their loads in flight (the
// kernel is bound by HBM latency, not by arithmetic).  x and G are loaded
// with one coalesced access per wavefront and array; the three flux
// components go through LDS for the transposed contractions.  Same results
// as the column kernel up to the order of the floating-point sums.
//
// GEO: the geometric factors are recomputed at each node from the element's
// 8 vertices (the same trilinear map and formulas as the set-up kernel that
// stores them) instead of being streamed: 48 bytes per node less to read and
// to hold, for about 200 float64 operations more per node.
template <int Q, bool DG, bool GEO = false>
__global__ __launch_bounds__(Q * 64) __attribute__((amdgpu_waves_per_eu(7)))
void k_apply_pw3(MeshDims md, const double *__restrict__ G, const double *__restrict__ Dg,
                 const double *__restrict__ x, double *__restrict__ y,
                 double *__restrict__ partials, const double *flag,
                 const double *__restrict__ fo, double *__restrict__ yE, GeoArgs geo = GeoArgs{}) {
  if (flag && flag[S_DONE] != 0.0) return;
  constexpr int Q2 = Q * Q, Q3 = Q2 * Q;
  static_assert(Q2 <= 64, "one plane per wavefront");
  __shared__ double su[Q3], sfx[Q3], sfy[Q3], sfz[Q3];
  __shared__ double sDT[Q2];
  __shared__ double red[Q];
  const int lane = threadIdx.x % 64;
  const int c = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const bool valid = lane < Q2;
  const int t = valid ? lane : 0;
  const int a = t % Q, b = t / Q;
  const int node = t + Q2 * c;
  const int64_t nel = int64_t(md.n[0]) * md.n[1] * md.n[2];
  const int64_t e = xcd_tile(blockIdx.x, gridDim.x);
  const bool active = valid && e < nel;
  const int p = Q - 1;
  const int ex = int(e % md.n[0]), ey = int((e / md.n[0]) % md.n[1]),
            ez = int(e / (int64_t(md.n[0]) * md.n[1]));
  double g[6];
  if constexpr (GEO) {
    // G = (w / det) A A^T with A = adj(J), J from the element's trilinear map
    const double xi[3] = {geo.gllx[a], geo.gllx[b], geo.gllx[c]};
    const double om[3] = {1.0 - xi[0], 1.0 - xi[1], 1.0 - xi[2]};
    const double w = geo.gllw[a] * geo.gllw[b] * geo.gllw[c];
    const int nv0 = md.n[0] + 1, nv1 = md.n[1] + 1;
    double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) {
      const int bx = cc & 1, by = (cc >> 1) & 1, bz = (cc >> 2) & 1;
      const int64_t vi = (ex + bx) + int64_t(nv0) * ((ey + by) + int64_t(nv1) * (ez + bz));
      const double gs0 = (bx ? 1.0 : -1.0) * (by ? xi[1] : om[1]) * (bz ? xi[2] : om[2]);
      const double gs1 = (by ? 1.0 : -1.0) * (bx ? xi[0] : om[0]) * (bz ? xi[2] : om[2]);
      const double gs2 = (bz ? 1.0 : -1.0) * (bx ? xi[0] : om[0]) * (by ? xi[1] : om[1]);
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const double X = geo.verts[vi * 3 + r];
        J[r][0] += X * gs0;
        J[r][1] += X * gs1;
        J[r][2] += X * gs2;
      }
    }
    double A[3][3];
    A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double det = J[0][0] * A[0][0] + J[0][1] * A[1][0] + J[0][2] * A[2][0];
    const double f = active ? w / det : 0.0;
    g[0] = f * (A[0][0] * A[0][0] + A[0][1] * A[0][1] + A[0][2] * A[0][2]);
    g[1] = f * (A[0][0] * A[1][0] + A[0][1] * A[1][1] + A[0][2] * A[1][2]);
    g[2] = f * (A[0][0] * A[2][0] + A[0][1] * A[2][1] + A[0][2] * A[2][2]);
    g[3] = f * (A[1][0] * A[1][0] + A[1][1] * A[1][1] + A[1][2] * A[1][2]);
    g[4] = f * (A[1][0] * A[2][0] + A[1][1] * A[2][1] + A[1][2] * A[2][2]);
    g[5] = f * (A[2][0] * A[2][0] + A[2][1] * A[2][1] + A[2][2] * A[2][2]);
  } else {
    // streamed data first: G (6 per node) and x
    const double *Ge = G + (e < nel ? e : 0) * 6 * Q3 + node;
#pragma unroll
    for (int i = 0; i < 6; ++i) g[i] = active ? Ge[i * Q3] : 0.0;
  }
  const int gx = ex * p + a, gy = ey * p + b, gz = ez * p + c;
  const bool dir = md.dirichlet;
  const int ox = dir ? 1 : 0;
  bool in = active;
  if (!DG && dir)
    in = in && gx > 0 && gx < md.ng[0] - 1 && gy > 0 && gy < md.ng[1] - 1 && gz > 0 &&
         gz < md.ng[2] - 1;
  const int64_t li = DG ? e * Q3 + node
                        : int64_t(gx - ox) + int64_t(md.nu[0]) * (int64_t(gy - ox) +
                                                                  int64_t(md.nu[1]) * (gz - ox));
  const double u = in ? x[li] : 0.0;
  if (threadIdx.x < Q2) sDT[(threadIdx.x % Q) * Q + threadIdx.x / Q] = Dg[threadIdx.x];
  double Da[Q], Db[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    Da[k] = Dg[a * Q + k];
    Db[k] = Dg[b * Q + k];
  }
  if (valid) su[node] = u;
  __syncthreads();
  double ux = 0.0, uy = 0.0, uz = 0.0;
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    ux += Da[k] * su[k + Q * b + Q2 * c];
    uy += Db[k] * su[a + Q * k + Q2 * c];
    uz += Dg[c * Q + k] * su[t + Q2 * k];
  }
  double fx = g[0] * ux + g[1] * uy + g[2] * uz;
  double fy = g[1] * ux + g[3] * uy + g[4] * uz;
  double fz = g[2] * ux + g[4] * uy + g[5] * uz;
  double v = 0.0;
  if (DG && active) {
    FaceRef fr[3];
    elem_faces(md, ex, ey, ez, fr);
    double h0 = 0.0, h1 = 0.0, h2 = 0.0;
    if (a == 0) add_face<Q2>(fo, fr[0].f0, 1, b + Q * c, v, h0, h1, h2);
    if (a == p) add_face<Q2>(fo, fr[0].f1, 0, b + Q * c, v, h0, h1, h2);
    if (b == 0) add_face<Q2>(fo, fr[1].f0, 1, a + Q * c, v, h0, h1, h2);
    if (b == p) add_face<Q2>(fo, fr[1].f1, 0, a + Q * c, v, h0, h1, h2);
    if (c == 0) add_face<Q2>(fo, fr[2].f0, 1, a + Q * b, v, h0, h1, h2);
    if (c == p) add_face<Q2>(fo, fr[2].f1, 0, a + Q * b, v, h0, h1, h2);
    fx += h0;
    fy += h1;
    fz += h2;
  }
  if (valid) {
    sfx[node] = fx;
    sfy[node] = fy;
    sfz[node] = fz;
  }
  __syncthreads();
  double acc = v;
  const double *DaT = sDT + a * Q, *DbT = sDT + b * Q;
#pragma unroll
  for (int k = 0; k < Q; ++k)
    acc += DaT[k] * sfx[k + Q * b + Q2 * c] + DbT[k] * sfy[a + Q * k + Q2 * c] +
           Dg[k * Q + c] * sfz[t + Q2 * k];
  if (DG) {
    if (active) y[li] = acc;
  } else if (in) {
    // element-interior nodes belong to this element only; the others are
    // summed over their elements by k_skeleton_gather (no atomics)
    const bool interior = a > 0 && a < p && b > 0 && b < p && c > 0 && c < p;
    if (interior)
      y[li] = acc;
    else
      yE[e * Q3 + node] = acc;
  }
  if (partials) {
    double d = in ? u * acc : 0.0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off);
    if (lane == 0) red[c] = d;
    __syncthreads();
    if (threadIdx.x == 0) {
      double tot = 0.0;
      for (int i = 0; i < Q; ++i) tot += red[i];
      partials[blockIdx.x] = tot;
    }
  }
}

// y on the element skeleton (GLL grid nodes with some coordinate on an
// element interface): the sum over the elements sharing the node of their
// element-local results yE, added in a fixed element order.  Nodes inside
// one element were stored by the element kernel.  One thread per skeleton
// node only: first the grid planes whose z coordinate is an element
// interface (every node of them), then, in the other planes, the grid lines
// whose y coordinate is one (every node), then the rest of those planes'
// nodes whose x coordinate is one.
struct SkeletonParts {
  int64_t nA, nB, nC;  // nodes of the three parts
  int fx, fy, fz;      // interface coordinates per direction among the unknowns
};

__host__ __device__ inline SkeletonParts skeleton_parts(const MeshDims &md) {
  SkeletonParts s;
  const int f = md.dirichlet ? -1 : 1;
  s.fx = md.n[0] + f;
  s.fy = md.n[1] + f;
  s.fz = md.n[2] + f;
  s.nA = int64_t(s.fz) * md.nu[0] * md.nu[1];
  s.nB = int64_t(md.nu[2] - s.fz) * s.fy * md.nu[0];
  s.nC = int64_t(md.nu[2] - s.fz) * (md.nu[1] - s.fy) * s.fx;
  return s;
}

template <int Q>
__global__ __launch_bounds__(256) void k_skeleton_gather(MeshDims md, SkeletonParts sp,
                                                         const double *__restrict__ yE,
                                                         double *__restrict__ y, const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;
  constexpr int Q3 = Q * Q * Q;
  constexpr int p = Q - 1;
  const int ox = md.dirichlet ? 1 : 0;
  const int nx = md.nu[0], ny = md.nu[1];
  // k-th grid coordinate of an interface, and k-th one strictly inside an element
  auto face = [&](int64_t k) { return int(k + ox) * p; };
  auto inner = [&](int64_t k) { return int(k + k / (p - 1) + 1); };
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int g[3];
  if (t < sp.nA) {
    const int64_t per = int64_t(nx) * ny;
    const int64_t kz = t / per, rem = t - kz * per, iy = rem / nx;
    g[0] = int(rem - iy * nx) + ox;
    g[1] = int(iy) + ox;
    g[2] = face(kz);
  } else if ((t -= sp.nA) < sp.nB) {
    const int64_t per = int64_t(sp.fy) * nx;
    const int64_t kz = t / per, rem = t - kz * per, ky = rem / nx;
    g[0] = int(rem - ky * nx) + ox;
    g[1] = face(ky);
    g[2] = inner(kz);
  } else if ((t -= sp.nB) < sp.nC) {
    const int64_t per = int64_t(ny - sp.fy) * sp.fx;
    const int64_t kz = t / per, rem = t - kz * per, ky = rem / sp.fx;
    g[0] = face(rem - ky * sp.fx);
    g[1] = inner(ky);
    g[2] = inner(kz);
  } else {
    return;
  }
  double acc = 0.0;
  for (int cb = 0; cb < 8; ++cb) {
    int e[3], l[3];
    bool ok = true;
    for (int d = 0; d < 3; ++d) {
      if (((cb >> d) & 1) == 0) {
        e[d] = g[d] / p;
        l[d] = g[d] - e[d] * p;
        if (e[d] >= md.n[d]) ok = false;
      } else {
        if (g[d] % p != 0 || g[d] == 0) ok = false;
        e[d] = g[d] / p - 1;
        l[d] = p;
      }
    }
    if (!ok) continue;
    const int64_t ei = e[0] + int64_t(md.n[0]) * (e[1] + int64_t(md.n[1]) * e[2]);
    acc += yE[ei * Q3 + l[0] + Q * (l[1] + Q * l[2])];
  }
  y[(g[0] - ox) + int64_t(nx) * ((g[1] - ox) + int64_t(ny) * (g[2] - ox))] = acc;
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
                   double *y, double *partials, const double *flag, const double *fo, double *yE,
                   const GeoArgs *geo, hipStream_t st) {
  constexpr int Q2 = Q * Q;
  constexpr int EPB = 256 / Q2;
  const int64_t nel = int64_t(md.n[0]) * md.n[1] * (md.dim == 3 ? md.n[2] : 1);
  const int nb = int((nel + EPB - 1) / EPB);
  if constexpr (Q >= 5 && Q <= 8) {
    if (md.dim == 3) {
      if (fo) {
        k_apply_pw3<Q, true><<<int(nel), Q * 64, 0, st>>>(md, G, D, x, y, partials, flag, fo,
                                                          nullptr);
      } else {
        if (!yE) return hipErrorInvalidValue;
        if (geo)
          k_apply_pw3<Q, false, true><<<int(nel), Q * 64, 0, st>>>(md, nullptr, D, x, y, partials, flag,
                                                                   nullptr, yE, *geo);
        else
          k_apply_pw3<Q, false><<<int(nel), Q * 64, 0, st>>>(md, G, D, x, y, partials, flag,
                                                             nullptr, yE);
        const SkeletonParts sp = skeleton_parts(md);
        const int64_t nsk = sp.nA + sp.nB + sp.nC;
        if (md.nu[0] > 0 && md.nu[1] > 0 && md.nu[2] > 0 && nsk > 0) {
          if ((nsk + 255) / 256 > int64_t(INT32_MAX)) return hipErrorInvalidValue;
          k_skeleton_gather<Q><<<unsigned((nsk + 255) / 256), 256, 0, st>>>(md, sp, yE, y, flag);
        }
      }
      return hipGetLastError();
    }
  }
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

bool apply_cg_uses_skeleton(const MeshDims &md) {
  return md.dim == 3 && md.p + 1 >= 5 && md.p + 1 <= 8;
}

int apply_cg_blocks(const MeshDims &md, bool dg) {
  const int Q = md.p + 1;
  (void)dg;
  if (md.dim == 3 && Q >= 5 && Q <= 8) return int(int64_t(md.n[0]) * md.n[1] * md.n[2]);
  const int EPB = 256 / (Q * Q);
  const int64_t nel = int64_t(md.n[0]) * md.n[1] * (md.dim == 3 ? md.n[2] : 1);
  return int((nel + EPB - 1) / EPB);
}

hipError_t launch_apply_cg(const MeshDims &md, const double *G, const double *D, const double *x,
                           double *y, double *partials, const double *flag, hipStream_t st,
                           const double *fo, double *yE, const GeoArgs *geo) {
  if (geo && !(md.dim == 3 && md.p + 1 >= 5 && md.p + 1 <= 8 && !fo)) return hipErrorInvalidValue;
  switch (md.p + 1) {
    case 2: return apply_q<2>(md, G, D, x, y, partials, flag, fo, yE, geo, st);
    case 3: return apply_q<3>(md, G, D, x, y, partials, flag, fo, yE, geo, st);
    case 4: return apply_q<4>(md, G, D, x, y, partials, flag, fo, yE, geo, st);
    case 5: return apply_q<5>(md, G, D, x, y, partials, flag, fo, yE, geo, st);
    case 6: return apply_q<6>(md, G, D, x, y, partials, flag, fo, yE, geo, st);
    case 7: return apply_q<7>(md, G, D, x, y, partials, flag, fo, yE, geo, st);
    case 8: return apply_q<8>(md, G, D, x, y, partials, flag, fo, yE, geo, st);
    case 9: return apply_q<9>(md, G, D, x, y, partials, flag, fo, yE, geo, st);
    case 10: return apply_q<10>(md, G, D, x, y, partials, flag, fo, yE, geo, st);
    case 11: return apply_q<11>(md, G, D, x, y, partials, flag, fo, yE, geo, st);
    case 12: return apply_q<12>(md, G, D, x, y, partials, flag, fo, yE, geo, st);
    case 13: return apply_q<13>(md, G, D, x, y, partials, flag, fo, yE, geo, st);
    case 14: return apply_q<14>(md, G, D, x, y, partials, flag, fo, yE, geo, st);
    case 15: return apply_q<15>(md, G, D, x, y, partials, flag, fo, yE, geo, st);
    case 16: return apply_q<16>(md, G, D, x, y, partials, flag, fo, yE, geo, st);
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

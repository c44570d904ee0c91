// Set-up kernels: GLL node coordinates, geometric factors of the high-order
// operator, the low-order refined Q1 stencils of every hierarchy level, the
// coarse-space restriction / prolongation and the dense coarse inverse.
//
// The node coordinates and the LOR stencils are computed in a fixed float64
// operation order without contraction (this file is built with
// -ffp-contract=off as well): the MDF orderings are decided by comparisons of
// values derived from them, and a reference implementation that follows the
// same order reproduces them bit for bit.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "lor_internal.h"

#pragma clang fp contract(off)

namespace lor {

namespace {

__device__ inline int64_t lex3(int x, int y, int z, int nx, int ny) {
  return int64_t(x) + int64_t(nx) * (int64_t(y) + int64_t(ny) * z);
}

// Q1 map of a structured element at reference point xi, pinned order:
// phi_c = (l(c_x,xi_0) * l(c_y,xi_1)) * l(c_z,xi_2); X_r = sum_c V_c,r phi_c.
template <int DIM>
__device__ void q1_map(const double *verts, const MeshDims &md, const int *e, const double *xi,
                       double *X) {
  const int nv0 = md.n[0] + 1, nv1 = md.n[1] + 1;
  double om[3], phi[8];
  for (int i = 0; i < DIM; ++i) om[i] = 1.0 - xi[i];
  for (int c = 0; c < (1 << DIM); ++c) {
    double f = (c & 1) ? xi[0] : om[0];
    for (int i = 1; i < DIM; ++i) f = f * (((c >> i) & 1) ? xi[i] : om[i]);
    phi[c] = f;
  }
  for (int r = 0; r < DIM; ++r) {
    double acc = 0.0;
    for (int c = 0; c < (1 << DIM); ++c) {
      const int vx = e[0] + (c & 1), vy = e[1] + ((c >> 1) & 1),
                vz = DIM == 3 ? e[2] + ((c >> 2) & 1) : 0;
      const int64_t vi = lex3(vx, vy, vz, nv0, nv1);
      acc = acc + verts[vi * DIM + r] * phi[c];
    }
    X[r] = acc;
  }
}

template <int DIM>
__global__ void k_node_coords(MeshDims md, const double *__restrict__ verts,
                              const double *__restrict__ gllx, double *__restrict__ coords) {
  const int64_t np = int64_t(md.ng[0]) * md.ng[1] * md.ng[2];
  for (int64_t g = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; g < np;
       g += int64_t(gridDim.x) * blockDim.x) {
    int gi[3] = {int(g % md.ng[0]), int((g / md.ng[0]) % md.ng[1]),
                 int(g / (int64_t(md.ng[0]) * md.ng[1]))};
    int e[3];
    double xi[3];
    for (int i = 0; i < DIM; ++i) {
      e[i] = min(gi[i] / md.p, md.n[i] - 1);
      xi[i] = gllx[gi[i] - e[i] * md.p];
    }
    double X[3];
    q1_map<DIM>(verts, md, e, xi, X);
    for (int r = 0; r < DIM; ++r) coords[r * np + g] = X[r];
  }
}

// E-vector node coordinates: every element maps its own GLL nodes (same
// operation order as the grid coordinates above).  Layout [node][dim].
template <int DIM>
__global__ void k_dg_coords(MeshDims md, const double *__restrict__ verts,
                            const double *__restrict__ gllx, double *__restrict__ coords) {
  const int Q = md.p + 1;
  const int nq = DIM == 3 ? Q * Q * Q : Q * Q;
  const int64_t nel = int64_t(md.n[0]) * md.n[1] * md.n[2];
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < nel * nq;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t e = t / nq;
    const int q = int(t % nq);
    const int ec[3] = {int(e % md.n[0]), int((e / md.n[0]) % md.n[1]),
                       int(e / (int64_t(md.n[0]) * md.n[1]))};
    const int l[3] = {q % Q, (q / Q) % Q, q / (Q * Q)};
    double xi[3];
    for (int i = 0; i < DIM; ++i) xi[i] = gllx[l[i]];
    double X[3];
    q1_map<DIM>(verts, md, ec, xi, X);
    for (int r = 0; r < DIM; ++r) coords[t * DIM + r] = X[r];
  }
}

// Geometric factors G = w |J| J^-1 J^-T (symmetric, d(d+1)/2 values per GLL
// node, element-major SoA [e][comp][node]) and w |J| for the collocated mass.
template <int DIM>
__global__ void k_geom(MeshDims md, const double *__restrict__ verts,
                       const double *__restrict__ gllx, const double *__restrict__ gllw,
                       const double *__restrict__ coef, double *__restrict__ G,
                       double *__restrict__ wdet, int *bad) {
  const int Q = md.p + 1;
  const int nq = DIM == 3 ? Q * Q * Q : Q * Q;
  const int64_t nel = int64_t(md.n[0]) * md.n[1] * (DIM == 3 ? md.n[2] : 1);
  const int ncomp = DIM == 3 ? 6 : 3;
  const int nv0 = md.n[0] + 1, nv1 = md.n[1] + 1;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < nel * nq;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t e = t / nq;
    const int q = int(t % nq);
    const int e3[3] = {int(e % md.n[0]), int((e / md.n[0]) % md.n[1]),
                       DIM == 3 ? int(e / (int64_t(md.n[0]) * md.n[1])) : 0};
    const int qi[3] = {q % Q, (q / Q) % Q, q / (Q * Q)};
    double xi[3], om[3];
    double w = 1.0;
    for (int i = 0; i < DIM; ++i) {
      xi[i] = gllx[qi[i]];
      om[i] = 1.0 - xi[i];
      w *= gllw[qi[i]];
    }
    double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int c = 0; c < (1 << DIM); ++c) {
      const int b[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
      const int vx = e3[0] + b[0], vy = e3[1] + b[1], vz = DIM == 3 ? e3[2] + b[2] : 0;
      const int64_t vi = lex3(vx, vy, vz, nv0, nv1);
      for (int s = 0; s < DIM; ++s) {
        double gsd = b[s] ? 1.0 : -1.0;
        for (int i = 0; i < DIM; ++i)
          if (i != s) gsd *= b[i] ? xi[i] : om[i];
        for (int r = 0; r < DIM; ++r) J[r][s] += verts[vi * DIM + r] * gsd;
      }
    }
    double det, A[3][3];
    if (DIM == 3) {
      A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
      A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
      A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
      A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
      A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
      A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
      A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
      A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
      A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
      det = J[0][0] * A[0][0] + J[0][1] * A[1][0] + J[0][2] * A[2][0];
    } else {
      A[0][0] = J[1][1];
      A[0][1] = -J[0][1];
      A[1][0] = -J[1][0];
      A[1][1] = J[0][0];
      det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    }
    if (!(det > 0.0)) atomicOr(bad, 1);
    // G = (w / det) * A A^T, with A = det * J^-1 (times the coefficient b
    // at the node: -div(b grad u), Section 4.2); G may be null when the
    // operator recomputes it
    const double f = coef ? (w / det) * coef[e * nq + q] : w / det;
    if (G) {
      double *Ge = G + e * ncomp * nq;
      int comp = 0;
      for (int r = 0; r < DIM; ++r)
        for (int c2 = r; c2 < DIM; ++c2) {
          double acc = 0.0;
          for (int s = 0; s < DIM; ++s) acc += A[r][s] * A[c2][s];
          Ge[comp * nq + q] = f * acc;
          ++comp;
        }
    }
    wdet[e * nq + q] = w * det;
  }
}

// Curved (isoparametric) elements: the geometric factors from the GLL node
// coordinates (SoA [dim][grid point]).  J[r][s] at node q of element e is the
// derivative along reference direction s of the interpolant of the element's
// node coordinates X_r: sum_a D[q_s][a] X_r(node q with its s-index set to a).
template <int DIM>
__global__ void k_geom_nodal(MeshDims md, const double *__restrict__ coords,
                             const double *__restrict__ D, const double *__restrict__ gllw,
                             const double *__restrict__ coef, double *__restrict__ G,
                             double *__restrict__ wdet, int *bad) {
  const int Q = md.p + 1;
  const int nq = DIM == 3 ? Q * Q * Q : Q * Q;
  const int64_t nel = int64_t(md.n[0]) * md.n[1] * (DIM == 3 ? md.n[2] : 1);
  const int ncomp = DIM == 3 ? 6 : 3;
  const int64_t fnp = int64_t(md.ng[0]) * md.ng[1] * md.ng[2];
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < nel * nq;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t e = t / nq;
    const int q = int(t % nq);
    const int e3[3] = {int(e % md.n[0]), int((e / md.n[0]) % md.n[1]),
                       DIM == 3 ? int(e / (int64_t(md.n[0]) * md.n[1])) : 0};
    const int qi[3] = {q % Q, (q / Q) % Q, DIM == 3 ? q / (Q * Q) : 0};
    double w = 1.0;
    for (int i = 0; i < DIM; ++i) w *= gllw[qi[i]];
    double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int sd = 0; sd < DIM; ++sd)
      for (int a = 0; a < Q; ++a) {
        int g[3];
        for (int i = 0; i < 3; ++i) g[i] = e3[i] * md.p + (i == sd ? a : qi[i]);
        const int64_t gi = g[0] + int64_t(md.ng[0]) * (g[1] + (DIM == 3 ? int64_t(md.ng[1]) * g[2] : 0));
        const double dq = D[qi[sd] * Q + a];
        for (int r = 0; r < DIM; ++r) J[r][sd] += dq * coords[r * fnp + gi];
      }
    double det, A[3][3];
    if (DIM == 3) {
      A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
      A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
      A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
      A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
      A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
      A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
      A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
      A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
      A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
      det = J[0][0] * A[0][0] + J[0][1] * A[1][0] + J[0][2] * A[2][0];
    } else {
      A[0][0] = J[1][1];
      A[0][1] = -J[0][1];
      A[1][0] = -J[1][0];
      A[1][1] = J[0][0];
      det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    }
    if (!(det > 0.0)) atomicOr(bad, 1);
    const double f = coef ? (w / det) * coef[e * nq + q] : w / det;
    double *Ge = G + e * ncomp * nq;
    int comp = 0;
    for (int r = 0; r < DIM; ++r)
      for (int c2 = r; c2 < DIM; ++c2) {
        double acc = 0.0;
        for (int sd = 0; sd < DIM; ++sd) acc += A[r][sd] * A[c2][sd];
        Ge[comp * nq + q] = f * acc;
        ++comp;
      }
    wdet[e * nq + q] = w * det;
  }
}

// LOR stencil of one level of the element-structured hierarchy.  For grid
// point g the 3^d slots are filled, in the order of the cells S = g - 1 + s
// (s = s_x + 2 s_y + 4 s_z ascending), with the Q1 stiffness entries
// K_S[corner of g][corner of g+o].  K_S uses 2^d Gauss points; every
// intermediate is computed in a fixed order (see the per-line comments).
struct KeptIdx {
  int fine[kMaxP + 1];  // level 1D index m -> GLL index kept[m]
};

template <int DIM>
__global__ void k_lor_stencil(MeshDims md, int s, KeptIdx kept, const double *__restrict__ fine,
                              double g0, double g1, const double *__restrict__ coef,
                              double *__restrict__ out) {
  constexpr int NC = 1 << DIM;
  constexpr int NS = DIM == 3 ? 27 : 9;
  const int lng[3] = {md.n[0] * s + 1, md.n[1] * s + 1, DIM == 3 ? md.n[2] * s + 1 : 1};
  const int64_t npts = int64_t(lng[0]) * lng[1] * lng[2];
  const int64_t fnp = int64_t(md.ng[0]) * md.ng[1] * md.ng[2];
  const double gq[2] = {g0, g1};
  const double wq = DIM == 3 ? 0.125 : 0.25;
  for (int64_t g = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; g < npts;
       g += int64_t(gridDim.x) * blockDim.x) {
    const int gi[3] = {int(g % lng[0]), int((g / lng[0]) % lng[1]),
                       int(g / (int64_t(lng[0]) * lng[1]))};
    double acc[NS];
    for (int sl = 0; sl < NS; ++sl) acc[sl] = 0.0;
    for (int sc = 0; sc < NC; ++sc) {
      int S[3] = {0, 0, 0};
      bool ok = true;
      for (int i = 0; i < DIM; ++i) {
        S[i] = gi[i] - 1 + ((sc >> i) & 1);
        if (S[i] < 0 || S[i] >= lng[i] - 1) ok = false;
      }
      if (!ok) continue;
      // corners of the cell: level grid point -> GLL grid point -> coordinates
      double X[NC][DIM];
      for (int c = 0; c < NC; ++c) {
        int64_t fi = 0, stride = 1;
        for (int i = 0; i < DIM; ++i) {
          const int G = S[i] + ((c >> i) & 1);
          const int e = min(G / s, md.n[i] - 1);
          const int f = e * md.p + kept.fine[G - e * s];
          fi += int64_t(f) * stride;
          stride *= md.ng[i];
        }
        for (int r = 0; r < DIM; ++r) X[c][r] = fine[r * fnp + fi];
      }
      int ca = 0;  // corner of g in S
      for (int i = 0; i < DIM; ++i) ca |= (gi[i] - S[i]) << i;
      double K[NC];
      for (int b = 0; b < NC; ++b) K[b] = 0.0;
      for (int q = 0; q < NC; ++q) {
        double lv[3][2];
        for (int i = 0; i < DIM; ++i) {
          const double xi = gq[(q >> i) & 1];
          lv[i][0] = 1.0 - xi;
          lv[i][1] = xi;
        }
        double gr[NC][DIM];
        for (int c = 0; c < NC; ++c) {
          const int bt[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
          for (int sd = 0; sd < DIM; ++sd) {
            // product of l over the other directions, ascending
            double val = 0.0;
            bool first = true;
            for (int t = 0; t < DIM; ++t) {
              if (t == sd) continue;
              val = first ? lv[t][bt[t]] : val * lv[t][bt[t]];
              first = false;
            }
            gr[c][sd] = bt[sd] ? val : -val;
          }
        }
        double J[DIM][DIM];
        for (int r = 0; r < DIM; ++r)
          for (int sd = 0; sd < DIM; ++sd) {
            double a = 0.0;
            for (int c = 0; c < NC; ++c) a = a + X[c][r] * gr[c][sd];
            J[r][sd] = a;
          }
        double A[DIM][DIM], det;
        if constexpr (DIM == 3) {
          A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
          A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
          A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
          A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
          A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
          A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
          A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
          A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
          A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
          det = J[0][0] * A[0][0] + J[0][1] * A[1][0] + J[0][2] * A[2][0];
        } else {
          A[0][0] = J[1][1];
          A[0][1] = -J[0][1];
          A[1][0] = -J[1][0];
          A[1][1] = J[0][0];
          det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        }
        const double coef = wq / det;
        double u[NC][DIM];
        for (int c = 0; c < NC; ++c)
          for (int r = 0; r < DIM; ++r) {
            double a = A[0][r] * gr[c][0] + A[1][r] * gr[c][1];
            if constexpr (DIM == 3) a = a + A[2][r] * gr[c][2];
            u[c][r] = a;
          }
        for (int b = 0; b < NC; ++b) {
          double dot = u[ca][0] * u[b][0] + u[ca][1] * u[b][1];
          if constexpr (DIM == 3) dot = dot + u[ca][2] * u[b][2];
          K[b] = K[b] + coef * dot;
        }
      }
      if (coef) {
        // the cell's coefficient: mean of b at its corners, GLL nodes of the
        // element holding the cell (corners ascending from 0.0, then 2^-d)
        const int Q = md.p + 1;
        int64_t eflat = 0, estride = 1;
        int mloc[3] = {0, 0, 0};
        for (int i = 0; i < DIM; ++i) {
          const int e = S[i] / s;
          mloc[i] = S[i] - e * s;
          eflat += int64_t(e) * estride;
          estride *= md.n[i];
        }
        const double *ce = coef + eflat * (DIM == 3 ? Q * Q * Q : Q * Q);
        double bs = 0.0;
        for (int c = 0; c < NC; ++c) {
          int lf = 0, ls = 1;
          for (int i = 0; i < DIM; ++i) {
            lf += kept.fine[mloc[i] + ((c >> i) & 1)] * ls;
            ls *= Q;
          }
          bs = bs + ce[lf];
        }
        bs = bs * (DIM == 3 ? 0.125 : 0.25);
        for (int b = 0; b < NC; ++b) K[b] = K[b] * bs;
      }
      for (int b = 0; b < NC; ++b) {
        int sl = 0, p3 = 1;
        for (int i = 0; i < DIM; ++i) {
          const int o = (S[i] + ((b >> i) & 1)) - gi[i];
          sl += (o + 1) * p3;
          p3 *= 3;
        }
        acc[sl] = acc[sl] + K[b];
      }
    }
    for (int sl = 0; sl < NS; ++sl) out[sl * npts + g] = acc[sl];
  }
}

// ---------------------------------------------------------------- coarse space
// P_0: Q1 interpolation of element-vertex values at the GLL grid nodes, in
// reference coordinates; weights 1 - x_a and x_a per direction.  Only the
// interior vertices are unknowns (Dirichlet).

// Weight of the vertex hat function at offset o (0 .. 2p-2) from the first
// grid node after the previous vertex: node a = o + 1 of the pair of
// elements sharing the vertex.
__device__ __forceinline__ double hat_weight(const double *__restrict__ gllx, int p, int o) {
  const int a = o + 1;
  return a <= p ? gllx[a] : 1.0 - gllx[a - p];
}

// rc = P_0^T r: one wavefront per interior vertex; lanes take (ox, oy) pairs
// of the vertex's (2p-1)^d support and loop over oz.
template <int DIM>
__global__ __launch_bounds__(256) void k_coarse_restrict(MeshDims md, const double *__restrict__ gllx,
                                                         const double *__restrict__ r,
                                                         double *__restrict__ rc, int nc) {
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= nc) return;  // the whole wavefront leaves; no block-level barrier follows
  const int ncx = md.n[0] - 1, ncy = md.n[1] - 1;
  const int v[3] = {c % ncx + 1, (c / ncx) % ncy + 1, DIM == 3 ? c / (ncx * ncy) + 1 : 0};
  const int p = md.p, w1 = 2 * p - 1;
  const int64_t sy = md.nu[0], sz = int64_t(md.nu[0]) * md.nu[1];
  double acc = 0.0;
  if (DIM == 3) {
    for (int t = lane; t < w1 * w1; t += 64) {
      const int ox = t % w1, oy = t / w1;
      const double wxy = hat_weight(gllx, p, ox) * hat_weight(gllx, p, oy);
      const double *src = r + ((v[0] - 1) * p + ox) + sy * ((v[1] - 1) * p + oy) + sz * ((v[2] - 1) * p);
#pragma unroll 4
      for (int oz = 0; oz < w1; ++oz) acc += wxy * hat_weight(gllx, p, oz) * src[sz * oz];
    }
  } else {
    for (int t = lane; t < w1 * w1; t += 64) {
      const int ox = t % w1, oy = t / w1;
      acc += hat_weight(gllx, p, ox) * hat_weight(gllx, p, oy) *
             r[((v[0] - 1) * p + ox) + sy * ((v[1] - 1) * p + oy)];
    }
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) rc[c] = acc;
}

// The same sum with the degree fixed at compile time: each lane takes every
// 64th point of the flattened (2p-1)^d support, all of its loads issued
// together; the 1D hat weights come from LDS.
template <int DIM, int P>
__global__ __launch_bounds__(256) void k_coarse_restrict_p(MeshDims md, const double *__restrict__ gllx,
                                                           const double *__restrict__ r,
                                                           double *__restrict__ rc, int nc) {
  constexpr int W1 = 2 * P - 1, W = DIM == 3 ? W1 * W1 * W1 : W1 * W1, NQ = (W + 63) / 64;
  __shared__ double hw[W1];
  if (int(threadIdx.x) < W1) hw[threadIdx.x] = hat_weight(gllx, P, int(threadIdx.x));
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= nc) return;  // no barrier follows
  const int ncx = md.n[0] - 1, ncy = md.n[1] - 1;
  const int v[3] = {c % ncx + 1, (c / ncx) % ncy + 1, DIM == 3 ? c / (ncx * ncy) + 1 : 0};
  const int64_t sy = md.nu[0], sz = int64_t(md.nu[0]) * md.nu[1];
  const double *src = r + (v[0] - 1) * P + sy * ((v[1] - 1) * P) + (DIM == 3 ? sz * ((v[2] - 1) * P) : 0);
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    const int q = lane + 64 * k;
    if (q < W) {
      const int ox = q % W1, oy = (q / W1) % W1, oz = DIM == 3 ? q / (W1 * W1) : 0;
      const double wq = hw[ox] * hw[oy] * (DIM == 3 ? hw[oz] : 1.0);
      acc += wq * src[ox + sy * oy + sz * oz];
    }
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) rc[c] = acc;
}

// z = P_0 xc on the unknowns: a workgroup covers 64 unknowns of each of four
// x-lines; lines (y, z) from the grid of blocks.
template <int DIM>
__global__ __launch_bounds__(256) void k_coarse_prolong(MeshDims md, const double *__restrict__ gllx,
                                                        const double *__restrict__ xc,
                                                        double *__restrict__ z, const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;
  const int ix = blockIdx.x * 64 + threadIdx.x;
  const int iy = blockIdx.y * 4 + threadIdx.y;
  if (ix >= md.nu[0] || iy >= md.nu[1]) return;
  const int gi[3] = {ix + 1, iy + 1, DIM == 3 ? int(blockIdx.z) + 1 : 0};
  const int ncx = md.n[0] - 1, ncy = md.n[1] - 1;
  int ev[3] = {0, 0, 0};
  double wl[3] = {1.0, 1.0, 1.0}, wh[3] = {0.0, 0.0, 0.0};
  for (int d = 0; d < DIM; ++d) {
    const int e = min(gi[d] / md.p, md.n[d] - 1);
    const int a = gi[d] - e * md.p;
    ev[d] = e;
    wl[d] = 1.0 - gllx[a];
    wh[d] = gllx[a];
  }
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < (1 << DIM); ++c) {
    double w = 1.0;
    int vi[3] = {1, 1, 1};
    bool ok = true;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int b = (c >> d) & 1;
      vi[d] = ev[d] + b;
      w *= b ? wh[d] : wl[d];
      ok = ok && vi[d] > 0 && vi[d] < md.n[d];
    }
    const int64_t ci = (vi[0] - 1) + int64_t(ncx) * ((vi[1] - 1) + (DIM == 3 ? int64_t(ncy) * (vi[2] - 1) : 0));
    acc += ok ? w * xc[ok ? ci : 0] : 0.0;
  }
  z[ix + int64_t(md.nu[0]) * (gi[1] - 1 + (DIM == 3 ? int64_t(md.nu[1]) * (gi[2] - 1) : 0))] = acc;
}

// y = A x for a dense row-major n x n matrix: eight rows per workgroup, one
// per wavefront; x is staged through LDS in tiles shared by the eight rows,
// and each lane keeps eight loads of its row in flight.
constexpr int kGemvTile = 2048;
constexpr int kGemvRows = 8;
// TA: float64 inverse, or its float32 copy with the mixed-precision
// preconditioner (products and sums in float64 either way)
template <typename TA>
__global__ __launch_bounds__(64 * kGemvRows) void k_gemv(int n, const TA *__restrict__ A,
                                                         const double *__restrict__ x,
                                                         double *__restrict__ y, const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;  // uniform over the grid
  __shared__ double xs[kGemvTile];
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * kGemvRows + (threadIdx.x >> 6);
  const bool live = row < n;
  const TA *a = A + int64_t(live ? row : 0) * n;
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int j0 = 0; j0 < n; j0 += kGemvTile) {
    const int m = min(kGemvTile, n - j0);
    __syncthreads();
    for (int t = threadIdx.x; t < m; t += 64 * kGemvRows) xs[t] = x[j0 + t];
    __syncthreads();
    const TA *aj = a + j0;
    int j = lane;
    for (; j + 448 < m; j += 512) {
      double av[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) av[q] = double(aj[j + 64 * q]);
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] += av[q] * xs[j + 64 * q];
    }
    for (; j < m; j += 64) acc[0] += double(aj[j]) * xs[j];
  }
  double sum = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_down(sum, off, 64);
  if (live && lane == 0) y[row] = sum;
}

// In-place Gauss-Jordan inversion of an SPD matrix, step k (no pivoting).
// Scalar Gauss-Jordan inverse of one bk x bk block (bk <= 128) by one
// workgroup: M (leading dimension ldm) -> Minv (bk x bk, dense).  The block is
// the pivot block of an SPD matrix after earlier elimination steps, so every
// pivot must be positive (otherwise *bad is set).
__global__ __launch_bounds__(1024) void k_small_inverse(const double *__restrict__ M, int ldm,
                                                        double *__restrict__ Minv, int bk, int *bad) {
  __shared__ double rowk[128], colk[128];
  const int tid = threadIdx.x;
  for (int t = tid; t < bk * bk; t += blockDim.x) Minv[t] = M[int64_t(t / bk) * ldm + t % bk];
  __syncthreads();
  for (int k = 0; k < bk; ++k) {
    const double piv = Minv[k * bk + k];
    if (tid == 0 && !(piv > 0.0)) atomicOr(bad, 1);
    for (int j = tid; j < bk; j += blockDim.x) {
      rowk[j] = j == k ? 1.0 / piv : Minv[k * bk + j] / piv;
      colk[j] = j == k ? 0.0 : Minv[j * bk + k];
    }
    __syncthreads();
    for (int t = tid; t < bk * bk; t += blockDim.x) {
      const int i = t / bk, j = t % bk;
      if (i == k)
        Minv[t] = rowk[j];
      else if (j == k)
        Minv[t] = -colk[i] * rowk[k];
      else
        Minv[t] -= colk[i] * rowk[j];
    }
    __syncthreads();
  }
}

// dst[i][j] = scale * src[i][j] for a rows x cols block (row-major, leading
// dimensions lds / ldd).
__global__ void k_copy_block(const double *__restrict__ src, int64_t lds, double *__restrict__ dst,
                             int64_t ldd, int rows, int cols, double scale) {
  const int64_t tot = int64_t(rows) * cols;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < tot;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = t / cols, j = t % cols;
    dst[i * ldd + j] = scale * src[i * lds + j];
  }
}

__global__ void k_fill(double *x, int64_t n, double v) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    x[i] = v;
}

template <int DIM, typename ST>
__global__ void k_sym_stencil(const double *__restrict__ soa, int64_t npts, ST *__restrict__ out) {
  constexpr int NS = DIM == 3 ? 27 : 9, C = NS / 2, W = rec_width<DIM, ST>();
  constexpr bool kFull = sizeof(ST) == 4;  // float records hold every slot
  for (int64_t g = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; g < npts;
       g += int64_t(gridDim.x) * blockDim.x)
    for (int j = 0; j < W; ++j) {
      const int slot = kFull ? j : C + j;
      out[g * W + j] = slot < NS ? ST(soa[int64_t(slot) * npts + g]) : ST(0);
    }
}

__global__ void k_to_float(const double *__restrict__ s, float *__restrict__ d, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    d[i] = float(s[i]);
}

inline int grid_for(int64_t n, int bs) {
  int64_t g = (n + bs - 1) / bs;
  return int(g > 65536 ? 65536 : (g < 1 ? 1 : g));
}

}  // namespace

hipError_t launch_node_coords(const MeshDims &md, const double *verts, const double *gllx,
                              double *coords, hipStream_t st) {
  const int64_t np = int64_t(md.ng[0]) * md.ng[1] * md.ng[2];
  if (md.dim == 3)
    k_node_coords<3><<<grid_for(np, 256), 256, 0, st>>>(md, verts, gllx, coords);
  else
    k_node_coords<2><<<grid_for(np, 256), 256, 0, st>>>(md, verts, gllx, coords);
  return hipGetLastError();
}

hipError_t launch_geom_cg(const MeshDims &md, const double *verts, const double *gllx,
                          const double *gllw, const double *coef, double *G, double *wdet, int *bad,
                          hipStream_t st) {
  const int Q = md.p + 1;
  const int64_t nel = int64_t(md.n[0]) * md.n[1] * (md.dim == 3 ? md.n[2] : 1);
  const int64_t tot = nel * (md.dim == 3 ? Q * Q * Q : Q * Q);
  if (md.dim == 3)
    k_geom<3><<<grid_for(tot, 256), 256, 0, st>>>(md, verts, gllx, gllw, coef, G, wdet, bad);
  else
    k_geom<2><<<grid_for(tot, 256), 256, 0, st>>>(md, verts, gllx, gllw, coef, G, wdet, bad);
  return hipGetLastError();
}

hipError_t launch_geom_nodal(const MeshDims &md, const double *coords, const double *D,
                             const double *gllw, const double *coef, double *G, double *wdet, int *bad,
                             hipStream_t st) {
  const int Q = md.p + 1;
  const int64_t nel = int64_t(md.n[0]) * md.n[1] * (md.dim == 3 ? md.n[2] : 1);
  const int64_t tot = nel * (md.dim == 3 ? Q * Q * Q : Q * Q);
  if (md.dim == 3)
    k_geom_nodal<3><<<grid_for(tot, 256), 256, 0, st>>>(md, coords, D, gllw, coef, G, wdet, bad);
  else
    k_geom_nodal<2><<<grid_for(tot, 256), 256, 0, st>>>(md, coords, D, gllw, coef, G, wdet, bad);
  return hipGetLastError();
}

hipError_t launch_dg_coords(const MeshDims &md, const double *verts, const double *gllx,
                            double *coords, hipStream_t st) {
  const int Q = md.p + 1;
  const int64_t n = int64_t(md.n[0]) * md.n[1] * md.n[2] * (md.dim == 3 ? Q * Q * Q : Q * Q);
  if (md.dim == 3)
    k_dg_coords<3><<<grid_for(n, 256), 256, 0, st>>>(md, verts, gllx, coords);
  else
    k_dg_coords<2><<<grid_for(n, 256), 256, 0, st>>>(md, verts, gllx, coords);
  return hipGetLastError();
}

hipError_t launch_lor_stencil(const MeshDims &md, int s, const int *kept_fine_idx,
                              const double *fine_coords, double g0, double g1, const double *coef,
                              double *stencil, hipStream_t st) {
  KeptIdx k{};
  for (int i = 0; i <= s; ++i) k.fine[i] = kept_fine_idx[i];
  const int64_t npts = int64_t(md.n[0] * s + 1) * (md.n[1] * s + 1) *
                       (md.dim == 3 ? md.n[2] * s + 1 : 1);
  if (md.dim == 3)
    k_lor_stencil<3><<<grid_for(npts, 128), 128, 0, st>>>(md, s, k, fine_coords, g0, g1, coef, stencil);
  else
    k_lor_stencil<2><<<grid_for(npts, 128), 128, 0, st>>>(md, s, k, fine_coords, g0, g1, coef, stencil);
  return hipGetLastError();
}

hipError_t launch_coarse_restrict(const MeshDims &md, const double *gllx, const double *r,
                                  double *rc, hipStream_t st) {
  const int nc = (md.n[0] - 1) * (md.n[1] - 1) * (md.dim == 3 ? md.n[2] - 1 : 1);
  if (nc <= 0) return hipSuccess;
  const int nb = (nc + 3) / 4;
#define LOR_RESTRICT_P(PP)                                                              \
  case PP:                                                                              \
    if (md.dim == 3) k_coarse_restrict_p<3, PP><<<nb, 256, 0, st>>>(md, gllx, r, rc, nc); \
    else k_coarse_restrict_p<2, PP><<<nb, 256, 0, st>>>(md, gllx, r, rc, nc);             \
    return hipGetLastError();
  switch (md.p) {
    LOR_RESTRICT_P(1)
    LOR_RESTRICT_P(2)
    LOR_RESTRICT_P(3)
    LOR_RESTRICT_P(4)
    LOR_RESTRICT_P(5)
    LOR_RESTRICT_P(6)
    LOR_RESTRICT_P(7)
    LOR_RESTRICT_P(8)
    default: break;
  }
#undef LOR_RESTRICT_P
  if (md.dim == 3)
    k_coarse_restrict<3><<<nb, 256, 0, st>>>(md, gllx, r, rc, nc);
  else
    k_coarse_restrict<2><<<nb, 256, 0, st>>>(md, gllx, r, rc, nc);
  return hipGetLastError();
}

hipError_t launch_coarse_prolong(const MeshDims &md, const double *gllx, const double *xc,
                                 double *z, const double *flag, hipStream_t st) {
  if (md.nu[2] > 65535) return hipErrorInvalidValue;  // grid z limit
  const dim3 grid((md.nu[0] + 63) / 64, (md.nu[1] + 3) / 4, md.dim == 3 ? md.nu[2] : 1);
  if (md.dim == 3)
    k_coarse_prolong<3><<<grid, dim3(64, 4), 0, st>>>(md, gllx, xc, z, flag);
  else
    k_coarse_prolong<2><<<grid, dim3(64, 4), 0, st>>>(md, gllx, xc, z, flag);
  return hipGetLastError();
}

hipError_t launch_gemv(int n, const double *A, const double *x, double *y, const double *flag,
                       hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_gemv<double><<<(n + kGemvRows - 1) / kGemvRows, 64 * kGemvRows, 0, st>>>(n, A, x, y, flag);
  return hipGetLastError();
}

hipError_t launch_gemv_f32(int n, const float *A, const double *x, double *y, const double *flag,
                           hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_gemv<float><<<(n + kGemvRows - 1) / kGemvRows, 64 * kGemvRows, 0, st>>>(n, A, x, y, flag);
  return hipGetLastError();
}

hipError_t launch_small_inverse(const double *M, int ldm, double *Minv, int bk, int *bad,
                                hipStream_t st) {
  if (bk < 1 || bk > 128) return hipErrorInvalidValue;
  k_small_inverse<<<1, 1024, 0, st>>>(M, ldm, Minv, bk, bad);
  return hipGetLastError();
}

hipError_t launch_copy_block(const double *src, int64_t lds, double *dst, int64_t ldd, int rows,
                             int cols, double scale, hipStream_t st) {
  k_copy_block<<<grid_for(int64_t(rows) * cols, 256), 256, 0, st>>>(src, lds, dst, ldd, rows, cols,
                                                                   scale);
  return hipGetLastError();
}

hipError_t launch_to_float(const double *src, float *dst, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_to_float<<<grid_for(n, 256), 256, 0, st>>>(src, dst, n);
  return hipGetLastError();
}

hipError_t launch_sym_stencil(const double *soa, int64_t npts, int dim, void *out, bool f32,
                              hipStream_t st) {
  const int g = grid_for(npts, 256);
  if (dim == 3) {
    if (f32)
      k_sym_stencil<3, float><<<g, 256, 0, st>>>(soa, npts, static_cast<float *>(out));
    else
      k_sym_stencil<3, double><<<g, 256, 0, st>>>(soa, npts, static_cast<double *>(out));
  } else {
    if (f32)
      k_sym_stencil<2, float><<<g, 256, 0, st>>>(soa, npts, static_cast<float *>(out));
    else
      k_sym_stencil<2, double><<<g, 256, 0, st>>>(soa, npts, static_cast<double *>(out));
  }
  return hipGetLastError();
}

hipError_t launch_fill(double *x, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_fill<<<grid_for(n, 256), 256, 0, st>>>(x, n, v);
  return hipGetLastError();
}

}  // namespace lor

// Discontinuous Galerkin parts of the path (Section 2, eq. ip and eq. br2;
// Section 3.5, eq. dg-as):
//   * face geometry and penalties, once at set-up;
//   * the face kernel of the matrix-free IP / BR2 operator;
//   * the diagonal of A_DG for the point-Jacobi part of the DG
//     preconditioner;
//   * E-vector <-> conforming L-vector transfers (E^T and E) fused with the
//     Jacobi step, and the collocated DG right-hand side.
//
// Faces.  Faces normal to direction s (s = 0, 1, 2 in turn) form a structured
// grid of shape n + e_s, lexicographic with x fastest.  Face f touches the
// "minus" element f - e_s (the face is its xi_s = 1 side) when f_s > 0 and the
// "plus" element f (its xi_s = 0 side) when f_s < n_s.  Face nodes are the
// element GLL nodes of that side, indexed by the tangential directions in
// increasing order (x fastest).
//
// The symmetric interior penalty form on one face,
//   -<{du/dn}, [v]> - <[u], {dv/dn}> + <sigma [u], [v]>,
// is split per face node q (weight omega_q = surface quadrature weight) into
//   value term   V_q = omega_q (sigma_q [u]_q - {du/dn}_q), added to the node
//                of each side with the sign of that side in [v], and
//   flux term    C_q a_q with C_q = -c omega_q [u]_q, a_q = J^-1 n on each
//                side, which the element kernel adds to the reference-space
//                flux G grad_xi u at the face node before the transposed
//                derivative contractions (c = 1/2 inside, 1 on the boundary).
// n is the unit normal of the minus element (the element's own outward normal
// on the boundary), so [u] = u^- - u^+ and {du/dn} = (a^- . grad_xi u^- +
// a^+ . grad_xi u^+) / 2 inside; on a (Dirichlet) boundary face [u] = u and
// {du/dn} = a . grad_xi u.
#include <hip/hip_runtime.h>

#include "lor_internal.h"

namespace lor {

namespace {

// Face f of global face index `face`: its direction s and multi-index f.
__device__ inline void face_decode(const MeshDims &md, int64_t face, int &s, int f[3]) {
  for (s = 0; s < 3; ++s) {
    int sh[3] = {md.n[0], md.n[1], md.n[2]};
    sh[s] += 1;
    const int64_t cnt = int64_t(sh[0]) * sh[1] * sh[2];
    if (face < cnt || s == md.dim - 1) {
      f[0] = int(face % sh[0]);
      f[1] = int((face / sh[0]) % sh[1]);
      f[2] = int(face / (int64_t(sh[0]) * sh[1]));
      return;
    }
    face -= cnt;
  }
}

__device__ inline int64_t elem_index(const MeshDims &md, const int e[3]) {
  return int64_t(e[0]) + int64_t(md.n[0]) * (int64_t(e[1]) + int64_t(md.n[1]) * e[2]);
}

// Jacobian of the Q1 map of element e at reference point xi: adj = det J^-1
// (the adjugate) and det.
template <int DIM>
__device__ void q1_jacobian(const double *verts, const MeshDims &md, const int e[3],
                            const double xi[3], double A[3][3], double &det) {
  const int nv0 = md.n[0] + 1, nv1 = md.n[1] + 1;
  double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double om[3];
  for (int i = 0; i < DIM; ++i) om[i] = 1.0 - xi[i];
  for (int c = 0; c < (1 << DIM); ++c) {
    const int b[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
    const int64_t vi = int64_t(e[0] + b[0]) +
                       int64_t(nv0) * (int64_t(e[1] + b[1]) + int64_t(nv1) * (DIM == 3 ? e[2] + b[2] : 0));
    for (int s = 0; s < DIM; ++s) {
      double g = b[s] ? 1.0 : -1.0;
      for (int i = 0; i < DIM; ++i)
        if (i != s) g *= b[i] ? xi[i] : om[i];
      for (int r = 0; r < DIM; ++r) J[r][s] += verts[vi * DIM + r] * g;
    }
  }
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
}

// Tangential directions of faces normal to s, in increasing order.
template <int DIM>
__device__ inline void face_local(int s, int q, int Q, int l[3]) {
  l[0] = l[1] = l[2] = 0;
  int t = 0;
  for (int d = 0; d < DIM; ++d) {
    if (d == s) continue;
    l[d] = t == 0 ? q % Q : q / Q;
    ++t;
  }
}

__device__ inline double block_sum64(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = 32; h > 0; h >>= 1) {
    if (int(threadIdx.x) < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Face geometry and penalty, one 64-thread block per face.  Output record
// (SoA per face, QF nodes): omega, sigma, a^-(3), a^+(3); a side that does
// not exist has a = 0.  IP: sigma = eta p^2 / h_e, h_e = min |K| / |e|
// (eq. ip), |K| = sum of w|J| over the element, |e| = sum of omega.  BR2
// (eq. br2 with the collocated lifting): sigma_q = eta c^2 sum_K
// omega_q / (w|J|)_q^K.  Pure Neumann meshes have no boundary faces: their
// records are zero.
template <int DIM>
__global__ __launch_bounds__(64) void k_dg_face_geom(MeshDims md, const double *__restrict__ verts,
                                                     const double *__restrict__ gllx,
                                                     const double *__restrict__ gllw,
                                                     const double *__restrict__ wdet, int method,
                                                     double eta, double *__restrict__ fg) {
  __shared__ double red[64];
  const int64_t face = blockIdx.x;
  int s, f[3];
  face_decode(md, face, s, f);
  const int Q = md.p + 1, p = md.p;
  const int QF = DIM == 3 ? Q * Q : Q;
  const int NQ = DIM == 3 ? Q * Q * Q : Q * Q;
  const bool hasm = f[s] > 0, hasp = f[s] < md.n[s];
  int em[3] = {f[0], f[1], f[2]};
  em[s] -= 1;
  const int64_t eim = hasm ? elem_index(md, em) : 0, eip = hasp ? elem_index(md, f) : 0;
  const bool bnd = !(hasm && hasp);
  double *out = fg + face * 8 * QF;
  if (bnd && !md.dirichlet) {
    for (int i = threadIdx.x; i < 8 * QF; i += 64) out[i] = 0.0;
    return;
  }
  double vm = 0.0, vp = 0.0;
  if (method == LOR_IP) {
    for (int i = threadIdx.x; i < NQ; i += 64) {
      if (hasm) vm += wdet[eim * NQ + i];
      if (hasp) vp += wdet[eip * NQ + i];
    }
    vm = block_sum64(vm, red);
    vp = block_sum64(vp, red);
  }
  double osum = 0.0;
  for (int q = threadIdx.x; q < QF; q += 64) {
    int l[3];
    face_local<DIM>(s, q, Q, l);
    double xi[3] = {gllx[l[0]], gllx[l[1]], gllx[l[2]]};
    xi[s] = hasm ? 1.0 : 0.0;
    double A[3][3], det;
    q1_jacobian<DIM>(verts, md, hasm ? em : f, xi, A, det);
    double area2 = 0.0;
    for (int r = 0; r < DIM; ++r) area2 += A[s][r] * A[s][r];
    double wt = 1.0;
    for (int d = 0; d < DIM; ++d)
      if (d != s) wt *= gllw[l[d]];
    osum += wt * sqrt(area2);
  }
  osum = block_sum64(osum, red);
  for (int q = threadIdx.x; q < QF; q += 64) {
    int l[3];
    face_local<DIM>(s, q, Q, l);
    double xi[3] = {gllx[l[0]], gllx[l[1]], gllx[l[2]]};
    double nrm[3] = {0, 0, 0}, omega = 0.0, am[3] = {0, 0, 0}, ap[3] = {0, 0, 0};
    double wm = 0.0, wp = 0.0;  // w|J| of the face node in each element
    for (int side = 0; side < 2; ++side) {
      if ((side == 0 && !hasm) || (side == 1 && !hasp)) continue;
      xi[s] = side == 0 ? 1.0 : 0.0;
      double A[3][3], det;
      q1_jacobian<DIM>(verts, md, side == 0 ? em : f, xi, A, det);
      const bool ref = side == 0 || !hasm;  // the side that defines n and omega
      if (ref) {
        const double sg = side == 0 ? 1.0 : -1.0;
        double area2 = 0.0;
        for (int r = 0; r < DIM; ++r) area2 += A[s][r] * A[s][r];
        const double area = sqrt(area2);
        for (int r = 0; r < DIM; ++r) nrm[r] = sg * A[s][r] / area;
        double wt = 1.0;
        for (int d = 0; d < DIM; ++d)
          if (d != s) wt *= gllw[l[d]];
        omega = wt * area;
      }
      double *a = side == 0 ? am : ap;
      for (int r = 0; r < DIM; ++r) {
        double acc = 0.0;
        for (int c = 0; c < DIM; ++c) acc += A[r][c] * nrm[c];
        a[r] = acc / det;
      }
      int ll[3] = {l[0], l[1], l[2]};
      ll[s] = side == 0 ? p : 0;
      const int loc = ll[0] + Q * (ll[1] + Q * ll[2]);
      (side == 0 ? wm : wp) = wdet[(side == 0 ? eim : eip) * NQ + loc];
    }
    double sigma;
    if (method == LOR_IP) {
      const double vol = bnd ? (hasm ? vm : vp) : fmin(vm, vp);
      sigma = eta * double(p) * double(p) * osum / vol;
    } else {
      const double c = bnd ? 1.0 : 0.5;
      double acc = 0.0;
      if (hasm) acc += omega / wm;
      if (hasp) acc += omega / wp;
      sigma = eta * c * c * acc;
    }
    out[0 * QF + q] = omega;
    out[1 * QF + q] = sigma;
    for (int r = 0; r < 3; ++r) {
      out[(2 + r) * QF + q] = am[r];
      out[(5 + r) * QF + q] = ap[r];
    }
  }
}

constexpr int face_fpb(int nq) {
  return 49152 / (16 * nq) >= 4 ? 4 : (49152 / (16 * nq) >= 1 ? 49152 / (16 * nq) : 1);
}

// Face kernel of A_DG: one 64-lane wave per face.  Both elements are staged
// in LDS (coalesced), then each lane takes face nodes: traces u^-, u^+ and the
// reference gradients on both sides, the jump and the averaged normal
// derivative, and writes the value and flux terms of each side (SoA per face
// and side: V, C a_0, C a_1, C a_2).
template <int DIM, int Q>
__global__ __launch_bounds__(256) void k_dg_face(MeshDims md, const double *__restrict__ Dg,
                                                 const double *__restrict__ fg,
                                                 const double *__restrict__ x,
                                                 double *__restrict__ fo, int64_t nfaces,
                                                 const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;
  constexpr int NQ = DIM == 3 ? Q * Q * Q : Q * Q;
  constexpr int QF = DIM == 3 ? Q * Q : Q;
  constexpr int FPB = face_fpb(NQ);
  __shared__ double sD[Q * Q];
  __shared__ double sx[FPB][2][NQ];
  const int tid = threadIdx.x, lf = tid / 64, lane = tid % 64;
  for (int i = tid; i < Q * Q; i += FPB * 64) sD[i] = Dg[i];
  const int64_t face = int64_t(blockIdx.x) * FPB + lf;
  const bool active = face < nfaces;
  int s = 0, f[3] = {0, 0, 0};
  if (active) face_decode(md, face, s, f);
  const bool hasm = active && f[s] > 0, hasp = active && f[s] < md.n[s];
  int em[3] = {f[0], f[1], f[2]};
  em[s] -= 1;
  const int64_t eim = hasm ? elem_index(md, em) : 0, eip = hasp ? elem_index(md, f) : 0;
  for (int i = lane; i < NQ; i += 64) {
    sx[lf][0][i] = hasm ? x[eim * NQ + i] : 0.0;
    sx[lf][1][i] = hasp ? x[eip * NQ + i] : 0.0;
  }
  __syncthreads();
  if (!active) return;
  const int p = Q - 1;
  const double *g = fg + face * 8 * QF;
  double *o0 = fo + (face * 2 + 0) * 4 * QF;
  double *o1 = fo + (face * 2 + 1) * 4 * QF;
  for (int q = lane; q < QF; q += 64) {
    int l[3];
    face_local<DIM>(s, q, Q, l);
    const double omega = g[q], sigma = g[QF + q];
    double am[3] = {0, 0, 0}, ap[3] = {0, 0, 0};
    for (int r = 0; r < DIM; ++r) {
      am[r] = g[(2 + r) * QF + q];
      ap[r] = g[(5 + r) * QF + q];
    }
    // traces and normal derivatives on both sides
    double u[2], dn[2];
    for (int side = 0; side < 2; ++side) {
      int ll[3] = {l[0], l[1], l[2]};
      ll[s] = side == 0 ? p : 0;
      const int loc = ll[0] + Q * (ll[1] + Q * ll[2]);
      const double *X = sx[lf][side];
      u[side] = X[loc];
      const double *a = side == 0 ? am : ap;
      double d = 0.0;
#pragma unroll
      for (int r = 0; r < DIM; ++r) {
        const int stride = r == 0 ? 1 : (r == 1 ? Q : Q * Q);
        const int base = loc - ll[r] * stride;
        double gr = 0.0;
#pragma unroll
        for (int k = 0; k < Q; ++k) gr += sD[ll[r] * Q + k] * X[base + k * stride];
        d += a[r] * gr;
      }
      dn[side] = d;
    }
    double V0 = 0.0, C0 = 0.0, V1 = 0.0, C1 = 0.0;
    if (hasm && hasp) {
      const double jump = u[0] - u[1];
      const double avg = 0.5 * (dn[0] + dn[1]);
      V0 = omega * (sigma * jump - avg);
      V1 = -V0;
      C0 = C1 = -0.5 * omega * jump;
    } else if (hasm) {
      V0 = omega * (sigma * u[0] - dn[0]);
      C0 = -omega * u[0];
    } else {
      V1 = omega * (sigma * u[1] - dn[1]);
      C1 = -omega * u[1];
    }
    o0[q] = V0;
    o1[q] = V1;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      o0[(1 + r) * QF + q] = C0 * am[r];
      o1[(1 + r) * QF + q] = C1 * ap[r];
    }
  }
}

// diag(A_DG) on the element-boundary nodes (some local index 0 or p), stored
// as its inverse; zero on element-interior nodes, which the point-Jacobi part
// of eq. dg-as does not touch.  Volume part: sum over the GLL nodes n on the
// lines through m of grad phi_m(n)^T G(n) grad phi_m(n).  Face part, for each
// face of the element through m: omega (sigma - a . grad phi_m) on the minus
// side, omega (sigma + a . grad phi_m) on the plus side (a taken along the
// minus normal), omega (sigma - 2 a . grad phi_m) on a boundary face.
template <int DIM>
__global__ void k_dg_diag(MeshDims md, const double *__restrict__ G, const double *__restrict__ Dg,
                          const double *__restrict__ fg, double *__restrict__ dinv) {
  const int Q = md.p + 1, p = md.p;
  const int NQ = DIM == 3 ? Q * Q * Q : Q * Q;
  const int QF = DIM == 3 ? Q * Q : Q;
  const int ncomp = DIM == 3 ? 6 : 3;
  const int64_t nel = int64_t(md.n[0]) * md.n[1] * md.n[2];
  const int64_t off[3] = {0, int64_t(md.n[0] + 1) * md.n[1] * md.n[2],
                          int64_t(md.n[0] + 1) * md.n[1] * md.n[2] +
                              int64_t(md.n[0]) * (md.n[1] + 1) * md.n[2]};
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < nel * NQ;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t e = t / NQ;
    const int m = int(t % NQ);
    const int l[3] = {m % Q, (m / Q) % Q, DIM == 3 ? m / (Q * Q) : 0};
    bool onb = false;
    for (int d = 0; d < DIM; ++d) onb = onb || l[d] == 0 || l[d] == p;
    if (!onb) {
      dinv[t] = 0.0;
      continue;
    }
    const int ec[3] = {int(e % md.n[0]), int((e / md.n[0]) % md.n[1]),
                       int(e / (int64_t(md.n[0]) * md.n[1]))};
    const double *Ge = G + e * ncomp * NQ;
    auto gcomp = [&](int r, int c, int n) {
      int a = r < c ? r : c, b = r < c ? c : r;
      const int idx = DIM == 3 ? (a == 0 ? b : (a == 1 ? 2 + b : 5)) : a + b;
      return Ge[idx * NQ + n];
    };
    const int strides[3] = {1, Q, Q * Q};
    double gself[3] = {0, 0, 0};
    for (int r = 0; r < DIM; ++r) gself[r] = Dg[l[r] * Q + l[r]];
    double dsum = 0.0;
    // node m itself
    for (int r = 0; r < DIM; ++r)
      for (int c = 0; c < DIM; ++c) dsum += gself[r] * gcomp(r, c, m) * gself[c];
    // the other nodes on the line through m in direction r
    for (int r = 0; r < DIM; ++r)
      for (int k = 0; k < Q; ++k) {
        if (k == l[r]) continue;
        const int n = m + (k - l[r]) * strides[r];
        const double dk = Dg[k * Q + l[r]];
        dsum += dk * gcomp(r, r, n) * dk;
      }
    // faces through m
    for (int s = 0; s < DIM; ++s) {
      if (l[s] != 0 && l[s] != p) continue;
      for (int side = 0; side < 2; ++side) {
        if ((side == 0 && l[s] != p) || (side == 1 && l[s] != 0)) continue;
        int f[3] = {ec[0], ec[1], ec[2]};
        if (side == 0) f[s] += 1;
        int sh[3] = {md.n[0], md.n[1], md.n[2]};
        sh[s] += 1;
        const int64_t face = off[s] + f[0] + int64_t(sh[0]) * (f[1] + int64_t(sh[1]) * f[2]);
        int q = 0, t2 = 0;
        for (int d = 0; d < DIM; ++d) {
          if (d == s) continue;
          q += t2 == 0 ? l[d] : l[d] * Q;
          ++t2;
        }
        const double *g = fg + face * 8 * QF;
        const double omega = g[q], sigma = g[QF + q];
        double ag = 0.0;
        for (int r = 0; r < DIM; ++r) ag += g[(2 + 3 * side + r) * QF + q] * gself[r];
        const bool bnd = f[s] == 0 || f[s] == md.n[s];
        if (bnd)
          dsum += omega * (sigma - 2.0 * ag);
        else
          dsum += omega * (sigma + (side == 0 ? -ag : ag));
      }
    }
    dinv[t] = 1.0 / dsum;
  }
}

// r_L = E^T r_E: each conforming unknown sums its copies in the elements that
// share it (fixed element order).
template <int DIM>
__global__ void k_dg_restrict(MeshDims md, const double *__restrict__ rE, double *__restrict__ rL,
                              const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;
  const int Q = md.p + 1;
  const int NQ = DIM == 3 ? Q * Q * Q : Q * Q;
  const int ox = md.dirichlet ? 1 : 0;
  const int64_t N = int64_t(md.nu[0]) * md.nu[1] * md.nu[2];
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < N;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int g[3] = {int(i % md.nu[0]) + ox, int((i / md.nu[0]) % md.nu[1]) + ox,
                      DIM == 3 ? int(i / (int64_t(md.nu[0]) * md.nu[1])) + ox : 0};
    double acc = 0.0;
    for (int c = 0; c < (1 << DIM); ++c) {
      int e[3] = {0, 0, 0}, l[3] = {0, 0, 0};
      bool ok = true;
      for (int d = 0; d < DIM; ++d) {
        if (((c >> d) & 1) == 0) {
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
      acc += rE[elem_index(md, e) * NQ + l[0] + Q * (l[1] + Q * l[2])];
    }
    rL[i] = acc;
  }
}

// z_E = D_B^-1 r_E + E z_L: point Jacobi on element-boundary nodes plus the
// conforming correction copied to every element copy of a node (zero on the
// Dirichlet boundary).
template <int DIM>
__global__ void k_dg_prolong_jacobi(MeshDims md, const double *__restrict__ rE,
                                    const double *__restrict__ dinv,
                                    const double *__restrict__ zL, double *__restrict__ zE,
                                    const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;
  const int Q = md.p + 1;
  const int NQ = DIM == 3 ? Q * Q * Q : Q * Q;
  const int ox = md.dirichlet ? 1 : 0;
  const int64_t nel = int64_t(md.n[0]) * md.n[1] * md.n[2];
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < nel * NQ;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t e = t / NQ;
    const int m = int(t % NQ);
    const int l[3] = {m % Q, (m / Q) % Q, DIM == 3 ? m / (Q * Q) : 0};
    const int ec[3] = {int(e % md.n[0]), int((e / md.n[0]) % md.n[1]),
                       int(e / (int64_t(md.n[0]) * md.n[1]))};
    bool in = true;
    int64_t li = 0, stride = 1;
    for (int d = 0; d < DIM; ++d) {
      const int gd = ec[d] * md.p + l[d];
      if (md.dirichlet && (gd == 0 || gd == md.ng[d] - 1)) in = false;
      li += int64_t(gd - ox) * stride;
      stride *= md.nu[d];
    }
    zE[t] = rE[t] * dinv[t] + (in ? zL[li] : 0.0);
  }
}

// b_E = (w|J|) f_E: the collocated element mass (layout of w|J| is the
// E-vector layout).
__global__ void k_dg_rhs(const double *__restrict__ wdet, const double *__restrict__ f,
                         double *__restrict__ b, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    b[i] = wdet[i] * f[i];
}

inline int grid_for(int64_t n, int bs) {
  int64_t g = (n + bs - 1) / bs;
  return int(g > 65536 ? 65536 : (g < 1 ? 1 : g));
}

template <int DIM, int Q>
hipError_t face_q(const MeshDims &md, const double *D, const double *fg, const double *x,
                  double *fo, int64_t nfaces, const double *flag, hipStream_t st) {
  constexpr int NQ = DIM == 3 ? Q * Q * Q : Q * Q;
  constexpr int FPB = face_fpb(NQ);
  const int nb = int((nfaces + FPB - 1) / FPB);
  k_dg_face<DIM, Q><<<nb, 64 * FPB, 0, st>>>(md, D, fg, x, fo, nfaces, flag);
  return hipGetLastError();
}

template <int DIM>
hipError_t face_dim(const MeshDims &md, const double *D, const double *fg, const double *x,
                    double *fo, int64_t nfaces, const double *flag, hipStream_t st) {
  switch (md.p + 1) {
    case 2: return face_q<DIM, 2>(md, D, fg, x, fo, nfaces, flag, st);
    case 3: return face_q<DIM, 3>(md, D, fg, x, fo, nfaces, flag, st);
    case 4: return face_q<DIM, 4>(md, D, fg, x, fo, nfaces, flag, st);
    case 5: return face_q<DIM, 5>(md, D, fg, x, fo, nfaces, flag, st);
    case 6: return face_q<DIM, 6>(md, D, fg, x, fo, nfaces, flag, st);
    case 7: return face_q<DIM, 7>(md, D, fg, x, fo, nfaces, flag, st);
    case 8: return face_q<DIM, 8>(md, D, fg, x, fo, nfaces, flag, st);
    case 9: return face_q<DIM, 9>(md, D, fg, x, fo, nfaces, flag, st);
    case 10: return face_q<DIM, 10>(md, D, fg, x, fo, nfaces, flag, st);
    case 11: return face_q<DIM, 11>(md, D, fg, x, fo, nfaces, flag, st);
    case 12: return face_q<DIM, 12>(md, D, fg, x, fo, nfaces, flag, st);
    case 13: return face_q<DIM, 13>(md, D, fg, x, fo, nfaces, flag, st);
    case 14: return face_q<DIM, 14>(md, D, fg, x, fo, nfaces, flag, st);
    case 15: return face_q<DIM, 15>(md, D, fg, x, fo, nfaces, flag, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int64_t dg_face_count(const MeshDims &md) {
  int64_t tot = 0;
  for (int s = 0; s < md.dim; ++s) {
    int64_t c = 1;
    for (int d = 0; d < 3; ++d) c *= md.n[d] + (d == s ? 1 : 0);
    tot += c;
  }
  return tot;
}

hipError_t launch_dg_face_geom(const MeshDims &md, const double *verts, const double *gllx,
                               const double *gllw, const double *wdet, int method, double eta,
                               double *fg, hipStream_t st) {
  const int64_t nf = dg_face_count(md);
  if (md.dim == 3)
    k_dg_face_geom<3><<<int(nf), 64, 0, st>>>(md, verts, gllx, gllw, wdet, method, eta, fg);
  else
    k_dg_face_geom<2><<<int(nf), 64, 0, st>>>(md, verts, gllx, gllw, wdet, method, eta, fg);
  return hipGetLastError();
}

hipError_t launch_dg_face(const MeshDims &md, const double *D, const double *fg, const double *x,
                          double *fo, const double *flag, hipStream_t st) {
  const int64_t nf = dg_face_count(md);
  return md.dim == 3 ? face_dim<3>(md, D, fg, x, fo, nf, flag, st)
                     : face_dim<2>(md, D, fg, x, fo, nf, flag, st);
}

hipError_t launch_dg_diag(const MeshDims &md, const double *G, const double *D, const double *fg,
                          double *dinv, hipStream_t st) {
  const int Q = md.p + 1;
  const int64_t n = int64_t(md.n[0]) * md.n[1] * md.n[2] * (md.dim == 3 ? Q * Q * Q : Q * Q);
  if (md.dim == 3)
    k_dg_diag<3><<<grid_for(n, 256), 256, 0, st>>>(md, G, D, fg, dinv);
  else
    k_dg_diag<2><<<grid_for(n, 256), 256, 0, st>>>(md, G, D, fg, dinv);
  return hipGetLastError();
}

hipError_t launch_dg_restrict(const MeshDims &md, const double *rE, double *rL, const double *flag,
                              hipStream_t st) {
  const int64_t N = int64_t(md.nu[0]) * md.nu[1] * md.nu[2];
  if (md.dim == 3)
    k_dg_restrict<3><<<grid_for(N, 256), 256, 0, st>>>(md, rE, rL, flag);
  else
    k_dg_restrict<2><<<grid_for(N, 256), 256, 0, st>>>(md, rE, rL, flag);
  return hipGetLastError();
}

hipError_t launch_dg_prolong_jacobi(const MeshDims &md, const double *rE, const double *dinv,
                                    const double *zL, double *zE, const double *flag,
                                    hipStream_t st) {
  const int Q = md.p + 1;
  const int64_t n = int64_t(md.n[0]) * md.n[1] * md.n[2] * (md.dim == 3 ? Q * Q * Q : Q * Q);
  if (md.dim == 3)
    k_dg_prolong_jacobi<3><<<grid_for(n, 256), 256, 0, st>>>(md, rE, dinv, zL, zE, flag);
  else
    k_dg_prolong_jacobi<2><<<grid_for(n, 256), 256, 0, st>>>(md, rE, dinv, zL, zE, flag);
  return hipGetLastError();
}

hipError_t launch_dg_rhs(const double *wdet, const double *f, double *b, int64_t n,
                         hipStream_t st) {
  k_dg_rhs<<<grid_for(n, 256), 256, 0, st>>>(wdet, f, b, n);
  return hipGetLastError();
}

}  // namespace lor

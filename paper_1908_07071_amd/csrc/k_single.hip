// Kernels of the box-patch preconditioners: B(1) (Section 4.1: one patch,
// the whole domain), B(n) (n overlapping subdomains) and vertex patches
// enlarged for isotropic overlap (Section 4.5).  Each patch is a box of
// elements; its V-cycle is the element-structured one of Section 3.3 on the
// box's part of the LOR level grids, with IC(0) smoothing in the chosen
// order and the exact solve on its part of T_p (a dense inverse applied by
// the coarse GEMV).
//
// Every vector is the points strictly inside a patch's box on one level
// (x fastest); for B(1) at level 0 that is the L-vector itself.
// The triangular sweeps follow the dependency levels of the elimination
// order (rows of one level are independent): a run of small levels goes to
// one workgroup that walks through them with a barrier between levels; a
// level with many rows gets a launch of its own over the whole GPU.  A box
// with no such level runs its whole V-cycle in one workgroup (k_box_vcycle,
// built from the same per-row and per-point steps).
#include <hip/hip_runtime.h>

#include "box_vcycle.h"
#include "lor_internal.h"

namespace lor {

namespace {

struct BoxDims {
  int m0, m1, m2;
};

// neighbour of row i at stencil slot s (the caller knows it is in the box)
template <int DIM>
__device__ __forceinline__ int nb_index(int i, int s, BoxDims b) {
  const int dx = s % 3 - 1, dy = (s / 3) % 3 - 1, dz = DIM == 3 ? s / 9 - 1 : 0;
  return i + dx + b.m0 * (dy + b.m1 * dz);
}

// forward: x_i = b_i - sum_{earlier m} l_im x_m (x and b may alias);
// backward: x_i = x_i / d_i - sum_{later m} l_mi x_m (in place).
template <int DIM, bool FWD>
__device__ __forceinline__ void sweep_row(int i, const double *__restrict__ Lv,
                                          const double *__restrict__ invD, const int *__restrict__ mask,
                                          const double *b, double *x, BoxDims bd) {
  constexpr int NS = DIM == 3 ? 27 : 9;
  const unsigned mk = unsigned(mask[i]);
  double acc = FWD ? b[i] : x[i] * invD[i];
  const double *li = Lv + int64_t(i) * NS;
  // every slot's factor value and neighbour value is loaded unconditionally
  // (the row itself stands in for a neighbour outside the mask), so that all
  // loads of a row are in flight together; the mask then selects the terms
  double lv[NS], xv[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const bool on = (mk >> s) & 1u;
    lv[s] = li[s];
    xv[s] = x[on ? nb_index<DIM>(i, s, bd) : i];
  }
#pragma unroll
  for (int s = 0; s < NS; ++s)
    if ((mk >> s) & 1u) acc -= lv[s] * xv[s];
  x[i] = acc;
}

template <int DIM, bool FWD>
__global__ __launch_bounds__(1024) void k_sweep_block(const int *__restrict__ sched,
                                                      const int *__restrict__ lptr, int l0, int l1,
                                                      const double *__restrict__ Lv,
                                                      const double *__restrict__ invD,
                                                      const int *__restrict__ mask, const double *b,
                                                      double *x, BoxDims bd, const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;
  for (int t = 0; t < l1 - l0; ++t) {
    const int l = FWD ? l0 + t : l1 - 1 - t;
    for (int q = lptr[l] + int(threadIdx.x); q < lptr[l + 1]; q += blockDim.x)
      sweep_row<DIM, FWD>(sched[q], Lv, invD, mask, b, x, bd);
    __syncthreads();  // the next level reads this level's rows
  }
}

template <int DIM, bool FWD>
__global__ __launch_bounds__(256) void k_sweep_level(const int *__restrict__ sched, int q0, int q1,
                                                     const double *__restrict__ Lv,
                                                     const double *__restrict__ invD,
                                                     const int *__restrict__ mask, const double *b,
                                                     double *x, BoxDims bd, const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;
  const int q = q0 + int(blockIdx.x * blockDim.x + threadIdx.x);
  if (q < q1) sweep_row<DIM, FWD>(sched[q], Lv, invD, mask, b, x, bd);
}

// r = b - A x on the interior box; A from the slot-major level stencil over
// the whole level grid (lng points per direction, boundary points included)
template <int DIM>
__device__ __forceinline__ void residual_at(int64_t i, const double *__restrict__ stencil, int64_t npts,
                                            int lng0, int lng1, BoxDims lo, BoxDims bd,
                                            const double *__restrict__ b, const double *__restrict__ x,
                                            double *__restrict__ r) {
  constexpr int NS = DIM == 3 ? 27 : 9;
  const int ix = int(i % bd.m0), iy = int((i / bd.m0) % bd.m1), iz = int(i / (int64_t(bd.m0) * bd.m1));
  const int64_t g = (ix + lo.m0) + int64_t(lng0) * ((iy + lo.m1) + (DIM == 3 ? int64_t(lng1) * (iz + lo.m2) : 0));
  double acc = b[i];
  for (int s = 0; s < NS; ++s) {
    const int dx = s % 3 - 1, dy = (s / 3) % 3 - 1, dz = DIM == 3 ? s / 9 - 1 : 0;
    const int qx = ix + dx, qy = iy + dy, qz = iz + dz;
    if (qx < 0 || qx >= bd.m0 || qy < 0 || qy >= bd.m1 || (DIM == 3 && (qz < 0 || qz >= bd.m2)))
      continue;  // a Dirichlet boundary point: its value is zero
    acc -= stencil[s * npts + g] * x[qx + int64_t(bd.m0) * (qy + int64_t(bd.m1) * qz)];
  }
  r[i] = acc;
}

template <int DIM>
__global__ __launch_bounds__(256) void k_box_residual(const double *__restrict__ stencil, int64_t npts,
                                                      int lng0, int lng1, BoxDims lo, BoxDims bd,
                                                      const double *__restrict__ b,
                                                      const double *__restrict__ x,
                                                      double *__restrict__ r, const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;
  const int64_t n = int64_t(bd.m0) * bd.m1 * bd.m2;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    residual_at<DIM>(i, stencil, npts, lng0, lng1, lo, bd, b, x, r);
}

// x_f += sum over the 2^d parents of P_f,c xc_c (1D tables per direction:
// parent index in the coarse box or -1, and weight)
template <int DIM>
__device__ __forceinline__ void prolong_at(int64_t i, const SingleXfer &t, const double *__restrict__ xc,
                                           double *__restrict__ x) {
  const int f[3] = {int(i % t.mf[0]), int((i / t.mf[0]) % t.mf[1]), int(i / (int64_t(t.mf[0]) * t.mf[1]))};
  double acc = 0.0;
  for (int c = 0; c < (1 << DIM); ++c) {
    int64_t ci = 0, stride = 1;
    double w = 1.0;
    bool ok = true;
    for (int d = 0; d < DIM; ++d) {
      const int b = (c >> d) & 1;
      const int pc = t.pc[d][2 * f[d] + b];
      if (pc < 0) ok = false;
      w *= t.pw[d][2 * f[d] + b];
      ci += int64_t(pc) * stride;
      stride *= t.mc[d];
    }
    if (ok) acc += w * xc[ci];
  }
  x[i] += acc;
}

template <int DIM>
__global__ __launch_bounds__(256) void k_box_prolong(SingleXfer t, const double *__restrict__ xc,
                                                     double *__restrict__ x, const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;
  const int64_t n = int64_t(t.mf[0]) * t.mf[1] * t.mf[2];
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    prolong_at<DIM>(i, t, xc, x);
}

// rc_c = sum over the fine points f with P_f,c != 0 of P_f,c r_f (R[d]
// entries per coarse index and direction, f = -1 for unused entries)
template <int DIM>
__device__ __forceinline__ void restrict_at(int64_t i, const SingleXfer &t, const double *__restrict__ r,
                                            double *__restrict__ rc) {
  const int c[3] = {int(i % t.mc[0]), int((i / t.mc[0]) % t.mc[1]), int(i / (int64_t(t.mc[0]) * t.mc[1]))};
  const int R0 = t.R[0], R1 = DIM >= 2 ? t.R[1] : 1, R2 = DIM == 3 ? t.R[2] : 1;
  double acc = 0.0;
  for (int a2 = 0; a2 < R2; ++a2) {
    const int f2 = DIM == 3 ? t.rf[2][c[2] * R2 + a2] : 0;
    if (f2 < 0) continue;
    const double w2 = DIM == 3 ? t.rw[2][c[2] * R2 + a2] : 1.0;
    for (int a1 = 0; a1 < R1; ++a1) {
      const int f1 = t.rf[1][c[1] * R1 + a1];
      if (f1 < 0) continue;
      const double w12 = w2 * t.rw[1][c[1] * R1 + a1];
      for (int a0 = 0; a0 < R0; ++a0) {
        const int f0 = t.rf[0][c[0] * R0 + a0];
        if (f0 < 0) continue;
        acc += w12 * t.rw[0][c[0] * R0 + a0] * r[f0 + int64_t(t.mf[0]) * (f1 + int64_t(t.mf[1]) * f2)];
      }
    }
  }
  rc[i] = acc;
}

template <int DIM>
__global__ __launch_bounds__(256) void k_box_restrict(SingleXfer t, const double *__restrict__ r,
                                                      double *__restrict__ rc, const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;
  const int64_t n = int64_t(t.mc[0]) * t.mc[1] * t.mc[2];
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    restrict_at<DIM>(i, t, r, rc);
}

// level-0 box <-> L-vector (Dirichlet numbering: grid index minus one)
template <int DIM, bool SCATTER>
__device__ __forceinline__ void move_at(int64_t i, const MeshDims &md, BoxDims lo, BoxDims bd,
                                        const double *__restrict__ src, const double *__restrict__ w,
                                        double *__restrict__ dst) {
  const int ix = int(i % bd.m0), iy = int((i / bd.m0) % bd.m1), iz = int(i / (int64_t(bd.m0) * bd.m1));
  const int64_t u = (ix + lo.m0 - 1) +
                    int64_t(md.nu[0]) * ((iy + lo.m1 - 1) + (DIM == 3 ? int64_t(md.nu[1]) * (iz + lo.m2 - 1) : 0));
  if (SCATTER)  // one fused multiply-add with a weight, as k_box_add_points does it
    dst[u] = w ? __builtin_fma(w[u], src[i], dst[u]) : dst[u] + src[i];
  else
    dst[i] = src[u];
}

template <int DIM, bool SCATTER>
__global__ __launch_bounds__(256) void k_box_move(MeshDims md, BoxDims lo, BoxDims bd,
                                                  const double *__restrict__ src,
                                                  const double *__restrict__ w,
                                                  double *__restrict__ dst, const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;
  const int64_t n = int64_t(bd.m0) * bd.m1 * bd.m2;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    move_at<DIM, SCATTER>(i, md, lo, bd, src, w, dst);
}

__global__ void k_axpy1(double *__restrict__ x, const double *__restrict__ y, int64_t n,
                        const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    x[i] += y[i];
}

// One row of y = A x by one wavefront, in the summation order of the coarse
// GEMV kernel (column tiles of 2048, eight partial sums per lane, then a
// shuffle tree), so that both give the same bits; the sum is in lane 0.
__device__ __forceinline__ double gemv_row_wave(int n, const double *__restrict__ a,
                                                const double *__restrict__ x, int lane) {
  constexpr int kTile = 2048;
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int j0 = 0; j0 < n; j0 += kTile) {
    const int m = min(kTile, n - j0);
    const double *aj = a + j0, *xj = x + j0;
    int j = lane;
    for (; j + 448 < m; j += 512) {
      double av[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) av[q] = aj[j + 64 * q];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] += av[q] * xj[j + 64 * q];
    }
    for (; j < m; j += 64) acc[0] += aj[j] * xj[j];
  }
  double sum = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_down(sum, off, 64);
  return sum;
}

// both triangular sweeps' levels in turn, a barrier after each level
template <int DIM, bool FWD>
__device__ __forceinline__ void wg_sweep(const BoxLevelDesc &lv, const double *b, double *x) {
  const BoxDims bd{lv.m[0], lv.m[1], lv.m[2]};
  const int *mask = FWD ? lv.emask : lv.lmask;
  for (int t = 0; t < lv.depth; ++t) {
    const int l = FWD ? t : lv.depth - 1 - t;
    const int q1 = lv.lptr[l + 1];
    for (int q = lv.lptr[l] + int(threadIdx.x); q < q1; q += kBoxThreads)
      sweep_row<DIM, FWD>(lv.sched[q], lv.Lv, lv.invD, mask, b, x, bd);
    __syncthreads();
  }
}

// The V-cycle of one box per workgroup: the steps of the per-level launches
// (pre-smoothing from zero, residual, restriction down to the deepest level
// the box reaches, the exact solve there if it is T_p, then prolongation,
// residual and post-smoothing back up), a barrier between steps.
// LDS: the vector a sweep pair works on sits in LDS (one level's worth,
// g.lds_rows values), so that the neighbour reads of every dependency level
// are LDS reads; the arithmetic is the same.
template <int DIM, bool LDS>
__global__ __launch_bounds__(kBoxThreads) void k_box_vcycle(const BoxDesc *__restrict__ boxes,
                                                            const int *__restrict__ list, BoxGrid g,
                                                            MeshDims md, const double *__restrict__ r,
                                                            double *__restrict__ z, int direct,
                                                            double *__restrict__ work, const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;
  const BoxDesc &bx = boxes[list[blockIdx.x]];
  if (bx.lv[0].n <= 0) return;
  const int tid = int(threadIdx.x);
  auto X = [&](int k) { return work + bx.lv[k].vo; };
  auto B = [&](int k) { return work + bx.lv[k].vo + bx.lv[k].vl; };
  auto R = [&](int k) { return work + bx.lv[k].vo + 2 * bx.lv[k].vl; };
  const double *b0 = direct ? r : B(0);
  double *x0 = direct ? z : X(0);
  auto bvec = [&](int k) -> const double * { return k == 0 ? b0 : B(k); };
  auto xvec = [&](int k) { return k == 0 ? x0 : X(k); };
  int K = 0;  // deepest level: the next one is empty or there is none
  while (K < g.L - 1 && bx.lv[K + 1].n > 0) ++K;
  const int top = min(K, g.L - 2);  // deepest level with sweeps
  if (!direct) {
    const BoxLevelDesc &l0 = bx.lv[0];
    const BoxDims lo{l0.lo[0], l0.lo[1], l0.lo[2]}, bd{l0.m[0], l0.m[1], l0.m[2]};
    for (int64_t i = tid; i < l0.n; i += kBoxThreads) move_at<DIM, false>(i, md, lo, bd, r, nullptr, B(0));
    __syncthreads();
  }
  extern __shared__ double xs[];
  for (int k = 0; k <= top; ++k) {
    const BoxLevelDesc lv = bx.lv[k];
    const BoxDims lo{lv.lo[0], lv.lo[1], lv.lo[2]}, bd{lv.m[0], lv.m[1], lv.m[2]};
    const double *bk = bvec(k);
    double *xk = xvec(k), *rk = R(k);
    if constexpr (LDS) {
      wg_sweep<DIM, true>(lv, bk, xs);
      wg_sweep<DIM, false>(lv, xs, xs);
      for (int64_t i = tid; i < lv.n; i += kBoxThreads) {
        residual_at<DIM>(i, g.stencil[k], g.npts[k], g.lng[k][0], g.lng[k][1], lo, bd, bk, xs, rk);
        xk[i] = xs[i];
      }
    } else {
      wg_sweep<DIM, true>(lv, bk, xk);
      wg_sweep<DIM, false>(lv, xk, xk);
      for (int64_t i = tid; i < lv.n; i += kBoxThreads)
        residual_at<DIM>(i, g.stencil[k], g.npts[k], g.lng[k][0], g.lng[k][1], lo, bd, bk, xk, rk);
    }
    __syncthreads();
    if (k < K) {
      const int64_t nc = int64_t(lv.xf.mc[0]) * lv.xf.mc[1] * lv.xf.mc[2];
      for (int64_t i = tid; i < nc; i += kBoxThreads) restrict_at<DIM>(i, lv.xf, rk, B(k + 1));
      __syncthreads();
    }
  }
  if (K == g.L - 1) {  // the box's part of T_p, solved exactly
    const BoxLevelDesc &lc = bx.lv[K];
    const int n = lc.n, lane = tid & 63;
    const double *bk = bvec(K);
    double *xk = xvec(K);
    for (int row = tid >> 6; row < n; row += kBoxThreads / 64) {
      const double s = gemv_row_wave(n, lc.ainv + int64_t(row) * n, bk, lane);
      if (lane == 0) xk[row] = s;
    }
    __syncthreads();
  }
  for (int k = top; k >= 0; --k) {
    const BoxLevelDesc lv = bx.lv[k];
    const BoxDims lo{lv.lo[0], lv.lo[1], lv.lo[2]}, bd{lv.m[0], lv.m[1], lv.m[2]};
    const double *bk = bvec(k);
    double *xk = xvec(k), *rk = R(k);
    if (k < K) {
      const int64_t nf = int64_t(lv.xf.mf[0]) * lv.xf.mf[1] * lv.xf.mf[2];
      for (int64_t i = tid; i < nf; i += kBoxThreads) prolong_at<DIM>(i, lv.xf, X(k + 1), xk);
      __syncthreads();
      for (int64_t i = tid; i < lv.n; i += kBoxThreads)
        residual_at<DIM>(i, g.stencil[k], g.npts[k], g.lng[k][0], g.lng[k][1], lo, bd, bk, xk, rk);
      __syncthreads();
    }
    if constexpr (LDS) {
      for (int64_t i = tid; i < lv.n; i += kBoxThreads) xs[i] = rk[i];
      __syncthreads();
      wg_sweep<DIM, true>(lv, xs, xs);
      wg_sweep<DIM, false>(lv, xs, xs);
      for (int64_t i = tid; i < lv.n; i += kBoxThreads) xk[i] += xs[i];
    } else {
      wg_sweep<DIM, true>(lv, rk, rk);
      wg_sweep<DIM, false>(lv, rk, rk);
      for (int64_t i = tid; i < lv.n; i += kBoxThreads) xk[i] += rk[i];
    }
    // the next level up reads this level's x; in LDS mode the next level's
    // load into LDS must also wait for this level's last LDS reads
    if (k > 0) __syncthreads();
  }
}

// z += w x_0 on the level-0 box of each listed box, one workgroup per box
template <int DIM>
__global__ __launch_bounds__(kBoxThreads) void k_box_add(const BoxDesc *__restrict__ boxes,
                                                         const int *__restrict__ list, MeshDims md,
                                                         const double *__restrict__ w,
                                                         double *__restrict__ z,
                                                         const double *__restrict__ work,
                                                         const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;
  const BoxLevelDesc &l0 = boxes[list[blockIdx.x]].lv[0];
  const BoxDims lo{l0.lo[0], l0.lo[1], l0.lo[2]}, bd{l0.m[0], l0.m[1], l0.m[2]};
  const double *x0 = work + l0.vo;
  for (int64_t i = threadIdx.x; i < l0.n; i += kBoxThreads) move_at<DIM, true>(i, md, lo, bd, x0, w, z);
}

// z_u += w_u x over every one-workgroup box holding point u, one thread per
// point, the boxes in colour order (the order of the per-colour launches)
__global__ __launch_bounds__(256) void k_box_add_points(const int64_t *__restrict__ ptr,
                                                        const int64_t *__restrict__ pts,
                                                        const int64_t *__restrict__ src, int64_t npt,
                                                        const double *__restrict__ w,
                                                        double *__restrict__ z,
                                                        const double *__restrict__ work,
                                                        const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < npt;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t u = pts[t];
    double acc = z[u];
    if (w) {
      const double wu = w[u];
      for (int64_t e = ptr[t]; e < ptr[t + 1]; ++e) acc = __builtin_fma(wu, work[src[e]], acc);
    } else {
      for (int64_t e = ptr[t]; e < ptr[t + 1]; ++e) acc = acc + work[src[e]];
    }
    z[u] = acc;
  }
}

inline int blocks_for(int64_t n, int bs) {
  int64_t g = (n + bs - 1) / bs;
  return int(g > 4096 ? 4096 : (g < 1 ? 1 : g));
}

}  // namespace

hipError_t launch_single_sweep(int dim, bool fwd, const SingleLevelDev &lv, const double *b, double *x,
                               const double *flag, hipStream_t st) {
  const BoxDims bd{lv.m[0], lv.m[1], lv.m[2]};
  const int nseg = int(lv.segs.size());
  for (int k = 0; k < nseg; ++k) {
    const SingleSeg &sg = lv.segs[fwd ? k : nseg - 1 - k];
    if (sg.grid) {
      const int q0 = lv.lptr_host[sg.l0], q1 = lv.lptr_host[sg.l0 + 1];
      const int nb = (q1 - q0 + 255) / 256;
      if (dim == 3) {
        if (fwd) k_sweep_level<3, true><<<nb, 256, 0, st>>>(lv.sched, q0, q1, lv.Lv, lv.invD, lv.emask, b, x, bd, flag);
        else k_sweep_level<3, false><<<nb, 256, 0, st>>>(lv.sched, q0, q1, lv.Lv, lv.invD, lv.lmask, x, x, bd, flag);
      } else {
        if (fwd) k_sweep_level<2, true><<<nb, 256, 0, st>>>(lv.sched, q0, q1, lv.Lv, lv.invD, lv.emask, b, x, bd, flag);
        else k_sweep_level<2, false><<<nb, 256, 0, st>>>(lv.sched, q0, q1, lv.Lv, lv.invD, lv.lmask, x, x, bd, flag);
      }
    } else {
      if (dim == 3) {
        if (fwd) k_sweep_block<3, true><<<1, 1024, 0, st>>>(lv.sched, lv.lptr, sg.l0, sg.l1, lv.Lv, lv.invD, lv.emask, b, x, bd, flag);
        else k_sweep_block<3, false><<<1, 1024, 0, st>>>(lv.sched, lv.lptr, sg.l0, sg.l1, lv.Lv, lv.invD, lv.lmask, x, x, bd, flag);
      } else {
        if (fwd) k_sweep_block<2, true><<<1, 1024, 0, st>>>(lv.sched, lv.lptr, sg.l0, sg.l1, lv.Lv, lv.invD, lv.emask, b, x, bd, flag);
        else k_sweep_block<2, false><<<1, 1024, 0, st>>>(lv.sched, lv.lptr, sg.l0, sg.l1, lv.Lv, lv.invD, lv.lmask, x, x, bd, flag);
      }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_single_residual(int dim, const double *stencil, int64_t npts, const int *lng,
                                  const int *lo, const int *m, const double *b, const double *x,
                                  double *r, const double *flag, hipStream_t st) {
  const BoxDims bd{m[0], m[1], m[2]};
  const BoxDims bl{lo[0], lo[1], lo[2]};
  const int64_t n = int64_t(m[0]) * m[1] * m[2];
  if (n <= 0) return hipSuccess;
  if (dim == 3)
    k_box_residual<3><<<blocks_for(n, 256), 256, 0, st>>>(stencil, npts, lng[0], lng[1], bl, bd, b, x, r, flag);
  else
    k_box_residual<2><<<blocks_for(n, 256), 256, 0, st>>>(stencil, npts, lng[0], lng[1], bl, bd, b, x, r, flag);
  return hipGetLastError();
}

hipError_t launch_box_gather(int dim, const MeshDims &md, const int *lo, const int *m,
                             const double *r, double *out, const double *flag, hipStream_t st) {
  const BoxDims bd{m[0], m[1], m[2]}, bl{lo[0], lo[1], lo[2]};
  const int64_t n = int64_t(m[0]) * m[1] * m[2];
  if (n <= 0) return hipSuccess;
  if (dim == 3) k_box_move<3, false><<<blocks_for(n, 256), 256, 0, st>>>(md, bl, bd, r, nullptr, out, flag);
  else k_box_move<2, false><<<blocks_for(n, 256), 256, 0, st>>>(md, bl, bd, r, nullptr, out, flag);
  return hipGetLastError();
}

hipError_t launch_box_scatter(int dim, const MeshDims &md, const int *lo, const int *m,
                              const double *x, const double *w, double *z, const double *flag,
                              hipStream_t st) {
  const BoxDims bd{m[0], m[1], m[2]}, bl{lo[0], lo[1], lo[2]};
  const int64_t n = int64_t(m[0]) * m[1] * m[2];
  if (n <= 0) return hipSuccess;
  if (dim == 3) k_box_move<3, true><<<blocks_for(n, 256), 256, 0, st>>>(md, bl, bd, x, w, z, flag);
  else k_box_move<2, true><<<blocks_for(n, 256), 256, 0, st>>>(md, bl, bd, x, w, z, flag);
  return hipGetLastError();
}

hipError_t launch_single_transfer(int dim, bool prolong, const SingleXfer &t, const double *in,
                                  double *out, const double *flag, hipStream_t st) {
  const int64_t n = prolong ? int64_t(t.mf[0]) * t.mf[1] * t.mf[2] : int64_t(t.mc[0]) * t.mc[1] * t.mc[2];
  if (n <= 0) return hipSuccess;
  if (prolong) {
    if (dim == 3) k_box_prolong<3><<<blocks_for(n, 256), 256, 0, st>>>(t, in, out, flag);
    else k_box_prolong<2><<<blocks_for(n, 256), 256, 0, st>>>(t, in, out, flag);
  } else {
    if (dim == 3) k_box_restrict<3><<<blocks_for(n, 256), 256, 0, st>>>(t, in, out, flag);
    else k_box_restrict<2><<<blocks_for(n, 256), 256, 0, st>>>(t, in, out, flag);
  }
  return hipGetLastError();
}

hipError_t launch_box_vcycles(int dim, const BoxDesc *boxes, const int *list, int count,
                              const BoxGrid &g, const MeshDims &md, const double *r, double *z,
                              int direct, double *work, const double *flag, hipStream_t st) {
  if (count == 0) return hipSuccess;
  if ((dim != 2 && dim != 3) || count < 0 || g.L < 1 || g.L > kMaxLevels) return hipErrorInvalidValue;
  if (g.lds_rows > 0 && g.lds_rows <= kBoxLdsRows) {
    const size_t lds = size_t(g.lds_rows) * sizeof(double);
    if (dim == 3) k_box_vcycle<3, true><<<count, kBoxThreads, lds, st>>>(boxes, list, g, md, r, z, direct, work, flag);
    else k_box_vcycle<2, true><<<count, kBoxThreads, lds, st>>>(boxes, list, g, md, r, z, direct, work, flag);
  } else {
    if (dim == 3) k_box_vcycle<3, false><<<count, kBoxThreads, 0, st>>>(boxes, list, g, md, r, z, direct, work, flag);
    else k_box_vcycle<2, false><<<count, kBoxThreads, 0, st>>>(boxes, list, g, md, r, z, direct, work, flag);
  }
  return hipGetLastError();
}

hipError_t launch_box_add(int dim, const BoxDesc *boxes, const int *list, int count,
                          const MeshDims &md, const double *w, double *z, const double *work,
                          const double *flag, hipStream_t st) {
  if (count == 0) return hipSuccess;
  if ((dim != 2 && dim != 3) || count < 0) return hipErrorInvalidValue;
  if (dim == 3) k_box_add<3><<<count, kBoxThreads, 0, st>>>(boxes, list, md, w, z, work, flag);
  else k_box_add<2><<<count, kBoxThreads, 0, st>>>(boxes, list, md, w, z, work, flag);
  return hipGetLastError();
}

hipError_t launch_box_add_points(const int64_t *ptr, const int64_t *pts, const int64_t *src, int64_t npt,
                                 const double *w, double *z, const double *work, const double *flag,
                                 hipStream_t st) {
  if (npt <= 0) return hipSuccess;
  k_box_add_points<<<blocks_for(npt, 256), 256, 0, st>>>(ptr, pts, src, npt, w, z, work, flag);
  return hipGetLastError();
}

hipError_t launch_axpy1(double *x, const double *y, int64_t n, const double *flag, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_axpy1<<<blocks_for(n, 256), 256, 0, st>>>(x, y, n, flag);
  return hipGetLastError();
}

}  // namespace lor

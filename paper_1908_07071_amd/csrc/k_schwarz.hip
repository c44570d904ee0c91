// Vertex-patch additive Schwarz: one element-structured LOR V-cycle per patch
// (Sections 3.2-3.4), summed into z (eq. as).
//
// One workgroup (a single wavefront) per patch.  The patch vectors of every
// level live in LDS as zero-padded boxes, so stencil neighbours outside the
// patch (the patch Dirichlet boundary) read zeros without branches.  The
// ILU(0) sweeps follow the dependency levels of the MDF order computed at
// set-up: rows of one level are independent and spread over the lanes; the
// wavefront synchronises between levels.  Stencils come from the global level
// operators (patch matrices are their principal sub-matrices), factors from
// the per-patch blocks.  The corrections of overlapping patches are added
// with FP64 atomics.
#include <hip/hip_runtime.h>

#include "lor_internal.h"

namespace lor {

namespace {

template <int DIM>
struct Box {
  int m[3];    // unknowns per direction
  int mp[3];   // padded extents (m + 2)
  int lo[3];   // first level-grid index per direction
  int n;       // unknowns
  __device__ int pad(int i) const {
    const int ix = i % m[0], iy = (i / m[0]) % m[1], iz = DIM == 3 ? i / (m[0] * m[1]) : 0;
    return (ix + 1) + mp[0] * ((iy + 1) + mp[1] * (DIM == 3 ? iz + 1 : 0));
  }
  __device__ int padded_size() const { return mp[0] * mp[1] * (DIM == 3 ? mp[2] : 1); }
};

template <int DIM>
__device__ inline int64_t level_gidx(const Box<DIM> &bx, int i, const int *lng) {
  const int ix = i % bx.m[0], iy = (i / bx.m[0]) % bx.m[1],
            iz = DIM == 3 ? i / (bx.m[0] * bx.m[1]) : 0;
  return int64_t(bx.lo[0] + ix) +
         int64_t(lng[0]) * (int64_t(bx.lo[1] + iy) + (DIM == 3 ? int64_t(lng[1]) * (bx.lo[2] + iz) : 0));
}

template <int DIM>
__device__ inline int slot_off(int s, const int *mp) {
  const int ox = s % 3 - 1, oy = (s / 3) % 3 - 1, oz = DIM == 3 ? s / 9 - 1 : 0;
  return ox + mp[0] * (oy + mp[1] * oz);
}

// forward sweep  w_i = y_i - sum_{earlier m} l_im w_m   (in place)
template <int DIM>
__device__ void sweep_fwd(double *Y, const Box<DIM> &bx, const char *blk, int depth) {
  constexpr int NS = DIM == 3 ? 27 : 9;
  const int n = bx.n;
  const int *idx = reinterpret_cast<const int *>(blk);
  const int *lvl = idx + n;
  const int *msk = lvl + n + 1;
  const double *val = reinterpret_cast<const double *>(blk + factor_vals_offset(n));
  int off[NS];
  for (int s = 0; s < NS; ++s) off[s] = slot_off<DIM>(s, bx.mp);
  for (int d = 0; d < depth; ++d) {
    for (int t = lvl[d] + threadIdx.x; t < lvl[d + 1]; t += blockDim.x) {
      const int pi = bx.pad(idx[t]);
      const int mk = msk[t];
      double acc = Y[pi];
      for (int s = 0; s < NS; ++s)
        if ((mk >> s) & 1) acc -= val[int64_t(s) * n + t] * Y[pi + off[s]];
      Y[pi] = acc;
    }
    __syncthreads();
  }
}

// backward sweep  y_i = w_i / D_i - sum_{later m} l_mi y_m   (in place)
template <int DIM>
__device__ void sweep_bwd(double *Y, const Box<DIM> &bx, const char *blk, int depth) {
  constexpr int NS = DIM == 3 ? 27 : 9;
  constexpr int C = NS / 2;
  const int n = bx.n;
  const int *idx = reinterpret_cast<const int *>(blk);
  const int *lvl = idx + n;
  const int *msk = lvl + n + 1;
  const double *val = reinterpret_cast<const double *>(blk + factor_vals_offset(n));
  int off[NS];
  for (int s = 0; s < NS; ++s) off[s] = slot_off<DIM>(s, bx.mp);
  for (int d = depth - 1; d >= 0; --d) {
    for (int t = lvl[d] + threadIdx.x; t < lvl[d + 1]; t += blockDim.x) {
      const int pi = bx.pad(idx[t]);
      const int mk = msk[t];
      double acc = Y[pi] * val[int64_t(C) * n + t];
      for (int s = 0; s < NS; ++s)
        if (s != C && !((mk >> s) & 1)) acc -= val[int64_t(s) * n + t] * Y[pi + off[s]];
      Y[pi] = acc;
    }
    __syncthreads();
  }
}

// R = B - A X on one level (A from the global level stencil)
template <int DIM>
__device__ void residual(double *R, const double *B, const double *X, const Box<DIM> &bx,
                         const double *__restrict__ st, int64_t npts, const int *lng) {
  constexpr int NS = DIM == 3 ? 27 : 9;
  int off[NS];
  for (int s = 0; s < NS; ++s) off[s] = slot_off<DIM>(s, bx.mp);
  for (int i = threadIdx.x; i < bx.n; i += blockDim.x) {
    const int pi = bx.pad(i);
    const int64_t g = level_gidx<DIM>(bx, i, lng);
    double acc = B[pi];
    for (int s = 0; s < NS; ++s) acc -= st[int64_t(s) * npts + g] * X[pi + off[s]];
    R[pi] = acc;
  }
  __syncthreads();
}

template <int DIM>
__global__ __launch_bounds__(64) void k_patch_vcycle(PatchArgs pa, const double *__restrict__ r,
                                                     double *__restrict__ z, const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;
  extern __shared__ double lds[];
  const int j = blockIdx.x;
  const int L = pa.nlev;
  const MeshDims &md = pa.md;
  const int v[3] = {j % pa.nv[0], (j / pa.nv[0]) % pa.nv[1],
                    DIM == 3 ? j / (pa.nv[0] * pa.nv[1]) : 0};
  int typ[3] = {1, 1, 1};
  Box<DIM> bx[kMaxLevels];
  for (int k = 0; k < L; ++k) {
    const int s = pa.s[k];
    int n = 1;
    for (int d = 0; d < 3; ++d) {
      if (d >= DIM) {
        bx[k].m[d] = 1;
        bx[k].mp[d] = 1;
        bx[k].lo[d] = 0;
        continue;
      }
      const int nn = md.n[d];
      const int lo = v[d] > 0 ? (v[d] - 1) * s + 1 : 1;
      const int hi = v[d] < nn ? (v[d] + 1) * s - 1 : nn * s - 1;
      bx[k].lo[d] = lo;
      bx[k].m[d] = hi - lo + 1;
      bx[k].mp[d] = bx[k].m[d] + 2;
      n *= max(bx[k].m[d], 0);
    }
    bx[k].n = n;
  }
  for (int d = 0; d < DIM; ++d) typ[d] = v[d] == 0 ? 0 : (v[d] == md.n[d] ? 2 : 1);
  if (bx[0].n <= 0) return;

  for (int i = threadIdx.x; i < pa.lds_total; i += blockDim.x) lds[i] = 0.0;
  __syncthreads();
  double *X[kMaxLevels], *B[kMaxLevels], *R[kMaxLevels];
  for (int k = 0; k < L; ++k) {
    const int ps = bx[k].padded_size();
    X[k] = lds + pa.lds_offs[k];
    B[k] = X[k] + ps;
    R[k] = B[k] + ps;
  }
  // gather the residual of the patch unknowns (level 0 = GLL grid)
  const int ox = md.dirichlet ? 1 : 0;
  for (int i = threadIdx.x; i < bx[0].n; i += blockDim.x) {
    const int64_t g = level_gidx<DIM>(bx[0], i, md.ng);
    const int gx = int(g % md.ng[0]), gy = int((g / md.ng[0]) % md.ng[1]),
              gz = DIM == 3 ? int(g / (int64_t(md.ng[0]) * md.ng[1])) : 0;
    const int64_t li = int64_t(gx - ox) +
                       int64_t(md.nu[0]) * (int64_t(gy - ox) + (DIM == 3 ? int64_t(md.nu[1]) * (gz - ox) : 0));
    B[0][bx[0].pad(i)] = r[li];
  }
  __syncthreads();

  const int nf = L - 1;  // levels with smoothing
  const int64_t fbase = int64_t(j) * (nf > 0 ? nf : 1);
  // ---------------- down
  for (int k = 0; k < nf; ++k) {
    if (bx[k].n <= 0) break;
    const char *blk = pa.fac + pa.fac_off[fbase + k];
    const int depth = pa.depth[fbase + k];
    for (int i = threadIdx.x; i < bx[k].n; i += blockDim.x) {
      const int pi = bx[k].pad(i);
      X[k][pi] = B[k][pi];
    }
    __syncthreads();
    sweep_fwd<DIM>(X[k], bx[k], blk, depth);
    sweep_bwd<DIM>(X[k], bx[k], blk, depth);
    residual<DIM>(R[k], B[k], X[k], bx[k], pa.stencil[k], pa.npts[k], pa.lng[k]);
    // restriction B_{k+1} = P^T R_k
    if (bx[k + 1].n > 0) {
      const XferTab *tb[3];
      for (int d = 0; d < DIM; ++d) tb[d] = &pa.xfer[k * 3 + typ[d]];
      const Box<DIM> &cb = bx[k + 1];
      const Box<DIM> &fb = bx[k];
      for (int i = threadIdx.x; i < cb.n; i += blockDim.x) {
        const int ci[3] = {i % cb.m[0], (i / cb.m[0]) % cb.m[1], DIM == 3 ? i / (cb.m[0] * cb.m[1]) : 0};
        double acc = 0.0;
        const int nz = DIM == 3 ? tb[2]->rcnt[ci[2]] : 1;
        for (int cz = 0; cz < nz; ++cz) {
          const int fz = DIM == 3 ? tb[2]->rf[ci[2]][cz] : 0;
          const double wz = DIM == 3 ? tb[2]->rw[ci[2]][cz] : 1.0;
          for (int cy = 0; cy < tb[1]->rcnt[ci[1]]; ++cy) {
            const int fy = tb[1]->rf[ci[1]][cy];
            const double wy = tb[1]->rw[ci[1]][cy] * wz;
            for (int cx = 0; cx < tb[0]->rcnt[ci[0]]; ++cx) {
              const int fx = tb[0]->rf[ci[0]][cx];
              acc += tb[0]->rw[ci[0]][cx] * wy * R[k][fx + fb.mp[0] * (fy + fb.mp[1] * fz)];
            }
          }
        }
        B[k + 1][cb.pad(i)] = acc;
      }
      __syncthreads();
    }
  }
  // ---------------- coarsest level: exact (at most one unknown)
  {
    const int kc = L - 1;
    if (bx[kc].n == 1 && threadIdx.x == 0) {
      const int64_t g = level_gidx<DIM>(bx[kc], 0, pa.lng[kc]);
      constexpr int C = DIM == 3 ? 13 : 4;
      const int pi = bx[kc].pad(0);
      X[kc][pi] = B[kc][pi] / pa.stencil[kc][int64_t(C) * pa.npts[kc] + g];
    }
    __syncthreads();
  }
  // ---------------- up
  for (int k = nf - 1; k >= 0; --k) {
    if (bx[k].n <= 0) continue;
    const char *blk = pa.fac + pa.fac_off[fbase + k];
    const int depth = pa.depth[fbase + k];
    if (bx[k + 1].n > 0) {
      const XferTab *tb[3];
      for (int d = 0; d < DIM; ++d) tb[d] = &pa.xfer[k * 3 + typ[d]];
      const Box<DIM> &cb = bx[k + 1];
      const Box<DIM> &fb = bx[k];
      for (int i = threadIdx.x; i < fb.n; i += blockDim.x) {
        const int fi[3] = {i % fb.m[0], (i / fb.m[0]) % fb.m[1], DIM == 3 ? i / (fb.m[0] * fb.m[1]) : 0};
        double acc = 0.0;
        for (int bz = 0; bz < (DIM == 3 ? 2 : 1); ++bz) {
          const int cz = DIM == 3 ? tb[2]->pc[fi[2]][bz] : 0;
          const double wz = DIM == 3 ? tb[2]->pw[fi[2]][bz] : 1.0;
          for (int by = 0; by < 2; ++by) {
            const int cy = tb[1]->pc[fi[1]][by];
            const double wy = tb[1]->pw[fi[1]][by] * wz;
            for (int bxx = 0; bxx < 2; ++bxx) {
              const int cx = tb[0]->pc[fi[0]][bxx];
              acc += tb[0]->pw[fi[0]][bxx] * wy * X[k + 1][cx + cb.mp[0] * (cy + cb.mp[1] * cz)];
            }
          }
        }
        X[k][fb.pad(i)] += acc;
      }
      __syncthreads();
    }
    residual<DIM>(R[k], B[k], X[k], bx[k], pa.stencil[k], pa.npts[k], pa.lng[k]);
    sweep_fwd<DIM>(R[k], bx[k], blk, depth);
    sweep_bwd<DIM>(R[k], bx[k], blk, depth);
    for (int i = threadIdx.x; i < bx[k].n; i += blockDim.x) {
      const int pi = bx[k].pad(i);
      X[k][pi] += R[k][pi];
    }
    __syncthreads();
  }
  // scatter-add the correction
  for (int i = threadIdx.x; i < bx[0].n; i += blockDim.x) {
    const int64_t g = level_gidx<DIM>(bx[0], i, md.ng);
    const int gx = int(g % md.ng[0]), gy = int((g / md.ng[0]) % md.ng[1]),
              gz = DIM == 3 ? int(g / (int64_t(md.ng[0]) * md.ng[1])) : 0;
    const int64_t li = int64_t(gx - ox) +
                       int64_t(md.nu[0]) * (int64_t(gy - ox) + (DIM == 3 ? int64_t(md.nu[1]) * (gz - ox) : 0));
    unsafeAtomicAdd(z + li, X[0][bx[0].pad(i)]);
  }
}

}  // namespace

hipError_t launch_patch_vcycle(const PatchArgs &pa, int npatch, const double *r, double *z,
                               const double *flag, hipStream_t st) {
  const size_t lds = size_t(pa.lds_total) * sizeof(double);
  if (pa.md.dim == 3) {
    hipError_t e = hipFuncSetAttribute((const void *)k_patch_vcycle<3>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return e;
    k_patch_vcycle<3><<<npatch, 64, lds, st>>>(pa, r, z, flag);
  } else {
    hipError_t e = hipFuncSetAttribute((const void *)k_patch_vcycle<2>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return e;
    k_patch_vcycle<2><<<npatch, 64, lds, st>>>(pa, r, z, flag);
  }
  return hipGetLastError();
}

}  // namespace lor

// Internal declarations shared by the host set-up code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lor.h"

namespace lor {

constexpr int kMaxP = 14;          // largest supported polynomial degree
constexpr int kMaxLevels = 6;      // 1 + ceil(log2(16)) = 5, one spare
constexpr int kMaxQ = kMaxP + 1;   // GLL points per direction

// 1D transfer between two consecutive levels of one patch direction.
// "fine" is level k, "coarse" level k+1; indices are into the zero-padded
// patch boxes (local index + 1), so a coarse node on the patch boundary
// reads the zero halo.
struct XferTab {
  int mf, mc;                 // unknowns per direction on the fine / coarse level
  int pc[2 * kMaxP][2];       // prolongation: padded coarse indices of fine f
  double pw[2 * kMaxP][2];    //               and their weights
  int rcnt[2 * kMaxP];        // restriction: number of fine nodes of coarse c
  int rf[2 * kMaxP][4];       //              padded fine indices
  double rw[2 * kMaxP][4];    //              weights (same as pw, transposed)
};

// Everything a device kernel needs to address the structured mesh.
struct MeshDims {
  int dim;
  int n[3];      // elements per direction (1 in unused directions)
  int p;
  int ng[3];     // GLL grid points per direction: n*p+1 (1 in unused dirs)
  int nu[3];     // unknowns per direction: ng-2 (Dirichlet) or ng (Neumann)
  int dirichlet; // 1: boundary nodes eliminated
};

// Patch data of the Schwarz preconditioner, by value into kernels.
struct PatchArgs {
  MeshDims md;
  int nlev;                          // levels of the element-structured hierarchy
  int s[kMaxLevels];                 // sub-intervals per element at each level
  int nv[3];                         // vertices per direction (n+1)
  const double *stencil[kMaxLevels]; // global level stencils, slot-major 3^d x npts
  int64_t npts[kMaxLevels];          // level grid points
  int lng[kMaxLevels][3];            // level grid points per direction
  const XferTab *xfer;               // [nlev-1][3] by (fine level, direction type)
  const char *fac;                   // factor pool
  const int64_t *fac_off;            // [J][nlev-1] byte offset of each block (-1: none)
  const int *depth;                  // [J][nlev-1] sweep depth
  int lds_offs[kMaxLevels];          // offsets (in doubles) of X_k in LDS; B_k, R_k follow
  int lds_total;                     // doubles of LDS per patch
};

// One (patch, level) factor block: int32 idx[n], lvl[n+1], mask[n]; then,
// 8-byte aligned, double val[27][n] (slot-major; center slot holds 1/D).
__host__ __device__ inline int64_t factor_block_bytes(int64_t n, int nslots) {
  int64_t ib = 4 * (3 * n + 1);
  ib = (ib + 15) & ~int64_t(15);
  return ib + 8 * int64_t(nslots) * n;
}
__host__ __device__ inline int64_t factor_vals_offset(int64_t n) {
  int64_t ib = 4 * (3 * n + 1);
  return (ib + 15) & ~int64_t(15);
}

// ---------------------------------------------------------------- host side
void gll_nodes_weights(int p, std::vector<double> &x, std::vector<double> &w);
void lagrange_derivative(const std::vector<double> &x, std::vector<double> &D);
std::vector<std::vector<int>> kept_points(int p);

// Result of the MDF ordering of one patch level.
struct MdfResult {
  std::vector<int> order;       // elimination order (patch-local indices)
  std::vector<int> level_ptr;   // dependency-level starts (depth+1 entries)
  std::vector<int> sched;       // rows in sweep order (sorted by level, then order)
  std::vector<double> L;        // n x nslots: l_im (earlier m) / l_mi (later m)
  std::vector<double> D;        // pivots
  std::vector<int> earlier;     // per row bit mask of slots holding earlier neighbours
};
// rows: n x nslots values (row-major), box shape m[0..dim-1].
// Returns LOR_OK or LOR_EPIVOT.
int mdf_factor(int dim, const int *m, std::vector<double> &rows, bool natural, MdfResult &out);

// ----------------------------------------------------- device launch wrappers
// "flag" (nullable) points at the Krylov scalar array: kernels return at once
// when its S_DONE entry is set.
hipError_t launch_node_coords(const MeshDims &md, const double *verts, const double *gllx,
                              double *coords, hipStream_t st);
hipError_t launch_geom_cg(const MeshDims &md, const double *verts, const double *gllx,
                          const double *gllw, double *G, double *wdet, int *bad, hipStream_t st);
hipError_t launch_lor_stencil(const MeshDims &md, int s, const int *kept_fine_idx,
                              const double *fine_coords, double g0, double g1, double *stencil,
                              hipStream_t st);
hipError_t launch_rhs_cg(const MeshDims &md, const double *wdet, const double *f, double *b,
                         hipStream_t st);
int apply_cg_blocks(const MeshDims &md);
hipError_t launch_apply_cg(const MeshDims &md, const double *G, const double *D,
                           const double *x, double *y, double *partials, const double *flag,
                           hipStream_t st);
hipError_t launch_coarse_restrict(const MeshDims &md, const double *gllx, const double *r,
                                  double *rc, hipStream_t st);
hipError_t launch_coarse_prolong(const MeshDims &md, const double *gllx, const double *xc,
                                 double *z, const double *flag, hipStream_t st);
hipError_t launch_gemv(int n, const double *A, const double *x, double *y, const double *flag,
                       hipStream_t st);
hipError_t launch_gauss_jordan(int n, double *A, double *rowbuf, double *colbuf, int *bad,
                               hipStream_t st);
hipError_t launch_patch_vcycle(const PatchArgs &pa, int npatch, const double *r, double *z,
                               const double *flag, hipStream_t st);
hipError_t launch_fill(double *x, int64_t n, double v, hipStream_t st);

// Krylov helpers.  Scalars live in a small device array.
enum Scal { S_RHO = 0, S_PQ, S_ALPHA, S_BETA, S_RR, S_BB, S_TOL2, S_DONE, S_ITERS, S_FAIL,
            S_RRTRUE, S_COUNT };
enum FinOp { FIN_PQ = 0, FIN_RR = 1, FIN_RHO = 2, FIN_BB = 3, FIN_FCG = 4, FIN_RRTRUE = 5 };
constexpr int kRedBlocks = 1024;  // most blocks of a two-stage reduction
int red_blocks(int64_t n);
hipError_t launch_dot_partials(const double *a, const double *b, int64_t n, double *partials,
                               const double *flag, hipStream_t st);
hipError_t launch_finalize(double *scal, const double *partials, int count, int which, int iter,
                           const double *partials2, hipStream_t st);
hipError_t launch_cg_update(double *x, double *r, double *rold, const double *p, const double *q,
                            int64_t n, const double *scal, double *partials, hipStream_t st);
hipError_t launch_p_update(double *p, double *q, const double *z, int64_t n, const double *scal,
                           hipStream_t st);
hipError_t launch_copy(double *dst, const double *src, int64_t n, hipStream_t st);
hipError_t launch_sub_dot(const double *b, const double *y, int64_t n, double *partials,
                          hipStream_t st);

}  // namespace lor

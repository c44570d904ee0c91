// Internal declarations shared by the host set-up code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lor.h"

namespace lor {

constexpr int kMaxP = 14;          // largest supported polynomial degree
constexpr int kMaxRhs = 4;         // right-hand sides per multi-RHS patch launch
constexpr int kMaxLevels = 6;      // 1 + ceil(log2(16)) = 5, one spare
constexpr int kMaxQ = kMaxP + 1;   // GLL points per direction

// 1D transfer between two consecutive levels of one patch direction.
// "fine" is level k, "coarse" level k+1; indices are patch-local along the
// direction.  A prolongation source outside [0, mc) lies on the patch
// boundary (zero) and is skipped.
struct XferTab {
  int mf, mc;                 // unknowns per direction on the fine / coarse level
  int pc[2 * kMaxP][2];       // prolongation: coarse indices of fine f
  double pw[2 * kMaxP][2];    //               and their weights
  int rcnt[2 * kMaxP];        // restriction: number of fine nodes of coarse c
  int rf[2 * kMaxP][4];       //              fine indices
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
  const double *stencil[kMaxLevels]; // global level stencils, point-major records
                                     // (rec_width): full in float, symmetric half in double
  int64_t npts[kMaxLevels];          // level grid points
  int lng[kMaxLevels][3];            // level grid points per direction
  const XferTab *xfer;               // [nlev-1][3] by (fine level, direction type)
  const char *fac;                   // factor pool
  const int64_t *fac_off;            // [J][nlev-1][2] byte offsets of the forward and
                                     // backward sweep blocks (-1: none)
  int lds_total;                     // LDS values per patch (largest patch)
  int fp32;                          // 1: stencils, factors and patch vectors in float
  int pou;                           // 1: corrections scaled by 1/c(i) (partition of unity)
  int plain;                         // 1: corrections added without atomics, one
                                     //    vertex-parity class of patches per launch
  int color;                         // parity class of this launch, -1: every patch
  const int *perm;                   // launch order: block b runs patch perm[b] (nullptr:
                                     //    vertex order)
  // Several right-hand sides of one matrix in one launch (nrhs > 0, see
  // launch_patch_vcycle_multi): right-hand side k reads rs[k], adds into
  // zs[k] and stops at flags[k]; otherwise nrhs == 0.
  int nrhs;
  const double *rs[kMaxRhs];
  double *zs[kMaxRhs];
  const double *flags[kMaxRhs];
};

// The patch corrections of several problems in one launch (see
// launch_patch_vcycle_jobs): problem k's blocks are [block0[k], block0[k+1]),
// laid out as in a multi-right-hand-side launch of p[k] (p[k].nrhs >= 1).
constexpr int kMaxJobs = 4;
struct PatchJobs {
  PatchArgs p[kMaxJobs];
  int njobs;
  int block0[kMaxJobs + 1];
};

// Sweep block: the data of one ILU(0) triangular sweep (forward or backward)
// of one (patch, level), laid out for a 64-lane wavefront.
//   header (kSweepHeader B): int32 nchunks, uint32 hdr0 (header of chunk 0),
//   8 B pad, uint8 q0[64] (quads lane l loads from chunk 0), 16 zero bytes.
//   chunks: a chunk is a run of consecutive dependency levels ("steps")
//   whose rows fit lanes 0-62: a row with at most kLaneCouplings couplings
//   takes one lane, a wider one the lane pair (2k, 2k+1), the even lane
//   holding the first couplings and the odd lane the rest, the two partial
//   sums added across the pair.  A chunk is stored as Q quads (16 B) per
//   lane, interleaved by lane: quad q of lane l at byte 16 * (q * 64 + l)
//   from the chunk start, so that one coalesced 1 KiB load brings every lane
//   its own quad.
//   Lane record (uint32 words): word 0 = row (bits 0-15) | step (16-21) |
//   quads of this lane's record in the next chunk (22-26) | kSweepPaired |
//   kSweepSecond | kSweepValid (lanes without a row only carry the next
//   size); for the backward sweep then 1 / D as T (zero in the second lane
//   of a pair); then one uint32 slot mask: bit s set for every stencil slot
//   s (the neighbour at offset (s%3-1, (s/3)%3-1, s/9-1), s != centre) that
//   this lane couples, and the coupling values as T in increasing slot order
//   (the record is zero beyond them).  The kernel turns a slot into the
//   neighbour's LDS offset from a 28-entry table of the level box (entry 27:
//   0, for padding couplings, which read the row itself with weight 0).  Lane
//   63 carries the header of the next chunk instead: Q (bits 0-7) | nsteps
//   (8-15) | W (16-23) | kChunkSplit,
//   W = the chunk's most couplings in a lane record, rounded up to even.
// Level stencils as the patch kernel reads them: point-major records, one
// per grid point g at g * rec_width.
//   float:  the full stencil, slots 0 .. 3^d - 1 in slot order, zero-padded
//           (128 B per point in 3D: one cache line, no neighbour reads);
//   double: the symmetric half, slots C .. 3^d - 1 (the centre and the
//           neighbours after it in slot order; C = (3^d - 1) / 2),
//           zero-padded.  Slot s < C of point g equals slot 3^d - 1 - s of
//           the neighbour g + offset(s) (the LOR matrices are symmetric bit
//           for bit).
template <int DIM, typename ST>
__host__ __device__ constexpr int rec_width() {
  return sizeof(ST) == 4 ? (DIM == 3 ? 32 : 12) : (DIM == 3 ? 16 : 8);
}
// index of the centre coefficient inside a record
template <int DIM, typename ST>
__host__ __device__ constexpr int rec_centre() {
  return sizeof(ST) == 4 ? (DIM == 3 ? 13 : 4) : 0;
}

constexpr int kChunkLanes = 63;   // lanes holding rows (lane 63: next header)
constexpr int kSweepHeader = 96;
constexpr int kSweepZero = 80;   // 16 zero bytes inside the header
constexpr int kMaxCouplings = 26;
constexpr int kLaneCouplings = 14;  // per lane record; wider rows take a lane pair
constexpr uint32_t kSweepPaired = 1u << 27;  // the row is split over lanes 2k, 2k+1
constexpr uint32_t kSweepSecond = 1u << 28;  // odd lane of a pair: partial sum only
constexpr uint32_t kSweepValid = 1u << 31;
constexpr uint32_t kChunkSplit = 1u << 24;   // the chunk holds split rows
template <typename T>
__host__ __device__ constexpr int sweep_head_words(bool fwd) {
  return fwd ? 1 : 1 + int(sizeof(T)) / 4;
}
// quads of a lane record with c couplings (head, slot mask, c values)
template <typename T>
__host__ __device__ constexpr int sweep_quads(bool fwd, int c) {
  return (sweep_head_words<T>(fwd) + 1 + c * int(sizeof(T)) / 4 + 3) / 4;
}
__host__ __device__ inline int64_t align16(int64_t b) { return (b + 15) & ~int64_t(15); }

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
// Elimination orders of a patch level's IC(0) smoother.
enum PatchOrdering { ORD_MDF = 0, ORD_NATURAL = 1, ORD_RCM = 2 };
// rows: n x nslots values (row-major), box shape m[0..dim-1]; ordering: a
// PatchOrdering.  Returns LOR_OK or LOR_EPIVOT.
int mdf_factor(int dim, const int *m, std::vector<double> &rows, int ordering, MdfResult &out);
// Reverse Cuthill-McKee order of a box of grid points with the stencil
// adjacency (offsets differing by at most one per direction).
std::vector<int> rcm_order(int dim, const int *m);
// Sweep block of one direction (layout at kChunkLanes).
template <typename T>
std::vector<char> pack_sweep(const MdfResult &res, int dim, const int *m, bool fwd);

// ----------------------------------------------------- device launch wrappers
// "flag" (nullable) points at the Krylov scalar array: kernels return at once
// when its S_DONE entry is set.
hipError_t launch_node_coords(const MeshDims &md, const double *verts, const double *gllx,
                              double *coords, hipStream_t st);
// coef: the coefficient b at every element's GLL nodes (n_el (p+1)^d), or
// nullptr for b = 1
hipError_t launch_geom_cg(const MeshDims &md, const double *verts, const double *gllx,
                          const double *gllw, const double *coef, double *G, double *wdet, int *bad,
                          hipStream_t st);
// curved elements: the same factors from the GLL node coordinates (SoA)
hipError_t launch_geom_nodal(const MeshDims &md, const double *coords, const double *D,
                             const double *gllw, const double *coef, double *G, double *wdet, int *bad,
                             hipStream_t st);
hipError_t launch_lor_stencil(const MeshDims &md, int s, const int *kept_fine_idx,
                              const double *fine_coords, double g0, double g1, const double *coef,
                              double *stencil, hipStream_t st);
hipError_t launch_rhs_cg(const MeshDims &md, const double *wdet, const double *f, double *b,
                         hipStream_t st);
// Blocks (= partial sums) of one operator launch.
int apply_cg_blocks(const MeshDims &md, bool dg);
// fo == nullptr: CG operator on the L-vector; otherwise the DG volume term on
// the E-vector plus the face records fo written by launch_dg_face.  CG with
// apply_cg_uses_skeleton(md): yE (n_el (p+1)^3 values) receives the
// element-boundary partial results, which a second kernel sums into y (y is
// then written completely, no zeroing needed); otherwise y must be zero on
// entry (shared nodes are accumulated atomically) and yE is unused.
bool apply_cg_uses_skeleton(const MeshDims &md);
// geo: recompute the geometric factors from the vertices instead of reading
// G (3D CG, 5 <= p + 1 <= 8 only)
struct GeoArgs {
  const double *verts = nullptr, *gllx = nullptr, *gllw = nullptr;
};
hipError_t launch_apply_cg(const MeshDims &md, const double *G, const double *D,
                           const double *x, double *y, double *partials, const double *flag,
                           hipStream_t st, const double *fo = nullptr, double *yE = nullptr,
                           const GeoArgs *geo = nullptr);

// DG (faces, penalties, diagonal, E-vector transfers)
int64_t dg_face_count(const MeshDims &md);
hipError_t launch_dg_coords(const MeshDims &md, const double *verts, const double *gllx,
                            double *coords, hipStream_t st);
hipError_t launch_dg_face_geom(const MeshDims &md, const double *verts, const double *gllx,
                               const double *gllw, const double *wdet, int method, double eta,
                               double *fg, hipStream_t st);
hipError_t launch_dg_face(const MeshDims &md, const double *D, const double *fg, const double *x,
                          double *fo, const double *flag, hipStream_t st);
hipError_t launch_dg_diag(const MeshDims &md, const double *G, const double *D, const double *fg,
                          double *dinv, hipStream_t st);
hipError_t launch_dg_restrict(const MeshDims &md, const double *rE, double *rL, const double *flag,
                              hipStream_t st);
hipError_t launch_dg_prolong_jacobi(const MeshDims &md, const double *rE, const double *dinv,
                                    const double *zL, double *zE, const double *flag,
                                    hipStream_t st);
hipError_t launch_dg_rhs(const double *wdet, const double *f, double *b, int64_t n,
                         hipStream_t st);
hipError_t launch_coarse_restrict(const MeshDims &md, const double *gllx, const double *r,
                                  double *rc, hipStream_t st);
hipError_t launch_coarse_prolong(const MeshDims &md, const double *gllx, const double *xc,
                                 double *z, const double *flag, hipStream_t st);
hipError_t launch_gemv(int n, const double *A, const double *x, double *y, const double *flag,
                       hipStream_t st);
// y = A x with the float32 copy of a float64 matrix (float64 products and sums)
hipError_t launch_gemv_f32(int n, const float *A, const double *x, double *y, const double *flag,
                           hipStream_t st);
// C = alpha A B + beta C in float64 on the matrix cores (row major, any sizes)
hipError_t launch_dgemm(int m, int n, int k, double alpha, const double *A, int64_t lda,
                        const double *B, int64_t ldb, double beta, double *C, int64_t ldc,
                        hipStream_t st);
hipError_t launch_small_inverse(const double *M, int ldm, double *Minv, int bk, int *bad,
                                hipStream_t st);
hipError_t launch_copy_block(const double *src, int64_t lds, double *dst, int64_t ldd, int rows,
                             int cols, double scale, hipStream_t st);
// In-place inverse of the dense SPD n x n matrix A (device, row-major);
// LOR_EPIVOT if a pivot is not positive.
int coarse_inverse(int n, double *A, hipStream_t st);
// Raises the patch kernel's dynamic LDS limit (call once before launches,
// outside any stream capture).
hipError_t prepare_patch_vcycle(const PatchArgs &pa);
// dense == nullptr: z += sum_j R_j^T V_j(R_j r) (atomically).  Otherwise the
// patch results V_j(R_j r) / dscale[j] are written into dense
// [npatch][(2p-1)^d] (grid point g_d = level-0 node - (v_d p - p + 1)) and z
// is not touched; dense must be zero where no patch unknown lies.
hipError_t launch_patch_vcycle(const PatchArgs &pa, int npatch, const double *r, double *z,
                               const double *flag, hipStream_t st, float *dense = nullptr,
                               const double *dscale = nullptr);
// z_k += sum_j R_j^T V_j(R_j r_k) for nrhs <= kMaxRhs right-hand sides of one
// matrix in one launch (flags[k]: the done flag of right-hand side k, or
// nullptr).  Block b takes right-hand side (b / 8) % nrhs of patch slot
// (b / (8 nrhs)) 8 + b % 8: the nrhs blocks of one patch land on the same
// XCD within a few dispatches of each other and share its L2 for the
// patch's factor and stencil records.  Not with the colored (plain) scatter.
hipError_t launch_patch_vcycle_multi(const PatchArgs &pa, int npatch, int nrhs,
                                     const double *const *r, double *const *z,
                                     const double *const *flags, hipStream_t st);
// The patch corrections of njobs problems (dimension and precision alike,
// up to kMaxJobs, each with jobs[k].nrhs right-hand sides in jobs[k].rs,
// zs, flags) in one launch sized for the largest patch of any of them.
hipError_t launch_patch_vcycle_jobs(const PatchArgs *jobs, int njobs, hipStream_t st);
// Warm start of the patch V-cycles for patches first .. first + count - 1
// (3D): y [count][(2p-1)^3] predictions on the patch grid, scale [count];
// z += y_j + V_j(r_j - A_j y_j) (scaled) for each.
hipError_t launch_patch_vcycle_warm(const PatchArgs &pa, int first, int count, const double *r,
                                    double *z, const float *y, const double *scale,
                                    const double *flag, hipStream_t st);
// ---- box-patch preconditioners: B(1), B(n), isotropic vertex patches (k_single.hip, box_patch.cpp)
// 1D transfer tables between the interior boxes of levels k and k+1: for
// every fine index its two parents (coarse index or -1) and weights, for
// every coarse index R[d] (fine index or -1, weight) pairs.
struct SingleXfer {
  int mf[3], mc[3], R[3];
  const int *pc[3];
  const double *pw[3];
  const int *rf[3];
  const double *rw[3];
};
// a run of dependency levels [l0, l1) swept by one workgroup, or one large
// level (grid = 1, l1 = l0 + 1) swept by a launch over the whole device
struct SingleSeg {
  int l0, l1, grid;
};
struct SingleLevelDev {
  int lo[3];                   // first level-grid index of the box's points
  int m[3];                    // interior box extents
  int64_t n;                   // rows
  int *sched = nullptr;        // rows by dependency level
  int *lptr = nullptr;         // level starts (depth + 1)
  std::vector<int> lptr_host;
  std::vector<SingleSeg> segs;
  double *Lv = nullptr;        // n x 3^d factor values (row i: l_im earlier, l_mi later)
  double *invD = nullptr;      // 1 / pivot
  int *emask = nullptr;        // slots of earlier in-box neighbours
  int *lmask = nullptr;        // slots of later in-box neighbours
  double *x = nullptr, *b = nullptr, *r = nullptr;  // level vectors (shared by the boxes)
  SingleXfer xf{};             // to the next coarser level
  double *ainv = nullptr;      // coarsest level: dense inverse
};
hipError_t launch_single_sweep(int dim, bool fwd, const SingleLevelDev &lv, const double *b, double *x,
                               const double *flag, hipStream_t st);
hipError_t launch_single_residual(int dim, const double *stencil, int64_t npts, const int *lng,
                                  const int *lo, const int *m, const double *b, const double *x,
                                  double *r, const double *flag, hipStream_t st);
// level-0 box of a patch <-> L-vector: out = r[box] (gather) or
// z[box] += w[box] * x (scatter, w may be nullptr for weight 1)
hipError_t launch_box_gather(int dim, const MeshDims &md, const int *lo, const int *m,
                             const double *r, double *out, const double *flag, hipStream_t st);
hipError_t launch_box_scatter(int dim, const MeshDims &md, const int *lo, const int *m,
                              const double *x, const double *w, double *z, const double *flag,
                              hipStream_t st);
hipError_t launch_single_transfer(int dim, bool prolong, const SingleXfer &t, const double *in,
                                  double *out, const double *flag, hipStream_t st);
hipError_t launch_axpy1(double *x, const double *y, int64_t n, const double *flag, hipStream_t st);

hipError_t launch_fill(double *x, int64_t n, double v, hipStream_t st);
hipError_t launch_to_float(const double *src, float *dst, int64_t n, hipStream_t st);
// slot-major float64 stencil (3^dim x npts) -> point-major records
// (rec_width values per point): full in float (f32), symmetric half in float64.
hipError_t launch_sym_stencil(const double *soa, int64_t npts, int dim, void *out, bool f32,
                              hipStream_t st);

// Learned patch correction (k_nn.hip).  bf16 values are uint16_t bit patterns.
hipError_t nn_gemm(int M, int N, int K, const uint16_t *A, int64_t ai, int64_t ak,
                   const uint16_t *B, int64_t bk, int64_t bj, float *C, int64_t ldc, bool acc,
                   hipStream_t st);
hipError_t nn_im2col(const uint16_t *act, int64_t rows, int G, int cin, int Kp, int64_t npad,
                     uint16_t *cols, const double *flag, hipStream_t st);
hipError_t nn_col2im_relu(const float *dcols, int64_t rows, int64_t npad, int G, int cin, int Kp,
                          const float *zprev, int ldzp, float *dz, uint16_t *dz16, hipStream_t st);
hipError_t nn_bias_relu(float *z, int64_t rows, int cout, int Np, const float *bias, uint16_t *a,
                        const double *flag, hipStream_t st);
hipError_t nn_input(const float *X, int64_t rows, int64_t npad, uint16_t *a0, const double *flag,
                    hipStream_t st);
hipError_t nn_output(const float *z, int Np, const float *X, int64_t rows, float *y,
                     const double *flag, hipStream_t st);
// per-block partial sums: at most kPartStride blocks, column c at part + c * kPartStride
constexpr int kPartStride = 1024;
int nn_red_blocks(int64_t n);
hipError_t nn_loss(const float *y, const float *T, const float *X, int64_t rows, int64_t npad,
                   int Np, const double *msum, float *dz, uint16_t *dz16, double *part, hipStream_t st);
hipError_t nn_colsum(const float *a, int64_t rows, int ld, int col0, int ncols, double *part,
                     hipStream_t st);
hipError_t nn_sum_partials(const double *part, int nblk, int ncols, double *dsum, float *fsum,
                           hipStream_t st);
hipError_t nn_adam(float *w, float *m, float *v, const float *g, int64_t n, float lr, float b1,
                   float b2, float eps, float c1, float c2, hipStream_t st);
hipError_t nn_pack(const float *wl, int K27, int cout, int Kp, int Np, uint16_t *Wb, float *bias,
                   hipStream_t st);
hipError_t nn_grad_gather(const float *dW, int K27, int cout, int Np, float *g, hipStream_t st);
hipError_t nn_gather(const MeshDims &md, int first, int count, const double *r, float *X,
                     double *scale, const double *flag, hipStream_t st);
hipError_t nn_scatter(const MeshDims &md, int first, int count, const float *y,
                      const double *scale, double *z, const double *flag, hipStream_t st);
hipError_t nn_fill(float *x, int64_t n, float v, hipStream_t st);
// Fused implicit-GEMM convolution layer (layer 0: 2 -> C channels, 1: C -> C,
// 2: C -> 1 masked output y) for C in {16, 32} and 3 <= G <= 15: zout
// [rows][Np] pre-activations (may be NULL), aout [rows][C] bf16 ReLU output
// of layers 0 and 1, y [rows] of layer 2 (X: the network input, for the mask).
bool nn_conv_supported(int channels, int G);
hipError_t nn_conv_prepare(int channels);
// Wf: the layer's weights in MFMA fragment order (nn_conv_frag of Wb [Kp][Np]).
hipError_t nn_conv_frag(const uint16_t *Wb, int Kp, int Np, uint16_t *Wf, hipStream_t st);
hipError_t nn_conv_layer(int channels, int layer, const uint16_t *ain, int nb, int G,
                         const uint16_t *Wf, const float *bias, float *zout, uint16_t *aout,
                         const float *X, float *y, const double *flag, hipStream_t st);

// Krylov helpers.  Scalars live in a small device array.
enum Scal { S_RHO = 0, S_PQ, S_ALPHA, S_BETA, S_RR, S_BB, S_TOL2, S_DONE, S_ITERS, S_FAIL,
            S_RRTRUE, S_MAXIT, S_COUNT };
enum FinOp { FIN_PQ = 0, FIN_RR = 1, FIN_RHO = 2, FIN_BB = 3, FIN_FCG = 4, FIN_RRTRUE = 5 };
constexpr int kRedBlocks = 1024;  // most blocks of a two-stage reduction
int red_blocks(int64_t n);
hipError_t launch_dot_partials(const double *a, const double *b, int64_t n, double *partials,
                               const double *flag, hipStream_t st);
// a.b and a.c partials in one pass over a
hipError_t launch_dot2_partials(const double *a, const double *b, const double *c, int64_t n,
                                double *pb, double *pc, const double *flag, hipStream_t st);
hipError_t launch_finalize(double *scal, const double *partials, int count, int which,
                           const double *partials2, hipStream_t st);
hipError_t launch_cg_update(double *x, double *r, double *rold, const double *p, const double *q,
                            int64_t n, const double *scal, double *partials, hipStream_t st);
hipError_t launch_p_update(double *p, double *q, const double *z, int64_t n, const double *scal,
                           hipStream_t st);
hipError_t launch_copy(double *dst, const double *src, int64_t n, hipStream_t st);
// partials of ||b - y||^2; res (optional, may equal y) receives b - y
hipError_t launch_sub_dot(const double *b, const double *y, int64_t n, double *partials,
                          hipStream_t st, double *res = nullptr);

}  // namespace lor

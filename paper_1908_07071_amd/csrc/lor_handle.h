// Handle of the C ABI (private to the library): mesh, discretization,
// preconditioner data and the default solve workspace.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>
#include <vector>

#include "box_vcycle.h"
#include "lor_internal.h"

using namespace lor;

struct lor_nn;

// One box patch: elements [a_d, b_d) and the data of each level.
struct BoxPatchDev {
  int a[3] = {0, 0, 0}, b[3] = {1, 1, 1};
  std::vector<SingleLevelDev> lv;
};

// Device workspace of one solve.  The handle holds one; a batched solve holds
// one per (problem, right-hand side) pair so that the pairs of one problem can
// run concurrently.
struct Work {
  double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *rold = nullptr, *tmp = nullptr;
  double *scal = nullptr, *part = nullptr, *part2 = nullptr;
  double *rc = nullptr, *xc = nullptr;  // coarse-space vectors
  double *yE = nullptr;                 // element-boundary operator results (CG skeleton path)
  double *fo = nullptr;                 // DG face records
  double *rL = nullptr, *zL = nullptr;  // DG: conforming vectors of E B E^T
  double *h_scal = nullptr;             // pinned host copy of scal
};

struct lor_handle {
  int dim = 3, n[3] = {1, 1, 1}, p = 1, method = LOR_CG, bc = LOR_BC_DIRICHLET;
  double penalty = 0.0;
  double t_setup = 0.0;  // seconds lor_setup took (host clock)
  int device = 0;        // HIP device current at lor_setup (holds the handle's memory)
  lor_options_t opt{};
  MeshDims md{};
  std::vector<double> verts, gllx, gllw, D;
  std::vector<double> coef;  // b at the elements' GLL nodes (empty: b = 1)
  std::vector<double> nodes; // curved elements: GLL-grid node coordinates (empty: Q1 maps)
  std::vector<std::vector<int>> kept;
  int L = 1;
  int64_t ndofs = 0, nfine = 0, nel = 0;
  int64_t ncg = 0;     // conforming unknowns (the L-vector of the Schwarz preconditioner)
  int64_t nfaces = 0;  // DG faces
  int J = 0, nc = 0;
  // device memory (owned)
  std::vector<void *> allocs;
  std::vector<size_t> alloc_size;  // bytes of each entry of allocs
  size_t bytes = 0;
  // caller-owned device workspace (lor_bind_workspace): every allocation
  // above moved into it; allocs is then empty
  bool bound = false;
  size_t bound_bytes = 0;
  // cached workspaces of batched solves (one per concurrent pair of this
  // handle), owned by the library and kept until lor_free
  std::vector<Work> bwork;
  std::vector<void *> ballocs;
  size_t bbytes = 0;
  double *d_verts = nullptr, *d_gllx = nullptr, *d_gllw = nullptr, *d_D = nullptr;
  double *d_coords = nullptr, *d_G = nullptr, *d_wdet = nullptr;
  double *d_stencil[kMaxLevels] = {};
  int64_t npts[kMaxLevels] = {};
  char *d_fac = nullptr;
  int64_t *d_fac_off = nullptr;
  int64_t fac_bytes = 0;
  XferTab *d_xfer = nullptr;
  double *d_A0inv = nullptr;
  float *d_A0inv_f = nullptr;  // mixed precision: float32 copy (the float64 one is released)
  double *d_fg = nullptr, *d_dinv = nullptr;
  double *d_coef = nullptr;
  int *d_perm = nullptr;       // patches by decreasing work (launch buckets)
  int order_used = 0;          // LOR_LAUNCH_VERTEX or LOR_LAUNCH_BUCKETS
  bool geo_onfly = false;      // operator recomputes G from the vertices (d_G not stored)
  double tune_ms[2] = {0, 0};  // autotuner: patch launch in vertex order, in buckets
  int npart = 0;
  Work w;                  // workspace of lor_pcg_solve / lor_apply_*
  lor_nn *nn = nullptr;    // patch network used instead of the V-cycles (LOR_NN_REPLACE)
  int nn_mode = 0;
  bool capturing = false;  // no event timing while a graph is captured
  PatchArgs pa{};
  std::vector<BoxPatchDev> boxes;  // box-patch modes: every patch's levels
  std::vector<double *> box_x, box_b, box_r;  // level vectors shared by the box patches
  double *d_box_w = nullptr;                  // partition-of-unity weights of the box patches
  // Box patches side by side: the patches of one colour have disjoint level-0
  // boxes and run on kBoxStreams streams, each with its own level vectors
  // (set 0: box_x / box_b / box_r); colours one after another.
  static constexpr int kBoxStreams = 4;
  std::vector<double *> box_sx[kBoxStreams - 1], box_sb[kBoxStreams - 1], box_sr[kBoxStreams - 1];
  std::vector<int> box_color;  // colour of every box (in box order)
  int box_ncolor = 0;
  hipStream_t box_st[kBoxStreams] = {};
  hipEvent_t box_ev[kBoxStreams + 1] = {};
  // boxes small enough for one workgroup each: all V-cycles in one launch,
  // then the corrections added to z one colour per launch
  std::vector<char> box_fused;        // per box
  std::vector<int64_t> box_vo;        // per box and level: offset of its x, b, r in d_box_work
  std::vector<int64_t> box_vl;        // per box and level: length of each of them
  int box_nfused = 0;                 // d_box_list[0 .. box_nfused): every one-workgroup box
  std::vector<int> box_list_off;      // colour c: d_box_list[box_nfused + box_list_off[c] ..)
  std::vector<int> box_unfused;       // per colour: boxes on the per-level launches
  BoxDesc *d_box_desc = nullptr;      // every box's level descriptors (device pointers)
  int *d_box_list = nullptr;
  double *d_box_work = nullptr;       // the one-workgroup boxes' level vectors
  BoxGrid box_grid{};
  // every box on the one-workgroup path: all corrections added in one launch,
  // per L-vector point its boxes in colour order (launch_box_add_points)
  int64_t box_add_npt = 0;
  int64_t *d_add_ptr = nullptr, *d_add_pts = nullptr, *d_add_src = nullptr;
  // host copies for parity export
  std::vector<int32_t> order_all, order_off, sched_all, sched_off;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool has_prec = false;
  // per-kernel event timing
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> tspans[3];
  hipEvent_t next_event() {
    if (ev_used == ev_pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      ev_pool.push_back(e);
    }
    return ev_pool[ev_used++];
  }

  template <class T>
  hipError_t alloc(T **ptr, size_t count) {
    void *p = nullptr;
    size_t b = std::max<size_t>(count * sizeof(T), 16);
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) return e;
    allocs.push_back(p);
    alloc_size.push_back(b);
    bytes += b;
    *ptr = static_cast<T *>(p);
    return hipSuccess;
  }
  // releases one allocation of allocs (no-op for pointers it does not hold)
  void release(void *p) {
    for (size_t i = 0; i < allocs.size(); ++i)
      if (allocs[i] == p) {
        (void)hipFree(p);
        bytes -= alloc_size[i];
        allocs.erase(allocs.begin() + i);
        alloc_size.erase(alloc_size.begin() + i);
        return;
      }
  }
  ~lor_handle() {
    for (void *p : allocs) (void)hipFree(p);
    for (void *p : ballocs) (void)hipFree(p);
    for (Work &bw : bwork)
      if (bw.h_scal) (void)hipHostFree(bw.h_scal);
    if (w.h_scal) (void)hipHostFree(w.h_scal);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : box_ev)
      if (e) (void)hipEventDestroy(e);
    for (hipStream_t t : box_st)
      if (t) (void)hipStreamDestroy(t);
  }
};


// z = B r with the coarse-space vectors (and, for DG, the conforming vectors
// of E B E^T) taken from `scratch` (device memory of `cap` doubles, 256-byte
// aligned) instead of the handle's workspace; no allocation, no memset and no
// event recording (lor_api.cpp).  LOR_ENOMEM if `cap` is too small.
size_t apply_P_scratch_doubles(const lor_handle *h);
int apply_P_scratch(lor_handle *h, double *scratch, size_t cap, const double *r, double *z,
                    hipStream_t st);
// Looks up, once per device, the device address of the static scratch array
// of the no-allocation entry point on the current device (noalloc.hip).
int noalloc_register_device(int device);

// Box-patch preconditioners (box_patch.cpp): B(1), B(n) slabs, isotropic
// vertex patches.  Set-up from the host copies of the level stencils, and
// the patch part of z = B r (B(1): all of it; the others add into z).
int build_boxes(lor_handle &h, const std::vector<std::vector<double>> &hst, hipStream_t st);
int apply_boxes(lor_handle *h, const double *r, double *z, const double *flag, hipStream_t st);
// writes the box descriptors and the shared level layout from the handle's
// current device pointers (after set-up and after the memory has moved)
int refresh_box_descs(lor_handle &h, hipStream_t st);
inline bool box_mode(int m) {
  return m == LOR_PATCH_SINGLE || m == LOR_PATCH_SLABS || m == LOR_PATCH_VERTEX_ISO;
}

// Patches of the Schwarz preconditioner through the attached network:
// z += sum_j R_j^T s_j net(R_j r / s_j) (nn_api.cpp).
int nn_apply_patches(lor_nn *nn, const double *r, double *z, const double *flag, hipStream_t st);
int nn_apply_patches_warm(lor_nn *nn, const double *r, double *z, const double *flag,
                          hipStream_t st);

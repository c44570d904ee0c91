// One workgroup per box patch: the whole V-cycle of a small box (Sections
// 3.3 and 4.5), every such box in one launch.
//
// A box qualifies when no dependency level of its sweeps has more than
// `sweep_grid_rows` rows and its finest level has at most kBoxFuseRows rows
// (and while the level vectors of all qualifying boxes fit kBoxWorkDoubles):
// then one workgroup walks every sweep level by level (a barrier between
// levels) and does the residuals, transfers, the exact solve on its part of
// T_p and the gather from r itself, with the same arithmetic, row for row,
// as the separate launches of the larger boxes (each sweep pair on an LDS
// copy of its vector when the launch's largest box fits kBoxLdsRows).  Each
// box keeps its own level vectors, so all of them run at once; the
// corrections are then added
// to z one colour of boxes per launch (boxes of one colour have disjoint
// level-0 point ranges), in the order the per-level path adds them.
#pragma once

#include <hip/hip_runtime.h>

#include "lor_internal.h"

namespace lor {

constexpr int kBoxThreads = 256;       // threads per box workgroup
constexpr int kBoxFuseRows = 1 << 16;  // largest finest-level box on the one-workgroup path
constexpr int64_t kBoxWorkDoubles = int64_t(1) << 28;  // level vectors of those boxes, at most
constexpr int kBoxLdsRows = 8192;      // sweeps on an LDS copy of the vector up to 64 KiB

// One level of one box (device pointers into the handle's allocations).
struct BoxLevelDesc {
  int lo[3], m[3];  // first level-grid index and extents of the interior box
  int n;            // rows; 0: the box has no interior points on this level
  int depth;        // dependency levels of the sweeps (0 on the coarsest level)
  const int *sched, *lptr;
  const double *Lv, *invD;
  const int *emask, *lmask;
  SingleXfer xf;         // to the next coarser level
  const double *ainv;    // coarsest level: dense inverse (n x n, row major)
  int64_t vo;            // this box's x, b, r of the level: work + vo, + vl, + 2 vl
  int64_t vl;
};

struct BoxDesc {
  BoxLevelDesc lv[kMaxLevels];
};

// What every box shares: the level stencils over the whole level grids.
struct BoxGrid {
  const double *stencil[kMaxLevels];
  int64_t npts[kMaxLevels];
  int lng[kMaxLevels][3];
  int L;
  int lds_rows;  // largest finest level of the boxes in the launch (LDS sweeps when <= kBoxLdsRows)
};

// V-cycles of `count` boxes, boxes[list[i]] for i < count, one workgroup
// each, in their own level vectors in `work`.  direct = 0: b_0 gathered
// from r, the correction left in the box's level-0 x.  direct = 1 (one box
// covering the domain): level 0 reads r and writes z itself.
// Nothing happens for count == 0; otherwise hipErrorInvalidValue for a bad
// dimension, count or level count.
hipError_t launch_box_vcycles(int dim, const BoxDesc *boxes, const int *list, int count,
                              const BoxGrid &g, const MeshDims &md, const double *r, double *z,
                              int direct, double *work, const double *flag, hipStream_t st);
// z += w x_0 over the level-0 boxes of boxes[list[i]], i < count (boxes with
// disjoint level-0 ranges; w may be null for weight 1).
hipError_t launch_box_add(int dim, const BoxDesc *boxes, const int *list, int count,
                          const MeshDims &md, const double *w, double *z, const double *work,
                          const double *flag, hipStream_t st);

// z_u += w_u x over the boxes holding point u, every point in one launch:
// points pts[t] (L-vector indices, t < npt), their entries
// [ptr[t], ptr[t+1]) of src (offsets in `work` of the boxes' level-0 x
// values, in colour order).
hipError_t launch_box_add_points(const int64_t *ptr, const int64_t *pts, const int64_t *src, int64_t npt,
                                 const double *w, double *z, const double *work, const double *flag,
                                 hipStream_t st);

}  // namespace lor

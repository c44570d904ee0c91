// Host-side planning with no device code: the colours of the box patches
// (boxes of one colour have disjoint level-0 point ranges, so their
// corrections can be added to z side by side) and the grouping of a batched
// solve's lockstep parts into captured chunks and streams.
#pragma once

#include <cstdint>
#include <vector>

namespace lor {

// A box's interior points on level 0: first grid index and extents per
// direction (n <= 0: the box has none and overlaps nothing).
struct BoxRange {
  int lo[3], m[3];
  int64_t n;
};

// Greedy colouring in box order: box j takes the smallest colour that no
// earlier box overlapping it has.  Returns the colour of every box and sets
// *ncolour (at least 1 for a non-empty list).
std::vector<int> greedy_box_colours(const std::vector<BoxRange> &boxes, int dim, int *ncolour);

// One lockstep part of a batched solve: up to four right-hand sides of one
// problem, their patch corrections in one launch when `multi`.
struct BatchPart {
  bool multi;       // the handle allows several right-hand sides per patch launch
  int dim, fp32;    // parts share a launch only with like dimension and precision
  int lds;          // LDS values per patch of the handle (similar sizes grouped together)
  int64_t blocks;   // patch blocks of the part's own launch
  double cost;      // unknowns times right-hand sides
};

// Groups of part indices, each one captured chunk: with more parts than
// streams, the multi parts whose launch has fewer than max_blocks blocks
// share groups (like dimension and precision, sorted by decreasing lds, up
// to max_jobs parts and max_blocks blocks per group); every other part is a
// group of its own.  Every part is in exactly one group.
std::vector<std::vector<int>> plan_batch_groups(const std::vector<BatchPart> &parts, int nstreams,
                                                int max_jobs, int64_t max_blocks);

// The stream of every group: the costliest group first, each to the least
// loaded of nstreams streams (ties: the lower stream).
std::vector<int> assign_streams(const std::vector<double> &costs, int nstreams);

}  // namespace lor

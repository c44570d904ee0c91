// Host-side planning: box colours and batched-solve groups (see host_plan.h).
#include "host_plan.h"

#include <algorithm>
#include <tuple>

namespace lor {

std::vector<int> greedy_box_colours(const std::vector<BoxRange> &boxes, int dim, int *ncolour) {
  auto overlap = [&](const BoxRange &a, const BoxRange &b) {
    if (a.n <= 0 || b.n <= 0) return false;
    for (int d = 0; d < dim; ++d)
      if (a.lo[d] + a.m[d] <= b.lo[d] || b.lo[d] + b.m[d] <= a.lo[d]) return false;
    return true;
  };
  std::vector<int> colour(boxes.size(), 0);
  int nc = boxes.empty() ? 0 : 1;
  std::vector<char> used;
  for (size_t j = 0; j < boxes.size(); ++j) {
    used.assign(boxes.size() + 1, 0);
    for (size_t i = 0; i < j; ++i)
      if (overlap(boxes[i], boxes[j])) used[colour[i]] = 1;
    int c = 0;
    while (used[c]) ++c;
    colour[j] = c;
    nc = std::max(nc, c + 1);
  }
  if (ncolour) *ncolour = nc;
  return colour;
}

std::vector<std::vector<int>> plan_batch_groups(const std::vector<BatchPart> &parts, int nstreams,
                                                int max_jobs, int64_t max_blocks) {
  std::vector<std::vector<int>> groups;
  const bool share = int(parts.size()) > nstreams && max_jobs > 1;
  std::vector<int> small;
  for (int a = 0; a < int(parts.size()); ++a) {
    if (share && parts[a].multi && parts[a].blocks < max_blocks)
      small.push_back(a);
    else
      groups.push_back({a});
  }
  auto key = [&](int a) { return std::make_tuple(parts[a].dim, parts[a].fp32, -parts[a].lds); };
  std::stable_sort(small.begin(), small.end(), [&](int x, int y) { return key(x) < key(y); });
  for (size_t i = 0; i < small.size();) {
    std::vector<int> g;
    int64_t nb = 0;
    const BatchPart &p0 = parts[small[i]];
    while (i < small.size() && int(g.size()) < max_jobs) {
      const BatchPart &pt = parts[small[i]];
      if (!g.empty() && (pt.dim != p0.dim || pt.fp32 != p0.fp32 || nb + pt.blocks > max_blocks)) break;
      g.push_back(small[i]);
      nb += pt.blocks;
      ++i;
    }
    groups.push_back(g);
  }
  return groups;
}

std::vector<int> assign_streams(const std::vector<double> &costs, int nstreams) {
  std::vector<int> order(costs.size()), out(costs.size(), 0);
  for (size_t g = 0; g < order.size(); ++g) order[g] = int(g);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return costs[a] > costs[b]; });
  std::vector<double> load(std::max(nstreams, 1), 0.0);
  for (int g : order) {
    int t = 0;
    for (int u = 1; u < int(load.size()); ++u)
      if (load[u] < load[t]) t = u;
    load[t] += costs[g];
    out[g] = t;
  }
  return out;
}

}  // namespace lor

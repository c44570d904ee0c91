// Host check of the planning helpers (csrc/host_plan.cpp): box colours and
// the grouping of a batched solve's parts.  Prints "OK" or the first
// violated property and exits with status 1.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

#include "host_plan.h"

using namespace lor;

static int fail(const char *what, long a, long b) {
  std::printf("FAIL %s (%ld, %ld)\n", what, a, b);
  return 1;
}

static bool overlap(const BoxRange &a, const BoxRange &b, int dim) {
  if (a.n <= 0 || b.n <= 0) return false;
  for (int d = 0; d < dim; ++d) {
    // some point index in both ranges
    const int lo = std::max(a.lo[d], b.lo[d]), hi = std::min(a.lo[d] + a.m[d], b.lo[d] + b.m[d]);
    if (lo >= hi) return false;
  }
  return true;
}

static int check_colours(const std::vector<BoxRange> &bx, int dim) {
  int nc = -1;
  const std::vector<int> c = greedy_box_colours(bx, dim, &nc);
  if (c.size() != bx.size()) return fail("colour count", long(c.size()), long(bx.size()));
  int mx = -1;
  for (size_t j = 0; j < bx.size(); ++j) {
    mx = std::max(mx, c[j]);
    if (bx[j].n <= 0 && c[j] != 0) return fail("empty box colour", long(j), c[j]);
    std::set<int> below;
    for (size_t i = 0; i < j; ++i) {
      if (!overlap(bx[i], bx[j], dim)) continue;
      if (c[i] == c[j]) return fail("overlapping boxes share a colour", long(i), long(j));
      below.insert(c[i]);
    }
    // greedy: every smaller colour is taken by an earlier overlapping box
    for (int k = 0; k < c[j]; ++k)
      if (!below.count(k)) return fail("colour not the smallest free one", long(j), k);
  }
  if (nc != (bx.empty() ? 0 : std::max(mx + 1, 1))) return fail("ncolour", nc, mx + 1);
  return 0;
}

int main() {
  std::mt19937 rng(7);
  // vertex boxes one element either way on a structured block: 2^d colours
  for (int dim = 2; dim <= 3; ++dim) {
    const int n = 6, s = 4;
    std::vector<BoxRange> bx;
    const int nv = n + 1, nz = dim == 3 ? nv : 1;
    for (int vz = 0; vz < nz; ++vz)
      for (int vy = 0; vy < nv; ++vy)
        for (int vx = 0; vx < nv; ++vx) {
          const int v[3] = {vx, vy, vz};
          BoxRange b{};
          b.n = 1;
          for (int d = 0; d < 3; ++d) {
            if (d >= dim) {
              b.lo[d] = 0;
              b.m[d] = 1;
              continue;
            }
            const int a0 = std::max(v[d] - 1, 0), a1 = std::min(v[d] + 1, n);
            b.lo[d] = a0 * s + 1;
            b.m[d] = std::max((a1 - a0) * s - 1, 0);
            b.n *= b.m[d];
          }
          bx.push_back(b);
        }
    if (check_colours(bx, dim)) return 1;
    int nc = 0;
    greedy_box_colours(bx, dim, &nc);
    if (nc != (1 << dim)) return fail("vertex boxes: colours", nc, 1 << dim);
  }
  // random boxes, some empty
  for (int t = 0; t < 200; ++t) {
    const int dim = 2 + t % 2, nb = 1 + int(rng() % 40);
    std::vector<BoxRange> bx(nb);
    for (BoxRange &b : bx) {
      b.n = 1;
      for (int d = 0; d < 3; ++d) {
        b.lo[d] = d < dim ? int(rng() % 30) : 0;
        b.m[d] = d < dim ? int(rng() % 9) : 1;
        b.n *= b.m[d];
      }
    }
    if (check_colours(bx, dim)) return 1;
  }
  // batch groups and streams
  for (int t = 0; t < 300; ++t) {
    const int np = int(rng() % 24), ns = 1 + int(rng() % 5), mj = 1 + int(rng() % 4);
    const int64_t mb = 2048;
    std::vector<BatchPart> parts(np);
    for (BatchPart &p : parts) {
      p.multi = rng() % 4 != 0;
      p.dim = 2 + int(rng() % 2);
      p.fp32 = int(rng() % 2);
      p.lds = int(rng() % 3000);
      p.blocks = int64_t(rng() % 4000);
      p.cost = double(1 + rng() % 1000);
    }
    const std::vector<std::vector<int>> g = plan_batch_groups(parts, ns, mj, mb);
    std::vector<int> seen(np, 0);
    for (const std::vector<int> &grp : g) {
      if (grp.empty()) return fail("empty group", t, 0);
      int64_t nb = 0;
      for (int a : grp) {
        if (a < 0 || a >= np) return fail("part index", t, a);
        ++seen[a];
        nb += parts[a].blocks;
      }
      if (grp.size() > 1) {
        if (np <= ns) return fail("shared group with no more parts than streams", t, np);
        if (int(grp.size()) > mj) return fail("group larger than max_jobs", t, long(grp.size()));
        if (nb > mb) return fail("group over max_blocks", t, long(nb));
        for (int a : grp) {
          if (!parts[a].multi || parts[a].blocks >= mb) return fail("large or single part shared", t, a);
          if (parts[a].dim != parts[grp[0]].dim || parts[a].fp32 != parts[grp[0]].fp32)
            return fail("mixed dimension or precision", t, a);
        }
      }
    }
    for (int a = 0; a < np; ++a)
      if (seen[a] != 1) return fail("part not in exactly one group", t, a);
    std::vector<double> costs;
    for (const std::vector<int> &grp : g) {
      double c = 0.0;
      for (int a : grp) c += parts[a].cost;
      costs.push_back(c);
    }
    const std::vector<int> st = assign_streams(costs, ns);
    if (st.size() != costs.size()) return fail("stream count", long(st.size()), long(costs.size()));
    std::set<int> used;
    for (int s : st) {
      if (s < 0 || s >= ns) return fail("stream index", t, s);
      used.insert(s);
    }
    // with no more groups than streams every group has a stream of its own
    if (int(costs.size()) <= ns && used.size() != costs.size()) return fail("streams shared", t, long(used.size()));
  }
  std::printf("OK\n");
  return 0;
}

// Minimum-discarded-fill ordering and the ILU(0) (= IC(0) for the symmetric
// LOR patch matrices) factor it produces (Section 3.4, complexity in the
// computational-cost table: O(n log n) with a min-heap).
//
// Reading of the method: the matrix carries the Q1 stencil pattern (two grid
// points are coupled iff their offsets differ by at most one per direction).
// Eliminating node i applies a_jl -= a_ji a_il / a_ii to every pair of not yet
// eliminated neighbours (j, l) of i inside the pattern and drops the rest.
// The discarded fill of a candidate m is the sum, over pairs of its remaining
// neighbours j < l that are not coupled, of ((a_mj * a_ml) / a_mm)^2.  The
// node with the smallest value goes next; exact ties go to the smallest
// patch-local index.  Every float64 operation below is written in a fixed
// order (and the file is compiled without contraction) so that an
// independent implementation following the same order agrees bit for bit.
#include <algorithm>
#include <cmath>
#include <queue>
#include <vector>

#include "lor_internal.h"

namespace lor {

namespace {

struct Stencil {
  int dim, ns, center;
  int off[27][3];
  bool coupled[27][27];
  int rel[27][27];     // slot of (o_l - o_j), -1 if outside the stencil
  int mirror[27];
  explicit Stencil(int d) : dim(d) {
    ns = d == 3 ? 27 : 9;
    center = ns / 2;
    for (int s = 0; s < ns; ++s) {
      off[s][0] = s % 3 - 1;
      off[s][1] = (s / 3) % 3 - 1;
      off[s][2] = d == 3 ? s / 9 - 1 : 0;
    }
    for (int a = 0; a < ns; ++a) {
      int mo[3] = {-off[a][0], -off[a][1], -off[a][2]};
      mirror[a] = slot(mo);
      for (int b = 0; b < ns; ++b) {
        int dlt[3];
        bool ok = true;
        for (int t = 0; t < 3; ++t) {
          dlt[t] = off[b][t] - off[a][t];
          if (dlt[t] < -1 || dlt[t] > 1) ok = false;
        }
        coupled[a][b] = ok;
        rel[a][b] = ok ? slot(dlt) : -1;
      }
    }
  }
  int slot(const int *o) const {
    int s = (o[0] + 1) + 3 * (o[1] + 1);
    if (dim == 3) s += 9 * (o[2] + 1);
    return s;
  }
};

struct HeapItem {
  double d;
  int idx;
  int ver;
};
struct HeapCmp {  // min-heap on (d, idx)
  bool operator()(const HeapItem &a, const HeapItem &b) const {
    if (a.d != b.d) return a.d > b.d;
    if (a.idx != b.idx) return a.idx > b.idx;
    return a.ver > b.ver;
  }
};

}  // namespace

// Reverse Cuthill-McKee (Cuthill and McKee 1969, reversed), one of the
// orderings Section 3.4 compares: on the stencil graph of the box (the values
// play no part), start from a node of minimum degree (smallest index among
// them), number the not yet numbered neighbours of each numbered node in
// increasing degree (ties to the smallest index), breadth first, and reverse.
std::vector<int> rcm_order(int dim, const int *m) {
  const Stencil st(dim);
  const int mx = m[0], my = m[1], mz = dim == 3 ? m[2] : 1;
  const int n = mx * my * mz;
  std::vector<int> deg(n, 0);
  auto for_nbrs = [&](int i, auto &&fn) {
    const int c[3] = {i % mx, (i / mx) % my, i / (mx * my)};
    for (int s = 0; s < st.ns; ++s) {
      if (s == st.center) continue;
      const int q[3] = {c[0] + st.off[s][0], c[1] + st.off[s][1], c[2] + st.off[s][2]};
      if (q[0] >= 0 && q[0] < mx && q[1] >= 0 && q[1] < my && q[2] >= 0 && q[2] < mz)
        fn(q[0] + mx * (q[1] + my * q[2]));
    }
  };
  for (int i = 0; i < n; ++i) for_nbrs(i, [&](int) { ++deg[i]; });
  std::vector<char> numbered(n, 0);
  std::vector<int> cm;
  cm.reserve(n);
  auto by_degree = [&](int a, int b) { return deg[a] != deg[b] ? deg[a] < deg[b] : a < b; };
  while (int(cm.size()) < n) {
    int start = -1;
    for (int i = 0; i < n; ++i)
      if (!numbered[i] && (start < 0 || by_degree(i, start))) start = i;
    numbered[start] = 1;
    size_t head = cm.size();
    cm.push_back(start);
    while (head < cm.size()) {
      const int u = cm[head++];
      int nxt[26], k = 0;
      for_nbrs(u, [&](int v) {
        if (!numbered[v]) nxt[k++] = v;
      });
      std::sort(nxt, nxt + k, by_degree);
      for (int t = 0; t < k; ++t) {
        numbered[nxt[t]] = 1;
        cm.push_back(nxt[t]);
      }
    }
  }
  std::reverse(cm.begin(), cm.end());
  return cm;
}

int mdf_factor(int dim, const int *m, std::vector<double> &a, int ordering, MdfResult &out) {
  const Stencil st(dim);
  const int ns = st.ns, C = st.center;
  const int mx = m[0], my = m[1], mz = dim == 3 ? m[2] : 1;
  const int n = mx * my * mz;
  std::vector<int> nb(size_t(n) * ns, -1);
  for (int i = 0; i < n; ++i) {
    int c[3] = {i % mx, (i / mx) % my, i / (mx * my)};
    for (int s = 0; s < ns; ++s) {
      int q[3] = {c[0] + st.off[s][0], c[1] + st.off[s][1], c[2] + st.off[s][2]};
      if (q[0] >= 0 && q[0] < mx && q[1] >= 0 && q[1] < my && q[2] >= 0 && q[2] < mz)
        nb[size_t(i) * ns + s] = q[0] + mx * (q[1] + my * q[2]);
      else
        a[size_t(i) * ns + s] = 0.0;
    }
  }
  std::vector<char> elim(n, 0);
  out.L.assign(size_t(n) * ns, 0.0);
  out.D.assign(n, 0.0);
  out.order.clear();
  out.order.reserve(n);

  auto disc = [&](int mm) -> double {
    int nbr[27], k = 0;
    const size_t base = size_t(mm) * ns;
    for (int s = 0; s < ns; ++s) {
      int j = nb[base + s];
      if (s != C && j >= 0 && !elim[j]) nbr[k++] = s;
    }
    double acc = 0.0;
    const double amm = a[base + C];
    for (int x = 0; x < k; ++x)
      for (int y = x + 1; y < k; ++y) {
        if (st.coupled[nbr[x]][nbr[y]]) continue;
        double f = (a[base + nbr[x]] * a[base + nbr[y]]) / amm;
        acc = acc + f * f;
      }
    return acc;
  };

  // returns the number of uneliminated neighbours written to nbr
  auto eliminate = [&](int i, int *nbr) -> int {
    const size_t bi = size_t(i) * ns;
    const double piv = a[bi + C];
    if (!(std::isfinite(piv) && piv > 0.0)) return -1;
    out.D[i] = piv;
    int k = 0;
    for (int s = 0; s < ns; ++s) {
      int j = nb[bi + s];
      if (s != C && j >= 0 && !elim[j]) nbr[k++] = s;
    }
    for (int x = 0; x < k; ++x) {
      const int sj = nbr[x];
      const int j = nb[bi + sj];
      const double lji = a[bi + sj] / piv;
      out.L[bi + sj] = lji;
      out.L[size_t(j) * ns + st.mirror[sj]] = lji;
      for (int y = 0; y < k; ++y) {
        const int sl = nbr[y];
        if (!st.coupled[sj][sl]) continue;
        const double t = (a[bi + sj] * a[bi + sl]) / piv;
        double &dst = a[size_t(j) * ns + st.rel[sj][sl]];
        dst = dst - t;
      }
    }
    elim[i] = 1;
    return k;
  };

  int nbr[27];
  if (ordering == ORD_NATURAL || ordering == ORD_RCM) {
    std::vector<int> fixed;
    if (ordering == ORD_RCM) fixed = rcm_order(dim, m);
    for (int t = 0; t < n; ++t) {
      const int i = ordering == ORD_RCM ? fixed[t] : t;
      if (eliminate(i, nbr) < 0) return LOR_EPIVOT;
      out.order.push_back(i);
    }
  } else {
    std::vector<double> dv(n);
    std::vector<int> ver(n, 0);
    std::priority_queue<HeapItem, std::vector<HeapItem>, HeapCmp> heap;
    for (int i = 0; i < n; ++i) {
      dv[i] = disc(i);
      heap.push({dv[i], i, 0});
    }
    while (int(out.order.size()) < n) {
      HeapItem it = heap.top();
      heap.pop();
      if (elim[it.idx] || it.ver != ver[it.idx]) continue;
      const int i = it.idx;
      out.order.push_back(i);
      int k = eliminate(i, nbr);
      if (k < 0) return LOR_EPIVOT;
      const size_t bi = size_t(i) * ns;
      for (int x = 0; x < k; ++x) {
        int j = nb[bi + nbr[x]];
        dv[j] = disc(j);
        ++ver[j];
        heap.push({dv[j], j, ver[j]});
      }
    }
  }

  // dependency levels of the forward sweep, rows grouped by level
  std::vector<int> pos(n), lev(n, 0);
  for (int t = 0; t < n; ++t) pos[out.order[t]] = t;
  out.earlier.assign(n, 0);
  int depth = 0;
  for (int t = 0; t < n; ++t) {
    const int i = out.order[t];
    int best = 0, mask = 0;
    for (int s = 0; s < ns; ++s) {
      int j = nb[size_t(i) * ns + s];
      if (s == C || j < 0) continue;
      if (pos[j] < t) {
        mask |= 1 << s;
        best = std::max(best, lev[j] + 1);
      }
    }
    lev[i] = best;
    out.earlier[i] = mask;
    depth = std::max(depth, best + 1);
  }
  std::vector<int> cnt(depth + 1, 0);
  for (int i = 0; i < n; ++i) cnt[lev[i] + 1]++;
  for (int d = 0; d < depth; ++d) cnt[d + 1] += cnt[d];
  out.level_ptr = cnt;
  out.sched.assign(n, 0);
  std::vector<int> fill(cnt.begin(), cnt.end() - 1);
  for (int t = 0; t < n; ++t) {
    const int i = out.order[t];
    out.sched[fill[lev[i]]++] = i;
  }
  return LOR_OK;
}

}  // namespace lor

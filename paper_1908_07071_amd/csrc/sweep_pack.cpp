// Packs the ILU(0) triangular sweeps of one patch level for the wavefront
// kernel (layout documented at kChunkLanes in lor_internal.h).
//
// Rows are taken in dependency-level order (forward: first level first,
// backward: last level first).  Each level becomes one step of the current
// chunk; when a row no longer fits the chunk's lanes, the chunk is closed and
// the rest of the level continues as a step of the next chunk (rows of one
// level are independent, so any split is a valid schedule).  A row with more
// than kLaneCouplings couplings takes an aligned lane pair; single-lane rows
// fill the lanes left free by that alignment first.
#include <algorithm>
#include <cstring>
#include <vector>

#include "lor_internal.h"

namespace lor {

namespace {

template <typename T>
void put(std::vector<uint32_t> &rec, int word, T v) {
  std::memcpy(&rec[word], &v, sizeof(T));
}

static_assert(kMaxCouplings <= 2 * kLaneCouplings, "every row must fit a lane pair");

// One lane's share of a row: couplings [c0, c1) of the row's list.
struct LaneRec {
  int row = -1, step = 0, c0 = 0, c1 = 0;
  bool paired = false, second = false;
};

struct Chunk {
  std::vector<LaneRec> lane = std::vector<LaneRec>(kChunkLanes);
  std::vector<int> holes;  // free lanes below `next`
  int next = 0, nsteps = 0, w = 0, q = 1;
  bool split = false;
  // places row i (n couplings) in step st; false if the lanes are full
  bool place(int i, int n, int st) {
    if (n > kLaneCouplings) {
      const int a = (next + 1) & ~1;
      if (a + 1 >= kChunkLanes) return false;
      if (a != next) holes.push_back(next);
      const int n0 = std::min(kLaneCouplings, 2 * ((n + 3) / 4));
      lane[a] = LaneRec{i, st, 0, n0, true, false};
      lane[a + 1] = LaneRec{i, st, n0, n, true, true};
      next = a + 2;
      split = true;
      return true;
    }
    int l;
    if (!holes.empty()) {
      l = holes.back();
      holes.pop_back();
    } else if (next < kChunkLanes) {
      l = next++;
    } else {
      return false;
    }
    lane[l] = LaneRec{i, st, 0, n, false, false};
    return true;
  }
};

}  // namespace

template <typename T>
std::vector<char> pack_sweep(const MdfResult &res, int dim, const int *m, bool fwd) {
  const int NS = dim == 3 ? 27 : 9, C = NS / 2;
  const int depth = int(res.level_ptr.size()) - 1;
  const int mx = m[0], my = m[1], mz = dim == 3 ? m[2] : 1;
  auto couplings = [&](int i, std::vector<int> &slots) {
    slots.clear();
    const int ix = i % mx, iy = (i / mx) % my, iz = i / (mx * my);
    for (int s = 0; s < NS; ++s) {
      if (s == C) continue;
      const int jx = ix + s % 3 - 1, jy = iy + (s / 3) % 3 - 1, jz = iz + (dim == 3 ? s / 9 - 1 : 0);
      if (jx < 0 || jx >= mx || jy < 0 || jy >= my || jz < 0 || jz >= mz) continue;
      const bool earlier = (res.earlier[i] >> s) & 1;
      if (earlier == fwd) slots.push_back(s);
    }
  };
  std::vector<Chunk> chunks(1);
  std::vector<int> slots;
  for (int q = 0; q < depth; ++q) {
    const int d = fwd ? q : depth - 1 - q;
    int st = -1;  // this level's step in the current chunk (opened by its first row)
    for (int t = res.level_ptr[d]; t < res.level_ptr[d + 1]; ++t) {
      const int i = res.sched[t];
      couplings(i, slots);
      const int n = int(slots.size());
      for (;;) {
        Chunk &c = chunks.back();
        if (st < 0 && c.nsteps == 63) {
          chunks.emplace_back();
          continue;
        }
        const int s_try = st < 0 ? c.nsteps : st;
        if (c.place(i, n, s_try)) {
          if (st < 0) st = c.nsteps++;
          break;
        }
        chunks.emplace_back();  // full: the rest of the level goes to a new chunk
        st = -1;
      }
    }
  }
  if (chunks.back().nsteps == 0) chunks.pop_back();
  const int hw = sweep_head_words<T>(fwd), sz = int(sizeof(T)) / 4;
  // Lanes of a chunk sorted by record length, longest first (lane pairs
  // first, on even lanes): quad q of the chunk is then loaded by a prefix of
  // the lanes, so a 128-byte line (8 lanes' quads) is fetched only where
  // most of it is used.  Rows keep their steps; the lane of a row is free.
  for (Chunk &c : chunks) {
    struct Unit {
      int first, lanes, quads;
    };
    std::vector<Unit> units;
    for (int l = 0; l < kChunkLanes; ++l) {
      const LaneRec &r = c.lane[l];
      if (r.row < 0 || r.second) continue;
      const int q0 = sweep_quads<T>(fwd, r.c1 - r.c0);
      if (r.paired) {
        const LaneRec &r2 = c.lane[l + 1];
        units.push_back({l, 2, std::max(q0, sweep_quads<T>(fwd, r2.c1 - r2.c0))});
      } else {
        units.push_back({l, 1, q0});
      }
    }
    std::stable_sort(units.begin(), units.end(), [](const Unit &a, const Unit &b) {
      return a.lanes != b.lanes ? a.lanes > b.lanes : a.quads > b.quads;
    });
    std::vector<LaneRec> sorted(kChunkLanes);
    int l = 0;
    for (const Unit &u : units)
      for (int k = 0; k < u.lanes; ++k) sorted[l++] = c.lane[u.first + k];
    c.lane.swap(sorted);
  }
  // per-lane quads, chunk width and size
  std::vector<std::vector<int>> lane_q(chunks.size(), std::vector<int>(64, 1));
  for (size_t ci = 0; ci < chunks.size(); ++ci) {
    Chunk &c = chunks[ci];
    for (int l = 0; l < kChunkLanes; ++l) {
      const LaneRec &r = c.lane[l];
      if (r.row < 0) continue;
      c.w = std::max(c.w, (r.c1 - r.c0 + 1) & ~1);
      lane_q[ci][l] = sweep_quads<T>(fwd, r.c1 - r.c0);
      c.q = std::max(c.q, lane_q[ci][l]);
    }
  }
  auto header = [](const Chunk &c) {
    return uint32_t(c.q) | (uint32_t(c.nsteps) << 8) | (uint32_t(c.w) << 16) | (c.split ? kChunkSplit : 0u);
  };
  int64_t bytes = kSweepHeader;
  for (const Chunk &c : chunks) bytes += int64_t(c.q) * 64 * 16;
  std::vector<char> out(bytes, 0);
  const int32_t nch = int32_t(chunks.size());
  const uint32_t h0 = chunks.empty() ? 0u : header(chunks[0]);
  std::memcpy(out.data(), &nch, 4);
  std::memcpy(out.data() + 4, &h0, 4);
  for (int l = 0; l < 64; ++l) out[16 + l] = char(chunks.empty() ? 0 : lane_q[0][l]);
  int64_t base = kSweepHeader;
  std::vector<uint32_t> rec;
  for (size_t ci = 0; ci < chunks.size(); ++ci) {
    const Chunk &c = chunks[ci];
    const int words = c.q * 4;
    auto nextq = [&](int l) -> uint32_t { return ci + 1 < chunks.size() ? uint32_t(lane_q[ci + 1][l]) : 0u; };
    for (int l = 0; l < kChunkLanes; ++l) {
      const LaneRec &r = c.lane[l];
      if (r.row < 0) {  // lanes without a row still learn their next size
        const uint32_t w0 = nextq(l) << 22;
        std::memcpy(out.data() + base + 16 * l, &w0, 4);
        continue;
      }
      rec.assign(words, 0u);
      rec[0] = uint32_t(r.row & 0xFFFF) | (uint32_t(r.step) << 16) | (nextq(l) << 22) | kSweepValid |
               (r.paired ? kSweepPaired : 0u) | (r.second ? kSweepSecond : 0u);
      if (!fwd && !r.second) put<T>(rec, 1, T(1.0 / res.D[r.row]));
      couplings(r.row, slots);
      uint32_t mask = 0;
      for (int q = r.c0; q < r.c1; ++q) {
        mask |= 1u << slots[q];
        put<T>(rec, hw + 1 + (q - r.c0) * sz, T(res.L[size_t(r.row) * NS + slots[q]]));
      }
      rec[hw] = mask;
      for (int qd = 0; qd < c.q; ++qd)
        std::memcpy(out.data() + base + 16 * (int64_t(qd) * 64 + l), &rec[4 * qd], 16);
    }
    // lane 63: header of the next chunk
    const uint32_t hn = ci + 1 < chunks.size() ? header(chunks[ci + 1]) : 0u;
    std::memcpy(out.data() + base + 16 * 63, &hn, 4);
    base += int64_t(c.q) * 64 * 16;
  }
  return out;
}

template std::vector<char> pack_sweep<double>(const MdfResult &, int, const int *, bool);
template std::vector<char> pack_sweep<float>(const MdfResult &, int, const int *, bool);

}  // namespace lor

// Packs the ILU(0) triangular sweeps of one patch level for the wavefront
// kernel (layout documented at kChunkRows in lor_internal.h).
//
// Rows are taken in dependency-level order (forward: first level first,
// backward: last level first).  A level holding more than kChunkRows rows is
// split into consecutive steps (rows of one level are independent, so any
// split is a valid schedule).  Consecutive steps are grouped into chunks of at
// most kChunkRows rows; lanes 0.. take the chunk's rows in order and lane 63
// carries the header of the next chunk.
#include <cstring>
#include <vector>

#include "lor_internal.h"

namespace lor {

namespace {

template <typename T>
void put(std::vector<uint32_t> &rec, int word, T v) {
  std::memcpy(&rec[word], &v, sizeof(T));
}

}  // namespace

template <typename T>
std::vector<char> pack_sweep(const MdfResult &res, int dim, const int *m, bool fwd) {
  const int NS = dim == 3 ? 27 : 9, C = NS / 2;
  const int depth = int(res.level_ptr.size()) - 1;
  const int mx = m[0], my = m[1], mz = dim == 3 ? m[2] : 1;
  int dl[27];
  for (int s = 0; s < NS; ++s) {
    const int ox = s % 3 - 1, oy = (s / 3) % 3 - 1, oz = dim == 3 ? s / 9 - 1 : 0;
    dl[s] = ox + mx * (oy + my * oz);
  }
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
  // steps in sweep order, each a list of rows
  std::vector<std::vector<int>> steps;
  for (int q = 0; q < depth; ++q) {
    const int d = fwd ? q : depth - 1 - q;
    std::vector<int> cur;
    for (int t = res.level_ptr[d]; t < res.level_ptr[d + 1]; ++t) {
      cur.push_back(res.sched[t]);
      if (int(cur.size()) == kChunkRows) {
        steps.push_back(cur);
        cur.clear();
      }
    }
    if (!cur.empty()) steps.push_back(cur);
  }
  // chunks of consecutive steps with at most kChunkRows rows
  struct Chunk {
    int first, nsteps, rows, w, q;
  };
  std::vector<Chunk> chunks;
  std::vector<int> slots;
  for (size_t s = 0; s < steps.size();) {
    Chunk c{int(s), 0, 0, 0, 0};
    while (s < steps.size() && c.rows + int(steps[s].size()) <= kChunkRows && c.nsteps < 63) {
      for (int i : steps[s]) {
        couplings(i, slots);
        c.w = std::max(c.w, int(slots.size()));
      }
      c.rows += int(steps[s].size());
      ++c.nsteps;
      ++s;
    }
    c.w = (c.w + 1) & ~1;  // whole pairs
    c.q = sweep_quads<T>(fwd, c.w);
    chunks.push_back(c);
  }
  auto header = [](const Chunk &c) {
    return uint32_t(c.q) | (uint32_t(c.nsteps) << 8) | (uint32_t(c.w) << 16);
  };
  // quads each lane loads in each chunk: its own record (at least the word
  // that tells it the size of its next record); lane 63 only the header
  const int hw = sweep_head_words<T>(fwd), pw = sweep_pair_words<T>();
  std::vector<std::vector<int>> lane_q(chunks.size(), std::vector<int>(64, 1));
  for (size_t ci = 0; ci < chunks.size(); ++ci) {
    const Chunk &c = chunks[ci];
    int lane = 0;
    for (int st = 0; st < c.nsteps; ++st)
      for (int i : steps[c.first + st]) {
        couplings(i, slots);
        const int w = int(slots.size() + 1) & ~1;
        lane_q[ci][lane++] = sweep_quads<T>(fwd, w);
      }
  }
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
    int lane = 0;
    for (int st = 0; st < c.nsteps; ++st) {
      for (int i : steps[c.first + st]) {
        rec.assign(words, 0u);
        rec[0] = uint32_t(i & 0xFFFF) | (uint32_t(st) << 16) | (nextq(lane) << 22) | (1u << 31);
        if (!fwd) put<T>(rec, 1, T(1.0 / res.D[i]));
        couplings(i, slots);
        for (size_t q = 0; q < slots.size(); ++q) {
          const int pr = int(q) / 2, hi = int(q) % 2;
          const int w0 = hw + pr * pw;
          put<T>(rec, w0 + hi * int(sizeof(T)) / 4, T(res.L[size_t(i) * NS + slots[q]]));
          const uint32_t o = uint32_t(uint16_t(int16_t(dl[slots[q]])));
          rec[w0 + pw - 1] |= hi ? (o << 16) : o;
        }
        for (int qd = 0; qd < c.q; ++qd)
          std::memcpy(out.data() + base + 16 * (int64_t(qd) * 64 + lane), &rec[4 * qd], 16);
        ++lane;
      }
    }
    for (; lane < 63; ++lane) {  // lanes without a row still learn their next size
      const uint32_t w0 = nextq(lane) << 22;
      std::memcpy(out.data() + base + 16 * lane, &w0, 4);
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

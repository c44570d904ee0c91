// Host check of the sweep-block packer.  For random symmetric positive
// definite 27-point (3D) and 9-point (2D) stencils on boxes of several
// shapes, the library's MDF factorization gives the IC(0) factor and its
// dependency levels; the packed forward and backward blocks are then
// replayed the way the patch kernel consumes them (double-buffered chunks,
// partial per-lane record loads, lane-pair partial sums, steps in order) and
// compared with a direct level-ordered triangular solve:
//   forward  w_i = y_i - sum_{earlier m} l_im w_m
//   backward y_i = w_i / D_i - sum_{later m} l_mi y_m
// The replay also checks the protocol's invariants: every load stays inside
// the block, pair partners agree, a step never reads a row it writes, every
// row is written exactly once.  Exit status 0 when every case passes.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "lor_internal.h"

using namespace lor;

static int failures = 0;
#define CHECK(c, ...)                                 \
  do {                                                \
    if (!(c)) {                                       \
      std::printf("FAIL line %d: ", __LINE__);        \
      std::printf(__VA_ARGS__);                       \
      std::printf("\n");                              \
      ++failures;                                     \
      return false;                                   \
    }                                                 \
  } while (0)

template <typename T>
static T word_as(const uint32_t *w, int b) {
  T v;
  std::memcpy(&v, w + b, sizeof(T));
  return v;
}

// Replays one packed block on Y (one wavefront of 64 lanes) of a dim-D box
// with extents m (the slot table of the kernel: offset of stencil slot s).
template <typename T, bool FWD>
static bool replay(const std::vector<char> &blk, std::vector<T> &Y, int dim, const int *m) {
  constexpr int QM = sweep_quads<T>(FWD, kLaneCouplings);
  constexpr int H = sweep_head_words<T>(FWD), SZ = sizeof(T) / 4;
  const int n = int(Y.size());
  const int NS = dim == 3 ? 27 : 9, C = NS / 2;
  int tab[28];
  for (int s = 0; s < 28; ++s)
    tab[s] = s < NS ? (s % 3 - 1) + m[0] * ((s / 3) % 3 - 1) + (dim == 3 ? m[0] * m[1] * (s / 9 - 1) : 0) : 0;
  int nch;
  uint32_t hdr;
  std::memcpy(&nch, blk.data(), 4);
  std::memcpy(&hdr, blk.data() + 4, 4);
  int myq[64];
  for (int l = 0; l < 64; ++l) myq[l] = static_cast<unsigned char>(blk[16 + l]);
  int64_t src = kSweepHeader;
  std::vector<int> written(n, 0);
  std::vector<uint32_t> R(64 * 4 * QM);
  for (int c = 0; c < nch; ++c) {
    for (int l = 0; l < 64; ++l) {
      CHECK(myq[l] <= QM, "lane %d loads %d quads, more than %d", l, myq[l], QM);
      for (int q = 0; q < QM; ++q) {
        const int64_t off = q < myq[l] ? src + 16 * (int64_t(q) * 64 + l) : kSweepZero;
        CHECK(off + 16 <= int64_t(blk.size()), "chunk %d lane %d reads past the block", c, l);
        std::memcpy(&R[(l * QM + q) * 4], blk.data() + off, 16);
      }
    }
    auto rec = [&](int l) { return &R[l * QM * 4]; };
    const int Q = hdr & 0xFF, nsteps = (hdr >> 8) & 0xFF, npairs = int((hdr >> 16) & 0xFF) / 2;
    const bool split = hdr & kChunkSplit;
    CHECK(Q >= 1 && Q <= QM && npairs <= kLaneCouplings / 2, "chunk %d header Q %d pairs %d", c, Q, npairs);
    const uint32_t hnext = rec(63)[0];
    int nq[64];
    for (int l = 0; l < 64; ++l) nq[l] = l == 63 ? 1 : int((rec(l)[0] >> 22) & 0x1F);
    for (int s = 0; s < nsteps; ++s) {
      T part[64];
      bool wr[64] = {};
      std::vector<int> reads, writes;
      for (int l = 0; l < 64; ++l) {
        part[l] = T(0);
        const uint32_t d0 = rec(l)[0];
        const int step = (d0 & kSweepValid) ? int((d0 >> 16) & 0x3F) : -1;
        if (step != s) continue;
        CHECK(l != 63, "the header lane holds a row");
        const int row = int(d0 & 0xFFFF);
        const bool second = d0 & kSweepSecond, paired = d0 & kSweepPaired;
        CHECK(row < n, "row %d outside the box (%d rows)", row, n);
        CHECK(split || (!paired && !second), "split row in a chunk without the split flag");
        T acc0 = FWD ? Y[row] : Y[row] * word_as<T>(rec(l), 1);
        if (split) acc0 = second ? T(0) : acc0;
        T acc1 = T(0);
        uint32_t mask = rec(l)[H];
        CHECK(!((mask >> C) & 1) && (mask >> NS) == 0, "slot mask %x of row %d", mask, row);
        CHECK(__builtin_popcount(mask) <= 2 * npairs, "row %d has more couplings than the chunk's width", row);
        for (int k = 0; k < 2 * npairs; ++k) {
          const int sl = mask ? __builtin_ctz(mask) : 27;
          mask &= mask - 1;
          const int j = row + tab[sl];
          CHECK(j >= 0 && j < n, "neighbour outside the box");
          const T v = word_as<T>(rec(l), H + 1 + k * SZ);
          CHECK(sl != 27 || v == T(0), "padding coupling with a nonzero value");
          if (j != row) reads.push_back(j);
          (k % 2 ? acc1 : acc0) -= v * Y[j];
        }
        part[l] = acc0 + acc1;
        if (!second) {
          wr[l] = true;
          writes.push_back(row);
        }
        if (paired) {
          const uint32_t dp = rec(l ^ 1)[0];
          CHECK((dp & kSweepValid) && int(dp & 0xFFFF) == row && int((dp >> 16) & 0x3F) == s &&
                    bool(dp & kSweepSecond) != second,
                "lane pair %d/%d does not hold one row", l, l ^ 1);
        }
      }
      for (int a : reads)
        for (int b : writes) CHECK(a != b, "row %d read and written in one step", a);
      T out[64];
      for (int l = 0; l < 64; ++l)
        if (wr[l]) out[l] = (rec(l)[0] & kSweepPaired) ? part[l] + part[l ^ 1] : part[l];
      for (int l = 0; l < 64; ++l)
        if (wr[l]) {
          const int row = int(rec(l)[0] & 0xFFFF);
          Y[row] = out[l];
          ++written[row];
        }
    }
    src += int64_t(Q) * 64 * 16;
    hdr = hnext;
    for (int l = 0; l < 64; ++l) myq[l] = nq[l];
  }
  CHECK(src == int64_t(blk.size()), "block of %lld bytes, chunks end at %lld", (long long)blk.size(),
        (long long)src);
  for (int i = 0; i < n; ++i) CHECK(written[i] == 1, "row %d written %d times", i, written[i]);
  return true;
}

// Random symmetric stencil rows with negative couplings, strictly
// diagonally dominant (n x 3^dim, slot order, x fastest).
static std::vector<double> random_rows(int dim, const int *m, unsigned seed) {
  const int NS = dim == 3 ? 27 : 9, C = NS / 2;
  const int mx = m[0], my = m[1], mz = dim == 3 ? m[2] : 1, n = mx * my * mz;
  auto nb = [&](int i, int s) {
    const int ix = i % mx, iy = (i / mx) % my, iz = i / (mx * my);
    const int jx = ix + s % 3 - 1, jy = iy + (s / 3) % 3 - 1, jz = iz + (dim == 3 ? s / 9 - 1 : 0);
    if (jx < 0 || jx >= mx || jy < 0 || jy >= my || jz < 0 || jz >= mz) return -1;
    return jx + mx * (jy + my * jz);
  };
  std::mt19937 g(seed);
  std::uniform_real_distribution<double> U(0.2, 1.5);
  std::vector<double> rows(size_t(n) * NS, 0.0);
  for (int i = 0; i < n; ++i)
    for (int s = C + 1; s < NS; ++s) {
      const int j = nb(i, s);
      if (j < 0) continue;
      const double w = U(g);
      rows[size_t(i) * NS + s] = -w;
      rows[size_t(j) * NS + (NS - 1 - s)] = -w;
    }
  for (int i = 0; i < n; ++i) {
    double d = 0.3;
    for (int s = 0; s < NS; ++s) d -= rows[size_t(i) * NS + s];
    rows[size_t(i) * NS + C] = d;
  }
  return rows;
}

template <typename T>
static void run_case(int dim, const int *m, std::vector<double> rows, unsigned seed, const char *kind) {
  const int NS = dim == 3 ? 27 : 9, C = NS / 2;
  const int mx = m[0], my = m[1], mz = dim == 3 ? m[2] : 1, n = mx * my * mz;
  auto nb = [&](int i, int s) {
    const int ix = i % mx, iy = (i / mx) % my, iz = i / (mx * my);
    const int jx = ix + s % 3 - 1, jy = iy + (s / 3) % 3 - 1, jz = iz + (dim == 3 ? s / 9 - 1 : 0);
    if (jx < 0 || jx >= mx || jy < 0 || jy >= my || jz < 0 || jz >= mz) return -1;
    return jx + mx * (jy + my * jz);
  };
  std::mt19937 g(seed + 1000);
  std::uniform_real_distribution<double> U(0.2, 1.5);
  MdfResult res;
  if (mdf_factor(dim, m, rows, false, res) != LOR_OK) {
    std::printf("FAIL: MDF factorization\n");
    ++failures;
    return;
  }
  std::vector<double> y0(n);
  for (auto &v : y0) v = U(g) - 0.85;
  const int depth = int(res.level_ptr.size()) - 1;
  std::vector<double> w = y0;
  for (int d = 0; d < depth; ++d)
    for (int t = res.level_ptr[d]; t < res.level_ptr[d + 1]; ++t) {
      const int i = res.sched[t];
      double a = w[i];
      for (int s = 0; s < NS; ++s) {
        const int j = s == C ? -1 : nb(i, s);
        if (j >= 0 && ((res.earlier[i] >> s) & 1)) a -= res.L[size_t(i) * NS + s] * w[j];
      }
      w[i] = a;
    }
  std::vector<double> y = w;
  for (int d = depth - 1; d >= 0; --d)
    for (int t = res.level_ptr[d]; t < res.level_ptr[d + 1]; ++t) {
      const int i = res.sched[t];
      double a = y[i] / res.D[i];
      for (int s = 0; s < NS; ++s) {
        const int j = s == C ? -1 : nb(i, s);
        if (j >= 0 && !((res.earlier[i] >> s) & 1)) a -= res.L[size_t(i) * NS + s] * y[j];
      }
      y[i] = a;
    }
  auto relerr = [](const std::vector<T> &a, const std::vector<double> &b) {
    double e = 0, s = 0;
    for (size_t i = 0; i < b.size(); ++i) {
      e = std::max(e, std::fabs(double(a[i]) - b[i]));
      s = std::max(s, std::fabs(b[i]));
    }
    return s > 0 ? e / s : e;
  };
  std::vector<T> Y(n);
  for (int i = 0; i < n; ++i) Y[i] = T(y0[i]);
  const int f0 = failures;
  const bool okf = replay<T, true>(pack_sweep<T>(res, dim, m, true), Y, dim, m);
  const double ef = relerr(Y, w);
  const bool okb = okf && replay<T, false>(pack_sweep<T>(res, dim, m, false), Y, dim, m);
  const double eb = relerr(Y, y);
  const double tol = sizeof(T) == 4 ? 2e-6 : 1e-13;
  const bool ok = okf && okb && failures == f0 && ef < tol && eb < tol;
  if (!ok && failures == f0) ++failures;
  std::printf("%-6s %-6s %dD %2dx%2dx%2d depth %4d: forward %.1e backward %.1e %s\n", kind,
              sizeof(T) == 4 ? "float" : "double", dim, mx, my, mz, depth, ef, eb, ok ? "ok" : "FAILED");
}

// Usage: sweep_pack_check [file]; the optional file holds further cases as
// text: the number of cases, then per case "dim m0 m1 m2" and the n x 3^dim
// stencil rows (for example LOR patch stencils).
int main(int argc, char **argv) {
  const int cases[][4] = {{3, 11, 11, 11}, {3, 11, 11, 5}, {3, 5, 11, 5}, {3, 5, 5, 5}, {3, 3, 3, 3}, {3, 1, 1, 1},
                          {3, 23, 23, 23}, {3, 13, 7, 9}, {2, 11, 11, 1}, {2, 29, 29, 1}, {2, 1, 3, 1}};
  unsigned seed = 1;
  for (const auto &c : cases) {
    const std::vector<double> rows = random_rows(c[0], c + 1, seed);
    run_case<float>(c[0], c + 1, rows, seed, "random");
    run_case<double>(c[0], c + 1, rows, seed, "random");
    ++seed;
  }
  if (argc > 1) {
    FILE *f = std::fopen(argv[1], "r");
    int ncase = 0;
    if (!f || std::fscanf(f, "%d", &ncase) != 1) {
      std::printf("FAIL: cannot read %s\n", argv[1]);
      return 1;
    }
    for (int c = 0; c < ncase; ++c) {
      int dim, m[3];
      if (std::fscanf(f, "%d %d %d %d", &dim, &m[0], &m[1], &m[2]) != 4) {
        std::printf("FAIL: bad case header\n");
        return 1;
      }
      const size_t cnt = size_t(m[0]) * m[1] * (dim == 3 ? m[2] : 1) * (dim == 3 ? 27 : 9);
      std::vector<double> rows(cnt);
      for (double &v : rows)
        if (std::fscanf(f, "%lf", &v) != 1) {
          std::printf("FAIL: short rows\n");
          return 1;
        }
      run_case<float>(dim, m, rows, seed, "file");
      run_case<double>(dim, m, rows, seed, "file");
      ++seed;
    }
    std::fclose(f);
  }
  std::printf("%s (%d failures)\n", failures ? "FAILED" : "all ok", failures);
  return failures != 0;
}

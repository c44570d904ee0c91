// C ABI of the library: set-up driver, operator / preconditioner application
// and the conjugate gradient loop.  See include/lor.h for the contract of
// every entry point.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <thread>
#include <tuple>
#include <vector>

#include "host_plan.h"
#include "lor_handle.h"

static_assert(LOR_ORD_MDF == ORD_MDF && LOR_ORD_NATURAL == ORD_NATURAL && LOR_ORD_RCM == ORD_RCM,
              "ordering codes of the C ABI and of the set-up agree");

namespace {

thread_local char g_detail[512] = "";

int hip_fail(hipError_t e, const char *what, int line) {
  std::snprintf(g_detail, sizeof(g_detail), "%s failed at lor_api.cpp:%d: %s", what, line,
                hipGetErrorString(e));
  return LOR_EHIP;
}

int invalid(const char *why, int line) {
  std::snprintf(g_detail, sizeof(g_detail), "invalid at lor_api.cpp:%d: %s", line, why);
  return LOR_EINVAL;
}

#define HIPCHK(x)                                          \
  do {                                                     \
    hipError_t e_ = (x);                                   \
    if (e_ != hipSuccess) return hip_fail(e_, #x, __LINE__); \
  } while (0)

inline int nslots(int dim) { return dim == 3 ? 27 : 9; }

// 1D transfer table for fine level k of a patch direction of the given type
// (0: vertex on the low boundary, 1: interior vertex, 2: high boundary).
// Built on a two-element line; the tables only depend on the position of the
// patch range relative to its element(s).
XferTab build_xfer(const lor_handle &h, int k, int type) {
  XferTab t{};
  const int nn = 2;
  const int v = type == 0 ? 0 : (type == 1 ? 1 : 2);
  const std::vector<int> &Xf = h.kept[k], &Xc = h.kept[k + 1];
  const int sf = int(Xf.size()) - 1, sc = int(Xc.size()) - 1;
  auto range = [&](int s, int &lo, int &hi) {
    lo = v > 0 ? (v - 1) * s + 1 : 1;
    hi = v < nn ? (v + 1) * s - 1 : nn * s - 1;
  };
  int flo, fhi, clo, chi;
  range(sf, flo, fhi);
  range(sc, clo, chi);
  t.mf = fhi - flo + 1;
  t.mc = chi - clo + 1;
  const std::vector<double> &x = h.gllx;
  for (int f = 0; f < t.mf; ++f) {
    const int G = flo + f;
    const int e = std::min(G / sf, nn - 1);
    const int a = Xf[G - e * sf];
    int cidx[2];
    double w[2];
    auto it = std::find(Xc.begin(), Xc.end(), a);
    if (it != Xc.end()) {
      cidx[0] = cidx[1] = e * sc + int(it - Xc.begin());
      w[0] = 1.0;
      w[1] = 0.0;
    } else {
      int hi = 0;
      while (Xc[hi] < a) ++hi;
      const int lo = hi - 1;
      const double xl = x[Xc[lo]], xh = x[Xc[hi]];
      cidx[0] = e * sc + lo;
      cidx[1] = e * sc + hi;
      w[0] = (xh - x[a]) / (xh - xl);
      w[1] = (x[a] - xl) / (xh - xl);
    }
    for (int b = 0; b < 2; ++b) {
      t.pc[f][b] = cidx[b] - clo;  // may be -1 or mc: on the patch boundary
      t.pw[f][b] = w[b];
      const int cl = cidx[b] - clo;
      if (w[b] != 0.0 && cl >= 0 && cl < t.mc) {
        const int c = t.rcnt[cl]++;
        t.rf[cl][c] = f;
        t.rw[cl][c] = w[b];
      }
    }
  }
  return t;
}

struct PatchBox {
  int lo[3], m[3], n;
};

PatchBox patch_box(const lor_handle &h, int j, int k) {
  PatchBox b{};
  const int s = int(h.kept[k].size()) - 1;
  const int nv0 = h.n[0] + 1, nv1 = h.n[1] + 1;
  const int v[3] = {j % nv0, (j / nv0) % nv1, h.dim == 3 ? j / (nv0 * nv1) : 0};
  b.n = 1;
  for (int d = 0; d < 3; ++d) {
    if (d >= h.dim) {
      b.lo[d] = 0;
      b.m[d] = 1;
      continue;
    }
    const int lo = v[d] > 0 ? (v[d] - 1) * s + 1 : 1;
    const int hi = v[d] < h.n[d] ? (v[d] + 1) * s - 1 : h.n[d] * s - 1;
    b.lo[d] = lo;
    b.m[d] = std::max(hi - lo + 1, 0);
    b.n *= b.m[d];
  }
  return b;
}

int build_coarse(lor_handle &h, const std::vector<double> &st0, hipStream_t st) {
  const int dim = h.dim, p = h.p;
  const int ncx = h.n[0] - 1, ncy = h.n[1] - 1, ncz = dim == 3 ? h.n[2] - 1 : 1;
  h.nc = std::max(ncx, 0) * std::max(ncy, 0) * std::max(ncz, 0);
  if (h.nc <= 0) {
    h.nc = 0;
    return LOR_OK;
  }
  const int NS = nslots(dim);
  const int ng[3] = {h.md.ng[0], h.md.ng[1], h.md.ng[2]};
  const int64_t npts = h.npts[0];
  std::vector<double> A0(size_t(h.nc) * h.nc, 0.0);
  auto cidx = [&](const int *v) -> int {
    for (int d = 0; d < dim; ++d)
      if (v[d] <= 0 || v[d] >= h.n[d]) return -1;
    return (v[0] - 1) + ncx * ((v[1] - 1) + (dim == 3 ? ncy * (v[2] - 1) : 0));
  };
  // parents of a fine grid index in one direction
  auto parents = [&](int d, int g, int *pv, double *pw) {
    const int e = std::min(g / p, h.n[d] - 1);
    const int a = g - e * p;
    pv[0] = e;
    pw[0] = 1.0 - h.gllx[a];
    pv[1] = e + 1;
    pw[1] = h.gllx[a];
  };
  unsigned nth = h.opt.nthreads > 0 ? unsigned(h.opt.nthreads) : std::max(1u, std::thread::hardware_concurrency());
  nth = std::min<unsigned>(nth, 64);
  std::vector<std::thread> pool;
  std::atomic<int> next{0};
  auto work = [&]() {
    for (;;) {
      const int c = next.fetch_add(1);
      if (c >= h.nc) break;
      const int v[3] = {c % ncx + 1, (c / ncx) % ncy + 1, dim == 3 ? c / (ncx * ncy) + 1 : 0};
      double *row = A0.data() + size_t(c) * h.nc;
      const int w1 = 2 * p - 1;
      const int cnt = dim == 3 ? w1 * w1 * w1 : w1 * w1;
      for (int t = 0; t < cnt; ++t) {
        const int o[3] = {t % w1, (t / w1) % w1, t / (w1 * w1)};
        int g[3] = {0, 0, 0};
        double wv = 1.0;
        for (int d = 0; d < dim; ++d) {
          g[d] = (v[d] - 1) * p + 1 + o[d];
          const int a = g[d] - (v[d] - 1) * p;
          wv *= a <= p ? h.gllx[a] : 1.0 - h.gllx[a - p];
        }
        const int64_t gi = g[0] + int64_t(ng[0]) * (g[1] + (dim == 3 ? int64_t(ng[1]) * g[2] : 0));
        for (int s = 0; s < NS; ++s) {
          const int off[3] = {s % 3 - 1, (s / 3) % 3 - 1, dim == 3 ? s / 9 - 1 : 0};
          int q[3] = {0, 0, 0};
          bool ok = true;
          for (int d = 0; d < dim; ++d) {
            q[d] = g[d] + off[d];
            if (q[d] <= 0 || q[d] >= ng[d] - 1) ok = false;
          }
          if (!ok) continue;
          const double kij = st0[size_t(s) * npts + gi] * wv;
          int pv[3][2];
          double pw[3][2];
          for (int d = 0; d < dim; ++d) parents(d, q[d], pv[d], pw[d]);
          for (int cc = 0; cc < (1 << dim); ++cc) {
            int vv[3] = {0, 0, 0};
            double w = kij;
            for (int d = 0; d < dim; ++d) {
              const int b = (cc >> d) & 1;
              vv[d] = pv[d][b];
              w *= pw[d][b];
            }
            const int ci = cidx(vv);
            if (ci >= 0 && w != 0.0) row[ci] += w;
          }
        }
      }
    }
  };
  for (unsigned t = 0; t < nth; ++t) pool.emplace_back(work);
  for (auto &th : pool) th.join();
  HIPCHK(h.alloc(&h.d_A0inv, size_t(h.nc) * h.nc));
  HIPCHK(hipMemcpyAsync(h.d_A0inv, A0.data(), A0.size() * sizeof(double), hipMemcpyHostToDevice, st));
  int rc = coarse_inverse(h.nc, h.d_A0inv, st);
  if (rc != LOR_OK) return rc;
  if (h.opt.precision == LOR_PREC_MIXED) {
    // the float32 preconditioner applies the coarse inverse in float32
    // storage too: half the bytes of the largest array of each application
    HIPCHK(h.alloc(&h.d_A0inv_f, size_t(h.nc) * h.nc));
    HIPCHK(launch_to_float(h.d_A0inv, h.d_A0inv_f, int64_t(h.nc) * h.nc, st));
    HIPCHK(hipStreamSynchronize(st));
    h.release(h.d_A0inv);
    h.d_A0inv = nullptr;
  }
  return LOR_OK;
}

int build_patches(lor_handle &h, const std::vector<std::vector<double>> &hst, hipStream_t st) {
  const int dim = h.dim, NS = nslots(dim), L = h.L, nf = L - 1;
  const bool mixed = h.opt.precision == LOR_PREC_MIXED;
  const int nv[3] = {h.n[0] + 1, h.n[1] + 1, dim == 3 ? h.n[2] + 1 : 1};
  h.J = nv[0] * nv[1] * nv[2];
  const int nfl = std::max(nf, 1);
  h.order_off.assign(size_t(h.J) * nf + 1, 0);
  h.sched_off.assign(size_t(h.J) * nf + 1, 0);
  // offsets into the concatenated orders (known sizes up front)
  {
    int32_t acc = 0;
    for (int j = 0; j < h.J; ++j)
      for (int k = 0; k < nf; ++k) {
        h.order_off[size_t(j) * nf + k] = acc;
        acc += patch_box(h, j, k).n;
      }
    h.order_off[size_t(h.J) * nf] = acc;
    h.order_all.assign(acc, 0);
  }
  std::vector<std::vector<int>> lvls(size_t(h.J) * nfl);
  std::vector<std::vector<char>> blocks(size_t(h.J) * nfl * 2);  // forward, backward
  std::atomic<int> next{0};
  std::atomic<int> err{LOR_OK};
  const int ntask = h.J * nf;
  auto work = [&]() {
    MdfResult res;
    std::vector<double> rows;
    for (;;) {
      const int task = next.fetch_add(1);
      if (task >= ntask || err.load() != LOR_OK) break;
      const int j = task / nf, k = task % nf;
      PatchBox b = patch_box(h, j, k);
      if (b.n <= 0) continue;
      const int64_t np = h.npts[k];
      const int lng0 = h.md.n[0] * (int(h.kept[k].size()) - 1) + 1;
      const int lng1 = h.md.n[1] * (int(h.kept[k].size()) - 1) + 1;
      rows.assign(size_t(b.n) * NS, 0.0);
      for (int i = 0; i < b.n; ++i) {
        const int ix = i % b.m[0], iy = (i / b.m[0]) % b.m[1], iz = i / (b.m[0] * b.m[1]);
        const int64_t g = int64_t(b.lo[0] + ix) +
                          int64_t(lng0) * (int64_t(b.lo[1] + iy) + (dim == 3 ? int64_t(lng1) * (b.lo[2] + iz) : 0));
        for (int s = 0; s < NS; ++s) rows[size_t(i) * NS + s] = hst[k][size_t(s) * np + g];
      }
      int rc = mdf_factor(dim, b.m, rows, h.opt.ordering, res);
      if (rc != LOR_OK) {
        err.store(rc);
        break;
      }
      if (mixed) {
        blocks[2 * (size_t(j) * nfl + k)] = pack_sweep<float>(res, dim, b.m, true);
        blocks[2 * (size_t(j) * nfl + k) + 1] = pack_sweep<float>(res, dim, b.m, false);
      } else {
        blocks[2 * (size_t(j) * nfl + k)] = pack_sweep<double>(res, dim, b.m, true);
        blocks[2 * (size_t(j) * nfl + k) + 1] = pack_sweep<double>(res, dim, b.m, false);
      }
      std::copy(res.order.begin(), res.order.end(), h.order_all.begin() + h.order_off[size_t(j) * nf + k]);
      lvls[size_t(j) * nfl + k] = res.level_ptr;
    }
  };
  unsigned nth = h.opt.nthreads > 0 ? unsigned(h.opt.nthreads) : std::max(1u, std::thread::hardware_concurrency());
  nth = std::min<unsigned>(nth, 64);
  std::vector<std::thread> thr;
  for (unsigned t = 0; t < nth; ++t) thr.emplace_back(work);
  for (auto &t : thr) t.join();
  if (err.load() != LOR_OK) return err.load();
  {
    int32_t acc = 0;
    for (int t = 0; t < ntask; ++t) {
      h.sched_off[t] = acc;
      acc += int32_t(lvls[t].size());
    }
    h.sched_off[ntask] = acc;
    h.sched_all.reserve(acc);
    for (int t = 0; t < ntask; ++t) h.sched_all.insert(h.sched_all.end(), lvls[t].begin(), lvls[t].end());
  }
  std::vector<int64_t> off(blocks.size(), -1);
  int64_t total = 0;
  for (size_t t = 0; t < blocks.size(); ++t) {
    if (blocks[t].empty()) continue;
    off[t] = total;
    total += align16(int64_t(blocks[t].size()));
  }
  h.fac_bytes = total;
  HIPCHK(h.alloc(&h.d_fac, size_t(std::max<int64_t>(total, 16))));
  HIPCHK(h.alloc(&h.d_fac_off, off.size()));
  {
    // upload through a staging buffer covering a contiguous range of the pool
    // (one copy per ~64 MiB rather than one per block; each block is freed
    // once staged)
    constexpr size_t kStage = size_t(64) << 20;
    std::vector<char> stage;
    int64_t r0 = 0;  // pool offset of stage[0]
    auto flush = [&]() -> hipError_t {
      if (stage.empty()) return hipSuccess;
      hipError_t e = hipMemcpyAsync(h.d_fac + r0, stage.data(), stage.size(), hipMemcpyHostToDevice, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      r0 += int64_t(stage.size());
      stage.clear();
      return e;
    };
    for (size_t t = 0; t < blocks.size(); ++t) {
      if (blocks[t].empty()) continue;
      if (!stage.empty() && size_t(off[t] - r0) + blocks[t].size() > kStage) HIPCHK(flush());
      stage.resize(size_t(off[t] - r0));  // alignment padding (zero)
      stage.insert(stage.end(), blocks[t].begin(), blocks[t].end());
      std::vector<char>().swap(blocks[t]);
    }
    HIPCHK(flush());
  }
  HIPCHK(hipMemcpyAsync(h.d_fac_off, off.data(), off.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));  // host blocks are freed on return
  // transfer tables
  std::vector<XferTab> xt(size_t(std::max(nf, 1)) * 3);
  for (int k = 0; k < nf; ++k)
    for (int t = 0; t < 3; ++t) xt[size_t(k) * 3 + t] = build_xfer(h, k, t);
  HIPCHK(h.alloc(&h.d_xfer, xt.size()));
  HIPCHK(hipMemcpyAsync(h.d_xfer, xt.data(), xt.size() * sizeof(XferTab), hipMemcpyHostToDevice, st));
  // kernel arguments
  PatchArgs &pa = h.pa;
  pa.md = h.md;
  pa.nlev = L;
  for (int d = 0; d < 3; ++d) pa.nv[d] = nv[d];
  for (int k = 0; k < L; ++k) {
    const int s = int(h.kept[k].size()) - 1;
    pa.s[k] = s;
    if (mixed) {
      const int W = dim == 3 ? rec_width<3, float>() : rec_width<2, float>();
      float *f32 = nullptr;
      HIPCHK(h.alloc(&f32, size_t(W) * h.npts[k]));
      HIPCHK(launch_sym_stencil(h.d_stencil[k], h.npts[k], dim, f32, true, st));
      pa.stencil[k] = reinterpret_cast<const double *>(f32);  // read as float by the kernel
    } else {
      const int W = dim == 3 ? rec_width<3, double>() : rec_width<2, double>();
      double *f64 = nullptr;
      HIPCHK(h.alloc(&f64, size_t(W) * h.npts[k]));
      HIPCHK(launch_sym_stencil(h.d_stencil[k], h.npts[k], dim, f64, false, st));
      pa.stencil[k] = f64;
    }
    pa.npts[k] = h.npts[k];
    for (int d = 0; d < 3; ++d) pa.lng[k][d] = d < dim ? h.n[d] * s + 1 : 1;
  }
  pa.xfer = h.d_xfer;
  pa.fac = h.d_fac;
  pa.fac_off = h.d_fac_off;
  // LDS of the largest patch: X_0, R_0 and B_1, the coarser levels inside
  // R_0's space.  That space must hold X_1, R_1 and X_k, B_k, R_k (k >= 2)
  // for every patch shape (each direction interior, 2 s - 1 points, or at
  // the boundary, s - 1).
  auto level_n = [&](int k, int mask) {
    int ps = 1;
    for (int d = 0; d < dim; ++d) {
      const bool interior = ((mask >> d) & 1) && h.n[d] >= 2;
      ps *= std::max(interior ? 2 * pa.s[k] - 1 : pa.s[k] - 1, 0);
    }
    return ps;
  };
  for (int mask = 0; mask < (1 << dim); ++mask) {
    int coarse = L > 1 ? 2 * level_n(1, mask) : 0;
    for (int k = 2; k < L; ++k) coarse += 3 * level_n(k, mask);
    if (coarse > level_n(0, mask))  // never for the kept-point rule
      return invalid("coarse patch levels do not fit the level-0 residual's LDS space", __LINE__);
  }
  const int full = (1 << dim) - 1;
  const int tot = 2 * level_n(0, full) + (L > 1 ? level_n(1, full) : 0);
  pa.lds_total = tot;
  pa.fp32 = mixed ? 1 : 0;
  pa.pou = h.opt.prolong_weights == LOR_PROLONG_POU ? 1 : 0;
  pa.plain = h.opt.deterministic ? 1 : 0;
  pa.color = -1;
  pa.perm = nullptr;
  // patch buckets: patches by decreasing work (rows over all smoothed levels;
  // interior patches, then face, edge and corner ones), so that the large
  // patches start in the first round of the launch and the small ones fill
  // its tail
  {
    std::vector<int64_t> work(h.J, 0);
    for (int j = 0; j < h.J; ++j)
      for (int k = 0; k < nf; ++k) work[j] += patch_box(h, j, k).n;
    std::vector<int> perm(h.J);
    for (int j = 0; j < h.J; ++j) perm[j] = j;
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return work[a] > work[b]; });
    HIPCHK(h.alloc(&h.d_perm, size_t(std::max(h.J, 1))));
    HIPCHK(hipMemcpyAsync(h.d_perm, perm.data(), perm.size() * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  if (size_t(tot) * (mixed ? sizeof(float) : sizeof(double)) > 160 * 1024)
    return invalid("patch vectors exceed the 160 KiB LDS of a CU (polynomial degree too high)", __LINE__);
  HIPCHK(prepare_patch_vcycle(pa));
  return LOR_OK;
}

int setup_impl(lor_handle &h, hipStream_t st) {
  const int dim = h.dim, p = h.p;
  gll_nodes_weights(p, h.gllx, h.gllw);
  lagrange_derivative(h.gllx, h.D);
  h.kept = kept_points(p);
  h.L = int(h.kept.size());
  MeshDims &md = h.md;
  md.dim = dim;
  md.p = p;
  md.dirichlet = h.bc == LOR_BC_DIRICHLET ? 1 : 0;
  for (int d = 0; d < 3; ++d) {
    md.n[d] = d < dim ? h.n[d] : 1;
    md.ng[d] = d < dim ? h.n[d] * p + 1 : 1;
    md.nu[d] = d < dim ? (md.dirichlet ? md.ng[d] - 2 : md.ng[d]) : 1;
  }
  h.nfine = int64_t(md.ng[0]) * md.ng[1] * md.ng[2];
  h.nel = int64_t(md.n[0]) * md.n[1] * md.n[2];
  const int Q = p + 1;
  const int nq = dim == 3 ? Q * Q * Q : Q * Q;
  const bool dg = h.method != LOR_CG;
  h.ncg = int64_t(md.nu[0]) * md.nu[1] * md.nu[2];
  h.ndofs = dg ? h.nel * nq : h.ncg;
  HIPCHK(h.alloc(&h.d_verts, h.verts.size()));
  HIPCHK(h.alloc(&h.d_gllx, Q));
  HIPCHK(h.alloc(&h.d_gllw, Q));
  HIPCHK(h.alloc(&h.d_D, Q * Q));
  HIPCHK(hipMemcpyAsync(h.d_verts, h.verts.data(), h.verts.size() * 8, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h.d_gllx, h.gllx.data(), Q * 8, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h.d_gllw, h.gllw.data(), Q * 8, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h.d_D, h.D.data(), Q * Q * 8, hipMemcpyHostToDevice, st));
  HIPCHK(h.alloc(&h.d_coords, size_t(h.nfine) * dim));
  if (h.nodes.empty()) {
    HIPCHK(launch_node_coords(md, h.d_verts, h.d_gllx, h.d_coords, st));
  } else {
    // curved elements: the caller's node coordinates (x fastest, dim per
    // node) into the SoA layout
    std::vector<double> soa(size_t(h.nfine) * dim);
    for (int64_t g = 0; g < h.nfine; ++g)
      for (int r = 0; r < dim; ++r) soa[size_t(r) * h.nfine + g] = h.nodes[size_t(g) * dim + r];
    HIPCHK(hipMemcpyAsync(h.d_coords, soa.data(), soa.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  const int ncomp = dim == 3 ? 6 : 3;
  // on request the plane kernel of 3D CG with straight elements and b = 1
  // recomputes the geometric factors from the vertices instead of storing them
  h.geo_onfly = !dg && h.coef.empty() && h.nodes.empty() && apply_cg_uses_skeleton(md) &&
                h.opt.operator_geometry == LOR_GEOM_ONFLY;
  if (!h.geo_onfly) HIPCHK(h.alloc(&h.d_G, size_t(h.nel) * ncomp * nq));
  HIPCHK(h.alloc(&h.d_wdet, size_t(h.nel) * nq));
  int *bad;
  HIPCHK(h.alloc(&bad, 1));
  HIPCHK(hipMemsetAsync(bad, 0, sizeof(int), st));
  if (!h.coef.empty()) {
    HIPCHK(h.alloc(&h.d_coef, h.coef.size()));
    HIPCHK(hipMemcpyAsync(h.d_coef, h.coef.data(), h.coef.size() * 8, hipMemcpyHostToDevice, st));
  }
  if (h.nodes.empty())
    HIPCHK(launch_geom_cg(md, h.d_verts, h.d_gllx, h.d_gllw, h.d_coef, h.d_G, h.d_wdet, bad, st));
  else
    HIPCHK(launch_geom_nodal(md, h.d_coords, h.d_D, h.d_gllw, h.d_coef, h.d_G, h.d_wdet, bad, st));
  int hb = 0;
  HIPCHK(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hb) return LOR_EJACOBIAN;
  if (dg) {
    // faces: geometry and penalty (eq. ip / eq. br2), face records, diag(A_DG)
    const int QF = dim == 3 ? Q * Q : Q;
    h.nfaces = dg_face_count(md);
    HIPCHK(h.alloc(&h.d_fg, size_t(h.nfaces) * 8 * QF));
    HIPCHK(h.alloc(&h.d_dinv, size_t(h.ndofs)));
    HIPCHK(launch_dg_face_geom(md, h.d_verts, h.d_gllx, h.d_gllw, h.d_wdet, h.method, h.penalty,
                               h.d_fg, st));
    HIPCHK(launch_dg_diag(md, h.d_G, h.d_D, h.d_fg, h.d_dinv, st));
  }
  h.npart = std::max(kRedBlocks, apply_cg_blocks(md, dg));
  HIPCHK(hipEventCreate(&h.ev0));
  HIPCHK(hipEventCreate(&h.ev1));
  if (!md.dirichlet) return LOR_OK;  // Neumann: operator only
  // LOR hierarchy stencils (Sections 3.1, 3.3)
  const int NS = nslots(dim);
  const double gm = 0.5 / std::sqrt(3.0);
  const double g0 = 0.5 - gm, g1 = 0.5 + gm;
  std::vector<std::vector<double>> hst(h.L);
  for (int k = 0; k < h.L; ++k) {
    const int s = int(h.kept[k].size()) - 1;
    h.npts[k] = int64_t(md.n[0] * s + 1) * (md.n[1] * s + 1) * (dim == 3 ? md.n[2] * s + 1 : 1);
    HIPCHK(h.alloc(&h.d_stencil[k], size_t(NS) * h.npts[k]));
    HIPCHK(launch_lor_stencil(md, s, h.kept[k].data(), h.d_coords, g0, g1, h.d_coef, h.d_stencil[k], st));
    hst[k].resize(size_t(NS) * h.npts[k]);
    HIPCHK(hipMemcpyAsync(hst[k].data(), h.d_stencil[k], hst[k].size() * 8, hipMemcpyDeviceToHost, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  if (box_mode(h.opt.patch_mode)) {
    int rc = build_boxes(h, hst, st);
    if (rc != LOR_OK) return rc;
    if (h.opt.patch_mode == LOR_PATCH_VERTEX_ISO) {
      rc = build_coarse(h, hst[0], st);
      if (rc != LOR_OK) return rc;
    }
    HIPCHK(hipStreamSynchronize(st));
    h.has_prec = true;
    return LOR_OK;
  }
  int rc = build_patches(h, hst, st);
  if (rc != LOR_OK) return rc;
  rc = build_coarse(h, hst[0], st);
  if (rc != LOR_OK) return rc;
  HIPCHK(hipStreamSynchronize(st));
  h.has_prec = true;
  return LOR_OK;
}

// Allocates the device workspace of one solve for handle h.  Buffers are
// appended to `owned` (hipMalloc'ed, freed by the owner) and counted in
// `bytes`; the pinned scalar copy is returned in w.h_scal.
int work_alloc(const lor_handle &h, Work &w, std::vector<void *> &owned, size_t &bytes,
               std::vector<size_t> *sizes = nullptr) {
  auto get = [&](double **ptr, size_t count) -> hipError_t {
    void *p = nullptr;
    const size_t b = std::max<size_t>(count * sizeof(double), 16);
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) return e;
    owned.push_back(p);
    if (sizes) sizes->push_back(b);
    bytes += b;
    *ptr = static_cast<double *>(p);
    return hipSuccess;
  };
  const int64_t N = h.ndofs;
  const int Q = h.p + 1;
  const int nq = h.dim == 3 ? Q * Q * Q : Q * Q, QF = h.dim == 3 ? Q * Q : Q;
  const bool dg = h.method != LOR_CG;
  HIPCHK(get(&w.r, N));
  HIPCHK(get(&w.z, N));
  HIPCHK(get(&w.p, N));
  HIPCHK(get(&w.q, N));
  HIPCHK(get(&w.rold, N));
  HIPCHK(get(&w.tmp, N));
  HIPCHK(get(&w.scal, S_COUNT));
  HIPCHK(get(&w.part, h.npart));
  HIPCHK(get(&w.part2, h.npart));
  if (h.nc > 0) {
    HIPCHK(get(&w.rc, h.nc));
    HIPCHK(get(&w.xc, h.nc));
  }
  if (!dg && apply_cg_uses_skeleton(h.md)) HIPCHK(get(&w.yE, size_t(h.nel) * nq));
  if (dg) {
    HIPCHK(get(&w.fo, size_t(h.nfaces) * 8 * QF));
    HIPCHK(get(&w.rL, size_t(h.ncg)));
    HIPCHK(get(&w.zL, size_t(h.ncg)));
  }
  HIPCHK(hipHostMalloc((void **)&w.h_scal, S_COUNT * sizeof(double), 0));
  return LOR_OK;
}

// Records an event pair around a launch when timing is on.
struct Span {
  lor_handle *h;
  int which;
  hipStream_t st;
  hipEvent_t a = nullptr;
  Span(lor_handle *hh, int w, hipStream_t s) : h(hh), which(w), st(s) {
    if (h->timing && !h->capturing && (a = h->next_event())) (void)hipEventRecord(a, st);
  }
  ~Span() {
    if (!a) return;
    hipEvent_t b = h->next_event();
    if (b && hipEventRecord(b, st) == hipSuccess) h->tspans[which].push_back({a, b});
  }
};

// The preconditioner in three parts, so that a batch can put the patch
// corrections of several right-hand sides of one matrix into one launch:
//   pre:     (DG) r_L = E^T r ; the coarse correction z_L = P_0 A_0^-1 P_0^T r_L
//            (it initialises z_L);
//   patches: z_L += sum_j P_j^T V_j(P_j r_L) (or the box patches, the network);
//   post:    (DG) z = D_B^-1 r on element-boundary nodes + E z_L.
// (r_L, z_L) are (r, z) for CG and the handle's L-vectors for DG (eq. dg-as).
void patch_io(const lor_handle *h, const Work &w, const double *r, double *z, const double **pr,
              double **pz) {
  if (h->method == LOR_CG) {
    *pr = r;
    *pz = z;
  } else {
    *pr = w.rL;
    *pz = w.zL;
  }
}

int apply_P_pre(lor_handle *h, Work &w, const double *r, double *z, const double *flag,
                hipStream_t st) {
  const double *pr;
  double *pz;
  patch_io(h, w, r, z, &pr, &pz);
  if (h->method != LOR_CG) HIPCHK(launch_dg_restrict(h->md, r, w.rL, flag, st));
  if (h->opt.patch_mode == LOR_PATCH_SINGLE) return LOR_OK;  // the box V-cycle writes z_L
  if (h->nc > 0) {
    Span sp(h, LOR_T_COARSE, st);
    HIPCHK(launch_coarse_restrict(h->md, h->d_gllx, pr, w.rc, st));
    if (h->d_A0inv_f)
      HIPCHK(launch_gemv_f32(h->nc, h->d_A0inv_f, w.rc, w.xc, flag, st));
    else
      HIPCHK(launch_gemv(h->nc, h->d_A0inv, w.rc, w.xc, flag, st));
    HIPCHK(launch_coarse_prolong(h->md, h->d_gllx, w.xc, pz, flag, st));
  } else {
    HIPCHK(launch_fill(pz, h->ncg, 0.0, st));
  }
  return LOR_OK;
}

int apply_P_patches(lor_handle *h, Work &w, const double *r, double *z, const double *flag,
                    hipStream_t st) {
  const double *pr;
  double *pz;
  patch_io(h, w, r, z, &pr, &pz);
  Span sp(h, LOR_T_PATCH, st);
  if (h->opt.patch_mode == LOR_PATCH_SINGLE || box_mode(h->opt.patch_mode))
    return apply_boxes(h, pr, pz, flag, st);
  if (h->nn && h->nn_mode == LOR_NN_REPLACE) return nn_apply_patches(h->nn, pr, pz, flag, st);
  if (h->nn && h->nn_mode == LOR_NN_WARMSTART) return nn_apply_patches_warm(h->nn, pr, pz, flag, st);
  HIPCHK(launch_patch_vcycle(h->pa, h->J, pr, pz, flag, st));
  return LOR_OK;
}

int apply_P_post(lor_handle *h, Work &w, const double *r, double *z, const double *flag,
                 hipStream_t st) {
  if (h->method != LOR_CG) HIPCHK(launch_dg_prolong_jacobi(h->md, r, h->d_dinv, w.zL, z, flag, st));
  return LOR_OK;
}

// CG: eq. as.  DG: eq. dg-as, z = D_B^-1 r on element-boundary nodes plus
// E B E^T r.
int apply_P_impl(lor_handle *h, Work &w, const double *r, double *z, const double *flag,
                 hipStream_t st) {
  int rc = apply_P_pre(h, w, r, z, flag, st);
  if (rc == LOR_OK) rc = apply_P_patches(h, w, r, z, flag, st);
  if (rc == LOR_OK) rc = apply_P_post(h, w, r, z, flag, st);
  return rc;
}

// Whether the batch can put the patch corrections of several right-hand
// sides of this handle into one launch (vertex patches, atomics, V-cycles).
bool multi_rhs_patches(const lor_handle *h) {
  return h->J > 0 && h->opt.patch_mode == LOR_PATCH_VERTEX && !h->pa.plain &&
         !(h->nn && h->nn_mode != LOR_NN_OFF);
}

}  // namespace

size_t apply_P_scratch_doubles(const lor_handle *h) {
  auto up = [](int64_t n) { return size_t((std::max<int64_t>(n, 0) + 31) / 32 * 32); };
  size_t need = 2 * up(h->nc);
  if (h->method != LOR_CG) need += 2 * up(h->ncg);
  return need;
}

int apply_P_scratch(lor_handle *h, double *scratch, size_t cap, const double *r, double *z,
                    hipStream_t st) {
  const size_t need = apply_P_scratch_doubles(h);
  if (need > cap) {
    std::snprintf(g_detail, sizeof(g_detail),
                  "lor_apply_P_noalloc: this handle needs %zu bytes of scratch, the static "
                  "buffer holds %zu",
                  need * sizeof(double), cap * sizeof(double));
    return LOR_ENOMEM;
  }
  auto up = [](int64_t n) { return size_t((std::max<int64_t>(n, 0) + 31) / 32 * 32); };
  Work w = h->w;  // operator buffers are not touched by B
  double *c = scratch;
  w.rc = c;
  c += up(h->nc);
  w.xc = c;
  c += up(h->nc);
  if (h->method != LOR_CG) {
    w.rL = c;
    c += up(h->ncg);
    w.zL = c;
  } else {
    w.rL = w.zL = nullptr;
  }
  const bool was = h->capturing;
  h->capturing = true;  // no timing events: nothing is created or recorded
  const int rc = apply_P_impl(h, w, r, z, nullptr, st);
  h->capturing = was;
  return rc;
}

namespace {

int apply_A_impl(lor_handle *h, Work &w, const double *x, double *y, double *partials,
                 const double *flag, hipStream_t st) {
  Span sp(h, LOR_T_APPLY_A, st);
  if (h->method != LOR_CG) HIPCHK(launch_dg_face(h->md, h->d_D, h->d_fg, x, w.fo, flag, st));
  GeoArgs geo{h->d_verts, h->d_gllx, h->d_gllw};
  HIPCHK(launch_apply_cg(h->md, h->d_G, h->d_D, x, y, partials, flag, st,
                         h->method != LOR_CG ? w.fo : nullptr, w.yE, h->geo_onfly ? &geo : nullptr));
  return LOR_OK;
}

constexpr int kChunk = 8;         // iterations between host checks / per captured graph
constexpr int kBatchStreams = 4;  // worker streams of a batched solve (HIP's hardware queues)
constexpr int64_t kJobBlocks = 2048;  // patch blocks of a shared launch: about 2/3 of one
                                      // round of resident patches on 256 CUs

// Enqueues x = 0, r = b, z = B r, p = z, rho = r.z and the scalars of a new
// solve (no memset nodes, so that the sequence can be captured).
int pcg_init(lor_handle *h, Work &w, const double *b, double *x, double rtol, int maxit,
             hipStream_t st) {
  const int64_t N = h->ndofs;
  double *s = w.scal;
  HIPCHK(launch_fill(x, N, 0.0, st));
  HIPCHK(launch_copy(w.r, b, N, st));
  HIPCHK(launch_fill(s, S_COUNT, 0.0, st));
  HIPCHK(launch_fill(s + S_TOL2, 1, rtol * rtol, st));
  HIPCHK(launch_fill(s + S_MAXIT, 1, double(maxit), st));
  const int nbv = red_blocks(N);
  HIPCHK(launch_dot_partials(b, b, N, w.part, nullptr, st));
  HIPCHK(launch_finalize(s, w.part, nbv, FIN_BB, nullptr, st));
  int rc = apply_P_impl(h, w, w.r, w.z, s, st);
  if (rc != LOR_OK) return rc;
  HIPCHK(launch_dot_partials(w.r, w.z, N, w.part, s, st));
  HIPCHK(launch_finalize(s, w.part, nbv, FIN_RHO, nullptr, st));
  HIPCHK(launch_copy(w.p, w.z, N, st));
  HIPCHK(launch_fill(w.q, N, 0.0, st));
  return LOR_OK;
}

// One (flexible) CG iteration in three parts around the preconditioner's
// patch corrections (see apply_P_pre): pre = q = A p, alpha, x and r, the
// recursive residual, and the preconditioner's first part; post = its last
// part, rho (and for FCG z.r_old), beta and p.  Every kernel returns at once
// after the device-side convergence flag is set, so the sequence can be
// replayed as a graph until the flag is seen on the host.
bool uses_fcg(const lor_handle *h) {
  // flexible CG whenever the preconditioner is not a fixed SPD operator
  // (float32 patch solves, or the nonlinear patch network)
  return h->opt.flexible != 0 || h->opt.precision == LOR_PREC_MIXED ||
         h->opt.prolong_weights == LOR_PROLONG_POU || (h->nn && h->nn_mode != LOR_NN_OFF);
}

int pcg_iter_pre(lor_handle *h, Work &w, double *x, hipStream_t st) {
  const int64_t N = h->ndofs;
  double *s = w.scal;
  const int nba = apply_cg_blocks(h->md, h->method != LOR_CG);
  const int nbv = red_blocks(N);
  int rc = apply_A_impl(h, w, w.p, w.q, w.part, s, st);
  if (rc != LOR_OK) return rc;
  HIPCHK(launch_finalize(s, w.part, nba, FIN_PQ, nullptr, st));
  HIPCHK(launch_cg_update(x, w.r, uses_fcg(h) ? w.rold : nullptr, w.p, w.q, N, s, w.part, st));
  HIPCHK(launch_finalize(s, w.part, nbv, FIN_RR, nullptr, st));
  return apply_P_pre(h, w, w.r, w.z, s, st);
}

int pcg_iter_post(lor_handle *h, Work &w, hipStream_t st) {
  const int64_t N = h->ndofs;
  double *s = w.scal;
  const bool fcg = uses_fcg(h);
  // the operator writes q completely (DG, or CG through the skeleton gather);
  // otherwise q is accumulated atomically and must be cleared each iteration
  const bool zero_q = h->method == LOR_CG && !apply_cg_uses_skeleton(h->md);
  const int nbv = red_blocks(N);
  int rc = apply_P_post(h, w, w.r, w.z, s, st);
  if (rc != LOR_OK) return rc;
  if (fcg)
    HIPCHK(launch_dot2_partials(w.z, w.r, w.rold, N, w.part, w.part2, s, st));
  else
    HIPCHK(launch_dot_partials(w.r, w.z, N, w.part, s, st));
  HIPCHK(launch_finalize(s, w.part, nbv, fcg ? FIN_FCG : FIN_RHO, fcg ? w.part2 : nullptr, st));
  HIPCHK(launch_p_update(w.p, zero_q ? w.q : nullptr, w.z, N, s, st));
  return LOR_OK;
}

// Enqueues `count` iterations of one solve.
int pcg_iterations(lor_handle *h, Work &w, double *x, int count, hipStream_t st) {
  for (int i = 0; i < count; ++i) {
    int rc = pcg_iter_pre(h, w, x, st);
    if (rc == LOR_OK) rc = apply_P_patches(h, w, w.r, w.z, w.scal, st);
    if (rc == LOR_OK) rc = pcg_iter_post(h, w, st);
    if (rc != LOR_OK) return rc;
  }
  return LOR_OK;
}

// Enqueues `count` iterations of up to kMaxRhs solves with the same handle in
// lockstep: the patch corrections of all of them in one launch.
int pcg_iterations_multi(lor_handle *h, Work *const *w, double *const *x, int n, int count,
                         hipStream_t st) {
  if (n < 1 || n > kMaxRhs) return LOR_EINVAL;
  const double *pr[kMaxRhs];
  double *pz[kMaxRhs];
  const double *fl[kMaxRhs];
  for (int k = 0; k < n; ++k) {
    patch_io(h, *w[k], w[k]->r, w[k]->z, &pr[k], &pz[k]);
    fl[k] = w[k]->scal;
  }
  for (int i = 0; i < count; ++i) {
    for (int k = 0; k < n; ++k) {
      int rc = pcg_iter_pre(h, *w[k], x[k], st);
      if (rc != LOR_OK) return rc;
    }
    {
      Span sp(h, LOR_T_PATCH, st);
      HIPCHK(launch_patch_vcycle_multi(h->pa, h->J, n, pr, pz, fl, st));
    }
    for (int k = 0; k < n; ++k) {
      int rc = pcg_iter_post(h, *w[k], st);
      if (rc != LOR_OK) return rc;
    }
  }
  return LOR_OK;
}

// Up to kMaxRhs right-hand sides of one handle, as one problem of a
// multi-problem patch launch.
struct PatchJob {
  lor_handle *h = nullptr;
  Work *w[kMaxRhs] = {};
  double *x[kMaxRhs] = {};
  int n = 0;
};

// The patch launch arguments of a job: the handle's, with the job's patch
// inputs, outputs and convergence flags (null flags: never stop).
PatchArgs job_patch_args(const PatchJob &jb, bool flags) {
  PatchArgs a = jb.h->pa;
  a.nrhs = jb.n;
  for (int k = 0; k < kMaxRhs; ++k) {
    a.rs[k] = nullptr;
    a.zs[k] = nullptr;
    a.flags[k] = nullptr;
  }
  for (int k = 0; k < jb.n; ++k) {
    patch_io(jb.h, *jb.w[k], jb.w[k]->r, jb.w[k]->z, &a.rs[k], &a.zs[k]);
    a.flags[k] = flags ? jb.w[k]->scal : nullptr;
  }
  return a;
}

// Enqueues `count` iterations of the solves of up to kMaxJobs jobs in
// lockstep: the patch corrections of all of them in one launch.
int pcg_iterations_jobs(const PatchJob *jobs, int njobs, int count, hipStream_t st) {
  if (njobs < 1 || njobs > kMaxJobs) return LOR_EINVAL;
  PatchArgs pa[kMaxJobs];
  for (int j = 0; j < njobs; ++j) pa[j] = job_patch_args(jobs[j], true);
  for (int i = 0; i < count; ++i) {
    for (int j = 0; j < njobs; ++j)
      for (int k = 0; k < jobs[j].n; ++k) {
        int rc = pcg_iter_pre(jobs[j].h, *jobs[j].w[k], jobs[j].x[k], st);
        if (rc != LOR_OK) return rc;
      }
    HIPCHK(launch_patch_vcycle_jobs(pa, njobs, st));
    for (int j = 0; j < njobs; ++j)
      for (int k = 0; k < jobs[j].n; ++k) {
        int rc = pcg_iter_post(jobs[j].h, *jobs[j].w[k], st);
        if (rc != LOR_OK) return rc;
      }
  }
  return LOR_OK;
}

// Enqueues the true residual ||b - A x||^2 (w.tmp receives b - A x) and
// copies the scalars to w.h_scal (synchronizes the stream).
int pcg_finish(lor_handle *h, Work &w, const double *b, const double *x, hipStream_t st) {
  const int64_t N = h->ndofs;
  const bool zero_q = h->method == LOR_CG && !apply_cg_uses_skeleton(h->md);
  if (zero_q) HIPCHK(launch_fill(w.tmp, N, 0.0, st));
  int rc = apply_A_impl(h, w, x, w.tmp, nullptr, nullptr, st);
  if (rc != LOR_OK) return rc;
  HIPCHK(launch_sub_dot(b, w.tmp, N, w.part, st, w.tmp));
  HIPCHK(launch_finalize(w.scal, w.part, red_blocks(N), FIN_RRTRUE, nullptr, st));
  HIPCHK(hipMemcpyAsync(w.h_scal, w.scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return LOR_OK;
}

constexpr int kMaxReplace = 4;  // residual replacements per solve

// Enqueues a restart of (flexible) CG from the true residual left in w.tmp
// by pcg_finish (rt = its squared norm): r = b - A x, z = B r, rho = r.z,
// p = z; the iteration count is kept.
int pcg_restart(lor_handle *h, Work &w, double rt, hipStream_t st) {
  const int64_t N = h->ndofs;
  double *s = w.scal;
  HIPCHK(launch_copy(w.r, w.tmp, N, st));
  HIPCHK(launch_fill(s + S_DONE, 1, 0.0, st));
  HIPCHK(launch_fill(s + S_FAIL, 1, 0.0, st));
  HIPCHK(launch_fill(s + S_RR, 1, rt, st));
  int rc = apply_P_impl(h, w, w.r, w.z, s, st);
  if (rc != LOR_OK) return rc;
  HIPCHK(launch_dot_partials(w.r, w.z, N, w.part, s, st));
  HIPCHK(launch_finalize(s, w.part, red_blocks(N), FIN_RHO, nullptr, st));
  HIPCHK(launch_copy(w.p, w.z, N, st));
  if (h->method == LOR_CG && !apply_cg_uses_skeleton(h->md)) HIPCHK(launch_fill(w.q, N, 0.0, st));
  return LOR_OK;
}

// Network-preconditioned solves (lor_nn_attach, nn_fallback): leave the
// network for the patch V-cycles when flexible CG breaks down or stalls.
// Called at every chunk boundary with the scalars in w.h_scal; rr_hist keeps
// the recursive residual of the last two boundaries.  On a switch the true
// residual of the current iterate is computed (x and r restart from b if
// the iterate is not finite) and CG restarts from it with the V-cycles.
constexpr double kStall = 0.25;  // ||r||^2 must fall by 4x (||r|| by 2x) per 16 iterations
int nn_fallback_check(lor_handle *h, Work &w, const double *b, double *x, double rtol, int maxit,
                      double rr_hist[2], int *fallback_iter, bool *restarted, hipStream_t st) {
  *restarted = false;
  if (*fallback_iter >= 0 || !h->nn || h->nn_mode == LOR_NN_OFF || !h->opt.nn_fallback) return LOR_OK;
  const double *hs = w.h_scal;
  const double rr = hs[S_RR], tol2 = rtol * rtol * hs[S_BB];
  const bool fail = hs[S_FAIL] != 0.0;
  const bool stalled = !(rr <= kStall * rr_hist[0]);
  rr_hist[0] = rr_hist[1];
  rr_hist[1] = rr;
  const int it = int(hs[S_ITERS]);
  if (!fail && (rr <= tol2 || !stalled)) return LOR_OK;
  if (it >= maxit) return LOR_OK;  // the iteration budget is spent
  *fallback_iter = it;
  h->nn_mode = LOR_NN_OFF;  // restored by lor_pcg_solve on exit
  int rc = pcg_finish(h, w, b, x, st);
  if (rc != LOR_OK) return rc;
  double rt = w.h_scal[S_RRTRUE];
  if (!std::isfinite(rt)) {
    HIPCHK(launch_fill(x, h->ndofs, 0.0, st));
    HIPCHK(launch_copy(w.tmp, b, h->ndofs, st));
    rt = w.h_scal[S_BB];
  }
  rc = pcg_restart(h, w, rt, st);
  if (rc != LOR_OK) return rc;
  *restarted = true;
  return LOR_OK;
}

// Residual replacement after pcg_finish: decides from w.h_scal whether the
// recursive residual met rtol while the true one did not, and if so enqueues
// a restart from the true residual: r = b - A x (left in w.tmp by
// pcg_finish), z = B r, rho = r.z, p = z, with the iteration count kept.
// Restarts stop once the true residual no longer falls by 4x (the float64
// attainable accuracy of the operator has been reached).  *restarted tells
// the caller to run more iterations.
int pcg_replace(lor_handle *h, Work &w, double rtol, int maxit, int &nrep, double &last_true,
                bool *restarted, hipStream_t st) {
  *restarted = false;
  const double *hs = w.h_scal;
  const double bb = hs[S_BB], rr = hs[S_RR], rt = hs[S_RRTRUE];
  const double tol2 = rtol * rtol * bb;
  if (hs[S_FAIL] != 0.0 || !(rr <= tol2) || rt <= tol2) return LOR_OK;
  if (int(hs[S_ITERS]) >= maxit || nrep >= kMaxReplace || !(rt < 0.0625 * last_true))
    return LOR_OK;
  last_true = rt;
  ++nrep;
  int rc = pcg_restart(h, w, rt, st);
  if (rc != LOR_OK) return rc;
  *restarted = true;
  return LOR_OK;
}

// Status and info from the scalars in w.h_scal.
int pcg_status(const lor_handle *h, const Work &w, double rtol, double t_solve, int nrep,
               lor_solve_info_t *info, int fallback_iter = -1) {
  const double *hs = w.h_scal;
  const double bb = hs[S_BB], rr = hs[S_RR], rt = hs[S_RRTRUE], fail = hs[S_FAIL];
  int status = LOR_OK;
  if (fail != 0.0)
    status = fail == 2.0 ? LOR_EINVAL : LOR_EBREAKDOWN;
  else if (!(rr <= rtol * rtol * bb))
    status = LOR_ENOCONV;
  else if (!(rt <= rtol * rtol * bb))
    status = LOR_EACCURACY;
  if (info) {
    info->iters = int(hs[S_ITERS]);
    info->status = status;
    info->rel_res = bb > 0 ? std::sqrt(rr / bb) : 0.0;
    info->rel_res_true = bb > 0 ? std::sqrt(rt / bb) : 0.0;
    info->t_solve = t_solve;
    info->t_setup = h->t_setup;
    info->replacements = nrep;
    info->fallback_iter = fallback_iter;
  }
  return status;
}

// Launch-order autotuner of the vertex-patch kernel: vertex order against
// patches by decreasing work (LOR_LAUNCH_AUTO), timed with HIP events over a
// few launches on the handle's workspace; the faster order is kept.
int tune_launch_order(lor_handle &h, hipStream_t st) {
  h.tune_ms[0] = h.tune_ms[1] = 0.0;
  if (!h.has_prec || box_mode(h.opt.patch_mode) || h.opt.deterministic || h.J <= 0) return LOR_OK;
  const int mode = h.opt.launch_order;
  if (mode == LOR_LAUNCH_VERTEX) {
    h.pa.perm = nullptr;
    h.order_used = LOR_LAUNCH_VERTEX;
    return LOR_OK;
  }
  if (mode == LOR_LAUNCH_BUCKETS) {
    h.pa.perm = h.d_perm;
    h.order_used = LOR_LAUNCH_BUCKETS;
    return LOR_OK;
  }
  const int64_t N = h.ncg;
  HIPCHK(launch_fill(h.w.r, h.ndofs, 1.0, st));
  hipEvent_t a = nullptr, b = nullptr;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&b));
  double best[2] = {0.0, 0.0};
  hipError_t e = hipSuccess;
  for (int rep = 0; rep < 2 && e == hipSuccess; ++rep)
    for (int o = 0; o < 2 && e == hipSuccess; ++o) {
      h.pa.perm = o ? h.d_perm : nullptr;
      const double *rr = h.w.r;  // ones
      e = launch_fill(h.w.z, N, 0.0, st);
      if (e == hipSuccess) e = launch_patch_vcycle(h.pa, h.J, rr, h.w.z, nullptr, st);  // warm
      if (e == hipSuccess) e = hipEventRecord(a, st);
      for (int t = 0; t < 3 && e == hipSuccess; ++t) e = launch_patch_vcycle(h.pa, h.J, rr, h.w.z, nullptr, st);
      if (e == hipSuccess) e = hipEventRecord(b, st);
      if (e == hipSuccess) e = hipEventSynchronize(b);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
      if (rep == 1) best[o] = ms / 3.0;
    }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  HIPCHK(e);
  h.tune_ms[0] = best[0];
  h.tune_ms[1] = best[1];
  const bool buckets = best[1] < best[0];
  h.pa.perm = buckets ? h.d_perm : nullptr;
  h.order_used = buckets ? LOR_LAUNCH_BUCKETS : LOR_LAUNCH_VERTEX;
  return LOR_OK;
}

}  // namespace

extern "C" {

int lor_default_options(lor_options_t *opt) {
  if (!opt) return LOR_EINVAL;
  std::memset(opt, 0, sizeof(*opt));
  opt->precision = LOR_PREC_FP64;
  opt->ordering = LOR_ORD_MDF;
  opt->flexible = 0;
  opt->nthreads = 0;
  opt->nn_fallback = 1;
  return LOR_OK;
}

const char *lor_last_error_detail(void) { return g_detail; }

const char *lor_error_string(int code) {
  switch (code) {
    case LOR_OK: return "success";
    case LOR_EINVAL: return "invalid argument";
    case LOR_EJACOBIAN: return "element map with non-positive Jacobian determinant";
    case LOR_EPIVOT: return "non-positive or non-finite pivot in a factorization";
    case LOR_EBREAKDOWN: return "conjugate gradient breakdown (p^T A p <= 0 or r^T z <= 0)";
    case LOR_ENOCONV: return "maximum number of iterations reached";
    case LOR_EHIP: return "HIP runtime error";
    case LOR_ENOMEM: return "workspace missing or too small";
    case LOR_ESTATE: return "call not valid in the current state";
    case LOR_EACCURACY:
      return "recursive residual converged but the true residual stays above the tolerance";
    default: return "unknown error";
  }
}

int lor_setup(const lor_mesh_t *mesh, int p, int method, double penalty, const lor_options_t *opt,
              void *stream, lor_handle_t **out) {
  g_detail[0] = '\0';
  if (!out) return LOR_EINVAL;
  *out = nullptr;
  const auto t0 = std::chrono::steady_clock::now();
  if (!mesh || !mesh->vertex_xyz) return LOR_EINVAL;
  if (mesh->dim != 2 && mesh->dim != 3) return LOR_EINVAL;
  if (p < 1 || p > kMaxP) return LOR_EINVAL;
  if (method < LOR_CG || method > LOR_BR2) return LOR_EINVAL;
  if (mesh->bc != LOR_BC_DIRICHLET && mesh->bc != LOR_BC_NEUMANN) return LOR_EINVAL;
  if (method != LOR_CG && !(std::isfinite(penalty) && penalty > 0.0)) return LOR_EINVAL;
  int64_t nv = 1;
  for (int d = 0; d < mesh->dim; ++d) {
    if (mesh->n[d] < 1 || mesh->n[d] > 4096) return LOR_EINVAL;
    nv *= mesh->n[d] + 1;
  }
  std::unique_ptr<lor_handle> h(new (std::nothrow) lor_handle());
  if (!h) return LOR_ENOMEM;
  h->dim = mesh->dim;
  for (int d = 0; d < 3; ++d) h->n[d] = d < mesh->dim ? mesh->n[d] : 1;
  h->p = p;
  h->method = method;
  h->bc = mesh->bc;
  h->penalty = penalty;
  if (opt) {
    h->opt = *opt;
    if (opt->precision != LOR_PREC_FP64 && opt->precision != LOR_PREC_MIXED) return LOR_EINVAL;
    if (opt->ordering != LOR_ORD_MDF && opt->ordering != LOR_ORD_NATURAL &&
        opt->ordering != LOR_ORD_RCM)
      return LOR_EINVAL;
    if (opt->prolong_weights != LOR_PROLONG_SUM && opt->prolong_weights != LOR_PROLONG_POU)
      return LOR_EINVAL;
    if (opt->patch_mode != LOR_PATCH_VERTEX && !box_mode(opt->patch_mode)) return LOR_EINVAL;
    if (box_mode(opt->patch_mode) && opt->precision != LOR_PREC_FP64)
      return invalid("the box-patch preconditioners run in float64 only", __LINE__);
    if (opt->patch_mode == LOR_PATCH_SLABS && (opt->nslabs < 1 || opt->nslabs > mesh->n[0]))
      return invalid("nslabs must lie in 1 .. n[0]", __LINE__);
    if (opt->sweep_grid_rows < 0) return LOR_EINVAL;
    if (opt->deterministic != 0 && opt->deterministic != 1) return LOR_EINVAL;
    if (opt->launch_order < LOR_LAUNCH_AUTO || opt->launch_order > LOR_LAUNCH_BUCKETS) return LOR_EINVAL;
    if (opt->operator_geometry != LOR_GEOM_STORED && opt->operator_geometry != LOR_GEOM_ONFLY)
      return LOR_EINVAL;
    if (opt->nn_fallback != 0 && opt->nn_fallback != 1) return LOR_EINVAL;
  } else {
    lor_default_options(&h->opt);
  }
  h->verts.assign(mesh->vertex_xyz, mesh->vertex_xyz + nv * mesh->dim);
  for (double v : h->verts)
    if (!std::isfinite(v)) return LOR_EINVAL;
  if (mesh->node_xyz) {
    if (method != LOR_CG) return invalid("curved elements need the CG discretization", __LINE__);
    int64_t nn = 1;
    for (int d = 0; d < mesh->dim; ++d) nn *= int64_t(mesh->n[d]) * p + 1;
    h->nodes.assign(mesh->node_xyz, mesh->node_xyz + nn * mesh->dim);
    for (double v : h->nodes)
      if (!std::isfinite(v)) return LOR_EINVAL;
  }
  if (mesh->coef) {
    if (method != LOR_CG) return invalid("a variable coefficient needs the CG discretization", __LINE__);
    int64_t ne = 1, nq = 1;
    for (int d = 0; d < mesh->dim; ++d) {
      ne *= mesh->n[d];
      nq *= p + 1;
    }
    h->coef.assign(mesh->coef, mesh->coef + ne * nq);
    bool pos = false;
    for (double v : h->coef) {
      if (!(std::isfinite(v) && v >= 0.0)) return invalid("coefficient negative or not finite", __LINE__);
      pos = pos || v > 0.0;
    }
    if (!pos) return invalid("coefficient zero everywhere", __LINE__);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIPCHK(hipGetDevice(&h->device));
  int rc = setup_impl(*h, st);
  if (rc != LOR_OK) return rc;
  rc = noalloc_register_device(h->device);
  if (rc != LOR_OK) return rc;
  rc = work_alloc(*h, h->w, h->allocs, h->bytes, &h->alloc_size);
  if (rc != LOR_OK) return rc;
  rc = tune_launch_order(*h, st);
  if (rc != LOR_OK) return rc;
  h->t_setup = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *out = h.release();
  return LOR_OK;
}

int lor_launch_order(const lor_handle_t *h, int *order, double *ms_vertex, double *ms_buckets) {
  if (!h || !order) return LOR_EINVAL;
  *order = h->order_used;
  if (ms_vertex) *ms_vertex = h->tune_ms[0];
  if (ms_buckets) *ms_buckets = h->tune_ms[1];
  return LOR_OK;
}

int lor_ndofs(const lor_handle_t *h, int64_t *n) {
  if (!h || !n) return LOR_EINVAL;
  *n = h->ndofs;
  return LOR_OK;
}

int lor_device_bytes(const lor_handle_t *h, size_t *bytes) {
  if (!h || !bytes) return LOR_EINVAL;
  *bytes = h->bytes + h->bbytes;
  return LOR_OK;
}

namespace {
constexpr size_t kWsAlign = 256;
size_t ws_round(size_t b) { return (b + kWsAlign - 1) / kWsAlign * kWsAlign; }
}  // namespace

int lor_workspace_bytes(const lor_handle_t *h, size_t *bytes) {
  if (!h || !bytes) return LOR_EINVAL;
  if (h->bound) {
    *bytes = h->bound_bytes;
    return LOR_OK;
  }
  size_t t = 0;
  for (size_t b : h->alloc_size) t += ws_round(b);
  *bytes = t;
  return LOR_OK;
}

int lor_bind_workspace(lor_handle_t *h, void *dev_ptr, size_t bytes, void *stream) {
  if (!h || !dev_ptr) return LOR_EINVAL;
  if (h->bound) return LOR_ESTATE;
  if (reinterpret_cast<uintptr_t>(dev_ptr) % kWsAlign) return LOR_EINVAL;
  if (h->allocs.size() != h->alloc_size.size()) return LOR_ESTATE;
  size_t need = 0;
  lor_workspace_bytes(h, &need);
  if (bytes < need) {
    std::snprintf(g_detail, sizeof(g_detail), "lor_bind_workspace: %zu bytes given, %zu needed",
                  bytes, need);
    return LOR_ENOMEM;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  char *base = static_cast<char *>(dev_ptr);
  const size_t na = h->allocs.size();
  std::vector<size_t> off(na);
  size_t o = 0;
  for (size_t a = 0; a < na; ++a) {
    off[a] = o;
    o += ws_round(h->alloc_size[a]);
  }
  // new address of a pointer into one of the handle's allocations; every
  // device pointer the handle keeps must resolve, or nothing is changed
  bool ok = true;
  auto reloc = [&](auto *p) -> decltype(p) {
    if (!p) return p;
    const char *c = reinterpret_cast<const char *>(p);
    for (size_t a = 0; a < na; ++a) {
      const char *b0 = static_cast<const char *>(h->allocs[a]);
      if (c >= b0 && c < b0 + h->alloc_size[a])
        return reinterpret_cast<decltype(p)>(base + off[a] + (c - b0));
    }
    ok = false;
    return p;
  };
  auto apply = [&](bool commit) {
    auto set = [&](auto *&field) {
      auto v = reloc(field);
      if (commit) field = v;
    };
    set(h->d_verts), set(h->d_gllx), set(h->d_gllw), set(h->d_D), set(h->d_coords);
    set(h->d_G), set(h->d_wdet), set(h->d_fac), set(h->d_fac_off), set(h->d_xfer);
    set(h->d_A0inv), set(h->d_A0inv_f), set(h->d_fg), set(h->d_dinv), set(h->d_coef);
    for (int k = 0; k < kMaxLevels; ++k) set(h->d_stencil[k]);
    Work &w = h->w;
    set(w.r), set(w.z), set(w.p), set(w.q), set(w.rold), set(w.tmp), set(w.scal), set(w.part);
    set(w.part2), set(w.rc), set(w.xc), set(w.yE), set(w.fo), set(w.rL), set(w.zL);
    for (int k = 0; k < kMaxLevels; ++k) set(h->pa.stencil[k]);
    set(h->pa.xfer), set(h->pa.fac), set(h->pa.fac_off), set(h->pa.perm), set(h->d_perm);
    for (BoxPatchDev &bp : h->boxes)
      for (SingleLevelDev &lv : bp.lv) {
        set(lv.sched), set(lv.lptr), set(lv.Lv), set(lv.invD), set(lv.emask), set(lv.lmask);
        set(lv.x), set(lv.b), set(lv.r), set(lv.ainv);
        for (int d = 0; d < 3; ++d) set(lv.xf.pc[d]), set(lv.xf.pw[d]), set(lv.xf.rf[d]), set(lv.xf.rw[d]);
      }
    for (double *&v : h->box_x) set(v);
    for (double *&v : h->box_b) set(v);
    for (double *&v : h->box_r) set(v);
    for (int t = 0; t < lor_handle::kBoxStreams - 1; ++t) {
      for (double *&v : h->box_sx[t]) set(v);
      for (double *&v : h->box_sb[t]) set(v);
      for (double *&v : h->box_sr[t]) set(v);
    }
    set(h->d_box_w), set(h->d_box_desc), set(h->d_box_list), set(h->d_box_work);
    set(h->d_add_ptr), set(h->d_add_pts), set(h->d_add_src);
  };
  apply(false);  // dry run: resolve every pointer before anything changes
  if (!ok) return LOR_ESTATE;
  for (size_t a = 0; a < na; ++a)
    HIPCHK(hipMemcpyAsync(base + off[a], h->allocs[a], h->alloc_size[a], hipMemcpyDeviceToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  apply(true);
  // the box descriptors hold device pointers: rewrite them at the new addresses
  const int rc = refresh_box_descs(*h, st);
  if (rc != LOR_OK) return rc;
  for (void *p : h->allocs) (void)hipFree(p);
  h->allocs.clear();
  h->alloc_size.clear();
  h->bytes = 0;
  h->bound = true;
  h->bound_bytes = need;
  return LOR_OK;
}

int lor_element_coords(const lor_handle_t *h, double *host_xyz) {
  if (!h || !host_xyz) return LOR_EINVAL;
  const int Q = h->p + 1;
  if (!h->nodes.empty()) {
    // curved elements: each element's own GLL nodes
    const int dim = h->dim, nq = dim == 3 ? Q * Q * Q : Q * Q;
    const int ng0 = h->md.ng[0], ng1 = h->md.ng[1];
    for (int64_t e = 0; e < h->nel; ++e) {
      const int e3[3] = {int(e % h->n[0]), int((e / h->n[0]) % h->n[1]), int(e / (int64_t(h->n[0]) * h->n[1]))};
      for (int q = 0; q < nq; ++q) {
        const int g[3] = {e3[0] * h->p + q % Q, e3[1] * h->p + (q / Q) % Q,
                          dim == 3 ? e3[2] * h->p + q / (Q * Q) : 0};
        const int64_t gi = g[0] + int64_t(ng0) * (g[1] + int64_t(ng1) * g[2]);
        for (int r = 0; r < dim; ++r) host_xyz[(e * nq + q) * dim + r] = h->nodes[size_t(gi) * dim + r];
      }
    }
    return LOR_OK;
  }
  const size_t nb = size_t(h->nel) * (h->dim == 3 ? Q * Q * Q : Q * Q) * h->dim * sizeof(double);
  double *tmp = nullptr;
  if (hipMalloc(&tmp, nb) != hipSuccess) return LOR_EHIP;
  hipError_t e = launch_dg_coords(h->md, h->d_verts, h->d_gllx, tmp, nullptr);
  if (e == hipSuccess) e = hipMemcpy(host_xyz, tmp, nb, hipMemcpyDeviceToHost);
  (void)hipFree(tmp);
  return e == hipSuccess ? LOR_OK : LOR_EHIP;
}

int lor_dof_coords(const lor_handle_t *h, double *host_xyz) {
  if (!h || !host_xyz) return LOR_EINVAL;
  const int dim = h->dim;
  if (h->method != LOR_CG) return lor_element_coords(h, host_xyz);
  std::vector<double> all(size_t(h->nfine) * dim);
  if (hipMemcpy(all.data(), h->d_coords, all.size() * 8, hipMemcpyDeviceToHost) != hipSuccess)
    return LOR_EHIP;
  const MeshDims &md = h->md;
  const int ox = md.dirichlet ? 1 : 0;
  for (int64_t i = 0; i < h->ndofs; ++i) {
    const int64_t gx = i % md.nu[0] + ox, gy = (i / md.nu[0]) % md.nu[1] + ox,
                  gz = dim == 3 ? i / (int64_t(md.nu[0]) * md.nu[1]) + ox : 0;
    const int64_t g = gx + int64_t(md.ng[0]) * (gy + int64_t(md.ng[1]) * gz);
    for (int r = 0; r < dim; ++r) host_xyz[i * dim + r] = all[size_t(r) * h->nfine + g];
  }
  return LOR_OK;
}

int lor_assemble_rhs(lor_handle_t *h, const double *f_dev, double *b_dev, void *stream) {
  if (!h || !f_dev || !b_dev) return LOR_EINVAL;
  if (h->method != LOR_CG) {
    HIPCHK(launch_dg_rhs(h->d_wdet, f_dev, b_dev, h->ndofs, static_cast<hipStream_t>(stream)));
    return LOR_OK;
  }
  HIPCHK(launch_rhs_cg(h->md, h->d_wdet, f_dev, b_dev, static_cast<hipStream_t>(stream)));
  return LOR_OK;
}

int lor_apply_A(lor_handle_t *h, const double *x_dev, double *y_dev, void *stream) {
  if (!h || !x_dev || !y_dev || x_dev == y_dev) return LOR_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (h->method == LOR_CG && !apply_cg_uses_skeleton(h->md))
    HIPCHK(hipMemsetAsync(y_dev, 0, h->ndofs * sizeof(double), st));
  return apply_A_impl(h, h->w, x_dev, y_dev, nullptr, nullptr, st);
}

int lor_apply_P(lor_handle_t *h, const double *r_dev, double *z_dev, void *stream) {
  if (!h || !r_dev || !z_dev || r_dev == z_dev) return LOR_EINVAL;
  if (!h->has_prec) return LOR_ESTATE;
  return apply_P_impl(h, h->w, r_dev, z_dev, nullptr, static_cast<hipStream_t>(stream));
}

int lor_apply_P_batch(lor_handle_t *const *hs, int n, const double *const *r, double *const *z,
                      void *stream) {
  if (!hs || !r || !z || n < 1) return LOR_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (!hs[i] || !r[i] || !z[i] || r[i] == z[i]) return LOR_EINVAL;
    if (!hs[i]->has_prec) return LOR_ESTATE;
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return LOR_EINVAL;  // one workspace per handle
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (int i0 = 0; i0 < n;) {
    // a run of handles whose patch corrections can share a launch
    int i1 = i0 + 1;
    if (multi_rhs_patches(hs[i0]))
      while (i1 < n && i1 - i0 < kMaxJobs && multi_rhs_patches(hs[i1]) &&
             hs[i1]->dim == hs[i0]->dim && hs[i1]->pa.fp32 == hs[i0]->pa.fp32)
        ++i1;
    if (i1 - i0 == 1) {
      const int rc = apply_P_impl(hs[i0], hs[i0]->w, r[i0], z[i0], nullptr, st);
      if (rc != LOR_OK) return rc;
      i0 = i1;
      continue;
    }
    PatchArgs pa[kMaxJobs];
    for (int i = i0; i < i1; ++i) {
      lor_handle *h = hs[i];
      const int rc = apply_P_pre(h, h->w, r[i], z[i], nullptr, st);
      if (rc != LOR_OK) return rc;
      PatchArgs &a = pa[i - i0];
      a = h->pa;
      a.nrhs = 1;
      for (int k = 0; k < kMaxRhs; ++k) {
        a.rs[k] = nullptr;
        a.zs[k] = nullptr;
        a.flags[k] = nullptr;
      }
      patch_io(h, h->w, r[i], z[i], &a.rs[0], &a.zs[0]);
    }
    HIPCHK(launch_patch_vcycle_jobs(pa, i1 - i0, st));
    for (int i = i0; i < i1; ++i) {
      const int rc = apply_P_post(hs[i], hs[i]->w, r[i], z[i], nullptr, st);
      if (rc != LOR_OK) return rc;
    }
    i0 = i1;
  }
  return LOR_OK;
}

int lor_pcg_solve(lor_handle_t *h, const double *b, double *x, double rtol, int maxit,
                  lor_solve_info_t *info, void *stream) {
  if (!h || !b || !x || b == x || !(rtol >= 0.0) || maxit < 0) return LOR_EINVAL;
  if (!h->has_prec) return LOR_ESTATE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Work &w = h->w;
  HIPCHK(hipEventRecord(h->ev0, st));
  // the network mode is switched off by a fallback for the rest of this
  // solve only
  struct ModeGuard {
    lor_handle *h;
    int mode;
    ~ModeGuard() { h->nn_mode = mode; }
  } guard{h, h->nn_mode};
  int rc = pcg_init(h, w, b, x, rtol, maxit, st);
  if (rc != LOR_OK) return rc;
  int nrep = 0, fallback_iter = -1;
  double last_true = HUGE_VAL, rr_hist[2] = {HUGE_VAL, HUGE_VAL};
  for (;;) {
    bool done = maxit == 0;
    while (!done) {
      rc = pcg_iterations(h, w, x, kChunk, st);
      if (rc != LOR_OK) return rc;
      HIPCHK(hipMemcpyAsync(w.h_scal, w.scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      done = w.h_scal[S_DONE] != 0.0;  // also set on the device at maxit
      bool switched = false;
      rc = nn_fallback_check(h, w, b, x, rtol, maxit, rr_hist, &fallback_iter, &switched, st);
      if (rc != LOR_OK) return rc;
      if (switched) done = false;
    }
    HIPCHK(hipEventRecord(h->ev1, st));
    rc = pcg_finish(h, w, b, x, st);
    if (rc != LOR_OK) return rc;
    bool again = false;
    rc = pcg_replace(h, w, rtol, maxit, nrep, last_true, &again, st);
    if (rc != LOR_OK) return rc;
    if (!again) break;
  }
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
  return pcg_status(h, w, rtol, ms * 1e-3, nrep, info, fallback_iter);
}

int lor_pcg_solve_batch(lor_handle_t *const *hs, int nprob, int nrhs, const double *const *b,
                        double *const *x, double rtol, int maxit, lor_solve_info_t *info,
                        void *stream) {
  if (!hs || !b || !x || nprob < 1 || nrhs < 1 || !(rtol >= 0.0) || maxit < 0) return LOR_EINVAL;
  const int npair = nprob * nrhs;
  for (int i = 0; i < nprob; ++i) {
    if (!hs[i]) return LOR_EINVAL;
    if (!hs[i]->has_prec) return LOR_ESTATE;
    if (hs[i]->nn && hs[i]->nn_mode != LOR_NN_OFF) return LOR_ESTATE;  // network buffers are shared
  }
  for (int k = 0; k < npair; ++k)
    if (!b[k] || !x[k] || b[k] == x[k]) return LOR_EINVAL;
  hipStream_t caller = static_cast<hipStream_t>(stream);
  struct Pair {
    lor_handle *h = nullptr;
    Work w;
    hipStream_t st = nullptr;
    int64_t it = 0;
    bool done = false, final = false;
    int nrep = 0;
    double last_true = HUGE_VAL;
  };
  // The right-hand sides of one problem form parts of up to kMaxRhs pairs
  // where the handle's preconditioner allows their patch corrections in one
  // launch, else parts of one pair.  A group is one captured chunk of
  // iterations of its parts in lockstep; with more parts than streams, small
  // parts of like dimension and precision share groups of up to kMaxJobs,
  // their patch corrections in one launch for all of them.
  struct Part {
    int first = 0, n = 1;
    bool multi = false;
    double cost = 0.0;
  };
  struct Group {
    std::vector<Part> parts;
    double cost = 0.0;
    hipStream_t st = nullptr;
    hipGraphExec_t chunk = nullptr;
  };
  std::vector<Pair> pairs(npair);
  std::vector<Group> groups;
  std::vector<hipStream_t> streams;
  hipEvent_t ready = nullptr, start = nullptr, stop = nullptr;
  int rc = LOR_OK;
  // graphs, streams and events are released on every exit path; the pairs'
  // workspaces are cached on their handles (allocated the first time a
  // handle needs that many, freed by lor_free)
  auto cleanup = [&]() {
    for (Group &g : groups)
      if (g.chunk) (void)hipGraphExecDestroy(g.chunk);
    for (hipStream_t t : streams) (void)hipStreamDestroy(t);
    if (ready) (void)hipEventDestroy(ready);
    if (start) (void)hipEventDestroy(start);
    if (stop) (void)hipEventDestroy(stop);
    for (int i = 0; i < nprob; ++i) hs[i]->capturing = false;
  };
  auto fail = [&](int code) {
    cleanup();
    return code;
  };
#define BCHK(x)                                              \
  do {                                                       \
    hipError_t e_ = (x);                                     \
    if (e_ != hipSuccess) return fail(hip_fail(e_, #x, __LINE__)); \
  } while (0)
  {
    std::vector<Part> parts;
    for (int i = 0; i < nprob; ++i) {
      const bool multi = multi_rhs_patches(hs[i]);
      const int step = multi ? kMaxRhs : 1;
      for (int j = 0; j < nrhs; j += step) {
        Part pt;
        pt.first = i * nrhs + j;
        pt.n = std::min(step, nrhs - j);
        pt.multi = multi;
        pt.cost = double(hs[i]->ndofs) * pt.n;
        parts.push_back(pt);
      }
    }
    // a part whose patch launch alone cannot fill the device shares one:
    // by dimension and precision, similar patch sizes together (the launch
    // reserves the largest patch's LDS for every patch), up to kMaxJobs
    // parts and kJobBlocks patch blocks per group
    std::vector<BatchPart> bp(parts.size());
    for (size_t a = 0; a < parts.size(); ++a) {
      const lor_handle *h = hs[parts[a].first / nrhs];
      bp[a] = BatchPart{parts[a].multi, h->dim, h->pa.fp32, h->pa.lds_total,
                        int64_t(h->J + 7) / 8 * 8 * parts[a].n, parts[a].cost};
    }
    for (const std::vector<int> &pl : plan_batch_groups(bp, kBatchStreams, kMaxJobs, kJobBlocks)) {
      Group g;
      for (int a : pl) {
        g.parts.push_back(parts[a]);
        g.cost += parts[a].cost;
      }
      groups.push_back(g);
    }
  }
  const int ns = std::min(kBatchStreams, int(groups.size()));
  for (int i = 0; i < ns; ++i) {
    hipStream_t t = nullptr;
    BCHK(hipStreamCreateWithFlags(&t, hipStreamNonBlocking));  // default priority
    streams.push_back(t);
  }
  BCHK(hipEventCreate(&ready));
  BCHK(hipEventCreate(&start));
  BCHK(hipEventCreate(&stop));
  // the caller's stream orders the inputs: every worker stream waits for it
  BCHK(hipEventRecord(ready, caller));
  for (hipStream_t t : streams) BCHK(hipStreamWaitEvent(t, ready, 0));
  {
    // a handle may serve several problems: its pairs take consecutive
    // cached workspaces
    std::vector<std::pair<lor_handle *, int>> used;
    // the costliest group first, each to the least loaded stream
    std::vector<double> costs(groups.size());
    for (size_t gi = 0; gi < groups.size(); ++gi) costs[gi] = groups[gi].cost;
    const std::vector<int> gs = assign_streams(costs, ns);
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      groups[gi].st = streams[gs[gi]];
      for (const Part &pt : groups[gi].parts)
        for (int k = pt.first; k < pt.first + pt.n; ++k) pairs[k].st = groups[gi].st;
    }
    for (int k = 0; k < npair; ++k) {
      Pair &q = pairs[k];
      q.h = hs[k / nrhs];
      int slot = 0;
      bool found = false;
      for (auto &u : used)
        if (u.first == q.h) {
          slot = u.second++;
          found = true;
        }
      if (!found) used.push_back({q.h, 1});
      while (int(q.h->bwork.size()) <= slot) {
        Work nw;
        rc = work_alloc(*q.h, nw, q.h->ballocs, q.h->bbytes);
        if (nw.h_scal) q.h->bwork.push_back(nw);
        if (rc != LOR_OK) return fail(rc);
      }
      q.w = q.h->bwork[slot];
    }
  }
  // one captured chunk of iterations per group (kernels become no-ops once a
  // pair has converged, so the chunk is replayed until every pair's flag is
  // set)
  for (Group &gr : groups) {
    PatchJob jobs[kMaxJobs];
    const int nj = int(gr.parts.size());
    for (int j = 0; j < nj; ++j) {
      const Part &pt = gr.parts[j];
      jobs[j].h = pairs[pt.first].h;
      jobs[j].n = pt.n;
      for (int k = 0; k < pt.n; ++k) {
        jobs[j].w[k] = &pairs[pt.first + k].w;
        jobs[j].x[k] = x[pt.first + k];
      }
      jobs[j].h->capturing = true;
    }
    hipGraph_t g = nullptr;
    BCHK(hipStreamBeginCapture(gr.st, hipStreamCaptureModeThreadLocal));
    if (nj > 1)
      rc = pcg_iterations_jobs(jobs, nj, kChunk, gr.st);
    else if (jobs[0].n > 1)
      rc = pcg_iterations_multi(jobs[0].h, jobs[0].w, jobs[0].x, jobs[0].n, kChunk, gr.st);
    else
      rc = pcg_iterations(jobs[0].h, *jobs[0].w[0], jobs[0].x[0], kChunk, gr.st);
    hipError_t e = hipStreamEndCapture(gr.st, &g);
    for (int j = 0; j < nj; ++j) jobs[j].h->capturing = false;
    if (rc != LOR_OK) {
      if (g) (void)hipGraphDestroy(g);
      return fail(rc);
    }
    BCHK(e);
    e = hipGraphInstantiate(&gr.chunk, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    BCHK(e);
  }
  // the timed span starts here: workspaces, streams and graphs are ready
  BCHK(hipEventRecord(start, streams[0]));
  for (hipStream_t t : streams)
    if (t != streams[0]) BCHK(hipStreamWaitEvent(t, start, 0));
  for (int k = 0; k < npair; ++k) {
    Pair &q = pairs[k];
    rc = pcg_init(q.h, q.w, b[k], x[k], rtol, maxit, q.st);
    if (rc != LOR_OK) return fail(rc);
    q.done = maxit == 0;
  }
  // the device sets each pair's flag at convergence or at maxit; the host
  // bound only guards against a flag that never comes
  const int64_t it_cap = int64_t(maxit + kChunk) * (kMaxReplace + 1);
  float ms = 0.f;
  for (;;) {
    for (;;) {
      bool any = false;
      for (Group &gr : groups) {
        bool live = false;
        for (const Part &pt : gr.parts)
          for (int k = pt.first; k < pt.first + pt.n; ++k) live = live || !pairs[k].done;
        if (!live) continue;
        any = true;
        BCHK(hipGraphLaunch(gr.chunk, gr.st));
        for (const Part &pt : gr.parts)
          for (int k = pt.first; k < pt.first + pt.n; ++k) {
            Pair &q = pairs[k];
            BCHK(hipMemcpyAsync(q.w.h_scal, q.w.scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost,
                                q.st));
            q.it += kChunk;
          }
      }
      if (!any) break;
      for (hipStream_t t : streams) BCHK(hipStreamSynchronize(t));
      for (Pair &q : pairs)
        if (!q.done) q.done = q.w.h_scal[S_DONE] != 0.0 || q.it >= it_cap;
    }
    // every worker stream has been synchronized: stop marks the end of the
    // iterations of all pairs
    BCHK(hipEventRecord(stop, streams[0]));
    BCHK(hipEventSynchronize(stop));
    BCHK(hipEventElapsedTime(&ms, start, stop));
    // true residuals; residual replacement for pairs whose recursive
    // residual drifted below rtol ahead of the true one
    bool again = false;
    for (int k = 0; k < npair; ++k) {
      Pair &q = pairs[k];
      if (q.final) continue;
      rc = pcg_finish(q.h, q.w, b[k], x[k], q.st);
      if (rc != LOR_OK) return fail(rc);
      bool restarted = false;
      rc = pcg_replace(q.h, q.w, rtol, maxit, q.nrep, q.last_true, &restarted, q.st);
      if (rc != LOR_OK) return fail(rc);
      if (restarted) {
        q.done = false;
        again = true;
      } else {
        q.final = true;
      }
    }
    if (!again) break;
  }
  int status = LOR_OK;
  for (int k = 0; k < npair; ++k) {
    Pair &q = pairs[k];
    const int sk = pcg_status(q.h, q.w, rtol, ms * 1e-3, q.nrep, info ? info + k : nullptr);
    if (status == LOR_OK) status = sk;
  }
#undef BCHK
  cleanup();
  return status;
}

int lor_export_maps(const lor_handle_t *h, int which, int32_t *out, int64_t *len) {
  if (!h || !len) return LOR_EINVAL;
  const std::vector<int32_t> *src = nullptr;
  std::vector<int32_t> tmp;
  switch (which) {
    case LOR_MAP_LDOF: {
      const MeshDims &md = h->md;
      const int ox = md.dirichlet ? 1 : 0;
      tmp.resize(h->ncg);
      for (int64_t i = 0; i < h->ncg; ++i) {
        const int64_t gx = i % md.nu[0] + ox, gy = (i / md.nu[0]) % md.nu[1] + ox,
                      gz = h->dim == 3 ? i / (int64_t(md.nu[0]) * md.nu[1]) + ox : 0;
        tmp[i] = int32_t(gx + int64_t(md.ng[0]) * (gy + int64_t(md.ng[1]) * gz));
      }
      src = &tmp;
      break;
    }
    case LOR_MAP_E2L: {
      if (h->method == LOR_CG) return LOR_EINVAL;
      const MeshDims &md = h->md;
      const int Q = md.p + 1, ox = md.dirichlet ? 1 : 0;
      const int nq = h->dim == 3 ? Q * Q * Q : Q * Q;
      tmp.resize(h->ndofs);
      for (int64_t t = 0; t < h->ndofs; ++t) {
        const int64_t e = t / nq;
        const int m = int(t % nq);
        const int l[3] = {m % Q, (m / Q) % Q, m / (Q * Q)};
        const int64_t ec[3] = {e % md.n[0], (e / md.n[0]) % md.n[1], e / (int64_t(md.n[0]) * md.n[1])};
        int64_t li = 0, stride = 1;
        bool in = true;
        for (int d = 0; d < h->dim; ++d) {
          const int64_t g = ec[d] * md.p + l[d];
          if (md.dirichlet && (g == 0 || g == md.ng[d] - 1)) in = false;
          li += (g - ox) * stride;
          stride *= md.nu[d];
        }
        tmp[t] = in ? int32_t(li) : -1;
      }
      src = &tmp;
      break;
    }
    case LOR_MAP_ORDER: src = &h->order_all; break;
    case LOR_MAP_ORDER_OFFSET: src = &h->order_off; break;
    case LOR_MAP_SCHEDULE: src = &h->sched_all; break;
    case LOR_MAP_SCHEDULE_OFFSET: src = &h->sched_off; break;
    default: return LOR_EINVAL;
  }
  *len = int64_t(src->size());
  if (out) std::copy(src->begin(), src->end(), out);
  return LOR_OK;
}

int lor_export_stencils(const lor_handle_t *h, int level, double *out, int64_t *len) {
  if (!h || !len) return LOR_EINVAL;
  if (!h->has_prec || level < 0 || level >= h->L) return LOR_EINVAL;
  const int64_t n = int64_t(nslots(h->dim)) * h->npts[level];
  *len = n;
  if (out && hipMemcpy(out, h->d_stencil[level], n * 8, hipMemcpyDeviceToHost) != hipSuccess)
    return LOR_EHIP;
  return LOR_OK;
}

int lor_timing(lor_handle_t *h, int enable) {
  if (!h) return LOR_EINVAL;
  if (hipDeviceSynchronize() != hipSuccess) return LOR_EHIP;
  if (enable) {  // a new record; disabling keeps the record for lor_timing_read
    for (auto &v : h->tspans) v.clear();
    h->ev_used = 0;
  }
  h->timing = enable != 0;
  return LOR_OK;
}

int lor_timing_read(const lor_handle_t *h, int which, double *total_ms, int64_t *count) {
  if (!h || which < 0 || which > 2 || !total_ms || !count) return LOR_EINVAL;
  double tot = 0.0;
  for (const auto &sp : h->tspans[which]) {
    if (hipEventSynchronize(sp.second) != hipSuccess) return LOR_EHIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, sp.first, sp.second) != hipSuccess) return LOR_EHIP;
    tot += ms;
  }
  *total_ms = tot;
  *count = int64_t(h->tspans[which].size());
  return LOR_OK;
}

int lor_gll(int p, double *x, double *w) {
  if (p < 1 || p > kMaxP || !x || !w) return LOR_EINVAL;
  std::vector<double> xv, wv;
  gll_nodes_weights(p, xv, wv);
  std::copy(xv.begin(), xv.end(), x);
  std::copy(wv.begin(), wv.end(), w);
  return LOR_OK;
}

int lor_mdf_order(int dim, const int *m, const double *rows, int ordering, int32_t *order,
                  int32_t *level_ptr, int32_t *depth, double *L, double *D) {
  if ((dim != 2 && dim != 3) || !m || !rows) return LOR_EINVAL;
  if (ordering != LOR_ORD_MDF && ordering != LOR_ORD_NATURAL && ordering != LOR_ORD_RCM)
    return LOR_EINVAL;
  int64_t n = 1;
  int mm[3] = {1, 1, 1};
  for (int d = 0; d < dim; ++d) {
    if (m[d] < 1 || m[d] > 4096) return LOR_EINVAL;
    mm[d] = m[d];
    n *= m[d];
  }
  if (n > (int64_t(1) << 24)) return LOR_EINVAL;
  const int NS = nslots(dim);
  std::vector<double> a(rows, rows + n * NS);
  MdfResult res;
  const int rc = mdf_factor(dim, mm, a, ordering, res);
  if (rc != LOR_OK) return rc;
  if (order) std::copy(res.order.begin(), res.order.end(), order);
  if (level_ptr) std::copy(res.level_ptr.begin(), res.level_ptr.end(), level_ptr);
  if (depth) *depth = int32_t(res.level_ptr.size()) - 1;
  if (L) std::copy(res.L.begin(), res.L.end(), L);
  if (D) std::copy(res.D.begin(), res.D.end(), D);
  return LOR_OK;
}

int lor_free(lor_handle_t *h) {
  delete h;
  return LOR_OK;
}

}  // extern "C"

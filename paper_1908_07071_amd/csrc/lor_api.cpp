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
#include <vector>

#include "lor_internal.h"

using namespace lor;

struct lor_handle {
  int dim = 3, n[3] = {1, 1, 1}, p = 1, method = LOR_CG, bc = LOR_BC_DIRICHLET;
  double penalty = 0.0;
  lor_options_t opt{};
  MeshDims md{};
  std::vector<double> verts, gllx, gllw, D;
  std::vector<std::vector<int>> kept;
  int L = 1;
  int64_t ndofs = 0, nfine = 0, nel = 0;
  int64_t ncg = 0;     // conforming unknowns (the L-vector of the Schwarz preconditioner)
  int64_t nfaces = 0;  // DG faces
  int J = 0, nc = 0;
  // device memory (owned)
  std::vector<void *> allocs;
  size_t bytes = 0;
  double *d_verts = nullptr, *d_gllx = nullptr, *d_gllw = nullptr, *d_D = nullptr;
  double *d_coords = nullptr, *d_G = nullptr, *d_wdet = nullptr;
  double *d_stencil[kMaxLevels] = {};
  int64_t npts[kMaxLevels] = {};
  char *d_fac = nullptr;
  int64_t *d_fac_off = nullptr;
  int64_t fac_bytes = 0;
  XferTab *d_xfer = nullptr;
  double *d_A0inv = nullptr, *d_rc = nullptr, *d_xc = nullptr;
  double *d_yE = nullptr;  // element-boundary partial results of the CG operator
  double *d_fg = nullptr, *d_fo = nullptr, *d_dinv = nullptr, *d_rL = nullptr, *d_zL = nullptr;
  double *d_r = nullptr, *d_z = nullptr, *d_p = nullptr, *d_q = nullptr, *d_rold = nullptr;
  double *d_tmp = nullptr, *d_scal = nullptr, *d_part = nullptr, *d_part2 = nullptr;
  int npart = 0;
  double *h_scal = nullptr;  // pinned
  PatchArgs pa{};
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
    bytes += b;
    *ptr = static_cast<T *>(p);
    return hipSuccess;
  }
  ~lor_handle() {
    for (void *p : allocs) (void)hipFree(p);
    if (h_scal) (void)hipHostFree(h_scal);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
  }
};

namespace {

thread_local char g_detail[512] = "";

int hip_fail(hipError_t e, const char *what, int line) {
  std::snprintf(g_detail, sizeof(g_detail), "%s failed at lor_api.cpp:%d: %s", what, line,
                hipGetErrorString(e));
  return LOR_EHIP;
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
  HIPCHK(h.alloc(&h.d_rc, h.nc));
  HIPCHK(h.alloc(&h.d_xc, h.nc));
  HIPCHK(hipMemcpyAsync(h.d_A0inv, A0.data(), A0.size() * sizeof(double), hipMemcpyHostToDevice, st));
  double *rowbuf, *colbuf;
  int *bad;
  HIPCHK(h.alloc(&rowbuf, h.nc));
  HIPCHK(h.alloc(&colbuf, h.nc));
  HIPCHK(h.alloc(&bad, 1));
  HIPCHK(hipMemsetAsync(bad, 0, sizeof(int), st));
  HIPCHK(launch_gauss_jordan(h.nc, h.d_A0inv, rowbuf, colbuf, bad, st));
  int hb = 0;
  HIPCHK(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return hb ? LOR_EPIVOT : LOR_OK;
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
      int rc = mdf_factor(dim, b.m, rows, h.opt.ordering == LOR_ORD_NATURAL, res);
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
  for (size_t t = 0; t < blocks.size(); ++t)
    if (!blocks[t].empty())
      HIPCHK(hipMemcpyAsync(h.d_fac + off[t], blocks[t].data(), blocks[t].size(), hipMemcpyHostToDevice, st));
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
    const int W = dim == 3 ? sym_width<3>() : sym_width<2>();
    if (mixed) {
      float *f32 = nullptr;
      HIPCHK(h.alloc(&f32, size_t(W) * h.npts[k]));
      HIPCHK(launch_sym_stencil(h.d_stencil[k], h.npts[k], dim, f32, true, st));
      pa.stencil[k] = reinterpret_cast<const double *>(f32);  // read as float by the kernel
    } else {
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
  // LDS of the largest patch: level 0 X, R; coarser levels X, B, R
  int tot = 0;
  for (int k = 0; k < L; ++k) {
    const int s = pa.s[k];
    int ps = 1;
    for (int d = 0; d < dim; ++d) ps *= std::max(h.n[d] >= 2 ? 2 * s - 1 : s - 1, 0);
    tot += (k == 0 ? 2 : 3) * ps;
  }
  pa.lds_total = tot;
  pa.fp32 = mixed ? 1 : 0;
  if (size_t(tot) * (mixed ? sizeof(float) : sizeof(double)) > 160 * 1024) return LOR_EINVAL;
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
  HIPCHK(launch_node_coords(md, h.d_verts, h.d_gllx, h.d_coords, st));
  const int ncomp = dim == 3 ? 6 : 3;
  HIPCHK(h.alloc(&h.d_G, size_t(h.nel) * ncomp * nq));
  HIPCHK(h.alloc(&h.d_wdet, size_t(h.nel) * nq));
  if (!dg && apply_cg_uses_skeleton(md)) HIPCHK(h.alloc(&h.d_yE, size_t(h.nel) * nq));
  int *bad;
  HIPCHK(h.alloc(&bad, 1));
  HIPCHK(hipMemsetAsync(bad, 0, sizeof(int), st));
  HIPCHK(launch_geom_cg(md, h.d_verts, h.d_gllx, h.d_gllw, h.d_G, h.d_wdet, bad, st));
  int hb = 0;
  HIPCHK(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hb) return LOR_EJACOBIAN;
  if (dg) {
    // faces: geometry and penalty (eq. ip / eq. br2), face records, diag(A_DG)
    const int QF = dim == 3 ? Q * Q : Q;
    h.nfaces = dg_face_count(md);
    HIPCHK(h.alloc(&h.d_fg, size_t(h.nfaces) * 8 * QF));
    HIPCHK(h.alloc(&h.d_fo, size_t(h.nfaces) * 8 * QF));
    HIPCHK(h.alloc(&h.d_dinv, size_t(h.ndofs)));
    HIPCHK(launch_dg_face_geom(md, h.d_verts, h.d_gllx, h.d_gllw, h.d_wdet, h.method, h.penalty,
                               h.d_fg, st));
    HIPCHK(launch_dg_diag(md, h.d_G, h.d_D, h.d_fg, h.d_dinv, st));
    HIPCHK(h.alloc(&h.d_rL, size_t(h.ncg)));
    HIPCHK(h.alloc(&h.d_zL, size_t(h.ncg)));
  }
  // Krylov work vectors
  const int64_t N = h.ndofs;
  HIPCHK(h.alloc(&h.d_r, N));
  HIPCHK(h.alloc(&h.d_z, N));
  HIPCHK(h.alloc(&h.d_p, N));
  HIPCHK(h.alloc(&h.d_q, N));
  HIPCHK(h.alloc(&h.d_rold, N));
  HIPCHK(h.alloc(&h.d_tmp, N));
  HIPCHK(h.alloc(&h.d_scal, S_COUNT));
  h.npart = std::max(kRedBlocks, apply_cg_blocks(md, dg));
  HIPCHK(h.alloc(&h.d_part, h.npart));
  HIPCHK(h.alloc(&h.d_part2, h.npart));
  HIPCHK(hipHostMalloc((void **)&h.h_scal, S_COUNT * sizeof(double), 0));
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
    HIPCHK(launch_lor_stencil(md, s, h.kept[k].data(), h.d_coords, g0, g1, h.d_stencil[k], st));
    hst[k].resize(size_t(NS) * h.npts[k]);
    HIPCHK(hipMemcpyAsync(hst[k].data(), h.d_stencil[k], hst[k].size() * 8, hipMemcpyDeviceToHost, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  int rc = build_patches(h, hst, st);
  if (rc != LOR_OK) return rc;
  rc = build_coarse(h, hst[0], st);
  if (rc != LOR_OK) return rc;
  HIPCHK(hipStreamSynchronize(st));
  h.has_prec = true;
  return LOR_OK;
}

// Records an event pair around a launch when timing is on.
struct Span {
  lor_handle *h;
  int which;
  hipStream_t st;
  hipEvent_t a = nullptr;
  Span(lor_handle *hh, int w, hipStream_t s) : h(hh), which(w), st(s) {
    if (h->timing && (a = h->next_event())) (void)hipEventRecord(a, st);
  }
  ~Span() {
    if (!a) return;
    hipEvent_t b = h->next_event();
    if (b && hipEventRecord(b, st) == hipSuccess) h->tspans[which].push_back({a, b});
  }
};

// Conforming Schwarz preconditioner on L-vectors (eq. as).
int apply_P_cg(lor_handle *h, const double *r, double *z, const double *flag, hipStream_t st) {
  if (h->nc > 0) {
    Span sp(h, LOR_T_COARSE, st);
    HIPCHK(launch_coarse_restrict(h->md, h->d_gllx, r, h->d_rc, st));
    HIPCHK(launch_gemv(h->nc, h->d_A0inv, h->d_rc, h->d_xc, flag, st));
    HIPCHK(launch_coarse_prolong(h->md, h->d_gllx, h->d_xc, z, flag, st));
  } else {
    HIPCHK(launch_fill(z, h->ncg, 0.0, st));
  }
  Span sp(h, LOR_T_PATCH, st);
  HIPCHK(launch_patch_vcycle(h->pa, h->J, r, z, flag, st));
  return LOR_OK;
}

// CG: eq. as.  DG: eq. dg-as, z = D_B^-1 r on element-boundary nodes plus
// E B E^T r.
int apply_P_impl(lor_handle *h, const double *r, double *z, const double *flag, hipStream_t st) {
  if (h->method == LOR_CG) return apply_P_cg(h, r, z, flag, st);
  HIPCHK(launch_dg_restrict(h->md, r, h->d_rL, flag, st));
  int rc = apply_P_cg(h, h->d_rL, h->d_zL, flag, st);
  if (rc != LOR_OK) return rc;
  HIPCHK(launch_dg_prolong_jacobi(h->md, r, h->d_dinv, h->d_zL, z, flag, st));
  return LOR_OK;
}

int apply_A_impl(lor_handle *h, const double *x, double *y, double *partials, const double *flag,
                 hipStream_t st) {
  Span sp(h, LOR_T_APPLY_A, st);
  if (h->method != LOR_CG) HIPCHK(launch_dg_face(h->md, h->d_D, h->d_fg, x, h->d_fo, flag, st));
  HIPCHK(launch_apply_cg(h->md, h->d_G, h->d_D, x, y, partials, flag, st,
                         h->method != LOR_CG ? h->d_fo : nullptr, h->d_yE));
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
    default: return "unknown error";
  }
}

int lor_setup(const lor_mesh_t *mesh, int p, int method, double penalty, const lor_options_t *opt,
              void *stream, lor_handle_t **out) {
  if (!out) return LOR_EINVAL;
  *out = nullptr;
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
    if (opt->ordering != LOR_ORD_MDF && opt->ordering != LOR_ORD_NATURAL) return LOR_EINVAL;
  } else {
    lor_default_options(&h->opt);
  }
  h->verts.assign(mesh->vertex_xyz, mesh->vertex_xyz + nv * mesh->dim);
  for (double v : h->verts)
    if (!std::isfinite(v)) return LOR_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = setup_impl(*h, st);
  if (rc != LOR_OK) return rc;
  *out = h.release();
  return LOR_OK;
}

int lor_ndofs(const lor_handle_t *h, int64_t *n) {
  if (!h || !n) return LOR_EINVAL;
  *n = h->ndofs;
  return LOR_OK;
}

int lor_device_bytes(const lor_handle_t *h, size_t *bytes) {
  if (!h || !bytes) return LOR_EINVAL;
  *bytes = h->bytes;
  return LOR_OK;
}

int lor_dof_coords(const lor_handle_t *h, double *host_xyz) {
  if (!h || !host_xyz) return LOR_EINVAL;
  const int dim = h->dim;
  if (h->method != LOR_CG) {
    double *tmp = nullptr;
    const size_t nb = size_t(h->ndofs) * dim * sizeof(double);
    if (hipMalloc(&tmp, nb) != hipSuccess) return LOR_EHIP;
    hipError_t e = launch_dg_coords(h->md, h->d_verts, h->d_gllx, tmp, nullptr);
    if (e == hipSuccess) e = hipMemcpy(host_xyz, tmp, nb, hipMemcpyDeviceToHost);
    (void)hipFree(tmp);
    return e == hipSuccess ? LOR_OK : LOR_EHIP;
  }
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
  return apply_A_impl(h, x_dev, y_dev, nullptr, nullptr, st);
}

int lor_apply_P(lor_handle_t *h, const double *r_dev, double *z_dev, void *stream) {
  if (!h || !r_dev || !z_dev || r_dev == z_dev) return LOR_EINVAL;
  if (!h->has_prec) return LOR_ESTATE;
  return apply_P_impl(h, r_dev, z_dev, nullptr, static_cast<hipStream_t>(stream));
}

int lor_pcg_solve(lor_handle_t *h, const double *b, double *x, double rtol, int maxit,
                  lor_solve_info_t *info, void *stream) {
  if (!h || !b || !x || b == x || !(rtol >= 0.0) || maxit < 0) return LOR_EINVAL;
  if (!h->has_prec) return LOR_ESTATE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t N = h->ndofs;
  const bool fcg = h->opt.flexible != 0 || h->opt.precision == LOR_PREC_MIXED;
  double *s = h->d_scal;
  HIPCHK(hipEventRecord(h->ev0, st));
  // x = 0, r = b, tol^2
  HIPCHK(hipMemsetAsync(x, 0, N * sizeof(double), st));
  HIPCHK(launch_copy(h->d_r, b, N, st));
  HIPCHK(launch_fill(s, S_COUNT, 0.0, st));
  HIPCHK(launch_fill(s + S_TOL2, 1, rtol * rtol, st));
  const int nbv = red_blocks(N);
  HIPCHK(launch_dot_partials(b, b, N, h->d_part, nullptr, st));
  HIPCHK(launch_finalize(s, h->d_part, nbv, FIN_BB, 0, nullptr, st));
  int rc = apply_P_impl(h, h->d_r, h->d_z, s, st);
  if (rc != LOR_OK) return rc;
  HIPCHK(launch_dot_partials(h->d_r, h->d_z, N, h->d_part, s, st));
  HIPCHK(launch_finalize(s, h->d_part, nbv, FIN_RHO, 0, nullptr, st));
  HIPCHK(launch_copy(h->d_p, h->d_z, N, st));
  HIPCHK(hipMemsetAsync(h->d_q, 0, N * sizeof(double), st));
  // the operator writes q completely (DG, or CG through the skeleton gather);
  // otherwise q is accumulated atomically and must be cleared each iteration
  const bool zero_q = h->method == LOR_CG && !apply_cg_uses_skeleton(h->md);
  const int nba = apply_cg_blocks(h->md, h->method != LOR_CG);
  const int chunk = 8;
  int it = 0;
  bool done = false;
  while (!done && it < maxit) {
    const int upto = std::min(maxit, it + chunk);
    for (; it < upto; ++it) {
      rc = apply_A_impl(h, h->d_p, h->d_q, h->d_part, s, st);
      if (rc != LOR_OK) return rc;
      HIPCHK(launch_finalize(s, h->d_part, nba, FIN_PQ, it + 1, nullptr, st));
      HIPCHK(launch_cg_update(x, h->d_r, fcg ? h->d_rold : nullptr, h->d_p, h->d_q, N, s, h->d_part, st));
      HIPCHK(launch_finalize(s, h->d_part, nbv, FIN_RR, it + 1, nullptr, st));
      rc = apply_P_impl(h, h->d_r, h->d_z, s, st);
      if (rc != LOR_OK) return rc;
      HIPCHK(launch_dot_partials(h->d_r, h->d_z, N, h->d_part, s, st));
      if (fcg) HIPCHK(launch_dot_partials(h->d_z, h->d_rold, N, h->d_part2, s, st));
      HIPCHK(launch_finalize(s, h->d_part, nbv, fcg ? FIN_FCG : FIN_RHO, it + 1,
                             fcg ? h->d_part2 : nullptr, st));
      HIPCHK(launch_p_update(h->d_p, zero_q ? h->d_q : nullptr, h->d_z, N, s, st));
    }
    HIPCHK(hipMemcpyAsync(h->h_scal, s, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    done = h->h_scal[S_DONE] != 0.0;
  }
  HIPCHK(hipEventRecord(h->ev1, st));
  // true residual ||b - A x|| (stream-ordered, after the timed region)
  if (zero_q) HIPCHK(hipMemsetAsync(h->d_tmp, 0, N * sizeof(double), st));
  rc = apply_A_impl(h, x, h->d_tmp, nullptr, nullptr, st);
  if (rc != LOR_OK) return rc;
  HIPCHK(launch_sub_dot(b, h->d_tmp, N, h->d_part, st));
  HIPCHK(launch_finalize(s, h->d_part, nbv, FIN_RRTRUE, 0, nullptr, st));
  HIPCHK(hipMemcpyAsync(h->h_scal, s, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const double bb = h->h_scal[S_BB];
  const double rr = h->h_scal[S_RR];
  const double rt = h->h_scal[S_RRTRUE];
  const int iters = int(h->h_scal[S_ITERS]);
  const double fail = h->h_scal[S_FAIL];
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
  int status = LOR_OK;
  if (fail != 0.0)
    status = fail == 2.0 ? LOR_EINVAL : LOR_EBREAKDOWN;
  else if (!h->h_scal[S_DONE])
    status = LOR_ENOCONV;
  if (info) {
    info->iters = iters;
    info->status = status;
    info->rel_res = bb > 0 ? std::sqrt(rr / bb) : 0.0;
    info->rel_res_true = bb > 0 ? std::sqrt(rt / bb) : 0.0;
    info->t_solve = ms * 1e-3;
  }
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

int lor_mdf_order(int dim, const int *m, const double *rows, int natural, int32_t *order,
                  int32_t *level_ptr, int32_t *depth, double *L, double *D) {
  if ((dim != 2 && dim != 3) || !m || !rows) return LOR_EINVAL;
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
  const int rc = mdf_factor(dim, mm, a, natural != 0, res);
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

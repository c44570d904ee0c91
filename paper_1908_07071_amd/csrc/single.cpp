// Set-up and application of the single-patch preconditioner B(1) (Section
// 4.1): one V-cycle of the element-structured LOR hierarchy (Section 3.3)
// over the whole domain, IC(0) smoothing in the chosen elimination order on
// every level but the last, and the exact solve on the last level, the
// original mesh T_p (its interior vertices), by a dense inverse.  Float64.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "lor_handle.h"

namespace {

#define SCHK(x)                                 \
  do {                                          \
    hipError_t e_ = (x);                        \
    if (e_ != hipSuccess) return LOR_EHIP;      \
  } while (0)

constexpr int kGridLevel = 8192;  // default: levels with more rows get a launch of their own

template <class T>
hipError_t upload(lor_handle &h, T **dst, const std::vector<T> &src, hipStream_t st) {
  hipError_t e = h.alloc(dst, std::max<size_t>(src.size(), 1));
  if (e != hipSuccess || src.empty()) return e;
  return hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st);
}

// 1D interpolation from level k+1 to level k on the interior indices of one
// direction (the paper's transfers, linear in reference coordinates).
struct Xfer1D {
  std::vector<int> pc;      // 2 per fine index
  std::vector<double> pw;
  std::vector<int> rf;      // R per coarse index
  std::vector<double> rw;
  int mf = 0, mc = 0, R = 1;
};

Xfer1D xfer_1d(const lor_handle &h, int k, int d) {
  Xfer1D t;
  const std::vector<int> &Xf = h.kept[k], &Xc = h.kept[k + 1];
  const int sf = int(Xf.size()) - 1, sc = int(Xc.size()) - 1, n = h.n[d];
  t.mf = std::max(n * sf - 1, 0);
  t.mc = std::max(n * sc - 1, 0);
  t.pc.assign(size_t(2) * t.mf, -1);
  t.pw.assign(size_t(2) * t.mf, 0.0);
  std::vector<std::vector<std::pair<int, double>>> lists(t.mc);
  const std::vector<double> &x = h.gllx;
  for (int f = 0; f < t.mf; ++f) {
    const int G = f + 1;
    const int e = std::min(G / sf, n - 1);
    const int a = Xf[G - e * sf];
    int C[2];
    double w[2];
    auto it = std::find(Xc.begin(), Xc.end(), a);
    if (it != Xc.end()) {
      C[0] = e * sc + int(it - Xc.begin());
      w[0] = 1.0;
      C[1] = -1;
      w[1] = 0.0;
    } else {
      int hi = 0;
      while (Xc[hi] < a) ++hi;
      const int lo = hi - 1;
      const double xl = x[Xc[lo]], xh = x[Xc[hi]];
      C[0] = e * sc + lo;
      C[1] = e * sc + hi;
      w[0] = (xh - x[a]) / (xh - xl);
      w[1] = (x[a] - xl) / (xh - xl);
    }
    for (int b = 0; b < 2; ++b) {
      const int c = C[b] - 1;  // interior coarse index; boundary values are zero
      if (C[b] < 0 || c < 0 || c >= t.mc || w[b] == 0.0) continue;
      t.pc[2 * f + b] = c;
      t.pw[2 * f + b] = w[b];
      lists[c].push_back({f, w[b]});
    }
  }
  t.R = 1;
  for (auto &l : lists) t.R = std::max<int>(t.R, int(l.size()));
  t.rf.assign(size_t(t.R) * std::max(t.mc, 1), -1);
  t.rw.assign(size_t(t.R) * std::max(t.mc, 1), 0.0);
  for (int c = 0; c < t.mc; ++c)
    for (size_t q = 0; q < lists[c].size(); ++q) {
      t.rf[size_t(c) * t.R + q] = lists[c][q].first;
      t.rw[size_t(c) * t.R + q] = lists[c][q].second;
    }
  return t;
}

}  // namespace

int build_single(lor_handle &h, const std::vector<std::vector<double>> &hst, hipStream_t st) {
  const int dim = h.dim, NS = dim == 3 ? 27 : 9, C = NS / 2, L = h.L;
  h.single.assign(L, SingleLevelDev{});
  h.J = 1;
  const int nf = L - 1;
  h.order_off.assign(size_t(nf) + 1, 0);
  h.sched_off.assign(size_t(nf) + 1, 0);
  h.order_all.clear();
  h.sched_all.clear();
  for (int k = 0; k < L; ++k) {
    SingleLevelDev &lv = h.single[k];
    const int s = int(h.kept[k].size()) - 1;
    int lng[3] = {1, 1, 1};
    lv.n = 1;
    for (int d = 0; d < 3; ++d) {
      lng[d] = d < dim ? h.n[d] * s + 1 : 1;
      lv.m[d] = d < dim ? std::max(lng[d] - 2, 0) : 1;
      lv.n *= lv.m[d];
    }
    const int64_t np = h.npts[k];
    auto grid_index = [&](int64_t i) {
      const int ix = int(i % lv.m[0]), iy = int((i / lv.m[0]) % lv.m[1]),
                iz = int(i / (int64_t(lv.m[0]) * lv.m[1]));
      return int64_t(ix + 1) + int64_t(lng[0]) * (int64_t(iy + 1) + (dim == 3 ? int64_t(lng[1]) * (iz + 1) : 0));
    };
    auto in_box = [&](int64_t i, int sl, int64_t *j) {
      const int ix = int(i % lv.m[0]), iy = int((i / lv.m[0]) % lv.m[1]),
                iz = int(i / (int64_t(lv.m[0]) * lv.m[1]));
      const int q[3] = {ix + sl % 3 - 1, iy + (sl / 3) % 3 - 1, dim == 3 ? iz + sl / 9 - 1 : 0};
      for (int d = 0; d < 3; ++d)
        if (q[d] < 0 || q[d] >= lv.m[d]) return false;
      *j = q[0] + int64_t(lv.m[0]) * (q[1] + int64_t(lv.m[1]) * q[2]);
      return true;
    };
    if (k < L - 1) {
      h.order_off[k + 1] = h.order_off[k] + int32_t(lv.n);
      if (lv.n <= 0) {
        h.sched_off[k + 1] = h.sched_off[k];
        continue;
      }
      if (lv.n > (int64_t(1) << 30) / NS) return LOR_EINVAL;
      std::vector<double> rows(size_t(lv.n) * NS);
      for (int64_t i = 0; i < lv.n; ++i) {
        const int64_t g = grid_index(i);
        for (int sl = 0; sl < NS; ++sl) rows[size_t(i) * NS + sl] = hst[k][size_t(sl) * np + g];
      }
      MdfResult res;
      const int rc = mdf_factor(dim, lv.m, rows, h.opt.ordering, res);
      if (rc != LOR_OK) return rc;
      h.order_all.insert(h.order_all.end(), res.order.begin(), res.order.end());
      h.sched_all.insert(h.sched_all.end(), res.level_ptr.begin(), res.level_ptr.end());
      h.sched_off[k + 1] = h.sched_off[k] + int32_t(res.level_ptr.size());
      std::vector<double> invD(lv.n);
      std::vector<int> lmask(lv.n);
      for (int64_t i = 0; i < lv.n; ++i) {
        invD[i] = 1.0 / res.D[i];
        int inbox = 0;
        int64_t j;
        for (int sl = 0; sl < NS; ++sl)
          if (sl != C && in_box(i, sl, &j)) inbox |= 1 << sl;
        lmask[i] = inbox & ~res.earlier[i];
      }
      lv.lptr_host = res.level_ptr;
      const int depth = int(res.level_ptr.size()) - 1;
      const int big = h.opt.sweep_grid_rows > 0 ? h.opt.sweep_grid_rows : kGridLevel;
      for (int l = 0; l < depth;) {
        const int cnt = res.level_ptr[l + 1] - res.level_ptr[l];
        if (cnt > big) {
          lv.segs.push_back({l, l + 1, 1});
          ++l;
          continue;
        }
        int l1 = l + 1;
        while (l1 < depth && res.level_ptr[l1 + 1] - res.level_ptr[l1] <= big) ++l1;
        lv.segs.push_back({l, l1, 0});
        l = l1;
      }
      SCHK(upload(h, &lv.sched, res.sched, st));
      SCHK(upload(h, &lv.lptr, res.level_ptr, st));
      SCHK(upload(h, &lv.Lv, res.L, st));
      SCHK(upload(h, &lv.invD, invD, st));
      SCHK(upload(h, &lv.emask, res.earlier, st));
      SCHK(upload(h, &lv.lmask, lmask, st));
      SCHK(h.alloc(&lv.r, size_t(lv.n)));
      if (k > 0) {
        SCHK(h.alloc(&lv.x, size_t(lv.n)));
        SCHK(h.alloc(&lv.b, size_t(lv.n)));
      }
      // transfers to level k + 1
      SingleXfer &t = lv.xf;
      for (int d = 0; d < 3; ++d) {
        t.mf[d] = t.mc[d] = t.R[d] = 1;
        t.pc[d] = t.rf[d] = nullptr;
        t.pw[d] = t.rw[d] = nullptr;
      }
      for (int d = 0; d < dim; ++d) {
        Xfer1D x1 = xfer_1d(h, k, d);
        t.mf[d] = x1.mf;
        t.mc[d] = x1.mc;
        t.R[d] = x1.R;
        int *pc, *rf;
        double *pw, *rw;
        SCHK(upload(h, &pc, x1.pc, st));
        SCHK(upload(h, &pw, x1.pw, st));
        SCHK(upload(h, &rf, x1.rf, st));
        SCHK(upload(h, &rw, x1.rw, st));
        t.pc[d] = pc;
        t.pw[d] = pw;
        t.rf[d] = rf;
        t.rw[d] = rw;
      }
      // keep the host rows alive only as long as the uploads need them
      SCHK(hipStreamSynchronize(st));
    } else if (lv.n > 0) {
      // T_p: the level matrix on the interior vertices, inverted
      if (lv.n > 40000) return LOR_EINVAL;
      const int n = int(lv.n);
      std::vector<double> A(size_t(n) * n, 0.0);
      for (int64_t i = 0; i < lv.n; ++i) {
        const int64_t g = grid_index(i);
        int64_t j;
        for (int sl = 0; sl < NS; ++sl)
          if (in_box(i, sl, &j)) A[size_t(i) * n + j] = hst[k][size_t(sl) * np + g];
      }
      SCHK(h.alloc(&lv.ainv, A.size()));
      SCHK(hipMemcpyAsync(lv.ainv, A.data(), A.size() * sizeof(double), hipMemcpyHostToDevice, st));
      const int rc = coarse_inverse(n, lv.ainv, st);
      if (rc != LOR_OK) return rc;
      SCHK(h.alloc(&lv.x, size_t(lv.n)));
      SCHK(h.alloc(&lv.b, size_t(lv.n)));
      SCHK(hipStreamSynchronize(st));
    }
  }
  return LOR_OK;
}

namespace {

int vcycle(lor_handle *h, int k, const double *b, double *x, const double *flag, hipStream_t st) {
  SingleLevelDev &lv = h->single[k];
  if (lv.n <= 0) return LOR_OK;
  if (k == h->L - 1) {
    SCHK(launch_gemv(int(lv.n), lv.ainv, b, x, flag, st));
    return LOR_OK;
  }
  const int dim = h->dim, s = int(h->kept[k].size()) - 1;
  const int lng[3] = {h->n[0] * s + 1, h->n[1] * s + 1, dim == 3 ? h->n[2] * s + 1 : 1};
  const double *A = h->d_stencil[k];
  // pre-smoothing from zero: x = M^-1 b
  SCHK(launch_single_sweep(dim, true, lv, b, x, flag, st));
  SCHK(launch_single_sweep(dim, false, lv, x, x, flag, st));
  SCHK(launch_single_residual(dim, A, h->npts[k], lng, lv.m, b, x, lv.r, flag, st));
  SingleLevelDev &cv = h->single[k + 1];
  if (cv.n > 0) {
    SCHK(launch_single_transfer(dim, false, lv.xf, lv.r, cv.b, flag, st));
    const int rc = vcycle(h, k + 1, cv.b, cv.x, flag, st);
    if (rc != LOR_OK) return rc;
    SCHK(launch_single_transfer(dim, true, lv.xf, cv.x, x, flag, st));
    SCHK(launch_single_residual(dim, A, h->npts[k], lng, lv.m, b, x, lv.r, flag, st));
  }
  // post-smoothing: x += M^-1 r (in place on r)
  SCHK(launch_single_sweep(dim, true, lv, lv.r, lv.r, flag, st));
  SCHK(launch_single_sweep(dim, false, lv, lv.r, lv.r, flag, st));
  SCHK(launch_axpy1(x, lv.r, lv.n, flag, st));
  return LOR_OK;
}

}  // namespace

int apply_single(lor_handle *h, const double *r, double *z, const double *flag, hipStream_t st) {
  if (h->single.empty()) return LOR_ESTATE;
  if (h->single[0].n <= 0) return LOR_OK;
  return vcycle(h, 0, r, z, flag, st);
}

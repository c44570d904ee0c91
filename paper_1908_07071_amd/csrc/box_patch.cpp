// Box-patch Schwarz preconditioners (host set-up and application):
//   B(1)  one patch, the whole domain (Section 4.1);
//   B(n)  n overlapping slabs of elements (Section 4.5);
//   vertex patches enlarged for isotropic overlap, plus the coarse space
//         (Section 4.5).
// A patch is a box of elements [a_d, b_d); its unknowns on level k are the
// level-grid points strictly inside it.  Its solver is one V-cycle of the
// element-structured LOR hierarchy (Section 3.3) restricted to the box: IC(0)
// smoothing in the chosen elimination order on every level but the last, the
// exact solve (a dense inverse) on the box's part of T_p.  Small boxes run
// their V-cycles one workgroup each, all in one launch; larger ones take
// per-level launches on four streams.  B(1) writes z directly, the others
// gather the patch residual and add the (optionally weighted) correction
// back, one colour of boxes (disjoint level-0 boxes) at a time.  Float64.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <utility>
#include <vector>

#include "host_plan.h"
#include "lor_handle.h"

namespace {

#define SCHK(x)                                 \
  do {                                          \
    hipError_t e_ = (x);                        \
    if (e_ != hipSuccess) return LOR_EHIP;      \
  } while (0)

constexpr int kGridLevel = 512;    // default: levels with more rows get a launch of their own
constexpr int kHostInverse = 512;  // coarsest box levels up to this size are inverted on the host

template <class T>
hipError_t upload(lor_handle &h, T **dst, const std::vector<T> &src, hipStream_t st) {
  hipError_t e = h.alloc(dst, std::max<size_t>(src.size(), 1));
  if (e != hipSuccess || src.empty()) return e;
  return hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st);
}

// 1D interpolation from level k+1 to level k between the interior indices of
// a box [a, b) in direction d (linear in reference coordinates, Section 3.3).
struct Xfer1D {
  std::vector<int> pc;  // 2 per fine index
  std::vector<double> pw;
  std::vector<int> rf;  // R per coarse index
  std::vector<double> rw;
  int mf = 0, mc = 0, R = 1;
};

Xfer1D xfer_1d(const lor_handle &h, int k, int d, int a, int b) {
  Xfer1D t;
  const std::vector<int> &Xf = h.kept[k], &Xc = h.kept[k + 1];
  const int sf = int(Xf.size()) - 1, sc = int(Xc.size()) - 1, n = h.n[d];
  const int lof = a * sf + 1, loc = a * sc + 1;
  t.mf = std::max((b - a) * sf - 1, 0);
  t.mc = std::max((b - a) * sc - 1, 0);
  t.pc.assign(size_t(2) * t.mf, -1);
  t.pw.assign(size_t(2) * t.mf, 0.0);
  std::vector<std::vector<std::pair<int, double>>> lists(t.mc);
  const std::vector<double> &x = h.gllx;
  for (int f = 0; f < t.mf; ++f) {
    const int G = lof + f;
    const int e = std::min(G / sf, n - 1);
    const int av = Xf[G - e * sf];
    int C[2];
    double w[2];
    auto it = std::find(Xc.begin(), Xc.end(), av);
    if (it != Xc.end()) {
      C[0] = e * sc + int(it - Xc.begin());
      w[0] = 1.0;
      C[1] = -1;
      w[1] = 0.0;
    } else {
      int hi = 0;
      while (Xc[hi] < av) ++hi;
      const int lo = hi - 1;
      const double xl = x[Xc[lo]], xh = x[Xc[hi]];
      C[0] = e * sc + lo;
      C[1] = e * sc + hi;
      w[0] = (xh - x[av]) / (xh - xl);
      w[1] = (x[av] - xl) / (xh - xl);
    }
    for (int q = 0; q < 2; ++q) {
      const int c = C[q] - loc;  // box-local coarse index; outside the box the value is zero
      if (C[q] < 0 || c < 0 || c >= t.mc || w[q] == 0.0) continue;
      t.pc[2 * f + q] = c;
      t.pw[2 * f + q] = w[q];
      lists[c].push_back({f, w[q]});
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

// in-place inverse of a small SPD matrix (Gauss-Jordan, no pivoting)
bool host_inverse(std::vector<double> &A, int n) {
  for (int k = 0; k < n; ++k) {
    const double piv = A[size_t(k) * n + k];
    if (!(std::isfinite(piv) && piv > 0.0)) return false;
    const double ip = 1.0 / piv;
    for (int j = 0; j < n; ++j) A[size_t(k) * n + j] *= ip;
    A[size_t(k) * n + k] = ip;
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      const double f = A[size_t(i) * n + k];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) A[size_t(i) * n + j] -= f * A[size_t(k) * n + j];
      A[size_t(i) * n + k] = -f * ip;
    }
  }
  return true;
}

// squared distance between two vertices, coordinates summed in order
double vdist2(const lor_handle &h, const int *v, const int *w) {
  const int nv0 = h.n[0] + 1, nv1 = h.n[1] + 1;
  const int64_t iv = v[0] + int64_t(nv0) * (v[1] + int64_t(nv1) * v[2]);
  const int64_t iw = w[0] + int64_t(nv0) * (w[1] + int64_t(nv1) * w[2]);
  double acc = 0.0;
  for (int t = 0; t < h.dim; ++t) {
    const double d = h.verts[size_t(iw) * h.dim + t] - h.verts[size_t(iv) * h.dim + t];
    acc = acc + d * d;
  }
  return acc;
}

}  // namespace

// The element boxes of the patch mode (see the oracle's readings): B(1) the
// domain; B(n) slabs along x with bounds i n / nslabs widened by one element
// on inner sides; isotropic vertex patches grown from each vertex, per
// direction and sense, until the vertex reached is at least 0.9 times the
// longest edge at the vertex away (squared lengths against 0.81 delta^2) or
// the boundary is reached.
std::vector<std::array<int, 6>> patch_boxes(const lor_handle &h) {
  std::vector<std::array<int, 6>> out;
  const int dim = h.dim;
  auto full = [&]() {
    std::array<int, 6> b{};
    for (int d = 0; d < 3; ++d) {
      b[d] = 0;
      b[3 + d] = d < dim ? h.n[d] : 1;
    }
    return b;
  };
  if (h.opt.patch_mode == LOR_PATCH_SINGLE) {
    out.push_back(full());
  } else if (h.opt.patch_mode == LOR_PATCH_SLABS) {
    const int ns = h.opt.nslabs, n = h.n[0];
    for (int i = 0; i < ns; ++i) {
      std::array<int, 6> b = full();
      const int a0 = int(int64_t(i) * n / ns), b0 = int(int64_t(i + 1) * n / ns);
      b[0] = std::max(a0 - 1, 0);
      b[3] = std::min(b0 + 1, n);
      out.push_back(b);
    }
  } else if (h.opt.patch_mode == LOR_PATCH_VERTEX_ISO) {
    const int nv[3] = {h.n[0] + 1, h.n[1] + 1, dim == 3 ? h.n[2] + 1 : 1};
    for (int j = 0; j < nv[0] * nv[1] * nv[2]; ++j) {
      const int v[3] = {j % nv[0], (j / nv[0]) % nv[1], j / (nv[0] * nv[1])};
      double delta2 = 0.0;
      for (int d = 0; d < dim; ++d)
        for (int sg = -1; sg <= 1; sg += 2) {
          int w[3] = {v[0], v[1], v[2]};
          w[d] += sg;
          if (w[d] >= 0 && w[d] <= h.n[d]) delta2 = std::max(delta2, vdist2(h, v, w));
        }
      std::array<int, 6> b{};
      for (int d = 0; d < 3; ++d) {
        if (d >= dim) {
          b[d] = 0;
          b[3 + d] = 1;
          continue;
        }
        int ext[2];
        for (int q = 0; q < 2; ++q) {
          const int sg = q == 0 ? -1 : 1;
          int k = 0;
          for (;;) {
            ++k;
            int w[3] = {v[0], v[1], v[2]};
            w[d] += sg * k;
            if (w[d] <= 0 || w[d] >= h.n[d] || vdist2(h, v, w) >= 0.81 * delta2) break;
          }
          ext[q] = k;
        }
        b[d] = std::max(v[d] - ext[0], 0);
        b[3 + d] = std::min(v[d] + ext[1], h.n[d]);
      }
      out.push_back(b);
    }
  }
  return out;
}

int build_boxes(lor_handle &h, const std::vector<std::vector<double>> &hst, hipStream_t st) {
  const int dim = h.dim, NS = dim == 3 ? 27 : 9, C = NS / 2, L = h.L, nf = L - 1;
  const std::vector<std::array<int, 6>> boxes = patch_boxes(h);
  h.boxes.assign(boxes.size(), BoxPatchDev{});
  h.J = int(boxes.size());
  h.order_off.assign(size_t(h.J) * nf + 1, 0);
  h.sched_off.assign(size_t(h.J) * nf + 1, 0);
  h.order_all.clear();
  h.sched_all.clear();
  std::vector<int64_t> maxn(L, 0);
  std::vector<double> count(size_t(h.ncg), 0.0);
  int t = 0;
  for (size_t j = 0; j < boxes.size(); ++j) {
    BoxPatchDev &bp = h.boxes[j];
    for (int d = 0; d < 3; ++d) {
      bp.a[d] = boxes[j][d];
      bp.b[d] = boxes[j][3 + d];
    }
    bp.lv.assign(L, SingleLevelDev{});
    for (int k = 0; k < L; ++k) {
      SingleLevelDev &lv = bp.lv[k];
      const int s = int(h.kept[k].size()) - 1;
      int lng[3] = {1, 1, 1};
      lv.n = 1;
      for (int d = 0; d < 3; ++d) {
        lng[d] = d < dim ? h.n[d] * s + 1 : 1;
        lv.lo[d] = d < dim ? bp.a[d] * s + 1 : 0;
        lv.m[d] = d < dim ? std::max((bp.b[d] - bp.a[d]) * s - 1, 0) : 1;
        lv.n *= lv.m[d];
      }
      maxn[k] = std::max(maxn[k], lv.n);
      const int64_t np = h.npts[k];
      auto grid_index = [&](int64_t i) {
        const int ix = int(i % lv.m[0]), iy = int((i / lv.m[0]) % lv.m[1]),
                  iz = int(i / (int64_t(lv.m[0]) * lv.m[1]));
        return int64_t(ix + lv.lo[0]) +
               int64_t(lng[0]) * (int64_t(iy + lv.lo[1]) + (dim == 3 ? int64_t(lng[1]) * (iz + lv.lo[2]) : 0));
      };
      auto in_box = [&](int64_t i, int sl, int64_t *jj) {
        const int ix = int(i % lv.m[0]), iy = int((i / lv.m[0]) % lv.m[1]),
                  iz = int(i / (int64_t(lv.m[0]) * lv.m[1]));
        const int q[3] = {ix + sl % 3 - 1, iy + (sl / 3) % 3 - 1, dim == 3 ? iz + sl / 9 - 1 : 0};
        for (int d = 0; d < 3; ++d)
          if (q[d] < 0 || q[d] >= lv.m[d]) return false;
        *jj = q[0] + int64_t(lv.m[0]) * (q[1] + int64_t(lv.m[1]) * q[2]);
        return true;
      };
      if (k == 0 && lv.n > 0) {
        for (int64_t i = 0; i < lv.n; ++i) {
          const int ix = int(i % lv.m[0]), iy = int((i / lv.m[0]) % lv.m[1]),
                    iz = int(i / (int64_t(lv.m[0]) * lv.m[1]));
          const int64_t u = (ix + lv.lo[0] - 1) +
                            int64_t(h.md.nu[0]) * ((iy + lv.lo[1] - 1) + (dim == 3 ? int64_t(h.md.nu[1]) * (iz + lv.lo[2] - 1) : 0));
          count[u] += 1.0;
        }
      }
      if (k < L - 1) {
        h.order_off[t + 1] = h.order_off[t] + int32_t(lv.n);
        if (lv.n <= 0) {
          h.sched_off[t + 1] = h.sched_off[t];
          ++t;
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
        h.sched_off[t + 1] = h.sched_off[t] + int32_t(res.level_ptr.size());
        ++t;
        std::vector<double> invD(lv.n);
        std::vector<int> lmask(lv.n);
        for (int64_t i = 0; i < lv.n; ++i) {
          invD[i] = 1.0 / res.D[i];
          int inbox = 0;
          int64_t jj;
          for (int sl = 0; sl < NS; ++sl)
            if (sl != C && in_box(i, sl, &jj)) inbox |= 1 << sl;
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
        SingleXfer &xf = lv.xf;
        for (int d = 0; d < 3; ++d) {
          xf.mf[d] = xf.mc[d] = xf.R[d] = 1;
          xf.pc[d] = xf.rf[d] = nullptr;
          xf.pw[d] = xf.rw[d] = nullptr;
        }
        for (int d = 0; d < dim; ++d) {
          Xfer1D x1 = xfer_1d(h, k, d, bp.a[d], bp.b[d]);
          xf.mf[d] = x1.mf;
          xf.mc[d] = x1.mc;
          xf.R[d] = x1.R;
          int *pc, *rf;
          double *pw, *rw;
          SCHK(upload(h, &pc, x1.pc, st));
          SCHK(upload(h, &pw, x1.pw, st));
          SCHK(upload(h, &rf, x1.rf, st));
          SCHK(upload(h, &rw, x1.rw, st));
          xf.pc[d] = pc;
          xf.pw[d] = pw;
          xf.rf[d] = rf;
          xf.rw[d] = rw;
        }
        SCHK(hipStreamSynchronize(st));  // the host vectors above go out of scope
      } else if (lv.n > 0) {
        // the box's part of T_p (its interior vertices), inverted
        if (lv.n > 40000) return LOR_EINVAL;
        const int n = int(lv.n);
        std::vector<double> A(size_t(n) * n, 0.0);
        for (int64_t i = 0; i < lv.n; ++i) {
          const int64_t g = grid_index(i);
          int64_t jj;
          for (int sl = 0; sl < NS; ++sl)
            if (in_box(i, sl, &jj)) A[size_t(i) * n + jj] = hst[k][size_t(sl) * np + g];
        }
        if (n <= kHostInverse) {
          if (!host_inverse(A, n)) return LOR_EPIVOT;
          SCHK(upload(h, &lv.ainv, A, st));
        } else {
          SCHK(h.alloc(&lv.ainv, A.size()));
          SCHK(hipMemcpyAsync(lv.ainv, A.data(), A.size() * sizeof(double), hipMemcpyHostToDevice, st));
          const int rc = coarse_inverse(n, lv.ainv, st);
          if (rc != LOR_OK) return rc;
        }
        SCHK(hipStreamSynchronize(st));
      }
    }
  }
  // level vectors of the per-level path (one set per stream)
  h.box_x.assign(L, nullptr);
  h.box_b.assign(L, nullptr);
  h.box_r.assign(L, nullptr);
  const bool single = h.opt.patch_mode == LOR_PATCH_SINGLE;
  for (int k = 0; k < L; ++k) {
    if (maxn[k] <= 0) continue;
    if (!(single && k == 0)) {  // B(1) reads r and writes z directly on level 0
      SCHK(h.alloc(&h.box_x[k], size_t(maxn[k])));
      SCHK(h.alloc(&h.box_b[k], size_t(maxn[k])));
    }
    SCHK(h.alloc(&h.box_r[k], size_t(maxn[k])));
  }
  for (BoxPatchDev &bp : h.boxes)
    for (int k = 0; k < L; ++k) {
      bp.lv[k].x = h.box_x[k];
      bp.lv[k].b = h.box_b[k];
      bp.lv[k].r = h.box_r[k];
    }
  // colours (greedy, in box order): boxes of one colour have disjoint
  // level-0 point ranges, so their corrections can be added side by side
  {
    std::vector<BoxRange> rg(h.boxes.size());
    for (size_t j = 0; j < h.boxes.size(); ++j) {
      const SingleLevelDev &l0 = h.boxes[j].lv[0];
      for (int d = 0; d < 3; ++d) {
        rg[j].lo[d] = l0.lo[d];
        rg[j].m[d] = l0.m[d];
      }
      rg[j].n = single ? 0 : l0.n;  // B(1): one box, one colour
    }
    h.box_color = greedy_box_colours(rg, dim, &h.box_ncolor);
  }
  // boxes for one workgroup each: no dependency level over `big` rows, a
  // finest level of at most kBoxFuseRows rows, level vectors of their own
  // while they fit kBoxWorkDoubles
  {
    const int big = h.opt.sweep_grid_rows > 0 ? h.opt.sweep_grid_rows : kGridLevel;
    const size_t nb = h.boxes.size();
    h.box_fused.assign(nb, 0);
    h.box_vo.assign(nb * L, 0);
    h.box_vl.assign(nb * L, 0);
    int64_t total = 0;
    std::vector<int> list;
    for (size_t j = 0; j < nb; ++j) {
      const BoxPatchDev &bp = h.boxes[j];
      bool ok = bp.lv[0].n > 0 && bp.lv[0].n <= kBoxFuseRows;
      int64_t need = 0;
      for (int k = 0; ok && k < L && bp.lv[k].n > 0; ++k) {
        const std::vector<int> &lp = bp.lv[k].lptr_host;
        for (size_t l = 0; ok && l + 1 < lp.size(); ++l) ok = lp[l + 1] - lp[l] <= big;
        need += 3 * ((bp.lv[k].n + 3) / 4 * 4);
      }
      if (!ok || total + need > kBoxWorkDoubles) continue;
      h.box_fused[j] = 1;
      list.push_back(int(j));
      for (int k = 0; k < L && bp.lv[k].n > 0; ++k) {
        const int64_t len = (bp.lv[k].n + 3) / 4 * 4;
        h.box_vo[j * L + k] = total;
        h.box_vl[j * L + k] = len;
        total += 3 * len;
      }
    }
    h.box_nfused = int(list.size());
    h.box_grid.L = L;
    h.box_grid.lds_rows = 0;
    for (int j : list) h.box_grid.lds_rows = std::max<int>(h.box_grid.lds_rows, int(h.boxes[j].lv[0].n));
    h.box_list_off.assign(size_t(h.box_ncolor) + 1, 0);
    h.box_unfused.assign(size_t(h.box_ncolor), 0);
    for (int c = 0; c < h.box_ncolor; ++c) {
      for (size_t j = 0; j < nb; ++j) {
        if (h.box_color[j] != c || h.boxes[j].lv[0].n <= 0) continue;
        if (h.box_fused[j]) list.push_back(int(j));
        else ++h.box_unfused[c];
      }
      h.box_list_off[c + 1] = int(list.size()) - h.box_nfused;
    }
    // every box on the one-workgroup path: the additions of all colours in
    // one launch, each point's boxes in colour order
    h.box_add_npt = 0;
    bool all = !single && h.box_nfused > 0;
    for (int c : h.box_unfused) all = all && c == 0;
    if (all) {
      std::vector<std::pair<int64_t, int64_t>> ent;  // (point, offset of its x value)
      for (size_t t = size_t(h.box_nfused); t < list.size(); ++t) {
        const int j = list[t];
        const SingleLevelDev &l0 = h.boxes[j].lv[0];
        const int64_t vo = h.box_vo[size_t(j) * L];
        for (int64_t i = 0; i < l0.n; ++i) {
          const int ix = int(i % l0.m[0]), iy = int((i / l0.m[0]) % l0.m[1]),
                    iz = int(i / (int64_t(l0.m[0]) * l0.m[1]));
          const int64_t u = (ix + l0.lo[0] - 1) +
                            int64_t(h.md.nu[0]) * ((iy + l0.lo[1] - 1) + (dim == 3 ? int64_t(h.md.nu[1]) * (iz + l0.lo[2] - 1) : 0));
          ent.push_back({u, vo + i});
        }
      }
      std::stable_sort(ent.begin(), ent.end(),
                       [](const std::pair<int64_t, int64_t> &a, const std::pair<int64_t, int64_t> &b) {
                         return a.first < b.first;
                       });
      std::vector<int64_t> ptr(1, 0), pts, src(ent.size());
      for (size_t e = 0; e < ent.size(); ++e) {
        if (e == 0 || ent[e].first != ent[e - 1].first) {
          if (e > 0) ptr.push_back(int64_t(e));
          pts.push_back(ent[e].first);
        }
        src[e] = ent[e].second;
      }
      ptr.push_back(int64_t(ent.size()));
      h.box_add_npt = int64_t(pts.size());
      SCHK(upload(h, &h.d_add_ptr, ptr, st));
      SCHK(upload(h, &h.d_add_pts, pts, st));
      SCHK(upload(h, &h.d_add_src, src, st));
      SCHK(hipStreamSynchronize(st));
    }
    if (h.box_nfused > 0) {
      SCHK(upload(h, &h.d_box_list, list, st));
      SCHK(hipStreamSynchronize(st));  // `list` goes out of scope below
      SCHK(h.alloc(&h.d_box_desc, nb));
      SCHK(h.alloc(&h.d_box_work, size_t(total)));
      const int rc = refresh_box_descs(h, st);
      if (rc != LOR_OK) return rc;
    }
  }
  bool unfused = false;
  for (int c : h.box_unfused) unfused = unfused || c > 0;
  if (!single && h.boxes.size() > 1 && unfused) {
    // the other streams' level vectors, the streams and their events
    for (int t = 0; t < lor_handle::kBoxStreams - 1; ++t) {
      h.box_sx[t].assign(L, nullptr);
      h.box_sb[t].assign(L, nullptr);
      h.box_sr[t].assign(L, nullptr);
      for (int k = 0; k < L; ++k) {
        if (maxn[k] <= 0) continue;
        SCHK(h.alloc(&h.box_sx[t][k], size_t(maxn[k])));
        SCHK(h.alloc(&h.box_sb[t][k], size_t(maxn[k])));
        SCHK(h.alloc(&h.box_sr[t][k], size_t(maxn[k])));
      }
    }
    for (hipStream_t &t : h.box_st) SCHK(hipStreamCreateWithFlags(&t, hipStreamNonBlocking));
    for (hipEvent_t &e : h.box_ev) SCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  if (h.opt.prolong_weights == LOR_PROLONG_POU && h.opt.patch_mode != LOR_PATCH_SINGLE) {
    std::vector<double> w(count.size());
    for (size_t i = 0; i < count.size(); ++i) w[i] = count[i] > 0.0 ? 1.0 / count[i] : 0.0;
    SCHK(upload(h, &h.d_box_w, w, st));
    SCHK(hipStreamSynchronize(st));
  }
  return LOR_OK;
}

int refresh_box_descs(lor_handle &h, hipStream_t st) {
  if (!h.d_box_desc) return LOR_OK;
  const int dim = h.dim, L = h.L;
  BoxGrid &g = h.box_grid;
  g.L = L;
  for (int k = 0; k < L; ++k) {
    const int s = int(h.kept[k].size()) - 1;
    g.stencil[k] = h.d_stencil[k];
    g.npts[k] = h.npts[k];
    for (int d = 0; d < 3; ++d) g.lng[k][d] = d < dim ? h.n[d] * s + 1 : 1;
  }
  std::vector<BoxDesc> desc(h.boxes.size());
  for (size_t j = 0; j < h.boxes.size(); ++j) {
    BoxDesc &bd = desc[j];
    std::memset(&bd, 0, sizeof(bd));
    for (int k = 0; k < L; ++k) {
      const SingleLevelDev &lv = h.boxes[j].lv[k];
      BoxLevelDesc &o = bd.lv[k];
      for (int d = 0; d < 3; ++d) {
        o.lo[d] = lv.lo[d];
        o.m[d] = lv.m[d];
      }
      o.n = int(std::max<int64_t>(lv.n, 0));
      o.depth = lv.lptr_host.empty() ? 0 : int(lv.lptr_host.size()) - 1;
      o.sched = lv.sched;
      o.lptr = lv.lptr;
      o.Lv = lv.Lv;
      o.invD = lv.invD;
      o.emask = lv.emask;
      o.lmask = lv.lmask;
      o.xf = lv.xf;
      o.ainv = lv.ainv;
      o.vo = h.box_vo[j * L + k];
      o.vl = h.box_vl[j * L + k];
    }
  }
  SCHK(hipMemcpyAsync(h.d_box_desc, desc.data(), desc.size() * sizeof(BoxDesc), hipMemcpyHostToDevice, st));
  SCHK(hipStreamSynchronize(st));
  return LOR_OK;
}

namespace {

// The level vectors a box patch's V-cycle works in (one set per stream).
struct BoxBufs {
  double *const *x, *const *b, *const *r;  // per level
};

BoxBufs box_bufs(const lor_handle *h, int set) {
  if (set == 0) return {h->box_x.data(), h->box_b.data(), h->box_r.data()};
  return {h->box_sx[set - 1].data(), h->box_sb[set - 1].data(), h->box_sr[set - 1].data()};
}

int vcycle(lor_handle *h, BoxPatchDev &bp, int k, const double *b, double *x, const double *flag,
           hipStream_t st, const BoxBufs &buf) {
  SingleLevelDev &lv = bp.lv[k];
  double *rk = buf.r[k];
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
  SCHK(launch_single_residual(dim, A, h->npts[k], lng, lv.lo, lv.m, b, x, rk, flag, st));
  SingleLevelDev &cv = bp.lv[k + 1];
  if (cv.n > 0) {
    double *cb = buf.b[k + 1], *cx = buf.x[k + 1];
    SCHK(launch_single_transfer(dim, false, lv.xf, rk, cb, flag, st));
    const int rc = vcycle(h, bp, k + 1, cb, cx, flag, st, buf);
    if (rc != LOR_OK) return rc;
    SCHK(launch_single_transfer(dim, true, lv.xf, cx, x, flag, st));
    SCHK(launch_single_residual(dim, A, h->npts[k], lng, lv.lo, lv.m, b, x, rk, flag, st));
  }
  // post-smoothing: x += M^-1 r (in place on r)
  SCHK(launch_single_sweep(dim, true, lv, rk, rk, flag, st));
  SCHK(launch_single_sweep(dim, false, lv, rk, rk, flag, st));
  SCHK(launch_axpy1(x, rk, lv.n, flag, st));
  return LOR_OK;
}

}  // namespace

int apply_boxes(lor_handle *h, const double *r, double *z, const double *flag, hipStream_t st) {
  if (h->boxes.empty()) return LOR_ESTATE;
  const bool single = h->opt.patch_mode == LOR_PATCH_SINGLE;
  if (single && h->boxes[0].lv[0].n <= 0) return LOR_OK;
  if (single && !h->box_fused[0]) {
    // one box, the whole domain: level 0 is the L-vector
    return vcycle(h, h->boxes[0], 0, r, z, flag, st, box_bufs(h, 0));
  }
  // every one-workgroup box's V-cycle in one launch (B(1): straight into z);
  // then colour by colour their corrections added to z in one launch, and
  // the other boxes' V-cycles on the side streams in turn (one after another
  // on `st` while a graph is captured): the same additions to z either way
  SCHK(launch_box_vcycles(h->dim, h->d_box_desc, h->d_box_list, h->box_nfused, h->box_grid, h->md, r, z,
                          single ? 1 : 0, h->d_box_work, flag, st));
  if (single) return LOR_OK;
  if (h->box_add_npt > 0) {  // every box above: all additions in one launch
    SCHK(launch_box_add_points(h->d_add_ptr, h->d_add_pts, h->d_add_src, h->box_add_npt, h->d_box_w, z,
                               h->d_box_work, flag, st));
    return LOR_OK;
  }
  constexpr int NS = lor_handle::kBoxStreams;
  const bool side = !h->capturing && h->box_st[0] != nullptr;
  for (int c = 0; c < h->box_ncolor; ++c) {
    const bool fork = side && h->box_unfused[c] > 0;
    if (fork) {
      SCHK(hipEventRecord(h->box_ev[NS], st));
      for (hipStream_t t : h->box_st) SCHK(hipStreamWaitEvent(t, h->box_ev[NS], 0));
    }
    const int l0 = h->box_list_off[c], cnt = h->box_list_off[c + 1] - l0;
    if (cnt > 0)
      SCHK(launch_box_add(h->dim, h->d_box_desc, h->d_box_list + h->box_nfused + l0, cnt, h->md, h->d_box_w,
                          z, h->d_box_work, flag, st));
    int turn = 0;
    for (size_t j = 0; h->box_unfused[c] > 0 && j < h->boxes.size(); ++j) {
      if (h->box_color[j] != c || h->box_fused[j]) continue;
      BoxPatchDev &bp = h->boxes[j];
      SingleLevelDev &lv0 = bp.lv[0];
      if (lv0.n <= 0) continue;
      const int set = fork ? turn++ % NS : 0;
      hipStream_t s = fork ? h->box_st[set] : st;
      const BoxBufs buf = box_bufs(h, set);
      double *b0 = buf.b[0], *x0 = buf.x[0];
      SCHK(launch_box_gather(h->dim, h->md, lv0.lo, lv0.m, r, b0, flag, s));
      const int rc = vcycle(h, bp, 0, b0, x0, flag, s, buf);
      if (rc != LOR_OK) return rc;
      SCHK(launch_box_scatter(h->dim, h->md, lv0.lo, lv0.m, x0, h->d_box_w, z, flag, s));
    }
    if (fork)
      for (int t = 0; t < NS; ++t) {
        SCHK(hipEventRecord(h->box_ev[t], h->box_st[t]));
        SCHK(hipStreamWaitEvent(st, h->box_ev[t], 0));
      }
  }
  return LOR_OK;
}

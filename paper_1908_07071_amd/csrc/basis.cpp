// Gauss-Lobatto nodes and weights on [0,1], Lagrange derivative matrix and
// the element-structured coarsening rule (Sections 3.1 and 3.3).
//
// The nodes and weights are computed by Newton's method in IEEE binary128
// arithmetic and rounded once to float64, i.e. they are the correctly rounded
// values: every independent implementation that rounds the exact values gets
// the same bits, which the bit-reproducible LOR stencils and orderings rely on.
#include <cmath>
#include <vector>

#include "lor_internal.h"

namespace lor {

using f128 = __float128;

static void legendre(int p, f128 x, f128 &pm1, f128 &pp) {
  f128 a = 1, b = x;
  for (int k = 2; k <= p; ++k) {
    f128 c = ((2 * k - 1) * x * b - (k - 1) * a) / k;
    a = b;
    b = c;
  }
  pm1 = a;
  pp = b;
}

void gll_nodes_weights(int p, std::vector<double> &xo, std::vector<double> &wo) {
  std::vector<f128> xs(p + 1);
  xs[0] = -1;
  xs[p] = 1;
  for (int j = 1; j < p; ++j) {
    f128 x = -std::cos(M_PI * double(j) / double(p));
    for (int it = 0; it < 100; ++it) {
      f128 pm1, pp;
      legendre(p, x, pm1, pp);
      f128 om = 1 - x * x;
      f128 dp = p * (pm1 - x * pp) / om;                 // P_p'
      f128 d2p = (2 * x * dp - f128(p) * (p + 1) * pp) / om;  // P_p'' from the ODE
      f128 step = dp / d2p;
      x -= step;
      f128 as = step < 0 ? -step : step;
      if (as < f128(1e-33)) break;
    }
    xs[j] = x;
  }
  xo.resize(p + 1);
  wo.resize(p + 1);
  for (int j = 0; j <= p; ++j) {
    f128 pm1, pp;
    legendre(p, xs[j], pm1, pp);
    f128 w = f128(2) / (f128(p) * (p + 1) * pp * pp);
    xo[j] = double((xs[j] + 1) / 2);
    wo[j] = double(w / 2);
  }
}

// Barycentric form: D_ij = (c_j / c_i) / (x_i - x_j), D_ii = -sum_{j!=i} D_ij.
void lagrange_derivative(const std::vector<double> &x, std::vector<double> &D) {
  const int n = int(x.size());
  std::vector<double> c(n, 1.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k)
      if (k != i) c[i] *= (x[i] - x[k]);
  D.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    double s = 0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double v = (c[i] / c[j]) / (x[i] - x[j]);
      D[i * n + j] = v;
      s += v;
    }
    D[i * n + i] = -s;
  }
}

// Section 3.3: from the kept list [0, i1, ..., im, p] delete i1, i3, ... until
// only the two end points remain.
std::vector<std::vector<int>> kept_points(int p) {
  std::vector<std::vector<int>> lv;
  std::vector<int> cur;
  for (int i = 0; i <= p; ++i) cur.push_back(i);
  lv.push_back(cur);
  while (cur.size() > 2) {
    std::vector<int> nxt{0};
    for (size_t k = 1; k + 1 < cur.size(); ++k)
      if ((k - 1) % 2 == 1) nxt.push_back(cur[k]);
    nxt.push_back(p);
    cur = nxt;
    lv.push_back(cur);
  }
  return lv;
}

}  // namespace lor

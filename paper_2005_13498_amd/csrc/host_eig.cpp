#include "host_eig.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace hub {

void sym_eig(int n, std::vector<double> A, std::vector<double>& vals, std::vector<double>& vecs) {
  std::vector<double> V(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) V[static_cast<size_t>(i) * n + i] = 1.0;
  auto at = [&](int i, int j) -> double& { return A[static_cast<size_t>(i) * n + j]; };
  double total = 0.0;
  for (double x : A) total += x * x;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += 2.0 * at(i, j) * at(i, j);
    if (off <= 1e-30 * total || off == 0.0) break;
    for (int p = 0; p < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const double apq = at(p, q);
        if (apq == 0.0) continue;
        // rotation angle that annihilates A[p][q]
        const double theta = (at(q, q) - at(p, p)) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = at(k, p), akq = at(k, q);
          at(k, p) = c * akp - s * akq;
          at(k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = at(p, k), aqk = at(q, k);
          at(p, k) = c * apk - s * aqk;
          at(q, k) = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double& vkp = V[static_cast<size_t>(k) * n + p];
          double& vkq = V[static_cast<size_t>(k) * n + q];
          const double a = vkp, b = vkq;
          vkp = c * a - s * b;
          vkq = s * a + c * b;
        }
      }
    }
  }
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int a, int b) { return at(a, a) < at(b, b); });
  vals.resize(n);
  vecs.assign(static_cast<size_t>(n) * n, 0.0);
  for (int k = 0; k < n; ++k) {
    vals[k] = at(order[k], order[k]);
    for (int i = 0; i < n; ++i) vecs[static_cast<size_t>(i) * n + k] = V[static_cast<size_t>(i) * n + order[k]];
  }
}

}  // namespace hub

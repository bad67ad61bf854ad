// Host eigensolver of the small symmetric Rayleigh-Ritz matrix H (k <= 192): Householder
// reduction to tridiagonal form with accumulated reflections, then the implicit QL
// iteration with Wilkinson-type shifts (Bowdler, Martin, Reinsch and Wilkinson, Numer.
// Math. 11 (1968); Golub and Van Loan, Matrix Computations, Sections 8.3-8.4).
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "isira.h"

namespace {

// a: k-by-k symmetric, row-major, overwritten.  On return d = diagonal, e[i] couples
// i and i+1 (e[k-1] = 0), and q (row-major) holds the accumulated orthogonal factor
// with a = q T q^T.
void tridiagonalize(int k, std::vector<double>& a, std::vector<double>& q, std::vector<double>& d,
                    std::vector<double>& e) {
  q.assign((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i) q[(size_t)i * k + i] = 1.0;
  std::vector<double> v(k), p(k);
  for (int j = 0; j + 2 < k; ++j) {
    // reflect x = a[j+1:k, j] onto alpha e_1
    double tail2 = 0.0;
    for (int i = j + 2; i < k; ++i) tail2 += a[(size_t)i * k + j] * a[(size_t)i * k + j];
    if (tail2 == 0.0) continue;  // already tridiagonal in this column
    const double xnorm = std::sqrt(tail2 + a[(size_t)(j + 1) * k + j] * a[(size_t)(j + 1) * k + j]);
    const double x0 = a[(size_t)(j + 1) * k + j];
    const double alpha = (x0 > 0.0) ? -xnorm : xnorm;
    for (int i = j + 1; i < k; ++i) v[i] = a[(size_t)i * k + j];
    v[j + 1] -= alpha;
    double vn2 = 0.0;
    for (int i = j + 1; i < k; ++i) vn2 += v[i] * v[i];
    const double vn = std::sqrt(vn2);
    for (int i = j + 1; i < k; ++i) v[i] /= vn;
    // A22 <- H A22 H with H = I - 2 v v^T:  p = 2 A22 v, K = v^T p, w = p - K v,
    // A22 -= v w^T + w v^T
    for (int i = j + 1; i < k; ++i) {
      double s = 0.0;
      for (int t = j + 1; t < k; ++t) s += a[(size_t)i * k + t] * v[t];
      p[i] = 2.0 * s;
    }
    double K = 0.0;
    for (int i = j + 1; i < k; ++i) K += v[i] * p[i];
    for (int i = j + 1; i < k; ++i) p[i] -= K * v[i];
    for (int i = j + 1; i < k; ++i)
      for (int t = j + 1; t < k; ++t) a[(size_t)i * k + t] -= v[i] * p[t] + p[i] * v[t];
    a[(size_t)(j + 1) * k + j] = alpha;
    a[(size_t)j * k + j + 1] = alpha;
    for (int i = j + 2; i < k; ++i) {
      a[(size_t)i * k + j] = 0.0;
      a[(size_t)j * k + i] = 0.0;
    }
    // Q <- Q H
    for (int r = 0; r < k; ++r) {
      double s = 0.0;
      for (int t = j + 1; t < k; ++t) s += q[(size_t)r * k + t] * v[t];
      s *= 2.0;
      for (int t = j + 1; t < k; ++t) q[(size_t)r * k + t] -= s * v[t];
    }
  }
  d.resize(k);
  e.assign(k, 0.0);
  for (int i = 0; i < k; ++i) d[i] = a[(size_t)i * k + i];
  for (int i = 0; i + 1 < k; ++i) e[i] = a[(size_t)(i + 1) * k + i];
}

// Implicit QL on (d, e); plane rotations are applied to the rows of zt, where row i of zt
// (contiguous) is column i of the orthogonal factor.
bool tridiagonal_ql(int k, std::vector<double>& d, std::vector<double>& e,
                    std::vector<double>& zt) {
  const double eps = 2.220446049250313e-16;
  for (int l = 0; l < k; ++l) {
    int iter = 0;
    for (;;) {
      int m = l;
      for (; m < k - 1; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= eps * dd) break;
      }
      if (m == l) break;
      if (++iter > 60) return false;
      // shift from the leading 2x2 block at l
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::sqrt(g * g + 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
      double s = 1.0, c = 1.0, p = 0.0;
      int i = m - 1;
      bool deflated = false;
      for (; i >= l; --i) {
        double f = s * e[i];
        const double b = c * e[i];
        r = std::sqrt(f * f + g * g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= p;
          e[m] = 0.0;
          deflated = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        double* __restrict__ z0 = zt.data() + (size_t)i * k;
        double* __restrict__ z1 = z0 + k;
        for (int t = 0; t < k; ++t) {
          const double a0 = z0[t], a1 = z1[t];
          z1[t] = s * a0 + c * a1;
          z0[t] = c * a0 - s * a1;
        }
      }
      if (deflated) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  return true;
}

}  // namespace

extern "C" int isira_symeig(int32_t k, const double* H, double* theta, double* S) {
  if (k < 1 || !H || !theta || !S) return ISIRA_E_ARG;
  if (k == 1) {
    theta[0] = H[0];
    S[0] = 1.0;
    return ISIRA_OK;
  }
  std::vector<double> a((size_t)k * k), q, d, e;
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) a[(size_t)i * k + j] = 0.5 * (H[i + (size_t)j * k] + H[j + (size_t)i * k]);
  tridiagonalize(k, a, q, d, e);
  std::vector<double> qt((size_t)k * k);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) qt[(size_t)j * k + i] = q[(size_t)i * k + j];
  if (!tridiagonal_ql(k, d, e, qt)) return ISIRA_E_STATE;
  std::vector<int> order(k);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return d[x] < d[y]; });
  for (int j = 0; j < k; ++j) {
    const int src = order[j];
    theta[j] = d[src];
    for (int i = 0; i < k; ++i) S[i + (size_t)j * k] = qt[(size_t)src * k + i];
  }
  return ISIRA_OK;
}

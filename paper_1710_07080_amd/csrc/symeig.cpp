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

// a: k-by-k symmetric, row-major; its lower triangle is read and overwritten.  On return
// d = diagonal, e[i] couples
// i and i+1 (e[k-1] = 0).  With accumulate, q (row-major) holds the orthogonal factor with
// a = q T q^T; otherwise refl keeps the unit Householder vectors (row j: reflector j,
// entries j+1..k-1, or all zero when step j reflected nothing), q = H_0 H_1 ... H_{k-3}.
void tridiagonalize(int k, std::vector<double>& a, std::vector<double>& q, std::vector<double>& d,
                    std::vector<double>& e, bool accumulate, std::vector<double>* refl) {
  if (accumulate) {
    q.assign((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i) q[(size_t)i * k + i] = 1.0;
  }
  if (refl) refl->assign((size_t)k * k, 0.0);
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
    // A22 -= v w^T + w v^T.  Only the lower triangle of A22 is read and updated (it is
    // symmetric); the product with v takes each stored entry once for both of its places.
    for (int i = j + 1; i < k; ++i) p[i] = 0.0;
    for (int i = j + 1; i < k; ++i) {
      const double* __restrict__ ai = a.data() + (size_t)i * k;
      const double vi = v[i];
      double s = ai[i] * vi;
      for (int t = j + 1; t < i; ++t) {
        s += ai[t] * v[t];
        p[t] += ai[t] * vi;
      }
      p[i] += s;
    }
    for (int i = j + 1; i < k; ++i) p[i] *= 2.0;
    double K = 0.0;
    for (int i = j + 1; i < k; ++i) K += v[i] * p[i];
    for (int i = j + 1; i < k; ++i) p[i] -= K * v[i];
    for (int i = j + 1; i < k; ++i) {
      double* __restrict__ ai = a.data() + (size_t)i * k;
      const double vi = v[i], pi = p[i];
      for (int t = j + 1; t <= i; ++t) ai[t] -= vi * p[t] + pi * v[t];
    }
    a[(size_t)(j + 1) * k + j] = alpha;
    for (int i = j + 2; i < k; ++i) a[(size_t)i * k + j] = 0.0;
    if (refl)
      for (int t = j + 1; t < k; ++t) (*refl)[(size_t)j * k + t] = v[t];
    if (!accumulate) continue;
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
// (contiguous) is column i of the orthogonal factor (eigenvalues only when zt is empty).
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
        if (zt.empty()) continue;  // eigenvalues only
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
  tridiagonalize(k, a, q, d, e, true, nullptr);
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

extern "C" int isira_symeig_lowest(int32_t k, const double* H, double* theta, double* s1) {
  if (k < 1 || !H || !theta || !s1) return ISIRA_E_ARG;
  if (k == 1) {
    theta[0] = H[0];
    s1[0] = 1.0;
    return ISIRA_OK;
  }
  std::vector<double> a((size_t)k * k), q, d, e, refl;
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) a[(size_t)i * k + j] = 0.5 * (H[i + (size_t)j * k] + H[j + (size_t)i * k]);
  tridiagonalize(k, a, q, d, e, false, &refl);
  std::vector<double> dt = d, et = e, none;
  if (!tridiagonal_ql(k, dt, et, none)) return ISIRA_E_STATE;
  std::sort(dt.begin(), dt.end());
  for (int j = 0; j < k; ++j) theta[j] = dt[j];
  // inverse iteration with T - theta_0 I (Gaussian elimination on the tridiagonal matrix
  // with partial pivoting, as in LAPACK's dlagtf/dlagts; a zero pivot is replaced by a
  // tiny one) from a fixed start vector; three steps, each normalized
  double tnorm = 0.0;
  for (int i = 0; i < k; ++i)
    tnorm = std::max(tnorm, std::fabs(d[i]) + (i > 0 ? std::fabs(e[i - 1]) : 0.0) +
                                (i + 1 < k ? std::fabs(e[i]) : 0.0));
  const double tiny = (tnorm > 0.0 ? tnorm : 1.0) * 2.220446049250313e-16;
  const double lam = theta[0];
  // factor P (T - lam I) = L U: U has diagonal u0, superdiagonals u1, u2; L unit lower with
  // multipliers mult; piv[i] = 1 when rows i and i+1 were swapped
  std::vector<double> u0(k), u1(k, 0.0), u2(k, 0.0), mult(k, 0.0);
  std::vector<int> piv(k, 0);
  {
    double diag = d[0] - lam, sup = k > 1 ? e[0] : 0.0;
    for (int i = 0; i + 1 < k; ++i) {
      const double sub = e[i];
      const double nd = d[i + 1] - lam, nsup = (i + 2 < k) ? e[i + 1] : 0.0;
      if (std::fabs(diag) >= std::fabs(sub)) {
        const double m = (diag != 0.0) ? sub / diag : 0.0;
        mult[i] = m;
        u0[i] = diag;
        u1[i] = sup;
        u2[i] = 0.0;
        diag = nd - m * sup;
        sup = nsup;
      } else {
        const double m = diag / sub;
        piv[i] = 1;
        mult[i] = m;
        u0[i] = sub;
        u1[i] = nd;
        u2[i] = nsup;
        diag = sup - m * nd;
        sup = -m * nsup;
      }
    }
    u0[k - 1] = diag;
  }
  for (int i = 0; i < k; ++i)
    if (std::fabs(u0[i]) < tiny) u0[i] = (u0[i] < 0.0 ? -tiny : tiny);
  std::vector<double> y(k);
  for (int i = 0; i < k; ++i) y[i] = 1.0 + 0.25 * std::sin(1.0 + i);
  for (int step = 0; step < 3; ++step) {
    for (int i = 0; i + 1 < k; ++i) {  // forward: apply P and L^-1
      if (piv[i]) std::swap(y[i], y[i + 1]);
      y[i + 1] -= mult[i] * y[i];
    }
    for (int i = k - 1; i >= 0; --i) {  // back: U^-1
      double v = y[i];
      if (i + 1 < k) v -= u1[i] * y[i + 1];
      if (i + 2 < k) v -= u2[i] * y[i + 2];
      y[i] = v / u0[i];
    }
    double nrm = 0.0;
    for (int i = 0; i < k; ++i) nrm += y[i] * y[i];
    nrm = std::sqrt(nrm);
    for (int i = 0; i < k; ++i) y[i] /= nrm;
  }
  // back to the basis of H: s1 = H_0 H_1 ... H_{k-3} y (reflector k-3 applied first)
  for (int j = k - 3; j >= 0; --j) {
    const double* v = refl.data() + (size_t)j * k;
    double t = 0.0;
    for (int i = j + 1; i < k; ++i) t += v[i] * y[i];
    t *= 2.0;
    for (int i = j + 1; i < k; ++i) y[i] -= t * v[i];
  }
  for (int i = 0; i < k; ++i) s1[i] = y[i];
  return ISIRA_OK;
}

// Dense FP64 linear algebra for the host setup (see dense.hpp).
#include "dense.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace ldgmg {

namespace {

// Householder reflector for x (length len, contiguous): on return x[0] = beta,
// x[1:] = v[1:] (v[0] = 1 implied) and tau such that (I - tau v v^T) x = beta e1.
double make_reflector(int len, double* x) {
  if (len <= 1) return 0.0;
  double sigma = 0.0;
  for (int i = 1; i < len; ++i) sigma += x[i] * x[i];
  if (sigma == 0.0) return 0.0;
  const double alpha = x[0];
  const double norm = std::sqrt(alpha * alpha + sigma);
  const double beta = alpha >= 0.0 ? -norm : norm;
  const double tau = (beta - alpha) / beta;
  const double scal = 1.0 / (alpha - beta);
  for (int i = 1; i < len; ++i) x[i] *= scal;
  x[0] = beta;
  return tau;
}

// Y: panel of reflectors stored in C (column-major, ld), rows r0..m-1,
// columns j0..j0+nb-1, unit diagonal implied.  Applies (I - Y T Y^T)^T to the
// ncol columns of B (column-major, leading dim ldb) restricted to rows r0..m-1.
void apply_panel_t(int m, int r0, int nb, const double* C, int ld, int j0,
                   const double* T, double* B, int ldb, int ncol,
                   std::vector<double>& Wbuf) {
  const int mm = m - r0;
  if (mm <= 0 || ncol <= 0) return;
  Wbuf.assign(static_cast<size_t>(nb) * ncol, 0.0);
  double* W = Wbuf.data();          // nb x ncol, column-major
  // W = Y^T B, four columns of B at a time so each Y column is reused
  int c = 0;
  for (; c + 4 <= ncol; c += 4) {
    const double* b0 = B + static_cast<size_t>(c) * ldb + r0;
    const double* b1 = b0 + ldb;
    const double* b2 = b1 + ldb;
    const double* b3 = b2 + ldb;
    for (int i = 0; i < nb; ++i) {
      const double* y = C + static_cast<size_t>(j0 + i) * ld + r0;
      // y[t] for t < i is zero, y[i] = 1
      double s0 = b0[i], s1 = b1[i], s2 = b2[i], s3 = b3[i];
      for (int t = i + 1; t < mm; ++t) {
        const double yt = y[t];
        s0 += yt * b0[t];
        s1 += yt * b1[t];
        s2 += yt * b2[t];
        s3 += yt * b3[t];
      }
      W[i + (c + 0) * nb] = s0;
      W[i + (c + 1) * nb] = s1;
      W[i + (c + 2) * nb] = s2;
      W[i + (c + 3) * nb] = s3;
    }
  }
  for (; c < ncol; ++c) {
    const double* b0 = B + static_cast<size_t>(c) * ldb + r0;
    for (int i = 0; i < nb; ++i) {
      const double* y = C + static_cast<size_t>(j0 + i) * ld + r0;
      double s0 = b0[i];
      for (int t = i + 1; t < mm; ++t) s0 += y[t] * b0[t];
      W[i + c * nb] = s0;
    }
  }
  // W = T^T W  (T upper triangular nb x nb, column-major)
  std::vector<double> tmp(nb);
  for (int cc = 0; cc < ncol; ++cc) {
    double* w = W + static_cast<size_t>(cc) * nb;
    for (int i = 0; i < nb; ++i) {
      double s = 0.0;
      for (int t = 0; t <= i; ++t) s += T[t + i * nb] * w[t];
      tmp[i] = s;
    }
    std::memcpy(w, tmp.data(), sizeof(double) * nb);
  }
  // B -= Y W
  c = 0;
  for (; c + 4 <= ncol; c += 4) {
    double* b0 = B + static_cast<size_t>(c) * ldb + r0;
    double* b1 = b0 + ldb;
    double* b2 = b1 + ldb;
    double* b3 = b2 + ldb;
    for (int i = 0; i < nb; ++i) {
      const double* y = C + static_cast<size_t>(j0 + i) * ld + r0;
      const double w0 = W[i + (c + 0) * nb], w1 = W[i + (c + 1) * nb];
      const double w2 = W[i + (c + 2) * nb], w3 = W[i + (c + 3) * nb];
      b0[i] -= w0;
      b1[i] -= w1;
      b2[i] -= w2;
      b3[i] -= w3;
      for (int t = i + 1; t < mm; ++t) {
        const double yt = y[t];
        b0[t] -= yt * w0;
        b1[t] -= yt * w1;
        b2[t] -= yt * w2;
        b3[t] -= yt * w3;
      }
    }
  }
  for (; c < ncol; ++c) {
    double* b0 = B + static_cast<size_t>(c) * ldb + r0;
    for (int i = 0; i < nb; ++i) {
      const double* y = C + static_cast<size_t>(j0 + i) * ld + r0;
      const double w0 = W[i + c * nb];
      b0[i] -= w0;
      for (int t = i + 1; t < mm; ++t) b0[t] -= y[t] * w0;
    }
  }
}

}  // namespace

bool ls_householder(int m, int n, int k, double* C, double* R, double* X) {
  const int NB = 32;
  std::vector<double> tau(n, 0.0), T(NB * NB), Wbuf;
  for (int j0 = 0; j0 < n; j0 += NB) {
    const int nb = std::min(NB, n - j0);
    // unblocked factorisation of the panel
    for (int j = j0; j < j0 + nb; ++j) {
      double* col = C + static_cast<size_t>(j) * m;
      tau[j] = make_reflector(m - j, col + j);
      if (tau[j] == 0.0) continue;
      const double beta = col[j];
      col[j] = 1.0;
      for (int c = j + 1; c < j0 + nb; ++c) {
        double* cc = C + static_cast<size_t>(c) * m;
        double s = 0.0;
        for (int t = j; t < m; ++t) s += col[t] * cc[t];
        s *= tau[j];
        for (int t = j; t < m; ++t) cc[t] -= s * col[t];
      }
      col[j] = beta;
    }
    // T of the compact WY form: I - Y T Y^T = H_j0 ... H_{j0+nb-1}
    std::fill(T.begin(), T.end(), 0.0);
    for (int i = 0; i < nb; ++i) {
      const int ji = j0 + i;
      T[i + i * nb] = tau[ji];
      if (i == 0 || tau[ji] == 0.0) continue;
      const double* vi = C + static_cast<size_t>(ji) * m;   // rows ji.., v[ji] = 1
      std::vector<double> z(i, 0.0);
      for (int t = 0; t < i; ++t) {                          // z = Y(:,0:i)^T v_i
        const double* vt = C + static_cast<size_t>(j0 + t) * m;
        double s = vt[ji];                                   // v_i[ji] = 1
        for (int r = ji + 1; r < m; ++r) s += vt[r] * vi[r];
        z[t] = s;
      }
      for (int t = 0; t < i; ++t) {                          // T(0:i,i) = -tau T(0:i,0:i) z
        double s = 0.0;
        for (int u = t; u < i; ++u) s += T[t + u * nb] * z[u];
        T[t + i * nb] = -tau[ji] * s;
      }
    }
    // trailing columns and right-hand sides (apply_panel_t treats the entries
    // above each reflector's unit diagonal as zero, so R stays in place)
    apply_panel_t(m, j0, nb, C, m, j0, T.data(), C + static_cast<size_t>(j0 + nb) * m, m,
                  n - j0 - nb, Wbuf);
    apply_panel_t(m, j0, nb, C, m, j0, T.data(), R, m, k, Wbuf);
  }
  double dmax = 0.0, dmin = INFINITY;
  for (int j = 0; j < n; ++j) {
    const double d = std::fabs(C[static_cast<size_t>(j) * m + j]);
    dmax = std::max(dmax, d);
    dmin = std::min(dmin, d);
  }
  if (!(dmin > 1e-13 * dmax)) return false;
  // back substitution R X = (Q^T R)[0:n]
  for (int c = 0; c < k; ++c) {
    const double* rhs = R + static_cast<size_t>(c) * m;
    double* x = X + static_cast<size_t>(c) * n;
    for (int i = n - 1; i >= 0; --i) {
      double s = rhs[i];
      for (int t = i + 1; t < n; ++t) s -= C[static_cast<size_t>(t) * m + i] * x[t];
      x[i] = s / C[static_cast<size_t>(i) * m + i];
    }
  }
  return true;
}

void sym_eig(int n, const double* Ain, double* w, double* Vout) {
  // a: working copy (row-major, symmetric); q: accumulated transform, column-major
  std::vector<double> a(Ain, Ain + static_cast<size_t>(n) * n);
  std::vector<double> q(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) q[static_cast<size_t>(i) * n + i] = 1.0;
  std::vector<double> v(n), p(n), wv(n), d(n), e(n, 0.0);
  // Householder tridiagonalisation
  for (int k = 0; k + 2 < n; ++k) {
    const int len = n - k - 1;
    for (int i = 0; i < len; ++i) v[i] = a[static_cast<size_t>(k + 1 + i) * n + k];
    const double tau = make_reflector(len, v.data());
    if (tau == 0.0) continue;
    const double beta = v[0];
    v[0] = 1.0;
    // p = tau * A' v   (A' = a[k+1:, k+1:])
    for (int i = 0; i < len; ++i) {
      const double* row = &a[static_cast<size_t>(k + 1 + i) * n + k + 1];
      double s = 0.0;
      for (int j = 0; j < len; ++j) s += row[j] * v[j];
      p[i] = tau * s;
    }
    double pv = 0.0;
    for (int i = 0; i < len; ++i) pv += p[i] * v[i];
    const double K = 0.5 * tau * pv;
    for (int i = 0; i < len; ++i) wv[i] = p[i] - K * v[i];
    for (int i = 0; i < len; ++i) {
      double* row = &a[static_cast<size_t>(k + 1 + i) * n + k + 1];
      const double vi = v[i], wi = wv[i];
      for (int j = 0; j < len; ++j) row[j] -= vi * wv[j] + wi * v[j];
    }
    a[static_cast<size_t>(k + 1) * n + k] = beta;
    a[static_cast<size_t>(k) * n + k + 1] = beta;
    for (int i = 1; i < len; ++i) {
      a[static_cast<size_t>(k + 1 + i) * n + k] = 0.0;
      a[static_cast<size_t>(k) * n + k + 1 + i] = 0.0;
    }
    // Q <- Q H on columns k+1..n-1 (column-major q): Q' -= tau (Q' v) v^T
    for (int r = 0; r < n; ++r) {
      double s = 0.0;
      for (int j = 0; j < len; ++j) s += q[static_cast<size_t>(k + 1 + j) * n + r] * v[j];
      s *= tau;
      for (int j = 0; j < len; ++j) q[static_cast<size_t>(k + 1 + j) * n + r] -= s * v[j];
    }
  }
  for (int i = 0; i < n; ++i) d[i] = a[static_cast<size_t>(i) * n + i];
  for (int i = 0; i + 1 < n; ++i) e[i] = a[static_cast<size_t>(i + 1) * n + i];
  // implicit QL iterations with shifts on (d, e)
  for (int l = 0; l < n; ++l) {
    int iter = 0;
    for (;;) {
      int m = l;
      for (; m + 1 < n; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= 1e-16 * dd) break;
      }
      if (m == l) break;
      if (++iter > 60) break;
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? std::fabs(r) : -std::fabs(r)));
      double s = 1.0, c = 1.0, pp = 0.0;
      int i;
      bool early = false;
      for (i = m - 1; i >= l; --i) {
        double f = s * e[i];
        const double b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= pp;
          e[m] = 0.0;
          early = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - pp;
        r = (d[i] - g) * s + 2.0 * c * b;
        pp = s * r;
        d[i + 1] = g + pp;
        g = c * r - b;
        double* qi = &q[static_cast<size_t>(i) * n];
        double* qi1 = &q[static_cast<size_t>(i + 1) * n];
        for (int t = 0; t < n; ++t) {
          f = qi1[t];
          qi1[t] = s * qi[t] + c * f;
          qi[t] = c * qi[t] - s * f;
        }
      }
      if (early) continue;
      d[l] -= pp;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  // sort ascending, write eigenvectors as columns of row-major V
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return d[x] < d[y]; });
  for (int j = 0; j < n; ++j) {
    w[j] = d[idx[j]];
    const double* col = &q[static_cast<size_t>(idx[j]) * n];
    for (int r = 0; r < n; ++r) Vout[static_cast<size_t>(r) * n + j] = col[r];
  }
}

void sym_pinv(int n, const double* A, double* out, double rel_tol) {
  std::vector<double> w(n), V(static_cast<size_t>(n) * n);
  sym_eig(n, A, w.data(), V.data());
  double wmax = 0.0;
  for (int i = 0; i < n; ++i) wmax = std::max(wmax, std::fabs(w[i]));
  std::vector<double> inv(n);
  for (int i = 0; i < n; ++i) inv[i] = std::fabs(w[i]) > rel_tol * wmax ? 1.0 / w[i] : 0.0;
  // out = V diag(inv) V^T (V row-major, so rows r and c are contiguous)
  for (int r = 0; r < n; ++r) {
    const double* vr = &V[static_cast<size_t>(r) * n];
    for (int c = r; c < n; ++c) {
      const double* vc = &V[static_cast<size_t>(c) * n];
      double s = 0.0;
      for (int t = 0; t < n; ++t) s += vr[t] * inv[t] * vc[t];
      out[static_cast<size_t>(r) * n + c] = s;
      out[static_cast<size_t>(c) * n + r] = s;
    }
  }
}

}  // namespace ldgmg

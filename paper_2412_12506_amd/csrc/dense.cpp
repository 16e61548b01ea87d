// Dense FP64 linear algebra for the host setup (see dense.hpp).
#include "dense.hpp"

#include <algorithm>
#include <thread>
#include <functional>
#include <atomic>
#include <cmath>
#include <cstring>
#include <immintrin.h>
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

// ---- bs x bs tiles, row-major ----------------------------------------------

// C += s * A B  (all bs x bs row-major).  A 4 x 8 block of C is held in eight
// AVX2 registers while the k loop streams one row of B per step.
void tile_nn(int bs, const double* A, const double* B, double* C, double s) {
  const __m256d vs = _mm256_set1_pd(s);
  int i0 = 0;
  for (; i0 + 4 <= bs; i0 += 4) {
    const double* a0 = A + static_cast<size_t>(i0) * bs;
    const double* a1 = a0 + bs;
    const double* a2 = a1 + bs;
    const double* a3 = a2 + bs;
    int j0 = 0;
    for (; j0 + 8 <= bs; j0 += 8) {
      __m256d c00 = _mm256_setzero_pd(), c01 = _mm256_setzero_pd();
      __m256d c10 = _mm256_setzero_pd(), c11 = _mm256_setzero_pd();
      __m256d c20 = _mm256_setzero_pd(), c21 = _mm256_setzero_pd();
      __m256d c30 = _mm256_setzero_pd(), c31 = _mm256_setzero_pd();
      const double* b = B + j0;
      for (int k = 0; k < bs; ++k, b += bs) {
        const __m256d b0 = _mm256_loadu_pd(b), b1 = _mm256_loadu_pd(b + 4);
        __m256d x = _mm256_broadcast_sd(a0 + k);
        c00 = _mm256_fmadd_pd(x, b0, c00);
        c01 = _mm256_fmadd_pd(x, b1, c01);
        x = _mm256_broadcast_sd(a1 + k);
        c10 = _mm256_fmadd_pd(x, b0, c10);
        c11 = _mm256_fmadd_pd(x, b1, c11);
        x = _mm256_broadcast_sd(a2 + k);
        c20 = _mm256_fmadd_pd(x, b0, c20);
        c21 = _mm256_fmadd_pd(x, b1, c21);
        x = _mm256_broadcast_sd(a3 + k);
        c30 = _mm256_fmadd_pd(x, b0, c30);
        c31 = _mm256_fmadd_pd(x, b1, c31);
      }
      double* c = C + static_cast<size_t>(i0) * bs + j0;
      _mm256_storeu_pd(c, _mm256_fmadd_pd(vs, c00, _mm256_loadu_pd(c)));
      _mm256_storeu_pd(c + 4, _mm256_fmadd_pd(vs, c01, _mm256_loadu_pd(c + 4)));
      c += bs;
      _mm256_storeu_pd(c, _mm256_fmadd_pd(vs, c10, _mm256_loadu_pd(c)));
      _mm256_storeu_pd(c + 4, _mm256_fmadd_pd(vs, c11, _mm256_loadu_pd(c + 4)));
      c += bs;
      _mm256_storeu_pd(c, _mm256_fmadd_pd(vs, c20, _mm256_loadu_pd(c)));
      _mm256_storeu_pd(c + 4, _mm256_fmadd_pd(vs, c21, _mm256_loadu_pd(c + 4)));
      c += bs;
      _mm256_storeu_pd(c, _mm256_fmadd_pd(vs, c30, _mm256_loadu_pd(c)));
      _mm256_storeu_pd(c + 4, _mm256_fmadd_pd(vs, c31, _mm256_loadu_pd(c + 4)));
    }
    for (; j0 < bs; ++j0) {
      double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
      for (int k = 0; k < bs; ++k) {
        const double b = B[static_cast<size_t>(k) * bs + j0];
        acc0 += a0[k] * b;
        acc1 += a1[k] * b;
        acc2 += a2[k] * b;
        acc3 += a3[k] * b;
      }
      C[static_cast<size_t>(i0) * bs + j0] += s * acc0;
      C[static_cast<size_t>(i0 + 1) * bs + j0] += s * acc1;
      C[static_cast<size_t>(i0 + 2) * bs + j0] += s * acc2;
      C[static_cast<size_t>(i0 + 3) * bs + j0] += s * acc3;
    }
  }
  for (; i0 < bs; ++i0) {
    const double* a = A + static_cast<size_t>(i0) * bs;
    double* c = C + static_cast<size_t>(i0) * bs;
    for (int k = 0; k < bs; ++k) {
      const double x = s * a[k];
      const double* b = B + static_cast<size_t>(k) * bs;
      for (int j = 0; j < bs; ++j) c[j] += x * b[j];
    }
  }
}

void tile_transpose(int bs, const double* A, double* At) {
  for (int i = 0; i < bs; ++i)
    for (int j = 0; j < bs; ++j) At[static_cast<size_t>(j) * bs + i] = A[static_cast<size_t>(i) * bs + j];
}

// lower Cholesky factor of a bs x bs tile in place (upper part left as is);
// false when a pivot is <= floor
bool tile_potrf(int bs, double* A, double floor) {
  for (int j = 0; j < bs; ++j) {
    double* aj = A + static_cast<size_t>(j) * bs;
    double d = aj[j];
    for (int t = 0; t < j; ++t) d -= aj[t] * aj[t];
    if (!(d > floor)) return false;
    const double ljj = std::sqrt(d);
    aj[j] = ljj;
    const double inv = 1.0 / ljj;
    for (int i = j + 1; i < bs; ++i) {
      double* ai = A + static_cast<size_t>(i) * bs;
      double v = ai[j];
      for (int t = 0; t < j; ++t) v -= ai[t] * aj[t];
      ai[j] = v * inv;
    }
  }
  return true;
}

// X <- X L^-T for the lower factor L (row by row: x L^T = g)
void tile_trsm_right_lt(int bs, const double* L, double* X) {
  for (int r = 0; r < bs; ++r) {
    double* x = X + static_cast<size_t>(r) * bs;
    for (int j = 0; j < bs; ++j) {
      const double* lj = L + static_cast<size_t>(j) * bs;
      double v = x[j];
      for (int t = 0; t < j; ++t) v -= x[t] * lj[t];
      x[j] = v / lj[j];
    }
  }
}

// Y <- L^-1 Y (forward substitution over the rows of Y)
void tile_trsm_left_l(int bs, const double* L, double* Y) {
  for (int r = 0; r < bs; ++r) {
    const double* lr = L + static_cast<size_t>(r) * bs;
    double* y = Y + static_cast<size_t>(r) * bs;
    for (int t = 0; t < r; ++t) {
      const double l = lr[t];
      const double* yt = Y + static_cast<size_t>(t) * bs;
      for (int j = 0; j < bs; ++j) y[j] -= l * yt[j];
    }
    const double inv = 1.0 / lr[r];
    for (int j = 0; j < bs; ++j) y[j] *= inv;
  }
}

// Y <- L^-T Y (backward substitution over the rows of Y)
void tile_trsm_left_lt(int bs, const double* L, double* Y) {
  for (int r = bs - 1; r >= 0; --r) {
    double* y = Y + static_cast<size_t>(r) * bs;
    for (int t = r + 1; t < bs; ++t) {
      const double l = L[static_cast<size_t>(t) * bs + r];
      const double* yt = Y + static_cast<size_t>(t) * bs;
      for (int j = 0; j < bs; ++j) y[j] -= l * yt[j];
    }
    const double inv = 1.0 / L[static_cast<size_t>(r) * bs + r];
    for (int j = 0; j < bs; ++j) y[j] *= inv;
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

bool ls_block_normal(int bs, int mb, int nb,
                     const std::vector<std::vector<std::pair<int, const double*>>>& rows, int pos,
                     double* Xout) {
  const size_t T = static_cast<size_t>(bs) * bs;
  // tiles of G = C^T C: lower tiles (i >= j) hold G and then its Cholesky
  // factor; upper tiles (k < j) receive the transposed factor tiles
  std::vector<double> G(static_cast<size_t>(nb) * nb * T, 0.0);
  auto g = [&](int i, int j) { return G.data() + (static_cast<size_t>(i) * nb + j) * T; };
  // transposed copies of the nonzero blocks of C, in the order of rows[a]
  std::vector<size_t> first(mb + 1, 0);
  for (int a = 0; a < mb; ++a) first[a + 1] = first[a] + rows[a].size();
  std::vector<double> Ct(first[mb] * T);
  for (int a = 0; a < mb; ++a)
    for (size_t q = 0; q < rows[a].size(); ++q) tile_transpose(bs, rows[a][q].second, &Ct[(first[a] + q) * T]);
  // Gram tiles: G_{b1 b2} += C_{a b1}^T C_{a b2} for b1 >= b2
  for (int a = 0; a < mb; ++a)
    for (size_t q1 = 0; q1 < rows[a].size(); ++q1)
      for (size_t q2 = 0; q2 < rows[a].size(); ++q2) {
        const int b1 = rows[a][q1].first, b2 = rows[a][q2].first;
        if (b1 >= b2) tile_nn(bs, &Ct[(first[a] + q1) * T], rows[a][q2].second, g(b1, b2), 1.0);
      }
  double gmax = 0.0;
  for (int b = 0; b < nb; ++b)
    for (int r = 0; r < bs; ++r) gmax = std::max(gmax, g(b, b)[static_cast<size_t>(r) * bs + r]);
  const double floor = 1e-24 * gmax;
  // right-looking tiled Cholesky, G = L L^T
  std::vector<double> tmp(T);
  std::vector<double> colT(static_cast<size_t>(nb) * T);
  for (int k = 0; k < nb; ++k) {
    if (!tile_potrf(bs, g(k, k), floor)) return false;
    for (int r = 0; r < bs; ++r)      // clear the strictly upper part of the diagonal factor tile
      for (int c = r + 1; c < bs; ++c) g(k, k)[static_cast<size_t>(r) * bs + c] = 0.0;
    for (int i = k + 1; i < nb; ++i) {
      tile_trsm_right_lt(bs, g(k, k), g(i, k));
      tile_transpose(bs, g(i, k), &colT[static_cast<size_t>(i) * T]);
    }
    for (int i = k + 1; i < nb; ++i)
      for (int j = k + 1; j <= i; ++j) tile_nn(bs, g(i, k), &colT[static_cast<size_t>(j) * T], g(i, j), -1.0);
    for (int j = k + 1; j < nb; ++j)
      std::memcpy(g(k, j), &colT[static_cast<size_t>(j) * T], T * sizeof(double));
  }
  // Y <- (L L^T)^-1 Y, tile rows of Y indexed by block column
  auto solve = [&](std::vector<double>& Y) {
    for (int k = 0; k < nb; ++k) {
      double* yk = &Y[static_cast<size_t>(k) * T];
      for (int j = 0; j < k; ++j) tile_nn(bs, g(k, j), &Y[static_cast<size_t>(j) * T], yk, -1.0);
      tile_trsm_left_l(bs, g(k, k), yk);
    }
    for (int k = nb - 1; k >= 0; --k) {
      double* yk = &Y[static_cast<size_t>(k) * T];
      for (int j = k + 1; j < nb; ++j) tile_nn(bs, g(k, j), &Y[static_cast<size_t>(j) * T], yk, -1.0);
      tile_trsm_left_lt(bs, g(k, k), yk);
    }
  };
  // X0 from C^T E: the transposed blocks of block row pos
  std::vector<double> X(static_cast<size_t>(nb) * T, 0.0);
  for (size_t q = 0; q < rows[pos].size(); ++q)
    std::memcpy(&X[static_cast<size_t>(rows[pos][q].first) * T], &Ct[(first[pos] + q) * T], T * sizeof(double));
  solve(X);
  // one refinement step: D = (C^T C)^-1 C^T (E - C X0)
  std::vector<double> R(static_cast<size_t>(mb) * T, 0.0), D(static_cast<size_t>(nb) * T, 0.0);
  for (int r = 0; r < bs; ++r) R[(static_cast<size_t>(pos) * bs + r) * bs + r] = 1.0;
  for (int a = 0; a < mb; ++a)
    for (const auto& bp : rows[a])
      tile_nn(bs, bp.second, &X[static_cast<size_t>(bp.first) * T], &R[static_cast<size_t>(a) * T], -1.0);
  for (int a = 0; a < mb; ++a)
    for (size_t q = 0; q < rows[a].size(); ++q)
      tile_nn(bs, &Ct[(first[a] + q) * T], &R[static_cast<size_t>(a) * T],
              &D[static_cast<size_t>(rows[a][q].first) * T], 1.0);
  solve(D);
  double xmax = 0.0, dmax = 0.0;
  for (size_t t = 0; t < X.size(); ++t) {
    X[t] += D[t];
    xmax = std::max(xmax, std::fabs(X[t]));
    dmax = std::max(dmax, std::fabs(D[t]));
  }
  if (!(dmax <= 1e-8 * xmax)) return false;
  const size_t n = static_cast<size_t>(nb) * bs;
  for (int b = 0; b < nb; ++b)
    for (int r = 0; r < bs; ++r)
      for (int c = 0; c < bs; ++c)
        Xout[static_cast<size_t>(c) * n + static_cast<size_t>(b) * bs + r] = X[static_cast<size_t>(b) * T + static_cast<size_t>(r) * bs + c];
  return true;
}

namespace {

// Sense-counting barrier for a fixed team of threads (spins, then yields).
class SpinBarrier {
 public:
  explicit SpinBarrier(int n) : n_(n) {}
  void wait() {
    if (n_ == 1) return;
    const int gen = gen_.load(std::memory_order_acquire);
    if (count_.fetch_add(1, std::memory_order_acq_rel) + 1 == n_) {
      count_.store(0, std::memory_order_relaxed);
      gen_.fetch_add(1, std::memory_order_release);
      return;
    }
    for (int spins = 0; gen_.load(std::memory_order_acquire) == gen; ++spins)
      if (spins > 2000) std::this_thread::yield();
  }

 private:
  const int n_;
  std::atomic<int> count_{0}, gen_{0};
};

// fn(tid) on nt threads, the caller being thread 0; fn must not throw.
void run_team(int nt, const std::function<void(int)>& fn) {
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) th.emplace_back(fn, t);
  fn(0);
  for (auto& t : th) t.join();
}

struct Rotation {
  int i;
  double c, s;
};

}  // namespace

void sym_eig(int n, const double* Ain, double* w, double* Vout, int nthreads) {
  const int nt = n >= 256 ? std::max(1, std::min(nthreads, n / 64)) : 1;
  // a: working copy, row-major and symmetric; after the reduction its
  // diagonal and subdiagonal hold the tridiagonal matrix and column k below
  // the subdiagonal holds the tail of reflector k (unit first entry implied)
  std::vector<double> a(Ain, Ain + static_cast<size_t>(n) * n);
  std::vector<double> tau(n, 0.0), v(n), p(n), wv(n);
  double tau_k = 0.0;
  SpinBarrier bar(nt);
  // 1. Householder tridiagonalisation A = Q T Q^T, trailing rows split over the team
  run_team(nt, [&](int tid) {
    for (int k = 0; k + 2 < n; ++k) {
      const int len = n - k - 1;
      if (tid == 0) {
        for (int i = 0; i < len; ++i) v[i] = a[static_cast<size_t>(k + 1 + i) * n + k];
        tau_k = make_reflector(len, v.data());
        tau[k] = tau_k;
        if (tau_k != 0.0) {
          for (int i = 0; i < len; ++i) a[static_cast<size_t>(k + 1 + i) * n + k] = v[i];  // beta, tail
          v[0] = 1.0;
        }
      }
      bar.wait();
      const double tk = tau_k;
      const int lo = static_cast<int>(static_cast<long long>(len) * tid / nt);
      const int hi = static_cast<int>(static_cast<long long>(len) * (tid + 1) / nt);
      if (tk != 0.0)
        for (int i = lo; i < hi; ++i) {        // p = tau A' v
          const double* row = &a[static_cast<size_t>(k + 1 + i) * n + k + 1];
          double s = 0.0;
          for (int j = 0; j < len; ++j) s += row[j] * v[j];
          p[i] = tk * s;
        }
      bar.wait();
      if (tid == 0 && tk != 0.0) {             // w = p - (tau p.v / 2) v
        double pv = 0.0;
        for (int i = 0; i < len; ++i) pv += p[i] * v[i];
        const double K = 0.5 * tk * pv;
        for (int i = 0; i < len; ++i) wv[i] = p[i] - K * v[i];
      }
      bar.wait();
      if (tk != 0.0)
        for (int i = lo; i < hi; ++i) {        // A' -= v w^T + w v^T
          double* row = &a[static_cast<size_t>(k + 1 + i) * n + k + 1];
          const double vi = v[i], wi = wv[i];
          for (int j = 0; j < len; ++j) row[j] -= vi * wv[j] + wi * v[j];
        }
      bar.wait();
    }
  });
  std::vector<double> d(n), e(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = a[static_cast<size_t>(i) * n + i];
  for (int i = 0; i + 1 < n; ++i) e[i] = a[static_cast<size_t>(i + 1) * n + i];
  // 2. Q (column-major): column j is H_0 ... H_{j-1} e_j; blocks of 16 columns
  // share each reflector load and are dealt to the team round robin
  // reflector k, contiguous: refl[k * n + i] = v_i (i < n - k - 1, v_0 = 1)
  for (int k = 0; k + 2 < n; ++k) {
    double* r = &a[static_cast<size_t>(k) * n];     // row k is no longer needed
    r[0] = 1.0;
    for (int i = 1; i < n - k - 1; ++i) r[i] = a[static_cast<size_t>(k + 1 + i) * n + k];
  }
  std::vector<double> q(static_cast<size_t>(n) * n, 0.0);
  const int CB = 16, nblk = (n + CB - 1) / CB;
  run_team(nt, [&](int tid) {
    for (int b = tid; b < nblk; b += nt) {
      const int j0 = b * CB, j1 = std::min(n, j0 + CB);
      for (int j = j0; j < j1; ++j) q[static_cast<size_t>(j) * n + j] = 1.0;
      for (int k = std::min(j1 - 1, n - 2) - 1; k >= 0; --k) {
        if (tau[k] == 0.0) continue;
        const double* vt = &a[static_cast<size_t>(k) * n];
        const int len = n - k - 1;
        for (int j = std::max(j0, k + 1); j < j1; ++j) {
          double* x = &q[static_cast<size_t>(j) * n + k + 1];
          double s = 0.0;
          for (int i = 0; i < len; ++i) s += vt[i] * x[i];
          s *= tau[k];
          for (int i = 0; i < len; ++i) x[i] -= s * vt[i];
        }
      }
    }
  });
  // 3. implicit QL iterations with Wilkinson-type shifts on (d, e), recording
  //    the rotations: the published tql2 procedure of Bowdler, Martin, Reinsch
  //    and Wilkinson (Handbook for Automatic Computation II, 1971) in its
  //    textbook form
  std::vector<Rotation> rot;
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
      bool early = false;
      for (int i = m - 1; i >= l; --i) {
        const double f = s * e[i];
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
        rot.push_back({i, c, s});
      }
      if (early) continue;
      d[l] -= pp;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  // 4. apply the rotations in order to the columns of Q, rows split over the team
  run_team(nt, [&](int tid) {
    const int lo = static_cast<int>(static_cast<long long>(n) * tid / nt);
    const int hi = static_cast<int>(static_cast<long long>(n) * (tid + 1) / nt);
    for (const Rotation& R : rot) {
      double* qi = &q[static_cast<size_t>(R.i) * n];
      double* qi1 = qi + n;
      for (int t = lo; t < hi; ++t) {
        const double f = qi1[t];
        qi1[t] = R.s * qi[t] + R.c * f;
        qi[t] = R.c * qi[t] - R.s * f;
      }
    }
  });
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

void sym_pinv(int n, const double* A, double* out, double rel_tol, int nthreads) {
  std::vector<double> w(n), V(static_cast<size_t>(n) * n);
  sym_eig(n, A, w.data(), V.data(), nthreads);
  double wmax = 0.0;
  for (int i = 0; i < n; ++i) wmax = std::max(wmax, std::fabs(w[i]));
  std::vector<double> inv(n);
  for (int i = 0; i < n; ++i) inv[i] = std::fabs(w[i]) > rel_tol * wmax ? 1.0 / w[i] : 0.0;
  // out = V diag(inv) V^T (V row-major, so rows r and c are contiguous); row r
  // owns the entries (r, c >= r) and their mirror images
  const int nt = n >= 256 ? std::max(1, std::min(nthreads, n / 64)) : 1;
  run_team(nt, [&](int tid) {
    std::vector<double> u(n);
    for (int r = tid; r < n; r += nt) {
      const double* vr = &V[static_cast<size_t>(r) * n];
      for (int t = 0; t < n; ++t) u[t] = vr[t] * inv[t];
      for (int c = r; c < n; ++c) {
        const double* vc = &V[static_cast<size_t>(c) * n];
        double s = 0.0;
        for (int t = 0; t < n; ++t) s += u[t] * vc[t];
        out[static_cast<size_t>(r) * n + c] = s;
        out[static_cast<size_t>(c) * n + r] = s;
      }
    }
  });
}

}  // namespace ldgmg

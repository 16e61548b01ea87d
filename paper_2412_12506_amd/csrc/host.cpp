// Host-side (FP64) setup of the LDG multigrid hierarchy.  See host.hpp.
//
// Discretisation (Section 2.1 / 3.1 of the paper), per uniform grid:
//   M (G_k u)_K = int_K d_k u w + sum_{faces of K normal to e_k} int_F (u^ - u_K) w n_k,
//   u^ from the more viscous side (ties: lower-coordinate side), u^ = 0 for the
//   operator part on Dirichlet faces and u^ = u_K on Neumann faces;
//   E = sum_F tau_F int_F [u][v], tau_F = tau0 min(mu_L, mu_R)/h (interior),
//   tau0 mu_K / h (Dirichlet);  E_p = sum_{interior F} cp h / max(mu_L, mu_R) int_F [p][q];
//   scalar:  A = sum_k G_k^T M_mu G_k + E;
//   Stokes:  eq:components with A_ij = delta_ij (sum_k G_k^T M_mu G_k + E) + gamma G_j^T M_mu G_i.
// Coarse levels (Section 2.2, operator coarsening), factor by factor:
//   G^{2h} = (M^{2h})^-1 I^T M^h G^h I,  M_mu^{2h} = I^T M_mu^h I,
//   E^{2h} = 1/2 I^T E^h I,  E_p^{2h} = 2 I^T E_p^h I,  then A^{2h} as on the fine grid.
#include "host.hpp"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <stdexcept>
#include <thread>

#include "dense.hpp"

namespace ldgmg {

namespace {

using Vec = std::vector<double>;

// Per calling thread, so that setups of different problems can run concurrently.
thread_local int g_threads = 1;

void parallel_for(int n, const std::function<void(int)>& fn) {
  const int nt = std::max(1, std::min(g_threads, n));
  if (nt == 1) {
    for (int i = 0; i < n; ++i) fn(i);
    return;
  }
  std::atomic<int> next{0};
  std::vector<std::thread> th;
  std::exception_ptr err = nullptr;
  std::atomic<bool> failed{false};
  for (int t = 0; t < nt; ++t) {
    th.emplace_back([&] {
      try {
        for (;;) {
          const int i = next.fetch_add(1);
          if (i >= n || failed.load()) break;
          fn(i);
        }
      } catch (...) {
        if (!failed.exchange(true)) err = std::current_exception();
      }
    });
  }
  for (auto& t : th) t.join();
  if (err) std::rethrow_exception(err);
}

// row-major dense helpers
void matmul(int r, int k, int c, const double* A, const double* B, double* C, bool acc = false) {
  if (!acc) std::fill(C, C + static_cast<size_t>(r) * c, 0.0);
  for (int i = 0; i < r; ++i)
    for (int t = 0; t < k; ++t) {
      const double a = A[static_cast<size_t>(i) * k + t];
      if (a == 0.0) continue;
      const double* b = B + static_cast<size_t>(t) * c;
      double* cc = C + static_cast<size_t>(i) * c;
      for (int j = 0; j < c; ++j) cc[j] += a * b[j];
    }
}
// C (+)= A^T B, A: k x r
void matmul_tn(int r, int k, int c, const double* A, const double* B, double* C, bool acc = false) {
  if (!acc) std::fill(C, C + static_cast<size_t>(r) * c, 0.0);
  for (int t = 0; t < k; ++t) {
    const double* b = B + static_cast<size_t>(t) * c;
    for (int i = 0; i < r; ++i) {
      const double a = A[static_cast<size_t>(t) * r + i];
      if (a == 0.0) continue;
      double* cc = C + static_cast<size_t>(i) * c;
      for (int j = 0; j < c; ++j) cc[j] += a * b[j];
    }
  }
}

// kron over dimensions with dimension 0 fastest: out[a][b] = prod_k mats[k][a_k][b_k]
Vec kron_dims(int dim, int q, const std::vector<const double*>& mats) {
  int bss = 1;
  for (int k = 0; k < dim; ++k) bss *= q;
  Vec out(static_cast<size_t>(bss) * bss);
  for (int a = 0; a < bss; ++a)
    for (int b = 0; b < bss; ++b) {
      double v = 1.0;
      int aa = a, bb = b;
      for (int k = 0; k < dim; ++k) {
        v *= mats[k][(aa % q) * q + (bb % q)];
        aa /= q;
        bb /= q;
      }
      out[static_cast<size_t>(a) * bss + b] = v;
    }
  return out;
}

// ---------------------------------------------------------------------------
// 1-D bases and Gauss-Legendre quadrature
// ---------------------------------------------------------------------------
// Legendre P_0..P_p and derivatives at t (three-term recurrence)
void legendre_all(int p, double t, double* P, double* dP) {
  P[0] = 1.0;
  dP[0] = 0.0;
  if (p >= 1) {
    P[1] = t;
    dP[1] = 1.0;
  }
  for (int k = 1; k < p; ++k) {
    P[k + 1] = ((2 * k + 1) * t * P[k] - k * P[k - 1]) / (k + 1);
    dP[k + 1] = dP[k - 1] + (2 * k + 1) * P[k];
  }
}

}  // namespace

void gauss_legendre(int q, Vec& x, Vec& w) {
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  std::vector<double> P(q + 1), dP(q + 1);
  for (int i = 0; i < q; ++i) {
    double t = std::cos(M_PI * (i + 0.75) / (q + 0.5));
    for (int it = 0; it < 100; ++it) {
      legendre_all(q, t, P.data(), dP.data());
      const double dt = P[q] / dP[q];
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    legendre_all(q, t, P.data(), dP.data());
    x[q - 1 - i] = t;
    w[q - 1 - i] = 2.0 / ((1.0 - t * t) * dP[q] * dP[q]);
  }
}

namespace {

struct Basis1D {
  int p, kind;
  Vec nodes;
  Basis1D(int p_, int kind_) : p(p_), kind(kind_) {
    if (kind == LDGMG_BASIS_GL_NODAL) {
      Vec w;
      gauss_legendre(p + 1, nodes, w);
    }
  }
  // values and derivatives of psi_0..psi_p at t
  void eval(double t, double* v, double* dv) const {
    if (kind == LDGMG_BASIS_LEGENDRE) {
      std::vector<double> P(p + 2), dP(p + 2);
      legendre_all(p, t, P.data(), dP.data());
      for (int i = 0; i <= p; ++i) {
        const double s = std::sqrt((2.0 * i + 1.0) / 2.0);
        v[i] = s * P[i];
        dv[i] = s * dP[i];
      }
      return;
    }
    for (int i = 0; i <= p; ++i) {
      double val = 1.0, der = 0.0;
      for (int j = 0; j <= p; ++j) {
        if (j == i) continue;
        const double f = 1.0 / (nodes[i] - nodes[j]);
        der = der * (t - nodes[j]) * f + val * f;
        val *= (t - nodes[j]) * f;
      }
      v[i] = val;
      dv[i] = der;
    }
  }
};

// invert a small dense matrix (Gauss-Jordan with partial pivoting)
Vec invert(int n, const Vec& A) {
  Vec a(A), inv(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) inv[static_cast<size_t>(i) * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[static_cast<size_t>(r) * n + c]) > std::fabs(a[static_cast<size_t>(piv) * n + c])) piv = r;
    if (piv != c)
      for (int j = 0; j < n; ++j) {
        std::swap(a[static_cast<size_t>(c) * n + j], a[static_cast<size_t>(piv) * n + j]);
        std::swap(inv[static_cast<size_t>(c) * n + j], inv[static_cast<size_t>(piv) * n + j]);
      }
    const double d = 1.0 / a[static_cast<size_t>(c) * n + c];
    for (int j = 0; j < n; ++j) {
      a[static_cast<size_t>(c) * n + j] *= d;
      inv[static_cast<size_t>(c) * n + j] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = a[static_cast<size_t>(r) * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        a[static_cast<size_t>(r) * n + j] -= f * a[static_cast<size_t>(c) * n + j];
        inv[static_cast<size_t>(r) * n + j] -= f * inv[static_cast<size_t>(c) * n + j];
      }
    }
  }
  return inv;
}

}  // namespace

void basis_eval(int p, int basis, double t, double* v, double* dv) {
  Basis1D b(p, basis);
  b.eval(t, v, dv);
}

void ElemOps::init(int dim_, int p_, double h_, int basis) {
  dim = dim_;
  p = p_;
  h = h_;
  q1 = p + 1;
  bss = 1;
  for (int k = 0; k < dim; ++k) bss *= q1;
  Basis1D b(p, basis);
  Vec xq, wq;
  gauss_legendre(p + 2, xq, wq);
  const int nq = p + 2;
  std::vector<double> V(static_cast<size_t>(q1) * nq), DV(static_cast<size_t>(q1) * nq), v(q1), dv(q1);
  for (int t = 0; t < nq; ++t) {
    b.eval(xq[t], v.data(), dv.data());
    for (int i = 0; i < q1; ++i) {
      V[static_cast<size_t>(i) * nq + t] = v[i];
      DV[static_cast<size_t>(i) * nq + t] = dv[i];
    }
  }
  m.assign(static_cast<size_t>(q1) * q1, 0.0);
  adv.assign(static_cast<size_t>(q1) * q1, 0.0);
  for (int i = 0; i < q1; ++i)
    for (int j = 0; j < q1; ++j) {
      double sm = 0, sa = 0;
      for (int t = 0; t < nq; ++t) {
        sm += wq[t] * V[static_cast<size_t>(i) * nq + t] * V[static_cast<size_t>(j) * nq + t];
        sa += wq[t] * V[static_cast<size_t>(i) * nq + t] * DV[static_cast<size_t>(j) * nq + t];
      }
      m[static_cast<size_t>(i) * q1 + j] = sm;
      adv[static_cast<size_t>(i) * q1 + j] = sa;
    }
  tm.assign(q1, 0.0);
  tp.assign(q1, 0.0);
  b.eval(-1.0, tm.data(), dv.data());
  b.eval(1.0, tp.data(), dv.data());
  const Vec minv = invert(q1, m);
  for (int c = 0; c < 2; ++c) {
    // P_c = m^-1 * int psi_i(t) psi_j(phi_c(t)) dt,  phi_c(t) = (t + 2c - 1)/2
    Vec mom(static_cast<size_t>(q1) * q1, 0.0);
    for (int t = 0; t < nq; ++t) {
      b.eval(0.5 * (xq[t] + (2 * c - 1)), v.data(), dv.data());
      for (int i = 0; i < q1; ++i)
        for (int j = 0; j < q1; ++j)
          mom[static_cast<size_t>(i) * q1 + j] += wq[t] * V[static_cast<size_t>(i) * nq + t] * v[j];
    }
    P[c].assign(static_cast<size_t>(q1) * q1, 0.0);
    matmul(q1, q1, q1, minv.data(), mom.data(), P[c].data());
  }
  const double jac = h / 2.0;
  const double jd = std::pow(jac, dim), jf = std::pow(jac, dim - 1);
  std::vector<const double*> mats(dim, m.data());
  M = kron_dims(dim, q1, mats);
  for (double& x : M) x *= jd;
  Minv = invert(bss, M);
  for (int k = 0; k < dim; ++k) {
    std::vector<const double*> mk(dim, m.data());
    mk[k] = adv.data();
    D[k] = kron_dims(dim, q1, mk);
    for (double& x : D[k]) x *= jf;
    for (int s1 = 0; s1 < 2; ++s1)
      for (int s2 = 0; s2 < 2; ++s2) {
        const Vec& a = s1 ? tp : tm;
        const Vec& bb = s2 ? tp : tm;
        Vec outer(static_cast<size_t>(q1) * q1);
        for (int i = 0; i < q1; ++i)
          for (int j = 0; j < q1; ++j) outer[static_cast<size_t>(i) * q1 + j] = a[i] * bb[j];
        std::vector<const double*> mt(dim, m.data());
        mt[k] = outer.data();
        T[k][s1][s2] = kron_dims(dim, q1, mt);
        for (double& x : T[k][s1][s2]) x *= jf;
      }
  }
  for (int c = 0; c < (1 << dim); ++c) {
    std::vector<const double*> mp(dim);
    for (int k = 0; k < dim; ++k) mp[k] = P[(c >> k) & 1].data();
    Ic[c] = kron_dims(dim, q1, mp);
  }
}

int PMat::slot(int i, int j) const {
  const int* b = ci.data() + rp[i];
  const int* e = ci.data() + rp[i + 1];
  const int* it = std::lower_bound(b, e, j);
  if (it != e && *it == j) return static_cast<int>(it - ci.data());
  return -1;
}

std::vector<int> level_sizes(int n) {
  std::vector<int> s{n};
  while (s.back() % 2 == 0 && s.back() > 2) s.push_back(s.back() / 2);
  return s;
}

void validate_problem(const ldgmg_problem& p) {
  if (p.dim != 2 && p.dim != 3) throw std::invalid_argument("dim must be 2 or 3");
  if (p.n < 2 || p.n > 4096) throw std::invalid_argument("n out of range");
  if (p.p < 1 || p.p > 5) throw std::invalid_argument("p must be in 1..5");
  if (p.basis != LDGMG_BASIS_LEGENDRE && p.basis != LDGMG_BASIS_GL_NODAL)
    throw std::invalid_argument("unknown basis");
  if (p.system != LDGMG_POISSON && p.system != LDGMG_STOKES) throw std::invalid_argument("unknown system");
  if (p.smoother < 0 || p.smoother > 2) throw std::invalid_argument("unknown smoother");
  if (p.sai_level < 0 || p.sai_level > 2) throw std::invalid_argument("sai_level must be 0..2");
  if (p.order < 0 || p.order > 3) throw std::invalid_argument("unknown order");
  if (p.nu1 < 0 || p.nu2 < 0 || p.nu1 > 16 || p.nu2 > 16) throw std::invalid_argument("nu out of range");
  if (p.precision != LDGMG_FP64 && p.precision != LDGMG_FP32 && p.precision != LDGMG_BF16S)
    throw std::invalid_argument("unknown precision");
  if (p.storage < LDGMG_STORE_AUTO || p.storage > LDGMG_STORE_TILED) throw std::invalid_argument("unknown storage");
  if (p.precision == LDGMG_BF16S && p.smoother != LDGMG_SMOOTH_SAI)
    throw std::invalid_argument("BF16 smoother storage is for the SAI smoothers only");
  if (!(p.tau0 > 0) || !(p.cp >= 0)) throw std::invalid_argument("penalty constants must be positive");
  if ((p.dev_alloc == nullptr) != (p.dev_free == nullptr))
    throw std::invalid_argument("dev_alloc and dev_free must be given together");
  if (!(p.delta >= 0) || !std::isfinite(p.delta)) throw std::invalid_argument("delta must be finite and >= 0");
  if (p.setup_device != 0 && p.setup_device != 1) throw std::invalid_argument("setup_device must be 0 or 1");
  if (p.delta > 0 && p.system != LDGMG_STOKES) throw std::invalid_argument("the density term is for Stokes");
  for (int k = 0; k < p.dim; ++k) {
    const int a = p.bc[2 * k], b = p.bc[2 * k + 1];
    if (a < 0 || a > 2 || b < 0 || b > 2) throw std::invalid_argument("unknown bc");
    if ((a == LDGMG_BC_PERIODIC) != (b == LDGMG_BC_PERIODIC))
      throw std::invalid_argument("periodic must be set on both faces of a dimension");
  }
  long long ne = 1;
  for (int k = 0; k < p.dim; ++k) ne *= p.n;
  if (p.mu)
    for (long long e = 0; e < ne; ++e)
      if (!(p.mu[e] > 0) || !std::isfinite(p.mu[e])) throw std::invalid_argument("viscosity must be finite and > 0");
  if (p.rho && p.delta > 0)
    for (long long e = 0; e < ne; ++e)
      if (!(p.rho[e] > 0) || !std::isfinite(p.rho[e])) throw std::invalid_argument("density must be finite and > 0");
}

namespace {

// ---------------------------------------------------------------------------
// grid helpers
// ---------------------------------------------------------------------------
struct GridInfo {
  int dim, n, ne;
  int bc[6];
  void idx(int e, int* out) const {
    for (int k = 0; k < dim; ++k) {
      out[k] = e % n;
      e /= n;
    }
  }
  int elem(const int* ix) const {
    int e = 0;
    for (int k = dim - 1; k >= 0; --k) e = e * n + ix[k];
    return e;
  }
  // neighbour across face (k, side in {-1,+1}); -1 on a non-periodic boundary
  int nbr(int e, int k, int side) const {
    int ix[3];
    idx(e, ix);
    int j = ix[k] + side;
    if (j < 0 || j >= n) {
      if (bc[2 * k] != LDGMG_BC_PERIODIC) return -1;
      j = (j + n) % n;
    }
    ix[k] = j;
    return elem(ix);
  }
  int btype(int k, int side) const { return bc[2 * k + (side < 0 ? 0 : 1)]; }
};

// build rows of a pooled matrix: rowfn(i, std::map<int, Key>&) fills the keys of
// row i, valfn(key bytes, out) evaluates a block.  Serial (pool interning).
template <class RowFn, class ValFn>
void build_pmat(PMat& P, int nbr, int nbc, int br, int bc_, RowFn&& rowfn, ValFn&& valfn) {
  P.nbr = nbr;
  P.nbc = nbc;
  P.pool.r = br;
  P.pool.c = bc_;
  P.rp.assign(nbr + 1, 0);
  P.ci.clear();
  P.id.clear();
  std::map<int, Key> row;
  for (int i = 0; i < nbr; ++i) {
    row.clear();
    rowfn(i, row);
    for (auto& kv : row) {
      P.ci.push_back(kv.first);
      P.id.push_back(P.pool.intern(kv.second.s, [&](double* out) { valfn(kv.second.s, out); }));
    }
    P.rp[i + 1] = static_cast<int>(P.ci.size());
  }
}

template <class T>
T read_at(const std::string& s, size_t& off) {
  T v;
  std::memcpy(&v, s.data() + off, sizeof(T));
  off += sizeof(T);
  return v;
}

// ---------------------------------------------------------------------------
// fine-level scalar factors
// ---------------------------------------------------------------------------
// u^ source for the lower / upper face of e in dimension k.
// returns 0: neighbour, 1: self, 2: Dirichlet, 3: Neumann
int src_lower(const GridInfo& g, const double* mu, int e, int k, int* L) {
  *L = g.nbr(e, k, -1);
  if (*L < 0) return g.btype(k, -1) == LDGMG_BC_DIRICHLET ? 2 : 3;
  return mu[*L] >= mu[e] ? 0 : 1;
}
int src_upper(const GridInfo& g, const double* mu, int e, int k, int* R) {
  *R = g.nbr(e, k, +1);
  if (*R < 0) return g.btype(k, +1) == LDGMG_BC_DIRICHLET ? 2 : 3;
  return mu[e] >= mu[*R] ? 1 : 0;
}

// G_k term codes: 0 D_k, 1 +T(-,-), 2 -T(+,+), 3 -T(-,+) [lower nbr], 4 +T(+,-) [upper nbr]
void build_gradient(PMat& G, const GridInfo& g, const ElemOps& em, const double* mu, int k) {
  const int bss = em.bss;
  build_pmat(G, g.ne, g.ne, bss, bss,
             [&](int e, std::map<int, Key>& row) {
               row[e].add(0);
               int L, R;
               const int sl = src_lower(g, mu, e, k, &L);
               if (sl == 0) {
                 row[L].add(3);
                 row[e].add(1);
               } else if (sl == 2) {
                 row[e].add(1);
               }
               const int su = src_upper(g, mu, e, k, &R);
               if (su == 0) {
                 row[R].add(4);
                 row[e].add(2);
               } else if (su == 2) {
                 row[e].add(2);
               }
             },
             [&](const std::string& key, double* out) {
               Vec acc(static_cast<size_t>(bss) * bss, 0.0);
               size_t off = 0;
               while (off < key.size()) {
                 const int code = read_at<int>(key, off);
                 const Vec* src = nullptr;
                 double s = 1.0;
                 switch (code) {
                   case 0: src = &em.D[k]; break;
                   case 1: src = &em.T[k][0][0]; break;
                   case 2: src = &em.T[k][1][1]; s = -1.0; break;
                   case 3: src = &em.T[k][0][1]; s = -1.0; break;
                   case 4: src = &em.T[k][1][0]; break;
                 }
                 for (size_t t = 0; t < acc.size(); ++t) acc[t] += s * (*src)[t];
               }
               matmul(bss, bss, bss, em.Minv.data(), acc.data(), out);
             });
}

void build_mu_mass(PMat& Mm, const GridInfo& g, const ElemOps& em, const double* mu) {
  const int bss = em.bss;
  build_pmat(Mm, g.ne, g.ne, bss, bss,
             [&](int e, std::map<int, Key>& row) { row[e].add(mu[e]); },
             [&](const std::string& key, double* out) {
               size_t off = 0;
               const double m = read_at<double>(key, off);
               for (int t = 0; t < bss * bss; ++t) out[t] = m * em.M[t];
             });
}

// penalty: kind 0 = scalar E (interior tau0 min(mu)/h, Dirichlet tau0 mu/h),
// kind 1 = pressure E_p (interior cp h / max(mu), no boundary terms).
// term: (k, code, tau) with code 0 +T(+,+), 1 +T(-,-), 2 -T(+,-) [upper nbr], 3 -T(-,+) [lower nbr]
void build_penalty(PMat& E, const GridInfo& g, const ElemOps& em, const double* mu, double c,
                   int kind) {
  const int bss = em.bss;
  const double h = em.h;
  auto face_tau = [&](int a, int b) {
    return kind == 0 ? c * std::min(mu[a], mu[b]) / h : c * h / std::max(mu[a], mu[b]);
  };
  build_pmat(E, g.ne, g.ne, bss, bss,
             [&](int e, std::map<int, Key>& row) {
               row[e];   // diagonal block always stored
               for (int k = 0; k < g.dim; ++k) {
                 const int L = g.nbr(e, k, -1);
                 if (L >= 0) {
                   const double tau = face_tau(L, e);
                   row[e].add(k).add(1).add(tau);
                   row[L].add(k).add(3).add(tau);
                 } else if (kind == 0 && g.btype(k, -1) == LDGMG_BC_DIRICHLET) {
                   row[e].add(k).add(1).add(c * mu[e] / h);
                 }
                 const int R = g.nbr(e, k, +1);
                 if (R >= 0) {
                   const double tau = face_tau(e, R);
                   row[e].add(k).add(0).add(tau);
                   row[R].add(k).add(2).add(tau);
                 } else if (kind == 0 && g.btype(k, +1) == LDGMG_BC_DIRICHLET) {
                   row[e].add(k).add(0).add(c * mu[e] / h);
                 }
               }
             },
             [&](const std::string& key, double* out) {
               std::fill(out, out + static_cast<size_t>(bss) * bss, 0.0);
               size_t off = 0;
               while (off < key.size()) {
                 const int k = read_at<int>(key, off);
                 const int code = read_at<int>(key, off);
                 const double tau = read_at<double>(key, off);
                 const Vec* src = nullptr;
                 double s = tau;
                 switch (code) {
                   case 0: src = &em.T[k][1][1]; break;
                   case 1: src = &em.T[k][0][0]; break;
                   case 2: src = &em.T[k][1][0]; s = -tau; break;
                   case 3: src = &em.T[k][0][1]; s = -tau; break;
                 }
                 for (int t = 0; t < bss * bss; ++t) out[t] += s * (*src)[t];
               }
             });
}

// ---------------------------------------------------------------------------
// coarsening
// ---------------------------------------------------------------------------
struct Family {   // parent/child maps between a fine and a coarse grid
  std::vector<int> parent, cpos;            // per fine element
  std::vector<std::vector<int>> children;   // per coarse element, indexed by cpos
};

Family make_family(const GridInfo& f, const GridInfo& c) {
  Family F;
  F.parent.resize(f.ne);
  F.cpos.resize(f.ne);
  F.children.assign(c.ne, std::vector<int>(1 << f.dim, -1));
  for (int e = 0; e < f.ne; ++e) {
    int ix[3], px[3];
    f.idx(e, ix);
    int cp = 0;
    for (int k = 0; k < f.dim; ++k) {
      px[k] = ix[k] / 2;
      cp |= (ix[k] & 1) << k;
    }
    const int pe = c.elem(px);
    F.parent[e] = pe;
    F.cpos[e] = cp;
    F.children[pe][cp] = e;
  }
  return F;
}

// C(Kc, Jc) = scale * L * sum_{f in ch(Kc)} sum_{(f,g)} I_f^T X_fg I_g ;  L = Mc^-1 (mode 1) or
// I (mode 0).  Fine blocks need the fine plain mass applied on the left (mode 1: X = M_f G_fg).
void coarsen_pmat(PMat& C, const PMat& F, const Family& fam, const GridInfo& cg,
                  const ElemOps& fem, const ElemOps& cem, double scale, bool grad) {
  const int bss = fem.bss;
  build_pmat(C, cg.ne, cg.ne, bss, bss,
             [&](int K, std::map<int, Key>& row) {
               for (int cp = 0; cp < static_cast<int>(fam.children[K].size()); ++cp) {
                 const int f = fam.children[K][cp];
                 for (int s = F.rp[f]; s < F.rp[f + 1]; ++s) {
                   const int g2 = F.ci[s];
                   row[fam.parent[g2]].add(cp).add(fam.cpos[g2]).add(F.id[s]);
                 }
               }
             },
             [&](const std::string& key, double* out) {
               Vec acc(static_cast<size_t>(bss) * bss, 0.0), t1(acc.size()), t2(acc.size());
               size_t off = 0;
               while (off < key.size()) {
                 const int cf = read_at<int>(key, off);
                 const int cgp = read_at<int>(key, off);
                 const int id = read_at<int>(key, off);
                 const double* X = F.pool.at(id);
                 if (grad) {          // M_f G
                   matmul(bss, bss, bss, fem.M.data(), X, t1.data());
                   X = t1.data();
                 }
                 matmul(bss, bss, bss, X, fem.Ic[cgp].data(), t2.data());          // X I_g
                 matmul_tn(bss, bss, bss, fem.Ic[cf].data(), t2.data(), acc.data(), true);  // I_f^T (.)
               }
               if (grad) {
                 matmul(bss, bss, bss, cem.Minv.data(), acc.data(), out);
               } else {
                 std::copy(acc.begin(), acc.end(), out);
               }
               for (int t = 0; t < bss * bss; ++t) out[t] *= scale;
             });
}

// ---------------------------------------------------------------------------
// products of factors
// ---------------------------------------------------------------------------
// columns of a pooled matrix: for column K the list of (row L, slot)
std::vector<std::vector<std::pair<int, int>>> transpose_pattern(const PMat& P) {
  std::vector<std::vector<std::pair<int, int>>> t(P.nbc);
  for (int L = 0; L < P.nbr; ++L)
    for (int s = P.rp[L]; s < P.rp[L + 1]; ++s) t[P.ci[s]].push_back({L, s});
  return t;
}

// R(K,J) = sum_t sum_L (Pa_t)_{L,K}^T Mmu_L (Pb_t)_{L,J}
void gram(PMat& R, const std::vector<std::pair<const PMat*, const PMat*>>& pairs, const PMat& Mmu,
          int bss) {
  std::vector<std::vector<std::vector<std::pair<int, int>>>> tp;
  for (auto& pr : pairs) tp.push_back(transpose_pattern(*pr.first));
  const int ne = Mmu.nbr;
  build_pmat(R, ne, ne, bss, bss,
             [&](int K, std::map<int, Key>& row) {
               for (size_t t = 0; t < pairs.size(); ++t) {
                 const PMat& Pb = *pairs[t].second;
                 for (auto& ls : tp[t][K]) {
                   const int L = ls.first;
                   const int idM = Mmu.id[Mmu.rp[L]];
                   for (int s = Pb.rp[L]; s < Pb.rp[L + 1]; ++s)
                     row[Pb.ci[s]].add(static_cast<int>(t)).add(pairs[t].first->id[ls.second]).add(idM).add(Pb.id[s]);
                 }
               }
             },
             [&](const std::string& key, double* out) {
               std::fill(out, out + static_cast<size_t>(bss) * bss, 0.0);
               Vec t1(static_cast<size_t>(bss) * bss), t2(t1.size());
               size_t off = 0;
               while (off < key.size()) {
                 const int t = read_at<int>(key, off);
                 const int ia = read_at<int>(key, off);
                 const int im = read_at<int>(key, off);
                 const int ib = read_at<int>(key, off);
                 matmul(bss, bss, bss, Mmu.pool.at(im), pairs[t].second->pool.at(ib), t1.data());
                 matmul_tn(bss, bss, bss, pairs[t].first->pool.at(ia), t1.data(), out, true);
               }
             });
}

// R(K,J) = (G_{J,K})^T M   (velocity row K, pressure column J of -G^T M)
void transpose_times_mass(PMat& R, const PMat& G, const ElemOps& em) {
  const int bss = em.bss;
  auto tp = transpose_pattern(G);
  build_pmat(R, G.nbc, G.nbr, bss, bss,
             [&](int K, std::map<int, Key>& row) {
               for (auto& ls : tp[K]) row[ls.first].add(G.id[ls.second]);
             },
             [&](const std::string& key, double* out) {
               size_t off = 0;
               const int id = read_at<int>(key, off);
               matmul_tn(bss, bss, bss, G.pool.at(id), em.M.data(), out);
             });
}

// R(K,J) = M G_{K,J}
void mass_times(PMat& R, const PMat& G, const ElemOps& em) {
  const int bss = em.bss;
  build_pmat(R, G.nbr, G.nbc, bss, bss,
             [&](int K, std::map<int, Key>& row) {
               for (int s = G.rp[K]; s < G.rp[K + 1]; ++s) row[G.ci[s]].add(G.id[s]);
             },
             [&](const std::string& key, double* out) {
               size_t off = 0;
               const int id = read_at<int>(key, off);
               matmul(bss, bss, bss, em.M.data(), G.pool.at(id), out);
             });
}

struct Piece {
  const PMat* P;
  int rc, cc;        // component block row / column
  double scale;
};

// system matrix from scalar pieces placed into (ncomp x ncomp) component blocks
void compose(PMat& A, const std::vector<Piece>& pieces, int ne, int bss, int ncomp) {
  const int bs = bss * ncomp;
  build_pmat(A, ne, ne, bs, bs,
             [&](int K, std::map<int, Key>& row) {
               for (size_t t = 0; t < pieces.size(); ++t) {
                 const PMat& P = *pieces[t].P;
                 for (int s = P.rp[K]; s < P.rp[K + 1]; ++s)
                   row[P.ci[s]].add(static_cast<int>(t)).add(P.id[s]);
               }
             },
             [&](const std::string& key, double* out) {
               std::fill(out, out + static_cast<size_t>(bs) * bs, 0.0);
               size_t off = 0;
               while (off < key.size()) {
                 const int t = read_at<int>(key, off);
                 const int id = read_at<int>(key, off);
                 const Piece& pc = pieces[t];
                 const double* blk = pc.P->pool.at(id);
                 for (int a = 0; a < bss; ++a)
                   for (int b = 0; b < bss; ++b)
                     out[static_cast<size_t>(pc.rc * bss + a) * bs + pc.cc * bss + b] +=
                         pc.scale * blk[static_cast<size_t>(a) * bss + b];
               }
             });
}

void assemble_system(HostLevel& L, int system, int gamma, double delta) {
  const int d = L.em.dim, bss = L.bss;
  PMat S;
  std::vector<std::pair<const PMat*, const PMat*>> lap;
  for (int k = 0; k < d; ++k) lap.push_back({&L.G[k], &L.G[k]});
  gram(S, lap, L.Mmu, bss);
  if (system == LDGMG_POISSON) {
    compose(L.A, {{&S, 0, 0, 1.0}, {&L.E, 0, 0, 1.0}}, L.ne, bss, 1);
    return;
  }
  std::vector<PMat> C;     // C[i*d+j] = G_j^T Mmu G_i  (stress-form coupling)
  if (gamma) {
    C.resize(d * d);
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) gram(C[i * d + j], {{&L.G[j], &L.G[i]}}, L.Mmu, bss);
  }
  std::vector<PMat> GtM(d), MG(d);
  for (int i = 0; i < d; ++i) {
    transpose_times_mass(GtM[i], L.G[i], L.em);
    mass_times(MG[i], L.G[i], L.em);
  }
  std::vector<Piece> pcs;
  for (int i = 0; i < d; ++i) {
    pcs.push_back({&S, i, i, 1.0});
    pcs.push_back({&L.E, i, i, 1.0});
    if (delta > 0) pcs.push_back({&L.Mrho, i, i, 1.0 / delta});   // eq:blockformunsteady
    if (gamma)
      for (int j = 0; j < d; ++j) pcs.push_back({&C[i * d + j], i, j, static_cast<double>(gamma)});
    pcs.push_back({&GtM[i], i, d, -1.0});
    pcs.push_back({&MG[i], d, i, -1.0});
  }
  pcs.push_back({&L.Ep, d, d, -1.0});
  compose(L.A, pcs, L.ne, bss, d + 1);
}

// ---------------------------------------------------------------------------
// smoothers
// ---------------------------------------------------------------------------
std::vector<int> diag_ids(const PMat& A) {
  std::vector<int> d(A.nbr);
  for (int i = 0; i < A.nbr; ++i) {
    const int s = A.slot(i, i);
    if (s < 0) throw std::runtime_error("missing diagonal block");
    d[i] = A.id[s];
  }
  return d;
}

void build_block_inverse(HostLevel& L) {
  const int bs = L.bs;
  const std::vector<int> did = diag_ids(L.A);
  const int nd = L.A.pool.size();
  std::vector<Vec> inv(nd);
  std::vector<char> used(nd, 0);
  for (int v : did) used[v] = 1;
  std::vector<int> todo;
  for (int i = 0; i < nd; ++i)
    if (used[i]) todo.push_back(i);
  parallel_for(static_cast<int>(todo.size()), [&](int t) {
    const int id = todo[t];
    const double* blk = L.A.pool.at(id);
    Vec sym(static_cast<size_t>(bs) * bs);
    for (int a = 0; a < bs; ++a)
      for (int b = 0; b < bs; ++b)
        sym[static_cast<size_t>(a) * bs + b] = 0.5 * (blk[static_cast<size_t>(a) * bs + b] + blk[static_cast<size_t>(b) * bs + a]);
    inv[id].assign(static_cast<size_t>(bs) * bs, 0.0);
    sym_pinv(bs, sym.data(), inv[id].data(), 0.0);
  });
  build_pmat(L.S, L.ne, L.ne, bs, bs,
             [&](int e, std::map<int, Key>& row) { row[e].add(did[e]); },
             [&](const std::string& key, double* out) {
               size_t off = 0;
               const int id = read_at<int>(key, off);
               std::copy(inv[id].begin(), inv[id].end(), out);
             });
  L.tpos.resize(L.S.nnzb());
  for (int s = 0; s < L.S.nnzb(); ++s) L.tpos[s] = s;
}

void build_colours(HostLevel& L) {
  const PMat& A = L.A;
  L.colour.assign(A.nbr, -1);
  int nc = 0;
  std::vector<char> used;
  for (int i = 0; i < A.nbr; ++i) {
    used.assign(nc + 1, 0);
    for (int s = A.rp[i]; s < A.rp[i + 1]; ++s) {
      const int j = A.ci[s];
      if (j != i && L.colour[j] >= 0) used[L.colour[j]] = 1;
    }
    int c = 0;
    while (used[c]) ++c;
    L.colour[i] = c;
    nc = std::max(nc, c + 1);
  }
  L.ncolours = nc;
  L.colour_rows.assign(nc, {});
  for (int i = 0; i < A.nbr; ++i) L.colour_rows[L.colour[i]].push_back(i);
}

// balancing vector per distinct diagonal block (Section 2.3.3 scalar, Section 3.3 Stokes)
std::vector<Vec> balance(const HostLevel& L, const std::vector<int>& did, int system, double zeta) {
  const int bs = L.bs, d = L.em.dim;
  std::vector<Vec> alpha(L.A.pool.size());
  for (int e = 0; e < L.ne; ++e) {
    const int id = did[e];
    if (!alpha[id].empty()) continue;
    const double* D = L.A.pool.at(id);
    Vec a(bs);
    if (system == LDGMG_POISSON) {
      double nf = 0;
      for (int t = 0; t < bs * bs; ++t) nf += D[t] * D[t];
      std::fill(a.begin(), a.end(), std::pow(std::sqrt(nf), -0.5));
    } else {
      const int nv = d * L.bss;
      double nA = 0, nD = 0;
      for (int r = 0; r < bs; ++r)
        for (int c = 0; c < nv; ++c) {
          const double v = D[static_cast<size_t>(r) * bs + c];
          if (r < nv) nA += v * v; else nD += v * v;
        }
      nA = std::sqrt(nA);
      nD = std::sqrt(nD);
      for (int r = 0; r < bs; ++r) a[r] = r < nv ? std::pow(nA, -0.5) : zeta * std::sqrt(nA) / nD;
    }
    alpha[id] = a;
  }
  return alpha;
}

std::vector<std::vector<int>> pattern_rows(const PMat& A, int ell) {
  const int n = A.nbr;
  std::vector<std::vector<int>> P(n);
  for (int i = 0; i < n; ++i) P[i] = {i};
  for (int l = 0; l < ell; ++l) {
    std::vector<std::vector<int>> Q(n);
    for (int i = 0; i < n; ++i) {
      std::vector<int> acc;
      for (int j : P[i])
        for (int s = A.rp[j]; s < A.rp[j + 1]; ++s) acc.push_back(A.ci[s]);
      std::sort(acc.begin(), acc.end());
      acc.erase(std::unique(acc.begin(), acc.end()), acc.end());
      Q[i] = std::move(acc);
    }
    P = std::move(Q);
  }
  return P;
}

void build_sai(HostLevel& L, int ell, int system, double zeta, const SaiBatchSolver* sai) {
  const int bs = L.bs, ne = L.ne;
  const PMat& A = L.A;
  const std::vector<int> did = diag_ids(A);
  const std::vector<Vec> alpha = balance(L, did, system, zeta);
  const auto J = pattern_rows(A, ell);            // symmetric pattern: row == column
  // per column: key of the balanced local least-squares problem
  std::vector<std::string> keys(ne);
  std::vector<std::vector<int>> Isets(ne);
  parallel_for(ne, [&](int i) {
    std::vector<int> I;
    for (int j : J[i])
      for (int s = A.rp[j]; s < A.rp[j + 1]; ++s) I.push_back(A.ci[s]);
    std::sort(I.begin(), I.end());
    I.erase(std::unique(I.begin(), I.end()), I.end());
    Key k;
    const int pos = static_cast<int>(std::lower_bound(I.begin(), I.end(), i) - I.begin());
    k.add(static_cast<int>(I.size())).add(static_cast<int>(J[i].size())).add(pos);
    for (int a : I) k.add(did[a]);
    for (int b : J[i]) k.add(did[b]);
    for (int a : I)
      for (int b : J[i]) {
        const int s = A.slot(a, b);
        k.add(s < 0 ? -1 : A.id[s]);
      }
    keys[i] = std::move(k.s);
    Isets[i] = std::move(I);
  });
  std::unordered_map<std::string, int> uniq;
  std::vector<int> col_ls(ne), rep;
  for (int i = 0; i < ne; ++i) {
    auto it = uniq.find(keys[i]);
    if (it == uniq.end()) {
      it = uniq.emplace(keys[i], static_cast<int>(rep.size())).first;
      rep.push_back(i);
    }
    col_ls[i] = it->second;
  }
  keys.clear();
  keys.shrink_to_fit();
  L.sai_unique = static_cast<int>(rep.size());
  // solve the representative problems: X = argmin || A~[I,J] X - E[I,i] ||
  const auto t_ls = std::chrono::steady_clock::now();
  std::vector<Vec> sol(rep.size());
  std::vector<char> solved(rep.size(), 0);
  if (sai && !rep.empty()) {   // the batch solver first (e.g. on the GPU); the host takes what it declines
    SaiBatch batch;
    batch.bs = bs;
    batch.pool = A.pool.data.data();
    batch.npool = A.pool.size();
    std::vector<double> al(alpha.size() * static_cast<size_t>(bs));
    for (size_t d = 0; d < alpha.size(); ++d)
      if (alpha[d].size() == static_cast<size_t>(bs)) std::copy(alpha[d].begin(), alpha[d].end(), al.begin() + d * bs);
    batch.alpha = al.data();
    batch.nalpha = static_cast<int>(alpha.size());
    batch.probs.resize(rep.size());
    parallel_for(static_cast<int>(rep.size()), [&](int u) {
      const int i = rep[u];
      const auto& I = Isets[i];
      const auto& Jc = J[i];
      SaiProblem& pb = batch.probs[u];
      pb.mb = static_cast<int>(I.size());
      pb.nb = static_cast<int>(Jc.size());
      pb.pos = static_cast<int>(std::lower_bound(I.begin(), I.end(), i) - I.begin());
      for (size_t a = 0; a < I.size(); ++a)
        for (size_t b = 0; b < Jc.size(); ++b) {
          const int s = A.slot(I[a], Jc[b]);
          if (s < 0) continue;
          pb.brow.push_back(static_cast<int>(a));
          pb.bcol.push_back(static_cast<int>(b));
          pb.bid.push_back(A.id[s]);
          pb.arow.push_back(did[I[a]]);
          pb.acol.push_back(did[Jc[b]]);
        }
      sol[u].assign(static_cast<size_t>(pb.nb) * bs * bs, 0.0);
      pb.X = sol[u].data();
    });
    const std::vector<char> ok = (*sai)(batch);
    for (size_t u = 0; u < rep.size() && u < ok.size(); ++u) solved[u] = ok[u];
    L.sai_device = static_cast<int>(std::count(solved.begin(), solved.end(), 1));
  }
  std::atomic<bool> singular{false};
  std::atomic<int> qr_fallback{0};
  parallel_for(static_cast<int>(rep.size()), [&](int u) {
    if (solved[u]) return;
    const int i = rep[u];
    const auto& I = Isets[i];
    const auto& Jc = J[i];
    const int m = static_cast<int>(I.size()) * bs, n = static_cast<int>(Jc.size()) * bs;
    const int pos = static_cast<int>(std::lower_bound(I.begin(), I.end(), i) - I.begin());
    Vec X(static_cast<size_t>(n) * bs);
    {
      // block-sparse normal equations (only the nonzero blocks of A~[I,J])
      const size_t T = static_cast<size_t>(bs) * bs;
      std::vector<std::vector<std::pair<int, const double*>>> brow(I.size());
      size_t nnz = 0;
      for (size_t a = 0; a < I.size(); ++a)
        for (size_t b = 0; b < Jc.size(); ++b) nnz += A.slot(I[a], Jc[b]) >= 0;
      Vec blocks(nnz * T);
      size_t q = 0;
      for (size_t a = 0; a < I.size(); ++a) {
        const Vec& al = alpha[did[I[a]]];
        for (size_t b = 0; b < Jc.size(); ++b) {
          const int s = A.slot(I[a], Jc[b]);
          if (s < 0) continue;
          const Vec& be = alpha[did[Jc[b]]];
          const double* blk = A.block(s);
          double* out = &blocks[q * T];
          for (int r = 0; r < bs; ++r)
            for (int c = 0; c < bs; ++c) out[static_cast<size_t>(r) * bs + c] = al[r] * blk[static_cast<size_t>(r) * bs + c] * be[c];
          brow[a].push_back({static_cast<int>(b), out});
          ++q;
        }
      }
      if (ls_block_normal(bs, static_cast<int>(I.size()), static_cast<int>(Jc.size()), brow, pos, X.data())) {
        sol[u] = std::move(X);
        return;
      }
      ++qr_fallback;
    }
    Vec C(static_cast<size_t>(m) * n, 0.0), R(static_cast<size_t>(m) * bs, 0.0);
    for (size_t a = 0; a < I.size(); ++a) {
      const Vec& al = alpha[did[I[a]]];
      for (size_t b = 0; b < Jc.size(); ++b) {
        const int s = A.slot(I[a], Jc[b]);
        if (s < 0) continue;
        const Vec& be = alpha[did[Jc[b]]];
        const double* blk = A.block(s);
        for (int r = 0; r < bs; ++r)
          for (int c = 0; c < bs; ++c)   // column-major C
            C[static_cast<size_t>(b * bs + c) * m + a * bs + r] = al[r] * blk[static_cast<size_t>(r) * bs + c] * be[c];
      }
    }
    for (int c = 0; c < bs; ++c) R[static_cast<size_t>(c) * m + pos * bs + c] = 1.0;
    if (!ls_householder(m, n, bs, C.data(), R.data(), X.data())) singular = true;
    sol[u] = std::move(X);
  });
  if (singular) throw std::runtime_error("rank-deficient SAI least-squares problem");
  L.sai_qr = qr_fallback.load();
  L.sai_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_ls).count();
  // B(j, i) = diag(alpha_j) X_b diag(alpha_i), stored row-wise with the pattern of A^ell
  std::vector<std::vector<std::pair<int, std::string>>> rows(ne);   // row j: (col i, key)
  for (int i = 0; i < ne; ++i)
    for (size_t b = 0; b < J[i].size(); ++b) {
      Key k;
      k.add(col_ls[i]).add(static_cast<int>(b)).add(did[J[i][b]]).add(did[i]);
      rows[J[i][b]].push_back({i, std::move(k.s)});
    }
  PMat& B = L.S;
  B.nbr = B.nbc = ne;
  B.pool.r = B.pool.c = bs;
  B.rp.assign(ne + 1, 0);
  B.ci.clear();
  B.id.clear();
  for (int j = 0; j < ne; ++j) {
    auto& r = rows[j];
    std::sort(r.begin(), r.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
    for (auto& ck : r) {
      B.ci.push_back(ck.first);
      B.id.push_back(B.pool.intern(ck.second, [&](double* out) {
        size_t off = 0;
        const int u = read_at<int>(ck.second, off);
        const int b = read_at<int>(ck.second, off);
        const int dj = read_at<int>(ck.second, off);
        const int di = read_at<int>(ck.second, off);
        const Vec& X = sol[u];
        const int n = static_cast<int>(X.size()) / bs;
        const Vec& aj = alpha[dj];
        const Vec& ai = alpha[di];
        for (int r2 = 0; r2 < bs; ++r2)
          for (int c = 0; c < bs; ++c)   // X column-major (n x bs): X[c*n + b*bs + r2]
            out[static_cast<size_t>(r2) * bs + c] = aj[r2] * X[static_cast<size_t>(c) * n + b * bs + r2] * ai[c];
      }));
    }
    B.rp[j + 1] = static_cast<int>(B.ci.size());
    std::vector<std::pair<int, std::string>>().swap(r);
  }
  L.tpos.resize(B.nnzb());
  for (int i = 0; i < ne; ++i)
    for (int s = B.rp[i]; s < B.rp[i + 1]; ++s) {
      const int t = B.slot(B.ci[s], i);
      if (t < 0) throw std::runtime_error("SAI pattern is not symmetric");
      L.tpos[s] = t;
    }
}

void build_bottom(HostLevel& L) {
  const int N = L.ne * L.bs, bs = L.bs;
  Vec dense(static_cast<size_t>(N) * N, 0.0);
  for (int i = 0; i < L.ne; ++i)
    for (int s = L.A.rp[i]; s < L.A.rp[i + 1]; ++s) {
      const int j = L.A.ci[s];
      const double* blk = L.A.block(s);
      for (int a = 0; a < bs; ++a)
        for (int b = 0; b < bs; ++b) dense[static_cast<size_t>(i * bs + a) * N + j * bs + b] += blk[a * bs + b];
    }
  for (int r = 0; r < N; ++r)
    for (int c = r + 1; c < N; ++c) {
      const double v = 0.5 * (dense[static_cast<size_t>(r) * N + c] + dense[static_cast<size_t>(c) * N + r]);
      dense[static_cast<size_t>(r) * N + c] = dense[static_cast<size_t>(c) * N + r] = v;
    }
  L.pinv.assign(static_cast<size_t>(N) * N, 0.0);
  sym_pinv(N, dense.data(), L.pinv.data(), 1e-12, g_threads);
}

}  // namespace

namespace {

// smoother of one non-bottom level from its assembled A (Sections 2.3, 3.3)
void build_smoother(HostLevel& L, const ldgmg_problem& pr, double zeta, const SaiBatchSolver* sai) {
  if (pr.smoother == LDGMG_SMOOTH_SAI) {
    build_sai(L, pr.sai_level, pr.system, zeta, sai);
  } else {
    build_block_inverse(L);
    if (pr.smoother == LDGMG_SMOOTH_GS) build_colours(L);
  }
}

double default_omega(const ldgmg_problem& pr) {
  return pr.omega > 0 ? pr.omega : (pr.smoother == LDGMG_SMOOTH_JACOBI ? 0.8 : 1.0);
}

double default_zeta(const ldgmg_problem& pr) {
  if (pr.zeta > 0) return pr.zeta;
  static const double tz[2][2][5] = {{{0.0382, 0.131, 0.0990, 0.153, 0.142}, {0.0462, 0.107, 0.113, 0.113, 0.113}},
                                     {{0.118, 0.131, 0.0814, 0.123, 0.0745}, {0.0384, 0.0928, 0.0930, 0.0930, 0.0930}}};
  return tz[pr.gamma ? 1 : 0][pr.dim - 2][pr.p - 1];
}

}  // namespace

std::unique_ptr<HostHierarchy> rebuild_smoother(const HostHierarchy& src, const ldgmg_problem& pr,
                                               const SaiBatchSolver* sai) {
  validate_problem(pr);
  const ldgmg_problem& q = src.prob;
  bool same = pr.dim == q.dim && pr.n == q.n && pr.p == q.p && pr.basis == q.basis && pr.system == q.system &&
              pr.gamma == q.gamma && pr.tau0 == q.tau0 && pr.cp == q.cp && pr.delta == q.delta;
  for (int f = 0; f < 6; ++f) same = same && pr.bc[f] == q.bc[f];
  if (same) {
    for (size_t e = 0; e < src.mu.size(); ++e)
      if ((pr.mu ? pr.mu[e] : 1.0) != src.mu[e]) {
        same = false;
        break;
      }
    for (size_t e = 0; e < src.rho.size(); ++e)
      if ((pr.rho ? pr.rho[e] : 1.0) != src.rho[e]) {
        same = false;
        break;
      }
  }
  if (!same) throw std::invalid_argument("rebuild_smoother: the problem differs from the source hierarchy's");
  const auto t0 = std::chrono::steady_clock::now();
  g_threads = pr.nthreads > 0 ? pr.nthreads : std::max(1u, std::thread::hardware_concurrency());
  auto H = std::make_unique<HostHierarchy>(src);   // operators, transfers, bottom pseudo-inverse
  H->prob = pr;
  H->prob.mu = nullptr;
  H->prob.rho = nullptr;
  H->omega = default_omega(pr);
  H->zeta = default_zeta(pr);
  for (size_t l = 0; l + 1 < H->levels.size(); ++l) {
    HostLevel& L = H->levels[l];
    const auto tl = std::chrono::steady_clock::now();
    L.S = PMat{};
    L.tpos.clear();
    L.colour_rows.clear();
    L.ncolours = 0;
    L.sai_unique = L.sai_qr = L.sai_device = 0;
    L.sai_seconds = 0;
    build_smoother(L, pr, H->zeta, sai);
    L.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - tl).count();
  }
  H->setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return H;
}

std::unique_ptr<HostHierarchy> build_host(const ldgmg_problem& pr, const SaiBatchSolver* sai) {
  validate_problem(pr);
  const auto t0 = std::chrono::steady_clock::now();
  g_threads = pr.nthreads > 0 ? pr.nthreads : std::max(1u, std::thread::hardware_concurrency());
  auto H = std::make_unique<HostHierarchy>();
  H->prob = pr;
  H->prob.mu = nullptr;
  const int d = pr.dim;
  long long ne0 = 1;
  for (int k = 0; k < d; ++k) ne0 *= pr.n;
  H->mu.assign(ne0, 1.0);
  if (pr.mu) std::copy(pr.mu, pr.mu + ne0, H->mu.begin());
  H->prob.rho = nullptr;
  if (pr.delta > 0) {
    H->rho.assign(ne0, 1.0);
    if (pr.rho) std::copy(pr.rho, pr.rho + ne0, H->rho.begin());
  }
  H->omega = default_omega(pr);
  H->zeta = default_zeta(pr);
  const std::vector<int> sizes = level_sizes(pr.n);
  const int ncomp = pr.system == LDGMG_STOKES ? d + 1 : 1;
  std::vector<GridInfo> grids;
  for (int n : sizes) {
    GridInfo g{};
    g.dim = d;
    g.n = n;
    g.ne = 1;
    for (int k = 0; k < d; ++k) g.ne *= n;
    for (int f = 0; f < 6; ++f) g.bc[f] = pr.bc[f];
    grids.push_back(g);
  }
  H->levels.resize(sizes.size());
  for (size_t l = 0; l < sizes.size(); ++l) {
    HostLevel& L = H->levels[l];
    const auto tl = std::chrono::steady_clock::now();
    L.n = sizes[l];
    L.ne = grids[l].ne;
    L.h = 1.0 / L.n;
    L.em.init(d, pr.p, L.h, pr.basis);
    L.bss = L.em.bss;
    L.ncomp = ncomp;
    L.bs = L.bss * ncomp;
    L.G.resize(d);
    if (l == 0) {
      const double* mu = H->mu.data();
      for (int k = 0; k < d; ++k) build_gradient(L.G[k], grids[0], L.em, mu, k);
      build_mu_mass(L.Mmu, grids[0], L.em, mu);
      build_penalty(L.E, grids[0], L.em, mu, pr.tau0, 0);
      if (ncomp > 1) {
        if (pr.delta > 0) {
          // unsteady: the pressure penalty sees mu + rho h^2 / delta (blending the
          // viscous and the projection limits); the velocity blocks gain M_rho / delta
          std::vector<double> mu_eff(H->mu);
          for (size_t e = 0; e < mu_eff.size(); ++e) mu_eff[e] += H->rho[e] * L.h * L.h / pr.delta;
          build_penalty(L.Ep, grids[0], L.em, mu_eff.data(), pr.cp, 1);
          build_mu_mass(L.Mrho, grids[0], L.em, H->rho.data());
        } else {
          build_penalty(L.Ep, grids[0], L.em, mu, pr.cp, 1);
        }
      }
    } else {
      HostLevel& F = H->levels[l - 1];
      const Family fam = make_family(grids[l - 1], grids[l]);
      for (int k = 0; k < d; ++k) coarsen_pmat(L.G[k], F.G[k], fam, grids[l], F.em, L.em, 1.0, true);
      coarsen_pmat(L.Mmu, F.Mmu, fam, grids[l], F.em, L.em, 1.0, false);
      coarsen_pmat(L.E, F.E, fam, grids[l], F.em, L.em, 0.5, false);
      if (ncomp > 1) coarsen_pmat(L.Ep, F.Ep, fam, grids[l], F.em, L.em, 2.0, false);
      if (pr.delta > 0) coarsen_pmat(L.Mrho, F.Mrho, fam, grids[l], F.em, L.em, 1.0, false);
    }
    assemble_system(L, pr.system, pr.gamma, pr.delta);
    const bool bottom = l + 1 == sizes.size();
    if (bottom) {
      build_bottom(L);
    } else {
      build_smoother(L, pr, H->zeta, sai);
    }
    L.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - tl).count();
  }
  H->setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return H;
}

}  // namespace ldgmg

// Host setup under AddressSanitizer and UndefinedBehaviorSanitizer: builds
// hierarchies of the library's host code (host.cpp, dense.cpp; no GPU code)
// for a spread of problems and exercises the threaded paths (SAI columns,
// block inverses, bottom eigensolver) and the smoother rebuild.  Compiled and
// run by tests/test_host_setup.py; exits non-zero on a failed check, and the
// sanitizers abort on the first error they find.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../paper_2412_12506_amd/csrc/host.hpp"

namespace {

ldgmg_problem base(int dim, int n, int p) {
  ldgmg_problem q{};
  q.dim = dim;
  q.n = n;
  q.p = p;
  q.basis = LDGMG_BASIS_LEGENDRE;
  q.system = LDGMG_POISSON;
  q.gamma = 1;
  for (int f = 0; f < 6; ++f) q.bc[f] = LDGMG_BC_DIRICHLET;
  q.tau0 = 1.0;
  q.cp = 0.1;
  q.smoother = LDGMG_SMOOTH_SAI;
  q.sai_level = 1;
  q.order = LDGMG_ORDER_OI;
  q.nu1 = q.nu2 = 3;
  q.precision = LDGMG_FP32;
  q.nthreads = 4;
  q.storage = LDGMG_STORE_AUTO;
  return q;
}

int check(const char* what, const ldgmg::HostHierarchy& H, int levels) {
  if (static_cast<int>(H.levels.size()) != levels) {
    std::printf("%s: %zu levels, expected %d\n", what, H.levels.size(), levels);
    return 1;
  }
  for (const auto& L : H.levels)
    if (L.A.nnzb() <= 0) {
      std::printf("%s: empty operator\n", what);
      return 1;
    }
  std::printf("%s: ok (%zu levels)\n", what, H.levels.size());
  return 0;
}

}  // namespace

int main() {
  int bad = 0;
  {
    ldgmg_problem q = base(3, 4, 3);
    bad += check("poisson 3D p=3 SAI_1", *ldgmg::build_host(q), 2);
  }
  {
    ldgmg_problem q = base(2, 8, 2);
    std::vector<double> mu(64, 1.0);
    for (int e = 0; e < 64; ++e)
      if ((e % 8) >= 2 && (e % 8) < 6 && (e / 8) >= 2 && (e / 8) < 6) mu[e] = 1e4;
    q.mu = mu.data();
    q.smoother = LDGMG_SMOOTH_GS;
    auto H = ldgmg::build_host(q);
    bad += check("interface 2D p=2 GS", *H, 3);
    q.smoother = LDGMG_SMOOTH_SAI;
    q.sai_level = 2;
    bad += check("interface 2D p=2 rebuilt with SAI_2", *ldgmg::rebuild_smoother(*H, q), 3);
  }
  {
    ldgmg_problem q = base(2, 8, 2);
    q.system = LDGMG_STOKES;
    std::vector<double> mu(64, 1.0), rho(64, 1.0);
    for (int e = 0; e < 64; ++e)
      if ((e % 8) >= 2 && (e % 8) < 6 && (e / 8) >= 2 && (e / 8) < 6) {
        mu[e] = 2e-4;
        rho[e] = 1e-3;
      }
    q.mu = mu.data();
    q.rho = rho.data();
    q.delta = 0.1 / 8;
    bad += check("unsteady stress Stokes 2D p=2 SAI_1", *ldgmg::build_host(q), 3);
    q.delta = 0.0;
    q.gamma = 0;
    q.smoother = LDGMG_SMOOTH_JACOBI;
    bad += check("standard Stokes 2D p=2 Jacobi", *ldgmg::build_host(q), 3);
  }
  {
    ldgmg_problem q = base(2, 10, 3);     // bottom of 400 unknowns: threaded eigensolver
    q.smoother = LDGMG_SMOOTH_JACOBI;
    q.nthreads = 3;
    for (int f = 0; f < 4; ++f) q.bc[f] = LDGMG_BC_NEUMANN;
    bad += check("Neumann 2D p=3 threaded bottom", *ldgmg::build_host(q), 2);
  }
  return bad ? 1 : 0;
}

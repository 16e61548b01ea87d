// Host-side (FP64) setup of the multigrid hierarchy.
//
// Block-sparse matrices are kept "pooled": every stored block position holds
// the id of a block in a per-matrix pool of distinct values, and each pool
// entry is computed once from a key that lists exactly the inputs of its
// arithmetic.  Translated copies of the same local configuration therefore get
// the same id (bit-identical values), which keeps host memory at O(nnzb) ints
// and makes the SAI cache of identical columns (Section 4, item (i)) exact.
#pragma once

#include <array>
#include <functional>
#include <cstdint>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/ldgmg.h"

namespace ldgmg {

struct Key {
  std::string s;
  Key& add(int v) { s.append(reinterpret_cast<const char*>(&v), sizeof v); return *this; }
  Key& add(double v) { s.append(reinterpret_cast<const char*>(&v), sizeof v); return *this; }
};

struct Pool {
  int r = 0, c = 0;
  std::vector<double> data;
  std::unordered_map<std::string, int> memo;
  int size() const { return (r > 0 && c > 0) ? static_cast<int>(data.size() / (static_cast<size_t>(r) * c)) : 0; }
  const double* at(int id) const { return data.data() + static_cast<size_t>(id) * r * c; }
  // returns the id for key, computing the block with fn(double* out) on a miss
  template <class F>
  int intern(const std::string& key, F&& fn) {
    auto it = memo.find(key);
    if (it != memo.end()) return it->second;
    const int id = size();
    data.resize(data.size() + static_cast<size_t>(r) * c, 0.0);
    fn(data.data() + static_cast<size_t>(id) * r * c);
    memo.emplace(key, id);
    return id;
  }
};

// pooled block-sparse matrix (CSR of blocks)
struct PMat {
  int nbr = 0, nbc = 0;
  std::vector<int> rp, ci, id;
  Pool pool;
  mutable double tile_passes = -1.0;   // cache of the device's tiling estimate (< 0: not computed)
  mutable int tile_perm_len = -1;      // and of the length of its tile order (rows plus padding)
  int nnzb() const { return static_cast<int>(ci.size()); }
  int slot(int i, int j) const;     // -1 if (i, j) is not stored
  const double* block(int s) const { return pool.at(id[s]); }
};

// Physical element matrices of Q_p on a cube of side h (scalar fields).
struct ElemOps {
  int dim = 0, p = 0, q1 = 0, bss = 0;
  double h = 0;
  std::vector<double> m, adv, tm, tp;        // 1-D reference matrices / traces
  std::vector<double> P[2];                  // 1-D child injection, (q1 x q1)
  std::vector<double> M, Minv;               // element mass and inverse (bss x bss)
  std::vector<double> D[3];                  // int w d_k u
  std::vector<double> T[3][2][2];            // face matrices [k][test side][trial side]
  std::vector<double> Ic[8];                 // child injection, bss x bss
  void init(int dim, int p, double h, int basis);
};

struct HostLevel {
  int n = 0, ne = 0, bs = 0, bss = 0, ncomp = 1;
  double h = 0;
  ElemOps em;
  std::vector<PMat> G;         // per dimension (scalar blocks)
  PMat Mmu, E, Ep;             // scalar blocks
  PMat Mrho;                   // density-weighted mass (unsteady Stokes), scalar blocks
  PMat A;                      // system blocks (bs x bs)
  PMat S;                      // smoother matrix: B (SAI) or D^-1 (block diagonal)
  std::vector<int> tpos;       // slot of S(j,i) for each slot (i,j) of S
  std::vector<int> colour;
  int ncolours = 0;
  std::vector<std::vector<int>> colour_rows;
  std::vector<double> pinv;    // bottom pseudo-inverse, dense (ne*bs)^2
  int sai_unique = 0;
  int sai_qr = 0;               // of those, solved by Householder QR (normal equations declined)
  int sai_device = 0;           // of those, solved by the batch solver (GPU setup)
  double sai_seconds = 0;       // time of the level's SAI least-squares solves
  double setup_seconds = 0;
};

struct HostHierarchy {
  ldgmg_problem prob{};
  std::vector<double> mu;      // fine-level viscosity
  std::vector<double> rho;     // fine-level density (unsteady Stokes; empty when steady)
  std::vector<HostLevel> levels;
  double omega = 0, zeta = 0;
  double setup_seconds = 0;
};

// One balanced SAI least-squares problem of a representative column (Section
// 2.3.3): min || C X - E ||_F with C = A~[I, J], mb x nb blocks of bs x bs given
// by its nonzero blocks, and E the identity block at block row pos.  X is
// (nb bs) x bs, column-major.
// Block (a, b) of C is diag(alpha[arow]) A_pool[bid] diag(alpha[acol]).
struct SaiProblem {
  int mb = 0, nb = 0, pos = 0;
  std::vector<int> brow, bcol;       // block coordinates of the nonzero blocks of C
  std::vector<int> bid, arow, acol;  // their pool block of A and balancing vectors
  double* X = nullptr;               // the solution (filled by the solver)
};
struct SaiBatch {
  int bs = 0;
  const double* pool = nullptr;      // A's distinct blocks, row-major bs x bs each
  int npool = 0;
  const double* alpha = nullptr;     // balancing vectors, bs each
  int nalpha = 0;
  std::vector<SaiProblem> probs;
};
// Solves a batch of SAI problems (e.g. on a GPU); returns, per problem,
// whether its X was written (the host solves the others).
using SaiBatchSolver = std::function<std::vector<char>(SaiBatch& batch)>;

// Throws std::runtime_error / std::invalid_argument on failure.  With `sai`,
// the SAI least-squares problems of every level go to that solver first.
std::unique_ptr<HostHierarchy> build_host(const ldgmg_problem& prob, const SaiBatchSolver* sai = nullptr);

// A hierarchy for prob that keeps src's operators, transfers and bottom
// pseudo-inverse and builds only the smoother of prob; prob must describe the
// same discrete problem as src (geometry, basis, system, penalties and the same
// viscosity values), else std::invalid_argument.
std::unique_ptr<HostHierarchy> rebuild_smoother(const HostHierarchy& src, const ldgmg_problem& prob,
                                               const SaiBatchSolver* sai = nullptr);

// q-point Gauss-Legendre rule on [-1, 1] (ascending nodes)
void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w);
// values (v) and derivatives (dv) of the 1-D basis functions psi_0..psi_p at t
void basis_eval(int p, int basis, double t, double* v, double* dv);

// Number of levels and per-level n for a fine n (halve while even and > 2).
std::vector<int> level_sizes(int n);

void validate_problem(const ldgmg_problem& p);

}  // namespace ldgmg

// Device hierarchy, V-cycle (Algorithm 1), Krylov drivers and the C-ABI.
//
// Precision: the V-cycle (matrices, smoothers, transfers, vectors) runs in the
// handle's precision T (float or double); the outer Krylov iteration, its
// operator A (fine level) and all inner products are FP64.  The bottom solve
// is an FP64 dense product with the pseudo-inverse.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <mutex>
#include <vector>

#include "../../include/ldgmg.h"
#include "host.hpp"
#include "launch.hpp"
#include "setup.hpp"

// Scratch for ldgmg_vcycle_batch_noalloc: 16M doubles (128 MiB) of device
// memory that each GPU holds from module load to process end; host code
// reaches it only through the address hipGetSymbolAddress gives per device.
constexpr long long kScratchDoubles = 16ll << 20;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace ldgmg {

namespace {

thread_local std::string g_err;

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct BudgetError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct StateError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct SingularError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    const hipError_t e_ = (x);                                                         \
    if (e_ != hipSuccess) throw HipError(std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

// tiled storage of one matrix (forward products on the matrix cores)
struct Tiled {
  const void* blk = nullptr;        // pool in the operand layout of the tiled kernel
  int* tab = nullptr;               // [rows][noff] pool ids, -1 where no block
  int* perm = nullptr;              // rows ordered by their row of tab, -1 where a tile is padded
  int nperm = 0;                    // entries of perm
  int* rows = nullptr;              // the same order unpadded (for tiles of fewer than 16 rows)
  int* off = nullptr;               // column offsets
  int noff = 0;
  bool quad = false;                // pool in the 4-step k mapping (read with FP32 x)
};

struct DevLevel {
  int index = 0;
  int n = 0, ne = 0, bs = 0, bss = 0, ncomp = 1;
  long long N = 0;                  // unknowns on the level
  int nnzA = 0, nnzS = 0;
  int* rpA = nullptr;
  int* ciA = nullptr;
  void* valA = nullptr;             // working precision
  int* rpS = nullptr;
  int* ciS = nullptr;
  int* tposS = nullptr;
  void* valS = nullptr;
  void* valST = nullptr;            // transposed copy: block (i,j) holds (S_ji)^T (fast kernels only)
  int* bidA = nullptr;              // pooled storage: block id per slot (null when expanded)
  int* bidS = nullptr;
  int* bidST = nullptr;
  Tiled tA, tS, tST;                // tiled storage (tab null when not tiled)
  bool p32 = false;                 // FP32 products in the tiled applies of the V-cycle
  float* r32 = nullptr;             // FP32 smoothing residual for those products (levels with tiled A and S, 16 | bs)
  float* x32 = nullptr;             // and the FP32 copy of x that the A applies read there (kept by x's producers)
  std::vector<int*> colour_rows;    // device lists per colour
  std::vector<int> colour_count;
  double* x = nullptr;              // level vectors are FP64 in both precisions
  double* b = nullptr;
  double* r = nullptr;
  double* t = nullptr;
  double* Ic = nullptr;             // child injection matrices [2^d][bss][bss]
  double* P1 = nullptr;             // 1-D child matrices [2][p+1][p+1]
  int q1 = 0;
  double* pinv = nullptr;           // bottom only
};

struct DevHier {
  int prec = LDGMG_FP32;
  int storage = LDGMG_STORE_AUTO;
  int device = 0;
  std::vector<DevLevel> L;
  double* val64 = nullptr;          // fine-level FP64 A values (own copy only in FP32 mode)
  int* bid64 = nullptr;             // its block ids when pooled
  Tiled t64;                        // and its tiled form
  bool own64 = false;
  double *kx = nullptr, *kr = nullptr, *kp = nullptr, *kq = nullptr, *kz = nullptr;
  double* scal = nullptr;           // scalar table
  double* partial = nullptr;        // reduction partials
  double* hscal = nullptr;          // pinned host mirror of scal
  double* Q = nullptr;              // GMRES basis
  int Qcap = 0;
  double* hvec = nullptr;           // device small vectors (GMRES coefficients)
  std::vector<void*> allocs;
  std::vector<size_t> sizes;
  size_t bytes = 0;
  // caller's device allocator (ldgmg_problem::dev_alloc / dev_free), or null: hipMalloc / hipFree
  void* (*ualloc)(size_t, void*) = nullptr;
  void (*ufree)(void*, void*) = nullptr;
  void* uctx = nullptr;
  // kernel of the fine operator (singular problems): nker unit vectors khat_i
  // (Euclidean norm 1) and their mean weights w_i = M khat_i / (khat_i^T M khat_i),
  // each [N]; bproj holds projected right-hand sides (kMaxRhs vectors)
  int nker = 0;
  double* khat = nullptr;
  double* kw = nullptr;
  double* bproj = nullptr;
  // batched solves (ldgmg_solve_batch): per level [kMaxRhs][N] x, b, r, t and the
  // fine-level Krylov vectors; allocated on the first batched call
  struct BatchLevel {
    double *x = nullptr, *b = nullptr, *r = nullptr, *t = nullptr;
  };
  std::vector<BatchLevel> BL;
  int bcap = 0;                     // right-hand sides the batch vectors hold (8 or kMaxRhs)
  double *bx = nullptr, *br = nullptr, *bp = nullptr, *bq = nullptr, *bz = nullptr;
  double* bscal = nullptr;          // per right-hand side scalars [kMaxRhs][8]
  double* hbscal = nullptr;         // pinned host mirror
  // CG iteration captured in a graph (ldgmg_cg_graph): the executable graph,
  // the handle generation it was captured at, its capture stream and the
  // device residual history
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int ggen = -1;
  hipStream_t capst = nullptr;
  double* ghist = nullptr;
  // fine-level launch timing (ldgmg_profile)
  bool prof = false;
  std::vector<hipEvent_t> evpool;
  struct Rec {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;

  void* raw_alloc(size_t n) {
    void* p = nullptr;
    if (n == 0) n = 16;
    if (ualloc) {
      p = ualloc(n, uctx);
      if (!p) throw BudgetError("the caller's dev_alloc returned NULL for " + std::to_string(n) + " bytes");
      return p;
    }
    const hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) throw BudgetError(std::string("hipMalloc failed: ") + hipGetErrorString(e));
    return p;
  }
  void* alloc(size_t n) {
    void* p = raw_alloc(n);
    allocs.push_back(p);
    sizes.push_back(n == 0 ? 16 : n);
    bytes += n == 0 ? 16 : n;
    return p;
  }
  // give one buffer of `alloc` back before the handle goes (its users on the
  // device must have finished: the caller synchronises first)
  void release(void* p) {
    for (size_t i = 0; i < allocs.size(); ++i)
      if (allocs[i] == p) {
        if (ufree) ufree(p, uctx);
        else (void)hipFree(p);
        bytes -= sizes[i];
        allocs.erase(allocs.begin() + static_cast<long>(i));
        sizes.erase(sizes.begin() + static_cast<long>(i));
        return;
      }
  }
  // temporary upload buffers: stream-ordered with HIP's pool, or the caller's
  // allocator (freed once the stream has drained)
  void* stage(size_t n, hipStream_t st) {
    if (ualloc) return raw_alloc(n);
    void* p = nullptr;
    HIPCHK(hipMallocAsync(&p, std::max<size_t>(16, n), st));
    return p;
  }
  void unstage(void* p, hipStream_t st) {
    if (ualloc) {
      HIPCHK(hipStreamSynchronize(st));
      ufree(p, uctx);
      return;
    }
    HIPCHK(hipFreeAsync(p, st));   // stream-ordered: no device-wide synchronisation
  }
  ~DevHier() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (capst) (void)hipStreamDestroy(capst);
    for (hipEvent_t e : evpool) (void)hipEventDestroy(e);
    for (void* p : allocs) {
      if (ufree) ufree(p, uctx);
      else (void)hipFree(p);
    }
    if (hscal) (void)hipHostFree(hscal);
    if (hbscal) (void)hipHostFree(hbscal);
  }
};

}  // namespace
}  // namespace ldgmg

struct ldgmg_hier {
  std::unique_ptr<ldgmg::HostHierarchy> host;
  std::unique_ptr<ldgmg::DevHier> dev;
  bool cg_guard = false;            // ldgmg_cg_guard
  bool fp32_products = false;       // ldgmg_fp32_products
  double rhs_check = 0.0;           // ldgmg_rhs_check tolerance (0: off)
  int graph_every = 0;              // ldgmg_cg_graph: replays between host checks (0: eager CG)
  int gen = 0;                      // bumped by every setting a captured graph depends on
};

namespace ldgmg {
namespace {

enum { S_BB = 0, S_RZ = 1, S_ALPHA = 2, S_RR = 3, S_BETA = 4, S_PQ = 5, S_TMP = 6, S_W = 7, S_K = 8 };
static_assert(kScalFrozen > S_K && kScalRRFinal < 64, "graph CG slots follow the others in the 64-entry table");
constexpr int kGraphHist = 4096;   // residual history entries of a replayed CG solve

// bytes per stored entry of the operators A and of the smoother S
size_t elem_bytes_A(int prec) { return prec == LDGMG_FP64 ? 8 : 4; }
size_t elem_bytes_S(int prec) { return prec == LDGMG_FP64 ? 8 : prec == LDGMG_BF16S ? 2 : 4; }

// pooled storage of one matrix with elements of `elem` bytes (LDGMG_STORE_*)
bool use_pool(const PMat& P, int bs, size_t elem, int storage) {
  if (!fast_bs(bs) || storage == LDGMG_STORE_EXPANDED) return false;
  if (storage == LDGMG_STORE_POOLED || storage == LDGMG_STORE_TILED) return true;
  const size_t bb = static_cast<size_t>(bs) * bs * elem;
  const size_t pool = static_cast<size_t>(P.pool.size()) * bb;
  return pool <= (static_cast<size_t>(64) << 20) && 4 * pool <= static_cast<size_t>(P.nnzb()) * bb;
}

// distinct column offsets (column - row) of a block-sparse matrix, ascending
std::vector<int> column_offsets(const PMat& P) {
  std::vector<int> o;
  for (int i = 0; i + 1 < static_cast<int>(P.rp.size()); ++i)
    for (int s2 = P.rp[i]; s2 < P.rp[i + 1]; ++s2) o.push_back(P.ci[s2] - i);
  std::sort(o.begin(), o.end());
  o.erase(std::unique(o.begin(), o.end()), o.end());
  return o;
}

constexpr int kMaxTiledOffsets = 64;
constexpr int kMinTiledRows = 4096;       // 256 tiles; below 1024 tiles the kernel takes a wavefront per row tile
constexpr double kMaxTiledPasses = 1.5;   // mean MFMA passes per tile and offset

// pool-id table [row][offset] of a matrix and its rows ordered by table row
// (stable, so that rows with equal blocks at every offset are side by side)
void tiled_table(const PMat& P, const std::vector<int>& off, std::vector<int>& tab, std::vector<int>& perm) {
  const int noff = static_cast<int>(off.size());
  tab.assign(static_cast<size_t>(P.nbr) * noff, -1);
  for (int i = 0; i < P.nbr; ++i)
    for (int s2 = P.rp[i]; s2 < P.rp[i + 1]; ++s2) {
      const int d = static_cast<int>(std::lower_bound(off.begin(), off.end(), P.ci[s2] - i) - off.begin());
      tab[static_cast<size_t>(i) * noff + d] = P.id[s2];
    }
  perm.resize(P.nbr);
  for (int i = 0; i < P.nbr; ++i) perm[i] = i;
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) {
    return std::lexicographical_compare(tab.begin() + static_cast<size_t>(a) * noff,
                                        tab.begin() + static_cast<size_t>(a + 1) * noff,
                                        tab.begin() + static_cast<size_t>(b) * noff,
                                        tab.begin() + static_cast<size_t>(b + 1) * noff);
  });
}

// the tile order of the tiled kernel: the rows ordered by table row, each
// group of equal table rows starting a 16-row tile (-1 pads the tile before
// it) when that costs at most a quarter more places.  In a padded order a
// tile holds one table row, so one MFMA pass per offset: no tile takes longer
// than the others, which matters where there are few tiles per SIMD.
constexpr double kMaxPadding = 1.25;
void tiled_order(const PMat& P, const std::vector<int>& off, std::vector<int>& tab, std::vector<int>& perm,
                 std::vector<int>* rows = nullptr) {
  tiled_table(P, off, tab, perm);
  if (rows) *rows = perm;
  const int noff = static_cast<int>(off.size());
  std::vector<int> pad;
  pad.reserve(perm.size() + perm.size() / 4 + 16);
  for (size_t e = 0; e < perm.size(); ++e) {
    const bool start = e == 0 || !std::equal(tab.begin() + static_cast<size_t>(perm[e]) * noff,
                                             tab.begin() + static_cast<size_t>(perm[e] + 1) * noff,
                                             tab.begin() + static_cast<size_t>(perm[e - 1]) * noff);
    if (start)
      while (pad.size() % 16) pad.push_back(-1);
    pad.push_back(perm[e]);
  }
  if (static_cast<double>(pad.size()) <= kMaxPadding * static_cast<double>(perm.size())) perm.swap(pad);
}

// mean number of MFMA passes (distinct blocks) per 16-row tile and offset in
// the tile order (and that order's length, both cached in P)
double tiled_passes(const PMat& P) {
  if (P.tile_passes >= 0.0) return P.tile_passes;
  const std::vector<int> off = column_offsets(P);
  std::vector<int> tab, perm;
  tiled_order(P, off, tab, perm);
  const int noff = static_cast<int>(off.size());
  const int np = static_cast<int>(perm.size());
  long long passes = 0, slots = 0;
  std::vector<int> ids;
  for (int t0 = 0; t0 < np; t0 += 16)
    for (int d = 0; d < noff; ++d) {
      ids.clear();
      for (int c = t0; c < std::min(np, t0 + 16); ++c) {
        if (perm[c] < 0) continue;
        const int v = tab[static_cast<size_t>(perm[c]) * noff + d];
        if (v >= 0) ids.push_back(v);
      }
      std::sort(ids.begin(), ids.end());
      passes += std::unique(ids.begin(), ids.end()) - ids.begin();
      slots += 1;
    }
  P.tile_passes = slots ? static_cast<double>(passes) / slots : 0.0;
  P.tile_perm_len = np;
  return P.tile_passes;
}

int tiled_perm_len(const PMat& P) {
  tiled_passes(P);
  return P.tile_perm_len;
}

// tiled storage (on top of pooled) for a matrix: TILED; or AUTO when pooled,
// large enough to fill the device and with few distinct blocks per tile
bool use_tiled(const PMat& P, int bs, size_t elem, int storage) {
  if (storage != LDGMG_STORE_TILED && storage != LDGMG_STORE_AUTO) return false;
  if (!use_pool(P, bs, elem, storage)) return false;
  if (static_cast<int>(column_offsets(P).size()) > kMaxTiledOffsets) return false;
  if (storage == LDGMG_STORE_TILED) return true;
  return P.nbr >= kMinTiledRows && tiled_passes(P) <= kMaxTiledPasses;
}

// device bytes of one matrix's blocks (and block ids when pooled, and the
// operand-layout pool and offset table when tiled).  The transposed copy of a
// smoother matrix follows the smoother matrix's choices.
size_t matrix_bytes(const PMat& P, int bs, size_t elem, int storage) {
  const size_t bb = static_cast<size_t>(bs) * bs * elem;
  if (!use_pool(P, bs, elem, storage)) return static_cast<size_t>(P.nnzb()) * bb;
  size_t b = static_cast<size_t>(P.pool.size()) * bb + P.nnzb() * sizeof(int);
  if (use_tiled(P, bs, elem, storage)) {
    const size_t noff = column_offsets(P).size();
    b += static_cast<size_t>(P.pool.size()) * tiled_block_elems(bs) * elem;
    b += static_cast<size_t>(P.nbr) * noff * sizeof(int) + std::max<size_t>(16, noff * sizeof(int));
    b += std::max<size_t>(16, static_cast<size_t>(tiled_perm_len(P)) * sizeof(int));   // tile order
    if (tiled_perm_len(P) != P.nbr) b += std::max<size_t>(16, static_cast<size_t>(P.nbr) * sizeof(int));   // unpadded
  }
  return b;
}

// bytes one level needs on the device in precision prec (expanded storage;
// used before the setup, from the stencil sizes)
size_t level_bytes(int ne, int bs, int bss, int dim, long long nnzA, long long nnzS, bool bottom,
                   bool gs, int prec) {
  const size_t ea = elem_bytes_A(prec), es = elem_bytes_S(prec);
  const size_t N = static_cast<size_t>(ne) * bs;
  size_t b = 0;
  b += (ne + 1) * 4 + nnzA * 4 + nnzA * static_cast<size_t>(bs) * bs * ea;
  if (!bottom) {
    b += (ne + 1) * 4 + nnzS * 8 + nnzS * static_cast<size_t>(bs) * bs * es * (fast_bs(bs) ? 2 : 1);
    if (gs) b += ne * 4;
  } else {
    b += N * N * 8;
  }
  b += 4 * N * 8;
  b += (static_cast<size_t>(1) << dim) * bss * bss * 8 + 2 * 64 * 8;
  return b;
}

// tiled form of a pooled matrix: the pool in the tiled kernel's operand layout
// (transposed blocks if asked), the column offsets and the pool-id table
template <typename T>
void make_tiled(DevHier& D, const PMat& P, int bs, bool transpose, bool quad, Tiled& t, hipStream_t st) {
  const std::vector<int> off = column_offsets(P);
  const int noff = static_cast<int>(off.size());
  // rows with equal blocks at every offset side by side (stable: interior rows
  // keep their grid order), so that a 16-row tile needs one pass per offset
  std::vector<int> tab, perm, rows;
  tiled_order(P, off, tab, perm, &rows);
  const long long nd = P.pool.size();
  T* blk = static_cast<T*>(D.alloc(static_cast<size_t>(nd) * tiled_block_elems(bs) * sizeof(T)));
  t.perm = static_cast<int*>(D.alloc(std::max<size_t>(16, perm.size() * sizeof(int))));
  HIPCHK(hipMemcpyAsync(t.perm, perm.data(), perm.size() * sizeof(int), hipMemcpyHostToDevice, st));
  if (perm.size() != rows.size()) {
    t.rows = static_cast<int*>(D.alloc(std::max<size_t>(16, rows.size() * sizeof(int))));
    HIPCHK(hipMemcpyAsync(t.rows, rows.data(), rows.size() * sizeof(int), hipMemcpyHostToDevice, st));
  } else {
    t.rows = t.perm;
  }
  t.tab = static_cast<int*>(D.alloc(tab.size() * sizeof(int)));
  t.off = static_cast<int*>(D.alloc(std::max<size_t>(16, off.size() * sizeof(int))));
  HIPCHK(hipMemcpyAsync(t.tab, tab.data(), tab.size() * sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(t.off, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice, st));
  double* pool = static_cast<double*>(D.stage(P.pool.data.size() * sizeof(double), st));
  HIPCHK(hipMemcpyAsync(pool, P.pool.data.data(), P.pool.data.size() * sizeof(double), hipMemcpyHostToDevice, st));
  expand_tiled<T>(nd, bs, pool, blk, transpose, quad, st);
  D.unstage(pool, st);
  HIPCHK(hipStreamSynchronize(st));   // the host tables above must outlive their copies
  t.blk = blk;
  t.nperm = static_cast<int>(perm.size());
  t.noff = noff;
  t.quad = quad;
}

template <typename TA, typename TS>   // element types of the stored operator and smoother blocks
// quad_S: the smoother matrix and its transpose take the 4-step k mapping (they
// read the FP32 smoothing residual)
void upload_level(DevHier& D, DevLevel& dl, const HostLevel& hl, bool bottom, bool quad_S, hipStream_t st) {
  dl.n = hl.n;
  dl.ne = hl.ne;
  dl.bs = hl.bs;
  dl.bss = hl.bss;
  dl.ncomp = hl.ncomp;
  dl.N = static_cast<long long>(hl.ne) * hl.bs;
  const size_t bb = static_cast<size_t>(hl.bs) * hl.bs;
  auto up_ints = [&](const std::vector<int>& v) {
    int* p = static_cast<int*>(D.alloc(v.size() * sizeof(int)));
    HIPCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice, st));
    return p;
  };
  const int storage = D.storage;
  // device blocks of type T for a pooled host matrix (transposed blocks if
  // asked): every slot's block (expanded), or the distinct blocks once with
  // the block id of every slot in `bid` (pooled; bid stays null otherwise)
  auto place = [&](auto tag, const PMat& P, bool transpose, int*& bid, Tiled& tiled, bool want_tiled, bool quad) {
    using T = decltype(tag);
    const bool pooled = use_pool(P, hl.bs, sizeof(T), storage);
    if (want_tiled) make_tiled<T>(D, P, hl.bs, transpose, quad, tiled, st);
    const int nd = P.pool.size();
    std::vector<int> order;
    if (pooled) {
      order.resize(nd);
      for (int i = 0; i < nd; ++i) order[i] = i;
    }
    const std::vector<int>& ids_h = pooled ? order : P.id;
    T* out = static_cast<T*>(D.alloc(ids_h.size() * bb * sizeof(T)));
    double* pool = static_cast<double*>(D.stage(P.pool.data.size() * sizeof(double), st));
    int* ids = static_cast<int*>(D.stage(ids_h.size() * sizeof(int), st));
    HIPCHK(hipMemcpyAsync(pool, P.pool.data.data(), P.pool.data.size() * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(ids, ids_h.data(), ids_h.size() * sizeof(int), hipMemcpyHostToDevice, st));
    expand_blocks<T>(static_cast<long long>(ids_h.size()), hl.bs, ids, pool, out, transpose, st);
    D.unstage(pool, st);
    D.unstage(ids, st);
    HIPCHK(hipStreamSynchronize(st));  // the host id list must outlive its copy
    bid = pooled ? up_ints(P.id) : nullptr;
    return out;
  };
  dl.nnzA = hl.A.nnzb();
  dl.rpA = up_ints(hl.A.rp);
  dl.ciA = up_ints(hl.A.ci);
  // where the smoothing reads FP32 vectors (quad_S) the operator reads the FP32 copy of x too: 4-step layout
  dl.valA = place(TA{}, hl.A, false, dl.bidA, dl.tA, use_tiled(hl.A, hl.bs, sizeof(TA), storage), quad_S);
  if (!bottom) {
    dl.nnzS = hl.S.nnzb();
    dl.rpS = up_ints(hl.S.rp);
    dl.ciS = up_ints(hl.S.ci);
    dl.tposS = up_ints(hl.tpos);
    const bool tiled_S = use_tiled(hl.S, hl.bs, sizeof(TS), storage);
    dl.valS = place(TS{}, hl.S, false, dl.bidS, dl.tS, tiled_S, quad_S && tiled_S);
    if (fast_bs(hl.bs)) {   // S^T applies stream a transposed copy through the forward kernel
      PMat st;
      st.nbr = hl.S.nbr;
      st.nbc = hl.S.nbc;
      st.rp = hl.S.rp;
      st.ci = hl.S.ci;
      st.id.resize(hl.S.id.size());
      for (size_t t = 0; t < st.id.size(); ++t) st.id[t] = hl.S.id[hl.tpos[t]];
      st.pool.r = hl.S.pool.r;
      st.pool.c = hl.S.pool.c;
      st.pool.data = hl.S.pool.data;
      dl.valST = place(TS{}, st, true, dl.bidST, dl.tST, tiled_S, quad_S && tiled_S);
    }
    for (const auto& rows : hl.colour_rows) {
      dl.colour_rows.push_back(up_ints(rows));
      dl.colour_count.push_back(static_cast<int>(rows.size()));
    }
  } else {
    dl.pinv = static_cast<double*>(D.alloc(hl.pinv.size() * sizeof(double)));
    HIPCHK(hipMemcpyAsync(dl.pinv, hl.pinv.data(), hl.pinv.size() * sizeof(double), hipMemcpyHostToDevice, st));
  }
  const size_t vb = static_cast<size_t>(dl.N) * sizeof(double);
  dl.x = static_cast<double*>(D.alloc(vb));
  dl.b = static_cast<double*>(D.alloc(vb));
  dl.r = static_cast<double*>(D.alloc(vb));
  dl.t = static_cast<double*>(D.alloc(vb));
  HIPCHK(hipMemsetAsync(dl.x, 0, vb, st));
  HIPCHK(hipMemsetAsync(dl.r, 0, vb, st));
  HIPCHK(hipMemsetAsync(dl.t, 0, vb, st));
  // child injection matrices (the same for every level: they depend on p only)
  const int nch = 1 << hl.em.dim;
  std::vector<double> ic(static_cast<size_t>(nch) * hl.bss * hl.bss);
  for (int c = 0; c < nch; ++c)
    std::copy(hl.em.Ic[c].begin(), hl.em.Ic[c].end(), ic.begin() + static_cast<size_t>(c) * hl.bss * hl.bss);
  dl.Ic = static_cast<double*>(D.alloc(ic.size() * sizeof(double)));
  HIPCHK(hipMemcpyAsync(dl.Ic, ic.data(), ic.size() * sizeof(double), hipMemcpyHostToDevice, st));
  dl.q1 = hl.em.q1;
  std::vector<double> p1(hl.em.P[0]);
  p1.insert(p1.end(), hl.em.P[1].begin(), hl.em.P[1].end());
  dl.P1 = static_cast<double*>(D.alloc(p1.size() * sizeof(double)));
  HIPCHK(hipMemcpyAsync(dl.P1, p1.data(), p1.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
}

// exact device bytes of ldgmg_upload for a host hierarchy (batch workspace excluded)
// levels that keep an FP32 smoothing residual for FP32 products: SAI smoother,
// A and S tiled, 16 | bs
bool fp32_residual_level(const HostHierarchy& H, int l, int prec) {
  const HostLevel& L = H.levels[l];
  const int storage = H.prob.storage;
  return l + 1 < static_cast<int>(H.levels.size()) && prec != LDGMG_FP64 && H.prob.smoother == LDGMG_SMOOTH_SAI &&
         L.bs % 16 == 0 && use_tiled(L.A, L.bs, elem_bytes_A(prec), storage) &&
         use_tiled(L.S, L.bs, elem_bytes_S(prec), storage);
}

std::vector<std::vector<double>> kernel_patterns(const HostHierarchy& H);

size_t estimate_from_host(const HostHierarchy& H, int prec) {
  const int storage = H.prob.storage;
  const size_t ea = elem_bytes_A(prec), es = elem_bytes_S(prec);
  size_t b = 0;
  const int nl = static_cast<int>(H.levels.size());
  for (int l = 0; l < nl; ++l) {
    const HostLevel& L = H.levels[l];
    const size_t N = static_cast<size_t>(L.ne) * L.bs;
    const bool bottom = l == nl - 1;
    b += (L.ne + 1) * 4 + L.A.nnzb() * 4 + matrix_bytes(L.A, L.bs, ea, storage);
    if (!bottom) {
      b += (L.ne + 1) * 4 + L.S.nnzb() * 4 + L.tpos.size() * 4 + matrix_bytes(L.S, L.bs, es, storage);
      if (fast_bs(L.bs)) b += matrix_bytes(L.S, L.bs, es, storage);   // transposed copy
      for (const auto& rows : L.colour_rows) b += std::max<size_t>(16, rows.size() * 4);
    } else {
      b += N * N * 8;
    }
    b += 4 * N * 8;
    if (fp32_residual_level(H, l, prec)) b += N * 8;   // FP32 residual and FP32 copy of x
    b += (static_cast<size_t>(1) << L.em.dim) * L.bss * L.bss * 8 + 2 * L.em.q1 * L.em.q1 * 8;
  }
  const HostLevel& F = H.levels[0];
  const size_t N = static_cast<size_t>(F.ne) * F.bs;
  if (prec != LDGMG_FP64) {
    const size_t bb8 = static_cast<size_t>(F.bs) * F.bs * 8;
    b += use_pool(F.A, F.bs, ea, storage) ? static_cast<size_t>(F.A.pool.size()) * bb8
                                          : static_cast<size_t>(F.A.nnzb()) * bb8;
    if (use_tiled(F.A, F.bs, ea, storage))   // operand-layout pool of the FP64 copy
      b += static_cast<size_t>(F.A.pool.size()) * tiled_block_elems(F.bs) * 8;
  }
  b += 5 * N * 8 + 64 * 8 + kRedBlocks * 8 * 2;
  b += 2 * kernel_patterns(H).size() * N * 8;   // kernel vectors and mean weights (singular operators)
  return b;
}

// Kernel of the fine operator.  Candidates: the constant function in one
// component (the scalar field of a problem with no Dirichlet face, the
// pressure of Stokes, the velocity components of Stokes with no Dirichlet
// face); a candidate k is kept when max_i |(A k)_i| <= 1e-10 max_i (|A| |k|)_i
// in FP64, evaluated per distinct block of the pooled A.  Per element the
// constant's coefficients are c1 (x) c1 (x) c1 with c1 = m^-1 (int psi_i),
// m the 1-D mass matrix.
std::vector<std::vector<double>> kernel_patterns(const HostHierarchy& H) {
  const HostLevel& F = H.levels[0];
  const int d = H.prob.dim, q1 = F.em.q1, bss = F.bss, bs = F.bs;
  bool any_dirichlet = false;
  for (int f = 0; f < 2 * d; ++f) any_dirichlet = any_dirichlet || H.prob.bc[f] == LDGMG_BC_DIRICHLET;
  std::vector<int> comps;
  if (H.prob.system == LDGMG_POISSON) {
    if (!any_dirichlet) comps.push_back(0);
  } else {
    if (!any_dirichlet)
      for (int c = 0; c < d; ++c) comps.push_back(c);
    comps.push_back(d);
  }
  std::vector<std::vector<double>> out;
  if (comps.empty()) return out;
  std::vector<double> t, w, v(q1), dv(q1);
  gauss_legendre(q1 + 1, t, w);
  std::vector<double> m(static_cast<size_t>(q1) * q1, 0.0), c1(q1, 0.0);
  for (size_t q = 0; q < t.size(); ++q) {
    basis_eval(F.em.p, H.prob.basis, t[q], v.data(), dv.data());
    for (int i = 0; i < q1; ++i) {
      c1[i] += w[q] * v[i];
      for (int j = 0; j < q1; ++j) m[static_cast<size_t>(i) * q1 + j] += w[q] * v[i] * v[j];
    }
  }
  // c1 = m^-1 (int psi_i): Gaussian elimination with partial pivoting (q1 <= 6)
  for (int k = 0; k < q1; ++k) {
    int pv = k;
    for (int i = k + 1; i < q1; ++i)
      if (std::fabs(m[static_cast<size_t>(i) * q1 + k]) > std::fabs(m[static_cast<size_t>(pv) * q1 + k])) pv = i;
    for (int j = 0; j < q1; ++j) std::swap(m[static_cast<size_t>(k) * q1 + j], m[static_cast<size_t>(pv) * q1 + j]);
    std::swap(c1[k], c1[pv]);
    for (int i = k + 1; i < q1; ++i) {
      const double f = m[static_cast<size_t>(i) * q1 + k] / m[static_cast<size_t>(k) * q1 + k];
      for (int j = k; j < q1; ++j) m[static_cast<size_t>(i) * q1 + j] -= f * m[static_cast<size_t>(k) * q1 + j];
      c1[i] -= f * c1[k];
    }
  }
  for (int k = q1 - 1; k >= 0; --k) {
    for (int j = k + 1; j < q1; ++j) c1[k] -= m[static_cast<size_t>(k) * q1 + j] * c1[j];
    c1[k] /= m[static_cast<size_t>(k) * q1 + k];
  }
  std::vector<double> cs(bss);
  for (int a = 0; a < bss; ++a) {
    double val = c1[a % q1] * c1[(a / q1) % q1];
    if (d == 3) val *= c1[a / (q1 * q1)];
    cs[a] = val;
  }
  const PMat& A = F.A;
  const int np = A.pool.size();
  for (int comp : comps) {
    std::vector<double> k(bs, 0.0);
    std::copy(cs.begin(), cs.end(), k.begin() + static_cast<size_t>(comp) * bss);
    // per distinct block: B k and |B| |k|
    std::vector<double> bk(static_cast<size_t>(np) * bs), ak(static_cast<size_t>(np) * bs);
    for (int id = 0; id < np; ++id) {
      const double* B = A.pool.at(id);
      for (int r = 0; r < bs; ++r) {
        double s1 = 0.0, s2 = 0.0;
        for (int c = 0; c < bs; ++c) {
          s1 += B[static_cast<size_t>(r) * bs + c] * k[c];
          s2 += std::fabs(B[static_cast<size_t>(r) * bs + c] * k[c]);
        }
        bk[static_cast<size_t>(id) * bs + r] = s1;
        ak[static_cast<size_t>(id) * bs + r] = s2;
      }
    }
    double worst = 0.0, scale = 0.0;
    std::vector<double> s1(bs), s2(bs);
    for (int i = 0; i < A.nbr; ++i) {
      std::fill(s1.begin(), s1.end(), 0.0);
      std::fill(s2.begin(), s2.end(), 0.0);
      for (int sl = A.rp[i]; sl < A.rp[i + 1]; ++sl)
        for (int r = 0; r < bs; ++r) {
          s1[r] += bk[static_cast<size_t>(A.id[sl]) * bs + r];
          s2[r] += ak[static_cast<size_t>(A.id[sl]) * bs + r];
        }
      for (int r = 0; r < bs; ++r) {
        worst = std::max(worst, std::fabs(s1[r]));
        scale = std::max(scale, s2[r]);
      }
    }
    if (worst <= 1e-10 * scale) out.push_back(k);
  }
  return out;
}

// the kernel vectors of the fine operator on the device: khat_i = k_i / ||k_i||
// and the mean weights w_i = M khat_i / (khat_i^T M khat_i), so that
// (w_i . x) khat_i is the M-orthogonal projection of x on khat_i
void upload_kernel(DevHier& D, const HostHierarchy& H, hipStream_t st) {
  const std::vector<std::vector<double>> pats = kernel_patterns(H);
  D.nker = static_cast<int>(pats.size());
  if (!D.nker) return;
  const HostLevel& F = H.levels[0];
  const long long N = static_cast<long long>(F.ne) * F.bs;
  const int bs = F.bs, bss = F.bss;
  std::vector<double> kh(static_cast<size_t>(D.nker) * N), kw(static_cast<size_t>(D.nker) * N);
  for (int i = 0; i < D.nker; ++i) {
    const std::vector<double>& k = pats[i];
    std::vector<double> mk(bs, 0.0);          // element mass applied per component block
    for (int c = 0; c < bs / bss; ++c)
      for (int a = 0; a < bss; ++a)
        for (int b = 0; b < bss; ++b)
          mk[c * bss + a] += F.em.M[static_cast<size_t>(a) * bss + b] * k[c * bss + b];
    double kk = 0.0, kmk = 0.0;
    for (int a = 0; a < bs; ++a) {
      kk += k[a] * k[a];
      kmk += k[a] * mk[a];
    }
    const double nrm = std::sqrt(kk * F.ne);   // ||k|| over the grid
    const double den = kmk / kk;               // khat^T M khat
    for (long long e = 0; e < F.ne; ++e)
      for (int a = 0; a < bs; ++a) {
        kh[static_cast<size_t>(i) * N + e * bs + a] = k[a] / nrm;
        kw[static_cast<size_t>(i) * N + e * bs + a] = mk[a] / nrm / den;
      }
  }
  D.khat = static_cast<double*>(D.alloc(kh.size() * sizeof(double)));
  D.kw = static_cast<double*>(D.alloc(kw.size() * sizeof(double)));
  HIPCHK(hipMemcpyAsync(D.khat, kh.data(), kh.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(D.kw, kw.data(), kw.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));   // the host vectors must outlive their copies
}

void upload(ldgmg_hier* h, hipStream_t st) {
  const HostHierarchy& H = *h->host;
  const size_t need = estimate_from_host(H, H.prob.precision);
  if (H.prob.hbm_budget && need > H.prob.hbm_budget)
    throw BudgetError("hierarchy needs " + std::to_string(need) + " bytes, over the HBM budget of " +
                      std::to_string(H.prob.hbm_budget));
  auto D = std::make_unique<DevHier>();
  D->prec = H.prob.precision;
  D->storage = H.prob.storage;
  D->ualloc = H.prob.dev_alloc;
  D->ufree = H.prob.dev_free;
  D->uctx = H.prob.alloc_ctx;
  HIPCHK(hipGetDevice(&D->device));
  const int nl = static_cast<int>(H.levels.size());
  D->L.resize(nl);
  for (int l = 0; l < nl; ++l) {
    D->L[l].index = l;
    if (D->prec == LDGMG_FP64)
      upload_level<double, double>(*D, D->L[l], H.levels[l], l == nl - 1, fp32_residual_level(H, l, D->prec), st);
    else if (D->prec == LDGMG_BF16S)
      upload_level<float, bf16s>(*D, D->L[l], H.levels[l], l == nl - 1, fp32_residual_level(H, l, D->prec), st);
    else
      upload_level<float, float>(*D, D->L[l], H.levels[l], l == nl - 1, fp32_residual_level(H, l, D->prec), st);
    if (fp32_residual_level(H, l, D->prec)) {
      if (!D->L[l].tA.tab || !D->L[l].tS.tab) throw std::logic_error("tiled storage differs from its estimate");
      D->L[l].r32 = static_cast<float*>(D->alloc(static_cast<size_t>(D->L[l].N) * sizeof(float)));
      D->L[l].x32 = static_cast<float*>(D->alloc(static_cast<size_t>(D->L[l].N) * sizeof(float)));
    }
  }
  const HostLevel& F = H.levels[0];
  DevLevel& f = D->L[0];
  if (D->prec == LDGMG_FP64) {
    D->val64 = static_cast<double*>(f.valA);
    D->bid64 = f.bidA;
    D->t64 = f.tA;
  } else {
    // the FP64 operator of the Krylov iteration follows the storage of A: the
    // distinct blocks (sharing A's block ids) when A is pooled
    const size_t bb = static_cast<size_t>(F.bs) * F.bs;
    std::vector<int> order;
    if (f.bidA) {
      order.resize(F.A.pool.size());
      for (size_t i = 0; i < order.size(); ++i) order[i] = static_cast<int>(i);
    }
    const std::vector<int>& ids_h = f.bidA ? order : F.A.id;
    D->val64 = static_cast<double*>(D->alloc(ids_h.size() * bb * sizeof(double)));
    D->bid64 = f.bidA;
    double* pool = static_cast<double*>(D->stage(F.A.pool.data.size() * sizeof(double), st));
    int* ids = static_cast<int*>(D->stage(ids_h.size() * sizeof(int), st));
    HIPCHK(hipMemcpyAsync(pool, F.A.pool.data.data(), F.A.pool.data.size() * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(ids, ids_h.data(), ids_h.size() * sizeof(int), hipMemcpyHostToDevice, st));
    expand_blocks<double>(static_cast<long long>(ids_h.size()), F.bs, ids, pool, D->val64, false, st);
    if (f.tA.tab) {                         // tiled A: the FP64 copy gets its own operand-layout pool
      const long long nd = F.A.pool.size();
      double* tb = static_cast<double*>(D->alloc(static_cast<size_t>(nd) * tiled_block_elems(F.bs) * sizeof(double)));
      expand_tiled<double>(nd, F.bs, pool, tb, false, false, st);
      D->t64 = f.tA;
      D->t64.blk = tb;
      D->t64.quad = false;                  // the 2-step k layout (FP64 x), whatever A's own
    }
    D->unstage(pool, st);
    D->unstage(ids, st);
    HIPCHK(hipStreamSynchronize(st));
    D->own64 = true;
  }
  const size_t vb = static_cast<size_t>(f.N) * sizeof(double);
  D->kx = static_cast<double*>(D->alloc(vb));
  D->kr = static_cast<double*>(D->alloc(vb));
  D->kp = static_cast<double*>(D->alloc(vb));
  D->kq = static_cast<double*>(D->alloc(vb));
  D->kz = static_cast<double*>(D->alloc(vb));
  D->scal = static_cast<double*>(D->alloc(64 * sizeof(double)));
  D->partial = static_cast<double*>(D->alloc(static_cast<size_t>(kRedBlocks) * 2 * sizeof(double)));
  HIPCHK(hipMemsetAsync(D->scal, 0, 64 * sizeof(double), st));
  HIPCHK(hipHostMalloc(&D->hscal, 64 * sizeof(double), hipHostMallocDefault));
  HIPCHK(hipStreamSynchronize(st));
  upload_kernel(*D, H, st);
  for (DevLevel& L : D->L) L.p32 = h->fp32_products;
  h->dev = std::move(D);
}

// ---------------------------------------------------------------------------
// level operations
// ---------------------------------------------------------------------------
struct Ctx {
  const HostHierarchy& H;
  DevHier& D;
  hipStream_t st;
  bool guard = false;               // CG stops at a breakdown (ldgmg_cg_guard)
};

// brackets one launch on level 0 with events when profiling is enabled
struct ProfScope {
  DevHier& D;
  hipStream_t st;
  int kind;
  hipEvent_t b = nullptr;
  ProfScope(DevHier& d, const DevLevel& L, hipStream_t s, int k) : D(d), st(s), kind(k) {
    if (!D.prof || L.index != 0 || D.recs.size() * 2 + 2 > D.evpool.size()) return;
    hipEvent_t a = D.evpool[D.recs.size() * 2];
    b = D.evpool[D.recs.size() * 2 + 1];
    HIPCHK(hipEventRecord(a, st));
    D.recs.push_back({kind, a, b});
  }
  ~ProfScope() {
    if (b) (void)hipEventRecord(b, st);
  }
};
enum { K_A = 0, K_SF = 1, K_ST = 2, K_A64 = 3, K_FUSED = 4 };

using Vd = double;   // vector / arithmetic type of the V-cycle

template <typename T>
void set_tiled(BsrArgs<T, Vd>& a, const Tiled& t) {
  a.tblk = static_cast<const T*>(t.blk);
  a.tab = t.tab;
  a.tperm = t.perm;
  a.toff = t.off;
  a.noff = t.noff;
  a.tnrows = t.nperm;
  a.trows = t.rows;
  a.tquad = t.quad;
}

template <typename T>
BsrArgs<T, Vd> argsA(const DevLevel& L) {
  BsrArgs<T, Vd> a;
  a.nrows = L.ne;
  a.bs = L.bs;
  a.rp = L.rpA;
  a.ci = L.ciA;
  a.bid = L.bidA;
  a.blk = static_cast<const T*>(L.valA);
  set_tiled(a, L.tA);
  a.p32 = L.p32;
  a.tpair = true;
  return a;
}
template <typename T>
BsrArgs<T, Vd> argsS(const DevLevel& L) {
  BsrArgs<T, Vd> a;
  a.nrows = L.ne;
  a.bs = L.bs;
  a.rp = L.rpS;
  a.ci = L.ciS;
  a.tpos = L.tposS;
  a.bid = L.bidS;
  a.blk = static_cast<const T*>(L.valS);
  set_tiled(a, L.tS);
  a.p32 = L.p32;
  return a;
}

// out = b - A x (or, given out32, the same rounded to FP32 into out32 only);
// x32 (optional): FP32 x read in place of x (FP32 products: the same operands)
template <typename T>
void residual(const DevLevel& L, const Vd* x, const Vd* b, Vd* out, hipStream_t st, float* out32 = nullptr,
              const float* x32 = nullptr) {
  BsrArgs<T, Vd> a = argsA<T>(L);
  a.x = x32 ? nullptr : x;
  a.x32 = x32;
  a.z = b;
  a.out = out32 ? nullptr : out;
  a.out32 = out32;
  a.alpha = -1.0;
  a.beta = 1.0;
  bsr_forward<T, Vd>(a, st);
}

template <typename T>
void residual(DevHier& D, const DevLevel& L, const Vd* x, const Vd* b, Vd* out, hipStream_t st,
              float* out32 = nullptr, const float* x32 = nullptr) {
  ProfScope ps(D, L, st, K_A);
  residual<T>(L, x, b, out, st, out32, x32);
}

// out = alpha S x + beta z   (transposed: S^T); out2 (optional, tiled): an FP32 copy of out
template <typename T>
void apply_S(const DevLevel& L, bool transposed, const Vd* x, const Vd* z, Vd* out, Vd alpha, Vd beta,
             hipStream_t st, const float* x32 = nullptr, float* out2 = nullptr) {
  BsrArgs<T, Vd> a = argsS<T>(L);
  a.x = x32 ? nullptr : x;
  a.x32 = x32;
  a.z = z;
  a.out = out;
  a.out2 = out2;
  a.alpha = alpha;
  a.beta = beta;
  if (transposed && L.valST) {
    a.blk = static_cast<const T*>(L.valST);
    a.bid = L.bidST;
    set_tiled(a, L.tST);
    bsr_forward<T, Vd>(a, st);
  } else if (transposed) {
    bsr_transposed<T, Vd>(a, st);
  } else {
    bsr_forward<T, Vd>(a, st);
  }
}

template <typename T>
void apply_S(DevHier& D, const DevLevel& L, bool transposed, const Vd* x, const Vd* z, Vd* out, Vd alpha,
             Vd beta, hipStream_t st, const float* x32 = nullptr, float* out2 = nullptr) {
  ProfScope ps(D, L, st, transposed ? K_ST : K_SF);
  apply_S<T>(L, transposed, x, z, out, alpha, beta, st, x32, out2);
}

// one smoothing step on level L with x (in/out), b.  `zero_x`: x is known to be 0.
// Uses L.r / L.t as scratch.  Returns the buffer holding the result (x or t).
// T: operator blocks, TS: smoother blocks (the block inverses of Jacobi and
// Gauss-Seidel share the operator's type)
template <typename T, typename TS>
Vd* smooth_step(const Ctx& c, DevLevel& L, Vd* x, const Vd* b, bool forward, bool zero_x) {
  const int sm = c.H.prob.smoother;
  const Vd omega = c.H.omega;
  Vd* r = L.r;
  Vd* t = L.t;
  if (sm == LDGMG_SMOOTH_SAI) {
    // with FP32 products the applies round their vector operand to FP32
    // anyway: the residual is written in FP32 only and read as such, and the
    // producers of x keep its FP32 copy for the operator applies
    float* r32 = L.p32 ? L.r32 : nullptr;
    float* x32 = L.p32 ? L.x32 : nullptr;
    if (zero_x) {             // x = S b  (eq:B1) or S^T b (eq:BT) from x = 0
      apply_S<TS>(c.D, L, !forward, b, nullptr, x, 1.0, 0.0, c.st, nullptr, x32);
      return x;
    }
    residual<T>(c.D, L, x, b, r, c.st, r32, x32);
    apply_S<TS>(c.D, L, !forward, r, x, x, 1.0, 1.0, c.st, r32, x32);
    return x;
  }
  if (sm == LDGMG_SMOOTH_JACOBI) {
    if (zero_x) {             // x = w D^-1 b
      apply_S<T>(c.D, L, false, b, nullptr, x, omega, 0.0, c.st);
      return x;
    }
    if (fast_bs(L.bs)) {      // t = x + w D^-1 (b - A x)
      BsrArgs<T, Vd> a = argsA<T>(L);
      a.x = x;
      a.z = b;
      a.out = t;
      a.dinv = static_cast<const T*>(L.valS);
      a.dbid = L.bidS;        // D^-1 is block diagonal: slot = row
      a.omega = omega;
      ProfScope ps(c.D, L, c.st, K_FUSED);
      bsr_forward<T, Vd>(a, c.st);
      return t;
    }
    residual<T>(c.D, L, x, b, r, c.st);
    apply_S<T>(c.D, L, false, r, x, x, omega, 1.0, c.st);
    return x;
  }
  // multi-coloured Gauss-Seidel: colours in order (forward) or reversed
  if (zero_x) fill_zero(x, L.N, c.st);     // a kernel, not a memset: the V-cycle may be captured in a graph
  const int nc = static_cast<int>(L.colour_rows.size());
  for (int k = 0; k < nc; ++k) {
    const int col = forward ? k : nc - 1 - k;
    if (fast_bs(L.bs)) {
      BsrArgs<T, Vd> a = argsA<T>(L);
      a.nrows = L.colour_count[col];
      a.rows = L.colour_rows[col];
      a.x = x;
      a.z = b;
      a.out = x;              // in place: rows of one colour are not coupled
      a.dinv = static_cast<const T*>(L.valS);
      a.dbid = L.bidS;
      a.omega = omega;
      ProfScope ps(c.D, L, c.st, K_FUSED);
      bsr_forward<T, Vd>(a, c.st);
    } else {
      BsrArgs<T, Vd> a = argsA<T>(L);
      a.nrows = L.colour_count[col];
      a.rows = L.colour_rows[col];
      a.x = x;
      a.z = b;
      a.out = r;
      a.alpha = -1.0;
      a.beta = 1.0;
      bsr_forward<T, Vd>(a, c.st);
      BsrArgs<T, Vd> s = argsS<T>(L);
      s.nrows = L.colour_count[col];
      s.rows = L.colour_rows[col];
      s.x = r;
      s.z = x;
      s.out = x;
      s.alpha = omega;
      s.beta = 1.0;
      bsr_forward<T, Vd>(s, c.st);
    }
  }
  return x;
}

int order_pre_forward(int order) { return order == LDGMG_ORDER_OO || order == LDGMG_ORDER_OI; }
int order_post_forward(int order) { return order == LDGMG_ORDER_OO || order == LDGMG_ORDER_IO; }

// x_l = V(E_l, 0, b_l) with b_l in L[l].b, result in L[l].x   (Algorithm 1)
template <typename T, typename TS>
void vcycle_level(const Ctx& c, int l) {
  DevLevel& L = c.D.L[l];
  const int nl = static_cast<int>(c.D.L.size());
  Vd* x = L.x;
  const Vd* b = L.b;
  if (l == nl - 1) {
    dense_gemv<Vd>(static_cast<int>(L.N), L.pinv, b, x, c.st);
    return;
  }
  const ldgmg_problem& P = c.H.prob;
  const bool pre_fwd = order_pre_forward(P.order), post_fwd = order_post_forward(P.order);
  auto keep = [&](Vd* res) {
    if (res != x) {             // Jacobi wrote into t: swap the roles of x and t
      std::swap(L.x, L.t);
      x = L.x;
    }
  };
  // the FP32 copy of x (SAI smoothing with FP32 products) follows x through the cycle
  float* x32 = P.smoother == LDGMG_SMOOTH_SAI && L.p32 ? L.x32 : nullptr;
  if (P.nu1 == 0) {
    fill_zero(x, L.N, c.st);
    if (x32) fill_zero(x32, L.N, c.st);
  }
  for (int s = 0; s < P.nu1; ++s) keep(smooth_step<T, TS>(c, L, x, b, pre_fwd, s == 0));
  residual<T>(c.D, L, x, b, L.r, c.st, nullptr, x32);
  DevLevel& Lc = c.D.L[l + 1];
  restrict_op<Vd>(P.dim, Lc.n, L.ncomp, L.bss, Lc.q1, Lc.P1, Lc.Ic, L.r, Lc.b, c.st);
  vcycle_level<T, TS>(c, l + 1);
  prolong_add<Vd>(P.dim, Lc.n, L.ncomp, L.bss, Lc.q1, Lc.P1, Lc.Ic, Lc.x, x, c.st, x32);
  for (int s = 0; s < P.nu2; ++s) keep(smooth_step<T, TS>(c, L, x, b, post_fwd, false));
}

// z = V r (FP64 vectors in and out; the stored blocks are FP32 or FP64)
void vcycle64(const Ctx& c, const double* r, double* z) {
  DevLevel& L = c.D.L[0];
  const size_t n = static_cast<size_t>(L.N);
  // the fine level reads r and writes z in place unless the two overlap
  const bool direct = r + n <= z || z + n <= r;
  double* const b0 = L.b;
  double* const x0 = L.x;
  double* const t0 = L.t;
  if (direct) {
    L.b = const_cast<double*>(r);         // read only
    L.x = z;
  } else {
    HIPCHK(hipMemcpyAsync(L.b, r, n * 8, hipMemcpyDeviceToDevice, c.st));
  }
  if (c.D.prec == LDGMG_FP64) vcycle_level<double, double>(c, 0);
  else if (c.D.prec == LDGMG_BF16S) vcycle_level<float, bf16s>(c, 0);
  else vcycle_level<float, float>(c, 0);
  // Jacobi smoothing swaps the roles of x and t: the result is in L.x
  if (L.x != z) HIPCHK(hipMemcpyAsync(z, L.x, n * 8, hipMemcpyDeviceToDevice, c.st));
  L.b = b0;
  L.x = x0;
  L.t = t0;
}

void apply_A64(const Ctx& c, const double* x, double* y) {
  const DevLevel& L = c.D.L[0];
  BsrArgs<double, double> a;
  a.nrows = L.ne;
  a.bs = L.bs;
  a.rp = L.rpA;
  a.ci = L.ciA;
  a.blk = c.D.val64;
  a.bid = c.D.bid64;
  set_tiled(a, c.D.t64);
  a.x = x;
  a.out = y;
  ProfScope ps(c.D, L, c.st, K_A64);
  bsr_forward<double, double>(a, c.st);
}

double dot_host(const Ctx& c, const double* a, const double* b, int slot) {
  dot_partial(c.D.L[0].N, a, b, c.D.partial, c.st);
  finalize(c.D.partial, c.D.scal, 0, slot, 0, c.st);
  HIPCHK(hipMemcpyAsync(c.D.hscal, c.D.scal, 64 * sizeof(double), hipMemcpyDeviceToHost, c.st));
  HIPCHK(hipStreamSynchronize(c.st));
  return c.D.hscal[slot];
}

double eta_from(const std::vector<double>& hist) {
  std::vector<double> y;
  for (double v : hist)
    if (v > 0) y.push_back(std::log10(v));
  const int n = static_cast<int>(y.size());
  if (n < 2) return NAN;
  double sx = 0, sy = 0, sxx = 0, sxy = 0;
  for (int k = 0; k < n; ++k) {
    sx += k;
    sy += y[k];
    sxx += static_cast<double>(k) * k;
    sxy += k * y[k];
  }
  const double slope = (n * sxy - sx * sy) / (n * sxx - sx * sx);
  if (slope >= 0) return INFINITY;
  return -1.0 / slope;
}

void finish_info(const Ctx& c, const double* b, double* x, double bnorm2, const std::vector<double>& hist,
                 int iters, bool conv, double krylov_rel, int vcycles, ldgmg_info* info) {
  if (!info) return;
  apply_A64(c, x, c.D.kq);
  axpby(c.D.L[0].N, b, c.D.kq, c.D.scal, -1, 1.0, -1, -1.0, c.st);   // kq = b - A x
  const double rr = dot_host(c, c.D.kq, c.D.kq, S_TMP);
  info->iters = iters;
  info->converged = conv ? 1 : 0;
  info->rel_res_true = bnorm2 > 0 ? std::sqrt(rr / bnorm2) : 0.0;
  info->rel_res_krylov = krylov_rel;
  info->eta = eta_from(hist);
  info->vcycles = vcycles;
  info->history_len = 0;
  if (info->history && info->history_cap > 0) {
    const int n = std::min(info->history_cap, static_cast<int>(hist.size()));
    for (int i = 0; i < n; ++i) info->history[i] = hist[i];
    info->history_len = n;
  }
}

// preconditioned CG (Hestenes-Stiefel), x0 = 0, z = V r
int solve_cg(const Ctx& c, const double* b, double* x, double rtol, int maxit, ldgmg_info* info) {
  DevHier& D = c.D;
  const long long N = D.L[0].N;
  HIPCHK(hipMemsetAsync(x, 0, N * 8, c.st));
  HIPCHK(hipMemcpyAsync(D.kr, b, N * 8, hipMemcpyDeviceToDevice, c.st));
  const double bb = dot_host(c, b, b, S_BB);
  if (!std::isfinite(bb)) throw std::invalid_argument("right-hand side contains NaN or Inf");
  std::vector<double> hist;
  if (bb == 0.0) {
    finish_info(c, b, x, bb, hist, 0, true, 0.0, 0, info);
    return LDGMG_OK;
  }
  const double tol2 = rtol * rtol * bb;
  vcycle64(c, D.kr, D.kz);
  int vcycles = 1;
  dot_partial(N, D.kr, D.kz, D.partial, c.st);
  finalize(D.partial, D.scal, 0, S_RZ, 0, c.st);
  HIPCHK(hipMemcpyAsync(D.kp, D.kz, N * 8, hipMemcpyDeviceToDevice, c.st));
  int it = 0;
  bool conv = false;
  double rr = bb;
  while (it < maxit) {
    apply_A64(c, D.kp, D.kq);
    dot_partial(N, D.kp, D.kq, D.partial, c.st);
    finalize(D.partial, D.scal, 1, S_ALPHA, S_RZ, c.st);          // alpha = rz / (p.q)
    cg_update(N, x, D.kr, D.kp, D.kq, D.scal, S_ALPHA, D.partial, c.st);
    finalize(D.partial, D.scal, 0, S_RR, 0, c.st);
    HIPCHK(hipMemcpyAsync(D.hscal, D.scal, 64 * sizeof(double), hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipStreamSynchronize(c.st));
    hist.push_back(std::sqrt(std::fabs(D.hscal[S_RZ])));
    ++it;
    rr = D.hscal[S_RR];
    if (!std::isfinite(rr)) throw std::runtime_error("CG breakdown (non-finite residual)");
    if (rr <= tol2) {
      conv = true;
      break;
    }
    // guarded: r^T V r <= 0 or p^T A p <= 0 shows that the preconditioner (or A)
    // is not positive definite on the Krylov space; stop unconverged
    if (c.guard && (!(D.hscal[S_RZ] > 0.0) || !(D.hscal[S_ALPHA] > 0.0))) break;
    vcycle64(c, D.kr, D.kz);
    ++vcycles;
    dot_partial(N, D.kr, D.kz, D.partial, c.st);
    finalize(D.partial, D.scal, 2, S_BETA, S_RZ, c.st);           // beta = rz_new / rz; rz = rz_new
    cg_dir(N, D.kp, D.kz, D.scal, S_BETA, c.st);
  }
  finish_info(c, b, x, bb, hist, it, conv, std::sqrt(rr / bb), vcycles, info);
  return conv ? LDGMG_OK : LDGMG_ENOCONV;
}

// The CG iteration of solve_cg (q = A p, alpha, x and r updates, r.r, the
// convergence test, z = V r, beta, p = z + beta p) captured once in a graph
// and replayed `every` times between host checks.  The test runs on the
// device: once it stops the recurrence (convergence, iteration limit,
// breakdown, guarded stop) alpha is 0, so the replays left in the batch leave
// x and r unchanged.  The first direction p = z comes from p = 0 and any
// finite beta, so every iteration is the same graph.  The results (iterations,
// x, history) are those of solve_cg; the replays after the stop cost device
// time only.  Used for right-hand sides whose solves are launch-bound.
int solve_cg_graph(ldgmg_hier* h, const Ctx& c, const double* b, double* x, double rtol, int maxit,
                   ldgmg_info* info) {
  DevHier& D = c.D;
  const long long N = D.L[0].N;
  double* xi = D.kx;                        // the graph's x: the caller's x changes between solves
  fill_zero(xi, N, c.st);
  HIPCHK(hipMemcpyAsync(D.kr, b, N * 8, hipMemcpyDeviceToDevice, c.st));
  const double bb = dot_host(c, b, b, S_BB);
  if (!std::isfinite(bb)) throw std::invalid_argument("right-hand side contains NaN or Inf");
  std::vector<double> hist;
  if (bb == 0.0) {
    HIPCHK(hipMemsetAsync(x, 0, N * 8, c.st));
    finish_info(c, b, x, bb, hist, 0, true, 0.0, 0, info);
    return LDGMG_OK;
  }
  const double tol2 = rtol * rtol * bb;
  vcycle64(c, D.kr, D.kz);
  dot_partial(N, D.kr, D.kz, D.partial, c.st);
  finalize(D.partial, D.scal, 0, S_RZ, 0, c.st);
  fill_zero(D.kp, N, c.st);                 // p = z + 0 p on the first replay
  cg_init(D.scal, tol2, maxit, c.st);
  if (!D.ghist) D.ghist = static_cast<double*>(D.alloc(kGraphHist * sizeof(double)));
  if (!D.gexec || D.ggen != h->gen) {
    if (D.gexec) HIPCHK(hipGraphExecDestroy(D.gexec));
    if (D.graph) HIPCHK(hipGraphDestroy(D.graph));
    D.gexec = nullptr;
    D.graph = nullptr;
    if (!D.capst) HIPCHK(hipStreamCreateWithFlags(&D.capst, hipStreamNonBlocking));
    Ctx cc{c.H, D, D.capst, c.guard};
    HIPCHK(hipStreamBeginCapture(D.capst, hipStreamCaptureModeRelaxed));
    try {
      // beta = rz_new / rz from the r.z partials of the previous replay (of
      // the prologue on the first, where beta is 0)
      finalize(D.partial, D.scal, 5, S_BETA, S_RZ, cc.st);
      cg_dir(N, D.kp, D.kz, D.scal, S_BETA, cc.st);
      apply_A64(cc, D.kp, D.kq);
      dot_partial(N, D.kp, D.kq, D.partial, cc.st);
      finalize(D.partial, D.scal, 4, S_ALPHA, S_RZ, cc.st);        // alpha = rz / (p.q), 0 once stopped
      cg_update(N, xi, D.kr, D.kp, D.kq, D.scal, S_ALPHA, D.partial, cc.st);
      finalize(D.partial, D.scal, 0, S_RR, 0, cc.st);
      cg_check(D.scal, D.ghist, kGraphHist, cc.guard, S_RZ, S_ALPHA, S_RR, cc.st);
      vcycle64(cc, D.kr, D.kz);
      dot_partial(N, D.kr, D.kz, D.partial, cc.st);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(D.capst, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    HIPCHK(hipStreamEndCapture(D.capst, &D.graph));
    HIPCHK(hipGraphInstantiate(&D.gexec, D.graph, nullptr, nullptr, 0));
    D.ggen = h->gen;
  }
  const int every = std::max(1, h->graph_every);
  int launched = 0;
  for (;;) {
    for (int k = 0; k < every; ++k) HIPCHK(hipGraphLaunch(D.gexec, c.st));
    launched += every;
    HIPCHK(hipMemcpyAsync(D.hscal, D.scal, 64 * sizeof(double), hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipStreamSynchronize(c.st));
    if (D.hscal[kScalFrozen] != 0.0) break;
    if (launched > maxit + every) throw std::runtime_error("graph CG: the recurrence did not stop at maxit");
  }
  const int status = static_cast<int>(D.hscal[kScalStatus]);
  const int it = static_cast<int>(D.hscal[kScalIt]);
  const double rr = D.hscal[kScalRRFinal];
  if (status == 3) throw std::runtime_error("CG breakdown (non-finite residual)");
  hist.resize(std::min(it, kGraphHist));
  if (!hist.empty())
    HIPCHK(hipMemcpyAsync(hist.data(), D.ghist, hist.size() * sizeof(double), hipMemcpyDeviceToHost, c.st));
  HIPCHK(hipMemcpyAsync(x, xi, N * 8, hipMemcpyDeviceToDevice, c.st));
  HIPCHK(hipStreamSynchronize(c.st));
  const bool conv = status == 1;
  // V-cycles the eager recurrence applies: one more than the iterations when
  // it stops at the limit (the last V-cycle follows the last check)
  const int vcycles = status == 0 ? it + 1 : it;
  finish_info(c, b, x, bb, hist, it, conv, std::sqrt(rr / bb), vcycles, info);
  return conv ? LDGMG_OK : LDGMG_ENOCONV;
}

// left-preconditioned GMRES on V A x = V b, x0 = 0, no restart, CGS2
int solve_gmres(const Ctx& c, const double* b, double* x, double rtol, int maxit, ldgmg_info* info) {
  DevHier& D = c.D;
  const long long N = D.L[0].N;
  maxit = std::max(1, std::min(maxit, 200));
  if (D.Qcap < maxit + 1) {
    D.Q = static_cast<double*>(D.alloc(static_cast<size_t>(maxit + 1) * N * 8));
    D.hvec = static_cast<double*>(D.alloc(static_cast<size_t>(2 * (maxit + 2)) * 8 +
                                          static_cast<size_t>(maxit + 2) * kMdotBlocks * 8));
    D.Qcap = maxit + 1;
  }
  double* h1 = D.hvec;
  double* h2 = D.hvec + (maxit + 2);
  double* part = D.hvec + 2 * (maxit + 2);
  HIPCHK(hipMemsetAsync(x, 0, N * 8, c.st));
  const double bb = dot_host(c, b, b, S_BB);
  if (!std::isfinite(bb)) throw std::invalid_argument("right-hand side contains NaN or Inf");
  std::vector<double> hist;
  if (bb == 0.0) {
    finish_info(c, b, x, bb, hist, 0, true, 0.0, 0, info);
    return LDGMG_OK;
  }
  vcycle64(c, b, D.kz);
  int vcycles = 1;
  const double beta2 = dot_host(c, D.kz, D.kz, S_W);
  const double beta = std::sqrt(beta2);
  scale_invsqrt(N, D.kz, D.Q, D.scal, S_W, c.st);
  std::vector<double> H(static_cast<size_t>(maxit + 1) * maxit, 0.0), cs(maxit), sn(maxit), g(maxit + 1, 0.0);
  g[0] = beta;
  hist.push_back(beta);
  std::vector<double> hh1(maxit + 2), hh2(maxit + 2);
  int k = 0;
  bool conv = false;
  for (int j = 0; j < maxit; ++j) {
    apply_A64(c, D.Q + static_cast<size_t>(j) * N, D.kq);
    vcycle64(c, D.kq, D.kz);
    ++vcycles;
    mdot(N, j + 1, D.Q, D.kz, part, h1, c.st);
    maxpy(N, j + 1, D.Q, h1, -1.0, D.kz, c.st);
    mdot(N, j + 1, D.Q, D.kz, part, h2, c.st);
    maxpy(N, j + 1, D.Q, h2, -1.0, D.kz, c.st);
    dot_partial(N, D.kz, D.kz, D.partial, c.st);
    finalize(D.partial, D.scal, 0, S_W, 0, c.st);
    HIPCHK(hipMemcpyAsync(hh1.data(), h1, (j + 1) * 8, hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipMemcpyAsync(hh2.data(), h2, (j + 1) * 8, hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipMemcpyAsync(D.hscal, D.scal, 64 * sizeof(double), hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipStreamSynchronize(c.st));
    const double wn = std::sqrt(D.hscal[S_W]);
    if (!std::isfinite(wn)) throw std::runtime_error("GMRES breakdown (non-finite vector)");
    double* hc = &H[static_cast<size_t>(j) * (maxit + 1)];      // column j
    for (int i = 0; i <= j; ++i) hc[i] = hh1[i] + hh2[i];
    hc[j + 1] = wn;
    if (wn > 0) scale_invsqrt(N, D.kz, D.Q + static_cast<size_t>(j + 1) * N, D.scal, S_W, c.st);
    for (int i = 0; i < j; ++i) {
      const double t = cs[i] * hc[i] + sn[i] * hc[i + 1];
      hc[i + 1] = -sn[i] * hc[i] + cs[i] * hc[i + 1];
      hc[i] = t;
    }
    const double den = std::hypot(hc[j], hc[j + 1]);
    cs[j] = hc[j] / den;
    sn[j] = hc[j + 1] / den;
    hc[j] = den;
    hc[j + 1] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    k = j + 1;
    hist.push_back(std::fabs(g[j + 1]));
    if (std::fabs(g[j + 1]) <= rtol * beta || wn == 0) {
      conv = std::fabs(g[j + 1]) <= rtol * beta;
      break;
    }
  }
  std::vector<double> y(k, 0.0);
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int t = i + 1; t < k; ++t) s -= H[static_cast<size_t>(t) * (maxit + 1) + i] * y[t];
    y[i] = s / H[static_cast<size_t>(i) * (maxit + 1) + i];
  }
  HIPCHK(hipMemcpyAsync(h1, y.data(), k * 8, hipMemcpyHostToDevice, c.st));
  maxpy(N, k, D.Q, h1, 1.0, x, c.st);
  finish_info(c, b, x, bb, hist, k, conv, std::fabs(g[k]) / beta, vcycles, info);
  return conv ? LDGMG_OK : LDGMG_ENOCONV;
}

// ---------------------------------------------------------------------------
// singular operators (a kernel of constants): right-hand side projection and
// the zero-mean convention for the solution
// ---------------------------------------------------------------------------
// out = b - sum_i (b . khat_i) khat_i: b projected on the range of the
// symmetric operator (the khat_i are orthonormal: one component each)
void project_rhs(const Ctx& c, const double* b, double* out) {
  DevHier& D = c.D;
  const long long N = D.L[0].N;
  if (out != b) HIPCHK(hipMemcpyAsync(out, b, N * 8, hipMemcpyDeviceToDevice, c.st));
  for (int i = 0; i < D.nker; ++i) {
    dot_partial(N, out, D.khat + static_cast<size_t>(i) * N, D.partial, c.st);
    finalize(D.partial, D.scal, 3, S_K, 0, c.st);                       // -(b . khat_i)
    axpby(N, D.khat + static_cast<size_t>(i) * N, out, D.scal, S_K, 0.0, -1, 1.0, c.st);
  }
}

// x <- x - sum_i (w_i . x) khat_i: the kernel components of x get zero mean
void remove_kernel(const Ctx& c, double* x) {
  DevHier& D = c.D;
  const long long N = D.L[0].N;
  for (int i = 0; i < D.nker; ++i) {
    dot_partial(N, x, D.kw + static_cast<size_t>(i) * N, D.partial, c.st);
    finalize(D.partial, D.scal, 3, S_K, 0, c.st);
    axpby(N, D.khat + static_cast<size_t>(i) * N, x, D.scal, S_K, 0.0, -1, 1.0, c.st);
  }
}

// |b . khat_i| <= tol ||b|| for every kernel vector, else SingularError
void check_rhs(const Ctx& c, const double* b, double tol) {
  DevHier& D = c.D;
  const long long N = D.L[0].N;
  const double bn = std::sqrt(dot_host(c, b, b, S_TMP));
  for (int i = 0; i < D.nker; ++i) {
    const double v = dot_host(c, b, D.khat + static_cast<size_t>(i) * N, S_K);
    if (!(std::fabs(v) <= tol * bn))
      throw SingularError("inconsistent right-hand side: |b . k| / ||b|| = " + std::to_string(std::fabs(v) / bn) +
                          " for kernel vector " + std::to_string(i) + " (tolerance " + std::to_string(tol) + ")");
  }
}

// ---------------------------------------------------------------------------
// batched V-cycle and CG: nk right-hand sides on one hierarchy; every level
// vector holds nk vectors at a stride of the level size
// ---------------------------------------------------------------------------
// batch vectors for nk right-hand sides: sets of 8, or of kMaxRhs once more
// than 8 are asked for (the 8-sets are then given back)
void ensure_batch(DevHier& D, int nk, hipStream_t st) {
  const int cap = nk <= 8 ? 8 : kMaxRhs;
  if (D.bcap >= cap) return;
  if (D.bcap) {
    HIPCHK(hipStreamSynchronize(st));
    for (auto& B : D.BL)
      for (double* p : {B.x, B.b, B.r, B.t}) D.release(p);
    for (double* p : {D.bx, D.br, D.bp, D.bq, D.bz}) D.release(p);
  }
  D.BL.assign(D.L.size(), DevHier::BatchLevel{});
  for (size_t l = 0; l < D.L.size(); ++l) {
    const size_t vb = static_cast<size_t>(D.L[l].N) * cap * sizeof(double);
    auto& B = D.BL[l];
    B.x = static_cast<double*>(D.alloc(vb));
    B.b = static_cast<double*>(D.alloc(vb));
    B.r = static_cast<double*>(D.alloc(vb));
    B.t = static_cast<double*>(D.alloc(vb));
    HIPCHK(hipMemsetAsync(B.r, 0, vb, st));
    HIPCHK(hipMemsetAsync(B.t, 0, vb, st));
  }
  const size_t vb = static_cast<size_t>(D.L[0].N) * cap * sizeof(double);
  D.bx = static_cast<double*>(D.alloc(vb));
  D.br = static_cast<double*>(D.alloc(vb));
  D.bp = static_cast<double*>(D.alloc(vb));
  D.bq = static_cast<double*>(D.alloc(vb));
  D.bz = static_cast<double*>(D.alloc(vb));
  if (!D.bscal) {
    D.bscal = static_cast<double*>(D.alloc(kMaxRhs * 8 * sizeof(double)));
    HIPCHK(hipMemsetAsync(D.bscal, 0, kMaxRhs * 8 * sizeof(double), st));
    HIPCHK(hipHostMalloc(&D.hbscal, kMaxRhs * 8 * sizeof(double), hipHostMallocDefault));
  }
  D.bcap = cap;
}

template <typename T>
void residual_multi(DevHier& D, const DevLevel& L, const Vd* x, const Vd* b, Vd* out, int nk, hipStream_t st,
                    int nrows = -1, const int* rows = nullptr) {
  ProfScope ps(D, L, st, K_A);
  BsrArgs<T, Vd> a = argsA<T>(L);
  if (rows) {
    a.nrows = nrows;
    a.rows = rows;
  }
  a.x = x;
  a.z = b;
  a.out = out;
  a.alpha = -1.0;
  a.beta = 1.0;
  bsr_forward_multi<T, Vd>(a, L.N, nk, st);
}

// out = alpha S x + beta z (S^T through the transposed copy)
template <typename T>
void apply_S_multi(DevHier& D, const DevLevel& L, bool transposed, const Vd* x, const Vd* z, Vd* out, Vd alpha,
                   Vd beta, int nk, hipStream_t st, int nrows = -1, const int* rows = nullptr) {
  if (transposed && !L.valST) {
    for (int q = 0; q < nk; ++q)
      apply_S<T>(D, L, true, x + q * L.N, z ? z + q * L.N : nullptr, out + q * L.N, alpha, beta, st);
    return;
  }
  ProfScope ps(D, L, st, transposed ? K_ST : K_SF);
  BsrArgs<T, Vd> a = argsS<T>(L);
  if (transposed) {
    a.blk = static_cast<const T*>(L.valST);
    a.bid = L.bidST;
    set_tiled(a, L.tST);
  }
  if (rows) {
    a.nrows = nrows;
    a.rows = rows;
  }
  a.x = x;
  a.z = z;
  a.out = out;
  a.alpha = alpha;
  a.beta = beta;
  bsr_forward_multi<T, Vd>(a, L.N, nk, st);
}

template <typename T, typename TS>
void smooth_step_multi(const Ctx& c, DevLevel& L, DevHier::BatchLevel& B, bool forward, bool zero_x, int nk) {
  const int sm = c.H.prob.smoother;
  const Vd omega = c.H.omega;
  const size_t vb = static_cast<size_t>(L.N) * nk * sizeof(Vd);
  if (sm == LDGMG_SMOOTH_SAI) {
    if (zero_x) {
      apply_S_multi<TS>(c.D, L, !forward, B.b, nullptr, B.x, 1.0, 0.0, nk, c.st);
      return;
    }
    residual_multi<T>(c.D, L, B.x, B.b, B.r, nk, c.st);
    apply_S_multi<TS>(c.D, L, !forward, B.r, B.x, B.x, 1.0, 1.0, nk, c.st);
    return;
  }
  if (sm == LDGMG_SMOOTH_JACOBI) {
    if (zero_x) {
      apply_S_multi<T>(c.D, L, false, B.b, nullptr, B.x, omega, 0.0, nk, c.st);
      return;
    }
    residual_multi<T>(c.D, L, B.x, B.b, B.r, nk, c.st);
    apply_S_multi<T>(c.D, L, false, B.r, B.x, B.x, omega, 1.0, nk, c.st);
    return;
  }
  if (zero_x) fill_zero(B.x, static_cast<long long>(vb / sizeof(Vd)), c.st);
  const int ncol = static_cast<int>(L.colour_rows.size());
  for (int k = 0; k < ncol; ++k) {
    const int col = forward ? k : ncol - 1 - k;
    residual_multi<T>(c.D, L, B.x, B.b, B.r, nk, c.st, L.colour_count[col], L.colour_rows[col]);
    apply_S_multi<T>(c.D, L, false, B.r, B.x, B.x, omega, 1.0, nk, c.st, L.colour_count[col], L.colour_rows[col]);
  }
}

template <typename T, typename TS>
void vcycle_level_multi(const Ctx& c, int l, int nk) {
  DevLevel& L = c.D.L[l];
  DevHier::BatchLevel& B = c.D.BL[l];
  const int nl = static_cast<int>(c.D.L.size());
  if (l == nl - 1) {
    for (int q = 0; q < nk; ++q)
      dense_gemv<Vd>(static_cast<int>(L.N), L.pinv, B.b + q * L.N, B.x + q * L.N, c.st);
    return;
  }
  const ldgmg_problem& P = c.H.prob;
  const bool pre_fwd = order_pre_forward(P.order), post_fwd = order_post_forward(P.order);
  if (P.nu1 == 0) fill_zero(B.x, L.N * nk, c.st);
  for (int s = 0; s < P.nu1; ++s) smooth_step_multi<T, TS>(c, L, B, pre_fwd, s == 0, nk);
  residual_multi<T>(c.D, L, B.x, B.b, B.r, nk, c.st);
  DevLevel& Lc = c.D.L[l + 1];
  DevHier::BatchLevel& Bc = c.D.BL[l + 1];
  for (int q = 0; q < nk; ++q)
    restrict_op<Vd>(P.dim, Lc.n, L.ncomp, L.bss, Lc.q1, Lc.P1, Lc.Ic, B.r + q * L.N, Bc.b + q * Lc.N, c.st);
  vcycle_level_multi<T, TS>(c, l + 1, nk);
  for (int q = 0; q < nk; ++q)
    prolong_add<Vd>(P.dim, Lc.n, L.ncomp, L.bss, Lc.q1, Lc.P1, Lc.Ic, Bc.x + q * Lc.N, B.x + q * L.N, c.st);
  for (int s = 0; s < P.nu2; ++s) smooth_step_multi<T, TS>(c, L, B, post_fwd, false, nk);
}

// z_q = V r_q for the nk vectors at r and z (stride N)
void vcycle64_multi(const Ctx& c, const double* r, double* z, int nk) {
  DevLevel& L = c.D.L[0];
  DevHier::BatchLevel& B = c.D.BL[0];
  const size_t vb = static_cast<size_t>(L.N) * nk * 8;
  HIPCHK(hipMemcpyAsync(B.b, r, vb, hipMemcpyDeviceToDevice, c.st));
  if (c.D.prec == LDGMG_FP64) vcycle_level_multi<double, double>(c, 0, nk);
  else if (c.D.prec == LDGMG_BF16S) vcycle_level_multi<float, bf16s>(c, 0, nk);
  else vcycle_level_multi<float, float>(c, 0, nk);
  HIPCHK(hipMemcpyAsync(z, B.x, vb, hipMemcpyDeviceToDevice, c.st));
}

void apply_A64_multi(const Ctx& c, const double* x, double* y, int nk) {
  const DevLevel& L = c.D.L[0];
  BsrArgs<double, double> a;
  a.nrows = L.ne;
  a.bs = L.bs;
  a.rp = L.rpA;
  a.ci = L.ciA;
  a.blk = c.D.val64;
  a.bid = c.D.bid64;
  set_tiled(a, c.D.t64);
  a.x = x;
  a.out = y;
  ProfScope ps(c.D, L, c.st, K_A64);
  bsr_forward_multi<double, double>(a, L.N, nk, c.st);
}

// nk preconditioned CG recurrences sharing every V-cycle and operator pass
int solve_cg_batch(const Ctx& c, const double* const* b, double* const* x, int nk, double rtol, int maxit,
                   ldgmg_info* infos) {
  DevHier& D = c.D;
  ensure_batch(D, nk, c.st);
  const long long N = D.L[0].N;
  double* sc = D.bscal;
  auto slot = [](int q, int s) { return q * 8 + s; };
  enum { BB = 0, RZ = 1, AL = 2, RR = 3, BE = 4, TMP = 5 };
  for (int q = 0; q < nk; ++q) {
    HIPCHK(hipMemcpyAsync(D.br + q * N, b[q], N * 8, hipMemcpyDeviceToDevice, c.st));
    dot_partial(N, b[q], b[q], D.partial, c.st);
    finalize(D.partial, sc, 0, slot(q, BB), 0, c.st);
  }
  HIPCHK(hipMemsetAsync(D.bx, 0, static_cast<size_t>(N) * nk * 8, c.st));
  HIPCHK(hipMemcpyAsync(D.hbscal, sc, kMaxRhs * 8 * 8, hipMemcpyDeviceToHost, c.st));
  HIPCHK(hipStreamSynchronize(c.st));
  std::vector<double> bb(nk), rr(nk), rel(nk, 0.0);
  std::vector<std::vector<double>> hist(nk);
  std::vector<int> iters(nk, 0);
  std::vector<char> done(nk, 0);
  for (int q = 0; q < nk; ++q) {
    bb[q] = D.hbscal[slot(q, BB)];
    if (!std::isfinite(bb[q])) throw std::invalid_argument("right-hand side contains NaN or Inf");
    done[q] = bb[q] == 0.0;
  }
  vcycle64_multi(c, D.br, D.bz, nk);
  // V-cycles spent on each right-hand side (a converged one is frozen while
  // the batch runs on for the others)
  std::vector<int> vcq(nk, 1);
  for (int q = 0; q < nk; ++q) {
    dot_partial(N, D.br + q * N, D.bz + q * N, D.partial, c.st);
    finalize(D.partial, sc, 0, slot(q, RZ), 0, c.st);
  }
  HIPCHK(hipMemcpyAsync(D.bp, D.bz, static_cast<size_t>(N) * nk * 8, hipMemcpyDeviceToDevice, c.st));
  int it = 0;
  while (it < maxit) {
    bool all = true;
    for (int q = 0; q < nk; ++q) all = all && done[q];
    if (all) break;
    apply_A64_multi(c, D.bp, D.bq, nk);
    for (int q = 0; q < nk; ++q) {
      if (done[q]) continue;
      dot_partial(N, D.bp + q * N, D.bq + q * N, D.partial, c.st);
      finalize(D.partial, sc, 1, slot(q, AL), slot(q, RZ), c.st);
      cg_update(N, D.bx + q * N, D.br + q * N, D.bp + q * N, D.bq + q * N, sc, slot(q, AL), D.partial, c.st);
      finalize(D.partial, sc, 0, slot(q, RR), 0, c.st);
    }
    HIPCHK(hipMemcpyAsync(D.hbscal, sc, kMaxRhs * 8 * 8, hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipStreamSynchronize(c.st));
    ++it;
    bool more = false;
    for (int q = 0; q < nk; ++q) {
      if (done[q]) continue;
      hist[q].push_back(std::sqrt(std::fabs(D.hbscal[slot(q, RZ)])));
      iters[q] = it;
      rr[q] = D.hbscal[slot(q, RR)];
      if (!std::isfinite(rr[q])) throw std::runtime_error("CG breakdown (non-finite residual)");
      if (rr[q] <= rtol * rtol * bb[q]) done[q] = 1;
      else if (c.guard && (!(D.hbscal[slot(q, RZ)] > 0.0) || !(D.hbscal[slot(q, AL)] > 0.0)))
        done[q] = 2;                                     // guarded breakdown
      else more = true;
    }
    if (!more) break;
    vcycle64_multi(c, D.br, D.bz, nk);
    for (int q = 0; q < nk; ++q) vcq[q] += done[q] ? 0 : 1;
    for (int q = 0; q < nk; ++q) {
      if (done[q]) continue;
      dot_partial(N, D.br + q * N, D.bz + q * N, D.partial, c.st);
      finalize(D.partial, sc, 2, slot(q, BE), slot(q, RZ), c.st);
      cg_dir(N, D.bp + q * N, D.bz + q * N, sc, slot(q, BE), c.st);
    }
  }
  bool all_conv = true;
  for (int q = 0; q < nk; ++q) {
    HIPCHK(hipMemcpyAsync(x[q], D.bx + q * N, N * 8, hipMemcpyDeviceToDevice, c.st));
    all_conv = all_conv && done[q] == 1;
    if (infos) {
      finish_info(c, b[q], x[q], bb[q], hist[q], iters[q], done[q] == 1,
                  bb[q] > 0 ? std::sqrt(std::fabs(rr[q]) / bb[q]) : 0.0, vcq[q], &infos[q]);
    }
  }
  HIPCHK(hipStreamSynchronize(c.st));
  return all_conv ? LDGMG_OK : LDGMG_ENOCONV;
}

template <typename T, typename TS>
void level_op_t(const Ctx& c, int l, int op, const void* in1, const void* in2, void* out) {
  DevLevel& L = c.D.L[l];
  const int nl = static_cast<int>(c.D.L.size());
  const Vd* a = static_cast<const Vd*>(in1);
  const Vd* b = static_cast<const Vd*>(in2);
  Vd* o = static_cast<Vd*>(out);
  const bool bottom = l == nl - 1;
  switch (op) {
    case LDGMG_OP_RESIDUAL:
      residual<T>(c.D, L, a, b, o, c.st);
      return;
    case LDGMG_OP_APPLY_A: {
      BsrArgs<T, Vd> x = argsA<T>(L);
      x.x = a;
      x.out = o;
      bsr_forward<T, Vd>(x, c.st);
      return;
    }
    case LDGMG_OP_APPLY_S:
    case LDGMG_OP_APPLY_ST:
      if (bottom) throw std::invalid_argument("no smoother on the bottom level");
      apply_S<TS>(c.D, L, op == LDGMG_OP_APPLY_ST, a, nullptr, o, 1.0, 0.0, c.st);
      return;
    case LDGMG_OP_SMOOTH_FWD:
    case LDGMG_OP_SMOOTH_REV: {
      if (bottom) throw std::invalid_argument("no smoother on the bottom level");
      HIPCHK(hipMemcpyAsync(o, a, static_cast<size_t>(L.N) * sizeof(Vd), hipMemcpyDeviceToDevice, c.st));
      if (c.H.prob.smoother == LDGMG_SMOOTH_SAI && L.p32 && L.x32) cast<double, float>(L.N, o, L.x32, c.st);
      Vd* res = smooth_step<T, TS>(c, L, o, b, op == LDGMG_OP_SMOOTH_FWD, false);
      if (res != o)
        HIPCHK(hipMemcpyAsync(o, res, static_cast<size_t>(L.N) * sizeof(Vd), hipMemcpyDeviceToDevice, c.st));
      return;
    }
    case LDGMG_OP_RESTRICT: {
      if (bottom) throw std::invalid_argument("no coarser level");
      DevLevel& Lc = c.D.L[l + 1];
      restrict_op<Vd>(c.H.prob.dim, Lc.n, L.ncomp, L.bss, Lc.q1, Lc.P1, Lc.Ic, a, o, c.st);
      return;
    }
    case LDGMG_OP_PROLONG_ADD: {
      if (bottom) throw std::invalid_argument("no coarser level");
      DevLevel& Lc = c.D.L[l + 1];
      prolong_add<Vd>(c.H.prob.dim, Lc.n, L.ncomp, L.bss, Lc.q1, Lc.P1, Lc.Ic, a, o, c.st);
      return;
    }
    case LDGMG_OP_BOTTOM:
      if (!bottom) throw std::invalid_argument("LDGMG_OP_BOTTOM needs the bottom level");
      dense_gemv<Vd>(static_cast<int>(L.N), L.pinv, a, o, c.st);
      return;
    default:
      throw std::invalid_argument("unknown op");
  }
}

void ensure_bproj(DevHier& D) {
  if (!D.bproj) D.bproj = static_cast<double*>(D.alloc(static_cast<size_t>(D.L[0].N) * kMaxRhs * sizeof(double)));
}

// one solve of ldgmg_solve: on a singular operator the right-hand side is
// checked (ldgmg_rhs_check) and projected on the range first, and the kernel
// components of the solution are given zero mean afterwards
int solve_one(ldgmg_hier* h, const double* b, double* x, int krylov, double rtol, int maxit, ldgmg_info* info,
              hipStream_t st) {
  DevHier& D = *h->dev;
  Ctx c{*h->host, D, st, h->cg_guard};
  const double* bb = b;
  if (D.nker) {
    if (h->rhs_check > 0) check_rhs(c, b, h->rhs_check);
    ensure_bproj(D);
    project_rhs(c, b, D.bproj);
    bb = D.bproj;
  }
  int rc;
  if (krylov != LDGMG_CG) rc = solve_gmres(c, bb, x, rtol, maxit, info);
  else if (h->graph_every > 0 && maxit > 0 && maxit <= kGraphHist && !D.prof) rc = solve_cg_graph(h, c, bb, x, rtol, maxit, info);
  else rc = solve_cg(c, bb, x, rtol, maxit, info);
  if (D.nker) {
    remove_kernel(c, x);
    HIPCHK(hipStreamSynchronize(st));
  }
  return rc;
}

// batched CG for nk <= kMaxRhs right-hand sides of one hierarchy, with the
// same treatment of singular operators as solve_one
int solve_cg_chunk(ldgmg_hier* h, const double* const* b, double* const* x, int nk, double rtol, int maxit,
                   ldgmg_info* infos, hipStream_t st) {
  DevHier& D = *h->dev;
  Ctx c{*h->host, D, st, h->cg_guard};
  std::vector<const double*> bb(b, b + nk);
  if (D.nker) {
    for (int q = 0; q < nk; ++q)
      if (h->rhs_check > 0) check_rhs(c, b[q], h->rhs_check);
    ensure_bproj(D);
    for (int q = 0; q < nk; ++q) {
      double* dst = D.bproj + static_cast<size_t>(q) * D.L[0].N;
      project_rhs(c, b[q], dst);
      bb[q] = dst;
    }
  }
  const int rc = solve_cg_batch(c, bb.data(), x, nk, rtol, maxit, infos);
  if (D.nker) {
    for (int q = 0; q < nk; ++q) remove_kernel(c, x[q]);
    HIPCHK(hipStreamSynchronize(st));
  }
  return rc;
}

// Continuous batching on one hierarchy: up to `slots` CG recurrences in
// flight, each exactly the recurrence of solve_cg on its own right-hand side,
// sharing every V-cycle stage and operator apply (multi-vector kernels over
// the slots in use).  A free slot is refilled from next() before every
// V-cycle stage: the new right-hand side starts with its first V-cycle there
// (r = b, z = V r, p = z) while the others take their (k+1)-th.  A slot whose
// recurrence stops (converged, maxit, guarded breakdown) is written out,
// reported through done() and freed at once.
int solve_cg_stream(ldgmg_hier* h, int slots, double rtol, int maxit,
                    int (*next)(void*, const double**, double**, long long*),
                    void (*done)(void*, long long, int, const ldgmg_info*), void* ctx, hipStream_t st) {
  DevHier& D = *h->dev;
  Ctx c{*h->host, D, st, h->cg_guard};
  ensure_batch(D, slots, st);
  if (D.nker) ensure_bproj(D);
  const long long N = D.L[0].N;
  double* sc = D.bscal;
  auto slot = [](int q, int s) { return q * 8 + s; };
  enum { BB = 0, RZ = 1, AL = 2, RR = 3, BE = 4 };
  struct Slot {
    bool used = false, fresh = false;
    const double* b = nullptr;   // the right-hand side the recurrence solves (projected when singular)
    double* x = nullptr;         // caller's solution vector
    long long tag = 0;
    int iters = 0, vcycles = 0;
    double bb = 0, rr = 0;
    std::vector<double> hist;
  };
  std::vector<Slot> S(slots);
  int worst = LDGMG_OK;
  auto finish = [&](int q, bool conv) {
    Slot& s = S[q];
    HIPCHK(hipMemcpyAsync(s.x, D.bx + q * N, N * 8, hipMemcpyDeviceToDevice, st));
    ldgmg_info info{};
    finish_info(c, s.b, s.x, s.bb, s.hist, s.iters, conv, s.bb > 0 ? std::sqrt(std::fabs(s.rr) / s.bb) : 0.0,
                s.vcycles, &info);
    if (D.nker) remove_kernel(c, s.x);
    HIPCHK(hipStreamSynchronize(st));
    if (!conv) worst = LDGMG_ENOCONV;
    const long long tag = s.tag;
    s = Slot{};
    done(ctx, tag, conv ? LDGMG_OK : LDGMG_ENOCONV, &info);
  };
  for (;;) {
    // admit waiting right-hand sides into free slots
    for (int q = 0; q < slots; ++q) {
      if (S[q].used) continue;
      const double* b = nullptr;
      double* x = nullptr;
      long long tag = 0;
      if (!next(ctx, &b, &x, &tag)) break;     // nothing waiting now
      if (!b || !x) throw std::invalid_argument("next() gave a null vector");
      Slot& s = S[q];
      s.used = s.fresh = true;
      s.b = b;
      s.x = x;
      s.tag = tag;
      if (D.nker) {
        if (h->rhs_check > 0) check_rhs(c, b, h->rhs_check);
        double* dst = D.bproj + static_cast<size_t>(q) * N;
        project_rhs(c, b, dst);
        s.b = dst;
      }
      HIPCHK(hipMemcpyAsync(D.br + q * N, s.b, N * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemsetAsync(D.bx + q * N, 0, N * 8, st));
      s.bb = dot_host(c, s.b, s.b, S_BB);
      if (!std::isfinite(s.bb)) throw std::invalid_argument("right-hand side contains NaN or Inf");
      if (s.bb == 0.0) {                 // x = 0 solves it: no iteration
        s.rr = 0.0;
        finish(q, true);
        --q;                             // the slot is free again
      }
    }
    int nk = 0;
    for (int q = 0; q < slots; ++q)
      if (S[q].used) nk = q + 1;
    if (nk == 0) break;                        // nothing in flight and nothing waiting
    // V-cycle stage of every slot in use: z = V r; fresh slots start p = z,
    // the others take beta = (r.z)_new / (r.z)_old and p = z + beta p
    vcycle64_multi(c, D.br, D.bz, nk);
    for (int q = 0; q < nk; ++q) {
      Slot& s = S[q];
      if (!s.used) continue;
      ++s.vcycles;
      dot_partial(N, D.br + q * N, D.bz + q * N, D.partial, st);
      if (s.fresh) {
        finalize(D.partial, sc, 0, slot(q, RZ), 0, st);
        HIPCHK(hipMemcpyAsync(D.bp + q * N, D.bz + q * N, N * 8, hipMemcpyDeviceToDevice, st));
        s.fresh = false;
      } else {
        finalize(D.partial, sc, 2, slot(q, BE), slot(q, RZ), st);
        cg_dir(N, D.bp + q * N, D.bz + q * N, sc, slot(q, BE), st);
      }
    }
    // operator stage: q = A p, alpha = (r.z) / (p.q), x += alpha p, r -= alpha q
    apply_A64_multi(c, D.bp, D.bq, nk);
    for (int q = 0; q < nk; ++q) {
      if (!S[q].used) continue;
      dot_partial(N, D.bp + q * N, D.bq + q * N, D.partial, st);
      finalize(D.partial, sc, 1, slot(q, AL), slot(q, RZ), st);
      cg_update(N, D.bx + q * N, D.br + q * N, D.bp + q * N, D.bq + q * N, sc, slot(q, AL), D.partial, st);
      finalize(D.partial, sc, 0, slot(q, RR), 0, st);
    }
    HIPCHK(hipMemcpyAsync(D.hbscal, sc, kMaxRhs * 8 * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int q = 0; q < nk; ++q) {
      Slot& s = S[q];
      if (!s.used) continue;
      s.hist.push_back(std::sqrt(std::fabs(D.hbscal[slot(q, RZ)])));
      ++s.iters;
      s.rr = D.hbscal[slot(q, RR)];
      if (!std::isfinite(s.rr)) throw std::runtime_error("CG breakdown (non-finite residual)");
      if (s.rr <= rtol * rtol * s.bb) finish(q, true);
      else if (c.guard && (!(D.hbscal[slot(q, RZ)] > 0.0) || !(D.hbscal[slot(q, AL)] > 0.0))) finish(q, false);
      else if (s.iters >= maxit) finish(q, false);
    }
  }
  return worst;
}

// device address of `scratch` on the current device, looked up once per device
double* scratch_address() {
  static std::mutex mu;
  static std::vector<void*> addr;
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  if (static_cast<int>(addr.size()) <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    addr[dev] = p;
  }
  return static_cast<double*>(addr[dev]);
}

// k V-cycles with the batch level vectors (x, b, r, t of k vectors per level)
// in the caller-given workspace ws; the handle's own batch vectors are not
// touched.  Every workspace vector is written before it is read.
void vcycle_batch_in(const Ctx& c, const double* const* b, double* const* x, int k, double* ws) {
  DevHier& D = c.D;
  std::vector<DevHier::BatchLevel> mine(D.L.size());
  size_t off = 0;
  for (size_t l = 0; l < D.L.size(); ++l) {
    const size_t n = static_cast<size_t>(D.L[l].N) * k;
    mine[l].x = ws + off;
    mine[l].b = ws + off + n;
    mine[l].r = ws + off + 2 * n;
    mine[l].t = ws + off + 3 * n;
    off += 4 * n;
  }
  std::swap(D.BL, mine);
  struct Restore {   // the handle's batch vectors come back whatever happens
    DevHier& D;
    std::vector<DevHier::BatchLevel>& v;
    ~Restore() { std::swap(D.BL, v); }
  } restore{D, mine};
  const long long N = D.L[0].N;
  for (int q = 0; q < k; ++q)
    HIPCHK(hipMemcpyAsync(D.BL[0].b + q * N, b[q], N * 8, hipMemcpyDeviceToDevice, c.st));
  if (D.prec == LDGMG_FP64) vcycle_level_multi<double, double>(c, 0, k);
  else if (D.prec == LDGMG_BF16S) vcycle_level_multi<float, bf16s>(c, 0, k);
  else vcycle_level_multi<float, float>(c, 0, k);
  for (int q = 0; q < k; ++q)
    HIPCHK(hipMemcpyAsync(x[q], D.BL[0].x + q * N, N * 8, hipMemcpyDeviceToDevice, c.st));
}

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

template <class F>
int guarded(F&& fn) {
  try {
    g_err.clear();
    return fn();
  } catch (const BudgetError& e) {
    return fail(LDGMG_ENOMEM, e.what());
  } catch (const HipError& e) {
    return fail(LDGMG_EHIP, e.what());
  } catch (const StateError& e) {
    return fail(LDGMG_ESTATE, e.what());
  } catch (const SingularError& e) {
    return fail(LDGMG_ESINGULAR, e.what());
  } catch (const std::invalid_argument& e) {
    return fail(LDGMG_EINVAL, e.what());
  } catch (const std::bad_alloc&) {
    return fail(LDGMG_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    const std::string m = e.what();
    if (m.find("rank-deficient") != std::string::npos) return fail(LDGMG_ESINGULAR, m);
    return fail(LDGMG_EHIP, m);
  }
}

void need_dev(ldgmg_hier* h) {
  if (!h) throw std::invalid_argument("null handle");
  if (!h->dev) throw StateError("handle has no device data (call ldgmg_upload)");
  int cur = -1;
  HIPCHK(hipGetDevice(&cur));
  if (cur != h->dev->device) throw StateError("current HIP device differs from the device of the handle");
}

void check_level(ldgmg_hier* h, int level) {
  if (!h || !h->host) throw std::invalid_argument("null handle");
  if (level < 0 || level >= static_cast<int>(h->host->levels.size())) throw std::invalid_argument("level out of range");
}

}  // namespace
}  // namespace ldgmg

using namespace ldgmg;

extern "C" {

int ldgmg_problem_default(ldgmg_problem* p) {
  if (!p) return fail(LDGMG_EINVAL, "null problem");
  std::memset(p, 0, sizeof(*p));
  p->dim = 2;
  p->n = 16;
  p->p = 2;
  p->basis = LDGMG_BASIS_LEGENDRE;
  p->system = LDGMG_POISSON;
  p->gamma = 1;
  for (int f = 0; f < 6; ++f) p->bc[f] = LDGMG_BC_DIRICHLET;
  p->mu = nullptr;
  p->tau0 = 1.0;
  p->cp = 0.1;
  p->smoother = LDGMG_SMOOTH_SAI;
  p->sai_level = 1;
  p->order = LDGMG_ORDER_OI;
  p->nu1 = 3;
  p->nu2 = 3;
  p->omega = 0.0;
  p->zeta = 0.0;
  p->precision = LDGMG_FP32;
  p->nthreads = 0;
  p->hbm_budget = 0;
  p->storage = LDGMG_STORE_AUTO;
  p->rho = nullptr;
  p->delta = 0.0;
  p->setup_device = 0;
  p->dev_alloc = nullptr;
  p->dev_free = nullptr;
  p->alloc_ctx = nullptr;
  return LDGMG_OK;
}

int ldgmg_estimate_bytes(const ldgmg_problem* p, size_t* bytes) {
  return guarded([&] {
    if (!p || !bytes) throw std::invalid_argument("null argument");
    validate_problem(*p);
    // interior stencils: |A| (tab:sizes) and the smoother pattern; 2% margin for interfaces
    const int d = p->dim;
    const bool stress = p->system == LDGMG_STOKES && p->gamma;
    const int sA = stress ? (d == 2 ? 7 : 13) : 2 * d + 1;
    const int sS[3][2] = {{1, 1}, {2 * d + 1, stress ? (d == 2 ? 7 : 13) : 2 * d + 1},
                          {d == 2 ? 13 : 25, stress ? (d == 2 ? 19 : 55) : (d == 2 ? 13 : 25)}};
    int bss = 1;
    for (int k = 0; k < d; ++k) bss *= p->p + 1;
    const int bs = bss * (p->system == LDGMG_STOKES ? d + 1 : 1);
    const std::vector<int> sizes = level_sizes(p->n);
    size_t b = 0;
    for (size_t l = 0; l < sizes.size(); ++l) {
      long long ne = 1;
      for (int k = 0; k < d; ++k) ne *= sizes[l];
      const bool bottom = l + 1 == sizes.size();
      const long long nnzA = static_cast<long long>(ne * sA * 1.02) + 1;
      const long long nnzS = p->smoother == LDGMG_SMOOTH_SAI
                                 ? static_cast<long long>(ne * sS[p->sai_level][stress ? 1 : 0] * 1.02) + 1
                                 : ne;
      b += level_bytes(static_cast<int>(ne), bs, bss, d, nnzA, nnzS, bottom, p->smoother == LDGMG_SMOOTH_GS,
                       p->precision);
      if (l == 0) {
        if (p->precision != LDGMG_FP64) b += static_cast<size_t>(nnzA) * bs * bs * 8;
        b += 5 * static_cast<size_t>(ne) * bs * 8 + 64 * 8 + kRedBlocks * 16;
      }
    }
    *bytes = b;
    return LDGMG_OK;
  });
}

int ldgmg_setup_host(const ldgmg_problem* p, ldgmg_handle* out) {
  return guarded([&] {
    if (!p || !out) throw std::invalid_argument("null argument");
    *out = nullptr;
    auto h = std::make_unique<ldgmg_hier>();
    if (p->setup_device) {
      const SaiBatchSolver gpu = gpu_sai_solve;
      h->host = build_host(*p, &gpu);
    } else {
      h->host = build_host(*p);
    }
    *out = h.release();
    return LDGMG_OK;
  });
}

int ldgmg_rebuild_smoother(ldgmg_handle src, const ldgmg_problem* p, ldgmg_handle* out) {
  return guarded([&] {
    if (!src || !src->host || !p || !out) throw std::invalid_argument("null argument");
    *out = nullptr;
    auto h = std::make_unique<ldgmg_hier>();
    if (p->setup_device) {
      const SaiBatchSolver gpu = gpu_sai_solve;
      h->host = rebuild_smoother(*src->host, *p, &gpu);
    } else {
      h->host = rebuild_smoother(*src->host, *p);
    }
    *out = h.release();
    return LDGMG_OK;
  });
}

int ldgmg_upload(ldgmg_handle h, void* stream) {
  return guarded([&] {
    if (!h || !h->host) throw std::invalid_argument("null handle");
    h->dev.reset();
    upload(h, static_cast<hipStream_t>(stream));
    return LDGMG_OK;
  });
}

int ldgmg_unload(ldgmg_handle h) {
  return guarded([&] {
    if (!h || !h->host) throw std::invalid_argument("null handle");
    h->dev.reset();
    return LDGMG_OK;
  });
}

int ldgmg_cg_guard(ldgmg_handle h, int enable) {
  return guarded([&] {
    if (!h || !h->host) throw std::invalid_argument("null handle");
    h->cg_guard = enable != 0;
    ++h->gen;                       // the guard is an argument of the captured test
    return LDGMG_OK;
  });
}

int ldgmg_cg_graph(ldgmg_handle h, int check_every) {
  return guarded([&] {
    if (!h || !h->host) throw std::invalid_argument("null handle");
    if (check_every < 0) throw std::invalid_argument("check_every must be >= 0");
    h->graph_every = check_every;
    return LDGMG_OK;
  });
}

int ldgmg_rhs_check(ldgmg_handle h, double tol) {
  return guarded([&] {
    if (!h || !h->host) throw std::invalid_argument("null handle");
    if (!(tol >= 0) || !std::isfinite(tol)) throw std::invalid_argument("tolerance must be finite and >= 0");
    h->rhs_check = tol;
    return LDGMG_OK;
  });
}

int ldgmg_kernel(ldgmg_handle h, int* count, double* host_out) {
  return guarded([&] {
    need_dev(h);
    if (!count) throw std::invalid_argument("null count");
    const DevHier& D = *h->dev;
    *count = D.nker;
    if (host_out && D.nker) {
      HIPCHK(hipMemcpy(host_out, D.khat, static_cast<size_t>(D.nker) * D.L[0].N * sizeof(double),
                       hipMemcpyDeviceToHost));
    }
    return LDGMG_OK;
  });
}

int ldgmg_fp32_products(ldgmg_handle h, int enable) {
  return guarded([&] {
    if (!h || !h->host) throw std::invalid_argument("null handle");
    if (enable && h->host->prob.precision == LDGMG_FP64)
      throw std::invalid_argument("FP32 products need FP32 or BF16 storage");
    h->fp32_products = enable != 0;
    ++h->gen;                       // other kernels: a captured iteration is stale
    if (h->dev)
      for (DevLevel& L : h->dev->L) L.p32 = h->fp32_products;
    return LDGMG_OK;
  });
}

int ldgmg_device_bytes(ldgmg_handle h, size_t* bytes) {
  return guarded([&] {
    if (!h || !h->host || !bytes) throw std::invalid_argument("null argument");
    *bytes = h->dev ? h->dev->bytes : 0;
    return LDGMG_OK;
  });
}

int ldgmg_level_storage(ldgmg_handle h, int level, int* pool_A, int* pool_S, int* tiled) {
  return guarded([&] {
    need_dev(h);
    check_level(h, level);
    const HostLevel& H = h->host->levels[level];
    const DevLevel& D = h->dev->L[level];
    if (pool_A) *pool_A = D.bidA ? H.A.pool.size() : 0;
    if (pool_S) *pool_S = D.bidS ? H.S.pool.size() : 0;
    if (tiled) *tiled = (D.tA.tab ? 1 : 0) | (D.tS.tab ? 2 : 0);
    return LDGMG_OK;
  });
}

int ldgmg_upload_bytes(ldgmg_handle h, size_t* bytes) {
  return guarded([&] {
    if (!h || !h->host || !bytes) throw std::invalid_argument("null argument");
    *bytes = estimate_from_host(*h->host, h->host->prob.precision);
    return LDGMG_OK;
  });
}

int ldgmg_setup(const ldgmg_problem* p, void* stream, ldgmg_handle* out) {
  ldgmg_handle h = nullptr;
  int rc = ldgmg_setup_host(p, &h);
  if (rc != LDGMG_OK) return rc;
  rc = ldgmg_upload(h, stream);
  if (rc != LDGMG_OK) {
    const std::string msg = g_err;
    delete h;
    g_err = msg;
    return rc;
  }
  *out = h;
  return LDGMG_OK;
}

int ldgmg_sizes(ldgmg_handle h, long long* ndofs, int* bs, int* nlevels) {
  return guarded([&] {
    if (!h || !h->host) throw std::invalid_argument("null handle");
    const HostLevel& F = h->host->levels[0];
    if (ndofs) *ndofs = static_cast<long long>(F.ne) * F.bs;
    if (bs) *bs = F.bs;
    if (nlevels) *nlevels = static_cast<int>(h->host->levels.size());
    return LDGMG_OK;
  });
}

int ldgmg_level_info(ldgmg_handle h, int level, int* n, int* nelem, int* nnzb_A, int* nnzb_S, int* ncolours) {
  return guarded([&] {
    check_level(h, level);
    const HostLevel& L = h->host->levels[level];
    if (n) *n = L.n;
    if (nelem) *nelem = L.ne;
    if (nnzb_A) *nnzb_A = L.A.nnzb();
    if (nnzb_S) *nnzb_S = L.S.nnzb();
    if (ncolours) *ncolours = L.ncolours;
    return LDGMG_OK;
  });
}

int ldgmg_rhs_volume(ldgmg_handle h, const double* f_qp, int nq, double* b_dev, void* stream) {
  return guarded([&] {
    need_dev(h);
    if (!f_qp || !b_dev || nq < 1 || nq > 16) throw std::invalid_argument("bad rhs arguments");
    const HostHierarchy& H = *h->host;
    if (H.prob.system != LDGMG_POISSON) throw std::invalid_argument("volume load is for scalar problems");
    const HostLevel& F = H.levels[0];
    const int d = H.prob.dim, q1 = F.em.q1;
    // 1-D table w_q psi_i(t_q) at the nq Gauss points the caller sampled f at
    std::vector<double> t, w, v(q1), dv(q1);
    gauss_legendre(nq, t, w);
    std::vector<double> tab(static_cast<size_t>(q1) * nq);
    for (int q = 0; q < nq; ++q) {
      basis_eval(F.em.p, H.prob.basis, t[q], v.data(), dv.data());
      for (int i = 0; i < q1; ++i) tab[static_cast<size_t>(i) * nq + q] = w[q] * v[i];
    }
    int nqd = 1;
    for (int k = 0; k < d; ++k) nqd *= nq;
    const double scale = std::pow(F.h / 2.0, d);
    std::vector<double> b(static_cast<size_t>(F.ne) * F.bs, 0.0);
    for (int e = 0; e < F.ne; ++e) {
      const double* fe = f_qp + static_cast<size_t>(e) * nqd;
      for (int a = 0; a < F.bs; ++a) {
        const int a0 = a % q1, a1 = (a / q1) % q1, a2 = a / (q1 * q1);
        double s = 0.0;
        for (int qq = 0; qq < nqd; ++qq) {
          const int q0 = qq % nq, qy = (qq / nq) % nq, qz = qq / (nq * nq);
          double wgt = tab[static_cast<size_t>(a0) * nq + q0] * tab[static_cast<size_t>(a1) * nq + qy];
          if (d == 3) wgt *= tab[static_cast<size_t>(a2) * nq + qz];
          s += wgt * fe[qq];
        }
        b[static_cast<size_t>(e) * F.bs + a] = scale * s;
      }
    }
    const hipStream_t st = static_cast<hipStream_t>(stream);
    HIPCHK(hipMemcpyAsync(b_dev, b.data(), b.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return LDGMG_OK;
  });
}

int ldgmg_vcycle(ldgmg_handle h, const double* b_dev, double* x_dev, void* stream) {
  return guarded([&] {
    need_dev(h);
    if (!b_dev || !x_dev) throw std::invalid_argument("null vector");
    Ctx c{*h->host, *h->dev, static_cast<hipStream_t>(stream)};
    vcycle64(c, b_dev, x_dev);
    return LDGMG_OK;
  });
}

int ldgmg_solve(ldgmg_handle h, const double* b_dev, double* x_dev, int krylov, double rtol, int maxit,
                ldgmg_info* info, void* stream) {
  return guarded([&] {
    need_dev(h);
    if (!b_dev || !x_dev) throw std::invalid_argument("null vector");
    if (!(rtol > 0) || maxit < 1) throw std::invalid_argument("rtol must be > 0 and maxit >= 1");
    if (krylov != LDGMG_CG && krylov != LDGMG_GMRES) throw std::invalid_argument("unknown krylov method");
    return solve_one(h, b_dev, x_dev, krylov, rtol, maxit, info, static_cast<hipStream_t>(stream));
  });
}

int ldgmg_vcycle_batch(ldgmg_handle h, const double* const* b_dev, double* const* x_dev, int k, void* stream) {
  return guarded([&] {
    need_dev(h);
    if (!b_dev || !x_dev || k < 1 || k > kMaxRhs) throw std::invalid_argument("bad batch arguments");
    Ctx c{*h->host, *h->dev, static_cast<hipStream_t>(stream)};
    ensure_batch(*h->dev, k, c.st);
    const long long N = h->dev->L[0].N;
    for (int q = 0; q < k; ++q) {
      if (!b_dev[q] || !x_dev[q]) throw std::invalid_argument("null vector in batch");
      HIPCHK(hipMemcpyAsync(h->dev->br + q * N, b_dev[q], N * 8, hipMemcpyDeviceToDevice, c.st));
    }
    vcycle64_multi(c, h->dev->br, h->dev->bz, k);
    for (int q = 0; q < k; ++q)
      HIPCHK(hipMemcpyAsync(x_dev[q], h->dev->bz + q * N, N * 8, hipMemcpyDeviceToDevice, c.st));
    return LDGMG_OK;
  });
}

int ldgmg_vcycle_batch_noalloc(ldgmg_handle h, const double* const* b_dev, double* const* x_dev, int k,
                               void* stream) {
  return guarded([&] {
    need_dev(h);
    if (!b_dev || !x_dev || k < 1 || k > kMaxRhs) throw std::invalid_argument("bad batch arguments");
    for (int q = 0; q < k; ++q)
      if (!b_dev[q] || !x_dev[q]) throw std::invalid_argument("null vector in batch");
    long long need = 0;
    for (const DevLevel& L : h->dev->L) need += 4 * L.N * k;
    if (need > kScratchDoubles)
      throw std::invalid_argument("ldgmg_vcycle_batch_noalloc: " + std::to_string(k) + " right-hand sides need " +
                                  std::to_string(need * 8) + " bytes of scratch, more than its " +
                                  std::to_string(kScratchDoubles * 8) + " bytes");
    Ctx c{*h->host, *h->dev, static_cast<hipStream_t>(stream)};
    vcycle_batch_in(c, b_dev, x_dev, k, scratch_address());
    return LDGMG_OK;
  });
}

int ldgmg_solve_batch(const ldgmg_handle* hs, const double* const* b_dev, double* const* x_dev, int k, int krylov,
                      double rtol, int maxit, ldgmg_info* infos, void* stream) {
  return guarded([&] {
    if (!hs || !b_dev || !x_dev || k < 1) throw std::invalid_argument("bad batch arguments");
    if (!(rtol > 0) || maxit < 1) throw std::invalid_argument("rtol must be > 0 and maxit >= 1");
    if (krylov != LDGMG_CG && krylov != LDGMG_GMRES) throw std::invalid_argument("unknown krylov method");
    for (int q = 0; q < k; ++q) {
      need_dev(hs[q]);
      if (!b_dev[q] || !x_dev[q]) throw std::invalid_argument("null vector in batch");
    }
    const hipStream_t st = static_cast<hipStream_t>(stream);
    // group the right-hand sides by hierarchy, in order of first appearance
    std::vector<ldgmg_hier*> order;
    std::vector<std::vector<int>> members;
    for (int q = 0; q < k; ++q) {
      size_t g = 0;
      while (g < order.size() && order[g] != hs[q]) ++g;
      if (g == order.size()) {
        order.push_back(hs[q]);
        members.emplace_back();
      }
      members[g].push_back(q);
    }
    int worst = LDGMG_OK;
    for (size_t g = 0; g < order.size(); ++g) {
      ldgmg_hier* h = order[g];
      const std::vector<int>& idx = members[g];
      if (krylov == LDGMG_GMRES) {
        for (int q : idx)
          if (solve_one(h, b_dev[q], x_dev[q], krylov, rtol, maxit, infos ? &infos[q] : nullptr, st) != LDGMG_OK)
            worst = LDGMG_ENOCONV;
        continue;
      }
      for (size_t c0 = 0; c0 < idx.size(); c0 += kMaxRhs) {
        const int nk = static_cast<int>(std::min<size_t>(kMaxRhs, idx.size() - c0));
        std::vector<const double*> bq(nk);
        std::vector<double*> xq(nk);
        std::vector<ldgmg_info> iq(nk);
        for (int j = 0; j < nk; ++j) {
          const int q = idx[c0 + j];
          bq[j] = b_dev[q];
          xq[j] = x_dev[q];
          iq[j] = infos ? infos[q] : ldgmg_info{};
        }
        if (solve_cg_chunk(h, bq.data(), xq.data(), nk, rtol, maxit, infos ? iq.data() : nullptr, st) != LDGMG_OK)
          worst = LDGMG_ENOCONV;
        if (infos)
          for (int j = 0; j < nk; ++j) infos[idx[c0 + j]] = iq[j];
      }
    }
    return worst;
  });
}

int ldgmg_solve_stream(ldgmg_handle h, int slots, double rtol, int maxit,
                       int (*next)(void* ctx, const double** b_dev, double** x_dev, long long* tag),
                       void (*done)(void* ctx, long long tag, int status, const ldgmg_info* info), void* ctx,
                       void* stream) {
  return guarded([&] {
    need_dev(h);
    if (slots < 1 || slots > kMaxRhs) throw std::invalid_argument("slots must be in 1..16");
    if (!(rtol > 0) || maxit < 1) throw std::invalid_argument("rtol must be > 0 and maxit >= 1");
    if (!next || !done) throw std::invalid_argument("null callback");
    return solve_cg_stream(h, slots, rtol, maxit, next, done, ctx, static_cast<hipStream_t>(stream));
  });
}

int ldgmg_level_op(ldgmg_handle h, int level, int op, const void* in1, const void* in2, void* out, void* stream) {
  return guarded([&] {
    need_dev(h);
    check_level(h, level);
    if (!in1 || !out) throw std::invalid_argument("null vector");
    if ((op == LDGMG_OP_RESIDUAL || op == LDGMG_OP_SMOOTH_FWD || op == LDGMG_OP_SMOOTH_REV) && !in2)
      throw std::invalid_argument("op needs in2");
    Ctx c{*h->host, *h->dev, static_cast<hipStream_t>(stream)};
    if (op == LDGMG_OP_APPLY_A64) {
      if (level != 0) throw std::invalid_argument("the FP64 operator lives on level 0");
      apply_A64(c, static_cast<const double*>(in1), static_cast<double*>(out));
      return LDGMG_OK;
    }
    if (h->dev->prec == LDGMG_FP64) level_op_t<double, double>(c, level, op, in1, in2, out);
    else if (h->dev->prec == LDGMG_BF16S) level_op_t<float, bf16s>(c, level, op, in1, in2, out);
    else level_op_t<float, float>(c, level, op, in1, in2, out);
    return LDGMG_OK;
  });
}

int ldgmg_export(ldgmg_handle h, int level, int what, int* row_ptr, int* col, double* blocks, int* nnzb,
                 int* dense_n) {
  return guarded([&] {
    check_level(h, level);
    const HostHierarchy& H = *h->host;
    if (what == LDGMG_EXPORT_PINV) {
      const HostLevel& B = H.levels.back();
      const int N = B.ne * B.bs;
      if (dense_n) *dense_n = N;
      if (blocks) std::copy(B.pinv.begin(), B.pinv.end(), blocks);
      return LDGMG_OK;
    }
    const HostLevel& L = H.levels[level];
    const PMat* P = nullptr;
    if (what == LDGMG_EXPORT_A) P = &L.A;
    else if (what == LDGMG_EXPORT_S) P = &L.S;
    else throw std::invalid_argument("unknown export");
    if (what == LDGMG_EXPORT_S && level + 1 == static_cast<int>(H.levels.size()))
      throw std::invalid_argument("no smoother on the bottom level");
    if (nnzb) *nnzb = P->nnzb();
    if (!blocks) return LDGMG_OK;
    if (row_ptr) std::copy(P->rp.begin(), P->rp.end(), row_ptr);
    if (col) std::copy(P->ci.begin(), P->ci.end(), col);
    const size_t bb = static_cast<size_t>(L.bs) * L.bs;
    for (int s = 0; s < P->nnzb(); ++s) std::copy(P->block(s), P->block(s) + bb, blocks + s * bb);
    return LDGMG_OK;
  });
}

int ldgmg_export_colours(ldgmg_handle h, int level, int* colours) {
  return guarded([&] {
    check_level(h, level);
    const HostLevel& L = h->host->levels[level];
    if (!colours) throw std::invalid_argument("null output");
    if (L.colour.empty()) throw std::invalid_argument("level has no colouring");
    std::copy(L.colour.begin(), L.colour.end(), colours);
    return LDGMG_OK;
  });
}

int ldgmg_setup_stats(ldgmg_handle h, int level, int* sai_unique, double* seconds) {
  return guarded([&] {
    check_level(h, level);
    const HostLevel& L = h->host->levels[level];
    if (sai_unique) *sai_unique = L.sai_unique;
    if (seconds) *seconds = L.setup_seconds;
    return LDGMG_OK;
  });
}

int ldgmg_setup_stats_device(ldgmg_handle h, int level, int* sai_device, int* sai_qr, double* sai_seconds) {
  return guarded([&] {
    check_level(h, level);
    const HostLevel& L = h->host->levels[level];
    if (sai_device) *sai_device = L.sai_device;
    if (sai_qr) *sai_qr = L.sai_qr;
    if (sai_seconds) *sai_seconds = L.sai_seconds;
    return LDGMG_OK;
  });
}

int ldgmg_profile(ldgmg_handle h, int enable) {
  return guarded([&] {
    need_dev(h);
    DevHier& D = *h->dev;
    if (D.evpool.empty() && enable) {
      D.evpool.resize(8192);
      for (auto& e : D.evpool) HIPCHK(hipEventCreate(&e));
    }
    D.recs.clear();
    D.prof = enable != 0;
    return LDGMG_OK;
  });
}

int ldgmg_profile_read(ldgmg_handle h, int kind, int* count, double* total_ms) {
  return guarded([&] {
    need_dev(h);
    DevHier& D = *h->dev;
    int cnt = 0;
    double tot = 0.0;
    for (const auto& r : D.recs) {
      if (r.kind != kind) continue;
      HIPCHK(hipEventSynchronize(r.b));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
      tot += ms;
      ++cnt;
    }
    if (count) *count = cnt;
    if (total_ms) *total_ms = tot;
    return LDGMG_OK;
  });
}

int ldgmg_destroy(ldgmg_handle h) {
  delete h;
  return LDGMG_OK;
}

const char* ldgmg_last_error(void) { return g_err.c_str(); }

}  // extern "C"

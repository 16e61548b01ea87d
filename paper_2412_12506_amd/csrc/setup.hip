// SAI least-squares setup on the GPU (Section 2.3.3: every block column of the
// balanced SAI matrix is an independent least-squares problem; Section 4: the
// distinct problems of a hierarchy are few and their cost is the setup's).
//
// The host lists the distinct problems (the SAI column cache); this file
// solves them in batches of equal shape, in FP64, by normal equations with one
// step of iterative refinement (as the host solver does):
//   C   = A~[I, J], dense column-major (m x n), scattered from its nonzero blocks
//   G   = C^T C                         (rocBLAS strided-batched GEMM)
//   G   = L L^T                         (rocSOLVER strided-batched Cholesky)
//   X   = G^-1 C^T E                    (E the identity block at block row pos)
//   dX  = G^-1 C^T (E - C X),  X += dX  (one refinement step)
// A problem is handed back to the host (Householder QR there) when its
// Cholesky factorisation fails, its solution is not finite, or the refinement
// step exceeds 1e-8 of the solution (kappa(C)^2 u not small).
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "setup.hpp"

namespace ldgmg {

namespace {

#define SETUP_HIP(x)                                                                                   \
  do {                                                                                                 \
    const hipError_t e_ = (x);                                                                         \
    if (e_ != hipSuccess) throw std::runtime_error(std::string("GPU SAI setup: ") + #x + ": " +       \
                                                   hipGetErrorString(e_));                             \
  } while (0)
#define SETUP_BLAS(x)                                                                                  \
  do {                                                                                                 \
    const rocblas_status s_ = (x);                                                                     \
    if (s_ != rocblas_status_success)                                                                  \
      throw std::runtime_error(std::string("GPU SAI setup: ") + #x + " failed (" + std::to_string(s_) + ")"); \
  } while (0)

// C[p] (column-major m x n) from its nonzero blocks: block q of problem
// bprob[q] at block coordinates (brow[q], bcol[q]) is
// diag(alpha[arow[q]]) pool[bid[q]] diag(alpha[acol[q]])
__global__ void k_scatter_blocks(long long nq, int bs, int m, long long mn, const double* __restrict__ pool,
                                 const double* __restrict__ alpha, const int* __restrict__ bprob,
                                 const int* __restrict__ brow, const int* __restrict__ bcol,
                                 const int* __restrict__ bid, const int* __restrict__ arow,
                                 const int* __restrict__ acol, double* __restrict__ C) {
  const long long bb = static_cast<long long>(bs) * bs;
  for (long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; t < nq * bb;
       t += static_cast<long long>(gridDim.x) * blockDim.x) {
    const long long q = t / bb;
    const int e = static_cast<int>(t - q * bb);
    const int r = e / bs, c = e % bs;
    const double v = alpha[static_cast<long long>(arow[q]) * bs + r] * pool[static_cast<long long>(bid[q]) * bb + e] *
                     alpha[static_cast<long long>(acol[q]) * bs + c];
    const long long row = static_cast<long long>(brow[q]) * bs + r;
    const long long col = static_cast<long long>(bcol[q]) * bs + c;
    C[bprob[q] * mn + col * m + row] = v;
  }
}

// R[p] (n x bs) = C[p]^T E[p] = rows pos[p] bs .. pos[p] bs + bs - 1 of C[p], transposed
__global__ void k_rhs_rows(int batch, int bs, int m, int n, long long mn, const int* __restrict__ pos,
                           const double* __restrict__ C, double* __restrict__ R) {
  const long long total = static_cast<long long>(batch) * n * bs;
  for (long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += static_cast<long long>(gridDim.x) * blockDim.x) {
    const long long p = t / (static_cast<long long>(n) * bs);
    const int rem = static_cast<int>(t - p * n * bs);
    const int c = rem / n, j = rem % n;           // R column-major: R[c n + j]
    R[t] = C[p * mn + static_cast<long long>(j) * m + static_cast<long long>(pos[p]) * bs + c];
  }
}

// Res[p] (m x bs) += E[p]: ones at (pos[p] bs + c, c)
__global__ void k_add_identity(int batch, int bs, int m, const int* __restrict__ pos, double* __restrict__ Res) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= batch * bs) return;
  const int p = t / bs, c = t % bs;
  Res[static_cast<long long>(p) * m * bs + static_cast<long long>(c) * m + static_cast<long long>(pos[p]) * bs + c] += 1.0;
}

int grid_of(long long n) { return static_cast<int>(std::min<long long>((n + 255) / 256, 65536)); }

template <typename T>
T* dalloc(std::vector<void*>& owned, size_t n) {
  void* p = nullptr;
  SETUP_HIP(hipMalloc(&p, std::max<size_t>(16, n * sizeof(T))));
  owned.push_back(p);
  return static_cast<T*>(p);
}

// one batch of problems of equal shape (mb, nb); dpool / dalpha: A's pool and
// the balancing vectors on the device
void solve_group(rocblas_handle hb, hipStream_t st, int bs, const double* dpool, const double* dalpha,
                 std::vector<SaiProblem*>& grp, std::vector<char>& ok, const std::vector<int>& index) {
  const int batch = static_cast<int>(grp.size());
  const int m = grp[0]->mb * bs, n = grp[0]->nb * bs;
  const long long mn = static_cast<long long>(m) * n, nn = static_cast<long long>(n) * n;
  const long long nk = static_cast<long long>(n) * bs, mk = static_cast<long long>(m) * bs;
  long long nq = 0;
  for (const SaiProblem* p : grp) nq += static_cast<long long>(p->brow.size());
  // per block: problem, coordinates, pool block, balancing vectors (6 ints)
  std::vector<int> meta(static_cast<size_t>(nq) * 6), pos(batch);
  long long q = 0;
  for (int p = 0; p < batch; ++p) {
    const SaiProblem& pb = *grp[p];
    for (size_t k = 0; k < pb.brow.size(); ++k, ++q) {
      meta[q] = p;
      meta[nq + q] = pb.brow[k];
      meta[2 * nq + q] = pb.bcol[k];
      meta[3 * nq + q] = pb.bid[k];
      meta[4 * nq + q] = pb.arow[k];
      meta[5 * nq + q] = pb.acol[k];
    }
    pos[p] = pb.pos;
  }
  std::vector<void*> owned;
  struct Free {
    std::vector<void*>& v;
    ~Free() {
      for (void* p : v) (void)hipFree(p);
    }
  } release{owned};
  int* dmeta = dalloc<int>(owned, meta.size());
  int* dpos = dalloc<int>(owned, batch);
  double* C = dalloc<double>(owned, static_cast<size_t>(batch) * mn);
  double* G = dalloc<double>(owned, static_cast<size_t>(batch) * nn);
  double* X = dalloc<double>(owned, static_cast<size_t>(batch) * nk);
  double* S = dalloc<double>(owned, static_cast<size_t>(batch) * nk);
  double* Res = dalloc<double>(owned, static_cast<size_t>(batch) * mk);
  rocblas_int* info = dalloc<rocblas_int>(owned, batch);
  SETUP_HIP(hipMemcpyAsync(dmeta, meta.data(), meta.size() * sizeof(int), hipMemcpyHostToDevice, st));
  SETUP_HIP(hipMemcpyAsync(dpos, pos.data(), batch * sizeof(int), hipMemcpyHostToDevice, st));
  SETUP_HIP(hipMemsetAsync(C, 0, static_cast<size_t>(batch) * mn * sizeof(double), st));
  k_scatter_blocks<<<grid_of(nq * bs * bs), 256, 0, st>>>(nq, bs, m, mn, dpool, dalpha, dmeta, dmeta + nq,
                                                          dmeta + 2 * nq, dmeta + 3 * nq, dmeta + 4 * nq,
                                                          dmeta + 5 * nq, C);
  SETUP_HIP(hipGetLastError());
  const double one = 1.0, zero = 0.0, minus = -1.0;
  // G = C^T C, then its Cholesky factor
  SETUP_BLAS(rocblas_dgemm_strided_batched(hb, rocblas_operation_transpose, rocblas_operation_none, n, n, m, &one, C,
                                           m, mn, C, m, mn, &zero, G, n, nn, batch));
  SETUP_BLAS(rocsolver_dpotrf_strided_batched(hb, rocblas_fill_lower, n, G, n, nn, info, batch));
  // X = G^-1 C^T E
  k_rhs_rows<<<grid_of(static_cast<long long>(batch) * nk), 256, 0, st>>>(batch, bs, m, n, mn, dpos, C, X);
  SETUP_HIP(hipGetLastError());
  SETUP_BLAS(rocsolver_dpotrs_strided_batched(hb, rocblas_fill_lower, n, bs, G, n, nn, X, n, nk, batch));
  // one refinement step: S = G^-1 C^T (E - C X); X += S
  SETUP_BLAS(rocblas_dgemm_strided_batched(hb, rocblas_operation_none, rocblas_operation_none, m, bs, n, &minus, C,
                                           m, mn, X, n, nk, &zero, Res, m, mk, batch));
  k_add_identity<<<(batch * bs + 255) / 256, 256, 0, st>>>(batch, bs, m, dpos, Res);
  SETUP_HIP(hipGetLastError());
  SETUP_BLAS(rocblas_dgemm_strided_batched(hb, rocblas_operation_transpose, rocblas_operation_none, n, bs, m, &one, C,
                                           m, mn, Res, m, mk, &zero, S, n, nk, batch));
  SETUP_BLAS(rocsolver_dpotrs_strided_batched(hb, rocblas_fill_lower, n, bs, G, n, nn, S, n, nk, batch));
  SETUP_BLAS(rocblas_daxpy(hb, static_cast<rocblas_int>(batch * nk), &one, S, 1, X, 1));
  std::vector<double> hx(static_cast<size_t>(batch) * nk), hs(static_cast<size_t>(batch) * nk);
  std::vector<rocblas_int> hinfo(batch);
  SETUP_HIP(hipMemcpyAsync(hx.data(), X, hx.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  SETUP_HIP(hipMemcpyAsync(hs.data(), S, hs.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  SETUP_HIP(hipMemcpyAsync(hinfo.data(), info, batch * sizeof(rocblas_int), hipMemcpyDeviceToHost, st));
  SETUP_HIP(hipStreamSynchronize(st));
  for (int p = 0; p < batch; ++p) {
    const double* xp = &hx[static_cast<size_t>(p) * nk];
    const double* sp = &hs[static_cast<size_t>(p) * nk];
    double xm = 0.0, sm = 0.0;
    bool finite = hinfo[p] == 0;
    for (long long t = 0; t < nk && finite; ++t) {
      finite = std::isfinite(xp[t]) && std::isfinite(sp[t]);
      xm = std::max(xm, std::fabs(xp[t]));
      sm = std::max(sm, std::fabs(sp[t]));
    }
    if (!finite || !(sm <= 1e-8 * xm)) continue;   // the host solves it by Householder QR
    std::copy(xp, xp + nk, grp[p]->X);
    ok[index[p]] = 1;
  }
}

// one rocBLAS handle and stream per device for the life of the process
// (creating a handle loads the library's kernels: done once)
struct BlasCtx {
  rocblas_handle hb = nullptr;
  hipStream_t st = nullptr;
};

BlasCtx& blas_ctx() {
  static std::mutex mu;
  static std::map<int, BlasCtx> ctx;
  int dev = -1;
  SETUP_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  BlasCtx& c = ctx[dev];
  if (!c.hb) {
    SETUP_HIP(hipStreamCreateWithFlags(&c.st, hipStreamNonBlocking));
    SETUP_BLAS(rocblas_create_handle(&c.hb));
    SETUP_BLAS(rocblas_set_stream(c.hb, c.st));
  }
  return c;
}

}  // namespace

std::vector<char> gpu_sai_solve(SaiBatch& batch) {
  std::vector<SaiProblem>& probs = batch.probs;
  const int bs = batch.bs;
  std::vector<char> ok(probs.size(), 0);
  if (probs.empty()) return ok;
  // one solver at a time per process: the handle and its stream are shared
  static std::mutex serial;
  std::lock_guard<std::mutex> lock(serial);
  BlasCtx& c = blas_ctx();
  // A's pool and the balancing vectors, once for every problem
  std::vector<void*> owned;
  struct Free {
    std::vector<void*>& v;
    ~Free() {
      for (void* p : v) (void)hipFree(p);
    }
  } release{owned};
  const size_t bb = static_cast<size_t>(bs) * bs;
  double* dpool = dalloc<double>(owned, static_cast<size_t>(batch.npool) * bb);
  double* dalpha = dalloc<double>(owned, static_cast<size_t>(batch.nalpha) * bs);
  SETUP_HIP(hipMemcpyAsync(dpool, batch.pool, static_cast<size_t>(batch.npool) * bb * sizeof(double),
                           hipMemcpyHostToDevice, c.st));
  SETUP_HIP(hipMemcpyAsync(dalpha, batch.alpha, static_cast<size_t>(batch.nalpha) * bs * sizeof(double),
                           hipMemcpyHostToDevice, c.st));
  // problems of equal shape, in chunks of at most ~2 GB of device workspace
  std::map<std::pair<int, int>, std::vector<int>> shapes;
  for (size_t u = 0; u < probs.size(); ++u) shapes[{probs[u].mb, probs[u].nb}].push_back(static_cast<int>(u));
  for (auto& kv : shapes) {
    const long long m = static_cast<long long>(kv.first.first) * bs, n = static_cast<long long>(kv.first.second) * bs;
    const long long per = (m * n + n * n + 2 * n * bs + m * bs) * 8 + 64;
    const size_t chunk = static_cast<size_t>(std::max<long long>(1, (2ll << 30) / per));
    const std::vector<int>& ids = kv.second;
    for (size_t c0 = 0; c0 < ids.size(); c0 += chunk) {
      std::vector<SaiProblem*> grp;
      std::vector<int> index;
      for (size_t k = c0; k < std::min(ids.size(), c0 + chunk); ++k) {
        grp.push_back(&probs[ids[k]]);
        index.push_back(ids[k]);
      }
      solve_group(c.hb, c.st, bs, dpool, dalpha, grp, ok, index);
    }
  }
  SETUP_HIP(hipStreamSynchronize(c.st));   // the pool buffers are freed after their last use
  return ok;
}

}  // namespace ldgmg

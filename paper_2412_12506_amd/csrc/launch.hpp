// Launch wrappers of the HIP kernels (kernels.hip).  All pointers are device
// pointers; every wrapper enqueues on `st` and throws std::runtime_error if the
// launch fails.  Sizes are trusted: the callers (device.hip) derive them from
// the hierarchy that allocated the buffers.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"   // storage types (bf16s)

namespace ldgmg {

constexpr int kRedBlocks = 1024;   // partial sums per dot product
constexpr int kRedThreads = 256;
constexpr int kMdotBlocks = 256;   // partial sums per vector of a multi-dot
constexpr int kMaxRhs = 16;        // right-hand sides per multi-vector BSR launch

// block sizes with a specialised (wave-mapped) kernel; others use the generic one
bool fast_bs(int bs);

// elements per vector load in the device block layout for block size bs
inline int device_vec_width(int bs, int elem_bytes) {
  if (!fast_bs(bs)) return 1;
  if (elem_bytes == 8) return bs % 2 == 0 ? 2 : 1;
  if (elem_bytes == 4) return bs % 4 == 0 ? 4 : 1;
  return bs % 8 == 0 ? 8 : bs % 4 == 0 ? 4 : bs % 2 == 0 ? 2 : 1;
}

// TM: element type of the stored blocks; T: vectors and arithmetic
template <typename TM, typename T>
struct BsrArgs {
  int nrows = 0;              // block rows to process
  int bs = 0;
  const int* rows = nullptr;  // optional list of block rows (nrows entries)
  const int* rp = nullptr;    // row pointer [nblockrows + 1]
  const int* ci = nullptr;    // block columns [nnzb]
  const int* tpos = nullptr;  // transposed kernel: slot of (j,i) for slot (i,j)
  const int* bid = nullptr;   // pooled storage: block of each slot [nnzb] (null: slot s owns block s)
  const TM* blk = nullptr;    // blocks [nnzb or pool size][bs*bs], device layout
  const T* x = nullptr;       // input vector
  const T* z = nullptr;       // added vector (MODE 0) / right-hand side (fused smoothing)
  T* out = nullptr;
  T alpha = T(1), beta = T(0);
  const TM* dinv = nullptr;   // fused smoothing: block inverses indexed by block row
  const int* dbid = nullptr;  // pooled block inverses: block of each row (null: row r owns block r)
  // tiled storage (forward products on the matrix cores; used when tab is set,
  // without dinv and rows): pool in the operand layout of k_bsr_tiled, the
  // column offsets and the [nrows][noff] table of pool ids (-1: no block)
  const TM* tblk = nullptr;
  const int* tab = nullptr;
  const int* tperm = nullptr; // block rows ordered by their row of tab, -1 where a tile is padded
  int tnrows = 0;             // entries of tperm (0: nrows)
  const int* trows = nullptr; // the same order unpadded, nrows entries (tiles of fewer than 16 rows)
  const int* toff = nullptr;
  int noff = 0;
  bool p32 = false;           // tiled storage: FP32 products on the matrix cores
  bool tquad = false;         // the tiled pool uses the 4-step k mapping (16 | bs; required for x32)
  bool tpair = false;         // FP32 blocks, FP32 vectors: two tiles per wavefront on large levels (set for the
                              // operator, whose FP32 block loads it halves; the smoother is faster with one)
  const float* x32 = nullptr; // with p32, one right-hand side and 16 | bs: FP32 input in place of x
  float* out2 = nullptr;      // tiled: an FP32 copy of out (rounded to nearest), or null
  float* out32 = nullptr;     // ... or FP32 output in place of out
  T omega = T(1);
};

// expand pooled FP64 blocks (row-major) into the operand layout of the tiled kernel
template <typename T>
void expand_tiled(long long nblk, int bs, const double* pool, T* out, bool transpose, bool quad, hipStream_t st);
// elements per pooled block in that layout
inline long long tiled_block_elems(int bs) { return static_cast<long long>((bs + 15) / 16) * 64 * ((bs + 3) / 4); }

// out = alpha M x + beta z, or (dinv != null) out = x + omega Dinv (z - M x)
template <typename TM, typename T> void bsr_forward(const BsrArgs<TM, T>& a, hipStream_t st);
// the same for nk <= kMaxRhs vectors at x + q*stride, z + q*stride, out + q*stride
template <typename TM, typename T>
void bsr_forward_multi(const BsrArgs<TM, T>& a, long long stride, int nk, hipStream_t st);
// out = alpha M^T x + beta z  (rows must be null; tpos required)
template <typename TM, typename T> void bsr_transposed(const BsrArgs<TM, T>& a, hipStream_t st);
// pooled FP64 row-major blocks -> device layout of T (optionally transposed)
template <typename T>
void expand_blocks(long long nslots, int bs, const int* ids, const double* pool, T* out, bool transpose,
                   hipStream_t st);
// transfers between a level (fine) and the next (coarse, nc elements per side); P1 = the
// 1-D child matrices [2][q1][q1] (sum-factorised kernels when bss <= 64), Ic = the full
// tensor-product child matrices [2^dim][bss][bss] (other block sizes)
template <typename T>
void restrict_op(int dim, int nc, int ncomp, int bss, int q1, const T* P1, const T* Ic, const T* rf, T* rc,
                 hipStream_t st);
// xf32 (optional): an FP32 copy of x_f, written with the result (rounded to nearest)
template <typename T>
void prolong_add(int dim, int nc, int ncomp, int bss, int q1, const T* P1, const T* Ic, const T* xc, T* xf,
                 hipStream_t st, float* xf32 = nullptr);
template <typename T> void dense_gemv(int N, const double* P, const T* in, T* out, hipStream_t st);

void dot_partial(long long n, const double* a, const double* b, double* partial, hipStream_t st);
// op 0: scal[dst] = v;  op 1: scal[dst] = scal[a] / v;  op 2: scal[dst] = v / scal[a], scal[a] = v;
// op 3: scal[dst] = -v;  op 4: op 1, or 0 once scal[kScalFrozen] is set;  op 5: op 2, with 0 for
// scal[dst] while scal[kScalIt] is 0
void finalize(const double* partial, double* scal, int op, int dst, int a, hipStream_t st);
// scalar-table slots of the CG recurrence replayed from a graph
constexpr int kScalFrozen = 9;    // 1 once the recurrence has stopped: alpha is 0 from then on
constexpr int kScalIt = 10;       // iterations done
constexpr int kScalStatus = 11;   // -1 running, 0 iteration limit, 1 converged, 2 guarded stop, 3 breakdown
constexpr int kScalTol2 = 12;     // rtol^2 b.b
constexpr int kScalMaxit = 13;
constexpr int kScalRRFinal = 14;  // r.r when the recurrence stopped
void fill_zero(double* p, long long n, hipStream_t st);
void fill_zero(float* p, long long n, hipStream_t st);
// scal: frozen 0, iterations 0, status -1, tol2 and maxit set
void cg_init(double* scal, double tol2, int maxit, hipStream_t st);
// after an iteration's r.r: count it, record sqrt|r.z| in hist (cap entries),
// and freeze the recurrence on convergence, breakdown, a guarded stop or maxit
void cg_check(double* scal, double* hist, int cap, bool guard, int s_rz, int s_alpha, int s_rr, hipStream_t st);
void cg_update(long long n, double* x, double* r, const double* p, const double* q, const double* scal,
               int ia, double* partial, hipStream_t st);
void cg_dir(long long n, double* p, const double* z, const double* scal, int ib, hipStream_t st);
// y = alpha x + beta y; alpha = scal[ia] if ia >= 0 else the literal (same for beta)
void axpby(long long n, const double* x, double* y, const double* scal, int ia, double alpha, int ib,
           double beta, hipStream_t st);
void scale_invsqrt(long long n, const double* x, double* y, const double* scal, int i, hipStream_t st);
template <typename S, typename D> void cast(long long n, const S* in, D* out, hipStream_t st);
// out[j] = Q_j . w for j < k (Q: k vectors of length n, contiguous); partial: k * kMdotBlocks
void mdot(long long n, int k, const double* Q, const double* w, double* partial, double* out, hipStream_t st);
// w += sign * sum_{j<k} h[j] Q_j   (h on the device)
void maxpy(long long n, int k, const double* Q, const double* h, double sign, double* w, hipStream_t st);

}  // namespace ldgmg

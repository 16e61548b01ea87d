// HIP kernels for gfx950 and their launch wrappers.  Layout and lane mapping:
// kernels.hpp.  Every wrapper enqueues on the given stream and checks the
// launch; bounds are the caller's (launch.hpp documents each wrapper).
#include "kernels.hpp"
#include "launch.hpp"

#include <stdexcept>
#include <cstdint>
#include <type_traits>
#include <string>

namespace ldgmg {

namespace {

template <typename T, int V> struct VecT;
template <> struct VecT<float, 4> { using type = float4; };
template <> struct VecT<float, 1> { using type = float; };
template <> struct VecT<double, 2> { using type = double2; };
template <> struct VecT<double, 1> { using type = double; };

// packed BF16 entries (two per 32-bit word, the lower half first)
struct bf16x2 {
  unsigned int w;
};
struct bf16x4 {
  uint2 w;
};
struct bf16x8 {
  uint4 w;
};
template <> struct VecT<bf16s, 8> { using type = bf16x8; };
template <> struct VecT<bf16s, 4> { using type = bf16x4; };
template <> struct VecT<bf16s, 2> { using type = bf16x2; };
template <> struct VecT<bf16s, 1> { using type = bf16s; };

__device__ __forceinline__ float half_of(unsigned int w, int h) {
  return __uint_as_float(h ? (w & 0xffff0000u) : (w << 16));
}

template <typename T> __device__ __forceinline__ T elem(const T& a, int) { return a; }
__device__ __forceinline__ float elem(const float4& a, int v) {
  return v == 0 ? a.x : v == 1 ? a.y : v == 2 ? a.z : a.w;
}
__device__ __forceinline__ double elem(const double2& a, int v) { return v == 0 ? a.x : a.y; }
__device__ __forceinline__ float elem(const bf16s& a, int) { return __uint_as_float(static_cast<unsigned int>(a.u) << 16); }
__device__ __forceinline__ float elem(const bf16x2& a, int v) { return half_of(a.w, v); }
__device__ __forceinline__ float elem(const bf16x4& a, int v) { return half_of(v < 2 ? a.w.x : a.w.y, v & 1); }
__device__ __forceinline__ float elem(const bf16x8& a, int v) {
  const unsigned int w = v < 2 ? a.w.x : v < 4 ? a.w.y : v < 6 ? a.w.z : a.w.w;
  return half_of(w, v & 1);
}

// stored entry -> arithmetic value (exact)
__device__ __forceinline__ float widen(float a) { return a; }
__device__ __forceinline__ double widen(double a) { return a; }
__device__ __forceinline__ float widen(bf16s a) { return elem(a, 0); }

// FP64 pool value -> stored entry: round to nearest even to FP32, and for BF16
// once more from FP32 to the upper 16 bits
template <typename T> __device__ __forceinline__ T narrow(double v) { return static_cast<T>(v); }
template <> __device__ __forceinline__ bf16s narrow<bf16s>(double v) {
  const unsigned int u = __float_as_uint(static_cast<float>(v));
  bf16s b;
  b.u = static_cast<uint16_t>((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
  return b;
}

template <typename VT> __device__ __forceinline__ VT vzero() { return VT{}; }

__device__ __forceinline__ float readlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ int readlane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ double readlane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), l);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), l);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// value of lane (g*BS + c) of the caller's group
template <typename T, int BS>
__device__ __forceinline__ T group_bcast(T v, int g, int c) {
  if constexpr (64 / BS == 1) return readlane(v, c);
  else return __shfl(v, g * BS + c);
}

constexpr int kWaves = 4;          // wavefronts per workgroup of the BSR kernels
constexpr long long kSplitTiles = 1024;   // below this many tiles: one wavefront per row tile
constexpr long long kPairTiles = 8192;    // from this many: two tiles per wavefront (FP32 blocks)
constexpr int kColSplitRows = 1024;       // at most this many block rows: a workgroup per block row
constexpr int kThreads = 64 * kWaves;

// ---------------------------------------------------------------------------
// forward BSR kernel
//   MODE 0: out_i = alpha (M x)_i + beta z_i            (z read only if beta != 0)
//   MODE 1: out_i = x_i + omega Dinv_i (z_i - (M x)_i)  (fused block-inverse smoothing;
//           out may alias x when the rows of one launch are not coupled)
// rows (optional) lists the block rows to process (nrows entries).
// POOL: blk holds the distinct blocks only and bid[slot] names the block of a
// slot (pooled storage); otherwise slot s owns block s.  dbid (optional) names
// the block inverse of a row in the same way.
// ---------------------------------------------------------------------------
template <typename TM, typename T, int BS, int MODE, bool POOL>
__global__ __launch_bounds__(kThreads) void k_bsr_fwd(int nrows, const int* __restrict__ rows,
                                                      const int* __restrict__ rp,
                                                      const int* __restrict__ ci,
                                                      const int* __restrict__ bid,
                                                      const TM* __restrict__ blk, const T* x,
                                                      const T* z, T* out, T alpha, T beta,
                                                      const TM* __restrict__ dinv,
                                                      const int* __restrict__ dbid, T omega) {
  using C = BlkCfg<TM, BS>;
  constexpr int V = C::V, G = C::G, NV = C::NV;
  constexpr int CH = BS < 8 ? BS : 8;   // slots whose column index and x entry are fetched together
  constexpr int NA = 4;                 // independent accumulators (breaks the FMA dependency chain)
  using VT = typename VecT<TM, V>::type;
  // Every load below is unconditional from an address that is valid for every
  // lane (idle lanes and missing slots point at row 0 / slot 0) and the unwanted
  // values are masked afterwards: a load inside a divergent branch forces a
  // wait for it before the branch joins, which would serialise the block loads.
  const int lane = threadIdx.x & 63;
  const int g = lane / BS;
  const int r = lane - g * BS;
  const int wave = blockIdx.x * kWaves + (threadIdx.x >> 6);
  const int idx = wave * G + g;
  const bool active = (g < G) && (idx < nrows);
  const int ridx = active ? idx : 0;
  const int row_l = rows ? rows[ridx] : ridx;
  const int row = active ? row_l : 0;
  const int s0 = rp[row];
  const int cnt = active ? rp[row + 1] - s0 : 0;
  int mc = cnt;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) mc = max(mc, __shfl_xor(mc, o));
  T acc[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) acc[i] = T(0);
  for (int k0 = 0; k0 < mc; k0 += CH) {
    // lane t < CH of each group fetches the column of slot k0 + t; every lane
    // then fetches its entries of those CH neighbour vectors, so the block
    // loads below wait for one memory latency only
    const bool own = r < CH && k0 + r < cnt;
    const int so = own ? s0 + k0 + r : 0;
    const int cl = ci[so];
    const int cidx = own ? cl : -1;
    int pid = 0;                            // pooled: block of slot k0 + r (slot 0's if none)
    if constexpr (POOL) pid = bid[so];
    T xv[CH];
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      const int j = group_bcast<int, BS>(cidx, g, t);
      const T xl = x[static_cast<size_t>(j >= 0 ? j : 0) * BS + r];
      xv[t] = j >= 0 ? xl : T(0);            // missing slot: multiplier 0
    }
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      if (k0 + t >= mc) break;                // wave-uniform
      size_t boff;
      if constexpr (POOL) {
        boff = static_cast<size_t>(group_bcast<int, BS>(pid, g, t)) * (BS * BS);
      } else {
        const int sl = k0 + t < cnt ? s0 + k0 + t : 0;
        boff = static_cast<size_t>(sl) * (BS * BS);
      }
      const VT* bp = reinterpret_cast<const VT*>(blk + boff) + r;
      VT a[NV];
#pragma unroll
      for (int q = 0; q < NV; ++q) a[q] = bp[q * BS];
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        // keep the widening of each loaded vector next to its use (otherwise the
        // scheduler widens the whole block at once and doubles the registers)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int v = 0; v < V; ++v)
          acc[(q * V + v) % NA] += static_cast<T>(elem(a[q], v)) * group_bcast<T, BS>(xv[t], g, q * V + v);
      }
    }
  }
  T sum = acc[0];
#pragma unroll
  for (int i = 1; i < NA; ++i) sum += acc[i];
  const size_t o = static_cast<size_t>(row) * BS + r;
  if constexpr (MODE == 1) {
    const T zo = z[o];
    const T res = active ? zo - sum : T(0);
    VT d[NV];
    const int drow = dbid ? dbid[row] : row;
    const VT* dp = reinterpret_cast<const VT*>(dinv + static_cast<size_t>(drow) * (BS * BS)) + r;
#pragma unroll
    for (int q = 0; q < NV; ++q) d[q] = dp[q * BS];
    T y[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) y[i] = T(0);
#pragma unroll
    for (int q = 0; q < NV; ++q) {
#pragma unroll
      for (int v = 0; v < V; ++v)
        y[(q * V + v) % NA] += static_cast<T>(elem(d[q], v)) * group_bcast<T, BS>(res, g, q * V + v);
    }
    T ys = y[0];
#pragma unroll
    for (int i = 1; i < NA; ++i) ys += y[i];
    const T xo = x[o];
    if (active) out[o] = xo + omega * ys;
  } else {
    if (beta != T(0)) {
      const T zo = z[o];
      if (active) out[o] = alpha * sum + beta * zo;
    } else {
      if (active) out[o] = alpha * sum;
    }
  }
}

// ---------------------------------------------------------------------------
// forward BSR kernel for matrices with few block rows (MODE 0; 16 | bs, bs >
// 32): the kWaves wavefronts of a workgroup share one block row, each taking a
// quarter of every block's columns, and add their partial rows in LDS.  A
// wavefront issues the block loads of up to CH slots before its first product,
// so a row costs about one memory latency per CH slots where the per-row
// kernel waits once per slot; on small levels nothing else hides those waits.
// ---------------------------------------------------------------------------
template <typename TM, typename T, int BS, bool POOL>
__global__ __launch_bounds__(kThreads) void k_bsr_fwd_cs(int nrows, const int* __restrict__ rows,
                                                         const int* __restrict__ rp,
                                                         const int* __restrict__ ci,
                                                         const int* __restrict__ bid,
                                                         const TM* __restrict__ blk, const T* x, const T* z,
                                                         T* out, T alpha, T beta) {
  using C = BlkCfg<TM, BS>;
  constexpr int V = C::V, NV = C::NV;
  static_assert(C::G == 1 && NV % kWaves == 0, "one block row per workgroup, columns in kWaves groups");
  constexpr int NQ = NV / kWaves;                // vector loads per slot and wavefront
  constexpr int NC = NQ * V;                     // columns per wavefront
  constexpr int CH = sizeof(TM) == 8 ? 4 : 8;    // slots whose loads are in flight together
  constexpr int NA = 4;
  using VT = typename VecT<TM, V>::type;
  __shared__ T part[kWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane < BS ? lane : 0;            // lanes past bs mirror row 0 and write nothing
  const int idx = blockIdx.x;                    // one block row per workgroup (grid = nrows)
  const int row = rows ? rows[idx] : idx;
  const int s0 = rp[row];
  const int cnt = rp[row + 1] - s0;
  const int cx = w * NC + (lane < NC ? lane : 0);   // lane l < NC holds column w NC + l of x
  T acc[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) acc[i] = T(0);
  for (int k0 = 0; k0 < cnt; k0 += CH) {
    VT a[CH][NQ];
    T xv[CH];
    // every load from a valid slot (clamped); a slot past the row's last one
    // gets x = 0, so no branch separates the loads from the products
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      const bool in = k0 + t < cnt;
      const int sl = in ? s0 + k0 + t : s0;
      const size_t boff = static_cast<size_t>(POOL ? bid[sl] : sl) * (BS * BS);
      const VT* bp = reinterpret_cast<const VT*>(blk + boff) + r;
#pragma unroll
      for (int q = 0; q < NQ; ++q) a[t][q] = bp[(w * NQ + q) * BS];
      const T xl = x[static_cast<size_t>(ci[sl]) * BS + cx];
      xv[t] = in ? xl : T(0);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < CH; ++t) {
#pragma unroll
      for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int v = 0; v < V; ++v)
          acc[(q * V + v) % NA] += static_cast<T>(elem(a[t][q], v)) * readlane(xv[t], q * V + v);
    }
  }
  T sum = acc[0];
#pragma unroll
  for (int i = 1; i < NA; ++i) sum += acc[i];
  part[w][lane] = sum;
  __syncthreads();
  if (w == 0 && lane < BS) {
    T y = part[0][lane];
#pragma unroll
    for (int i = 1; i < kWaves; ++i) y += part[i][lane];
    const size_t o = static_cast<size_t>(row) * BS + lane;
    out[o] = beta != T(0) ? alpha * y + beta * z[o] : alpha * y;
  }
}

// ---------------------------------------------------------------------------
// multi-right-hand-side forward BSR kernel: out_q = alpha (M x_q) + beta z_q for
// q < nk <= kMaxRhs vectors stored with a stride.  Each block is read from HBM
// once for all right-hand sides; a lane's entries of the nk neighbour vectors
// are staged in LDS ([slot][rhs]) and read back as broadcasts, so a column of
// a block costs one widening and nk FP64 FMAs.  (On gfx950 FP64 matrix cores
// have the same rate as FP64 vector FMA, so the FP64 accumulation that keeps
// the Krylov iteration counts stays on the vector units.)
// ---------------------------------------------------------------------------
template <typename TM, typename T, int BS>
__global__ __launch_bounds__(kThreads) void k_bsr_fwd_multi(int nrows, const int* __restrict__ rows,
                                                            const int* __restrict__ rp,
                                                            const int* __restrict__ ci,
                                                            const int* __restrict__ bid,
                                                            const TM* __restrict__ blk, const T* x,
                                                            const T* z, T* out, long long stride, int nk,
                                                            T alpha, T beta) {
  using C = BlkCfg<TM, BS>;
  constexpr int V = C::V, G = C::G, NV = C::NV;
  using VT = typename VecT<TM, V>::type;
  __shared__ T xs[kWaves][64][kMaxRhs];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int g = lane / BS;
  const int r = lane - g * BS;
  const int wave = blockIdx.x * kWaves + wid;
  const int idx = wave * G + g;
  const bool active = (g < G) && (idx < nrows);
  const int ridx = active ? idx : 0;
  const int row_l = rows ? rows[ridx] : ridx;
  const int row = active ? row_l : 0;
  const int s0 = rp[row];
  const int cnt = active ? rp[row + 1] - s0 : 0;
  int mc = cnt;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) mc = max(mc, __shfl_xor(mc, o));
  T acc[kMaxRhs];
#pragma unroll
  for (int q = 0; q < kMaxRhs; ++q) acc[q] = T(0);
  for (int k = 0; k < mc; ++k) {
    const bool has = k < cnt;
    const int sl = has ? s0 + k : 0;
    const int j = ci[sl];
#pragma unroll
    for (int q = 0; q < kMaxRhs; ++q) {
      if (q < nk) {                                  // nk is uniform
        const T xv = x[q * stride + static_cast<long long>(j) * BS + r];
        xs[wid][lane][q] = has ? xv : T(0);
      }
    }
    // make this wavefront's LDS writes visible to its other lanes
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int pb = bid ? bid[sl] : sl;          // pooled storage: block of the slot
    const VT* bp = reinterpret_cast<const VT*>(blk + static_cast<size_t>(pb) * (BS * BS)) + r;
    VT a[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) a[q] = bp[q * BS];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const T av = static_cast<T>(elem(a[q], v));
        const T* xc = &xs[wid][g * BS + q * V + v][0];
#pragma unroll
        for (int qq = 0; qq < kMaxRhs; ++qq)
          if (qq < nk) acc[qq] += av * xc[qq];
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  const long long o = static_cast<long long>(row) * BS + r;
#pragma unroll
  for (int q = 0; q < kMaxRhs; ++q) {
    if (q < nk) {
      if (beta != T(0)) {
        const T zo = z[q * stride + o];
        if (active) out[q * stride + o] = alpha * acc[q] + beta * zo;
      } else {
        if (active) out[q * stride + o] = alpha * acc[q];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// transposed BSR kernel: out_i = alpha sum_{(i,j) stored} (M_ji)^T x_j + beta z_i.
// tpos[s] is the slot of block (j, i) for slot s = (i, j) (symmetric pattern).
// Lane r accumulates row r of each (M_ji) scaled by x_j[r]; the BS partial
// vectors of a group are then summed across lanes.
// ---------------------------------------------------------------------------
template <typename TM, typename T, int BS>
__global__ __launch_bounds__(kThreads) void k_bsr_tr(int nrows, const int* __restrict__ rp,
                                                     const int* __restrict__ ci,
                                                     const int* __restrict__ tpos,
                                                     const TM* __restrict__ blk, const T* x,
                                                     const T* z, T* out, T alpha, T beta) {
  using C = BlkCfg<TM, BS>;
  constexpr int V = C::V, G = C::G, NV = C::NV;
  constexpr bool POW2 = (BS & (BS - 1)) == 0;
  using VT = typename VecT<TM, V>::type;
  const int lane = threadIdx.x & 63;
  const int g = lane / BS;
  const int r = lane - g * BS;
  const int wid = threadIdx.x >> 6;
  const int wave = blockIdx.x * kWaves + wid;
  const int idx = wave * G + g;
  const bool active = (g < G) && (idx < nrows);
  const int row = active ? idx : 0;
  const int s0 = rp[row];
  const int cnt = active ? rp[row + 1] - s0 : 0;
  int mc = cnt;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) mc = max(mc, __shfl_xor(mc, o));
  T acc[BS];
#pragma unroll
  for (int c = 0; c < BS; ++c) acc[c] = T(0);
  for (int k = 0; k < mc; ++k) {
    const bool has = k < cnt;
    const int s = has ? s0 + k : 0;
    const int t = tpos[s];
    const int j = ci[s];
    const T xl = x[static_cast<size_t>(j) * BS + r];
    const T xr = has ? xl : T(0);
    const VT* bp = reinterpret_cast<const VT*>(blk + static_cast<size_t>(t) * (BS * BS)) + r;
    VT a[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) a[q] = bp[q * BS];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
#pragma unroll
      for (int v = 0; v < V; ++v) acc[q * V + v] += static_cast<T>(elem(a[q], v)) * xr;
    }
  }
  T y;
  if constexpr (POW2) {
    // butterfly transpose-reduction inside the aligned group of BS lanes:
    // after the stage with offset o the lane keeps the half selected by bit o
    // of its index, so lane r ends with the sum for column r.
#pragma unroll
    for (int o = BS / 2; o >= 1; o >>= 1) {
      const bool upper = (r & o) != 0;
#pragma unroll
      for (int i = 0; i < o; ++i) {
        const T mine = upper ? acc[i + o] : acc[i];
        const T send = upper ? acc[i] : acc[i + o];
        acc[i] = mine + __shfl_xor(send, o);
      }
    }
    y = acc[0];
  } else {
    __shared__ T red[kWaves][G][BS][BS + 1];
    if (g < G) {
#pragma unroll
      for (int c = 0; c < BS; ++c) red[wid][g][r][c] = acc[c];
    }
    __syncthreads();
    y = T(0);
    if (g < G) {
      for (int rr = 0; rr < BS; ++rr) y += red[wid][g][rr][r];
    }
  }
  if (active) {
    const size_t o = static_cast<size_t>(row) * BS + r;
    out[o] = beta != T(0) ? alpha * y + beta * z[o] : alpha * y;
  }
}

// ---------------------------------------------------------------------------
// tiled forward BSR kernel on the matrix cores: out = alpha M x + beta z
// for a pooled matrix addressed by column offset, for nk <= 16 right-hand sides
// (vectors q at x + q stride, z + q stride, out + q stride).  tab[row * noff +
// d] is the pool id of block (row, row + off[d]) or -1; perm lists the block
// rows ordered by their row of tab (rows with the same blocks are adjacent).
// The 16 columns of an MFMA tile are (row, right-hand side) pairs: with kp the
// power of two >= nk, a wavefront takes the 16 / kp block rows
// perm[e0 .. e0 + 16 / kp - 1] and column c = (row c / kp, vector c % kp).  For
// each offset it groups the columns by block id and accumulates
// Y(bs x 16) += B(bs x bs) X(bs x 16), column c of X being its vector's block at
// the row + off[d] (zero outside the group), with v_mfma_f64_16x16x4f64
// (products and sums in FP64) or v_mfma_f32_16x16x4f32 (FP32 products).
// MFMA operands: A lane l = (row l % 16, k lane l / 16), B lane l = (k lane
// l / 16, column l % 16); result lane l = rows l / 16 + 4 i (FP64) or
// 4 (l / 16) + i (FP32), i < 4, of column l % 16.
// With MT = ceil(bs/16) row tiles and KS = ceil(bs/4) k steps, k lane q of
// step s takes the block column tile_k(s, q): for a matrix laid out for FP32
// x ("quad", 16 | bs) 16 (s / 4) + 4 q + s % 4, so that steps 4j .. 4j+3 of a
// lane are 4 contiguous entries of x (one 16-byte load of FP32 x, two of
// FP64); otherwise 8 (s / 2) + 2 q + s % 2 when 8 divides bs (the four k lanes
// of a column read 64 contiguous bytes of FP64 x per 16-byte load), else
// q KS + s.
// Pool layout, E entries per 16 bytes (E = 16 / entry size when E divides KS,
// else 1): entry [block][m][s / E][lane][s % E] = B(16 m + lane % 16,
// tile_k(s, lane / 16)), zero outside the block; one 16-byte load of a
// wavefront reads 1 KB contiguously.
// ---------------------------------------------------------------------------
typedef double v4d __attribute__((ext_vector_type(4)));

typedef float v4f __attribute__((ext_vector_type(4)));

typedef unsigned int v4u __attribute__((ext_vector_type(4)));

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// entries per 16-byte group of the pool layout
template <typename TM>
__host__ __device__ constexpr int tile_vec(int KS) {
  return KS % (16 / static_cast<int>(sizeof(TM))) == 0 ? 16 / static_cast<int>(sizeof(TM)) : 1;
}

// block column of k lane q at step s
__host__ __device__ constexpr int tile_k(int bs, int KS, int s, int q, bool quad) {
  return quad && bs % 16 == 0 ? 16 * (s >> 2) + 4 * q + (s & 3)
                              : bs % 8 == 0 ? 8 * (s >> 1) + 2 * q + (s & 1) : q * KS + s;
}

// the KS operands of this lane in row tile p (= pool block + m 64 KS), widened
// to the operand type OP (FP64, or FP32 for stored FP32 / BF16: exact either way)
template <typename TM, int KS, typename OP>
__device__ __forceinline__ void load_widen(const TM* p, int lane, OP (&out)[KS]) {
  constexpr int E = tile_vec<TM>(KS);
  if constexpr (E > 1) {
    using VT = typename VecT<TM, E>::type;
    const VT* v = reinterpret_cast<const VT*>(p) + lane;
#pragma unroll
    for (int q = 0; q < KS / E; ++q) {
      const VT w = v[q * 64];
#pragma unroll
      for (int e = 0; e < E; ++e) out[q * E + e] = static_cast<OP>(elem(w, e));
    }
  } else {
#pragma unroll
    for (int s = 0; s < KS; ++s) out[s] = static_cast<OP>(widen(p[s * 64 + lane]));
  }
}

// one 16x16x4 MFMA step: FP64, or FP32 operands with FP32 accumulation
__device__ __forceinline__ v4d mfma_step(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma_step(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// FP32 x split into three BF16 parts, x = hi + mid + lo: hi keeps the top 8
// significand bits (truncated), mid the next 8 of the remainder, lo the last 8
// (the remainders are exact in FP32 and lo fits a BF16 exactly when
// |x| >= 2^-103; below that lo may be subnormal and loses under 2^-133).  Each
// group of 8 steps 8c .. 8c+7 becomes one 8-element operand per part.
template <int KS>
__device__ __forceinline__ void split_bf16x3(const float (&f)[KS], v8bf (&xs)[3][KS / 8]) {
#pragma unroll
  for (int c = 0; c < KS / 8; ++c) {
    unsigned w[3][8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float v = f[8 * c + e];
      const unsigned uh = __float_as_uint(v) & 0xFFFF0000u;
      const float r1 = v - __uint_as_float(uh);
      const unsigned um = __float_as_uint(r1) & 0xFFFF0000u;
      const float r2 = r1 - __uint_as_float(um);
      w[0][e] = uh;
      w[1][e] = um;
      w[2][e] = __float_as_uint(r2);
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const v4u p{(w[t][0] >> 16) | (w[t][1] & 0xFFFF0000u), (w[t][2] >> 16) | (w[t][3] & 0xFFFF0000u),
                  (w[t][4] >> 16) | (w[t][5] & 0xFFFF0000u), (w[t][6] >> 16) | (w[t][7] & 0xFFFF0000u)};
      xs[t][c] = __builtin_bit_cast(v8bf, p);
    }
  }
}

// the KS operands of the x block at xp for k lane kq (zero when !use), in the
// k mapping of the pool layout
template <int BS, int KS, bool QUAD, typename XT, typename OP>
__device__ __forceinline__ void load_x(const XT* xp, int kq, bool use, OP (&xb)[KS]) {
  if constexpr (QUAD && std::is_same<XT, float>::value) {   // steps 4j..4j+3: one 16-byte load
    const float4* x4 = reinterpret_cast<const float4*>(xp + 4 * kq);
#pragma unroll
    for (int j = 0; j < KS / 4; ++j) {
      const float4 v = x4[4 * j];
      xb[4 * j] = use ? v.x : OP(0);
      xb[4 * j + 1] = use ? v.y : OP(0);
      xb[4 * j + 2] = use ? v.z : OP(0);
      xb[4 * j + 3] = use ? v.w : OP(0);
    }
  } else if constexpr (QUAD) {   // steps 4j..4j+3: columns 16j + 4 kq + {0..3}, two 16-byte loads
    const double2* x2 = reinterpret_cast<const double2*>(xp + 4 * kq);
#pragma unroll
    for (int j = 0; j < KS / 4; ++j) {
      const double2 v0 = x2[8 * j], v1 = x2[8 * j + 1];
      xb[4 * j] = use ? static_cast<OP>(v0.x) : OP(0);
      xb[4 * j + 1] = use ? static_cast<OP>(v0.y) : OP(0);
      xb[4 * j + 2] = use ? static_cast<OP>(v1.x) : OP(0);
      xb[4 * j + 3] = use ? static_cast<OP>(v1.y) : OP(0);
    }
  } else if constexpr (BS % 8 == 0) {    // steps 2j, 2j+1: columns 8j + 2 kq + {0, 1}, one 16-byte load
    const double2* x2 = reinterpret_cast<const double2*>(xp + 2 * kq);
#pragma unroll
    for (int q = 0; q < KS / 2; ++q) {
      const double2 v = x2[4 * q];
      xb[2 * q] = use ? static_cast<OP>(v.x) : OP(0);
      xb[2 * q + 1] = use ? static_cast<OP>(v.y) : OP(0);
    }
  } else {
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int c = tile_k(BS, KS, s, kq, QUAD);
      const double v = xp[c < BS ? c : 0];
      xb[s] = (use && c < BS) ? static_cast<OP>(v) : OP(0);
    }
  }
}

// the epilogue of k_bsr_tiled for one tile: out = alpha Y + beta z (and the
// FP32 copy out2 when given) for the rows of block row rb / BS held by this
// lane
template <int BS, bool P32, int MW, typename OT, typename ACC>
__device__ __forceinline__ void tiled_store(const ACC (&acc)[MW], size_t rb, int mw, int kq, OT* out,
                                            const double* z, double alpha, double beta,
                                            float* __restrict__ out2) {
  if constexpr (P32 && BS % 16 == 0) {
    // FP32 result layout: lane l holds rows 16 m + 4 (l/16) + i, four
    // consecutive entries per row tile: with 16-byte aligned out and z (a
    // wavefront-uniform test) every z load is issued before the first use and
    // the results leave in 16-byte stores
    if (((reinterpret_cast<uintptr_t>(out) | reinterpret_cast<uintptr_t>(z)) & 15) == 0) {
      double y[MW][4];
#pragma unroll
      for (int m = 0; m < MW; ++m)
#pragma unroll
        for (int i = 0; i < 4; ++i) y[m][i] = alpha * static_cast<double>(acc[m][i]);
      if (beta != 0.0) {
        double2 zv[MW][2];
#pragma unroll
        for (int m = 0; m < MW; ++m) {
          const double2* zp = reinterpret_cast<const double2*>(z + rb + 16 * (mw + m) + 4 * kq);
          zv[m][0] = zp[0];
          zv[m][1] = zp[1];
        }
#pragma unroll
        for (int m = 0; m < MW; ++m) {
          y[m][0] = __builtin_fma(beta, zv[m][0].x, y[m][0]);
          y[m][1] = __builtin_fma(beta, zv[m][0].y, y[m][1]);
          y[m][2] = __builtin_fma(beta, zv[m][1].x, y[m][2]);
          y[m][3] = __builtin_fma(beta, zv[m][1].y, y[m][3]);
        }
      }
#pragma unroll
      for (int m = 0; m < MW; ++m) {
        OT* op = out + rb + 16 * (mw + m) + 4 * kq;
        if constexpr (std::is_same<OT, float>::value) {
          *reinterpret_cast<float4*>(op) = float4{static_cast<float>(y[m][0]), static_cast<float>(y[m][1]),
                                                  static_cast<float>(y[m][2]), static_cast<float>(y[m][3])};
        } else {
          reinterpret_cast<double2*>(op)[0] = double2{y[m][0], y[m][1]};
          reinterpret_cast<double2*>(op)[1] = double2{y[m][2], y[m][3]};
          if (out2)                          // the FP32 copy (wavefront-uniform test)
            *reinterpret_cast<float4*>(out2 + rb + 16 * (mw + m) + 4 * kq) =
                float4{static_cast<float>(y[m][0]), static_cast<float>(y[m][1]), static_cast<float>(y[m][2]),
                       static_cast<float>(y[m][3])};
        }
      }
      return;
    }
  }
#pragma unroll
  for (int m = 0; m < MW; ++m)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      // result layout: FP64 lane l holds rows l/16 + 4i, FP32 rows 4(l/16) + i
      const int r = 16 * (mw + m) + (P32 ? 4 * kq + i : kq + 4 * i);
      if (r < BS) {
        const double y = alpha * static_cast<double>(acc[m][i]);
        const OT v = static_cast<OT>(beta != 0.0 ? __builtin_fma(beta, z[rb + r], y) : y);
        out[rb + r] = v;
        if (out2) out2[rb + r] = static_cast<float>(v);
      }
    }
}

// P32: FP32 products (operands rounded to FP32: the stored FP32 / BF16 entries
// exactly, the vector entries to nearest) accumulated in FP32; the result is
// combined with z in FP64.  XT / OT: element type of x / out; FP32 x (already
// rounded by its producer, so the same operand values) or FP32 out only with
// FP32 products, one right-hand side and 16 | bs.  QUAD: the matrix is laid out
// with the 4-step k mapping (required for FP32 x).  SPLIT: one wavefront per
// row tile of a tile (MT wavefronts per tile, one right-hand side), for
// matrices with too few tiles to fill the device; the products are the same.
// NG: consecutive tiles per wavefront (1 or 2; 2 with FP32 products and one
// right-hand side): a pass loads the block operands once and multiplies them
// with the x columns of every tile (zero columns where a tile's rows do not
// hold that block), halving the block loads per MFMA.
template <typename TM, int BS, int LKP, bool P32, typename XT = double, typename OT = double, bool QUAD = false,
          bool SPLIT = false, int NG = 1>
__global__ __launch_bounds__(kThreads) void k_bsr_tiled(int nrows, int noff, const int* __restrict__ off,
                                                        const int* __restrict__ tab,
                                                        const int* __restrict__ perm,
                                                        const TM* __restrict__ blk, const XT* x,
                                                        const double* z, OT* out, double alpha,
                                                        double beta, long long stride, int nk,
                                                        float* __restrict__ out2) {
  static_assert(std::is_same<XT, double>::value || (P32 && QUAD && BS % 16 == 0), "FP32 x: FP32 products, quad layout");
  static_assert(!QUAD || BS % 16 == 0, "the quad layout needs 16 | bs");
  static_assert(!SPLIT || LKP == 0, "one wavefront per row tile: one right-hand side");
  static_assert(NG == 1 || (NG == 2 && P32 && !SPLIT && LKP == 0), "two tiles per wavefront: FP32 products, one vector");
  constexpr int MT = (BS + 15) / 16, KS = (BS + 3) / 4;
  constexpr int MW = SPLIT ? 1 : MT;            // row tiles of this wavefront
  constexpr int MG = SPLIT ? 1 : sizeof(TM) == 8 ? 1 : 4;   // row tiles whose operands are held at once
  using OP = typename std::conditional<P32, float, double>::type;
  using ACC = typename std::conditional<P32, v4f, v4d>::type;
  // BF16 blocks times FP32 x on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16)
  constexpr bool BFX = std::is_same<TM, bf16s>::value && std::is_same<XT, float>::value && QUAD && KS % 8 == 0;
  const int lane = threadIdx.x & 63;
  // workgroups are dealt to the 8 XCDs in turn: give each XCD a contiguous
  // range of tiles so that neighbouring rows share its L2
  const int nb = gridDim.x, n8 = nb >> 3;
  const int b = blockIdx.x;
  const int lb = b < 8 * n8 ? (b & 7) * n8 + (b >> 3) : b;
  const int wv = lb * kWaves + (threadIdx.x >> 6);
  const int tile = SPLIT ? wv / MT : wv * NG;
  const int mw = SPLIT ? wv - tile * MT : 0;   // first row tile of this wavefront
  const int e0 = tile * (16 >> LKP);        // 16 / kp block rows per tile
  if (e0 >= nrows) return;                  // the whole wavefront; no barrier follows
  const int col = lane & 15, kq = lane >> 4;
  const int q = col & ((1 << LKP) - 1);     // right-hand side of this column
  int rowg[NG];
  bool rvg[NG];
#pragma unroll
  for (int h = 0; h < NG; ++h) {            // tile h of this wavefront
    const int e = e0 + 16 * h + (col >> LKP);
    const int pr = e < nrows ? perm[e] : -1;  // -1: a padded place of the tile order
    rvg[h] = pr >= 0 && q < nk;
    rowg[h] = rvg[h] ? pr : 0;
  }
  const size_t qoff = static_cast<size_t>(rvg[0] ? q : 0) * stride;
  ACC acc[NG][MW];
#pragma unroll
  for (int h = 0; h < NG; ++h)
#pragma unroll
    for (int m = 0; m < MW; ++m) acc[h][m] = ACC{0, 0, 0, 0};
  for (int d = 0; d < noff; ++d) {
    const int o = off[d];
    int myid[NG];
    unsigned long long rem[NG], left = 0;
#pragma unroll
    for (int h = 0; h < NG; ++h) {
      const int t = tab[static_cast<size_t>(rowg[h]) * noff + d];
      myid[h] = rvg[h] ? t : -1;
      rem[h] = __ballot(myid[h] >= 0) & 0xFFFFull;
      left |= rem[h];
    }
    while (left) {                          // one MFMA pass per distinct block of this offset
      int id = -1;
#pragma unroll
      for (int h = NG - 1; h >= 0; --h)      // a block not yet served, first tile first
        if (rem[h]) id = __shfl(myid[h], __ffsll(static_cast<long long>(rem[h])) - 1);
      OP xb[NG][KS];
      left = 0;
#pragma unroll
      for (int h = 0; h < NG; ++h) {
        const unsigned long long sel = __ballot(myid[h] == id) & 0xFFFFull;
        const bool use = (sel >> col) & 1ull;
        load_x<BS, KS, QUAD>(x + (use ? qoff + static_cast<size_t>(rowg[h] + o) * BS : 0), kq, use, xb[h]);
        rem[h] &= ~sel;
        left |= rem[h];
      }
      const TM* bp = blk + static_cast<size_t>(id) * (MT * 64 * KS) + static_cast<size_t>(mw) * 64 * KS;
      if constexpr (BFX) {
        // BF16 blocks and FP32 x: a 16-byte pool group holds a lane's steps
        // 8c .. 8c+7 and is the block operand as stored; x enters as its three
        // exact BF16 parts, so every product is exact and the sums are FP32
        v8bf ab[MW][KS / 8];
        const v4u* g4 = reinterpret_cast<const v4u*>(bp) + lane;
#pragma unroll
        for (int m = 0; m < MW; ++m)
#pragma unroll
          for (int c = 0; c < KS / 8; ++c) ab[m][c] = __builtin_bit_cast(v8bf, g4[(m * (KS / 8) + c) * 64]);
#pragma unroll
        for (int h = 0; h < NG; ++h) {
          v8bf xs[3][KS / 8];
          split_bf16x3<KS>(xb[h], xs);
#pragma unroll
          for (int c = 0; c < KS / 8; ++c)
#pragma unroll
            for (int t = 2; t >= 0; --t)
#pragma unroll
              for (int m = 0; m < MW; ++m)
                acc[h][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab[m][c], xs[t][c], acc[h][m], 0, 0, 0);
        }
        continue;
      }
      // MG row tiles at a time: their operands are loaded first and their
      // independent accumulations interleaved, so no MFMA waits on the last
#pragma unroll
      for (int m0 = 0; m0 < MW; m0 += MG) {
        OP a[MG][KS];
#pragma unroll
        for (int g = 0; g < MG; ++g)
          if (m0 + g < MW) load_widen<TM, KS, OP>(bp + (m0 + g) * 64 * KS, lane, a[g]);
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
          for (int h = 0; h < NG; ++h)
#pragma unroll
            for (int g = 0; g < MG; ++g)
              if (m0 + g < MW) acc[h][m0 + g] = mfma_step(a[g][s], xb[h][s], acc[h][m0 + g]);
      }
    }
  }
#pragma unroll
  for (int h = 0; h < NG; ++h) {
    if (rvg[h]) tiled_store<BS, P32, MW, OT>(acc[h], qoff + static_cast<size_t>(rowg[h]) * BS, mw, kq, out, z,
                                             alpha, beta, out2);
  }
}

// pooled blocks (row-major FP64) -> the operand layout of k_bsr_tiled
template <typename T>
__global__ void k_expand_tiled(long long nblk, int bs, int MT, int KS, const double* __restrict__ pool,
                               T* __restrict__ out, int transpose, int quad) {
  const long long per = static_cast<long long>(MT) * 64 * KS;
  const long long bb = static_cast<long long>(bs) * bs;
  for (long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; t < nblk * per;
       t += static_cast<long long>(gridDim.x) * blockDim.x) {
    const long long b = t / per;
    const int rem = static_cast<int>(t - b * per);
    const int E = tile_vec<T>(KS);
    const int e = rem % E;
    const int l = (rem / E) % 64;
    const int gq = rem / (64 * E);          // m KS / E + s / E
    const int m = gq / (KS / E);
    const int s = (gq % (KS / E)) * E + e;
    const int r = 16 * m + l % 16, c = tile_k(bs, KS, s, l / 16, quad != 0);
    double v = 0.0;
    if (r < bs && c < bs) v = transpose ? pool[b * bb + static_cast<long long>(c) * bs + r] : pool[b * bb + static_cast<long long>(r) * bs + c];
    out[t] = narrow<T>(v);
  }
}

// generic BSR kernel for any block size: one lane per scalar row.
// Blocks use the V = 1 layout (entry (r, c) at c * bs + r).
template <typename TM, typename T>
__global__ __launch_bounds__(256) void k_bsr_generic(int nrows, int bs, const int* __restrict__ rows,
                                                     const int* __restrict__ rp,
                                                     const int* __restrict__ ci,
                                                     const int* __restrict__ tpos,
                                                     const TM* __restrict__ blk, const T* x,
                                                     const T* z, T* out, T alpha, T beta) {
  const long long tid = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  const long long idx = tid / bs;
  const int r = static_cast<int>(tid - idx * bs);
  if (idx >= nrows) return;
  const int row = rows ? rows[idx] : static_cast<int>(idx);
  T acc = T(0);
  const size_t bb = static_cast<size_t>(bs) * bs;
  for (int s = rp[row]; s < rp[row + 1]; ++s) {
    const int j = ci[s];
    const T* xj = x + static_cast<size_t>(j) * bs;
    if (tpos) {   // (M_ji)^T[r][c] = M_ji[c][r], stored at r * bs + c
      const TM* b = blk + static_cast<size_t>(tpos[s]) * bb + static_cast<size_t>(r) * bs;
      for (int c = 0; c < bs; ++c) acc += static_cast<T>(widen(b[c])) * xj[c];
    } else {
      const TM* b = blk + static_cast<size_t>(s) * bb + r;
      for (int c = 0; c < bs; ++c) acc += static_cast<T>(widen(b[static_cast<size_t>(c) * bs])) * xj[c];
    }
  }
  const size_t o = static_cast<size_t>(row) * bs + r;
  out[o] = beta != T(0) ? alpha * acc + beta * z[o] : alpha * acc;
}

// expand pooled FP64 blocks (row-major) into the device layout of type T
template <typename T>
__global__ void k_expand(long long nslots, int bs, int V, const int* __restrict__ ids,
                         const double* __restrict__ pool, T* __restrict__ out, int transpose) {
  const long long bb = static_cast<long long>(bs) * bs;
  const long long total = nslots * bb;
  for (long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += static_cast<long long>(gridDim.x) * blockDim.x) {
    const long long s = t / bb;
    const int e = static_cast<int>(t - s * bb);
    const int r = e / bs, c = e - (e / bs) * bs;
    const double v = transpose ? pool[ids[s] * bb + static_cast<long long>(c) * bs + r]
                               : pool[ids[s] * bb + e];
    const size_t dst = (static_cast<size_t>(c / V) * bs + r) * V + (c % V);
    out[s * bb + dst] = narrow<T>(v);
  }
}

// restriction r_c = I^T r_f: one thread per (coarse element, component, coarse dof)
template <typename T>
__global__ void k_restrict(int dim, int nc, int ncomp, int bss, const T* __restrict__ Ic,
                           const T* __restrict__ rf, T* __restrict__ rc) {
  long long nce = nc;
  for (int k = 1; k < dim; ++k) nce *= nc;
  const long long total = nce * ncomp * bss;
  const long long tid = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (tid >= total) return;
  const int a = static_cast<int>(tid % bss);
  const long long rest = tid / bss;
  const int comp = static_cast<int>(rest % ncomp);
  const long long K = rest / ncomp;
  const int nf = 2 * nc;
  const int kx = static_cast<int>(K % nc), ky = static_cast<int>((K / nc) % nc);
  const int kz = dim == 3 ? static_cast<int>(K / (static_cast<long long>(nc) * nc)) : 0;
  T sum = T(0);
  const int nchild = 1 << dim;
  for (int cp = 0; cp < nchild; ++cp) {
    const long long fx = 2 * kx + (cp & 1), fy = 2 * ky + ((cp >> 1) & 1);
    const long long fz = dim == 3 ? 2 * kz + ((cp >> 2) & 1) : 0;
    const long long f = fx + nf * (fy + static_cast<long long>(nf) * fz);
    const T* rfe = rf + (f * ncomp + comp) * bss;
    const T* I = Ic + static_cast<size_t>(cp) * bss * bss;
    for (int b = 0; b < bss; ++b) sum += I[static_cast<size_t>(b) * bss + a] * rfe[b];
  }
  rc[(K * ncomp + comp) * bss + a] = sum;
}

// prolongation and correction x_f += I x_c: one thread per (fine element, component, dof)
template <typename T>
__global__ void k_prolong_add(int dim, int nc, int ncomp, int bss, const T* __restrict__ Ic,
                              const T* __restrict__ xc, T* __restrict__ xf, float* __restrict__ xf32) {
  const int nf = 2 * nc;
  long long nfe = nf;
  for (int k = 1; k < dim; ++k) nfe *= nf;
  const long long total = nfe * ncomp * bss;
  const long long tid = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (tid >= total) return;
  const int b = static_cast<int>(tid % bss);
  const long long rest = tid / bss;
  const int comp = static_cast<int>(rest % ncomp);
  const long long f = rest / ncomp;
  const int fx = static_cast<int>(f % nf), fy = static_cast<int>((f / nf) % nf);
  const int fz = dim == 3 ? static_cast<int>(f / (static_cast<long long>(nf) * nf)) : 0;
  const int cp = (fx & 1) | ((fy & 1) << 1) | ((fz & 1) << 2);
  const long long K = (fx >> 1) + static_cast<long long>(nc) * ((fy >> 1) + static_cast<long long>(nc) * (fz >> 1));
  const T* I = Ic + (static_cast<size_t>(cp) * bss + b) * bss;
  const T* xce = xc + (K * ncomp + comp) * bss;
  T sum = T(0);
  for (int a = 0; a < bss; ++a) sum += I[a] * xce[a];
  const T y = xf[tid] + sum;
  xf[tid] = y;
  if (xf32) xf32[tid] = static_cast<float>(y);
}

// Sum-factorised transfers (bss = (p+1)^d <= 64), one lane per scalar
// coefficient.  The tensor-product child matrix is applied one direction at a
// time with lane shuffles: (p+1) products per lane and direction instead of
// bss.  P1 holds the 1-D child matrices, P1[c][i][j] = coefficient i on child c
// of the coarse basis function j.
template <int Q1, int DIM>
struct XferShape {
  static constexpr int BSS = DIM == 3 ? Q1 * Q1 * Q1 : Q1 * Q1;   // nodes per element component
  static constexpr int G = 64 / BSS;                              // coarse elements per wavefront
  static constexpr int NCH = 1 << DIM;                            // children per coarse element
};

// Work unit of both transfer kernels: one (coarse element, component) pair per
// group of BSS lanes, covering all 2^d children of the element.  Lane li holds
// node li, whose degree index in direction k is digit k of li in base Q1.
template <int Q1, int DIM>
struct XferLane {
  unsigned g;
  bool valid;
  int li, dg[3];
  size_t coarse;                                  // offset of the lane's coarse value
  size_t fine[XferShape<Q1, DIM>::NCH];           // offset of the lane's value in each child
  __device__ XferLane(int nc, int ncomp, unsigned nwork) {
    using S = XferShape<Q1, DIM>;
    const unsigned lane = threadIdx.x & 63u;
    g = lane / S::BSS;
    const unsigned work = ((blockIdx.x * blockDim.x + threadIdx.x) >> 6) * S::G + g;
    valid = g < S::G && work < nwork;
    const unsigned wk = valid ? work : 0u;
    li = valid ? static_cast<int>(lane - g * S::BSS) : 0;
    dg[0] = li % Q1;
    dg[1] = (li / Q1) % Q1;
    dg[2] = DIM == 3 ? li / (Q1 * Q1) : 0;
    const unsigned K = wk / ncomp, comp = wk - K * ncomp;
    const unsigned kx = K % nc, ky = (K / nc) % nc, kz = DIM == 3 ? K / (static_cast<unsigned>(nc) * nc) : 0u;
    const size_t nf = 2u * nc;
    coarse = (static_cast<size_t>(K) * ncomp + comp) * S::BSS + li;
#pragma unroll
    for (int cp = 0; cp < S::NCH; ++cp) {
      const size_t f = (2 * kx + (cp & 1)) + nf * ((2 * ky + ((cp >> 1) & 1)) + nf * (DIM == 3 ? 2 * kz + (cp >> 2) : 0u));
      fine[cp] = (f * ncomp + comp) * S::BSS + li;
    }
  }
};

// x_f += I x_c over the children of every coarse element (Section 2.2: the
// interpolation is the injection of the coarse polynomial into the children).
// The tensor-product child matrices are applied direction by direction as a
// tree: the direction-k pass turns each of the 2^k partial results into one
// per child index c_k in {0, 1}, and one shuffle of an input value serves both.
template <typename T, int Q1, int DIM>
__global__ __launch_bounds__(256) void k_prolong_tree(int nc, int ncomp, const T* __restrict__ P1,
                                                      const T* __restrict__ xc, T* __restrict__ xf, unsigned nwork,
                                                      float* __restrict__ xf32) {
  using S = XferShape<Q1, DIM>;
  const XferLane<Q1, DIM> L(nc, ncomp, nwork);
  T old[S::NCH], v[S::NCH];
#pragma unroll
  for (int cp = 0; cp < S::NCH; ++cp) old[cp] = xf[L.fine[cp]];
  v[0] = xc[L.coarse];
  int stride = 1;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const int base = static_cast<int>(L.g * S::BSS) + L.li - L.dg[k] * stride;
    const T* P0 = P1 + L.dg[k] * Q1;            // row dg of the child-0 matrix
    const T* Pc = P1 + (Q1 + L.dg[k]) * Q1;     // row dg of the child-1 matrix
    T nv[S::NCH];
#pragma unroll
    for (int t = 0; t < (1 << k); ++t) {
      T a0 = T(0), a1 = T(0);
#pragma unroll
      for (int j = 0; j < Q1; ++j) {
        const T u = __shfl(v[t], base + j * stride);
        a0 += P0[j] * u;
        a1 += Pc[j] * u;
      }
      nv[t] = a0;
      nv[t + (1 << k)] = a1;
    }
#pragma unroll
    for (int t = 0; t < (2 << k); ++t) v[t] = nv[t];
    stride *= Q1;
  }
#pragma unroll
  for (int cp = 0; cp < S::NCH; ++cp)
    if (L.valid) {
      const T y = old[cp] + v[cp];
      xf[L.fine[cp]] = y;
      if (xf32) xf32[L.fine[cp]] = static_cast<float>(y);   // the FP32 copy, when kept
    }
}

// r_c = I^T r_f (Section 2.2: the restriction is the adjoint of the
// interpolation, which on residual vectors of the discrete system is I^T),
// the tree of the prolongation run backwards: the direction-k pass pairs the
// partial results of child index c_k = 0 and 1 and applies the transposed
// child matrices.
template <typename T, int Q1, int DIM>
__global__ __launch_bounds__(256) void k_restrict_tree(int nc, int ncomp, const T* __restrict__ P1,
                                                       const T* __restrict__ rf, T* __restrict__ rc, unsigned nwork) {
  using S = XferShape<Q1, DIM>;
  const XferLane<Q1, DIM> L(nc, ncomp, nwork);
  T v[S::NCH];
#pragma unroll
  for (int cp = 0; cp < S::NCH; ++cp) v[cp] = rf[L.fine[cp]];
  int stride = 1;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const int base = static_cast<int>(L.g * S::BSS) + L.li - L.dg[k] * stride;
    const int half = S::NCH >> (k + 1);
#pragma unroll
    for (int t = 0; t < half; ++t) {
      T a = T(0);
#pragma unroll
      for (int j = 0; j < Q1; ++j) {
        // column dg of the child matrices: P1[c][j][dg]
        a += P1[j * Q1 + L.dg[k]] * __shfl(v[2 * t], base + j * stride);
        a += P1[(Q1 + j) * Q1 + L.dg[k]] * __shfl(v[2 * t + 1], base + j * stride);
      }
      v[t] = a;
    }
    stride *= Q1;
  }
  if (L.valid) rc[L.coarse] = v[0];
}

// dense FP64 GEMV (bottom pseudo-inverse): one wavefront per row
template <typename T>
__global__ __launch_bounds__(256) void k_dense_gemv(int N, const double* __restrict__ P,
                                                    const T* __restrict__ in, T* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= N) return;
  double s = 0.0;
  const double* pr = P + static_cast<size_t>(row) * N;
  for (int c = lane; c < N; c += 64) s += pr[c] * static_cast<double>(in[c]);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) out[row] = static_cast<T>(s);
}

// ---------------------------------------------------------------------------
// FP64 vector kernels of the Krylov iterations
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double sh[kRedThreads / 64];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kRedThreads / 64; ++i) t += sh[i];
  return t;   // valid in thread 0
}

__global__ __launch_bounds__(kRedThreads) void k_dot(long long n, const double* __restrict__ a,
                                                     const double* __restrict__ b,
                                                     double* __restrict__ partial) {
  double s = 0.0;
  for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<long long>(gridDim.x) * blockDim.x)
    s += a[i] * b[i];
  const double t = block_sum(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// x += alpha p; r -= alpha q; partial sums of r.r   (alpha = scal[ia])
__global__ __launch_bounds__(kRedThreads) void k_cg_update(long long n, double* __restrict__ x,
                                                           double* __restrict__ r,
                                                           const double* __restrict__ p,
                                                           const double* __restrict__ q,
                                                           const double* __restrict__ scal, int ia,
                                                           double* __restrict__ partial) {
  const double alpha = scal[ia];
  double s = 0.0;
  for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<long long>(gridDim.x) * blockDim.x) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    s += ri * ri;
  }
  const double t = block_sum(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// p = z + beta p   (beta = scal[ib])
__global__ void k_cg_dir(long long n, double* __restrict__ p, const double* __restrict__ z,
                         const double* __restrict__ scal, int ib) {
  const double beta = scal[ib];
  for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<long long>(gridDim.x) * blockDim.x)
    p[i] = z[i] + beta * p[i];
}

// reduce partial sums in a fixed order and update the scalar table:
//   op 0: scal[dst] = v
//   op 1: scal[dst] = scal[a] / v
//   op 2: scal[dst] = v / scal[a]; scal[a] = v
//   op 3: scal[dst] = -v
__global__ __launch_bounds__(kRedThreads) void k_finalize(int nparts, const double* __restrict__ partial,
                                                          double* __restrict__ scal, int op, int dst,
                                                          int a) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) s += partial[i];
  const double v = block_sum(s);
  if (threadIdx.x == 0) {
    if (op == 0) {
      scal[dst] = v;
    } else if (op == 1) {
      scal[dst] = scal[a] / v;
    } else if (op == 4) {                  // op 1 that yields 0 once the recurrence is frozen
      scal[dst] = scal[kScalFrozen] != 0.0 ? 0.0 : scal[a] / v;
    } else if (op == 5) {                  // op 2 that yields 0 before the first iteration
      scal[dst] = scal[kScalIt] == 0.0 ? 0.0 : v / scal[a];
      scal[a] = v;
    } else if (op == 3) {
      scal[dst] = -v;
    } else {
      scal[dst] = v / scal[a];
      scal[a] = v;
    }
  }
}

template <typename S, typename D>
__global__ void k_cast(long long n, const S* __restrict__ in, D* __restrict__ out) {
  for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<long long>(gridDim.x) * blockDim.x)
    out[i] = static_cast<D>(in[i]);
}

// y = alpha x + beta y with alpha, beta from the scalar table (index < 0 -> literal)
__global__ void k_axpby(long long n, const double* __restrict__ x, double* __restrict__ y,
                        const double* __restrict__ scal, int ia, double alpha_lit, int ib,
                        double beta_lit) {
  const double alpha = ia >= 0 ? scal[ia] : alpha_lit;
  const double beta = ib >= 0 ? scal[ib] : beta_lit;
  for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<long long>(gridDim.x) * blockDim.x)
    y[i] = alpha * x[i] + (beta == 0.0 ? 0.0 : beta * y[i]);
}

// y = x / sqrt(scal[i])  (normalise by a stored squared norm)
__global__ void k_scale_invsqrt(long long n, const double* __restrict__ x, double* __restrict__ y,
                                const double* __restrict__ scal, int i) {
  const double s = 1.0 / sqrt(scal[i]);
  for (long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
       t += static_cast<long long>(gridDim.x) * blockDim.x)
    y[t] = x[t] * s;
}

// partial[j][blk] = sum over the block's chunk of Q_j . w   (blockIdx.y = j)
__global__ __launch_bounds__(kRedThreads) void k_mdot(long long n, const double* __restrict__ Q,
                                                      const double* __restrict__ w,
                                                      double* __restrict__ partial) {
  const int j = blockIdx.y;
  const double* q = Q + static_cast<size_t>(j) * n;
  double s = 0.0;
  for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<long long>(gridDim.x) * blockDim.x)
    s += q[i] * w[i];
  const double t = block_sum(s);
  if (threadIdx.x == 0) partial[static_cast<size_t>(j) * gridDim.x + blockIdx.x] = t;
}

// out[j] = sum_b partial[j][b]  (one block per j, fixed order)
__global__ __launch_bounds__(kRedThreads) void k_finalize_many(int nparts, const double* __restrict__ partial,
                                                               double* __restrict__ out) {
  double s = 0.0;
  const double* p = partial + static_cast<size_t>(blockIdx.x) * nparts;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) s += p[i];
  const double v = block_sum(s);
  if (threadIdx.x == 0) out[blockIdx.x] = v;
}

__global__ void k_fill_zero_f(long long n, float* __restrict__ p) {
  for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<long long>(gridDim.x) * blockDim.x)
    p[i] = 0.0f;
}

__global__ void k_fill_zero(long long n, double* __restrict__ p) {
  for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<long long>(gridDim.x) * blockDim.x)
    p[i] = 0.0;
}

// device-side CG bookkeeping of a replayed iteration (one thread)
__global__ void k_cg_init(double* scal, double tol2, double maxit) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  scal[kScalFrozen] = 0.0;
  scal[kScalIt] = 0.0;
  scal[kScalStatus] = -1.0;
  scal[kScalTol2] = tol2;
  scal[kScalMaxit] = maxit;
  scal[kScalRRFinal] = 0.0;
}

__global__ void k_cg_check(double* scal, double* hist, int cap, int guard, int s_rz, int s_alpha, int s_rr) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (scal[kScalFrozen] != 0.0) return;
  const double it = scal[kScalIt] + 1.0;
  scal[kScalIt] = it;
  const int k = static_cast<int>(it) - 1;
  if (k < cap) hist[k] = sqrt(fabs(scal[s_rz]));
  const double rr = scal[s_rr];
  double status = -1.0;
  if (!isfinite(rr)) status = 3.0;                          // breakdown
  else if (rr <= scal[kScalTol2]) status = 1.0;             // converged
  else if (guard && (!(scal[s_rz] > 0.0) || !(scal[s_alpha] > 0.0))) status = 2.0;   // guarded stop
  else if (it >= scal[kScalMaxit]) status = 0.0;            // iteration limit
  if (status >= 0.0) {
    scal[kScalFrozen] = 1.0;
    scal[kScalStatus] = status;
    scal[kScalRRFinal] = rr;
  }
}

// w += sign * sum_{j<k} h[j] Q_j
__global__ void k_maxpy(long long n, int k, const double* __restrict__ Q, const double* __restrict__ h,
                        double sign, double* __restrict__ w) {
  for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<long long>(gridDim.x) * blockDim.x) {
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += h[j] * Q[static_cast<size_t>(j) * n + i];
    w[i] += sign * s;
  }
}

void check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

int grid_for(long long n, int threads, int cap = 4096) {
  long long g = (n + threads - 1) / threads;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return static_cast<int>(g);
}

template <typename TM, typename T, int BS>
void launch_fwd_bs(const BsrArgs<TM, T>& a, hipStream_t st) {
  constexpr int G = 64 / BS;
  const long long waves = (a.nrows + G - 1) / G;
  const int blocks = static_cast<int>((waves + kWaves - 1) / kWaves);
  if (blocks == 0) return;
  if constexpr (std::is_same<T, double>::value && BS % 16 == 0 && BS > 32 && BlkCfg<TM, BS>::NV % kWaves == 0) {
    if (!a.dinv && a.nrows <= kColSplitRows) {   // few block rows: a workgroup per row
      if (a.bid)
        k_bsr_fwd_cs<TM, T, BS, true><<<a.nrows, kThreads, 0, st>>>(a.nrows, a.rows, a.rp, a.ci, a.bid, a.blk,
                                                                     a.x, a.z, a.out, a.alpha, a.beta);
      else
        k_bsr_fwd_cs<TM, T, BS, false><<<a.nrows, kThreads, 0, st>>>(a.nrows, a.rows, a.rp, a.ci, nullptr,
                                                                      a.blk, a.x, a.z, a.out, a.alpha, a.beta);
      check_launch("bsr_fwd_cs");
      return;
    }
  }
  if (a.dinv && a.bid)
    k_bsr_fwd<TM, T, BS, 1, true><<<blocks, kThreads, 0, st>>>(a.nrows, a.rows, a.rp, a.ci, a.bid, a.blk, a.x,
                                                               a.z, a.out, a.alpha, a.beta, a.dinv, a.dbid,
                                                               a.omega);
  else if (a.dinv)
    k_bsr_fwd<TM, T, BS, 1, false><<<blocks, kThreads, 0, st>>>(a.nrows, a.rows, a.rp, a.ci, nullptr, a.blk,
                                                                a.x, a.z, a.out, a.alpha, a.beta, a.dinv,
                                                                a.dbid, a.omega);
  else if (a.bid)
    k_bsr_fwd<TM, T, BS, 0, true><<<blocks, kThreads, 0, st>>>(a.nrows, a.rows, a.rp, a.ci, a.bid, a.blk, a.x,
                                                               a.z, a.out, a.alpha, a.beta, nullptr, nullptr,
                                                               T(0));
  else
    k_bsr_fwd<TM, T, BS, 0, false><<<blocks, kThreads, 0, st>>>(a.nrows, a.rows, a.rp, a.ci, nullptr, a.blk,
                                                                a.x, a.z, a.out, a.alpha, a.beta, nullptr,
                                                                nullptr, T(0));
  check_launch("bsr_fwd");
}

template <typename TM, typename T, int BS>
void launch_tiled_bs(const BsrArgs<TM, T>& a, long long stride, int nk, hipStream_t st) {
  // FP32 products for FP32 / BF16 storage only: FP64 blocks keep FP64 products
  constexpr bool P32 = !std::is_same<TM, double>::value;
  constexpr int MT = (BS + 15) / 16;        // row tiles per tile
  const int nt = a.tnrows > 0 ? a.tnrows : a.nrows;   // places of the tile order
  if (a.p32 && !P32) throw std::invalid_argument("bsr_tiled: FP32 products need FP32 or BF16 storage");
  if (a.x32 || a.out32) {                   // an FP32 vector in or out (smoothing residuals)
    if constexpr (P32 && BS % 16 == 0) {
      if (!a.p32 || nk != 1 || (a.x32 && !a.tquad))
        throw std::invalid_argument("bsr_tiled: FP32 vectors need FP32 products, one right-hand side and, "
                                    "for FP32 x, the quad layout");
      const long long tiles = (nt + 15) / 16;
      const bool split = tiles < kSplitTiles;
      // FP32 blocks of a matrix that asks for it: two tiles per wavefront (one
      // load of a pass's blocks for both) where that still leaves two
      // wavefronts per SIMD; BF16 blocks are half the load and keep one
      constexpr bool kPair = std::is_same<TM, float>::value;
      const int per = kPair && a.tpair && tiles >= kPairTiles ? 2 : 1;   // tiles per wavefront
      const int blocks = static_cast<int>(((split ? tiles * MT : (tiles + per - 1) / per) + kWaves - 1) / kWaves);
      if (blocks == 0) return;
#define TILED32(XT_, OT_, Q_, X_, O_)                                                                          \
  if (split)                                                                                                   \
    k_bsr_tiled<TM, BS, 0, true, XT_, OT_, Q_, true><<<blocks, kThreads, 0, st>>>(                             \
        nt, a.noff, a.toff, a.tab, a.tperm, a.tblk, X_, a.z, O_, a.alpha, a.beta, 0, 1, a.out2);                  \
  else if (per == 2) {                                                                                         \
    if constexpr (kPair)                                                                                       \
      k_bsr_tiled<TM, BS, 0, true, XT_, OT_, Q_, false, 2><<<blocks, kThreads, 0, st>>>(                       \
          nt, a.noff, a.toff, a.tab, a.tperm, a.tblk, X_, a.z, O_, a.alpha, a.beta, 0, 1, a.out2);                \
  } else                                                                                                       \
    k_bsr_tiled<TM, BS, 0, true, XT_, OT_, Q_><<<blocks, kThreads, 0, st>>>(                                   \
        nt, a.noff, a.toff, a.tab, a.tperm, a.tblk, X_, a.z, O_, a.alpha, a.beta, 0, 1, a.out2);
      if (a.x32 && a.out32) {
        TILED32(float, float, true, a.x32, a.out32)
      } else if (a.x32) {
        TILED32(float, double, true, a.x32, a.out)
      } else if (a.tquad) {
        TILED32(double, float, true, a.x, a.out32)
      } else {
        TILED32(double, float, false, a.x, a.out32)
      }
#undef TILED32
      check_launch("bsr_tiled");
      return;
    } else {
      throw std::invalid_argument("bsr_tiled: FP32 vectors need FP32 products and 16 | bs");
    }
  }
  if (a.tquad && !(P32 && BS % 16 == 0))
    throw std::invalid_argument("bsr_tiled: the quad layout needs FP32 or BF16 storage and 16 | bs");
  int lkp = 0;                              // log2 of the power of two >= nk
  while ((1 << lkp) < nk) ++lkp;
  // tiles of 16 / kp rows: the unpadded order (padding to 16 rows would leave
  // empty tiles there)
  const int* order = lkp > 0 && a.trows ? a.trows : a.tperm;
  const int no = lkp > 0 && a.trows ? a.nrows : nt;
  const int rpt = 16 >> lkp;                // block rows per tile
  const long long tiles = (no + rpt - 1) / rpt;
  const int blocks = static_cast<int>((tiles + kWaves - 1) / kWaves);
  if (blocks == 0) return;
  if (lkp == 0 && tiles < kSplitTiles) {    // few tiles: one wavefront per row tile
    const int bsplit = static_cast<int>((tiles * MT + kWaves - 1) / kWaves);
    if constexpr (P32 && BS % 16 == 0) {
      if (a.tquad) {
        if (a.p32)
          k_bsr_tiled<TM, BS, 0, true, double, double, true, true><<<bsplit, kThreads, 0, st>>>(
              no, a.noff, a.toff, a.tab, order, a.tblk, a.x, a.z, a.out, a.alpha, a.beta, stride, nk, a.out2);
        else
          k_bsr_tiled<TM, BS, 0, false, double, double, true, true><<<bsplit, kThreads, 0, st>>>(
              no, a.noff, a.toff, a.tab, order, a.tblk, a.x, a.z, a.out, a.alpha, a.beta, stride, nk, a.out2);
        check_launch("bsr_tiled");
        return;
      }
    }
    if (P32 && a.p32)
      k_bsr_tiled<TM, BS, 0, P32, double, double, false, true><<<bsplit, kThreads, 0, st>>>(
          no, a.noff, a.toff, a.tab, order, a.tblk, a.x, a.z, a.out, a.alpha, a.beta, stride, nk, a.out2);
    else
      k_bsr_tiled<TM, BS, 0, false, double, double, false, true><<<bsplit, kThreads, 0, st>>>(
          no, a.noff, a.toff, a.tab, order, a.tblk, a.x, a.z, a.out, a.alpha, a.beta, stride, nk, a.out2);
    check_launch("bsr_tiled");
    return;
  }
  switch (lkp) {
#define TILED(LK)                                                                                              \
  case LK:                                                                                                     \
    if constexpr (P32 && BS % 16 == 0) {                                                                       \
      if (a.tquad) {                                                                                           \
        if (a.p32)                                                                                             \
          k_bsr_tiled<TM, BS, LK, true, double, double, true><<<blocks, kThreads, 0, st>>>(                    \
              no, a.noff, a.toff, a.tab, order, a.tblk, a.x, a.z, a.out, a.alpha, a.beta, stride, nk, a.out2);  \
        else                                                                                                   \
          k_bsr_tiled<TM, BS, LK, false, double, double, true><<<blocks, kThreads, 0, st>>>(                   \
              no, a.noff, a.toff, a.tab, order, a.tblk, a.x, a.z, a.out, a.alpha, a.beta, stride, nk, a.out2);  \
        break;                                                                                                 \
      }                                                                                                        \
    }                                                                                                          \
    if (P32 && a.p32)                                                                                          \
      k_bsr_tiled<TM, BS, LK, P32><<<blocks, kThreads, 0, st>>>(no, a.noff, a.toff, a.tab, order,       \
                                                               a.tblk, a.x, a.z, a.out, a.alpha, a.beta,       \
                                                               stride, nk, a.out2);                                    \
    else                                                                                                       \
      k_bsr_tiled<TM, BS, LK, false><<<blocks, kThreads, 0, st>>>(no, a.noff, a.toff, a.tab, order,     \
                                                                 a.tblk, a.x, a.z, a.out, a.alpha, a.beta,     \
                                                                 stride, nk, a.out2);                                  \
    break;
    TILED(0) TILED(1) TILED(2) TILED(3) TILED(4)
#undef TILED
    default:
      throw std::invalid_argument("bsr_tiled: at most 16 right-hand sides");
  }
  check_launch("bsr_tiled");
}

template <typename TM, typename T, int BS>
void launch_tr_bs(const BsrArgs<TM, T>& a, hipStream_t st) {
  constexpr int G = 64 / BS;
  const long long waves = (a.nrows + G - 1) / G;
  const int blocks = static_cast<int>((waves + kWaves - 1) / kWaves);
  if (blocks == 0) return;
  k_bsr_tr<TM, T, BS><<<blocks, kThreads, 0, st>>>(a.nrows, a.rp, a.ci, a.tpos, a.blk, a.x, a.z, a.out,
                                               a.alpha, a.beta);
  check_launch("bsr_tr");
}

template <typename TM, typename T, int BS>
void launch_fwd_multi_bs(const BsrArgs<TM, T>& a, long long stride, int nk, hipStream_t st) {
  constexpr int G = 64 / BS;
  const long long waves = (a.nrows + G - 1) / G;
  const int blocks = static_cast<int>((waves + kWaves - 1) / kWaves);
  if (blocks == 0) return;
  k_bsr_fwd_multi<TM, T, BS><<<blocks, kThreads, 0, st>>>(a.nrows, a.rows, a.rp, a.ci, a.bid, a.blk, a.x, a.z,
                                                          a.out, stride, nk, a.alpha, a.beta);
  check_launch("bsr_fwd_multi");
}

#define LDGMG_FOR_BS(X) X(4) X(8) X(9) X(12) X(16) X(25) X(27) X(32) X(36) X(48) X(64)

}  // namespace

bool fast_bs(int bs) {
  switch (bs) {
#define CASE(B) case B:
    LDGMG_FOR_BS(CASE)
#undef CASE
    return true;
    default:
      return false;
  }
}

template <typename TM, typename T>
void bsr_forward(const BsrArgs<TM, T>& a, hipStream_t st) {
  if constexpr (std::is_same<T, double>::value) {
    if (a.tab && !a.dinv && !a.rows) {     // tiled storage: matrix cores
      switch (a.bs) {
#define CASE(B) \
  case B:       \
    launch_tiled_bs<TM, T, B>(a, 0, 1, st); \
    return;
        LDGMG_FOR_BS(CASE)
#undef CASE
        default:
          throw std::runtime_error("tiled storage needs a block size with a wave-mapped kernel");
      }
    }
  }
  switch (a.bs) {
#define CASE(B) \
  case B:       \
    launch_fwd_bs<TM, T, B>(a, st); \
    return;
    LDGMG_FOR_BS(CASE)
#undef CASE
    default:
      break;
  }
  if (a.dinv) throw std::runtime_error("fused smoothing needs a block size <= 64");
  if (a.bid) throw std::runtime_error("pooled storage needs a block size with a wave-mapped kernel");
  const long long n = static_cast<long long>(a.nrows) * a.bs;
  if (n == 0) return;
  k_bsr_generic<TM, T><<<static_cast<int>((n + 255) / 256), 256, 0, st>>>(a.nrows, a.bs, a.rows, a.rp, a.ci,
                                                                        nullptr, a.blk, a.x, a.z, a.out,
                                                                        a.alpha, a.beta);
  check_launch("bsr_generic");
}

template <typename TM, typename T>
void bsr_forward_multi(const BsrArgs<TM, T>& a, long long stride, int nk, hipStream_t st) {
  if (nk < 1 || nk > kMaxRhs) throw std::invalid_argument("bsr_forward_multi: bad right-hand-side count");
  if (a.dinv) throw std::invalid_argument("bsr_forward_multi: no fused smoothing");
  if constexpr (std::is_same<T, double>::value) {
    if (a.tab && !a.rows) {                 // tiled storage: (row, vector) columns on the matrix cores
      switch (a.bs) {
#define CASE(B) \
  case B:       \
    launch_tiled_bs<TM, T, B>(a, stride, nk, st); \
    return;
        LDGMG_FOR_BS(CASE)
#undef CASE
        default:
          throw std::runtime_error("tiled storage needs a block size with a wave-mapped kernel");
      }
    }
  }
  switch (a.bs) {
#define CASE(B) \
  case B:       \
    launch_fwd_multi_bs<TM, T, B>(a, stride, nk, st); \
    return;
    LDGMG_FOR_BS(CASE)
#undef CASE
    default:
      break;
  }
  for (int q = 0; q < nk; ++q) {   // other block sizes: one apply per right-hand side
    BsrArgs<TM, T> b = a;
    b.x = a.x + q * stride;
    b.z = a.z ? a.z + q * stride : nullptr;
    b.out = a.out + q * stride;
    bsr_forward<TM, T>(b, st);
  }
}

template <typename TM, typename T>
void bsr_transposed(const BsrArgs<TM, T>& a, hipStream_t st) {
  if (a.bid) throw std::runtime_error("pooled storage: transposed applies use the transposed copy");
  switch (a.bs) {
#define CASE(B) \
  case B:       \
    launch_tr_bs<TM, T, B>(a, st); \
    return;
    LDGMG_FOR_BS(CASE)
#undef CASE
    default:
      break;
  }
  const long long n = static_cast<long long>(a.nrows) * a.bs;
  if (n == 0) return;
  k_bsr_generic<TM, T><<<static_cast<int>((n + 255) / 256), 256, 0, st>>>(a.nrows, a.bs, nullptr, a.rp, a.ci,
                                                                        a.tpos, a.blk, a.x, a.z, a.out,
                                                                        a.alpha, a.beta);
  check_launch("bsr_generic_t");
}

template <typename T>
void expand_blocks(long long nslots, int bs, const int* ids, const double* pool, T* out, bool transpose,
                   hipStream_t st) {
  if (nslots == 0) return;
  const int V = device_vec_width(bs, sizeof(T));
  const long long total = nslots * bs * bs;
  k_expand<T><<<grid_for(total, 256, 65536), 256, 0, st>>>(nslots, bs, V, ids, pool, out, transpose ? 1 : 0);
  check_launch("expand");
}

template <typename T>
void expand_tiled(long long nblk, int bs, const double* pool, T* out, bool transpose, bool quad, hipStream_t st) {
  if (quad && bs % 16 != 0) throw std::invalid_argument("expand_tiled: the quad layout needs 16 | bs");
  if (nblk == 0) return;
  const int MT = (bs + 15) / 16, KS = (bs + 3) / 4;
  const long long total = nblk * MT * 64 * KS;
  k_expand_tiled<T><<<grid_for(total, 256, 65536), 256, 0, st>>>(nblk, bs, MT, KS, pool, out, transpose ? 1 : 0,
                                                                 quad ? 1 : 0);
  check_launch("expand_tiled");
}

template <typename T, int Q1, int DIM>
void launch_xfer_tree(bool prolong, int nc, int ncomp, long long nwork, const T* P1, const T* in, T* out,
                      hipStream_t st, float* out32) {
  constexpr int G = XferShape<Q1, DIM>::G;
  const long long waves = (nwork + G - 1) / G;
  const int blocks = static_cast<int>((waves + 3) / 4);
  if (prolong)
    k_prolong_tree<T, Q1, DIM><<<blocks, 256, 0, st>>>(nc, ncomp, P1, in, out, static_cast<unsigned>(nwork), out32);
  else
    k_restrict_tree<T, Q1, DIM><<<blocks, 256, 0, st>>>(nc, ncomp, P1, in, out, static_cast<unsigned>(nwork));
  check_launch(prolong ? "prolong_tree" : "restrict_tree");
}

// Transfers whose element component fits one wavefront (Q1^d <= 64) run as a
// tree over the children; returns false for the others.
template <typename T>
bool xfer_tree(bool prolong, int dim, int q1, int nc, int ncomp, long long nwork, const T* P1, const T* in,
               T* out, hipStream_t st, float* out32 = nullptr) {
  if (nwork >= (1LL << 31)) throw std::invalid_argument("transfer: more than 2^31 coarse element components");
  if (dim == 3) {
    switch (q1) {
      case 2: launch_xfer_tree<T, 2, 3>(prolong, nc, ncomp, nwork, P1, in, out, st, out32); return true;
      case 3: launch_xfer_tree<T, 3, 3>(prolong, nc, ncomp, nwork, P1, in, out, st, out32); return true;
      case 4: launch_xfer_tree<T, 4, 3>(prolong, nc, ncomp, nwork, P1, in, out, st, out32); return true;
      default: return false;
    }
  }
  switch (q1) {
    case 2: launch_xfer_tree<T, 2, 2>(prolong, nc, ncomp, nwork, P1, in, out, st, out32); return true;
    case 3: launch_xfer_tree<T, 3, 2>(prolong, nc, ncomp, nwork, P1, in, out, st, out32); return true;
    case 4: launch_xfer_tree<T, 4, 2>(prolong, nc, ncomp, nwork, P1, in, out, st, out32); return true;
    case 5: launch_xfer_tree<T, 5, 2>(prolong, nc, ncomp, nwork, P1, in, out, st, out32); return true;
    case 6: launch_xfer_tree<T, 6, 2>(prolong, nc, ncomp, nwork, P1, in, out, st, out32); return true;
    default: return false;
  }
}

template <typename T>
void restrict_op(int dim, int nc, int ncomp, int bss, int q1, const T* P1, const T* Ic, const T* rf, T* rc,
                 hipStream_t st) {
  long long nce = nc;
  for (int k = 1; k < dim; ++k) nce *= nc;
  if (xfer_tree<T>(false, dim, q1, nc, ncomp, nce * ncomp, P1, rf, rc, st)) return;
  const long long total = nce * ncomp * bss;
  k_restrict<T><<<static_cast<int>((total + 255) / 256), 256, 0, st>>>(dim, nc, ncomp, bss, Ic, rf, rc);
  check_launch("restrict");
}

template <typename T>
void prolong_add(int dim, int nc, int ncomp, int bss, int q1, const T* P1, const T* Ic, const T* xc, T* xf,
                 hipStream_t st, float* xf32) {
  long long nfe = 2 * nc;
  for (int k = 1; k < dim; ++k) nfe *= 2 * nc;
  long long nce = nc;
  for (int k = 1; k < dim; ++k) nce *= nc;
  if (xfer_tree<T>(true, dim, q1, nc, ncomp, nce * ncomp, P1, xc, xf, st, xf32)) return;
  const long long total = nfe * ncomp * bss;
  k_prolong_add<T><<<static_cast<int>((total + 255) / 256), 256, 0, st>>>(dim, nc, ncomp, bss, Ic, xc, xf, xf32);
  check_launch("prolong");
}

template <typename T>
void dense_gemv(int N, const double* P, const T* in, T* out, hipStream_t st) {
  k_dense_gemv<T><<<(N + 3) / 4, 256, 0, st>>>(N, P, in, out);
  check_launch("dense_gemv");
}

void dot_partial(long long n, const double* a, const double* b, double* partial, hipStream_t st) {
  k_dot<<<kRedBlocks, kRedThreads, 0, st>>>(n, a, b, partial);
  check_launch("dot");
}

void finalize(const double* partial, double* scal, int op, int dst, int a, hipStream_t st) {
  k_finalize<<<1, kRedThreads, 0, st>>>(kRedBlocks, partial, scal, op, dst, a);
  check_launch("finalize");
}

void fill_zero(float* p, long long n, hipStream_t st) {
  if (n <= 0) return;
  const long long want = (n + 255) / 256;
  k_fill_zero_f<<<static_cast<int>(want < 4096 ? want : 4096), 256, 0, st>>>(n, p);
  check_launch("fill_zero");
}

void fill_zero(double* p, long long n, hipStream_t st) {
  if (n <= 0) return;
  const long long want = (n + 255) / 256;
  const int blocks = static_cast<int>(want < 4096 ? want : 4096);
  k_fill_zero<<<blocks, 256, 0, st>>>(n, p);
  check_launch("fill_zero");
}

void cg_init(double* scal, double tol2, int maxit, hipStream_t st) {
  k_cg_init<<<1, 64, 0, st>>>(scal, tol2, static_cast<double>(maxit));
  check_launch("cg_init");
}

void cg_check(double* scal, double* hist, int cap, bool guard, int s_rz, int s_alpha, int s_rr, hipStream_t st) {
  k_cg_check<<<1, 64, 0, st>>>(scal, hist, cap, guard ? 1 : 0, s_rz, s_alpha, s_rr);
  check_launch("cg_check");
}

void cg_update(long long n, double* x, double* r, const double* p, const double* q, const double* scal,
               int ia, double* partial, hipStream_t st) {
  k_cg_update<<<kRedBlocks, kRedThreads, 0, st>>>(n, x, r, p, q, scal, ia, partial);
  check_launch("cg_update");
}

void cg_dir(long long n, double* p, const double* z, const double* scal, int ib, hipStream_t st) {
  k_cg_dir<<<grid_for(n, 256), 256, 0, st>>>(n, p, z, scal, ib);
  check_launch("cg_dir");
}

void axpby(long long n, const double* x, double* y, const double* scal, int ia, double alpha, int ib,
           double beta, hipStream_t st) {
  k_axpby<<<grid_for(n, 256), 256, 0, st>>>(n, x, y, scal, ia, alpha, ib, beta);
  check_launch("axpby");
}

void scale_invsqrt(long long n, const double* x, double* y, const double* scal, int i, hipStream_t st) {
  k_scale_invsqrt<<<grid_for(n, 256), 256, 0, st>>>(n, x, y, scal, i);
  check_launch("scale_invsqrt");
}

template <typename S, typename D>
void cast(long long n, const S* in, D* out, hipStream_t st) {
  k_cast<S, D><<<grid_for(n, 256), 256, 0, st>>>(n, in, out);
  check_launch("cast");
}

void mdot(long long n, int k, const double* Q, const double* w, double* partial, double* out, hipStream_t st) {
  dim3 grid(kMdotBlocks, k);
  k_mdot<<<grid, kRedThreads, 0, st>>>(n, Q, w, partial);
  check_launch("mdot");
  k_finalize_many<<<k, kRedThreads, 0, st>>>(kMdotBlocks, partial, out);
  check_launch("finalize_many");
}

void maxpy(long long n, int k, const double* Q, const double* h, double sign, double* w, hipStream_t st) {
  k_maxpy<<<grid_for(n, 256), 256, 0, st>>>(n, k, Q, h, sign, w);
  check_launch("maxpy");
}

template void bsr_forward<float, double>(const BsrArgs<float, double>&, hipStream_t);
template void bsr_forward<double, double>(const BsrArgs<double, double>&, hipStream_t);
template void bsr_transposed<float, double>(const BsrArgs<float, double>&, hipStream_t);
template void bsr_forward_multi<float, double>(const BsrArgs<float, double>&, long long, int, hipStream_t);
template void bsr_forward_multi<double, double>(const BsrArgs<double, double>&, long long, int, hipStream_t);
template void bsr_transposed<double, double>(const BsrArgs<double, double>&, hipStream_t);
template void bsr_forward<bf16s, double>(const BsrArgs<bf16s, double>&, hipStream_t);
template void bsr_transposed<bf16s, double>(const BsrArgs<bf16s, double>&, hipStream_t);
template void bsr_forward_multi<bf16s, double>(const BsrArgs<bf16s, double>&, long long, int, hipStream_t);
template void expand_blocks<bf16s>(long long, int, const int*, const double*, bf16s*, bool, hipStream_t);
template void expand_tiled<float>(long long, int, const double*, float*, bool, bool, hipStream_t);
template void expand_tiled<double>(long long, int, const double*, double*, bool, bool, hipStream_t);
template void expand_tiled<bf16s>(long long, int, const double*, bf16s*, bool, bool, hipStream_t);
template void expand_blocks<float>(long long, int, const int*, const double*, float*, bool, hipStream_t);
template void expand_blocks<double>(long long, int, const int*, const double*, double*, bool, hipStream_t);
template void restrict_op<double>(int, int, int, int, int, const double*, const double*, const double*, double*,
                                  hipStream_t);
template void prolong_add<double>(int, int, int, int, int, const double*, const double*, const double*, double*,
                                  hipStream_t, float*);
template void dense_gemv<float>(int, const double*, const float*, float*, hipStream_t);
template void dense_gemv<double>(int, const double*, const double*, double*, hipStream_t);
template void cast<double, float>(long long, const double*, float*, hipStream_t);
template void cast<float, double>(long long, const float*, double*, hipStream_t);

}  // namespace ldgmg

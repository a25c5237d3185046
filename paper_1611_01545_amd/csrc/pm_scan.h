// Header-only device-wide exclusive scan into 64-bit offsets (out[0..n], out[n] =
// total), parameterised by a value getter so each caller scans what it needs
// without materialising the values.
#pragma once
#include "pm_common.h"

namespace pmscan {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

template <typename T>
__global__ void k_fill(T* p, int64_t n, T v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

struct GetU32 {
  const uint32_t* p;
  __device__ int64_t operator()(int64_t i) const { return p[i]; }
};
struct GetU64Lo {
  const uint64_t* p;
  __device__ int64_t operator()(int64_t i) const { return (int64_t)(p[i] & 0xffffffffull); }
};
// Full per-cell count of a compressed species: the byte, or the escape table entry.
struct GetCount {
  const uint8_t* count;
  const uint64_t* esc;
  const pm_shdr* hdr;
  __device__ int64_t operator()(int64_t i) const {
    const uint32_t c = count[i];
    return c != 255u ? (int64_t)c : escaped(i);
  }
  // the full count of a cell whose byte is 255, from the escape table
  __device__ int64_t escaped(int64_t i) const {
    int64_t lo = 0, hi = hdr->n_esc;  // binary search (esc sorted by cell)
    while (lo < hi) {
      int64_t mid = (lo + hi) >> 1;
      if ((int64_t)esc[2 * mid] < i) lo = mid + 1; else hi = mid;
    }
    if (lo < hdr->n_esc && (int64_t)esc[2 * lo] == i) return (int64_t)esc[2 * lo + 1];
    return 255;  // inconsistent table: treated as 255 (sum check flags it)
  }
};

// Element access in two phases: each getter's plain load first, then what needs the loaded
// value (GetCount's escape lookup), so that a thread issues the loads of all its items
// before it uses any (with a branch between them the compiler waited for each load).
template <typename Get>
struct Phase {
  using R = int64_t;
  __device__ static R raw(const Get& g, int64_t i) { return g(i); }
  __device__ static int64_t fix(const Get&, int64_t, R r) { return r; }
};
template <>
struct Phase<GetCount> {
  using R = uint32_t;
  __device__ static R raw(const GetCount& g, int64_t i) { return g.count[i]; }
  __device__ static int64_t fix(const GetCount& g, int64_t i, R c) {
    return c != 255u ? (int64_t)c : g.escaped(i);
  }
};

// LDS index of tile element e with one pad word per SCAN_ITEMS: a thread's SCAN_ITEMS
// consecutive elements then start 17 words apart, not 16 (which put every lane on the
// same banks)
__device__ inline int scan_pad(int e) { return e + e / SCAN_ITEMS; }

__device__ inline int64_t wave_incl_scan(int64_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int64_t t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

// Inclusive prefix sum over the 64 lanes of a wave by DPP: shifts by 1, 2, 4 and 8
// within each row of 16 lanes, then the last lane of rows 0 and 2 added into rows 1 and
// 3, then lane 31 added into rows 2 and 3; lanes with no source add 0. Unlike a scan by
// shuffles it needs no lane-index registers.
__device__ inline int wave_incl_scan_dpp(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);
  return v;
}

// Exclusive scan of 32-bit values over the block's threads with one barrier. wsum:
// blockDim.x / 64 ints of LDS that the caller leaves alone until its next barrier.
__device__ inline int block_excl_scan_i32(int v, int* wsum) {
  const int inc = wave_incl_scan_dpp(v);
  if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = inc;
  __syncthreads();
  int base = inc - v;
  for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) base += wsum[w];
  return base;
}

// Exclusive scan over the block's threads (blockDim.x a multiple of 64, <= 1024).
__device__ inline int64_t block_excl_scan(int64_t v, int64_t* lds_w, int64_t* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int64_t inc = wave_incl_scan(v);
  if (lane == 63) lds_w[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t s = 0;
    for (int i = 0; i < nw; ++i) {
      int64_t t = lds_w[i];
      lds_w[i] = s;
      s += t;
    }
    lds_w[nw] = s;
  }
  __syncthreads();
  int64_t r = lds_w[w] + inc - v;
  if (total) *total = lds_w[nw];
  __syncthreads();
  return r;
}

template <typename Get>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(Get g, int64_t n,
                                                              int64_t* bsum) {
  __shared__ int64_t lw[SCAN_THREADS / 64 + 1];
  using PH = Phase<Get>;
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  typename PH::R r[SCAN_ITEMS];
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const int64_t i = base + k * SCAN_THREADS + threadIdx.x;
    r[k] = PH::raw(g, i < n ? i : n - 1);  // n > 0 whenever a block runs
  }
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const int64_t i = base + k * SCAN_THREADS + threadIdx.x;
    if (i < n) s += PH::fix(g, i, r[k]);
  }
  int64_t tot;
  block_excl_scan(s, lw, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

static __global__ __launch_bounds__(1024) void k_scan_blocks(int64_t* bsum, int64_t nb,
                                                      int64_t* total_out) {
  __shared__ int64_t lw[1024 / 64 + 1];
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += 1024) {
    int64_t i = b0 + threadIdx.x;
    int64_t v = i < nb ? bsum[i] : 0;
    int64_t tot;
    int64_t ex = block_excl_scan(v, lw, &tot);
    if (i < nb) bsum[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) *total_out = carry;
}

template <typename Get>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_down(Get g, int64_t n,
                                                            const int64_t* bsum,
                                                            int64_t* out) {
  __shared__ int64_t vals[SCAN_TILE + SCAN_TILE / SCAN_ITEMS];
  __shared__ int64_t lw[SCAN_THREADS / 64 + 1];
  using PH = Phase<Get>;
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  {
    typename PH::R r[SCAN_ITEMS];
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
      const int64_t i = base + k * SCAN_THREADS + threadIdx.x;
      r[k] = PH::raw(g, i < n ? i : n - 1);  // n > 0 whenever a block runs
    }
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
      const int64_t i = base + k * SCAN_THREADS + threadIdx.x;
      vals[scan_pad(k * SCAN_THREADS + threadIdx.x)] = i < n ? PH::fix(g, i, r[k]) : 0;
    }
  }
  __syncthreads();
  int64_t loc[SCAN_ITEMS];
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    loc[k] = s;
    s += vals[scan_pad(threadIdx.x * SCAN_ITEMS + k)];
  }
  int64_t ex = block_excl_scan(s, lw, nullptr);
  int64_t off = bsum[blockIdx.x] + ex;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) vals[scan_pad(threadIdx.x * SCAN_ITEMS + k)] = off + loc[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const int64_t i = base + k * SCAN_THREADS + threadIdx.x;
    if (i < n) out[i] = vals[scan_pad(k * SCAN_THREADS + threadIdx.x)];
  }
}

// bsum_ext (nullable): caller-provided block sums of at least cdiv(n, SCAN_TILE) entries
// instead of the context's scratch
template <typename Get>
pm_status scan_generic(pm_context* c, Get g, int64_t n, int64_t* out,
                       int64_t* bsum_ext = nullptr) {
  int64_t nb = cdiv(n, SCAN_TILE);
  if (nb == 0) {
    hipLaunchKernelGGL(k_fill<int64_t>, dim3(1), dim3(64), 0, c->stream, out, 1,
                       (int64_t)0);
    PM_LAUNCH_CHECK();
    return PM_OK;
  }
  int64_t* bsum = bsum_ext ? bsum_ext : (int64_t*)scratch(c, SC_BSUM, (size_t)nb * sizeof(int64_t));
  if (!bsum) return PM_ERR_NOMEM;
  hipLaunchKernelGGL(k_scan_reduce<Get>, dim3((unsigned)nb), dim3(SCAN_THREADS), 0,
                     c->stream, g, n, bsum);
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, c->stream, bsum, nb, out + n);
  hipLaunchKernelGGL(k_scan_down<Get>, dim3((unsigned)nb), dim3(SCAN_THREADS), 0,
                     c->stream, g, n, bsum, out);
  PM_LAUNCH_CHECK();
  return PM_OK;
}


}  // namespace pmscan

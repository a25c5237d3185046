// Device-wide building blocks: fills, exclusive scans into 64-bit offsets, and a
// stable LSD radix sort of (uint32 key, uint32 value) pairs. They serve the cell
// ordering of the compressed format (a stable counting order of particles by cell,
// Sec. 2.4 "linked list" reused for compression).
#include "pm_scan.h"

using namespace pmscan;

namespace {

// ------------------------------------------------------------------ radix sort --
constexpr int RS_THREADS = 256;
constexpr int RS_ROUNDS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ROUNDS;
constexpr int64_t RS_GMAX = 1024;  // workgroups of a sort whose length is on the device

// The pair count is n_host, or *n_dev when given (a count produced on the device, so
// that the host never waits for it). Workgroup b of nblk takes the contiguous range
// [lo, hi) of whole rounds of RS_THREADS pairs; ranges follow the workgroup order, so the
// digit histogram laid out [digit][workgroup] and scanned gives stable destinations.
__device__ inline void rs_range(int64_t n_host, const int64_t* n_dev, int64_t nblk,
                                int64_t b, int64_t& lo, int64_t& hi) {
  const int64_t n = n_dev ? *n_dev : n_host;
  const int64_t per = ((n + nblk - 1) / nblk + RS_THREADS - 1) / RS_THREADS * RS_THREADS;
  lo = b * per < n ? b * per : n;
  hi = lo + per < n ? lo + per : n;
}

__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const uint32_t* keys, int64_t n,
                                                        const int64_t* n_dev, int shift,
                                                        int64_t nblk, uint32_t* hist) {
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  int64_t lo, hi;
  rs_range(n, n_dev, nblk, blockIdx.x, lo, hi);
  for (int64_t i = lo + threadIdx.x; i < hi; i += RS_THREADS)
    atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1u);
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

// Scatter of one digit pass, a tile of up to RS_TILE pairs at a time: each round of
// RS_THREADS pairs is ranked by a wave multi-split (stable: round, wave, lane), the
// tile's pairs are placed in LDS in digit order, and then written out in that order, so
// that a digit's pairs of the tile go to consecutive destinations (one run per digit
// and tile, instead of one or two pairs per digit and round: the written lines are whole
// and the scatter of a sort of 1.07 G pairs stops re-fetching them).
__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(const uint32_t* kin,
                                                           const uint32_t* vin, int64_t n,
                                                           const int64_t* n_dev, int shift,
                                                           int64_t nblk,
                                                           const int64_t* hoff,
                                                           uint32_t* kout, uint32_t* vout) {
  __shared__ int64_t dbase[256];        // destination of the digit's next pair
  __shared__ uint32_t tcnt[256];        // the tile's pairs per digit, so far
  __shared__ int tstart[256];           // their first LDS slot
  __shared__ uint32_t wcnt[RS_THREADS / 64][256];
  __shared__ int wsum[RS_THREADS / 64];
  __shared__ uint32_t skey[RS_TILE], sval[RS_TILE];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  int64_t lo, hi;
  rs_range(n, n_dev, nblk, blockIdx.x, lo, hi);
  dbase[threadIdx.x] = hoff[(int64_t)threadIdx.x * nblk + blockIdx.x];
  for (int64_t tb = lo; tb < hi; tb += RS_TILE) {  // uniform across the block
    const int64_t te = tb + RS_TILE < hi ? tb + RS_TILE : hi;
    tcnt[threadIdx.x] = 0;
    uint32_t key[RS_ROUNDS], val[RS_ROUNDS], lrank[RS_ROUNDS];
#pragma unroll
    for (int r = 0; r < RS_ROUNDS; ++r) {
      const int64_t i = tb + (int64_t)r * RS_THREADS + threadIdx.x;
      key[r] = i < te ? kin[i] : 0u;
      val[r] = i < te ? vin[i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < RS_ROUNDS; ++r) {
      const bool valid = tb + (int64_t)r * RS_THREADS + threadIdx.x < te;
      const uint32_t d = (key[r] >> shift) & 255u;
#pragma unroll
      for (int q = 0; q < RS_THREADS / 64; ++q) wcnt[q][threadIdx.x] = 0;
      __syncthreads();
      uint64_t match = __ballot(valid);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const uint64_t m = __ballot(valid && ((d >> b) & 1u));
        match &= ((d >> b) & 1u) ? m : ~m;
      }
      const uint32_t rank = (uint32_t)__popcll(match & lt);
      if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(match);
      __syncthreads();
      if (valid) {
        uint32_t pre = tcnt[d];
        for (int q = 0; q < w; ++q) pre += wcnt[q][d];
        lrank[r] = pre + rank;
      }
      __syncthreads();
      uint32_t add = 0;
#pragma unroll
      for (int q = 0; q < RS_THREADS / 64; ++q) add += wcnt[q][threadIdx.x];
      tcnt[threadIdx.x] += add;
    }
    __syncthreads();
    // first LDS slot of each digit
    const int start = pmscan::block_excl_scan_i32((int)tcnt[threadIdx.x], wsum);
    tstart[threadIdx.x] = start;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RS_ROUNDS; ++r) {
      if (tb + (int64_t)r * RS_THREADS + threadIdx.x < te) {
        const int slot = tstart[(key[r] >> shift) & 255u] + (int)lrank[r];
        skey[slot] = key[r];
        sval[slot] = val[r];
      }
    }
    __syncthreads();
    const int cnt = (int)(te - tb);
    for (int slot = threadIdx.x; slot < cnt; slot += RS_THREADS) {
      const uint32_t k = skey[slot];
      const uint32_t d = (k >> shift) & 255u;
      const int64_t dst = dbase[d] + (slot - tstart[d]);
      kout[dst] = k;
      vout[dst] = sval[slot];
    }
    __syncthreads();
    dbase[threadIdx.x] += tcnt[threadIdx.x];
    __syncthreads();
  }
}

__global__ void k_iota(int64_t* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = i;
}

// Grid folds in two launches: FOLD_G workgroups reduce strided slices of the partials
// to one pair each, then one workgroup reduces those.
constexpr int FOLD_T = 256;
constexpr int FOLD_G = 256;

__device__ inline void block_minmax(int& a, int& b) {
  __shared__ int smn[FOLD_T / 64], smx[FOLD_T / 64];
  for (int d = 32; d >= 1; d >>= 1) {
    a = min(a, __shfl_xor(a, d, 64));
    b = max(b, __shfl_xor(b, d, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    smn[threadIdx.x >> 6] = a;
    smx[threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int q = 1; q < FOLD_T / 64; ++q) {
      a = min(a, smn[q]);
      b = max(b, smx[q]);
    }
}

__global__ __launch_bounds__(FOLD_T) void k_fold_minmax_part(const int32_t* mn,
                                                             const int32_t* mx, int64_t n,
                                                             int32_t* part) {
  int a = 65536, b = -1;
  for (int64_t i = (int64_t)blockIdx.x * FOLD_T + threadIdx.x; i < n;
       i += (int64_t)FOLD_T * gridDim.x) {
    a = min(a, mn[i]);
    b = max(b, mx[i]);
  }
  block_minmax(a, b);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = b;
  }
}

__global__ __launch_bounds__(FOLD_T) void k_fold_minmax(const int32_t* part, int g,
                                                        pm_shdr* h) {
  int a = 65536, b = -1;
  for (int i = threadIdx.x; i < g; i += FOLD_T) {
    a = min(a, part[2 * i]);
    b = max(b, part[2 * i + 1]);
  }
  block_minmax(a, b);
  if (threadIdx.x == 0) {
    h->j_min = a;
    h->j_max = b;
  }
}

__global__ __launch_bounds__(FOLD_T) void k_fold_max_part(const uint32_t* part, int64_t n,
                                                          uint32_t* out) {
  int a = 0, b = 0;  // values as non-negative float bit patterns fit int
  for (int64_t i = (int64_t)blockIdx.x * FOLD_T + threadIdx.x; i < n;
       i += (int64_t)FOLD_T * gridDim.x)
    b = max(b, (int)part[i]);
  block_minmax(a, b);
  if (threadIdx.x == 0) out[blockIdx.x] = (uint32_t)b;
}

}  // namespace

pm_status fold_minmax_to_header(pm_context* c, const int32_t* mn, const int32_t* mx,
                                int64_t n, pm_shdr* hdr) {
  const int g = (int)std::min<int64_t>(FOLD_G, std::max<int64_t>(1, (n + FOLD_T - 1) / FOLD_T));
  int32_t* part = (int32_t*)scratch(c, SC_FOLD, (size_t)2 * FOLD_G * sizeof(int32_t));
  if (!part) return PM_ERR_NOMEM;
  hipLaunchKernelGGL(k_fold_minmax_part, dim3(g), dim3(FOLD_T), 0, c->stream, mn, mx, n, part);
  hipLaunchKernelGGL(k_fold_minmax, dim3(1), dim3(FOLD_T), 0, c->stream, part, g, hdr);
  PM_LAUNCH_CHECK();
  return PM_OK;
}

// max of non-negative float bit patterns (or any values below 2^31)
pm_status fold_max_u32(pm_context* c, const uint32_t* part, int64_t n, uint32_t* out) {
  const int g = (int)std::min<int64_t>(FOLD_G, std::max<int64_t>(1, (n + FOLD_T - 1) / FOLD_T));
  uint32_t* p2 = (uint32_t*)scratch(c, SC_FOLD, (size_t)2 * FOLD_G * sizeof(int32_t));
  if (!p2) return PM_ERR_NOMEM;
  hipLaunchKernelGGL(k_fold_max_part, dim3(g), dim3(FOLD_T), 0, c->stream, part, n, p2);
  hipLaunchKernelGGL(k_fold_max_part, dim3(1), dim3(FOLD_T), 0, c->stream, p2, (int64_t)g, out);
  PM_LAUNCH_CHECK();
  return PM_OK;
}

pm_status run_iota(pm_context* c, int64_t* p, int64_t n) {
  if (n <= 0) return PM_OK;
  hipLaunchKernelGGL(k_iota, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, c->stream, p, n);
  PM_LAUNCH_CHECK();
  return PM_OK;
}

pm_status launch_fill_u32(pm_context* c, uint32_t* p, int64_t n, uint32_t v) {
  if (n <= 0) return PM_OK;
  int64_t blocks = cdiv(n, 256);
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill<uint32_t>, dim3((unsigned)blocks), dim3(256), 0, c->stream, p,
                     n, v);
  PM_LAUNCH_CHECK();
  return PM_OK;
}

pm_status launch_fill_u64(pm_context* c, uint64_t* p, int64_t n, uint64_t v) {
  if (n <= 0) return PM_OK;
  int64_t blocks = cdiv(n, 256);
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill<uint64_t>, dim3((unsigned)blocks), dim3(256), 0, c->stream, p,
                     n, v);
  PM_LAUNCH_CHECK();
  return PM_OK;
}

pm_status scan_u32(pm_context* c, const uint32_t* in, int64_t n, int64_t* out) {
  return scan_generic(c, GetU32{in}, n, out);
}
pm_status scan_u64lo(pm_context* c, const uint64_t* in, int64_t n, int64_t* out) {
  return scan_generic(c, GetU64Lo{in}, n, out);
}
pm_status scan_counts(pm_context* c, const uint8_t* count, const uint64_t* esc,
                      const pm_shdr* hdr, int64_t n, int64_t* out) {
  return scan_generic(c, GetCount{count, esc, hdr}, n, out);
}

namespace {
pm_status radix_sort_impl(pm_context* c, uint32_t** keys, uint32_t** vals,
                          uint32_t** keys_alt, uint32_t** vals_alt, int64_t n,
                          const int64_t* n_dev, int64_t nblk, int bits) {
  uint32_t* hist = (uint32_t*)scratch(c, SC_HIST, (size_t)nblk * 256 * sizeof(uint32_t));
  int64_t* hoff = (int64_t*)scratch(c, SC_HOFF, ((size_t)nblk * 256 + 1) * sizeof(int64_t));
  if (!hist || !hoff) return PM_ERR_NOMEM;
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nblk), dim3(RS_THREADS), 0, c->stream,
                       *keys, n, n_dev, shift, nblk, hist);
    PM_LAUNCH_CHECK();
    pm_status s = scan_u32(c, hist, nblk * 256, hoff);
    if (s != PM_OK) return s;
    hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nblk), dim3(RS_THREADS), 0, c->stream,
                       *keys, *vals, n, n_dev, shift, nblk, hoff, *keys_alt, *vals_alt);
    PM_LAUNCH_CHECK();
    uint32_t* t = *keys;
    *keys = *keys_alt;
    *keys_alt = t;
    t = *vals;
    *vals = *vals_alt;
    *vals_alt = t;
  }
  return PM_OK;
}
}  // namespace

pm_status radix_sort_pairs(pm_context* c, uint32_t** keys, uint32_t** vals,
                           uint32_t** keys_alt, uint32_t** vals_alt, int64_t n,
                           int bits) {
  if (n <= 1 || bits <= 0) return PM_OK;
  return radix_sort_impl(c, keys, vals, keys_alt, vals_alt, n, nullptr, cdiv(n, RS_TILE),
                         bits);
}

pm_status radix_sort_pairs_dev(pm_context* c, uint32_t** keys, uint32_t** vals,
                               uint32_t** keys_alt, uint32_t** vals_alt, int64_t n_max,
                               const int64_t* n_dev, int bits) {
  if (n_max <= 1 || bits <= 0) return PM_OK;
  int64_t nblk = cdiv(n_max, RS_TILE);
  if (nblk > RS_GMAX) nblk = RS_GMAX;
  return radix_sort_impl(c, keys, vals, keys_alt, vals_alt, n_max, n_dev, nblk, bits);
}

// The compressed phase-space format of Sec. 2.4 on the GPU: encode from float
// particles, decode to bin centres, per-cell offsets of a compressed stream, the
// count/escape table, the byte stream and the float64 global reductions.
#include <cstring>
#include <mutex>

#include "pm_codec.h"
#include "pm_scan.h"

using namespace pmscan;

namespace {

constexpr int T256 = 256;

__global__ void k_init_hdr(pm_shdr* h) {
  h->v_max = 0.f;
  h->j_min = 65536;
  h->j_max = -1;
  h->flags = 0;
  h->n_esc = 0;
  h->reserved = 0;
}

// v_max of a species: largest |v_a| (bit pattern of a non-negative float orders
// like an unsigned integer).
__global__ __launch_bounds__(T256) void k_absmax(const float* v, int64_t n3, pm_shdr* h,
                                                DevErr* err) {
  float m = 0.f;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * T256 + threadIdx.x; i < n3;
       i += (int64_t)gridDim.x * T256) {
    float a = fabsf(v[i]);
    if (!(a <= 3.0e38f)) bad = true;
    else m = fmaxf(m, a);
  }
  for (int d = 32; d >= 1; d >>= 1) m = fmaxf(m, __shfl_xor(m, d, 64));
  if ((threadIdx.x & 63) == 0) atomicMax((unsigned int*)&h->v_max, __float_as_uint(m));
  if (bad) latch_error(err, ERRBIT_RANGE);
}

__global__ __launch_bounds__(T256) void k_encode_keys(const float* x, int64_t n, Geom g,
                                                     uint32_t* keys, uint32_t* vals,
                                                     DevErr* err) {
  int64_t p = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (p >= n) return;
  uint32_t u[3];
  bool ok = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) ok &= pos_code(x[3 * p + a], g.SL, g.S, u[a]);
  if (!ok) latch_error(err, ERRBIT_RANGE);
  keys[p] = cell_key(g, u[0] >> 8, u[1] >> 8, u[2] >> 8);
  vals[p] = (uint32_t)p;
}

// Block min/max of the velocity codes, stored at the block's index (no atomics).
__device__ inline void block_minmax_store(int jmin, int jmax, int32_t* pmn, int32_t* pmx) {
  __shared__ int smn[T256 / 64], smx[T256 / 64];
  for (int d = 32; d >= 1; d >>= 1) {
    jmin = min(jmin, __shfl_xor(jmin, d, 64));
    jmax = max(jmax, __shfl_xor(jmax, d, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    smn[threadIdx.x >> 6] = jmin;
    smx[threadIdx.x >> 6] = jmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < T256 / 64; ++q) {
      jmin = min(jmin, smn[q]);
      jmax = max(jmax, smx[q]);
    }
    pmn[blockIdx.x] = jmin;
    pmx[blockIdx.x] = jmax;
  }
}

// P position bytes, V velocity bytes per axis (P = 1, V = 2: the paper's format)
template <int P, int V>
__global__ __launch_bounds__(T256) void k_encode_gather(
    const float* x, const float* v, int64_t n, Geom g, const uint32_t* keys_sorted,
    const uint32_t* idx_sorted, void* pos_, void* vel_, int64_t* perm,
    uint32_t* run_start, pm_shdr* h, int32_t* pmn, int32_t* pmx) {
  using PT = typename PosCode<P>::T;
  using VT = typename VelCode<V>::T;
  PT* pos = (PT*)pos_;
  VT* vel = (VT*)vel_;
  // S and S / L of the P-byte code (powers-of-two multiples of the 1-byte ones)
  const int64_t S = g.S << (8 * (P - 1));
  const double SL = P == 1 ? g.SL : g.SL * 256.0;
  constexpr uint32_t OFF_MASK = (1u << (8 * P)) - 1u;
  int64_t j = (int64_t)blockIdx.x * T256 + threadIdx.x;
  int jmin = 65536, jmax = -1;
  if (j < n) {
    uint32_t p = idx_sorted[j];
    float vmax = h->v_max;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      uint32_t u;
      pos_code(x[3 * (int64_t)p + a], SL, S, u);
      pos[3 * j + a] = (PT)(u & OFF_MASK);
      int c = vel_code_v<V>(v[3 * (int64_t)p + a], vmax);
      vel[3 * j + a] = (VT)c;
      jmin = min(jmin, c);
      jmax = max(jmax, c);
    }
    if (perm) perm[j] = (int64_t)p;
    const uint32_t k = keys_sorted[j];
    if (j == 0 || keys_sorted[j - 1] != k) run_start[k] = (uint32_t)j;  // first of its cell
  }
  block_minmax_store(jmin, jmax, pmn, pmx);
}

// Particle count of each occupied cell, from the sorted keys: stored by the last
// particle of the cell's run (runs are contiguous after the sort).
__global__ __launch_bounds__(T256) void k_run_counts(const uint32_t* keys_sorted, int64_t n,
                                                    const uint32_t* run_start,
                                                    uint32_t* count32) {
  int64_t j = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (j >= n) return;
  const uint32_t k = keys_sorted[j];
  if (j == n - 1 || keys_sorted[j + 1] != k) count32[k] = (uint32_t)(j + 1 - run_start[k]);
}

// Full count -> u8 byte and escape flag (count >= 255).
struct CountSrc {
  const uint32_t* c32;
  const uint64_t* c64;
  __device__ uint32_t operator()(int64_t i) const {
    return c32 ? c32[i] : (uint32_t)(c64[i] & 0xffffffffull);
  }
};

// Per block of T256 cells: the byte counts, and the block's number of escapes in bcnt.
__global__ __launch_bounds__(T256) void k_count_bytes(CountSrc src, int64_t ncell,
                                                     uint8_t* count, uint32_t* bcnt) {
  const int64_t i = (int64_t)blockIdx.x * T256 + threadIdx.x;
  const uint32_t c = i < ncell ? src(i) : 0u;
  if (i < ncell) count[i] = (uint8_t)(c >= 255u ? 255u : c);
  const int ne = __syncthreads_count(c >= 255u);
  if (threadIdx.x == 0) bcnt[blockIdx.x] = (uint32_t)ne;
}

// The escape table in cell order: one thread per block of T256 cells writes that block's
// escapes from boff[b] (the exclusive prefix of the block counts, boff[nb] the total);
// blocks without escapes, nearly all of them, read one word.
__global__ __launch_bounds__(T256) void k_escapes(CountSrc src, int64_t ncell, int64_t nb,
                                                 const uint32_t* bcnt, const int64_t* boff,
                                                 uint64_t* esc, int64_t cap, pm_shdr* h,
                                                 DevErr* err) {
  const int64_t b = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (b == 0) {
    const int64_t ne = boff[nb];
    h->n_esc = ne;
    if (ne > cap) latch_error(err, ERRBIT_CAPACITY, ne);
  }
  if (b >= nb || bcnt[b] == 0) return;
  int64_t k = boff[b];
  const int64_t i1 = min((b + 1) * T256, ncell);
  for (int64_t i = b * T256; i < i1; ++i) {
    const uint32_t c = src(i);
    if (c >= 255u) {
      if (k < cap) {
        esc[2 * k] = (uint64_t)i;
        esc[2 * k + 1] = (uint64_t)c;
      }
      ++k;
    }
  }
}

__global__ void k_check_total(const int64_t* off, int64_t ncell, int64_t n, DevErr* err) {
  if (off[ncell] != n) latch_error(err, ERRBIT_CORRUPT);
}

__device__ inline int64_t find_cell(const int64_t* off, int64_t ncell, int64_t j) {
  // largest c with off[c] <= j (cells with zero particles are skipped)
  int64_t lo = 0, hi = ncell;  // off[lo] <= j < off[hi]
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) >> 1;
    if (off[mid] <= j) lo = mid; else hi = mid;
  }
  return lo;
}

template <int P, int V>
__global__ __launch_bounds__(T256) void k_decode(const void* pos_, const void* vel_,
                                                const pm_shdr* h, const int64_t* off,
                                                int64_t n, Geom g, float* x, float* v) {
  const typename PosCode<P>::T* pos = (const typename PosCode<P>::T*)pos_;
  const typename VelCode<V>::T* vel = (const typename VelCode<V>::T*)vel_;
  int64_t j = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (j >= n) return;
  uint32_t cell[3];
  key_cell(g, (uint32_t)find_cell(off, g.ncell3, j), cell[0], cell[1], cell[2]);
  float vmax = h->v_max;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const uint32_t u = (cell[a] << (8 * P)) | pos[3 * j + a];
    // 2-byte codes reach 2^26: the bin centre in float64, rounded once (as the 1-byte
    // form's float32 arithmetic is exact)
    x[3 * j + a] = P == 1 ? pos_decode(u, g.LS)
                          : (float)(((double)u + 0.5) * ((double)g.LS * 0x1p-8));
    v[3 * j + a] = vel_decode_v<V>(vel[3 * j + a], vmax);
  }
}

// ---------------------------------------------------------------- byte stream --
// Block sum of the checksum terms, stored at the block's index (integer: exact).
__device__ inline void block_sum_store(uint64_t s, uint64_t* part) {
  __shared__ uint64_t sm[T256 / 64];
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < T256 / 64; ++q) s += sm[q];
    part[blockIdx.x] = s;
  }
}

struct GetPackBytes {
  const int64_t* off;
  int64_t rb;  // record bytes: 3 (P + V)
  __device__ int64_t operator()(int64_t c) const {
    int64_t k = off[c + 1] - off[c];
    return 1 + (k >= 255 ? 4 : 0) + rb * k;
  }
};

__global__ __launch_bounds__(T256) void k_pack_cells(const int64_t* off, const int64_t* boff,
                                                    int64_t ncell, uint8_t* body,
                                                    int64_t cap_body, uint64_t* csum) {
  int64_t c = (int64_t)blockIdx.x * T256 + threadIdx.x;
  uint64_t s = 0;
  if (c < ncell && boff[ncell] <= cap_body) {
    int64_t k = off[c + 1] - off[c];
    int64_t o = boff[c];
    if (k >= 255) {
      uint8_t b[5] = {255, (uint8_t)(k & 255), (uint8_t)((k >> 8) & 255),
                      (uint8_t)((k >> 16) & 255), (uint8_t)((k >> 24) & 255)};
      for (int q = 0; q < 5; ++q) {
        body[o + q] = b[q];
        s += (2ull * (uint64_t)(o + q) + 1ull) * b[q];
      }
    } else {
      body[o] = (uint8_t)k;
      s += (2ull * (uint64_t)o + 1ull) * (uint64_t)k;
    }
  }
  block_sum_store(s, csum);
}

template <int P, int V>
__global__ __launch_bounds__(T256) void k_pack_records(const void* pos_, const void* vel_,
                                                      const int64_t* off, const int64_t* boff,
                                                      int64_t n, int64_t ncell, uint8_t* body,
                                                      int64_t cap_body, uint64_t* csum) {
  constexpr int RB = 3 * (P + V);  // record: x, y, z codes, then vx, vy, vz (little-endian)
  const typename PosCode<P>::T* pos = (const typename PosCode<P>::T*)pos_;
  const typename VelCode<V>::T* vel = (const typename VelCode<V>::T*)vel_;
  int64_t j = (int64_t)blockIdx.x * T256 + threadIdx.x;
  uint64_t s = 0;
  if (j < n && boff[ncell] <= cap_body) {
    int64_t c = find_cell(off, ncell, j);
    int64_t k = off[c + 1] - off[c];
    int64_t o = boff[c] + (k >= 255 ? 5 : 1) + RB * (j - off[c]);
    // counts inconsistent with n (latched by the offset check): write nothing
    if (o + RB > boff[ncell]) o = -1;
    uint8_t b[RB];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const uint32_t w = pos[3 * j + a];
#pragma unroll
      for (int q = 0; q < P; ++q) b[P * a + q] = (uint8_t)((w >> (8 * q)) & 255u);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const uint32_t w = vel[3 * j + a];
#pragma unroll
      for (int q = 0; q < V; ++q) b[3 * P + V * a + q] = (uint8_t)((w >> (8 * q)) & 255u);
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      if (o < 0) break;
      body[o + q] = b[q];
      s += (2ull * (uint64_t)(o + q) + 1ull) * b[q];
    }
  }
  block_sum_store(s, csum);
}

// csum[0..nparts) -> csum[nparts] (sum mod 2^64, fixed order per thread, exact anyway)
__global__ __launch_bounds__(1024) void k_fold_sum(uint64_t* csum, int64_t nparts) {
  __shared__ uint64_t sm[16];
  uint64_t a = 0;
  for (int64_t i = threadIdx.x; i < nparts; i += 1024) a += csum[i];
  for (int d = 32; d >= 1; d >>= 1) a += __shfl_xor(a, d, 64);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < 16; ++q) a += sm[q];
    csum[nparts] = a;
  }
}

__global__ void k_pack_header(uint8_t* buf, int64_t cap, const int64_t* boff, int64_t ncell,
                              const uint64_t* csum, const pm_shdr* h, int32_t sid, int32_t B,
                              int64_t n, int64_t nc, double mass, uint32_t widths,
                              int64_t* used, DevErr* err) {
  int64_t body = boff[ncell];
  int64_t total = PM_STREAM_HEADER + body;
  *used = total;
  if (total > cap) {
    latch_error(err, ERRBIT_CAPACITY, total);
    return;
  }
  uint8_t hb[PM_STREAM_HEADER];
  for (int i = 0; i < PM_STREAM_HEADER; ++i) hb[i] = 0;
  auto put = [&](int o, const void* p, int len) {
    const uint8_t* q = (const uint8_t*)p;
    for (int i = 0; i < len; ++i) hb[o + i] = q[i];
  };
  const char magic[4] = {'P', 'M', 'C', '1'};
  uint32_t ver = 1, usid = (uint32_t)sid, ub = (uint32_t)B;
  const uint64_t cs = *csum;
  uint64_t un = (uint64_t)n, unc = (uint64_t)nc, ubl = (uint64_t)body;
  float vmax = h->v_max;
  put(0, magic, 4);
  put(4, &ver, 4);
  put(8, &usid, 4);
  put(12, &ub, 4);
  put(16, &un, 8);
  put(24, &unc, 8);
  put(32, &vmax, 4);
  put(36, &widths, 4);  // code widths, 0 for the paper's 1-byte positions, 2-byte velocities
  put(40, &mass, 8);
  put(48, &cs, 8);
  put(56, &ubl, 8);
  for (int i = 0; i < PM_STREAM_HEADER; ++i) buf[i] = hb[i];
}

// ------------------------------------------------------------------ reductions --
constexpr int RED_BLOCKS = 512;

__global__ __launch_bounds__(T256) void k_reduce_mesh(const float* rho, int64_t n,
                                                     double* part) {
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * T256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * T256)
    s += (double)rho[i];
  __shared__ double lw[T256 / 64];
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
  if ((threadIdx.x & 63) == 0) lw[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = lw[0] + lw[1] + lw[2] + lw[3];
}

// Per block: sum of v and of the CIC-interpolated acceleration a_i over one species'
// particles (decoded bin centres for compressed streams), in float64, stored at the
// block's index. off: cell offsets of a compressed stream (finds each particle's cell).
struct RedSpecies {
  pm_species sp;
  const int64_t* off;
};

__device__ inline void cic_accumulate(const float* acc, int64_t ng, const float xm[3],
                                      double a[3]) {
  int64_t i[3];
  float f[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const float fl = floorf(xm[q]);
    f[q] = xm[q] - fl;
    int64_t k = (int64_t)fl % ng;
    i[q] = k < 0 ? k + ng : k;
  }
  const int64_t n3 = ng * ng * ng;
#pragma unroll
  for (int dz = 0; dz < 2; ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) {
        const float w = (dx ? f[0] : 1.f - f[0]) * (dy ? f[1] : 1.f - f[1]) *
                        (dz ? f[2] : 1.f - f[2]);
        const int64_t node = (((i[2] + dz) % ng) * ng + (i[1] + dy) % ng) * ng +
                             (i[0] + dx) % ng;
#pragma unroll
        for (int q = 0; q < 3; ++q) a[q] += (double)(w * acc[q * n3 + node]);
      }
}

template <int P, int V>
__global__ __launch_bounds__(T256) void k_reduce_particles(RedSpecies rs, const float* acc,
                                                          Geom g, double* part) {
  const pm_species& sp = rs.sp;
  const typename PosCode<P>::T* pos = (const typename PosCode<P>::T*)sp.pos;
  const typename VelCode<V>::T* vel = (const typename VelCode<V>::T*)sp.vel;
  double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const float fng = g.ngL;
  const float rs_cell = (float)g.r / 256.f;  // mesh cells per 1-byte position quantum
  for (int64_t j = (int64_t)blockIdx.x * T256 + threadIdx.x; j < sp.n;
       j += (int64_t)gridDim.x * T256) {
    float xm[3];
    if (sp.layout == PM_FLOAT) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        s[a] += (double)sp.v[3 * j + a];
        xm[a] = sp.x[3 * j + a] * fng;  // mesh units (exact for a power-of-two box)
      }
    } else {
      uint32_t cell[3];
      key_cell(g, (uint32_t)find_cell(rs.off, g.ncell3, j), cell[0], cell[1], cell[2]);
      const float vmax = sp.hdr->v_max;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        s[a] += (double)vel_decode_v<V>(vel[3 * j + a], vmax);
        const uint32_t u = (cell[a] << (8 * P)) | pos[3 * j + a];
        // bin centre in mesh units: exact in float32 for 1-byte codes, in float64 (then
        // rounded once) for 2-byte codes
        xm[a] = P == 1 ? ((float)u + 0.5f) * rs_cell
                       : (float)(((double)u + 0.5) * ((double)g.r * 0x1p-16));
      }
    }
    if (acc) cic_accumulate(acc, g.ng, xm, s + 3);
  }
  __shared__ double lw[6][T256 / 64];
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    for (int d = 32; d >= 1; d >>= 1) s[a] += __shfl_xor(s[a], d, 64);
    if ((threadIdx.x & 63) == 0) lw[a][threadIdx.x >> 6] = s[a];
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int a = threadIdx.x;
    part[6 * blockIdx.x + a] = lw[a][0] + lw[a][1] + lw[a][2] + lw[a][3];
  }
}

struct RedMeta {
  int n_sp;
  double mass[4];
  int64_t count[4];
};

// Fixed-order final sums (deterministic). out[0] mesh mass, out[1] particle mass,
// out[2..4] total momentum, out[5..7] total sum m a; per species s, out[8 + 6 s ..] =
// m_s sum v (3) and m_s sum a (3).
__global__ void k_reduce_final(const double* pmesh, int nmesh_part, double cell_vol,
                               const double* ppart, RedMeta meta, double* out) {
  double m = 0.0;
  for (int i = 0; i < nmesh_part; ++i) m += pmesh[i];
  out[0] = m * cell_vol;
  double mt = 0.0, tot[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int s = 0; s < meta.n_sp; ++s) {
    mt += meta.mass[s] * (double)meta.count[s];
    double sum[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = 0; b < RED_BLOCKS; ++b) {
      const double* q = ppart + 6 * (int64_t)(s * RED_BLOCKS + b);
      for (int a = 0; a < 6; ++a) sum[a] += q[a];
    }
    for (int a = 0; a < 6; ++a) {
      out[8 + 6 * s + a] = meta.mass[s] * sum[a];
      tot[a] += meta.mass[s] * sum[a];
    }
  }
  out[1] = mt;
  for (int a = 0; a < 6; ++a) out[2 + a] = tot[a];
}

}  // namespace

pm_status run_cell_offsets(pm_context* c, const pm_species* sp, int64_t* off) {
  ProfScope ps(c, ST_OFFSETS);
  return scan_counts_into(c, sp, off, nullptr);
}

// cell offsets of a compressed stream and the check that the counts sum to n; bsum
// (nullable) holds the scan's block sums
pm_status scan_counts_into(pm_context* c, const pm_species* sp, int64_t* off, int64_t* bsum) {
  pm_status s = scan_generic(c, GetCount{sp->count, sp->esc, sp->hdr}, c->g.ncell3, off, bsum);
  if (s != PM_OK) return s;
  hipLaunchKernelGGL(k_check_total, dim3(1), dim3(1), 0, c->stream, off, c->g.ncell3, sp->n,
                     c->err);
  PM_LAUNCH_CHECK();
  return PM_OK;
}

pm_status run_finalize_counts(pm_context* c, const uint32_t* cnt32, const uint64_t* cnt64,
                              pm_species* out) {
  const int64_t nc3 = c->g.ncell3;
  const int64_t nb = cdiv(nc3, T256);  // blocks of T256 cells
  uint32_t* bcnt = (uint32_t*)scratch(c, SC_FLAG, (size_t)nb * 4);
  int64_t* boff = (int64_t*)scratch(c, SC_FOFF, (size_t)(nb + 1) * 8);
  if (!bcnt || !boff) return PM_ERR_NOMEM;
  CountSrc src{cnt32, cnt64};
  hipLaunchKernelGGL(k_count_bytes, dim3((unsigned)nb), dim3(T256), 0, c->stream, src, nc3,
                     out->count, bcnt);
  PM_LAUNCH_CHECK();
  pm_status s = scan_u32(c, bcnt, nb, boff);
  if (s != PM_OK) return s;
  hipLaunchKernelGGL(k_escapes, dim3((unsigned)cdiv(nb, T256)), dim3(T256), 0, c->stream, src,
                     nc3, nb, bcnt, boff, out->esc, out->cap_esc, out->hdr, c->err);
  PM_LAUNCH_CHECK();
  return PM_OK;
}

pm_status run_encode(pm_context* c, const pm_species* in, pm_species* out, int64_t* perm) {
  ProfScope ps(c, ST_CODEC);
  const int64_t n = in->n;
  const Geom& g = c->g;
  hipLaunchKernelGGL(k_init_hdr, dim3(1), dim3(1), 0, c->stream, out->hdr);
  PM_LAUNCH_CHECK();
  uint32_t* cnt32 = (uint32_t*)scratch(c, SC_COUNT32, (size_t)g.ncell3 * 4);
  if (!cnt32) return PM_ERR_NOMEM;
  pm_status s = launch_fill_u32(c, cnt32, g.ncell3, 0u);
  if (s != PM_OK) return s;
  if (n > 0) {
    int64_t blocks = cdiv(3 * n, T256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_absmax, dim3((unsigned)blocks), dim3(T256), 0, c->stream, in->v,
                       3 * n, out->hdr, c->err);
    uint32_t* ka = (uint32_t*)scratch(c, SC_KEYA, (size_t)n * 4);
    uint32_t* va = (uint32_t*)scratch(c, SC_VALA, (size_t)n * 4);
    uint32_t* kb = (uint32_t*)scratch(c, SC_KEYB, (size_t)n * 4);
    uint32_t* vb = (uint32_t*)scratch(c, SC_VALB, (size_t)n * 4);
    if (!ka || !va || !kb || !vb) return PM_ERR_NOMEM;
    unsigned nbk = (unsigned)cdiv(n, T256);
    hipLaunchKernelGGL(k_encode_keys, dim3(nbk), dim3(T256), 0, c->stream, in->x, n, g, ka,
                       va, c->err);
    PM_LAUNCH_CHECK();
    int bits = 3 * (g.lgB + g.lgnb);
    s = radix_sort_pairs(c, &ka, &va, &kb, &vb, n, bits);
    if (s != PM_OK) return s;
    const int64_t nb = (int64_t)nbk;
    int32_t* part = (int32_t*)scratch(c, SC_PARTS, (size_t)nb * 8);
    uint32_t* rstart = (uint32_t*)scratch(c, SC_FLAG, (size_t)g.ncell3 * 4);
    if (!part || !rstart) return PM_ERR_NOMEM;
    s = width_dispatch(width_kind(*out), [&](auto P_, auto V_) {
      hipLaunchKernelGGL((k_encode_gather<decltype(P_)::value, decltype(V_)::value>),
                         dim3(nbk), dim3(T256), 0, c->stream, in->x, in->v, n, g, ka, va,
                         (void*)out->pos, (void*)out->vel, perm, rstart, out->hdr, part,
                         part + nb);
      return PM_OK;
    });
    if (s != PM_OK) return s;
    PM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_run_counts, dim3(nbk), dim3(T256), 0, c->stream, ka, n, rstart, cnt32);
    PM_LAUNCH_CHECK();
    if ((s = fold_minmax_to_header(c, part, part + nb, nb, out->hdr)) != PM_OK) return s;
  }
  return run_finalize_counts(c, cnt32, nullptr, out);
}

pm_status run_decode(pm_context* c, const pm_species* in, pm_species* out) {
  const int64_t n = in->n;
  int64_t* off = (int64_t*)scratch(c, SC_OFF, (size_t)(c->g.ncell3 + 1) * 8);
  if (!off) return PM_ERR_NOMEM;
  pm_status s = run_cell_offsets(c, in, off);
  if (s != PM_OK || n == 0) return s;
  s = width_dispatch(width_kind(*in), [&](auto P_, auto V_) {
    hipLaunchKernelGGL((k_decode<decltype(P_)::value, decltype(V_)::value>),
                       dim3((unsigned)cdiv(n, T256)), dim3(T256), 0, c->stream,
                       (const void*)in->pos, (const void*)in->vel, in->hdr, off, n, c->g,
                       out->x, out->v);
    return PM_OK;
  });
  if (s != PM_OK) return s;
  PM_LAUNCH_CHECK();
  return PM_OK;
}

pm_status run_pack(pm_context* c, const pm_species* sp, int32_t sid, uint8_t* buf,
                   int64_t cap, int64_t* used) {
  const int64_t nc3 = c->g.ncell3;
  int64_t* off = (int64_t*)scratch(c, SC_OFF, (size_t)(nc3 + 1) * 8);
  int64_t* boff = (int64_t*)scratch(c, SC_FOFF, (size_t)(nc3 + 1) * 8);
  const int64_t nbc = cdiv(nc3, T256), nbr = cdiv(sp->n, T256);
  uint64_t* csum = (uint64_t*)scratch(c, SC_PARTS, (size_t)(nbc + nbr + 1) * 8);
  if (!off || !boff || !csum) return PM_ERR_NOMEM;
  pm_status s = run_cell_offsets(c, sp, off);
  if (s != PM_OK) return s;
  const int64_t rb = 3 * (width_pos(*sp) + width_vel(*sp));
  s = scan_generic_pack(c, off, nc3, boff, rb);
  if (s != PM_OK) return s;
  int64_t cap_body = cap - PM_STREAM_HEADER;
  uint8_t* body = buf + PM_STREAM_HEADER;
  hipLaunchKernelGGL(k_pack_cells, dim3((unsigned)nbc), dim3(T256), 0, c->stream,
                     off, boff, nc3, body, cap_body, csum);
  if (nbr > 0) {
    s = width_dispatch(width_kind(*sp), [&](auto P_, auto V_) {
      hipLaunchKernelGGL((k_pack_records<decltype(P_)::value, decltype(V_)::value>),
                         dim3((unsigned)nbr), dim3(T256), 0, c->stream, (const void*)sp->pos,
                         (const void*)sp->vel, off, boff, sp->n, nc3, body, cap_body,
                         csum + nbc);
      return PM_OK;
    });
    if (s != PM_OK) return s;
  }
  hipLaunchKernelGGL(k_fold_sum, dim3(1), dim3(1024), 0, c->stream, csum, nbc + nbr);
  hipLaunchKernelGGL(k_pack_header, dim3(1), dim3(1), 0, c->stream, buf, cap, boff, nc3,
                     csum + nbc + nbr, sp->hdr, sid, c->g.B, sp->n, c->g.nc, sp->mass,
                     (uint32_t)sp->widths, used, c->err);
  PM_LAUNCH_CHECK();
  return PM_OK;
}

pm_status scan_generic_pack(pm_context* c, const int64_t* off, int64_t n, int64_t* out,
                            int64_t rb) {
  return scan_generic(c, GetPackBytes{off, rb}, n, out);
}

namespace {
// Float64 reductions with the caller's choice of buffers: part (RED_BLOCKS * 25 doubles),
// off_of(s) the cell offsets of compressed species s ((ncell3 + 1) int64), bsum the scan's
// block sums (nullptr: the context's scratch).
template <typename OffOf>
pm_status reduce_core(pm_context* c, const pm_species* sp, int n_sp, const float* rho,
                      const float* acc, double* out, double* part, OffOf off_of,
                      int64_t* bsum) {
  if (n_sp < 0 || n_sp > 4) return PM_ERR_ARG;
  double* pmesh = part;
  double* ppart = part + RED_BLOCKS;
  RedMeta meta{};
  meta.n_sp = n_sp;
  int nmp = 0;
  if (rho) {
    nmp = RED_BLOCKS;
    hipLaunchKernelGGL(k_reduce_mesh, dim3(RED_BLOCKS), dim3(T256), 0, c->stream, rho,
                       c->g.ng * c->g.ng * c->g.ng, pmesh);
  }
  for (int s = 0; s < n_sp; ++s) {
    meta.mass[s] = sp[s].mass;
    meta.count[s] = sp[s].n;
    RedSpecies rs{sp[s], nullptr};
    if (sp[s].layout == PM_COMPRESSED) {
      int64_t* off = off_of(s);
      if (!off) return PM_ERR_NOMEM;
      pm_status st = scan_counts_into(c, &sp[s], off, bsum);
      if (st != PM_OK) return st;
      rs.off = off;
    }
    double* pp = ppart + 6 * (int64_t)s * RED_BLOCKS;
    const int kind = sp[s].layout == PM_COMPRESSED ? width_kind(sp[s]) : 0;
    pm_status st = width_dispatch(kind, [&](auto P_, auto V_) {
      hipLaunchKernelGGL((k_reduce_particles<decltype(P_)::value, decltype(V_)::value>),
                         dim3(RED_BLOCKS), dim3(T256), 0, c->stream, rs, acc, c->g, pp);
      return PM_OK;
    });
    if (st != PM_OK) return st;
  }
  const double dv = c->g.box * c->g.box * c->g.box / ((double)c->g.ng * c->g.ng * c->g.ng);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(1), 0, c->stream, pmesh, nmp, dv, ppart,
                     meta, out);
  PM_LAUNCH_CHECK();
  return PM_OK;
}
}  // namespace

pm_status run_reduce(pm_context* c, const pm_species* sp, int n_sp, const float* rho,
                     const float* acc, double* out) {
  double* part = (double*)scratch(c, SC_MISC, (size_t)(RED_BLOCKS * (6 * 4 + 1)) * 8);
  if (!part) return PM_ERR_NOMEM;
  return reduce_core(c, sp, n_sp, rho, acc, out, part, [&](int s) {
    return (int64_t*)scratch(c, SC_SPOFF0 + s, (size_t)(c->g.ncell3 + 1) * 8);
  }, nullptr);
}

// ------------------------------------------------------- allocation-free reduce --
// For callers that cannot allocate device memory. Every buffer of pm_reduce_noalloc lives
// in one fixed array per device: the per-workgroup partial sums, the cell offsets of one
// compressed species at a time (species are reduced one after the other on the stream)
// and the block sums of their scan. Its device address is taken once per device, when a
// context is created there; calls that overlap on one device share the array and race.
namespace noalloc {
constexpr int64_t NC3_MAX = 32768;  // compressed species: n_cell^3 <= 32^3
constexpr size_t PART_BYTES = (size_t)RED_BLOCKS * (6 * 4 + 1) * 8;
constexpr size_t OFF_BYTES = (size_t)(NC3_MAX + 1) * 8;
constexpr size_t BSUM_BYTES = 256;  // cdiv(NC3_MAX + 1, 4096) int64 block sums
constexpr size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t BYTES = a256(PART_BYTES) + a256(OFF_BYTES) + BSUM_BYTES;
static __device__ __align__(256) unsigned char scratch[BYTES];

std::mutex mu;
unsigned char* addr[256] = {};
}  // namespace noalloc

pm_status noalloc_init(pm_context* c) {
  if (c->device < 0 || c->device >= 256) return PM_ERR_DEVICE;
  std::lock_guard<std::mutex> lock(noalloc::mu);
  if (!noalloc::addr[c->device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc::scratch)) != hipSuccess || !p)
      return PM_ERR_DEVICE;
    noalloc::addr[c->device] = (unsigned char*)p;
  }
  c->na_scratch = noalloc::addr[c->device];
  return PM_OK;
}

pm_status run_reduce_noalloc(pm_context* c, const pm_species* sp, int n_sp,
                             const float* rho, const float* acc, double* out) {
  using namespace noalloc;
  if (!c->na_scratch) return PM_ERR_DEVICE;
  for (int s = 0; s < n_sp; ++s)
    if (sp[s].layout == PM_COMPRESSED && c->g.ncell3 > NC3_MAX) return PM_ERR_SHAPE;
  unsigned char* base = c->na_scratch;
  double* part = (double*)base;
  int64_t* off = (int64_t*)(base + a256(PART_BYTES));
  int64_t* bsum = (int64_t*)(base + a256(PART_BYTES) + a256(OFF_BYTES));
  return reduce_core(c, sp, n_sp, rho, acc, out, part, [&](int) { return off; }, bsum);
}

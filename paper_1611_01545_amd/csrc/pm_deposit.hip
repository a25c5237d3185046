// Cloud-in-cell mass deposit (Sec. 2.1; CIC is named in Sec. 2.3), both species on
// one mesh (Sec. 2.1 footnote).
//
// Compressed particles are cell-sorted, so a workgroup owns a cube of R^3 mesh nodes
// (R = T r, T compression cells of r mesh cells each) and gathers exactly the
// particles that can reach those nodes: its own T^3 cells plus the one-cell shell
// on the -x/-y/-z faces, whose particles reach the tile's lowest node plane through
// their upper CIC corner. Every node has exactly one owner, so the tile is written
// with plain stores and no mesh-wide atomics or halo pass are needed. The paper's
// CPU code avoids write races with a strided loop over cells (Sec. 2.3); here the
// races inside the tile are resolved by LDS atomics.
//
// Weights are exact: a compressed position sits at the bin centre (2u+1)/(512 n_c),
// i.e. at (2u+1) r / 512 mesh cells, so each axis weight is an integer multiple of
// 1/512 and their product an integer multiple of 2^-27. Each species' weights are
// summed as integers in LDS (exact, so independent of the order of the atomics): a
// 32-bit word per node that wraps, plus a 16-bit count of its wraps, so 48 bits per
// node in 6 bytes. Each species' sum is scaled by its mass in FP64, rounded once to
// float and added to the thread's float node densities in a fixed species order: every
// run, and the recomputation in the adjoint, gives bit-identical densities.
//
// The tile loop is bound by latency (cell offsets, then particle codes, per species),
// so what pays is tiles in flight: the 26 KB of LDS and 74 VGPRs of a 16^3-node tile
// let six workgroups share a CU (64-bit sums in LDS and FP64 densities held four), and
// the prefix over the tile's cells is a DPP wave scan with a single barrier.
#include "pm_codec.h"
#include "pm_scan.h"

namespace {

constexpr int DEP_THREADS = 256;
constexpr int MAX_SP = 4;

struct DepSpecies {
  int64_t n;           // particles (bounds guard against inconsistent counts)
  const void* pos;     // position codes, P bytes per axis
  const int64_t* off;  // [ncell3 + 1]
  double unit;         // density per weight unit 2^-27: m_s n_g^3 2^-27
};
struct DepArgs {
  DepSpecies sp[MAX_SP];
  int n_sp;
  int T;   // tile side in cells
  int r;   // mesh cells per compression cell
  int R;   // tile side in nodes
};

// byte offset of the cell starts after the weight sums (low words, then carries)
__host__ __device__ inline size_t dep_cst_offset(int R3) {
  return ((size_t)R3 * 4 + (size_t)((R3 + 1) / 2) * 4 + 7) & ~(size_t)7;
}

__device__ inline int wrapc(int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); }

// TT: tile side in cells (compile time, 0: runtime A.T); PB: position bytes per axis. With
// PB = 2 the offset inside a cell has 17 fractional bits of a mesh cell per axis, and each
// node's weight (the exact product, a multiple of 2^-51) is rounded to a multiple of
// 2^-27, the unit of the 1-byte form, so that the same integer sums apply.
template <int TT, int PB = 1>
__global__ __launch_bounds__(DEP_THREADS) void k_deposit_tile(DepArgs A, Geom g, float* rho) {
  using PT = typename PosCode<PB>::T;
  constexpr int FB = 8 * PB + 1;              // fractional bits of a mesh coordinate
  constexpr int ONE = 1 << FB;                // one mesh cell
  constexpr uint32_t FMASK = (uint32_t)ONE - 1u;
  extern __shared__ unsigned char smem[];
  // compile-time tiles have T r = 16 nodes per side (T = 16 / r)
  const int T = TT ? TT : A.T, R = TT ? 16 : A.R, r = TT ? 16 / TT : A.r;
  const bool spread = !TT && r == 1;  // the coarse mesh of the two-level force
  const int E = T + 1;              // extended cells per side
  const int NE = E * E * E;
  const int R3 = R * R * R;
  __shared__ int wsum[DEP_THREADS / 64];
  // a node's weight sum is hi 2^32 + lo: lo wraps in the LDS atomics, and each wrap
  // increments a 16-bit carry counter (two per word)
  uint32_t* wlo = (uint32_t*)smem;                    // [R3]
  uint32_t* whi = wlo + R3;                           // [(R3 + 1) / 2]
  int64_t* cst = (int64_t*)(smem + dep_cst_offset(R3));  // [NE] stream start of each extended cell
  int* pre = (int*)(cst + NE);                        // [NE + 1] particle prefix over extended cells
  const int nt = (int)(g.nc / T);
  const int64_t tile = xcd_tile(blockIdx.x, (int64_t)nt * nt * nt);
  const int tx = (int)(tile % nt), ty = (int)((tile / nt) % nt), tz = (int)(tile / ((int64_t)nt * nt));
  const int ncs = (int)g.nc;

  for (int i = threadIdx.x; i < R3; i += DEP_THREADS) wlo[i] = 0u;
  // per-thread density of its nodes i = threadIdx.x + k DEP_THREADS (R <= 16, so at most
  // 16 nodes), summed over species (and segments) in a fixed order
  constexpr int NPT = 4096 / DEP_THREADS;
  float racc[NPT];
#pragma unroll
  for (int k = 0; k < NPT; ++k) racc[k] = 0.0f;

  for (int s = 0; s < A.n_sp; ++s) {
    const DepSpecies sp = A.sp[s];
    // counts of the extended cells, then an exclusive prefix (single pass per wave)
    __syncthreads();
    for (int i = threadIdx.x; i < (R3 + 1) / 2; i += DEP_THREADS) whi[i] = 0u;
    for (int e = threadIdx.x; e < NE; e += DEP_THREADS) {
      int ex = e % E, ey = (e / E) % E, ez = e / (E * E);
      int cx = wrapc(tx * T + ex - 1, ncs), cy = wrapc(ty * T + ey - 1, ncs),
          cz = wrapc(tz * T + ez - 1, ncs);
      uint32_t key = cell_key(g, cx, cy, cz);
      const int64_t o0 = sp.off[key], o1 = sp.off[key + 1];
      cst[e] = o0;
      pre[e + 1] = (int)(o1 - o0);
    }
    __syncthreads();
    {
      // block-wide inclusive prefix of pre[1..NE]: each thread owns K consecutive
      const int K = (NE + DEP_THREADS - 1) / DEP_THREADS;
      const int e0 = 1 + threadIdx.x * K;
      int loc = 0;
      for (int k = 0; k < K; ++k)
        if (e0 + k <= NE) loc += pre[e0 + k];
      int base = pmscan::block_excl_scan_i32(loc, wsum);
      for (int k = 0; k < K; ++k)
        if (e0 + k <= NE) {
          base += pre[e0 + k];
          pre[e0 + k] = base;
        }
      if (threadIdx.x == 0) pre[0] = 0;
    }
    __syncthreads();
    const int P = pre[NE];
    // U particles per thread per round: their code loads are issued together
    constexpr int U = 2;
    static_assert(DEP_THREADS * U == 512, "the spread order is a transpose of 8 x 64 slots");
    // the carries count at most 2^16 wraps, i.e. 2^48 weight units per node: segments
    // of 2^21 particles (each adds < 2^27 to a node) are flushed one by one; every
    // tile of a realistic input has a single segment
    constexpr int SEG = 1 << 21;
    for (int s0 = 0;; s0 += SEG) {
      const int s1 = P - s0 > SEG ? s0 + SEG : P;
      for (int rb = s0; rb < s1; rb += DEP_THREADS * U) {  // uniform across the block
        int eu[U];
        int64_t ju[U];
        uint32_t pb[U][3];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          // slot l of the round takes particle l, or, with one mesh cell per compression
          // cell (8 neutrinos per cell on 8^3 nodes), particle (l % 8) 64 + l / 8: the
          // lanes of one atomic then hit the nodes of eight different cells instead of
          // the same eight nodes (spread)
          const int l = (int)threadIdx.x + u * DEP_THREADS;
          const int q = rb + (spread ? ((l & 7) << 6) + (l >> 3) : l);
          // extended cell of flat particle q: largest e with pre[e] <= q
          int lo = 0, hi = NE;
          while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (pre[mid] <= q) lo = mid; else hi = mid;
          }
          eu[u] = lo;
          const int64_t j = cst[lo] + (q - pre[lo]);
          // counts inconsistent with n are latched by the offset check; q >= s1 is padding
          ok[u] = q < s1 && j < sp.n;
          ju[u] = ok[u] ? j : 0;  // n > 0 whenever P > 0
        }
        // all code loads of the round, then the arithmetic
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int a = 0; a < 3; ++a) pb[u][a] = ((const PT*)sp.pos)[3 * ju[u] + a];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (!ok[u]) continue;
          const int e = eu[u];
          const int ex = e % E, ey = (e / E) % E, ez = e / (E * E);
          int li[3], f[3];
          const int le[3] = {ex - 1, ey - 1, ez - 1};
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            // position inside the cell in units of 2^-FB mesh cells (1/512 for PB = 1)
            int gl = (2 * (int)pb[u][a] + 1) * r;
            li[a] = le[a] * r + (gl >> FB);
            f[a] = (int)((uint32_t)gl & FMASK);
          }
#pragma unroll
          for (int dz = 0; dz < 2; ++dz) {
            int nz = li[2] + dz;
            int wz = dz ? f[2] : ONE - f[2];
            if (nz < 0 || nz >= R || wz == 0) continue;
#pragma unroll
            for (int dy = 0; dy < 2; ++dy) {
              int ny = li[1] + dy;
              int wy = dy ? f[1] : ONE - f[1];
              if (ny < 0 || ny >= R || wy == 0) continue;
#pragma unroll
              for (int dx = 0; dx < 2; ++dx) {
                int nx = li[0] + dx;
                int wx = dx ? f[0] : ONE - f[0];
                if (nx < 0 || nx >= R || wx == 0) continue;
                uint32_t W;  // units of 2^-27
                if constexpr (PB == 1) {
                  W = (uint32_t)(wx * wy) * (uint32_t)wz;  // exact
                } else {
                  const uint64_t w3 = (uint64_t)wx * (uint64_t)wy * (uint64_t)wz;
                  W = (uint32_t)((w3 + (1ull << 23)) >> 24);  // 2^-51 -> 2^-27, rounded
                }
                const int i = (nz * R + ny) * R + nx;
                const uint32_t old = atomicAdd(&wlo[i], W);
                if (old > 0xffffffffu - W) atomicAdd(&whi[i >> 1], 1u << ((i & 1) * 16));
              }
            }
          }
        }
      }
      // the segment's integer weight sums into the thread's node densities
      __syncthreads();
#pragma unroll
      for (int k = 0; k < NPT; ++k) {
        const int i = threadIdx.x + k * DEP_THREADS;
        if (i < R3) {
          const uint64_t w =
              ((uint64_t)((whi[i >> 1] >> ((i & 1) * 16)) & 0xffffu) << 32) | wlo[i];
          racc[k] += (float)((double)w * sp.unit);
          wlo[i] = 0u;
        }
      }
      if (s1 >= P) break;
      __syncthreads();
      for (int i = threadIdx.x; i < (R3 + 1) / 2; i += DEP_THREADS) whi[i] = 0u;
      __syncthreads();
    }
  }
  const int64_t ng = g.ng;
  if (TT) {
    // R = 16: node i = threadIdx.x + 256 k has lx = i & 15, ly = (i >> 4) & 15, lz = k
    const int64_t ng2 = ng * ng;
    float* dst = rho + (int64_t)tz * 16 * ng2 +
                 ((int64_t)ty * 16 + ((threadIdx.x >> 4) & 15)) * ng + (int64_t)tx * 16 +
                 (threadIdx.x & 15);
#pragma unroll
    for (int k = 0; k < NPT; ++k) dst[k * ng2] = racc[k];
  } else {
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const int i = threadIdx.x + k * DEP_THREADS;
      if (i < R3) {
        int lx = i % R, ly = (i / R) % R, lz = i / (R * R);
        int64_t gx = (int64_t)tx * R + lx, gy = (int64_t)ty * R + ly,
                gz = (int64_t)tz * R + lz;
        rho[(gz * ng + gy) * ng + gx] = racc[k];
      }
    }
  }
}

// ---------------------------------------------------------- float-layout path --
// Unsorted float particles: fixed-point weights accumulated with 64-bit global atomics
// (still order independent), then converted.
__global__ __launch_bounds__(256) void k_deposit_float(const float* x, int64_t n, int64_t ng,
                                                      float ngL, double scale,
                                                      unsigned long long* acc) {
  int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= n) return;
  int64_t i[3];
  double f[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double u = (double)(x[3 * p + a] * ngL);  // mesh units (exact for a power-of-two box)
    double fl = floor(u);
    f[a] = u - fl;
    int64_t k = (int64_t)fl % ng;
    i[a] = k < 0 ? k + ng : k;
  }
#pragma unroll
  for (int dz = 0; dz < 2; ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) {
        double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
        unsigned long long q = (unsigned long long)__double2ll_rn(w * scale);
        if (!q) continue;
        int64_t nz = (i[2] + dz) % ng, ny = (i[1] + dy) % ng, nx = (i[0] + dx) % ng;
        atomicAdd(&acc[(nz * ng + ny) * ng + nx], q);
      }
}

__global__ __launch_bounds__(256) void k_fixed_to_float(const unsigned long long* acc, int64_t n,
                                                       double unit, float* rho) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) rho[i] = (float)((double)acc[i] * unit);
}

}  // namespace

int deposit_tile_cells(const Geom& g) {
  // 16 nodes per tile side (T r = 16), except with one mesh cell per compression cell
  // (the coarse mesh of the two-level force): 8^3-cell tiles, since 16^3 cells would
  // hold 83 KB of LDS and run one workgroup per CU
  int T = g.r == 1 ? 8 : 16 / g.r;
  if (T < 1) T = 1;
  if (T > g.nc) T = (int)g.nc;
  return T;
}

pm_status run_deposit_tile(pm_context* c, const pm_species* sp, int n_sp,
                           int64_t* const* offs, float* rho) {
  const Geom& g = c->g;
  if (n_sp > MAX_SP) return PM_ERR_ARG;
  const double ng3 = (double)g.ng * g.ng * g.ng / (g.box * g.box * g.box);  // 1 / Delta^3
  DepArgs A{};
  A.n_sp = 0;
  for (int s = 0; s < n_sp; ++s) {
    if (sp[s].n == 0 || sp[s].mass == 0.0) continue;
    A.sp[A.n_sp].n = sp[s].n;
    A.sp[A.n_sp].pos = sp[s].pos;
    A.sp[A.n_sp].off = offs[s];
    A.sp[A.n_sp].unit = sp[s].mass * ng3 * 0x1p-27;
    A.n_sp++;
  }
  A.r = g.r;
  A.T = deposit_tile_cells(g);
  A.R = A.T * g.r;
  if (A.R > 16) return PM_ERR_SHAPE;  // at most 16 nodes per thread
  int nt = (int)(g.nc / A.T);
  const size_t ne = (size_t)(A.T + 1) * (A.T + 1) * (A.T + 1);
  size_t lds = dep_cst_offset(A.R * A.R * A.R) + ne * 8 + (ne + 1) * 4;
  ProfScope ps(c, ST_DEPOSIT);
  const dim3 grid((unsigned)((int64_t)nt * nt * nt));
  // the compile-time variants assume T r = 16; one position width for every species
  const int kind = common_width_kind(sp, n_sp);
  if (kind < 0) return PM_ERR_ARG;
  if (width_pos(sp[0]) == 1) {
    if (A.T == 4 && A.r == 4)
      hipLaunchKernelGGL(k_deposit_tile<4>, grid, dim3(DEP_THREADS), lds, c->stream, A, g, rho);
    else if (A.T == 8 && A.r == 2)
      hipLaunchKernelGGL(k_deposit_tile<8>, grid, dim3(DEP_THREADS), lds, c->stream, A, g, rho);
    else
      hipLaunchKernelGGL(k_deposit_tile<0>, grid, dim3(DEP_THREADS), lds, c->stream, A, g, rho);
  } else {
    if (A.T == 4 && A.r == 4)
      hipLaunchKernelGGL((k_deposit_tile<4, 2>), grid, dim3(DEP_THREADS), lds, c->stream, A, g,
                         rho);
    else
      hipLaunchKernelGGL((k_deposit_tile<0, 2>), grid, dim3(DEP_THREADS), lds, c->stream, A, g,
                         rho);
  }
  PM_LAUNCH_CHECK();
  return PM_OK;
}

pm_status run_deposit(pm_context* c, const pm_species* sp, int n_sp, float* rho) {
  const Geom& g = c->g;
  if (n_sp <= 0 || n_sp > MAX_SP) return PM_ERR_ARG;
  int layout = sp[0].layout;
  for (int s = 1; s < n_sp; ++s)
    if (sp[s].layout != layout) return PM_ERR_ARG;
  if (layout == PM_COMPRESSED) {
    int64_t* offs[MAX_SP];
    for (int s = 0; s < n_sp; ++s) {
      offs[s] = (int64_t*)scratch(c, SC_SPOFF0 + s, (size_t)(g.ncell3 + 1) * 8);
      if (!offs[s]) return PM_ERR_NOMEM;
      pm_status st = run_cell_offsets(c, &sp[s], offs[s]);
      if (st != PM_OK) return st;
    }
    return run_deposit_tile(c, sp, n_sp, offs, rho);
  }
  // float layout
  ProfScope ps(c, ST_DEPOSIT);
  const int64_t n3 = g.ng * g.ng * g.ng;
  unsigned long long* acc = (unsigned long long*)scratch(c, SC_ACC64, (size_t)n3 * 8);
  if (!acc) return PM_ERR_NOMEM;
  pm_status st = launch_fill_u64(c, (uint64_t*)acc, n3, 0ull);
  if (st != PM_OK) return st;
  double mmax = 0.0;
  for (int s = 0; s < n_sp; ++s) mmax = fmax(mmax, sp[s].mass);
  for (int s = 0; s < n_sp; ++s) {
    if (sp[s].n == 0 || sp[s].mass == 0.0) continue;
    double scale = 0x1p32 * (sp[s].mass / mmax);
    hipLaunchKernelGGL(k_deposit_float, dim3((unsigned)cdiv(sp[s].n, 256)), dim3(256), 0,
                       c->stream, sp[s].x, sp[s].n, g.ng, g.ngL, scale, acc);
  }
  double unit = mmax > 0 ? mmax * 0x1p-32 * (double)n3 / (g.box * g.box * g.box) : 0.0;
  hipLaunchKernelGGL(k_fixed_to_float, dim3((unsigned)cdiv(n3, 256)), dim3(256), 0, c->stream,
                     acc, n3, unit, rho);
  PM_LAUNCH_CHECK();
  return PM_OK;
}

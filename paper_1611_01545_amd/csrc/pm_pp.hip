// The cell-local particle-particle (PP) force of eq. (4) (Sec. 2.1) on compressed
// streams: for every particle, the direct sum over the particles of all species that
// share its cell of the PM mesh,
//   a_i = G sum_{j != i, same mesh cell, r_ij >= r_soft} m_j (x_j - x_i) / r_ij^3,
// truncated below the softening length r_soft. The cell-sorted stream is the paper's
// linked list: a mesh cell lies inside one compression cell (r^3 mesh cells each), so a
// particle's partners are found among the particles of its compression cell, one
// contiguous range per species.
//
// One wave per brick of the stream order (four per workgroup), lanes on consecutive
// particles, grid.y over species: the brick's cell offsets of every species are staged
// in LDS, where each particle finds its cell (a binary search over the whole offset
// array in global memory, 27 dependent loads per particle at 512^3 cells, held the
// kernel at 49 ms at 2048^3). Positions are the bin centres in mesh
// units, (u + 1/2) r / 256, exact in float32, so the mesh cell and every difference x_j - x_i
// are exact; the cut is decided on the integer code differences (|du|^2 >= (r_soft S / L)^2),
// the force is summed in float32 in stream order (deterministic). The arithmetic is plain
// vector ALU work: about 20 flops per interacting pair.
#include "pm_codec.h"

namespace {

constexpr int PWB = 4;  // bricks (waves) per workgroup
constexpr int PCAP = 4096;  // bytes of partner codes a wave stages in LDS
constexpr int PMAXSP = 4;

struct PPSpecies {
  int64_t n;
  const void* pos;     // position codes, P bytes per axis
  const int64_t* off;  // cell offsets [ncell3 + 1]
  float mass;
  float* app;          // [n][3] accelerations, stream order
};

struct PPArgs {
  PPSpecies sp[PMAXSP];
  int n_sp;
  float g_scale;  // G / Delta^2 (distances in mesh units)
  double cut2;    // (r_soft S / L)^2 in squared position codes
};

// P: position bytes per axis (codes u = cell 256^P + offset; (2u + 1) r < 2^28)
template <int P>
__global__ __launch_bounds__(64 * PWB) void k_pp_accel(PPArgs A, Geom g, uint32_t* part) {
  using PC = typename PosCode<P>::T;
  using DT = typename std::conditional<P == 1, int, int64_t>::type;  // code differences
  constexpr int SH = 8 * P, FB = 8 * P + 1;
  // [PWB][n_sp][B^3 + 1] cell offsets of the bricks, then [PWB][PCAP] bytes of their codes
  extern __shared__ int64_t pso[];
  const int s = blockIdx.y;
  const PPSpecies& S = A.sp[s];
  const PC* spos = (const PC*)S.pos;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t b = (int64_t)blockIdx.x * PWB + wv;
  const int B3 = 1 << (3 * g.lgB);
  int64_t* so = pso + (int64_t)wv * A.n_sp * (B3 + 1);
  float m = 0.f;
  if (b < g.nbrick && S.n > 0) {  // uniform across the wave
    const int64_t k0 = b * B3;  // first cell key of the brick
    for (int t = 0; t < A.n_sp; ++t)
      for (int c = lane; c <= B3; c += 64)
        so[t * (B3 + 1) + c] = A.sp[t].n ? A.sp[t].off[k0 + c] : 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int64_t* mo = so + s * (B3 + 1);
    const int64_t base = mo[0], np = mo[B3] - base;
    // the brick's codes of every species in LDS when they fit (the partners' codes are
    // then LDS reads instead of three byte loads per partner)
    PC* sc = (PC*)(pso + (int64_t)PWB * A.n_sp * (B3 + 1)) + (int64_t)wv * (PCAP / sizeof(PC));
    int64_t tot = 0;
    for (int t = 0; t < A.n_sp; ++t) tot += so[t * (B3 + 1) + B3] - so[t * (B3 + 1)];
    const bool staged = 3 * tot * (int64_t)sizeof(PC) <= PCAP;
    int sbase[PMAXSP];
    if (staged) {
      int at = 0;
      for (int t = 0; t < A.n_sp; ++t) {
        sbase[t] = at;
        const int64_t j0 = so[t * (B3 + 1)], nt = 3 * (so[t * (B3 + 1) + B3] - j0);
        const PC* tp = (const PC*)A.sp[t].pos + 3 * j0;
        for (int c = lane; c < nt; c += 64) sc[at + c] = tp[c];
        at += (int)nt;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    for (int64_t q = lane; q < np; q += 64) {
      const int64_t i = base + q;
      if (i >= S.n) break;  // offsets inconsistent with n: latched by the offset check
      int lc = 0, hc = B3;  // local cell: the largest l with mo[l] <= i
      while (hc - lc > 1) {
        const int mid = (lc + hc) >> 1;
        if (mo[mid] <= i) lc = mid; else hc = mid;
      }
      const int64_t key = k0 + lc;
      uint32_t cx, cy, cz;
      key_cell(g, (uint32_t)key, cx, cy, cz);
      const int ui[3] = {(int)((cx << SH) | spos[3 * i]), (int)((cy << SH) | spos[3 * i + 1]),
                         (int)((cz << SH) | spos[3 * i + 2])};
      // mesh cell of a code: floor((2 u + 1) r / 2^FB)
      const int ci[3] = {((2 * ui[0] + 1) * g.r) >> FB, ((2 * ui[1] + 1) * g.r) >> FB,
                         ((2 * ui[2] + 1) * g.r) >> FB};
      const float unit = (float)g.r * (P == 1 ? (1.0f / 256.0f) : (1.0f / 65536.0f));
      float ax = 0.f, ay = 0.f, az = 0.f;
      for (int t = 0; t < A.n_sp; ++t) {
        const PPSpecies& T = A.sp[t];
        if (T.n == 0) continue;
        const int64_t j0 = so[t * (B3 + 1) + lc], j1 = so[t * (B3 + 1) + lc + 1];
        float sx = 0.f, sy = 0.f, sz = 0.f;
        // partner j's codes: the staged copy in LDS, or the stream
        const PC* tpos = (const PC*)T.pos;
        const PC* tloc = sc + (staged ? sbase[t] : 0);
        const int64_t jb = so[t * (B3 + 1)];  // the brick's first particle of species t
        for (int64_t j = j0; j < j1; ++j) {
          if (t == s && j == i) continue;
          int uj0, uj1, uj2;
          if (staged) {
            const int l = 3 * (int)(j - jb);
            uj0 = (int)((cx << SH) | tloc[l]);
            uj1 = (int)((cy << SH) | tloc[l + 1]);
            uj2 = (int)((cz << SH) | tloc[l + 2]);
          } else {
            uj0 = (int)((cx << SH) | tpos[3 * j]);
            uj1 = (int)((cy << SH) | tpos[3 * j + 1]);
            uj2 = (int)((cz << SH) | tpos[3 * j + 2]);
          }
          if ((((2 * uj0 + 1) * g.r) >> FB) != ci[0] || (((2 * uj1 + 1) * g.r) >> FB) != ci[1] ||
              (((2 * uj2 + 1) * g.r) >> FB) != ci[2])
            continue;
          const DT d0 = uj0 - ui[0], d1 = uj1 - ui[1], d2 = uj2 - ui[2];
          const DT r2c = d0 * d0 + d1 * d1 + d2 * d2;
          if ((double)r2c < A.cut2) continue;
          const float dx = (float)d0 * unit, dy = (float)d1 * unit, dz = (float)d2 * unit;
          const float r2 = dx * dx + dy * dy + dz * dz;
          const float inv = 1.0f / sqrtf(r2);
          const float w = inv * inv * inv;
          sx += dx * w;
          sy += dy * w;
          sz += dz * w;
        }
        ax += T.mass * sx;
        ay += T.mass * sy;
        az += T.mass * sz;
      }
      ax *= A.g_scale;
      ay *= A.g_scale;
      az *= A.g_scale;
      S.app[3 * i] = ax;
      S.app[3 * i + 1] = ay;
      S.app[3 * i + 2] = az;
      m = fmaxf(m, fmaxf(fabsf(ax), fmaxf(fabsf(ay), fabsf(az))));
    }
  }
  // per-block max |a| (non-negative float bits order as integers), folded afterwards
  __shared__ float wm[PWB];
  for (int d = 32; d >= 1; d >>= 1) m = fmaxf(m, __shfl_xor(m, d, 64));
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < PWB; ++q) m = fmaxf(m, wm[q]);
    part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = __float_as_uint(m);
  }
}

__global__ void k_add_max(const float* a, const float* b, float* out) { *out = *a + *b; }

}  // namespace

pm_status run_pp_accel(pm_context* c, const pm_species* sp, int n_sp, int64_t* const* offs,
                       double r_soft, float* const* app, float* pmax) {
  if (n_sp <= 0 || n_sp > PMAXSP) return PM_ERR_ARG;
  const Geom& g = c->g;
  PPArgs A{};
  A.n_sp = n_sp;
  const double delta = g.box / (double)g.ng;
  A.g_scale = (float)(c->cfg.G / (delta * delta));
  const int kind = common_width_kind(sp, n_sp);
  if (kind < 0) return PM_ERR_ARG;
  const int P = width_pos(sp[0]);
  const double rc = r_soft * g.SL * (P == 1 ? 1.0 : 256.0);  // r_soft in position codes
  A.cut2 = rc * rc;
  int64_t nmax = 0;
  for (int s = 0; s < n_sp; ++s) {
    A.sp[s].n = sp[s].n;
    A.sp[s].pos = sp[s].pos;
    A.sp[s].off = offs[s];
    A.sp[s].mass = (float)sp[s].mass;
    A.sp[s].app = app[s];
    nmax = sp[s].n > nmax ? sp[s].n : nmax;
  }
  (void)nmax;
  const int64_t nb = cdiv(g.nbrick, PWB);
  uint32_t* part = (uint32_t*)scratch(c, SC_PPMAX, (size_t)nb * n_sp * 4);
  if (!part) return PM_ERR_NOMEM;
  const size_t lds =
      (size_t)PWB * n_sp * (((size_t)1 << (3 * g.lgB)) + 1) * sizeof(int64_t) + (size_t)PWB * PCAP;
  {
    ProfScope ps(c, ST_PP);
    if (P == 1)
      hipLaunchKernelGGL(k_pp_accel<1>, dim3((unsigned)nb, (unsigned)n_sp), dim3(64 * PWB),
                         lds, c->stream, A, g, part);
    else
      hipLaunchKernelGGL(k_pp_accel<2>, dim3((unsigned)nb, (unsigned)n_sp), dim3(64 * PWB),
                         lds, c->stream, A, g, part);
    PM_LAUNCH_CHECK();
  }
  return fold_max_u32(c, part, nb * n_sp, (uint32_t*)pmax);
}

// a_max of the kick's velocity bound with the PP term: the mesh's max |a| plus the PP
// accelerations' max |a| (a bound on every component of their sum)
pm_status run_add_max(pm_context* c, const float* a, const float* b, float* out) {
  hipLaunchKernelGGL(k_add_max, dim3(1), dim3(1), 0, c->stream, a, b, out);
  PM_LAUNCH_CHECK();
  return PM_OK;
}

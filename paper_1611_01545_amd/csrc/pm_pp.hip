// The cell-local particle-particle (PP) force of eq. (4) (Sec. 2.1) on compressed
// streams: for every particle, the direct sum over the particles of all species that
// share its cell of the PM mesh,
//   a_i = G sum_{j != i, same mesh cell, r_ij >= r_soft} m_j (x_j - x_i) / r_ij^3,
// truncated below the softening length r_soft. The cell-sorted stream is the paper's
// linked list: a mesh cell lies inside one compression cell (r^3 mesh cells each), so a
// particle's partners are found among the particles of its compression cell, one
// contiguous range per species.
//
// One thread per particle, grid.y over species. Positions are the bin centres in mesh
// units, (u + 1/2) r / 256, exact in float32, so the mesh cell and every difference x_j - x_i
// are exact; the cut is decided on the integer code differences (|du|^2 >= (r_soft S / L)^2),
// the force is summed in float32 in stream order (deterministic). The arithmetic is plain
// vector ALU work: about 20 flops per interacting pair.
#include "pm_codec.h"

namespace {

constexpr int PT = 256;
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

__device__ inline int64_t pp_find_cell(const int64_t* off, int64_t ncell, int64_t j) {
  int64_t lo = 0, hi = ncell;  // largest c with off[c] <= j
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (off[mid] <= j) lo = mid; else hi = mid;
  }
  return lo;
}

// P: position bytes per axis (codes u = cell 256^P + offset; (2u + 1) r < 2^28)
template <int P>
__global__ __launch_bounds__(PT) void k_pp_accel(PPArgs A, Geom g, uint32_t* part) {
  using PC = typename PosCode<P>::T;
  using DT = typename std::conditional<P == 1, int, int64_t>::type;  // code differences
  constexpr int SH = 8 * P, FB = 8 * P + 1;
  const int s = blockIdx.y;
  const PPSpecies& S = A.sp[s];
  const PC* spos = (const PC*)S.pos;
  const int64_t i = (int64_t)blockIdx.x * PT + threadIdx.x;
  float m = 0.f;
  if (i < S.n) {
    const int64_t key = pp_find_cell(S.off, g.ncell3, i);
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
      const int64_t j0 = T.off[key], j1 = T.off[key + 1];
      float sx = 0.f, sy = 0.f, sz = 0.f;
      const PC* tpos = (const PC*)T.pos;
      for (int64_t j = j0; j < j1; ++j) {
        if (t == s && j == i) continue;
        const int uj0 = (int)((cx << SH) | tpos[3 * j]);
        const int uj1 = (int)((cy << SH) | tpos[3 * j + 1]);
        const int uj2 = (int)((cz << SH) | tpos[3 * j + 2]);
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
    m = fmaxf(fabsf(ax), fmaxf(fabsf(ay), fabsf(az)));
  }
  // per-block max |a| (non-negative float bits order as integers), folded afterwards
  __shared__ float wm[PT / 64];
  for (int d = 32; d >= 1; d >>= 1) m = fmaxf(m, __shfl_xor(m, d, 64));
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < PT / 64; ++q) m = fmaxf(m, wm[q]);
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
  const int64_t nb = cdiv(nmax > 0 ? nmax : 1, PT);
  uint32_t* part = (uint32_t*)scratch(c, SC_PPMAX, (size_t)nb * n_sp * 4);
  if (!part) return PM_ERR_NOMEM;
  {
    ProfScope ps(c, ST_PP);
    if (P == 1)
      hipLaunchKernelGGL(k_pp_accel<1>, dim3((unsigned)nb, (unsigned)n_sp), dim3(PT), 0,
                         c->stream, A, g, part);
    else
      hipLaunchKernelGGL(k_pp_accel<2>, dim3((unsigned)nb, (unsigned)n_sp), dim3(PT), 0,
                         c->stream, A, g, part);
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

// The two-level particle-mesh force of Sec. 2.1 on one device: the long-range force on
// a coarse mesh spanning the box (a context with the long-range kernel part), the
// short-range force on the fine mesh (a context with the short-range part), and the PP
// force of eq. (4) inside the fine mesh's cells, summed in the kick of the fine context.
//
// The paper solves the short-range part on per-tile meshes with a buffer of 24 fine
// cells so that each node works in its own memory. One device holds the whole box's fine
// mesh, which is then a single periodic tile: no buffer, no per-tile transforms (a batch
// of power-of-two tile meshes with such buffers would transform at least 8 times the
// fine mesh's cells).
//
// k_interp_bricks interpolates a context's force meshes to compressed particles (the
// inverse force interpolation of Sec. 2.3, Fig. 2): one wave per brick of the stream
// order, whose particles are one contiguous range (a brick of 4^3 cells holds 64 CDM or
// 512 neutrinos at the paper's 1:8 ratio, so a 256-thread workgroup per brick left
// three quarters of its threads idle on CDM bricks); lanes take consecutive particles
// (coalesced code loads and result stores) and find their cell among the brick's cell
// offsets staged in LDS. A particle's mesh coordinate per axis is
// (2 u + 1) r / 512 mesh cells (u its position code, r mesh cells per compression cell),
// an exact binary fraction, so the node index and the CIC weights (multiples of 1/512)
// are exact; the 8-node sum is float32 in a fixed order.
#include "pm_codec.h"

namespace {

constexpr int IWB = 4;  // bricks (waves) per workgroup
constexpr int ISN = 5;  // nodes per side of a brick staged in LDS, at most
constexpr int IMAXSP = 4;

struct ISpecies {
  int64_t n;
  const void* pos;     // position codes, P bytes per axis
  const int64_t* off;  // cell offsets [ncell3 + 1]
  float* out;          // [n][3], stream order
};

struct IArgs {
  ISpecies sp[IMAXSP];
  int n_sp;
  int accumulate;
};

template <int P>  // position bytes per axis
__global__ __launch_bounds__(64 * IWB) void k_interp_bricks(IArgs A, Geom g,
                                                           const float* __restrict__ acc) {
  using PC = typename PosCode<P>::T;
  constexpr int SH = 8 * P, FB = 8 * P + 1;
  constexpr uint32_t FMASK = (1u << FB) - 1u;
  constexpr float UNIT = 1.0f / (float)(1u << FB);
  const ISpecies& S = A.sp[blockIdx.y];
  if (S.n == 0) return;
  const PC* spos = (const PC*)S.pos;
  __shared__ int64_t so_all[IWB][8 * 8 * 8 + 1];  // each brick's cell offsets (B <= 8)
  // a brick spanning at most ISN - 1 mesh cells per side (the coarse mesh of the two-level
  // force: one mesh cell per compression cell) stages its (B r + 1)^3 nodes of the three
  // force meshes in LDS: 375 loads per brick instead of 24 per particle
  __shared__ float sn_all[IWB][3][ISN * ISN * ISN];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t b = (int64_t)blockIdx.x * IWB + wv;
  if (b >= g.nbrick) return;  // the whole wave
  int64_t* so = so_all[wv];
  const int B3 = 1 << (3 * g.lgB);
  const int64_t k0 = b * B3;  // first cell key of the brick
  for (int i = lane; i <= B3; i += 64) so[i] = S.off[k0 + i];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int64_t base = so[0];
  const int64_t np = so[B3] - base;  // the brick's particles
  const int64_t n = g.ng, n3 = n * n * n;
  const int nm = (int)n - 1;  // n is a power of two
  const float* ax = acc;
  const float* ay = acc + n3;
  const float* az = acc + 2 * n3;
  const int NB = g.B * g.r + 1;  // nodes per side of the brick's mesh region
  const bool staged = NB <= ISN;
  const uint32_t nbm = (1u << g.lgnb) - 1u;
  const int ox = (int)(((uint32_t)b & nbm) << g.lgB) * g.r;  // first node of the brick
  const int oy = (int)((((uint32_t)b >> g.lgnb) & nbm) << g.lgB) * g.r;
  const int oz = (int)(((uint32_t)b >> (2 * g.lgnb)) << g.lgB) * g.r;
  float(*sn)[ISN * ISN * ISN] = sn_all[wv];
  if (staged) {
    for (int i = lane; i < NB * NB * NB; i += 64) {
      const int lx = i % NB, ly = (i / NB) % NB, lz = i / (NB * NB);
      const int64_t qn = ((int64_t)((oz + lz) & nm) * n + ((oy + ly) & nm)) * n + ((ox + lx) & nm);
      sn[0][i] = ax[qn];
      sn[1][i] = ay[qn];
      sn[2][i] = az[qn];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  for (int64_t q = lane; q < np; q += 64) {
    const int64_t j = base + q;
    if (j >= S.n) break;  // offsets inconsistent with n: latched by the offset check
    // local cell: the largest l with so[l] <= j (skips empty cells)
    int lo = 0, hi = B3;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (so[mid] <= j) lo = mid; else hi = mid;
    }
    uint32_t cx, cy, cz;
    key_cell(g, (uint32_t)(k0 + lo), cx, cy, cz);
    // mesh coordinate (2u + 1) r / 2^FB per axis (2^FB = 512 for 1-byte codes): node =
    // t >> FB, weight of node + 1 = (t mod 2^FB) / 2^FB; (2u + 1) r < 2^28
    const int tx = (2 * (int)((cx << SH) | spos[3 * j]) + 1) * g.r;
    const int ty = (2 * (int)((cy << SH) | spos[3 * j + 1]) + 1) * g.r;
    const int tz = (2 * (int)((cz << SH) | spos[3 * j + 2]) + 1) * g.r;
    const int ix = (tx >> FB) & nm, iy = (ty >> FB) & nm, iz = (tz >> FB) & nm;
    const float fx = (float)((uint32_t)tx & FMASK) * UNIT;
    const float fy = (float)((uint32_t)ty & FMASK) * UNIT;
    const float fz = (float)((uint32_t)tz & FMASK) * UNIT;
    const float wx[2] = {1.0f - fx, fx}, wy[2] = {1.0f - fy, fy}, wz[2] = {1.0f - fz, fz};
    const int xs[2] = {ix, (ix + 1) & nm}, ys[2] = {iy, (iy + 1) & nm};
    const int zs[2] = {iz, (iz + 1) & nm};
    float sx = 0.f, sy = 0.f, sz = 0.f;
    if (staged) {
      // the particle's nodes relative to the brick's first node: 0 .. B r
      const int lx = (ix - ox) & nm, ly = (iy - oy) & nm, lz = (iz - oz) & nm;
#pragma unroll
      for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
          for (int dx = 0; dx < 2; ++dx) {
            const int i = ((lz + dz) * NB + (ly + dy)) * NB + (lx + dx);
            const float w = wz[dz] * wy[dy] * wx[dx];
            sx += w * sn[0][i];
            sy += w * sn[1][i];
            sz += w * sn[2][i];
          }
    } else {
#pragma unroll
      for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
          for (int dx = 0; dx < 2; ++dx) {
            const int64_t qn = ((int64_t)zs[dz] * n + ys[dy]) * n + xs[dx];
            const float w = wz[dz] * wy[dy] * wx[dx];
            sx += w * ax[qn];
            sy += w * ay[qn];
            sz += w * az[qn];
          }
    }
    float* o = S.out + 3 * j;
    if (A.accumulate) {
      sx += o[0];
      sy += o[1];
      sz += o[2];
    }
    o[0] = sx;
    o[1] = sy;
    o[2] = sz;
  }
}

}  // namespace

pm_status run_interp_accel(pm_context* c, const pm_species* sp, int n_sp,
                           int64_t* const* offs, const float* acc, float* const* out,
                           int accumulate) {
  if (n_sp <= 0 || n_sp > IMAXSP) return PM_ERR_ARG;
  const Geom& g = c->g;
  IArgs A{};
  A.n_sp = n_sp;
  A.accumulate = accumulate ? 1 : 0;
  for (int s = 0; s < n_sp; ++s) {
    A.sp[s].n = sp[s].n;
    A.sp[s].pos = sp[s].pos;
    A.sp[s].off = offs[s];
    A.sp[s].out = out[s];
  }
  const int kind = common_width_kind(sp, n_sp);
  if (kind < 0) return PM_ERR_ARG;
  ProfScope ps(c, ST_INTERP);
  if (width_pos(sp[0]) == 1)
    hipLaunchKernelGGL(k_interp_bricks<1>, dim3((unsigned)cdiv(g.nbrick, IWB), (unsigned)n_sp),
                       dim3(64 * IWB), 0, c->stream, A, g, acc);
  else
    hipLaunchKernelGGL(k_interp_bricks<2>, dim3((unsigned)cdiv(g.nbrick, IWB), (unsigned)n_sp),
                       dim3(64 * IWB), 0, c->stream, A, g, acc);
  PM_LAUNCH_CHECK();
  return PM_OK;
}

// A fine (short-range) and a coarse (long-range) context form a two-level pair when they
// split the same kernel at the same length and share the particle format and units.
bool split_pair_ok(const pm_context* f, const pm_context* c) {
  const pm_config &a = f->cfg, &b = c->cfg;
  if (a.kernel != PM_KERNEL_SHORT || b.kernel != PM_KERNEL_LONG) return false;
  if (f->stream != c->stream || f->device != c->device) return false;
  if (a.n_cell != b.n_cell || a.brick != b.brick || a.box != b.box || a.G != b.G) return false;
  if (a.r_split != b.r_split || b.n_mesh > a.n_mesh) return false;
  // the same softening length on both meshes
  const double ea = a.soft_cells / (double)a.n_mesh, eb = b.soft_cells / (double)b.n_mesh;
  return fabs(ea - eb) <= 1e-12 * fmax(ea, eb);
}

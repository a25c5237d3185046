// Adjoint (vector-Jacobian product) of the particle-mesh step and of a density loss.
//
// The paper's code runs the forward step only; the adjoint here makes the step usable
// inside gradient-based fitting. For the step v' = v + c_k a(x), x' = x + c_d v' with
// a = K rho (the force operator of eqs. (1)-(3) applied to the CIC density), given the
// cotangents lx' = dL/dx' and lv' = dL/dv':
//   g_v = lv' + c_d lx'            -> dL/dv
//   g_a = c_k g_v
//   mu_a(c) = sum_j W(x_j - x_c) g_a,ja            (transpose of the interpolation)
//   nu = sum_a K_a^T mu_a = sum_a IDFT(+i k_a G DFT(mu_a))
//   dL/dx_i = lx'_i + sum_c grad W(x_i - x_c) [ g_a,i . a(c) + m_i n^3 nu(c) ]
// The two terms of the last line are the direct dependence of the interpolated force on
// the particle position and the dependence through the density it deposits; CIC is
// node-centred, so grad W has the one-sided derivative +-n per axis that floor gives.
//
// Compressed states are differentiated straight-through at the decoded bin centres;
// the forward re-sort is recomputed to map the new stream order of the cotangents back
// to the old order. The tiled scatter of compressed states sums fixed-point integers
// (the result does not depend on the order of the atomics); the per-particle scatter of
// the other shapes sums with float atomics (summation order not fixed).
#include "pm_codec.h"
#include "pm_scan.h"

int deposit_tile_cells(const Geom& g);

namespace {

constexpr int AT = 256;

struct Cic {
  int64_t i[3];  // lower node per axis (periodic)
  float f[3];    // fractional offset per axis
};

__device__ __forceinline__ Cic cic_of(const float* x, int64_t ng, float ngL) {
  Cic r;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float u = x[a] * ngL;  // mesh units (exact for a power-of-two box)
    float fl = floorf(u);
    r.f[a] = u - fl;
    int64_t k = (int64_t)fl % ng;
    r.i[a] = k < 0 ? k + ng : k;
  }
  return r;
}

__device__ __forceinline__ int64_t cic_node(const Cic& q, int dx, int dy, int dz, int64_t ng) {
  return (((q.i[2] + dz) % ng) * ng + (q.i[1] + dy) % ng) * ng + (q.i[0] + dx) % ng;
}

// g_v = lv1 + c_d lx1 into lv0 (old order), lx0 = lx1 (old order). perm: new -> old.
// One thread per component, so that the loads are contiguous across the wave.
__global__ __launch_bounds__(AT) void k_vjp_init(const float* lx1, const float* lv1,
                                                 const int64_t* perm, int64_t n, float cd,
                                                 float* lx0, float* lv0) {
  const int64_t i = (int64_t)blockIdx.x * AT + threadIdx.x;
  if (i >= 3 * n) return;
  const int64_t j = i / 3;
  const int64_t o = perm ? perm[j] : j;
  const int64_t d = 3 * o + (i - 3 * j);
  const float lx = lx1[i];
  lv0[d] = lv1[i] + cd * lx;
  lx0[d] = lx;
}

// mu_a(c) += W(x_j - x_c) c_k g_v,ja for the three components.
__global__ __launch_bounds__(AT) void k_scatter_vec(const float* x, const float* gv, int64_t n,
                                                    int64_t ng, float ngL, float ck, float* mu) {
  const int64_t p = (int64_t)blockIdx.x * AT + threadIdx.x;
  if (p >= n) return;
  const int64_t n3 = ng * ng * ng;
  const Cic q = cic_of(x + 3 * p, ng, ngL);
  const float g0 = ck * gv[3 * p], g1 = ck * gv[3 * p + 1], g2 = ck * gv[3 * p + 2];
#pragma unroll
  for (int dz = 0; dz < 2; ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) {
        const float w = (dx ? q.f[0] : 1.f - q.f[0]) * (dy ? q.f[1] : 1.f - q.f[1]) *
                        (dz ? q.f[2] : 1.f - q.f[2]);
        const int64_t node = cic_node(q, dx, dy, dz, ng);
        unsafeAtomicAdd(&mu[node], w * g0);
        unsafeAtomicAdd(&mu[n3 + node], w * g1);
        unsafeAtomicAdd(&mu[2 * n3 + node], w * g2);
      }
}

// out_i (+)= sum_c grad W(x_i - x_c) q(c) with
//   q(c) = s_scale s(c) + c_k g_v,i . a(c)      (the second term only if acc is given).
__global__ __launch_bounds__(AT) void k_gather_grad(const float* x, int64_t n, int64_t ng,
                                                    float ngL, const float* s, float s_scale,
                                                    const float* acc, const float* gv,
                                                    float ck, float* out, int accumulate) {
  const int64_t p = (int64_t)blockIdx.x * AT + threadIdx.x;
  if (p >= n) return;
  const int64_t n3 = ng * ng * ng;
  const Cic q = cic_of(x + 3 * p, ng, ngL);
  float g0 = 0.f, g1 = 0.f, g2 = 0.f;
  if (acc) {
    g0 = ck * gv[3 * p];
    g1 = ck * gv[3 * p + 1];
    g2 = ck * gv[3 * p + 2];
  }
  const float fn = ngL;  // d W / d x per axis is +-n / L
  float gr[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int dz = 0; dz < 2; ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) {
        const int64_t node = cic_node(q, dx, dy, dz, ng);
        float val = s_scale * s[node];
        if (acc) val += g0 * acc[node] + g1 * acc[n3 + node] + g2 * acc[2 * n3 + node];
        const float wx = dx ? q.f[0] : 1.f - q.f[0];
        const float wy = dy ? q.f[1] : 1.f - q.f[1];
        const float wz = dz ? q.f[2] : 1.f - q.f[2];
        gr[0] += (dx ? fn : -fn) * wy * wz * val;
        gr[1] += (dy ? fn : -fn) * wx * wz * val;
        gr[2] += (dz ? fn : -fn) * wx * wy * val;
      }
#pragma unroll
  for (int a = 0; a < 3; ++a) out[3 * p + a] = (accumulate ? out[3 * p + a] : 0.f) + gr[a];
}

// r = rho - rho_t in place of rho; per-block partial sums of r^2 in double.
__global__ __launch_bounds__(AT) void k_residual(float* rho, const float* rho_t, int64_t n3,
                                                 double* part) {
  __shared__ double sh[AT];
  const int64_t i0 = (int64_t)blockIdx.x * AT * 4 + threadIdx.x;
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = i0 + (int64_t)k * AT;
    if (i < n3) {
      const float r = rho[i] - rho_t[i];
      rho[i] = r;
      acc += (double)r * (double)r;
    }
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = AT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Fixed-order sum of the partials (one workgroup).
__global__ __launch_bounds__(AT) void k_fold_double(const double* part, int64_t m, double* out) {
  __shared__ double sh[AT];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += AT) acc += part[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = AT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

__global__ void k_zero_f32(float* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * AT + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

// ------------------------------------------------ compressed layout, tiled --
// The scatter mu_a(c) = c_k sum_j W(x_j - x_c) g_v,ja and the gradient gather read the
// particles' compressed codes directly (cell-sorted streams), like the deposit and the
// kick: exact CIC weights from the codes, no decoded positions in HBM.
constexpr int MAXSP = 4;
constexpr int ST = 512;  // scatter threads per workgroup

struct AdjSpecies {
  int64_t n;
  const uint8_t* pos;
  const int64_t* off;  // cell offsets [ncell3 + 1]
  const float* gv;     // g_v = dL/dv per particle, stream order
  float* lx;           // dL/dx per particle, stream order (gather adds to it)
  float sscale;        // m / Delta^3 (density per unit weight)
};
struct AdjArgs {
  AdjSpecies sp[MAXSP];
  int n_sp;
  float ck;
};

__device__ inline int wrapc(int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); }

// One workgroup per tile of TT^3 cells = 16^3 mesh nodes (r = 16 / TT). Particles of the
// one-cell shell on the -x/-y/-z faces reach the tile's lowest node plane and are
// included, as in the deposit. Each species' contributions w g are summed in LDS as
// 32-bit fixed-point integers (integer LDS atomics are several times faster than float
// ones, and integer sums do not depend on the order of the atomics): the unit 2^-q is
// chosen per tile and species from the largest |g| and the particle count so that no
// sum can overflow. Each species is then converted into per-thread float sums of the
// thread's nodes, in species order, and the tile is written with plain stores: every
// node has one owner. A species whose cotangents in the tile are not all finite is
// summed with float atomics instead, so that inf and NaN propagate.
template <int TT>
__global__ __launch_bounds__(ST) void k_scatter_tile(AdjArgs A, Geom g, float* mu) {
  constexpr int T = TT, R = 16, r = 16 / TT, E = T + 1, NE = E * E * E, R3 = R * R * R;
  constexpr int NW = ST / 64, NPT = R3 / ST;
  __shared__ int F[3 * R3];  // one species' sums (fixed point, or float bits)
  __shared__ int64_t cst[NE];
  __shared__ int pre[NE + 1];
  __shared__ int wsum[NW];
  __shared__ float wgm[NW];
  __shared__ int wnf[NW];
  const int nt = (int)(g.nc / T);
  const int64_t tile = xcd_tile(blockIdx.x, (int64_t)nt * nt * nt);
  const int tx = (int)(tile % nt), ty = (int)((tile / nt) % nt),
            tz = (int)(tile / ((int64_t)nt * nt));
  const int ncs = (int)g.nc;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < 3 * R3; i += ST) F[i] = 0;
  float racc[3][NPT];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int k = 0; k < NPT; ++k) racc[c][k] = 0.f;
  for (int s = 0; s < A.n_sp; ++s) {
    const AdjSpecies sp = A.sp[s];
    __syncthreads();
    for (int e = threadIdx.x; e < NE; e += ST) {
      const int ex = e % E, ey = (e / E) % E, ez = e / (E * E);
      const int cx = wrapc(tx * T + ex - 1, ncs), cy = wrapc(ty * T + ey - 1, ncs),
                cz = wrapc(tz * T + ez - 1, ncs);
      const uint32_t key = cell_key(g, cx, cy, cz);
      const int64_t o0 = sp.off[key], o1 = sp.off[key + 1];
      cst[e] = o0;
      pre[e + 1] = (int)(o1 - o0);
    }
    __syncthreads();
    {
      constexpr int K = (NE + ST - 1) / ST;
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
    constexpr int U = 4;
    // the largest |g| of the species' particles in the tile: from the first batch's
    // registers when one batch holds them all, otherwise from a pass of its own (one
    // wave per extended cell)
    const bool one = P <= ST * U;
    float gm = 0.f;
    int nf = 0;
    if (!one)
      for (int e = w; e < NE; e += NW)
        for (int q = lane; q < pre[e + 1] - pre[e]; q += 64) {
          const int64_t j = cst[e] + q;
          if (j < sp.n)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              const float v = fabsf(sp.gv[3 * j + a]);
              nf |= !(v <= 3.4028234e38f);  // inf or NaN
              gm = fmaxf(gm, v);
            }
        }
    int eu[U];
    bool ok[U];
    uint32_t pb[U][3];
    float gg[U][3];
    auto load_batch = [&](int q0) {
      int64_t ju[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = q0 + u * ST;
        int lo = 0, hi = NE;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (pre[mid] <= q) lo = mid; else hi = mid;
        }
        eu[u] = lo;
        const int64_t j = cst[lo] + (q - pre[lo]);
        ok[u] = q < P && j < sp.n;
        ju[u] = ok[u] ? j : 0;  // n > 0 whenever P > 0
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          pb[u][a] = sp.pos[3 * ju[u] + a];
          gg[u][a] = sp.gv[3 * ju[u] + a];
        }
    };
    load_batch(threadIdx.x);
    if (one)
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const float v = ok[u] ? fabsf(gg[u][a]) : 0.f;
          nf |= !(v <= 3.4028234e38f);
          gm = fmaxf(gm, v);
        }
    for (int d = 32; d >= 1; d >>= 1) {
      gm = fmaxf(gm, __shfl_xor(gm, d, 64));
      nf |= __shfl_xor(nf, d, 64);
    }
    if (lane == 0) {
      wgm[w] = gm;
      wnf[w] = nf;
    }
    __syncthreads();
    for (int q = 0; q < NW; ++q) {
      gm = fmaxf(gm, wgm[q]);
      nf |= wnf[q];
    }
    // unit 2^-qs: P gm 2^qs < 2^30, so a node's sum of at most P rounded contributions
    // stays below 2^30 + P / 2 < 2^31
    const bool fixed = !nf;
    const float t = (float)P * gm;
    const int qs = t > 0.f ? 29 - ilogbf(t) : 0;
    for (int q0 = threadIdx.x; q0 < P; q0 += ST * U) {
      if (q0 != (int)threadIdx.x) load_batch(q0);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (!ok[u]) continue;
        const int e = eu[u];
        const int le[3] = {e % E - 1, (e / E) % E - 1, e / (E * E) - 1};
        int li[3], f[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int gl = (2 * (int)pb[u][a] + 1) * r;  // 1/512 mesh cells
          li[a] = le[a] * r + (gl >> 9);
          f[a] = gl & 511;
        }
#pragma unroll
        for (int dz = 0; dz < 2; ++dz) {
          const int nz = li[2] + dz, wz = dz ? f[2] : 512 - f[2];
          if (nz < 0 || nz >= R || wz == 0) continue;
#pragma unroll
          for (int dy = 0; dy < 2; ++dy) {
            const int ny = li[1] + dy, wy = dy ? f[1] : 512 - f[1];
            if (ny < 0 || ny >= R || wy == 0) continue;
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
              const int nx = li[0] + dx, wx = dx ? f[0] : 512 - f[0];
              if (nx < 0 || nx >= R || wx == 0) continue;
              const float wt = (float)((uint32_t)(wx * wy) * (uint32_t)wz) * 0x1p-27f;
              const int node = (nz * R + ny) * R + nx;
#pragma unroll
              for (int a = 0; a < 3; ++a) {
                const float cv = wt * gg[u][a];
                if (fixed)
                  atomicAdd(&F[a * R3 + node], __float2int_rn(ldexpf(cv, qs)));
                else
                  atomicAdd((float*)&F[a * R3 + node], cv);
              }
            }
          }
        }
      }
    }
    // this species' sums into the thread's float node sums, then cleared
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int k = 0; k < NPT; ++k) {
        const int i = c * R3 + threadIdx.x + k * ST;
        const int v = F[i];
        racc[c][k] += fixed ? ldexpf((float)v, -qs) : __int_as_float(v);
        F[i] = 0;
      }
  }
  // node i = threadIdx.x + ST k: lx = i & 15, ly = (i >> 4) & 15, lz = i >> 8
  const int64_t ng = g.ng, ng2 = ng * ng, n3 = ng2 * ng;
  float* dst = mu + ((int64_t)tz * 16 + (threadIdx.x >> 8)) * ng2 +
               ((int64_t)ty * 16 + ((threadIdx.x >> 4) & 15)) * ng + (int64_t)tx * 16 +
               (threadIdx.x & 15);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int k = 0; k < NPT; ++k) dst[c * n3 + k * (ST / 256) * ng2] = A.ck * racc[c][k];
}

// Gradient gather on bricks of B^3 cells = 16^3 nodes: the four meshes a_x, a_y, a_z
// and nu are staged for the nodes [0, 16]^3 of the brick, then for every particle of the
// brick's cells lx += sum_c grad W(x - x_c) [c_k g_v . a(c) + m n^3 nu(c)].
constexpr int GT = 512;  // gather threads per workgroup
constexpr int GR = 16, GR1 = GR + 1;

__global__ __launch_bounds__(GT) void k_gather_brick(AdjArgs A, Geom g, const float* acc,
                                                     const float* nu) {
  constexpr int FS = GR1 * GR1 * GR1;
  __shared__ float Fm[4 * FS];  // a_x, a_y, a_z, nu on the brick's nodes
  extern __shared__ int64_t loff[];  // [B^3 + 1]: sized at launch, so that two
                                     // workgroups fit one CU's LDS at B = 4
  const int B = g.B, B3 = B * B * B, r = g.r;
  const int64_t b = xcd_tile(blockIdx.x, g.nbrick);
  const uint32_t kbase = (uint32_t)(b * B3);
  const int64_t ng = g.ng, n3 = ng * ng * ng;
  uint32_t bcx, bcy, bcz;
  key_cell(g, kbase, bcx, bcy, bcz);
  const int64_t ox = (int64_t)bcx * r, oy = (int64_t)bcy * r, oz = (int64_t)bcz * r;
  {
    // rows of 16 nodes as float4 loads plus the x = 16 halo column; all loads of a
    // thread are issued before its LDS writes
    constexpr int ROWS = 4 * GR1 * GR1, NQ = ROWS * 4;
    constexpr int PQ = (NQ + GT - 1) / GT, PH = (ROWS + GT - 1) / GT;
    const bool wrapx = ox + GR >= ng;
    float4 vq[PQ];
    float vh[PH];
#pragma unroll
    for (int k = 0; k < PQ; ++k) {
      const int i = min((int)threadIdx.x + k * GT, NQ - 1);
      const int row = i >> 2, q = i & 3;
      const int c = row / (GR1 * GR1), rem = row - c * (GR1 * GR1);
      const int lz = rem / GR1, ly = rem - lz * GR1;
      int64_t gz = oz + lz, gy = oy + ly;
      gz -= gz >= ng ? ng : 0;
      gy -= gy >= ng ? ng : 0;
      const float* src = c < 3 ? acc + (int64_t)c * n3 : nu;
      vq[k] = *(const float4*)(src + (gz * ng + gy) * ng + ox + 4 * q);
    }
#pragma unroll
    for (int k = 0; k < PH; ++k) {
      const int row = min((int)threadIdx.x + k * GT, ROWS - 1);
      const int c = row / (GR1 * GR1), rem = row - c * (GR1 * GR1);
      const int lz = rem / GR1, ly = rem - lz * GR1;
      int64_t gz = oz + lz, gy = oy + ly;
      gz -= gz >= ng ? ng : 0;
      gy -= gy >= ng ? ng : 0;
      const float* src = c < 3 ? acc + (int64_t)c * n3 : nu;
      vh[k] = src[(gz * ng + gy) * ng + (wrapx ? 0 : ox + GR)];
    }
#pragma unroll
    for (int k = 0; k < PQ; ++k) {
      const int i = threadIdx.x + k * GT;
      if (i < NQ) {
        float* d = Fm + (i >> 2) * GR1 + 4 * (i & 3);
        d[0] = vq[k].x;
        d[1] = vq[k].y;
        d[2] = vq[k].z;
        d[3] = vq[k].w;
      }
    }
#pragma unroll
    for (int k = 0; k < PH; ++k) {
      const int row = threadIdx.x + k * GT;
      if (row < ROWS) Fm[row * GR1 + GR] = vh[k];
    }
  }
  const float fn = g.ngL;  // d W / d x per axis is +-n / L
  for (int s = 0; s < A.n_sp; ++s) {
    const AdjSpecies sp = A.sp[s];
    __syncthreads();  // staged meshes ready / previous species done with loff
    for (int i = threadIdx.x; i <= B3; i += GT) loff[i] = sp.off[kbase + i];
    __syncthreads();
    const int64_t j0 = min(loff[0], sp.n), j1 = min(loff[B3], sp.n);
    for (int64_t j = j0 + threadIdx.x; j < j1; j += GT) {
      uint32_t pb[3];
      float gvv[3], lxx[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        pb[a] = sp.pos[3 * j + a];
        gvv[a] = sp.gv[3 * j + a];
        lxx[a] = sp.lx[3 * j + a];
      }
      int lo = 0, hi = B3;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (loff[mid] <= j) lo = mid; else hi = mid;
      }
      uint32_t cx, cy, cz;
      key_cell(g, kbase + (uint32_t)lo, cx, cy, cz);
      const uint32_t cell[3] = {cx, cy, cz};
      const int64_t org[3] = {ox, oy, oz};
      int li[3];
      float f[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int64_t gg = (2 * (int64_t)((cell[a] << 8) | pb[a]) + 1) * r;  // 1/512 cells
        li[a] = (int)((gg >> 9) - org[a]);
        f[a] = (float)(gg & 511) * (1.0f / 512.0f);
      }
      const float g0 = A.ck * gvv[0], g1 = A.ck * gvv[1], g2 = A.ck * gvv[2];
      float gr[3] = {0.f, 0.f, 0.f};
#pragma unroll
      for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
          for (int dx = 0; dx < 2; ++dx) {
            const int node = ((li[2] + dz) * GR1 + (li[1] + dy)) * GR1 + (li[0] + dx);
            const float val = g0 * Fm[node] + g1 * Fm[FS + node] + g2 * Fm[2 * FS + node] +
                              sp.sscale * Fm[3 * FS + node];
            const float wx = dx ? f[0] : 1.f - f[0];
            const float wy = dy ? f[1] : 1.f - f[1];
            const float wz = dz ? f[2] : 1.f - f[2];
            gr[0] += (dx ? fn : -fn) * wy * wz * val;
            gr[1] += (dy ? fn : -fn) * wx * wz * val;
            gr[2] += (dz ? fn : -fn) * wx * wy * val;
          }
#pragma unroll
      for (int a = 0; a < 3; ++a) sp.lx[3 * j + a] = lxx[a] + gr[a];
    }
  }
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Float positions of every species (decoded bin centres for compressed states) and,
// for compressed states, the cell offsets. `pool` receives the decoded arrays.
struct Positions {
  const float* x[4];
  int64_t* offs[4];
};

pm_status positions(pm_context* c, const pm_species* sp, int n_sp, int scratch_id,
                    Positions& P, bool decode = true) {
  pm_status s;
  for (int i = 0; i < n_sp; ++i) {
    P.x[i] = sp[i].x;
    P.offs[i] = nullptr;
  }
  if (sp[0].layout != PM_COMPRESSED) return PM_OK;
  if (!decode) {
    for (int i = 0; i < n_sp; ++i) {
      P.x[i] = nullptr;
      P.offs[i] = (int64_t*)scratch(c, SC_SPOFF0 + i, (size_t)(c->g.ncell3 + 1) * 8);
      if (!P.offs[i]) return PM_ERR_NOMEM;
      if ((s = run_cell_offsets(c, &sp[i], P.offs[i])) != PM_OK) return s;
    }
    return PM_OK;
  }
  size_t bytes = 0;
  for (int i = 0; i < n_sp; ++i) bytes += 2 * align256((size_t)sp[i].n * 12);
  char* pool = (char*)scratch(c, scratch_id, bytes);
  if (!pool) return PM_ERR_NOMEM;
  size_t at = 0;
  for (int i = 0; i < n_sp; ++i) {
    pm_species dec = {};
    dec.layout = PM_FLOAT;
    dec.n = sp[i].n;
    dec.mass = sp[i].mass;
    dec.x = (float*)(pool + at);
    at += align256((size_t)sp[i].n * 12);
    dec.v = (float*)(pool + at);
    at += align256((size_t)sp[i].n * 12);
    if ((s = run_decode(c, &sp[i], &dec)) != PM_OK) return s;
    P.x[i] = dec.x;
    P.offs[i] = (int64_t*)scratch(c, SC_SPOFF0 + i, (size_t)(c->g.ncell3 + 1) * 8);
    if (!P.offs[i]) return PM_ERR_NOMEM;
    if ((s = run_cell_offsets(c, &sp[i], P.offs[i])) != PM_OK) return s;
  }
  return PM_OK;
}

pm_status deposit_all(pm_context* c, const pm_species* sp, int n_sp, const Positions& P,
                      float* rho) {
  if (sp[0].layout == PM_COMPRESSED) return run_deposit_tile(c, sp, n_sp, P.offs, rho);
  return run_deposit(c, sp, n_sp, rho);
}

}  // namespace

pm_status run_step_vjp(pm_context* c, const pm_species* in, int n_sp, double dt,
                       float* const* lx1, float* const* lv1, float* const* lx0,
                       float* const* lv0) {
  const int64_t ng = c->g.ng, n3 = ng * ng * ng;
  const float ck = (float)dt, cd = (float)dt;
  pm_status s;
  // compressed states with 16-node tiles and bricks use the tiled scatter and gather on
  // the codes; other shapes and float states decode and use the per-particle kernels
  const Geom& g = c->g;
  const bool comp = in[0].layout == PM_COMPRESSED;
  const int tt = comp ? deposit_tile_cells(g) : 0;
  // (the tiled kernels read the paper's 1-byte position codes; other code widths decode)
  const bool tiled = comp && tt * g.r == 16 && (tt == 4 || tt == 8) && g.B * g.r == 16 &&
                     common_width_kind(in, n_sp) == 0;
  Positions P;
  if ((s = positions(c, in, n_sp, SC_VJP2, P, !tiled)) != PM_OK) return s;
  // forward recomputation: density, acceleration mesh (in the context mesh)
  float* acc = c->mesh;
  if ((s = deposit_all(c, in, n_sp, P, acc)) != PM_OK) return s;
  if ((s = run_force(c, acc, acc, c->nyq, c->amax)) != PM_OK) return s;
  // the re-sort of compressed streams: new stream position -> old
  int64_t* perm[4] = {nullptr, nullptr, nullptr, nullptr};
  if (in[0].layout == PM_COMPRESSED) {
    const int64_t nc3 = c->g.ncell3;
    size_t bytes = 0;
    for (int i = 0; i < n_sp; ++i) {
      const int64_t cap = in[i].n / 255 + 1;
      bytes += align256((size_t)in[i].n * 8) + align256((size_t)nc3) +
               align256((size_t)in[i].n * 3 * width_pos(in[i])) +
               align256((size_t)in[i].n * 3 * width_vel(in[i])) +
               align256((size_t)cap * 16) + align256(sizeof(pm_shdr));
    }
    char* pool = (char*)scratch(c, SC_VJP3, bytes);
    if (!pool) return PM_ERR_NOMEM;
    pm_species out[4];
    size_t at = 0;
    for (int i = 0; i < n_sp; ++i) {
      const int64_t n = in[i].n, cap = n / 255 + 1;
      out[i] = in[i];
      perm[i] = (int64_t*)(pool + at);
      at += align256((size_t)n * 8);
      out[i].count = (uint8_t*)(pool + at);
      at += align256((size_t)nc3);
      out[i].pos = (uint8_t*)(pool + at);
      at += align256((size_t)n * 3 * width_pos(in[i]));
      out[i].vel = (uint16_t*)(pool + at);
      at += align256((size_t)n * 3 * width_vel(in[i]));
      out[i].esc = (uint64_t*)(pool + at);
      out[i].cap_esc = cap;
      at += align256((size_t)cap * 16);
      out[i].hdr = (pm_shdr*)(pool + at);
      at += align256(sizeof(pm_shdr));
    }
    if ((s = run_kick_compressed_all(c, in, out, n_sp, P.offs, acc, c->amax, dt, dt, perm)) !=
        PM_OK)
      return s;
  }
  // cotangents into old order; g_v lands in lv0
  float* mu = (float*)scratch(c, SC_VJP, (size_t)3 * n3 * sizeof(float));
  if (!mu) return PM_ERR_NOMEM;
  AdjArgs T{};
  T.ck = ck;
  for (int i = 0; i < n_sp; ++i) {
    if (in[i].n == 0) continue;
    AdjSpecies& a = T.sp[T.n_sp++];
    a.n = in[i].n;
    a.pos = in[i].pos;
    a.off = P.offs[i];
    a.gv = lv0[i];
    a.lx = lx0[i];
    a.sscale = (float)(in[i].mass * (double)n3 / (c->g.box * c->g.box * c->g.box));
  }
  {
    ProfScope ps(c, ST_ADJOINT);
    if (!tiled)
      hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)cdiv(3 * n3, AT)), dim3(AT), 0,
                         c->stream, mu, 3 * n3);
    for (int i = 0; i < n_sp; ++i) {
      if (in[i].n == 0) continue;
      const unsigned nb = (unsigned)cdiv(in[i].n, AT);
      hipLaunchKernelGGL(k_vjp_init, dim3((unsigned)cdiv(3 * in[i].n, AT)), dim3(AT), 0,
                         c->stream, lx1[i], lv1[i], perm[i], in[i].n, cd, lx0[i], lv0[i]);
      if (!tiled)
        hipLaunchKernelGGL(k_scatter_vec, dim3(nb), dim3(AT), 0, c->stream, P.x[i], lv0[i],
                           in[i].n, ng, c->g.ngL, ck, mu);
    }
    if (tiled && T.n_sp > 0) {
      const int64_t nt = g.nc / tt;
      const dim3 grid((unsigned)(nt * nt * nt));
      if (tt == 4)
        hipLaunchKernelGGL(k_scatter_tile<4>, grid, dim3(ST), 0, c->stream, T, g, mu);
      else
        hipLaunchKernelGGL(k_scatter_tile<8>, grid, dim3(ST), 0, c->stream, T, g, mu);
    } else if (tiled) {
      hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)cdiv(3 * n3, AT)), dim3(AT), 0,
                         c->stream, mu, 3 * n3);
    }
    PM_LAUNCH_CHECK();
  }
  {
    ProfScope ps(c, ST_ADJOINT);
    if ((s = run_force_transpose(c, mu, c->nyq)) != PM_OK) return s;
  }
  {
    ProfScope ps(c, ST_ADJOINT);
    if (tiled) {
      if (T.n_sp > 0)
        hipLaunchKernelGGL(k_gather_brick, dim3((unsigned)g.nbrick), dim3(GT),
                           (size_t)(g.B * g.B * g.B + 1) * 8, c->stream, T, g, acc, mu);
    } else {
      for (int i = 0; i < n_sp; ++i) {
        if (in[i].n == 0) continue;
        const float sscale = (float)(in[i].mass * (double)n3 / (c->g.box * c->g.box * c->g.box));
        hipLaunchKernelGGL(k_gather_grad, dim3((unsigned)cdiv(in[i].n, AT)), dim3(AT), 0,
                           c->stream, P.x[i], in[i].n, ng, c->g.ngL, mu, sscale, acc, lv0[i], ck,
                           lx0[i], 1);
      }
    }
    PM_LAUNCH_CHECK();
  }
  return PM_OK;
}

pm_status run_loss_vjp(pm_context* c, const pm_species* sp, int n_sp, const float* rho_t,
                       double* loss, float* const* lam_x) {
  const int64_t ng = c->g.ng, n3 = ng * ng * ng;
  pm_status s;
  Positions P;
  if ((s = positions(c, sp, n_sp, SC_VJP2, P)) != PM_OK) return s;
  float* r = c->mesh;
  if ((s = deposit_all(c, sp, n_sp, P, r)) != PM_OK) return s;
  ProfScope ps(c, ST_ADJOINT);
  const int64_t nb = cdiv(n3, 4 * AT);
  double* part = (double*)scratch(c, SC_PARTS, (size_t)nb * sizeof(double));
  if (!part) return PM_ERR_NOMEM;
  hipLaunchKernelGGL(k_residual, dim3((unsigned)nb), dim3(AT), 0, c->stream, r, rho_t, n3,
                     part);
  if (loss)
    hipLaunchKernelGGL(k_fold_double, dim3(1), dim3(AT), 0, c->stream, part, nb, loss);
  for (int i = 0; i < n_sp; ++i) {
    if (sp[i].n == 0) continue;
    const float sscale = (float)(2.0 * sp[i].mass * (double)n3 / (c->g.box * c->g.box * c->g.box));
    hipLaunchKernelGGL(k_gather_grad, dim3((unsigned)cdiv(sp[i].n, AT)), dim3(AT), 0,
                       c->stream, P.x[i], sp[i].n, ng, c->g.ngL, r, sscale, nullptr, nullptr, 0.f,
                       lam_x[i], 0);
  }
  PM_LAUNCH_CHECK();
  return PM_OK;
}

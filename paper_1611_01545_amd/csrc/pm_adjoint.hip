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
// to the old order. The scatter uses float atomics (summation order not fixed).
#include "pm_codec.h"

pm_status run_kick_compressed_all(pm_context* c, const pm_species* in, pm_species* out,
                                  int n_sp, int64_t* const* offs, const float* acc,
                                  const float* amax, double ck, double cd,
                                  int64_t* const* perm);

namespace {

constexpr int AT = 256;

struct Cic {
  int64_t i[3];  // lower node per axis (periodic)
  float f[3];    // fractional offset per axis
};

__device__ __forceinline__ Cic cic_of(const float* x, int64_t ng) {
  Cic r;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float u = x[a] * (float)ng;  // exact: ng is a power of two
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
__global__ __launch_bounds__(AT) void k_vjp_init(const float* lx1, const float* lv1,
                                                 const int64_t* perm, int64_t n, float cd,
                                                 float* lx0, float* lv0) {
  const int64_t j = (int64_t)blockIdx.x * AT + threadIdx.x;
  if (j >= n) return;
  const int64_t o = perm ? perm[j] : j;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float lx = lx1[3 * j + a];
    lv0[3 * o + a] = lv1[3 * j + a] + cd * lx;
    lx0[3 * o + a] = lx;
  }
}

// mu_a(c) += W(x_j - x_c) c_k g_v,ja for the three components.
__global__ __launch_bounds__(AT) void k_scatter_vec(const float* x, const float* gv, int64_t n,
                                                    int64_t ng, float ck, float* mu) {
  const int64_t p = (int64_t)blockIdx.x * AT + threadIdx.x;
  if (p >= n) return;
  const int64_t n3 = ng * ng * ng;
  const Cic q = cic_of(x + 3 * p, ng);
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
                                                    const float* s, float s_scale,
                                                    const float* acc, const float* gv,
                                                    float ck, float* out, int accumulate) {
  const int64_t p = (int64_t)blockIdx.x * AT + threadIdx.x;
  if (p >= n) return;
  const int64_t n3 = ng * ng * ng;
  const Cic q = cic_of(x + 3 * p, ng);
  float g0 = 0.f, g1 = 0.f, g2 = 0.f;
  if (acc) {
    g0 = ck * gv[3 * p];
    g1 = ck * gv[3 * p + 1];
    g2 = ck * gv[3 * p + 2];
  }
  const float fn = (float)ng;
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

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Float positions of every species (decoded bin centres for compressed states) and,
// for compressed states, the cell offsets. `pool` receives the decoded arrays.
struct Positions {
  const float* x[4];
  int64_t* offs[4];
};

pm_status positions(pm_context* c, const pm_species* sp, int n_sp, int scratch_id,
                    Positions& P) {
  pm_status s;
  for (int i = 0; i < n_sp; ++i) {
    P.x[i] = sp[i].x;
    P.offs[i] = nullptr;
  }
  if (sp[0].layout != PM_COMPRESSED) return PM_OK;
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
  Positions P;
  if ((s = positions(c, in, n_sp, SC_VJP2, P)) != PM_OK) return s;
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
               align256((size_t)in[i].n * 3) + align256((size_t)in[i].n * 6) +
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
      at += align256((size_t)n * 3);
      out[i].vel = (uint16_t*)(pool + at);
      at += align256((size_t)n * 6);
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
  {
    ProfScope ps(c, ST_ADJOINT);
    hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)cdiv(3 * n3, AT)), dim3(AT), 0, c->stream,
                       mu, 3 * n3);
    for (int i = 0; i < n_sp; ++i) {
      if (in[i].n == 0) continue;
      const unsigned nb = (unsigned)cdiv(in[i].n, AT);
      hipLaunchKernelGGL(k_vjp_init, dim3(nb), dim3(AT), 0, c->stream, lx1[i], lv1[i],
                         perm[i], in[i].n, cd, lx0[i], lv0[i]);
      hipLaunchKernelGGL(k_scatter_vec, dim3(nb), dim3(AT), 0, c->stream, P.x[i], lv0[i],
                         in[i].n, ng, ck, mu);
    }
    PM_LAUNCH_CHECK();
  }
  {
    ProfScope ps(c, ST_ADJOINT);
    if ((s = run_force_transpose(c, mu, c->nyq)) != PM_OK) return s;
  }
  {
    ProfScope ps(c, ST_ADJOINT);
    for (int i = 0; i < n_sp; ++i) {
      if (in[i].n == 0) continue;
      const float sscale = (float)(in[i].mass * (double)n3);
      hipLaunchKernelGGL(k_gather_grad, dim3((unsigned)cdiv(in[i].n, AT)), dim3(AT), 0,
                         c->stream, P.x[i], in[i].n, ng, mu, sscale, acc, lv0[i], ck, lx0[i],
                         1);
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
    const float sscale = (float)(2.0 * sp[i].mass * (double)n3);
    hipLaunchKernelGGL(k_gather_grad, dim3((unsigned)cdiv(sp[i].n, AT)), dim3(AT), 0,
                       c->stream, P.x[i], sp[i].n, ng, r, sscale, nullptr, nullptr, 0.f,
                       lam_x[i], 0);
  }
  PM_LAUNCH_CHECK();
  return PM_OK;
}

// The C ABI of libpm (include/pm.h): argument checks, context and scratch management,
// and the order of the kernel launches of each call.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "pm_common.h"

namespace {

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2_i(int64_t v) {
  int r = 0;
  while ((int64_t)1 << (r + 1) <= v) ++r;
  return r;
}

pm_status check_species(const pm_context* c, const pm_species* s, bool need_float_ptrs) {
  if (!s) return PM_ERR_ARG;
  if (s->n < 0 || s->n >= ((int64_t)1 << 32) - 1) return PM_ERR_ARG;
  if (!(s->mass >= 0.0) || !std::isfinite(s->mass)) return PM_ERR_ARG;
  if (s->layout == PM_FLOAT) {
    if (s->n > 0 && need_float_ptrs && (!s->x || !s->v)) return PM_ERR_ARG;
    return PM_OK;
  }
  if (s->layout == PM_COMPRESSED) {
    if (!s->count || !s->hdr) return PM_ERR_ARG;
    if (!widths_valid(s->widths)) return PM_ERR_ARG;
    if (s->n > 0 && (!s->pos || !s->vel)) return PM_ERR_ARG;
    if (s->cap_esc < 0 || (s->cap_esc > 0 && !s->esc)) return PM_ERR_ARG;
    return PM_OK;
  }
  return PM_ERR_ARG;
}

pm_status ensure_step_meshes(pm_context* c) {
  if (c->mesh) return PM_OK;
  const int64_t n3 = c->g.ng * c->g.ng * c->g.ng;
  if (hipMalloc(&c->mesh, (size_t)3 * n3 * sizeof(float)) != hipSuccess) {
    c->mesh = nullptr;
    return PM_ERR_NOMEM;
  }
  return PM_OK;
}

}  // namespace

void* scratch(pm_context* c, int id, size_t bytes) {
  DevBuf& b = c->scratch[id];
  if (bytes == 0) bytes = 1;
  if (b.bytes >= bytes) return b.p;
  if (b.p) {
    hipStreamSynchronize(c->stream);  // the old buffer may still be in use
    hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  size_t want = bytes + bytes / 8;  // headroom against repeated growth
  if (hipMalloc(&b.p, want) != hipSuccess) {
    b.p = nullptr;
    return nullptr;
  }
  b.bytes = want;
  return b.p;
}

void prof_begin(pm_context* c, int stage) {
  if (!c->prof) return;
  size_t i = c->prof_used;
  if (2 * i + 2 > c->prof_pool.size()) {
    for (int k = 0; k < 2; ++k) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      c->prof_pool.push_back(e);
    }
    c->prof_stage.push_back(0);
  }
  c->prof_stage[i] = stage;
  hipEventRecord(c->prof_pool[2 * i], c->stream);
  c->prof_open = (int)i;
  c->prof_used = i + 1;
}

void prof_end(pm_context* c) {
  if (!c->prof || c->prof_open < 0) return;
  hipEventRecord(c->prof_pool[2 * c->prof_open + 1], c->stream);
  c->prof_open = -1;
}

// pm_kick.hip
int deposit_tile_cells(const Geom& g);

extern "C" {

const char* pm_status_str(pm_status s) {
  switch (s) {
    case PM_OK: return "ok";
    case PM_ERR_ARG: return "invalid argument";
    case PM_ERR_SHAPE: return "unsupported mesh or cell size";
    case PM_ERR_NOMEM: return "device allocation failed";
    case PM_ERR_DEVICE: return "HIP call failed";
    case PM_ERR_CAPACITY: return "output capacity exceeded";
    case PM_ERR_CORRUPT: return "corrupt or inconsistent compressed data";
    case PM_ERR_RANGE: return "value out of range";
  }
  return "unknown status";
}

pm_status pm_create(const pm_config* cfg, void* stream, pm_ctx* out) {
  if (!cfg || !out) return PM_ERR_ARG;
  *out = nullptr;
  const int64_t ng = cfg->n_mesh, nc = cfg->n_cell, B = cfg->brick;
  if (!is_pow2(ng) || ng < 8 || ng > 2048) return PM_ERR_SHAPE;
  if (!is_pow2(nc) || nc > 1024 || nc > ng || ng / nc > 16) return PM_ERR_SHAPE;
  if (!is_pow2(B) || B > 8 || B > nc) return PM_ERR_SHAPE;
  if (!(cfg->soft_cells >= 0.0) || !std::isfinite(cfg->soft_cells)) return PM_ERR_ARG;
  if (!std::isfinite(cfg->G)) return PM_ERR_ARG;
  if (!(cfg->box > 0.0) || !std::isfinite(cfg->box)) return PM_ERR_ARG;
  if (cfg->prec != PM_PREC_F32) return PM_ERR_ARG;
  if (cfg->kernel != PM_KERNEL_FULL && cfg->kernel != PM_KERNEL_LONG &&
      cfg->kernel != PM_KERNEL_SHORT)
    return PM_ERR_ARG;
  if (cfg->kernel != PM_KERNEL_FULL && (!(cfg->r_split > 0.0) || !std::isfinite(cfg->r_split)))
    return PM_ERR_ARG;
  pm_context* c = new (std::nothrow) pm_context();
  if (!c) return PM_ERR_NOMEM;
  c->cfg = *cfg;
  c->stream = (hipStream_t)stream;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return PM_ERR_DEVICE;
  }
  Geom& g = c->g;
  g.ng = ng;
  g.nc = nc;
  g.B = (int32_t)B;
  g.r = (int32_t)(ng / nc);
  g.lgB = ilog2_i(B);
  g.lgnb = ilog2_i(nc / B);
  g.ncell3 = nc * nc * nc;
  g.nbrick = (nc / B) * (nc / B) * (nc / B);
  g.S = 256 * nc;
  g.box = cfg->box;
  g.ngL = (float)((double)ng / cfg->box);
  g.SL = (double)g.S / cfg->box;
  g.LS = (float)(cfg->box / (double)g.S);
  pm_status s = PM_OK;
  if (hipMalloc(&c->err, sizeof(DevErr)) != hipSuccess ||
      hipMalloc(&c->amax, 64) != hipSuccess ||
      hipMalloc(&c->nyq, (size_t)3 * ng * ng * sizeof(float2)) != hipSuccess) {
    s = PM_ERR_NOMEM;
  }
  if (s == PM_OK && hipMemsetAsync(c->err, 0, sizeof(DevErr), c->stream) != hipSuccess)
    s = PM_ERR_DEVICE;
  if (s == PM_OK) s = build_kernel_table(c);
  if (s == PM_OK) s = noalloc_init(c);
  if (s == PM_OK && hipStreamSynchronize(c->stream) != hipSuccess) s = PM_ERR_DEVICE;
  if (s != PM_OK) {
    pm_destroy(c);
    return s;
  }
  *out = c;
  return PM_OK;
}

pm_status pm_query_sizes(const pm_config* cfg, int64_t n_max, int n_sp, pm_sizes* out) {
  if (!cfg || !out || n_max < 0 || n_sp < 1 || n_sp > 4) return PM_ERR_ARG;
  const int64_t ng = cfg->n_mesh, nc = cfg->n_cell, B = cfg->brick;
  if (!is_pow2(ng) || ng < 8 || ng > 2048) return PM_ERR_SHAPE;
  if (!is_pow2(nc) || nc > 1024 || nc > ng || ng / nc > 16) return PM_ERR_SHAPE;
  if (!is_pow2(B) || B > 8 || B > nc) return PM_ERR_SHAPE;
  const int64_t n3 = ng * ng * ng, n2 = ng * ng, h1 = ng / 2 + 1, nc3 = nc * nc * nc;
  const int64_t nb = (nc / B) * (nc / B) * (nc / B), N = n_max;
  // grown scratch buffers carry 1/8 headroom
  auto grown = [](int64_t b) { return b + b / 8; };
  *out = pm_sizes{};
  // pm_create: kernel tables (by |n|^2 and the octant copy), twiddles, gradient symbol,
  // three Nyquist planes, error word and max |a|
  out->context_bytes = (3 * (ng / 2) * (ng / 2) + 1) * 4 + h1 * h1 * h1 * 4 + ng * 8 + ng * 4 +
                       3 * n2 * 8 + (int64_t)sizeof(DevErr) + 64;
  out->step_mesh_bytes = 3 * n3 * 4;
  // pm_encode / pm_step of N particles in n_sp species
  const int64_t rs_blocks = N / 4096 + 1;  // radix-sort workgroups (encode: uncapped)
  int64_t st = 0;
  st += grown(n3 * 4);                                  // spectrum scratch mesh
  st += grown(3 * n2 * 4);                              // per-row max |a| partials (bound)
  st += n_sp * grown((nc3 + 1) * 8);                    // cell offsets per species
  st += grown((nc3 + 1) * 8);                           // decode/pack offsets
  st += grown((nb + 1) * 8) + grown(nb * 4);            // re-sort: brick starts and totals
  st += grown(nc3 * 8 * n_sp);                          // new counts per cell
  st += grown(nc3 * 4) * 2 + grown((nc3 + 1) * 8);      // escape flags, their scan, counts
  st += grown(N * 3) + grown(N * 6) + grown(N * 2);     // new codes and digits, old order
  st += 4 * grown(N * 4);                               // mover keys and indices, two copies
  st += grown(nb * 4 * n_sp) + grown((nb + 1) * 8);     // movers per brick, their offsets
  st += grown(std::max<int64_t>(nb * 8 * n_sp, (N / 256 + 1) * 8));  // grid partials
  st += grown(rs_blocks * 256 * 4) + grown((rs_blocks * 256 + 1) * 8);  // radix histograms
  st += grown((std::max<int64_t>(std::max<int64_t>(nc3, N), rs_blocks * 256) / 4096 + 1) * 8);
  st += grown(4096) + grown(512 * 25 * 8) + grown(32);  // folds, reductions, mover counts
  st += grown(N * 12 + n_sp * 256);                     // extra accelerations (PP, long range)
  out->step_scratch_bytes = st;
  // pm_step_vjp adds the three adjoint meshes, the decoded positions and the recomputed
  // re-sort (permutations and a copy of the stream)
  int64_t vj = grown(3 * n3 * 4) + grown(N * 24 + n_sp * 512);
  vj += grown(N * 8 + N * 3 + N * 6 + n_sp * (nc3 + (N / 255 + 1) * 16 + 2048));
  out->vjp_scratch_bytes = vj;
  out->float_deposit_scratch_bytes = grown(n3 * 8);   // 64-bit fixed-point node sums
  out->compressed_species_bytes = nc3 + 9 * N + (N / 255 + 1) * 16 + (int64_t)sizeof(pm_shdr);
  out->float_species_bytes = 24 * N;
  return PM_OK;
}

pm_status pm_scratch_bytes(pm_ctx c, int64_t* bytes) {
  if (!c || !bytes) return PM_ERR_ARG;
  int64_t t = 0;
  for (const auto& b : c->scratch) t += (int64_t)b.bytes;
  *bytes = t;
  return PM_OK;
}

pm_status pm_destroy(pm_ctx c) {
  if (!c) return PM_ERR_ARG;
  hipStreamSynchronize(c->stream);
  hipFree(c->ktab);
  hipFree(c->gtab);
  hipFree(c->tw);
  hipFree(c->gk);
  hipFree(c->mesh);
  hipFree(c->nyq);
  hipFree(c->err);
  hipFree(c->amax);
  for (auto& b : c->scratch)
    if (b.p) hipFree(b.p);
  for (auto e : c->prof_pool) hipEventDestroy(e);
  delete c;
  return PM_OK;
}

pm_status pm_sync(pm_ctx c) {
  if (!c) return PM_ERR_ARG;
  PM_HIP_CHECK(hipStreamSynchronize(c->stream));
  DevErr e{};
  PM_HIP_CHECK(hipMemcpy(&e, c->err, sizeof(DevErr), hipMemcpyDeviceToHost));
  if (e.bits == 0) return PM_OK;
  c->last_detail = e.detail;
  DevErr z{};
  PM_HIP_CHECK(hipMemcpy(c->err, &z, sizeof(DevErr), hipMemcpyHostToDevice));
  if (e.bits & ERRBIT_CAPACITY) return PM_ERR_CAPACITY;
  if (e.bits & ERRBIT_CORRUPT) return PM_ERR_CORRUPT;
  if (e.bits & ERRBIT_RANGE) return PM_ERR_RANGE;
  return PM_ERR_ARG;
}

pm_status pm_last_error_detail(pm_ctx c, int64_t* needed) {
  if (!c || !needed) return PM_ERR_ARG;
  *needed = c->last_detail;
  return PM_OK;
}

pm_status pm_encode(pm_ctx c, const pm_species* in, pm_species* out, int64_t* perm) {
  if (!c || !in || !out) return PM_ERR_ARG;
  pm_status s;
  if ((s = check_species(c, in, true)) != PM_OK || in->layout != PM_FLOAT) return PM_ERR_ARG;
  if ((s = check_species(c, out, false)) != PM_OK || out->layout != PM_COMPRESSED)
    return PM_ERR_ARG;
  if (out->n != in->n) return PM_ERR_ARG;
  return run_encode(c, in, out, perm);
}

pm_status pm_decode(pm_ctx c, const pm_species* in, pm_species* out) {
  if (!c || !in || !out) return PM_ERR_ARG;
  if (check_species(c, in, false) != PM_OK || in->layout != PM_COMPRESSED) return PM_ERR_ARG;
  if (check_species(c, out, true) != PM_OK || out->layout != PM_FLOAT) return PM_ERR_ARG;
  if (out->n != in->n) return PM_ERR_ARG;
  return run_decode(c, in, out);
}

pm_status pm_deposit(pm_ctx c, const pm_species* sp, int n_sp, float* rho) {
  if (!c || !sp || !rho || n_sp <= 0 || n_sp > 4) return PM_ERR_ARG;
  for (int i = 0; i < n_sp; ++i)
    if (check_species(c, &sp[i], true) != PM_OK) return PM_ERR_ARG;
  return run_deposit(c, sp, n_sp, rho);
}

pm_status pm_force(pm_ctx c, const float* rho, float* acc, float* a_max) {
  if (!c || !rho || !acc) return PM_ERR_ARG;
  const int64_t n3 = c->g.ng * c->g.ng * c->g.ng;
  // rho may alias the x component only
  if (rho != acc && rho + n3 > acc && rho < acc + 3 * n3) return PM_ERR_ARG;
  return run_force(c, rho, acc, c->nyq, a_max ? a_max : c->amax);
}

static pm_status kick_all(pm_context* c, const pm_species* in, pm_species* out, int n_sp,
                          const float* acc, const float* a_max, double ck, double cd,
                          int64_t* const* offs, int64_t* const* perm = nullptr) {
  pm_status s;
  if (in[0].layout == PM_FLOAT) {
    for (int i = 0; i < n_sp; ++i) {
      if ((s = run_kick_float(c, &in[i], &out[i], acc, ck, cd)) != PM_OK) return s;
      if (perm && perm[i] && (s = run_iota(c, perm[i], in[i].n)) != PM_OK) return s;
    }
    return PM_OK;
  }
  int64_t* own[4] = {nullptr, nullptr, nullptr, nullptr};
  if (!offs) {
    for (int i = 0; i < n_sp; ++i) {
      own[i] = (int64_t*)scratch(c, SC_SPOFF0 + i, (size_t)(c->g.ncell3 + 1) * 8);
      if (!own[i]) return PM_ERR_NOMEM;
      if ((s = run_cell_offsets(c, &in[i], own[i])) != PM_OK) return s;
    }
    offs = own;
  }
  return run_kick_compressed_all(c, in, out, n_sp, offs, acc, a_max, ck, cd, perm);
}

static pm_status check_kick_args(pm_context* c, const pm_species* in, pm_species* out,
                                 int n_sp) {
  if (!in || !out || n_sp <= 0 || n_sp > 4) return PM_ERR_ARG;
  for (int i = 0; i < n_sp; ++i) {
    if (check_species(c, &in[i], true) != PM_OK) return PM_ERR_ARG;
    if (check_species(c, &out[i], true) != PM_OK) return PM_ERR_ARG;
    if (in[i].layout != out[i].layout || in[i].n != out[i].n) return PM_ERR_ARG;
    if (in[i].layout != in[0].layout) return PM_ERR_ARG;
    if (in[i].layout == PM_COMPRESSED &&
        (width_kind(in[i]) != width_kind(in[0]) || width_kind(out[i]) != width_kind(in[0])))
      return PM_ERR_ARG;
    if (in[i].layout == PM_COMPRESSED &&
        (in[i].pos == out[i].pos || in[i].vel == out[i].vel || in[i].count == out[i].count ||
         in[i].hdr == out[i].hdr))
      return PM_ERR_ARG;
  }
  return PM_OK;
}

pm_status pm_kick_drift(pm_ctx c, const pm_species* in, pm_species* out, int n_sp,
                        const float* acc, const float* a_max, double c_kick, double c_drift) {
  if (!c || !acc) return PM_ERR_ARG;
  pm_status s = check_kick_args(c, in, out, n_sp);
  if (s != PM_OK) return s;
  if (!std::isfinite(c_kick) || !std::isfinite(c_drift)) return PM_ERR_ARG;
  if (in[0].layout == PM_COMPRESSED && !a_max) return PM_ERR_ARG;
  return kick_all(c, in, out, n_sp, acc, a_max, c_kick, c_drift, nullptr);
}

pm_status pm_kick_drift_perm(pm_ctx c, const pm_species* in, pm_species* out, int n_sp,
                             const float* acc, const float* a_max, double c_kick,
                             double c_drift, int64_t* const* perm) {
  if (!c || !acc || !perm) return PM_ERR_ARG;
  pm_status s = check_kick_args(c, in, out, n_sp);
  if (s != PM_OK) return s;
  if (!std::isfinite(c_kick) || !std::isfinite(c_drift)) return PM_ERR_ARG;
  if (in[0].layout == PM_COMPRESSED && !a_max) return PM_ERR_ARG;
  return kick_all(c, in, out, n_sp, acc, a_max, c_kick, c_drift, nullptr, perm);
}

pm_status pm_step(pm_ctx c, const pm_species* in, pm_species* out, int n_sp, double dt) {
  if (!c) return PM_ERR_ARG;
  pm_status s = check_kick_args(c, in, out, n_sp);
  if (s != PM_OK) return s;
  if (!std::isfinite(dt)) return PM_ERR_ARG;
  if ((s = ensure_step_meshes(c)) != PM_OK) return s;
  float* mesh = c->mesh;
  if (in[0].layout == PM_COMPRESSED) {
    int64_t* offs[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int i = 0; i < n_sp; ++i) {
      offs[i] = (int64_t*)scratch(c, SC_SPOFF0 + i, (size_t)(c->g.ncell3 + 1) * 8);
      if (!offs[i]) return PM_ERR_NOMEM;
      if ((s = run_cell_offsets(c, &in[i], offs[i])) != PM_OK) return s;
    }
    if ((s = run_deposit_tile(c, in, n_sp, offs, mesh)) != PM_OK) return s;
    if ((s = run_force(c, mesh, mesh, c->nyq, c->amax)) != PM_OK) return s;
    return kick_all(c, in, out, n_sp, mesh, c->amax, dt, dt, offs);
  }
  if ((s = run_deposit(c, in, n_sp, mesh)) != PM_OK) return s;
  if ((s = run_force(c, mesh, mesh, c->nyq, c->amax)) != PM_OK) return s;
  return kick_all(c, in, out, n_sp, mesh, c->amax, dt, dt, nullptr);
}

pm_status pm_pp_accel(pm_ctx c, const pm_species* sp, int n_sp, double r_soft,
                      float* const* app, float* app_max) {
  if (!c || !sp || !app || n_sp <= 0 || n_sp > 4) return PM_ERR_ARG;
  if (!(r_soft >= 0.0) || !std::isfinite(r_soft)) return PM_ERR_ARG;
  for (int i = 0; i < n_sp; ++i) {
    if (check_species(c, &sp[i], true) != PM_OK || sp[i].layout != PM_COMPRESSED)
      return PM_ERR_ARG;
    if (sp[i].n > 0 && !app[i]) return PM_ERR_ARG;
  }
  int64_t* offs[4] = {nullptr, nullptr, nullptr, nullptr};
  pm_status s;
  for (int i = 0; i < n_sp; ++i) {
    offs[i] = (int64_t*)scratch(c, SC_SPOFF0 + i, (size_t)(c->g.ncell3 + 1) * 8);
    if (!offs[i]) return PM_ERR_NOMEM;
    if ((s = run_cell_offsets(c, &sp[i], offs[i])) != PM_OK) return s;
  }
  return run_pp_accel(c, sp, n_sp, offs, r_soft, app, app_max ? app_max : c->amax + 1);
}

pm_status pm_step_pp(pm_ctx c, const pm_species* in, pm_species* out, int n_sp, double dt,
                     double r_soft, int64_t* const* perm) {
  if (!c) return PM_ERR_ARG;
  pm_status s = check_kick_args(c, in, out, n_sp);
  if (s != PM_OK) return s;
  if (!std::isfinite(dt) || !(r_soft >= 0.0) || !std::isfinite(r_soft)) return PM_ERR_ARG;
  if (in[0].layout != PM_COMPRESSED) return PM_ERR_ARG;
  if ((s = ensure_step_meshes(c)) != PM_OK) return s;
  float* mesh = c->mesh;
  int64_t* offs[4] = {nullptr, nullptr, nullptr, nullptr};
  size_t bytes = 0;
  for (int i = 0; i < n_sp; ++i) {
    offs[i] = (int64_t*)scratch(c, SC_SPOFF0 + i, (size_t)(c->g.ncell3 + 1) * 8);
    if (!offs[i]) return PM_ERR_NOMEM;
    if ((s = run_cell_offsets(c, &in[i], offs[i])) != PM_OK) return s;
    bytes += ((size_t)in[i].n * 12 + 255) & ~(size_t)255;
  }
  char* pool = (char*)scratch(c, SC_PPACC, bytes);
  if (!pool) return PM_ERR_NOMEM;
  float* app[4] = {nullptr, nullptr, nullptr, nullptr};
  size_t at = 0;
  for (int i = 0; i < n_sp; ++i) {
    app[i] = (float*)(pool + at);
    at += ((size_t)in[i].n * 12 + 255) & ~(size_t)255;
  }
  if ((s = run_deposit_tile(c, in, n_sp, offs, mesh)) != PM_OK) return s;
  if ((s = run_force(c, mesh, mesh, c->nyq, c->amax)) != PM_OK) return s;
  if ((s = run_pp_accel(c, in, n_sp, offs, r_soft, app, c->amax + 1)) != PM_OK) return s;
  if ((s = run_add_max(c, c->amax, c->amax + 1, c->amax + 2)) != PM_OK) return s;
  return run_kick_compressed_all(c, in, out, n_sp, offs, mesh, c->amax + 2, dt, dt, perm,
                                 app);
}

pm_status pm_interp_accel(pm_ctx c, const pm_species* sp, int n_sp, const float* acc,
                          float* const* out, int accumulate) {
  if (!c || !sp || !acc || !out || n_sp <= 0 || n_sp > 4) return PM_ERR_ARG;
  for (int i = 0; i < n_sp; ++i) {
    if (check_species(c, &sp[i], true) != PM_OK || sp[i].layout != PM_COMPRESSED)
      return PM_ERR_ARG;
    if (sp[i].n > 0 && !out[i]) return PM_ERR_ARG;
  }
  int64_t* offs[4] = {nullptr, nullptr, nullptr, nullptr};
  pm_status s;
  for (int i = 0; i < n_sp; ++i) {
    offs[i] = (int64_t*)scratch(c, SC_SPOFF0 + i, (size_t)(c->g.ncell3 + 1) * 8);
    if (!offs[i]) return PM_ERR_NOMEM;
    if ((s = run_cell_offsets(c, &sp[i], offs[i])) != PM_OK) return s;
  }
  return run_interp_accel(c, sp, n_sp, offs, acc, out, accumulate);
}

pm_status pm_step_p3m(pm_ctx f, pm_ctx cc, const pm_species* in, pm_species* out, int n_sp,
                      double dt, double r_soft, int64_t* const* perm) {
  if (!f || !cc || f == cc) return PM_ERR_ARG;
  if (!split_pair_ok(f, cc)) return PM_ERR_ARG;
  pm_status s = check_kick_args(f, in, out, n_sp);
  if (s != PM_OK) return s;
  if (!std::isfinite(dt) || !(r_soft >= 0.0) || !std::isfinite(r_soft)) return PM_ERR_ARG;
  if (in[0].layout != PM_COMPRESSED) return PM_ERR_ARG;
  if ((s = ensure_step_meshes(f)) != PM_OK) return s;
  if ((s = ensure_step_meshes(cc)) != PM_OK) return s;
  // cell offsets depend on the counts, n_cell and brick only: the pair shares them
  int64_t* offs[4] = {nullptr, nullptr, nullptr, nullptr};
  size_t bytes = 0;
  for (int i = 0; i < n_sp; ++i) {
    offs[i] = (int64_t*)scratch(f, SC_SPOFF0 + i, (size_t)(f->g.ncell3 + 1) * 8);
    if (!offs[i]) return PM_ERR_NOMEM;
    if ((s = run_cell_offsets(f, &in[i], offs[i])) != PM_OK) return s;
    bytes += ((size_t)in[i].n * 12 + 255) & ~(size_t)255;
  }
  char* pool = (char*)scratch(f, SC_LRACC, bytes > 0 ? bytes : 256);
  if (!pool) return PM_ERR_NOMEM;
  float* app[4] = {nullptr, nullptr, nullptr, nullptr};
  size_t at = 0;
  for (int i = 0; i < n_sp; ++i) {
    app[i] = (float*)(pool + at);
    at += ((size_t)in[i].n * 12 + 255) & ~(size_t)255;
  }
  // long range: coarse deposit, force, interpolation into app
  float* cm = cc->mesh;
  if ((s = run_deposit_tile(cc, in, n_sp, offs, cm)) != PM_OK) return s;
  if ((s = run_force(cc, cm, cm, cc->nyq, cc->amax)) != PM_OK) return s;
  const bool pp = r_soft > 0.0;
  if (pp && (s = run_pp_accel(f, in, n_sp, offs, r_soft, app, f->amax + 1)) != PM_OK) return s;
  if ((s = run_interp_accel(cc, in, n_sp, offs, cm, app, pp ? 1 : 0)) != PM_OK) return s;
  // short range on the fine mesh
  float* fm = f->mesh;
  if ((s = run_deposit_tile(f, in, n_sp, offs, fm)) != PM_OK) return s;
  if ((s = run_force(f, fm, fm, f->nyq, f->amax)) != PM_OK) return s;
  // velocity bound: max |a_short| + max |a_long| (+ max |a_pp|)
  if ((s = run_add_max(f, f->amax, cc->amax, f->amax + 2)) != PM_OK) return s;
  if (pp && (s = run_add_max(f, f->amax + 2, f->amax + 1, f->amax + 2)) != PM_OK) return s;
  return run_kick_compressed_all(f, in, out, n_sp, offs, fm, f->amax + 2, dt, dt, perm, app);
}

pm_status pm_step_vjp(pm_ctx c, const pm_species* in, int n_sp, double dt,
                      float* const* lam_x1, float* const* lam_v1, float* const* lam_x0,
                      float* const* lam_v0) {
  if (!c || !in || n_sp <= 0 || n_sp > 4 || !lam_x1 || !lam_v1 || !lam_x0 || !lam_v0)
    return PM_ERR_ARG;
  for (int i = 0; i < n_sp; ++i) {
    if (check_species(c, &in[i], true) != PM_OK || in[i].layout != in[0].layout)
      return PM_ERR_ARG;
    if (in[i].n > 0 && (!lam_x1[i] || !lam_v1[i] || !lam_x0[i] || !lam_v0[i]))
      return PM_ERR_ARG;
    // results are written in another particle order than the cotangents are read
    for (int j = 0; j < n_sp; ++j)
      if (in[i].n > 0 && in[j].n > 0 &&
          (lam_x0[i] == lam_x1[j] || lam_x0[i] == lam_v1[j] || lam_v0[i] == lam_x1[j] ||
           lam_v0[i] == lam_v1[j]))
        return PM_ERR_ARG;
  }
  if (!std::isfinite(dt)) return PM_ERR_ARG;
  pm_status s = ensure_step_meshes(c);
  if (s != PM_OK) return s;
  return run_step_vjp(c, in, n_sp, dt, lam_x1, lam_v1, lam_x0, lam_v0);
}

pm_status pm_loss_density_vjp(pm_ctx c, const pm_species* sp, int n_sp, const float* rho_t,
                              double* loss, float* const* lam_x) {
  if (!c || !sp || n_sp <= 0 || n_sp > 4 || !rho_t || !lam_x) return PM_ERR_ARG;
  for (int i = 0; i < n_sp; ++i) {
    if (check_species(c, &sp[i], true) != PM_OK || sp[i].layout != sp[0].layout)
      return PM_ERR_ARG;
    if (sp[i].n > 0 && !lam_x[i]) return PM_ERR_ARG;
  }
  pm_status s = ensure_step_meshes(c);
  if (s != PM_OK) return s;
  return run_loss_vjp(c, sp, n_sp, rho_t, loss, lam_x);
}

pm_status pm_reduce(pm_ctx c, const pm_species* sp, int n_sp, const float* rho,
                    const float* acc, double* out) {
  if (!c || !out || n_sp < 0 || n_sp > 4 || (n_sp > 0 && !sp)) return PM_ERR_ARG;
  for (int i = 0; i < n_sp; ++i)
    if (check_species(c, &sp[i], true) != PM_OK) return PM_ERR_ARG;
  return run_reduce(c, sp, n_sp, rho, acc, out);
}

pm_status pm_reduce_noalloc(pm_ctx c, const pm_species* sp, int n_sp, const float* rho,
                            const float* acc, double* out) {
  if (!c || !out || n_sp < 0 || n_sp > 4 || (n_sp > 0 && !sp)) return PM_ERR_ARG;
  for (int i = 0; i < n_sp; ++i)
    if (check_species(c, &sp[i], true) != PM_OK) return PM_ERR_ARG;
  return run_reduce_noalloc(c, sp, n_sp, rho, acc, out);
}

pm_status pm_pack(pm_ctx c, const pm_species* sp, int32_t species_id, uint8_t* buf,
                  int64_t cap, int64_t* used) {
  if (!c || !sp || !buf || !used || cap < 64) return PM_ERR_ARG;
  if (check_species(c, sp, false) != PM_OK || sp->layout != PM_COMPRESSED) return PM_ERR_ARG;
  return run_pack(c, sp, species_id, buf, cap, used);
}

pm_status pm_pack_size(pm_ctx c, const pm_species* sp, int64_t* bytes) {
  if (!c || !sp || !bytes) return PM_ERR_ARG;
  if (check_species(c, sp, false) != PM_OK || sp->layout != PM_COMPRESSED) return PM_ERR_ARG;
  pm_shdr h;
  PM_HIP_CHECK(hipStreamSynchronize(c->stream));
  PM_HIP_CHECK(hipMemcpy(&h, sp->hdr, sizeof(h), hipMemcpyDeviceToHost));
  const int64_t rb = 3 * (width_pos(*sp) + width_vel(*sp));
  *bytes = 64 + rb * sp->n + c->g.ncell3 + 4 * h.n_esc;
  return PM_OK;
}

pm_status pm_unpack(pm_ctx c, const uint8_t* buf, int64_t len, pm_species* out, double* mass,
                    int32_t* species_id) {
  if (!c || !buf || !out || len < 0) return PM_ERR_ARG;
  if (check_species(c, out, false) != PM_OK || out->layout != PM_COMPRESSED) return PM_ERR_ARG;
  if (len < 64) return PM_ERR_CORRUPT;
  uint32_t ver, sid, brick, wword;
  uint64_t n, nc, csum, blen;
  float vmax;
  double m;
  if (std::memcmp(buf, "PMC1", 4) != 0) return PM_ERR_CORRUPT;
  std::memcpy(&ver, buf + 4, 4);
  std::memcpy(&sid, buf + 8, 4);
  std::memcpy(&brick, buf + 12, 4);
  std::memcpy(&n, buf + 16, 8);
  std::memcpy(&nc, buf + 24, 8);
  std::memcpy(&vmax, buf + 32, 4);
  std::memcpy(&wword, buf + 36, 4);
  std::memcpy(&m, buf + 40, 8);
  std::memcpy(&csum, buf + 48, 8);
  std::memcpy(&blen, buf + 56, 8);
  if (ver != 1 || brick != (uint32_t)c->g.B || nc != (uint64_t)c->g.nc) return PM_ERR_CORRUPT;
  if (blen != (uint64_t)(len - 64) || n != (uint64_t)out->n) return PM_ERR_CORRUPT;
  if (!(vmax >= 0.f) || !std::isfinite(vmax)) return PM_ERR_CORRUPT;
  // code widths: a valid word, equal to the destination's
  if (wword > 0xffffu || !widths_valid((int32_t)wword)) return PM_ERR_CORRUPT;
  if ((int32_t)wword != out->widths) return PM_ERR_ARG;
  const int P = width_pos(*out), V = width_vel(*out);
  const uint64_t RB = 3 * (uint64_t)(P + V);
  const uint8_t* body = buf + 64;
  uint64_t cs = 0;
  for (uint64_t i = 0; i < blen; ++i) cs += (2ull * i + 1ull) * body[i];
  if (cs != csum) return PM_ERR_CORRUPT;
  const int64_t ncell = c->g.ncell3;
  std::vector<uint8_t> count((size_t)ncell);
  std::vector<uint64_t> esc;
  std::vector<uint8_t> pos((size_t)n * 3 * P);
  std::vector<uint8_t> vel((size_t)n * 3 * V);
  uint64_t off = 0, p = 0;
  int32_t jmin = 65536, jmax = -1;
  for (int64_t cc = 0; cc < ncell; ++cc) {
    if (off >= blen) return PM_ERR_CORRUPT;
    uint64_t k = body[off++];
    if (k == 255) {
      if (off + 4 > blen) return PM_ERR_CORRUPT;
      uint32_t kk;
      std::memcpy(&kk, body + off, 4);
      off += 4;
      if (kk < 255) return PM_ERR_CORRUPT;
      k = kk;
      esc.push_back((uint64_t)cc);
      esc.push_back(k);
    }
    count[(size_t)cc] = (uint8_t)(k >= 255 ? 255 : k);
    if (p + k > n || off + RB * k > blen) return PM_ERR_CORRUPT;
    for (uint64_t q = 0; q < k; ++q, ++p, off += RB) {
      // little-endian codes in the stream; the device arrays hold them in the host's
      // byte order, which is little-endian on every machine this library runs on
      const uint8_t* r = body + off;
      std::memcpy(&pos[3 * P * p], r, 3 * P);
      for (int a = 0; a < 3; ++a) {
        int32_t w = r[3 * P + V * a];
        if (V == 2) w |= (int32_t)r[3 * P + V * a + 1] << 8;
        jmin = w < jmin ? w : jmin;
        jmax = w > jmax ? w : jmax;
      }
      std::memcpy(&vel[3 * V * p], r + 3 * P, 3 * V);
    }
  }
  if (p != n || off != blen) return PM_ERR_CORRUPT;
  const int64_t n_esc = (int64_t)esc.size() / 2;
  if (n_esc > out->cap_esc) {
    c->last_detail = n_esc;
    return PM_ERR_CAPACITY;
  }
  pm_shdr h{};
  h.v_max = vmax;
  h.j_min = jmin;
  h.j_max = jmax;
  h.n_esc = n_esc;
  PM_HIP_CHECK(hipStreamSynchronize(c->stream));
  PM_HIP_CHECK(hipMemcpy(out->count, count.data(), (size_t)ncell, hipMemcpyHostToDevice));
  if (n > 0) {
    PM_HIP_CHECK(hipMemcpy(out->pos, pos.data(), pos.size(), hipMemcpyHostToDevice));
    PM_HIP_CHECK(hipMemcpy(out->vel, vel.data(), vel.size(), hipMemcpyHostToDevice));
  }
  if (n_esc > 0)
    PM_HIP_CHECK(hipMemcpy(out->esc, esc.data(), esc.size() * 8, hipMemcpyHostToDevice));
  PM_HIP_CHECK(hipMemcpy(out->hdr, &h, sizeof(h), hipMemcpyHostToDevice));
  if (mass) *mass = m;
  if (species_id) *species_id = (int32_t)sid;
  return PM_OK;
}

pm_status pm_profile(pm_ctx c, int enable) {
  if (!c) return PM_ERR_ARG;
  PM_HIP_CHECK(hipStreamSynchronize(c->stream));
  c->prof = enable ? 1 : 0;
  c->prof_used = 0;
  c->prof_open = -1;
  return PM_OK;
}

pm_status pm_profile_read(pm_ctx c, double* ms, int64_t* launches, int cap) {
  if (!c || !ms || !launches || cap < 0) return PM_ERR_ARG;
  PM_HIP_CHECK(hipStreamSynchronize(c->stream));
  for (int k = 0; k < cap; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  for (size_t i = 0; i < c->prof_used; ++i) {
    int st = c->prof_stage[i];
    float t = 0.f;
    if (hipEventElapsedTime(&t, c->prof_pool[2 * i], c->prof_pool[2 * i + 1]) != hipSuccess)
      continue;
    if (st < cap) {
      ms[st] += t;
      launches[st] += 1;
    }
  }
  return PM_OK;
}

pm_status pm_kernel_table(pm_ctx c, float* out, int64_t cap) {
  if (!c || !out || cap < c->ktab_n) return PM_ERR_ARG;
  PM_HIP_CHECK(hipMemcpyAsync(out, c->ktab, (size_t)c->ktab_n * sizeof(float),
                              hipMemcpyDeviceToDevice, c->stream));
  return PM_OK;
}

}  // extern "C"

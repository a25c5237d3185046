// Internal declarations shared by the HIP translation units of libpm.
// Not part of the public ABI (see include/pm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "pm.h"

// ---------------------------------------------------------------- error latch --
// Device-side errors are OR-ed into a context word and returned by pm_sync().
enum : int32_t {
  ERRBIT_CAPACITY = 1,
  ERRBIT_CORRUPT = 2,
  ERRBIT_RANGE = 4,
  ERRBIT_ARG = 8,
};

struct DevErr {
  int32_t bits;
  int32_t pad;
  int64_t detail;  // e.g. capacity needed
};

__device__ inline void latch_error(DevErr* e, int32_t bit, int64_t detail = 0) {
  atomicOr(&e->bits, bit);
  if (detail) atomicMax((unsigned long long*)&e->detail, (unsigned long long)detail);
}

// ------------------------------------------------------------ XCD mapping --
// Workgroups are dispatched round-robin over the chip's 8 XCDs, each with its own L2.
// Giving every XCD a contiguous range of tiles keeps neighbouring tiles (which share
// halo cache lines) on the same L2.
__device__ inline int64_t xcd_tile(int64_t bid, int64_t ntiles) {
  if (ntiles % 8) return bid;
  return (bid & 7) * (ntiles >> 3) + (bid >> 3);
}

// ------------------------------------------------------- partial reductions --
// Whole-grid min/max without atomics: every workgroup stores its partial result at
// its own index, and a one-block kernel folds the partials.
pm_status fold_minmax_to_header(pm_context* c, const int32_t* mn, const int32_t* mx,
                                int64_t n, pm_shdr* hdr);   // hdr->j_min / j_max
pm_status fold_max_u32(pm_context* c, const uint32_t* part, int64_t n, uint32_t* out);

// ----------------------------------------------------------------- geometry --
// Cell keys: bricks of B^3 cells in x-fastest order, cells x-fastest inside a brick.
struct Geom {
  int64_t ng;      // mesh side
  int64_t nc;      // compression-cell side
  int32_t B;       // brick side (cells)
  int32_t r;       // ng / nc
  int32_t lgB;     // log2(B)
  int32_t lgnb;    // log2(nc / B)
  int64_t ncell3;  // nc^3
  int64_t nbrick;  // (nc/B)^3
  int64_t S;       // 256 nc (position codes per box side)
  double box;      // box side L (positions in [0, L))
  float ngL;       // ng / L: mesh cells per unit length (float)
  double SL;       // S / L: position codes per unit length
  float LS;        // L / S: length of one position code (float)
};

__host__ __device__ inline uint32_t cell_key(const Geom& g, uint32_t cx, uint32_t cy,
                                             uint32_t cz) {
  uint32_t m = (uint32_t)g.B - 1;
  uint32_t bx = cx >> g.lgB, by = cy >> g.lgB, bz = cz >> g.lgB;
  uint32_t b = (((bz << g.lgnb) + by) << g.lgnb) + bx;
  uint32_t l = ((((cz & m) << g.lgB) + (cy & m)) << g.lgB) + (cx & m);
  return (b << (3 * g.lgB)) + l;
}

__host__ __device__ inline void key_cell(const Geom& g, uint32_t key, uint32_t& cx,
                                         uint32_t& cy, uint32_t& cz) {
  uint32_t m = (uint32_t)g.B - 1;
  uint32_t b = key >> (3 * g.lgB), l = key & ((1u << (3 * g.lgB)) - 1);
  uint32_t nbm = (1u << g.lgnb) - 1;
  cx = ((b & nbm) << g.lgB) + (l & m);
  cy = (((b >> g.lgnb) & nbm) << g.lgB) + ((l >> g.lgB) & m);
  cz = ((b >> (2 * g.lgnb)) << g.lgB) + (l >> (2 * g.lgB));
}

// Code widths of a compressed species (pm_species.widths): 0 is the paper's 1-byte
// positions and 2-byte velocities, otherwise P | V << 8 with P, V in {1, 2}.
inline int width_pos(const pm_species& s) { return s.widths == 0 ? 1 : (s.widths & 255); }
inline int width_vel(const pm_species& s) { return s.widths == 0 ? 2 : (s.widths >> 8); }
// kind 0: (1, 2), 1: (2, 2), 2: (1, 1), 3: (2, 1)
inline int width_kind(const pm_species& s) {
  return (width_pos(s) - 1) | ((2 - width_vel(s)) << 1);
}
inline bool widths_valid(int32_t w) {
  if (w == 0) return true;
  const int p = w & 255, v = w >> 8;
  return (p == 1 || p == 2) && (v == 1 || v == 2) && w != (1 | (2 << 8));
}
// the one widths kind of the species of a call, or -1 when they differ
inline int common_width_kind(const pm_species* sp, int n_sp) {
  const int k = width_kind(sp[0]);
  for (int i = 1; i < n_sp; ++i)
    if (width_kind(sp[i]) != k) return -1;
  return k;
}

// --------------------------------------------------------------- scratch pool --
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct pm_context {
  pm_config cfg;
  hipStream_t stream;
  int device;
  Geom g;
  // gravity kernel table G(|n|^2)/n^3 (float) and twiddles exp(-2 pi i k/n), k<n
  float* ktab = nullptr;
  int64_t ktab_n = 0;
  float* gtab = nullptr;  // the same kernel values on the octant [kx][|ky|][|kz|] <= n/2
  float2* tw = nullptr;
  float* gk = nullptr;    // gradient symbol D(k), k < ng (fourth-order difference)
  // owned meshes for pm_step: 3 x ng^3 floats + 3 Nyquist planes (complex ng^2)
  float* mesh = nullptr;
  float2* nyq = nullptr;
  DevErr* err = nullptr;
  float* amax = nullptr;  // device scalar
  // grow-on-demand scratch
  DevBuf scratch[40];
  // this device's fixed array of pm_reduce_noalloc (device address, set by pm_create)
  unsigned char* na_scratch = nullptr;
  int64_t last_detail = 0;
  // stage profiler (pm_profile)
  int prof = 0;
  std::vector<hipEvent_t> prof_pool;
  std::vector<int> prof_stage;   // stage of pair i (events 2i, 2i+1)
  size_t prof_used = 0;          // pairs in use
  int prof_open = -1;            // pair index currently open
};

enum ProfStage {
  ST_OFFSETS = 0, ST_DEPOSIT, ST_FFT_R2C, ST_FFT_YF, ST_FFT_Z, ST_FFT_YI, ST_FFT_C2R,
  ST_KICK, ST_RESORT, ST_CODEC, ST_ADJOINT, ST_PP, ST_INTERP, ST_GRAD, ST_N
};
// Record a begin/end event pair around a group of launches (no-op unless profiling).
void prof_begin(pm_context* c, int stage);
void prof_end(pm_context* c);
struct ProfScope {
  pm_context* c;
  ProfScope(pm_context* cc, int stage) : c(cc) { prof_begin(c, stage); }
  ~ProfScope() { prof_end(c); }
};

enum ScratchId {
  SC_OFF = 0,      // int64 [ncell3+1] cell offsets (species A)
  SC_OFF2,         // int64 [nbrick+1] first new stream position of each brick (re-sort)
  SC_CNT,          // uint64 [ncell3] counts (stay | arrivals-before << 32)
  SC_BSUM,         // int64 block sums for scans
  SC_KEYA,         // uint32 [N]
  SC_VALA,         // uint32 [N]
  SC_KEYB,         // uint32 [N]
  SC_VALB,         // uint32 [N]
  SC_HIST,         // uint32 radix histograms
  SC_HOFF,         // int64 radix offsets
  SC_TPOS,         // uint8 [N][3]
  SC_TVEL,         // uint16 [N][3]
  SC_TDST,         // uint32 [N]
  SC_MCNT,         // uint32 [nbrick] movers per brick
  SC_MOFF,         // int64 [nbrick+1]
  SC_ACC64,        // uint64 [ng^3] fixed-point accumulator (float layout deposit)
  SC_FLAG,         // uint32: escape counts per block of cells / misc
  SC_FOFF,         // int64: their offsets / misc
  SC_MISC,         // small
  SC_VJP,          // float [3][ng^3] adjoint meshes
  SC_VJP2,         // decoded positions of compressed species (adjoint)
  SC_VJP3,         // recomputed re-sort of the adjoint: permutations and stream copies
  SC_COUNT32,      // uint32 [ncell3]
  SC_SPOFF0,       // int64 [ncell3+1] cell offsets of species 0..3
  SC_SPOFF1,
  SC_SPOFF2,
  SC_SPOFF3,
  SC_PARTS,        // per-workgroup partial results of grid reductions
  SC_SPEC,         // float [ng^3] spectrum scratch of the force transforms
  SC_FOLD,         // first-stage results of the grid min / max folds
  SC_NMOV,         // int64 [4]: mover count of each species (device-side)
  SC_PPMAX,        // per-workgroup max |a| of the PP force
  SC_PPACC,        // float [N][3] PP accelerations of pm_step_pp
  SC_LRACC,        // float [N][3] long-range accelerations of pm_step_p3m
  SC_BTOT,         // uint32 [nbrick] new particles per brick (re-sort)
  SC_N
};

void* scratch(pm_context* c, int id, size_t bytes);  // grows; nullptr on failure

#define PM_HIP_CHECK(expr)                         \
  do {                                             \
    hipError_t _e = (expr);                        \
    if (_e != hipSuccess) return PM_ERR_DEVICE;    \
  } while (0)

#define PM_LAUNCH_CHECK()                          \
  do {                                             \
    hipError_t _e = hipGetLastError();             \
    if (_e != hipSuccess) return PM_ERR_DEVICE;    \
  } while (0)

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ------------------------------------------------------------ launch wrappers --
// scan / sort / fill (pm_scan.hip)
pm_status launch_fill_u32(pm_context* c, uint32_t* p, int64_t n, uint32_t v);
pm_status launch_fill_u64(pm_context* c, uint64_t* p, int64_t n, uint64_t v);
pm_status run_iota(pm_context* c, int64_t* p, int64_t n);  // p[i] = i
// exclusive scans into int64 out[n+1]
pm_status scan_u32(pm_context* c, const uint32_t* in, int64_t n, int64_t* out);
pm_status scan_u64lo(pm_context* c, const uint64_t* in, int64_t n, int64_t* out);
pm_status scan_counts(pm_context* c, const uint8_t* count, const uint64_t* esc,
                      const pm_shdr* hdr, int64_t n, int64_t* out);
// stable LSD radix sort of (key, val) pairs on the low `bits` of key; results land in
// *keys/*vals (which may be swapped with the alternate buffers).
pm_status radix_sort_pairs(pm_context* c, uint32_t** keys, uint32_t** vals,
                           uint32_t** keys_alt, uint32_t** vals_alt, int64_t n,
                           int bits);
// the same with the pair count read on the device (*n_dev <= n_max): nothing waits on
// the host for a count the device produced
pm_status radix_sort_pairs_dev(pm_context* c, uint32_t** keys, uint32_t** vals,
                               uint32_t** keys_alt, uint32_t** vals_alt, int64_t n_max,
                               const int64_t* n_dev, int bits);

// codec (pm_codec.hip)
pm_status run_encode(pm_context* c, const pm_species* in, pm_species* out, int64_t* perm);
pm_status run_decode(pm_context* c, const pm_species* in, pm_species* out);
pm_status run_cell_offsets(pm_context* c, const pm_species* sp, int64_t* off);
pm_status scan_counts_into(pm_context* c, const pm_species* sp, int64_t* off, int64_t* bsum);
pm_status run_finalize_counts(pm_context* c, const uint32_t* cnt32, const uint64_t* cnt64,
                              pm_species* out);
pm_status run_pack(pm_context* c, const pm_species* sp, int32_t sid, uint8_t* buf,
                   int64_t cap, int64_t* used);
pm_status run_reduce(pm_context* c, const pm_species* sp, int n_sp, const float* rho,
                     const float* acc, double* out);
// the same reductions with every buffer in a fixed device array (no allocation)
pm_status noalloc_init(pm_context* c);
pm_status run_reduce_noalloc(pm_context* c, const pm_species* sp, int n_sp,
                             const float* rho, const float* acc, double* out);

// deposit (pm_deposit.hip)
pm_status run_deposit(pm_context* c, const pm_species* sp, int n_sp, float* rho);
pm_status run_deposit_tile(pm_context* c, const pm_species* sp, int n_sp,
                           int64_t* const* offs, float* rho);

// FFT (pm_fft.hip)
pm_status build_kernel_table(pm_context* c);
pm_status run_force(pm_context* c, const float* rho, float* acc, float2* nyq,
                    float* amax);
// adjoint transform: nu = sum_a IDFT(+i k_a G DFT(mu_a)); mu in acc[3] (destroyed),
// result written to acc component 0.
pm_status run_force_transpose(pm_context* c, float* acc, float2* nyq);

// kick-drift (pm_kick.hip)
pm_status run_kick_float(pm_context* c, const pm_species* in, pm_species* out,
                         const float* acc, double ck, double cd);
// All species of a compressed state: the fused kick and the re-sort. offs[s]: input cell
// offsets; perm[s] (nullable): new stream position -> old; app[s] (nullable array):
// per-particle accelerations added to the interpolated force (the PP term).
pm_status run_kick_compressed_all(pm_context* c, const pm_species* in, pm_species* out,
                                  int n_sp, int64_t* const* offs, const float* acc,
                                  const float* amax, double ck, double cd,
                                  int64_t* const* perm, const float* const* app = nullptr);
// PP force of eq. (4) inside the mesh cells (pm_pp.hip): app[s] float [n][3], stream
// order; pmax receives max |a| over all particles and axes
pm_status run_pp_accel(pm_context* c, const pm_species* sp, int n_sp, int64_t* const* offs,
                       double r_soft, float* const* app, float* pmax);
pm_status run_add_max(pm_context* c, const float* a, const float* b, float* out);
// two-level force (pm_split.hip): CIC interpolation of force meshes to compressed
// particles (out per species [n][3], stream order; accumulate adds), and the check that
// two contexts form a fine/coarse pair of the split
pm_status run_interp_accel(pm_context* c, const pm_species* sp, int n_sp,
                           int64_t* const* offs, const float* acc, float* const* out,
                           int accumulate);
bool split_pair_ok(const pm_context* fine, const pm_context* coarse);
pm_status run_kick_compressed(pm_context* c, const pm_species* in, pm_species* out,
                              const float* acc, const float* amax, double ck, double cd,
                              uint32_t* perm_new_to_old);

// adjoint (pm_adjoint.hip)
pm_status run_step_vjp(pm_context* c, const pm_species* in, int n_sp, double dt,
                       float* const* lx1, float* const* lv1, float* const* lx0,
                       float* const* lv0);
pm_status run_loss_vjp(pm_context* c, const pm_species* sp, int n_sp, const float* rho_t,
                       double* loss, float* const* lam_x);

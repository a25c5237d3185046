/*
 * pm.h - C ABI of the MI355X particle-mesh (PM) step with compressed particles.
 *
 * The library advances a periodic box of two particle species (cold dark matter and
 * neutrinos) by one particle-mesh gravity step, as described in Emberson et al.,
 * "Cosmological neutrino simulations at extreme scale" (arXiv:1611.01545):
 *   - cloud-in-cell (CIC) mass deposit of all species on one mesh (Sec. 2.1 and its
 *     footnote; CIC is named in Sec. 2.3),
 *   - FFT solution of the Poisson equation, eqs. (1)-(2), and the spectral force of
 *     eq. (3), with Plummer softening of the kernel,
 *   - CIC interpolation of the force back to the particles (Fig. 2,
 *     "inverse_force_interpolation"),
 *   - a kick-drift leapfrog update,
 * on particles stored in the compressed phase-space format of Sec. 2.4: per-cell
 * particle counts (one byte, 255 + a 4-byte count as escape), one byte per axis of
 * position offset inside the cell and a 2-byte velocity histogram index per axis.
 *
 * Conventions for every entry point:
 *   - periodic box of side L (pm_config.box); positions in [0, L); mesh arrays are
 *     float [z][y][x] (x fastest);
 *     particle float arrays are [n][3] with columns x, y, z;
 *   - all pointers documented "device" are device memory on the context's GPU; the
 *     caller owns them and keeps them alive until the work is done;
 *   - calls validate their arguments on the host, then enqueue asynchronously on the
 *     context's HIP stream and return; errors detected on the device (capacity
 *     exceeded, out-of-range input) are latched and returned by pm_sync();
 *   - counts and indices are 64-bit;
 *   - a context is not thread-safe; calls on one context are ordered by its stream.
 *
 * Status codes: PM_OK on success; PM_ERR_ARG for a null or inconsistent argument;
 * PM_ERR_SHAPE for mesh/cell sizes the library does not support; PM_ERR_NOMEM when a
 * device allocation fails; PM_ERR_DEVICE when a HIP call fails; PM_ERR_CAPACITY when
 * an output buffer is too small (pm_last_error_detail reports the size needed);
 * PM_ERR_CORRUPT for a byte stream that fails its integrity checks; PM_ERR_RANGE for
 * non-finite input.
 */
#ifndef PM_H
#define PM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pm_status {
  PM_OK = 0,
  PM_ERR_ARG = 1,
  PM_ERR_SHAPE = 2,
  PM_ERR_NOMEM = 3,
  PM_ERR_DEVICE = 4,
  PM_ERR_CAPACITY = 5,
  PM_ERR_CORRUPT = 6,
  PM_ERR_RANGE = 7
} pm_status;

typedef struct pm_context* pm_ctx;

/* Arithmetic of the mesh and particle kernels: float32 meshes, FFTs and kicks, with
 * positions exact in the fixed-point codes of compressed species and float64 global
 * reductions and kernel-table construction. No other precision is built. */
enum { PM_PREC_F32 = 0 };

/* Sizes and physics constants of a context.
 *   n_mesh     PM mesh side n_g: a power of two, 8 <= n_mesh <= 2048.
 *   n_cell     compression mesh side n_c (Sec. 2.4 uses (n_p/2)^3 cells): a power of
 *              two, 1 <= n_cell <= 1024, dividing n_mesh, n_mesh/n_cell <= 16.
 *   brick      cells per brick side B of the stream order: a power of two dividing
 *              n_cell, B <= 8. Cells are ordered brick by brick (x fastest), and x
 *              fastest inside a brick; B = 1 is plain row-major order.
 *   prec       PM_PREC_F32 (anything else: PM_ERR_ARG).
 *   box        box side L > 0: float positions lie in [0, L), the mesh spacing is
 *              Delta = L / n_mesh and densities are mass per unit volume. A power of two
 *              keeps every position conversion exact (L = 1 is the unit box).
 *   G          gravitational constant (1/(4 pi) makes 4 pi G = 1).
 *   soft_cells Plummer softening length in mesh cells (>= 0).
 *   kernel     which part of the two-level force split the context's force computes
 *              (PM_KERNEL_*; 0 is the one-level kernel).
 *   reserved   0.
 *   r_split    split length r_s of the two-level force in units of length (> 0 for
 *              PM_KERNEL_LONG and PM_KERNEL_SHORT, ignored otherwise). */
typedef struct pm_config {
  int64_t n_mesh;
  int64_t n_cell;
  int32_t brick;
  int32_t prec;
  double box;
  double G;
  double soft_cells;
  int32_t kernel;
  int32_t reserved;
  double r_split;
} pm_config;

/* Two-level force split (Sec. 2.1: a long-range force on a coarse mesh spanning the box,
 * a short-range force on a mesh 4 times finer; the paper gives no split kernel). With
 * G(k) the softened kernel of pm_force and k the wave vector (2 pi n / L):
 *   PM_KERNEL_FULL   G(k), one level;
 *   PM_KERNEL_LONG   G(k) exp(-k^2 r_s^2) / prod_a sinc(n_a / n_mesh)^4, sinc(t) =
 *                    sin(pi t) / (pi t): the long-range part for the coarse mesh, with
 *                    that mesh's CIC deposit and interpolation windows divided out;
 *   PM_KERNEL_SHORT  G(k) (1 - exp(-k^2 r_s^2)): the short-range part for the fine mesh.
 * A two-level pair is a fine context (PM_KERNEL_SHORT) and a coarse one
 * (PM_KERNEL_LONG) with the same r_split, softening length (soft_cells times the
 * mesh spacing), n_cell, brick, box and G; pm_step_p3m steps them together. The
 * paper's configuration is n_mesh(coarse) = n_cell = (n_p/2), n_mesh(fine) = 4 n_cell,
 * and r_s = 1.25 coarse cells (the short-range force of a point mass is then below 1%
 * of Newton's beyond 24 fine cells, the tile buffer the paper uses). */
enum { PM_KERNEL_FULL = 0, PM_KERNEL_LONG = 1, PM_KERNEL_SHORT = 2 };

/* Device-resident header of one compressed species (32 bytes).
 *   v_max  half-range of the velocity histogram (the paper keeps it in the file
 *          header, one per species, Sec. 2.4);
 *   j_min, j_max  smallest / largest velocity code present (65536 / -1 if none);
 *   flags  0 for a valid state;
 *   n_esc  number of escape entries in use. */
typedef struct pm_shdr {
  float v_max;
  int32_t j_min;
  int32_t j_max;
  int32_t flags;
  int64_t n_esc;
  int64_t reserved;
} pm_shdr;

enum { PM_FLOAT = 0, PM_COMPRESSED = 1 };

/* One particle species.
 *   layout  PM_FLOAT: x, v are device float [n][3] (positions in [0,1)).
 *           PM_COMPRESSED: count, pos, vel, esc, hdr describe the Sec. 2.4 format:
 *             count  device uint8 [n_cell^3], one per cell in stream order; 255 means
 *                    "see the escape table";
 *             pos    device uint8 [n][3], position offset inside the cell, in units
 *                    of 1/(256 n_cell);
 *             vel    device uint16 [n][3], velocity bin in [0, 65535] over
 *                    [-v_max, v_max];
 *             esc    device uint64 [cap_esc][2], (cell, count) for every cell with
 *                    count >= 255, sorted by cell;
 *             hdr    device pm_shdr.
 *   widths  code widths of a compressed species (Sec. 2.4, closing remark: a memory-light
 *           variant keeps positions and velocities in 8 or 16 bits): 0 for the format
 *           above (1-byte positions, 2-byte velocities), else P | V << 8 with P, V in
 *           {1, 2}. P = 2: pos holds uint16 [n][3] offsets in units of 1/(65536 n_cell)
 *           (S = 65536 n_cell position steps per box side); V = 1: vel holds uint8
 *           [n][3] indices into 256 bins over [-v_max, v_max] (code floor(v 128 / v_max
 *           + 128) clamped to [0, 255], bin centre (j - 127.5) v_max / 128). The pointers
 *           keep their C types and are read as those arrays. All species of one call
 *           have the same widths (PM_ERR_ARG otherwise). Ignored for PM_FLOAT.
 *   n       particle count (>= 0); mass  mass per particle. */
typedef struct pm_species {
  int32_t layout;
  int32_t widths;
  int64_t n;
  double mass;
  float* x;
  float* v;
  uint8_t* count;
  uint8_t* pos;
  uint16_t* vel;
  uint64_t* esc;
  int64_t cap_esc;
  pm_shdr* hdr;
} pm_species;

/* Message for a status code (static string). */
const char* pm_status_str(pm_status s);

/* Device memory of a configuration, for planning (host only, no GPU call). Bytes:
 *   context_bytes     what pm_create allocates (kernel tables, twiddles, gradient
 *                     symbol, Nyquist planes), exact;
 *   step_mesh_bytes   the context's force meshes (3 n_mesh^3 floats, allocated by the
 *                     first pm_step, pm_step_vjp or pm_loss_density_vjp), exact;
 *   step_scratch_bytes  upper bound of the scratch that pm_encode and pm_step (also
 *                     pm_step_pp and, for the fine context, pm_step_p3m) grow for
 *                     n_max particles in total over n_sp species (1 <= n_sp <= 4);
 *   vjp_scratch_bytes   upper bound of what pm_step_vjp adds to that;
 *   float_deposit_scratch_bytes  what a PM_FLOAT deposit adds (8 n_mesh^3);
 *   compressed_species_bytes  one compressed species of n_max particles with
 *                     cap_esc = n_max / 255 + 1 (caller-owned);
 *   float_species_bytes  one float species of n_max particles (caller-owned).
 * Scratch is grown on first use and kept until pm_destroy; pm_scratch_bytes reports
 * what a context holds. */
typedef struct pm_sizes {
  int64_t context_bytes;
  int64_t step_mesh_bytes;
  int64_t step_scratch_bytes;
  int64_t vjp_scratch_bytes;
  int64_t float_deposit_scratch_bytes;
  int64_t compressed_species_bytes;
  int64_t float_species_bytes;
} pm_sizes;

pm_status pm_query_sizes(const pm_config* cfg, int64_t n_max, int n_sp, pm_sizes* out);
/* Scratch bytes a context currently holds (host value). */
pm_status pm_scratch_bytes(pm_ctx ctx, int64_t* bytes);

/* Create a context on the current HIP device; `stream` is a hipStream_t (NULL for
 * the default stream). Builds the gravity-kernel table in float64 on the GPU. */
pm_status pm_create(const pm_config* cfg, void* stream, pm_ctx* out);
pm_status pm_destroy(pm_ctx ctx);

/* Wait for all enqueued work; return the first latched device error (and clear it). */
pm_status pm_sync(pm_ctx ctx);
/* After PM_ERR_CAPACITY: the capacity (elements) that would have been needed. */
pm_status pm_last_error_detail(pm_ctx ctx, int64_t* needed);

/* Compress float particles (Sec. 2.4): position code u = floor(x S / L) mod S per axis
 * (S = 256 n_cell, cell u >> 8, byte u & 255; with out->widths P = 2, S = 65536 n_cell,
 * cell u >> 16, offset u & 65535); v_max = largest |v_a| of the species; cells of the
 * n_cell^3 mesh in stream order; particles of a cell in input order.
 * in: PM_FLOAT; out: PM_COMPRESSED with out->n == in->n. perm (device int64 [n],
 * nullable) receives, for each stream position, the input index of that particle. */
pm_status pm_encode(pm_ctx ctx, const pm_species* in, pm_species* out, int64_t* perm);

/* Decompress to bin centres (u + 1/2) L / S (S = 256^P n_cell), in stream order (Sec. 2.4,
 * used for restarts).
 * in: PM_COMPRESSED; out: PM_FLOAT with out->n == in->n. */
pm_status pm_decode(pm_ctx ctx, const pm_species* in, pm_species* out);

/* CIC mass density rho(c) = Delta^-3 sum_s m_s sum_i W(x_i - x_c) of all species
 * (Sec. 2.1 footnote: both species on the same mesh). rho: device float [n_mesh^3].
 * Species must all be PM_FLOAT or all PM_COMPRESSED. Deterministic: PM_COMPRESSED
 * sums each species' exact CIC weights as integers per node, scales each sum by the
 * species' mass in FP64, rounds it to float and adds the species in a fixed order
 * (with 2-byte positions each node's weight is the exact product rounded to a multiple
 * of 2^-27, the 1-byte form's exact unit); PM_FLOAT sums all contributions in 64-bit
 * fixed point. */
pm_status pm_deposit(pm_ctx ctx, const pm_species* sp, int n_sp, float* rho);

/* Accelerations a_a(c) from a density mesh, eqs. (2)-(3): a = IDFT(-i D(k) G(k) DFT(rho))
 * with the softened kernel G(k) = -4 pi G eps K1(k eps)/k, G(0) = 0, eps =
 * soft_cells Delta, and for the gradient of eq. (3) the symbol of the fourth-order
 * central difference, D(k_a) = (8 sin(k_a Delta) - sin(2 k_a Delta)) / (6 Delta) (zero on
 * the Nyquist index). acc: device float
 * [3][n_mesh^3]; rho may alias acc (component x). a_max (device float, nullable)
 * receives max |a_a(c)| over the mesh. rho is not preserved when it aliases acc. */
pm_status pm_force(pm_ctx ctx, const float* rho, float* acc, float* a_max);

/* Interpolate acc to the particles (CIC), kick v' = v + c_kick a, drift
 * x' = x + c_drift v' (mod L). PM_FLOAT: in and out may be the same arrays.
 * PM_COMPRESSED: in and out must be distinct; positions drift in fixed point
 * (u' = u + floor(v' c_drift S / L + 1/2), S = 256^P n_cell), velocities are re-binned with
 * v_max' = the smallest power of two >= max|v_decoded| + |c_kick| a_max, and the
 * stream is re-sorted stably into cell order. a_max: device float from pm_force
 * (required for PM_COMPRESSED). */
pm_status pm_kick_drift(pm_ctx ctx, const pm_species* in, pm_species* out, int n_sp,
                        const float* acc, const float* a_max, double c_kick,
                        double c_drift);

/* pm_kick_drift that also reports, per species, the re-sort of compressed streams:
 * perm[s] (device int64 [n], nullable) receives for each new stream position the
 * old stream position of that particle (identity for PM_FLOAT). The format stores no
 * particle identities (Sec. 2.4); this map is what carries cotangents and test
 * comparisons across the re-sort. perm is a host array of n_sp device pointers. */
pm_status pm_kick_drift_perm(pm_ctx ctx, const pm_species* in, pm_species* out, int n_sp,
                             const float* acc, const float* a_max, double c_kick,
                             double c_drift, int64_t* const* perm);

/* One full step (deposit, force, kick-drift) with c_kick = c_drift = dt, using the
 * context's own mesh buffers. Same layout rules as pm_kick_drift. */
pm_status pm_step(pm_ctx ctx, const pm_species* in, pm_species* out, int n_sp, double dt);

/* The particle-particle force of eq. (4) (Sec. 2.1) inside the cells of the PM mesh:
 * a_i = G sum_j m_j (x_j - x_i) / |x_j - x_i|^3 over the particles j != i of every species
 * that share particle i's mesh cell (side L / n_mesh), truncated below the softening length
 * r_soft (pairs closer than r_soft exert no force; the paper takes r_soft = L / (20 n_p)).
 * Compressed species only (positions at bin centres; the cut is decided on the integer
 * code differences, |du|^2 >= (r_soft 256 n_cell / L)^2). app: host array of n_sp device
 * float [n][3] results in stream order; app_max (device float, nullable) receives the
 * largest |a| component. Float32 sums in stream order (deterministic). */
pm_status pm_pp_accel(pm_ctx ctx, const pm_species* sp, int n_sp, double r_soft,
                      float* const* app, float* app_max);

/* pm_step with the PP force added to the interpolated mesh force in the kick (the P^3M
 * step of Sec. 2.1 on one mesh): v' = v + dt (a_mesh + a_pp), x' = x + dt v'; the velocity
 * bound of the re-encode uses max |a_mesh| + max |a_pp|. Compressed species only. perm
 * (nullable host array of n_sp device int64 [n] pointers, entries nullable) receives the
 * re-sort as in pm_kick_drift_perm. */
pm_status pm_step_pp(pm_ctx ctx, const pm_species* in, pm_species* out, int n_sp, double dt,
                     double r_soft, int64_t* const* perm);

/* CIC interpolation of the context's force meshes to the particles (the inverse force
 * interpolation of Sec. 2.3, Fig. 2) without the kick: acc is device float
 * [3][n_mesh^3] (as pm_force writes it); out is a host array of n_sp device float [n][3]
 * results in stream order. accumulate = 0 writes out, 1 adds to it. Compressed species
 * only (mesh positions (u + 1/2) n_mesh / (256 n_cell) per axis, exact in float32).
 * Float32 sums over the 8 nodes in a fixed order. */
pm_status pm_interp_accel(pm_ctx ctx, const pm_species* sp, int n_sp, const float* acc,
                          float* const* out, int accumulate);

/* One step of the two-level force (Sec. 2.1): the long-range force on the coarse
 * context's mesh (deposit, pm_force with PM_KERNEL_LONG, interpolation), the short-range
 * force on the fine context's mesh (PM_KERNEL_SHORT), and for r_soft > 0 the PP force of
 * eq. (4) inside the fine mesh's cells (pm_pp_accel); then the kick-drift-re-encode of
 * pm_step with v' = v + dt (a_short + a_long + a_pp), x' = x + dt v'. The velocity bound
 * of the re-encode uses max |a_short| + max |a_long| (meshes) + max |a_pp|. Compressed
 * species only; fine and coarse must be a two-level pair (see PM_KERNEL_LONG) created on
 * the same stream; PM_ERR_ARG otherwise. perm as in pm_step_pp. Scratch (the long-range
 * and PP accelerations, 12 bytes per particle each) is the fine context's. */
pm_status pm_step_p3m(pm_ctx fine, pm_ctx coarse, const pm_species* in, pm_species* out,
                      int n_sp, double dt, double r_soft, int64_t* const* perm);

/* Adjoint of pm_step at state `in` (straight-through for the quantisation of
 * compressed states). lam_x1, lam_v1: per species device float [n][3] cotangents of
 * the step's outputs, in the output's particle order; lam_x0, lam_v0: results, in
 * the input's particle order (no result array may be one of the cotangent arrays:
 * PM_ERR_ARG). Arrays are passed as arrays of n_sp device pointers (host arrays of
 * pointers). The step is recomputed (deposit, force and, for compressed states, the
 * re-sort that maps output order to input order); the cotangent of the interpolated
 * force is scattered to three meshes, taken through the transposed force operator
 * (eqs. (1)-(3): the conjugate spectral multiplier +i k G) and gathered with the
 * gradient of the CIC weights. For compressed states on 16-node tiles (r = 2, 4 or 8
 * mesh cells per compression cell) the scatter sums 32-bit fixed-point integers per
 * tile and species, and the result is the same on every call; other shapes and float
 * states sum with float atomics, and results may then differ between calls in the
 * last bits. */
pm_status pm_step_vjp(pm_ctx ctx, const pm_species* in, int n_sp, double dt,
                      float* const* lam_x1, float* const* lam_v1, float* const* lam_x0,
                      float* const* lam_v0);

/* Density loss L = sum_c (rho(c) - rho_t(c))^2 of the species' CIC density against a
 * target mesh (device float [n_mesh^3]); loss (device double, nullable) and
 * dL/dx per species (host array of n_sp device float [n][3] pointers). */
pm_status pm_loss_density_vjp(pm_ctx ctx, const pm_species* sp, int n_sp,
                              const float* rho_target, double* loss,
                              float* const* lam_x);

/* Float64 global reductions on the GPU: the conserved quantities that check the method
 * (Sec. 2.1: the CIC deposit and interpolation with a real odd gradient conserve mass and
 * momentum). out: device double [8 + 6 n_sp]:
 *   out[0]        sum_c rho(c) Delta^3 (0 if rho is NULL),
 *   out[1]        sum_s m_s N_s,
 *   out[2..4]     sum_i m_i v_i over all species,
 *   out[5..7]     sum_i m_i a_i over all species, a_i the CIC interpolation of acc at the
 *                 particle (0 if acc is NULL; it vanishes up to rounding when acc is the
 *                 force of the same particles' density),
 *   out[8+6s..]   per species s: m_s sum_i v_i (3), then m_s sum_i a_i (3).
 * Compressed species use decoded bin centres and velocities. acc: device float
 * [3][n_mesh^3] or NULL. Asynchronous; 0 <= n_sp <= 4. */
pm_status pm_reduce(pm_ctx ctx, const pm_species* sp, int n_sp, const float* rho,
                    const float* acc, double* out);

/* pm_reduce for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. Same arguments, results
 * and kernels as pm_reduce; it calls no allocator. Every buffer it needs (partial sums,
 * the cell offsets of one compressed species, the scan's block sums) lives in one fixed
 * array of 365 KB per device, held until the process ends, whose address pm_create takes
 * once per device. Limit: compressed species need n_cell <= 32 (n_cell^3 <= 32768;
 * PM_ERR_SHAPE beyond); float species and the meshes are not limited. Calls that
 * overlap on one device (any context) share the array and race: order them on one
 * stream or synchronise between them. */
pm_status pm_reduce_noalloc(pm_ctx ctx, const pm_species* sp, int n_sp, const float* rho,
                            const float* acc, double* out);

/* Byte stream of one compressed species (Sec. 2.4 layout): a 64-byte header
 * {"PMC1", version 1, species_id, brick, N, n_cell, v_max, widths, mass, checksum,
 * body length}, then for every cell its count byte (255 + uint32 count when >= 255)
 * followed by its particles' records: 3 P position bytes (x, y, z) then 3 V velocity
 * bytes (vx, vy, vz), multi-byte codes little-endian; with the paper's widths (header
 * word 0) a record is 9 bytes (x, y, z bytes; vx, vy, vz uint16). The widths word is
 * P | V << 8 otherwise. The checksum is sum_i (2 i + 1) b_i mod 2^64 over the body
 * bytes. buf: device uint8 [cap]; used: device int64 (bytes written). */
pm_status pm_pack(pm_ctx ctx, const pm_species* sp, int32_t species_id, uint8_t* buf,
                  int64_t cap, int64_t* used);
/* Exact stream length of a compressed species (host value; synchronises). */
pm_status pm_pack_size(pm_ctx ctx, const pm_species* sp, int64_t* bytes);

/* Parse and verify a byte stream held in HOST memory into a compressed species
 * (synchronous). Checks magic, version, brick and n_cell against the context, the code
 * widths against out->widths (PM_ERR_ARG when they differ, PM_ERR_CORRUPT when the word
 * is not a valid one), body length, checksum, and that the counts sum to N == out->n;
 * returns PM_ERR_CORRUPT otherwise. The species mass and id from the header are returned via the pointers
 * (nullable). */
pm_status pm_unpack(pm_ctx ctx, const uint8_t* host_buf, int64_t len, pm_species* out,
                    double* mass, int32_t* species_id);

/* Per-stage timing with HIP events recorded on the context's stream around each
 * kernel group. pm_profile(ctx, 1) clears the totals and starts recording, 0 stops.
 * pm_profile_read synchronises and returns, for stage ids 0..cap-1, the summed
 * milliseconds and the number of timed launches:
 *   0 cell offsets   1 deposit          2 FFT x r2c     3 FFT y forward
 *   4 FFT z sweeps   5 FFT y inverse    6 FFT x c2r     7 interpolate-kick-drift
 *   8 re-sort        9 encode/decode   10 adjoint scatter/gather   11 PP force
 *  12 force interpolation without the kick (pm_interp_accel, the long range of
 *     pm_step_p3m)   13 force components from the potential (difference stencil) */
pm_status pm_profile(pm_ctx ctx, int enable);
pm_status pm_profile_read(pm_ctx ctx, double* ms, int64_t* launches, int cap);

/* Diagnostics: copy the float32 kernel table L G(|n|^2)/n_mesh^3 (device float
 * [3 (n_mesh/2)^2 + 1], indexed by the integer |n|^2), with the split factor of the
 * context's kernel part (the long part's window division, which is not a function of
 * |n|^2, is applied in the force only). */
pm_status pm_kernel_table(pm_ctx ctx, float* out, int64_t cap);

#ifdef __cplusplus
}
#endif

#endif /* PM_H */

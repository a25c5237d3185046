// CIC force interpolation (Fig. 2 "inverse_force_interpolation"), kick and drift, fused
// with the re-encode of compressed particles and the stable re-sort of the stream into
// cell order (Sec. 2.4: particles are written cell by cell).
//
// Compressed path, per species:
//   k_vmax_next     v_max' = smallest power of two >= V + |c_k| A_max (V: largest
//                   decoded |v| of the input, from its extreme velocity codes; A_max:
//                   largest |a| on the mesh). Interpolation is a convex combination of
//                   mesh values, so no kicked component exceeds the bound.
//   k_kick_pair     two bricks adjacent along x per workgroup (R = 16 nodes per brick
//   k_kick_brick    side), or one brick of any shape: the force nodes staged in LDS,
//                   then waves take 64-particle chunks independently (no barrier):
//                   decode, gather a from the 8 CIC nodes, v' = v + c_k a, fixed-point
//                   drift u' = u + floor(v' c_d S + 1/2), new codes, and the digit: the
//                   new cell inside the brick, or B^3 for a particle that leaves it (a
//                   "mover", whose new cell key is kept). Stayers are counted per new
//                   cell and movers per brick with LDS atomics.
//   movers          compacted in old order (ballots over the digits, one wave per
//                   brick), stably radix-sorted by new cell.
//   k_arrivals      per new cell: arrivals, and how many of them come from earlier
//                   bricks (they precede the cell's stayers in stream order);
//   k_brick_arrivals  per brick, its run of the sorted movers (its arrivals).
//   scan            new cell offsets.
//   k_place_stayers stayers and arrivals written at their final stream positions, per
//                   brick by one wave: the stayers' first position in each new cell
//                   staged in LDS and their stable rank from a multi-split of the
//                   digits, then the brick's arrivals, so that one wave writes all of the
//                   brick's output range.
#include <type_traits>

#include "pm_codec.h"
#include "pm_scan.h"

namespace {

constexpr int KT = 256;  // threads per workgroup

// ------------------------------------------------------------ float layout --
__global__ __launch_bounds__(KT) void k_kick_float(const float* x, const float* v, float* xo,
                                                  float* vo, int64_t n, const float* acc,
                                                  int64_t ng, float ngL, float box, float ck,
                                                  float cd) {
  int64_t p = (int64_t)blockIdx.x * KT + threadIdx.x;
  if (p >= n) return;
  const int64_t n3 = ng * ng * ng;
  int64_t i[3];
  float f[3], xv[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    xv[a] = x[3 * p + a];
    float u = xv[a] * ngL;  // mesh units (exact for a power-of-two box)
    float fl = floorf(u);
    f[a] = u - fl;
    int64_t k = (int64_t)fl % ng;
    i[a] = k < 0 ? k + ng : k;
  }
  float ax = 0.f, ay = 0.f, az = 0.f;
#pragma unroll
  for (int dz = 0; dz < 2; ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) {
        float w = (dx ? f[0] : 1.f - f[0]) * (dy ? f[1] : 1.f - f[1]) * (dz ? f[2] : 1.f - f[2]);
        int64_t node = (((i[2] + dz) % ng) * ng + (i[1] + dy) % ng) * ng + (i[0] + dx) % ng;
        ax += w * acc[node];
        ay += w * acc[n3 + node];
        az += w * acc[2 * n3 + node];
      }
  const float a3[3] = {ax, ay, az};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float v1 = v[3 * p + a] + ck * a3[a];
    float x1 = xv[a] + cd * v1;
    x1 -= box * floorf(x1 / box);  // periodic wrap into [0, L)
    if (x1 >= box || x1 < 0.f) x1 = 0.f;
    vo[3 * p + a] = v1;
    xo[3 * p + a] = x1;
  }
}

// ------------------------------------------------------- compressed layout --
template <int VB = 2>  // velocity bytes per axis
__global__ void k_vmax_next(const pm_shdr* hin, pm_shdr* hout, const float* amax, double ck,
                            int64_t n) {
  double V = 0.0;
  if (n > 0 && hin->j_max >= 0) {
    double a = fabs((double)vel_decode_v<VB>((uint32_t)hin->j_min, hin->v_max));
    double b = fabs((double)vel_decode_v<VB>((uint32_t)hin->j_max, hin->v_max));
    V = a > b ? a : b;
  }
  double bound = V + fabs(ck) * (double)(*amax);
  float vm = 0.f;
  if (bound > 0.0) {
    int e;
    double m = frexp(bound, &e);
    vm = (float)(m == 0.5 ? bound : ldexp(1.0, e));
  }
  hout->v_max = vm;
  hout->j_min = 65536;
  hout->j_max = -1;
  hout->flags = 0;
  hout->n_esc = 0;
  hout->reserved = 0;
}

constexpr int KB = 512;  // threads per workgroup of the brick kicks
constexpr int NWK = KB / 64;
constexpr int MAXSP = 4;

struct KickSpecies {
  int64_t n;
  const void* pos;     // position codes, P bytes per axis
  const void* vel;     // velocity codes, V bytes per axis
  const pm_shdr* hin;
  pm_shdr* hout;
  const int64_t* off;  // input cell offsets [ncell3 + 1]
  void* tpos;          // new codes, old stream order
  void* tvel;
  uint16_t* tdig;      // new local cell in the brick, or B^3 for movers
  uint32_t* mkey;      // movers: new cell key, at the old stream index
  uint64_t* cnt;       // per cell: stayers (low 32 bits)
  uint32_t* mcnt;      // movers per brick
  int32_t* pmn;        // per-brick extreme new velocity codes, folded into hout
  int32_t* pmx;
  const float* app;    // nullable: per-particle acceleration added to the mesh force
};
struct KickArgs {
  KickSpecies sp[MAXSP];
  int n_sp;
  const float* acc;  // [3][ng^3]
  float ck;
  double cdS;        // c_d S / L (position codes per unit velocity)
};

// Codec constants of one species (uniform), V velocity bytes per axis (half range
// H = 2^(8V - 1)): wd = v_max / H, ce = H / v_max' (v_max' a power of two: exponent
// field of 2^(8V - 1 - e) is 253 + 8V minus that of v_max').
struct Codec {
  float vmi, vmo, wd, ce;
};
template <int V>
__device__ inline Codec codec_of(const KickSpecies& S) {
  Codec k;
  k.vmi = S.hin->v_max;
  k.vmo = S.hout->v_max;
  k.wd = k.vmi * (V == 2 ? 0x1p-15f : 0x1p-7f);
  k.ce = __uint_as_float(((253u + 8u * V) - (__float_as_uint(k.vmo) >> 23)) << 23);
  return k;
}
// float32 codec forms valid for every species (see vel_code_p2, vel_decode_w)
__device__ inline bool codec_fast(const KickArgs& A) {
  bool fast = true;
  for (int s = 0; s < A.n_sp; ++s) {
    const float vi = A.sp[s].hin->v_max, vo = A.sp[s].hout->v_max;
    fast = fast && vi >= 0x1p-90f && vi <= 0x1p90f && vo >= 0x1p-90f && vo <= 0x1p90f &&
           (__float_as_uint(vo) & 0x7fffffu) == 0;
  }
  return fast;
}

// One lane kicks particle j of one species in one brick (jr: its index from the
// brick's first particle of that species): decode, gather a through `gather(li, f)`
// (node index inside the brick, CIC fractions), kick, fixed-point drift, new codes.
// Writes the new codes and the particle's digit (new local cell, or B^3 when it leaves
// the brick; movers also get their new cell key), counts stayers per new cell and movers
// in LDS, and folds the new velocity codes into the lane's running extremes jmn, jmx
// (reduced over the wave once per kernel, by VelExt). No barrier: waves are
// independent, and the lanes of a wave may take particles of different bricks. The cell
// search range [lo0, hi0) spans a power-of-two number of cells.
// P position bytes and V velocity bytes per axis (P = 1, V = 2: the paper's format).
template <bool FAST, int P, int V, typename Gather>
__device__ inline void kick_lane(const KickSpecies& S, const KickArgs& A, const Geom& g,
                                 const Codec& cd, int64_t j, uint32_t jr, const uint32_t* rel,
                                 int lo0, int hi0, const uint32_t bc[3], uint32_t* run,
                                 uint32_t* mvc, int& jmn, int& jmx, bool& bad, Gather gather) {
  using PC = typename PosCode<P>::T;
  using VC = typename VelCode<V>::T;
  constexpr int SH = 8 * P, FB = 8 * P + 1;  // offset bits, fractional bits of a mesh cell
  constexpr uint32_t FMASK = (1u << FB) - 1u, OMASK = (1u << SH) - 1u;
  constexpr float UNIT = 1.0f / (float)(1u << FB);
  const int B3 = g.B * g.B * g.B;
  const uint32_t mB = (uint32_t)g.B - 1;
  {
    const PC* pp = (const PC*)S.pos + 3 * j;
    const VC* vp = (const VC*)S.vel + 3 * j;
    uint32_t pb[3], vc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      pb[a] = pp[a];
      vc[a] = vp[a];
    }
    int lo = lo0;  // local cell: largest l in [lo0, hi0) with rel[l] <= jr
    for (int st = (hi0 - lo0) >> 1; st > 0; st >>= 1) lo += rel[lo + st] <= jr ? st : 0;
    const uint32_t lc[3] = {(uint32_t)lo & mB, ((uint32_t)lo >> g.lgB) & mB,
                            (uint32_t)lo >> (2 * g.lgB)};
    int li[3];
    float f[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      // position in 2^-FB mesh cells (1/512 for P = 1) from the brick's corner node
      const uint32_t gl = (2 * ((lc[a] << SH) | pb[a]) + 1) * (uint32_t)g.r;
      li[a] = (int)(gl >> FB);
      f[a] = (float)(gl & FMASK) * UNIT;
    }
    float acc3[3];
    gather(li, f, acc3);
    if (S.app) {
#pragma unroll
      for (int a = 0; a < 3; ++a) acc3[a] += S.app[3 * j + a];
    }
    const int64_t SP = g.S << (8 * (P - 1));  // position steps per box side
    const uint32_t Sm = (uint32_t)SP - 1;
    const double Sd = (double)SP, invS = 1.0 / Sd;  // powers of two
    PC* tp = (PC*)S.tpos + 3 * j;
    VC* tv = (VC*)S.tvel + 3 * j;
    uint32_t un[3], nl[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float v0 = FAST ? vel_decode_w_v<V>(vc[a], cd.wd) : vel_decode_v<V>(vc[a], cd.vmi);
      const float v1 = v0 + A.ck * acc3[a];
      const double d = floor((double)v1 * A.cdS + 0.5);
      const bool okd = fabs(d) < 4.0e15;
      bad |= !okd;
      // d mod S, exact in float64 (d is an integer below 2^52, S a power of two)
      const double dm = okd ? d - Sd * floor(d * invS) : 0.0;
      un[a] = ((((bc[a] + lc[a]) << SH) | pb[a]) + (uint32_t)dm) & Sm;
      nl[a] = (un[a] >> SH) - bc[a];  // new local cell (wraps above B when outside)
      const int jv = FAST ? vel_code_p2_v<V>(v1, cd.ce) : vel_code_v<V>(v1, cd.vmo);
      tp[a] = (PC)(un[a] & OMASK);
      tv[a] = (VC)jv;
      jmn = min(jmn, jv);
      jmx = max(jmx, jv);
    }
    if (nl[0] <= mB && nl[1] <= mB && nl[2] <= mB) {
      const uint32_t digit = (((nl[2] << g.lgB) | nl[1]) << g.lgB) | nl[0];
      S.tdig[j] = (uint16_t)digit;
      atomicAdd(&run[digit], 1u);
    } else {
      S.tdig[j] = (uint16_t)B3;
      S.mkey[j] = cell_key(g, un[0] >> SH, un[1] >> SH, un[2] >> SH);
      atomicAdd(mvc, 1u);
    }
  }
}

// A workgroup-uniform 64-bit value read from LDS, moved to scalar registers.
__device__ inline int64_t uniform64(int64_t v) {
  const uint64_t u = (uint64_t)v;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Each lane's extreme new velocity codes per species over all the chunks it kicked
// (statically indexed, so they stay in registers), reduced over the wave and folded into
// the workgroup's smm[2 s], smm[2 s + 1] once at the end.
struct VelExt {
  int mn[MAXSP], mx[MAXSP];
  __device__ VelExt() {
#pragma unroll
    for (int t = 0; t < MAXSP; ++t) {
      mn[t] = 65536;
      mx[t] = -1;
    }
  }
  __device__ void fold(int s, int a, int b) {
#pragma unroll
    for (int t = 0; t < MAXSP; ++t)
      if (t == s) {
        mn[t] = min(mn[t], a);
        mx[t] = max(mx[t], b);
      }
  }
  __device__ void flush(int n_sp, int* smm) const {
#pragma unroll
    for (int t = 0; t < MAXSP; ++t) {
      if (t >= n_sp) break;
      int a = mn[t], b = mx[t];
      for (int d = 32; d >= 1; d >>= 1) {
        a = min(a, __shfl_xor(a, d, 64));
        b = max(b, __shfl_xor(b, d, 64));
      }
      if ((threadIdx.x & 63) == 0 && b >= 0) {
        atomicMin(&smm[2 * t], a);
        atomicMax(&smm[2 * t + 1], b);
      }
    }
  }
};

// Chunks of 64 particles over a list of segments (one species' particles in one brick,
// or in one z half of it), dealt to the waves of the workgroup in turn. seg(i) gives
// segment i's (species, brick slot, stream range, local cell search range).
struct Seg {
  int s, k;
  int64_t j0, j1;
  int lo, hi;
};

// ---- one brick per workgroup (any shape; R = B r nodes per side) ----
// With STAGE the brick's force nodes [b R, b R + R]^3 are copied to LDS first and every
// particle gathers its 8 CIC nodes from there.
// RS: staged tile side in nodes (compile time), or 0: gather from HBM; P, V: code widths
template <int RS, int P = 1, int V = 2>
__global__ __launch_bounds__(KB) void k_kick_brick(KickArgs A, Geom g, DevErr* err) {
  constexpr bool STAGE = RS > 0;
  const int B = g.B, B3 = B * B * B, L = B3 + 1;
  constexpr int R1 = RS + 1;
  extern __shared__ unsigned char smem[];
  float* F = (float*)smem;  // [3][R1^3] when STAGE
  const int fsz = STAGE ? 3 * R1 * R1 * R1 : 0;
  uint32_t* rel = (uint32_t*)(smem + fsz * 4);  // [MAXSP][L]
  uint32_t* run = rel + MAXSP * L;              // [MAXSP][L]
  __shared__ int64_t l0s[MAXSP];
  __shared__ uint32_t mvc[MAXSP];
  __shared__ int smm[2 * MAXSP];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t b = xcd_tile(blockIdx.x, g.nbrick);
  const uint32_t kbase = (uint32_t)(b * B3);
  const int64_t ng = g.ng, n3 = ng * ng * ng;
  uint32_t bc[3];
  key_cell(g, kbase, bc[0], bc[1], bc[2]);
  const int64_t ox = (int64_t)bc[0] * g.r, oy = (int64_t)bc[1] * g.r, oz = (int64_t)bc[2] * g.r;
  const int n_sp = A.n_sp;
  for (int i = threadIdx.x; i < n_sp * L; i += KB) {
    const int s = i / L, l = i - s * L;
    const int64_t v0 = A.sp[s].off[kbase];
    rel[i] = (uint32_t)(A.sp[s].off[kbase + l] - v0);
    run[i] = 0;
    if (l == 0) l0s[s] = v0;
  }
  if (threadIdx.x < MAXSP) mvc[threadIdx.x] = 0;
  if (threadIdx.x < 2 * MAXSP) smm[threadIdx.x] = (threadIdx.x & 1) ? -1 : 65536;
  if constexpr (STAGE) {
    // rows of RS nodes (x) as float4 loads, then the x = RS halo column; node (lz, ly)
    // of component c is row (c R1 + lz) R1 + ly. Rows past the end repeat the last row
    // (a duplicate load, not stored), so no load sits behind a branch.
    static_assert(RS % 4 == 0, "staged tile side must be a multiple of 4");
    constexpr int Q = RS / 4;
    constexpr int ROWS = 3 * R1 * R1;
    constexpr int NQ = ROWS * Q;
    constexpr int PQ = (NQ + KB - 1) / KB;
    constexpr int PH = (ROWS + KB - 1) / KB;
    constexpr int RR = R1 * R1;
    constexpr int DR = KB / Q;
    constexpr int DC = DR / RR, DLZ = (DR % RR) / R1, DLY = DR % R1;
    static_assert(KB % Q == 0, "a workgroup covers whole rows");
    const uint32_t mu = (uint32_t)(ng - 1), ngu = (uint32_t)ng;
    const uint32_t oxq = (uint32_t)ox + 4 * (threadIdx.x % Q);
    const uint32_t hx = ((uint32_t)ox + RS) & mu;
    const float* pc0 = A.acc;
    const float* pc1 = A.acc + n3;
    const float* pc2 = A.acc + 2 * n3;
    const int row0 = threadIdx.x / Q;
    float4 vq[PQ];
    float vh[PH];
    {
      int c = row0 / RR, lz = (row0 % RR) / R1, ly = row0 % R1;
#pragma unroll
      for (int k = 0; k < PQ; ++k) {
        const bool over = c >= 3;
        const int cc = over ? 2 : c, zz = over ? R1 - 1 : lz, yy = over ? R1 - 1 : ly;
        const float* pc = cc == 0 ? pc0 : (cc == 1 ? pc1 : pc2);
        const uint32_t gz = ((uint32_t)oz + zz) & mu, gy = ((uint32_t)oy + yy) & mu;
        vq[k] = *(const float4*)(pc + ((uint64_t)(gz * ngu + gy) * ngu + oxq));
        ly += DLY;
        lz += DLZ;
        c += DC;
        if (ly >= R1) { ly -= R1; ++lz; }
        if (lz >= R1) { lz -= R1; ++c; }
      }
    }
#pragma unroll
    for (int k = 0; k < PH; ++k) {
      const int row = min((int)threadIdx.x + k * KB, ROWS - 1);
      const int c = row / RR, rem = row - c * RR;
      const int lz = rem / R1, ly = rem - lz * R1;
      const float* pc = c == 0 ? pc0 : (c == 1 ? pc1 : pc2);
      const uint32_t gz = ((uint32_t)oz + lz) & mu, gy = ((uint32_t)oy + ly) & mu;
      vh[k] = pc[(uint64_t)(gz * ngu + gy) * ngu + hx];
    }
    {
      int c = row0 / RR, lz = (row0 % RR) / R1, ly = row0 % R1;
      const int q4 = 4 * (threadIdx.x % Q);
#pragma unroll
      for (int k = 0; k < PQ; ++k) {
        if (c < 3) {
          float* d = F + ((c * R1 + lz) * R1 + ly) * R1 + q4;
          d[0] = vq[k].x;
          d[1] = vq[k].y;
          d[2] = vq[k].z;
          d[3] = vq[k].w;
        }
        ly += DLY;
        lz += DLZ;
        c += DC;
        if (ly >= R1) { ly -= R1; ++lz; }
        if (lz >= R1) { lz -= R1; ++c; }
      }
    }
#pragma unroll
    for (int k = 0; k < PH; ++k) {
      const int row = threadIdx.x + k * KB;
      if (row < ROWS) F[row * R1 + RS] = vh[k];
    }
  }
  __syncthreads();

  auto gather = [&](const int li[3], const float f[3], float acc3[3]) {
    acc3[0] = acc3[1] = acc3[2] = 0.f;
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
      for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
          const float wgt = (dx ? f[0] : 1.f - f[0]) * (dy ? f[1] : 1.f - f[1]) *
                            (dz ? f[2] : 1.f - f[2]);
          if constexpr (STAGE) {
            const int node = ((li[2] + dz) * R1 + (li[1] + dy)) * R1 + (li[0] + dx);
            acc3[0] += wgt * F[node];
            acc3[1] += wgt * F[R1 * R1 * R1 + node];
            acc3[2] += wgt * F[2 * R1 * R1 * R1 + node];
          } else {
            const int64_t m = ng - 1;
            const int64_t nz = (oz + li[2] + dz) & m, ny = (oy + li[1] + dy) & m,
                          nx = (ox + li[0] + dx) & m;
            const int64_t node = (nz * ng + ny) * ng + nx;
            acc3[0] += wgt * A.acc[node];
            acc3[1] += wgt * A.acc[n3 + node];
            acc3[2] += wgt * A.acc[2 * n3 + node];
          }
        }
  };
  bool bad = false;
  VelExt ext;
  auto run_all = [&](auto fast_tag) {
    constexpr bool FAST = decltype(fast_tag)::value;
    int64_t cbase = 0;  // chunks of the earlier species
    for (int s = 0; s < n_sp; ++s) {
      const KickSpecies& S = A.sp[s];
      const int64_t l0 = l0s[s];
      const int64_t j0 = min(l0, S.n), j1 = min(l0 + (int64_t)rel[s * L + B3], S.n);
      const int64_t nch = j1 > j0 ? (j1 - j0 + 63) >> 6 : 0;
      const Codec cd = codec_of<V>(S);
      // this wave's chunks of species s: global chunk index = cbase + c, dealt round-robin
      int64_t c = ((int64_t)w - cbase) % NWK;
      if (c < 0) c += NWK;
      int jmn = 65536, jmx = -1;
      for (; c < nch; c += NWK) {
        const int64_t j = j0 + 64 * c + (threadIdx.x & 63);
        if (j < j1)
          kick_lane<FAST, P, V>(S, A, g, cd, j, (uint32_t)(j - l0), rel + s * L, 0, B3, bc,
                                run + s * L, &mvc[s], jmn, jmx, bad, gather);
      }
      ext.fold(s, jmn, jmx);
      cbase += nch;
    }
  };
  if (codec_fast(A)) run_all(std::true_type{});
  else run_all(std::false_type{});
  ext.flush(n_sp, smm);
  __syncthreads();
  for (int i = threadIdx.x; i < n_sp * L; i += KB) {
    const int s = i / L, l = i - s * L;
    if (l < B3) A.sp[s].cnt[kbase + l] = (uint64_t)run[i];
  }
  if ((int)threadIdx.x < n_sp) {
    const int s = threadIdx.x;
    A.sp[s].mcnt[b] = mvc[s];
    A.sp[s].pmn[b] = smm[2 * s];
    A.sp[s].pmx[b] = smm[2 * s + 1];
  }
  if (bad) latch_error(err, ERRBIT_RANGE);
}

// ---- two bricks adjacent along x per workgroup, R = 16, in NZ passes over z ----
// Pass h stages the force nodes x in [x0, x0 + 2R], y in [y0, y0 + R], z in
// [z0 + h R/NZ, z0 + (h + 1) R/NZ] (33 x 17 x 5 nodes for NZ = 4) and kicks the
// particles of both bricks' cells in that z slice (whole cell layers). Consecutive
// passes share a node layer, which stays in LDS: the layers form a ring, and passes
// after the first stage only their R/NZ new layers. Rows of the staged tile are 2R
// nodes long, which the memory system serves much faster than rows of R; with NZ = 4
// and 256 threads the tile is 34 KB and four workgroups share a CU, each staging while
// the others compute.
constexpr int PR = 16;
template <int NT, int NZ, int P = 1, int V = 2>  // threads per workgroup, z passes, widths
__global__ __launch_bounds__(NT, 4) void k_kick_pair(KickArgs A, Geom g, DevErr* err) {
  constexpr int KB = NT, NWK = NT / 64;
  constexpr int X1 = 2 * PR + 1, Y1 = PR + 1, Z1 = PR / NZ + 1;
  constexpr int TS = X1 * Y1 * Z1;  // nodes per component
  const int B = g.B, B3 = B * B * B, L = B3 + 1, H = B3 / NZ;  // H: cells per z pass
  extern __shared__ unsigned char smem[];
  float* F = (float*)smem;                          // [3][Z1][Y1][X1]
  uint32_t* rel = (uint32_t*)(smem + 3 * TS * 4);   // [2][MAXSP][L]
  uint32_t* run = rel + 2 * MAXSP * L;              // [2][MAXSP][L]
  __shared__ int64_t l0s[2 * MAXSP];
  __shared__ uint32_t mvc[2 * MAXSP];
  __shared__ int smm[2 * MAXSP];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t p = xcd_tile(blockIdx.x, g.nbrick / 2);
  const int64_t b0 = 2 * p;  // bricks b0, b0 + 1 (x index even, same row)
  const uint32_t kb0 = (uint32_t)(b0 * B3);
  const int64_t ng = g.ng, n3 = ng * ng * ng;
  uint32_t bc0[3];
  key_cell(g, kb0, bc0[0], bc0[1], bc0[2]);
  const int64_t ox = (int64_t)bc0[0] * g.r, oy = (int64_t)bc0[1] * g.r,
                oz = (int64_t)bc0[2] * g.r;
  const int n_sp = A.n_sp;
  for (int i = threadIdx.x; i < 2 * MAXSP * L; i += KB) {
    const int k = i / (MAXSP * L), rem = i - k * (MAXSP * L);
    const int s = rem / L, l = rem - s * L;
    uint32_t v = 0;
    if (s < n_sp) {
      const int64_t v0 = A.sp[s].off[kb0 + k * B3];
      v = (uint32_t)(A.sp[s].off[kb0 + k * B3 + l] - v0);
      if (l == 0) l0s[k * MAXSP + s] = v0;
    }
    rel[i] = v;
    run[i] = 0;
  }
  if (threadIdx.x < 2 * MAXSP) {
    mvc[threadIdx.x] = 0;
    smm[threadIdx.x] = (threadIdx.x & 1) ? -1 : 65536;
  }
  const bool fast = codec_fast(A);
  bool bad = false;
  VelExt ext;

  // The z passes share their boundary layer: pass h needs node layers 4h..4h+4 (for
  // PR / NZ = 4), pass h + 1 starts at 4h + 4. F holds the Z1 layers as a ring, layer
  // 4h + lz in slot (4h + lz) mod Z1, so that pass 0 stages Z1 layers and every later
  // pass only the Z1 - 1 new ones.
  auto stage = [&](int h, auto nl_tag) {
    constexpr int NL = decltype(nl_tag)::value;  // layers loaded: Z1, or Z1 - 1
    constexpr int LZ0 = Z1 - NL;                  // first local layer loaded
    constexpr int Q = 2 * PR / 4;
    constexpr int ROWS = 3 * NL * Y1;
    constexpr int NQ = ROWS * Q;
    constexpr int PQ = (NQ + KB - 1) / KB;
    constexpr int PH = (ROWS + KB - 1) / KB;
    constexpr int RR = NL * Y1;
    constexpr int DR = KB / Q;
    constexpr int DC = DR / RR, DLZ = (DR % RR) / Y1, DLY = DR % Y1;
    static_assert(KB % Q == 0, "a workgroup covers whole rows");
    const uint32_t mu = (uint32_t)(ng - 1), ngu = (uint32_t)ng;
    const uint32_t oz2 = (uint32_t)oz + h * (PR / NZ) + LZ0;
    const int hb = (h * (PR / NZ) + LZ0) % Z1;  // slot of the first loaded layer
    const uint32_t oxq = (uint32_t)ox + 4 * (threadIdx.x % Q);
    const uint32_t hx = ((uint32_t)ox + 2 * PR) & mu;
    const float* pc0 = A.acc;
    const float* pc1 = A.acc + n3;
    const float* pc2 = A.acc + 2 * n3;
    const int row0 = threadIdx.x / Q;
    float4 vq[PQ];
    float vh[PH];
    {
      int c = row0 / RR, lz = (row0 % RR) / Y1, ly = row0 % Y1;
#pragma unroll
      for (int k = 0; k < PQ; ++k) {
        const bool over = c >= 3;
        const int cc = over ? 2 : c, zz = over ? NL - 1 : lz, yy = over ? Y1 - 1 : ly;
        const float* pc = cc == 0 ? pc0 : (cc == 1 ? pc1 : pc2);
        const uint32_t gz = (oz2 + zz) & mu, gy = ((uint32_t)oy + yy) & mu;
        vq[k] = *(const float4*)(pc + ((uint64_t)(gz * ngu + gy) * ngu + oxq));
        ly += DLY;
        lz += DLZ;
        c += DC;
        if (ly >= Y1) { ly -= Y1; ++lz; }
        if (lz >= NL) { lz -= NL; ++c; }
      }
    }
#pragma unroll
    for (int k = 0; k < PH; ++k) {
      const int row = min((int)threadIdx.x + k * KB, ROWS - 1);
      const int c = row / RR, rem = row - c * RR;
      const int lz = rem / Y1, ly = rem - lz * Y1;
      const float* pc = c == 0 ? pc0 : (c == 1 ? pc1 : pc2);
      const uint32_t gz = (oz2 + lz) & mu, gy = ((uint32_t)oy + ly) & mu;
      vh[k] = pc[(uint64_t)(gz * ngu + gy) * ngu + hx];
    }
    __syncthreads();  // the previous pass is done with the slots rewritten here
    {
      int c = row0 / RR, lz = (row0 % RR) / Y1, ly = row0 % Y1;
      const int q4 = 4 * (threadIdx.x % Q);
#pragma unroll
      for (int k = 0; k < PQ; ++k) {
        if (c < 3) {
          int sl = hb + lz;
          sl -= sl >= Z1 ? Z1 : 0;
          float* d = F + ((c * Z1 + sl) * Y1 + ly) * X1 + q4;
          d[0] = vq[k].x;
          d[1] = vq[k].y;
          d[2] = vq[k].z;
          d[3] = vq[k].w;
        }
        ly += DLY;
        lz += DLZ;
        c += DC;
        if (ly >= Y1) { ly -= Y1; ++lz; }
        if (lz >= NL) { lz -= NL; ++c; }
      }
    }
#pragma unroll
    for (int k = 0; k < PH; ++k) {
      const int row = threadIdx.x + k * KB;
      if (row < ROWS) {
        const int c = row / RR, rem = row - c * RR;
        const int lz = rem / Y1, ly = rem - lz * Y1;
        int sl = hb + lz;
        sl -= sl >= Z1 ? Z1 : 0;
        F[((c * Z1 + sl) * Y1 + ly) * X1 + 2 * PR] = vh[k];
      }
    }
    __syncthreads();
  };

  // A pass deals 64-particle chunks over each species' particles of the z slice, brick
  // b0's then brick b0 + 1's (the two ranges are apart in the stream), so that a lane's
  // brick k is its own: a species with few particles per slice (16 CDM particles per
  // brick at one per cell) fills one chunk instead of two part-empty ones.
  auto pass = [&](auto fast_tag, int h) {
    constexpr bool FAST = decltype(fast_tag)::value;
    int64_t cbase = 0;  // chunks of the earlier species of this pass
    const int lane = threadIdx.x & 63;
    {
      int k = 0;  // this lane's brick, set per chunk
      auto gather = [&](const int li[3], const float f[3], float acc3[3]) {
        const int tx = li[0] + k * PR, ty = li[1];
        // ring slots of the node layers tz and tz + 1 (local to this pass)
        int z0 = li[2] - h * (PR / NZ) + (h * (PR / NZ)) % Z1;
        z0 -= z0 >= Z1 ? Z1 : 0;
        const int z1 = z0 + 1 == Z1 ? 0 : z0 + 1;
        acc3[0] = acc3[1] = acc3[2] = 0.f;
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
          for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
              const float wgt = (dx ? f[0] : 1.f - f[0]) * (dy ? f[1] : 1.f - f[1]) *
                                (dz ? f[2] : 1.f - f[2]);
              const int node = ((dz ? z1 : z0) * Y1 + (ty + dy)) * X1 + (tx + dx);
              acc3[0] += wgt * F[node];
              acc3[1] += wgt * F[TS + node];
              acc3[2] += wgt * F[2 * TS + node];
            }
      };
      for (int s = 0; s < n_sp; ++s) {
        const KickSpecies& S = A.sp[s];
        int64_t l0[2], j0[2], nk[2];  // per brick: first particle, slice start, slice size
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
          const uint32_t* rs = rel + (kk * MAXSP + s) * L;
          l0[kk] = uniform64(l0s[kk * MAXSP + s]);
          j0[kk] = min(l0[kk] + (int64_t)__builtin_amdgcn_readfirstlane(rs[h * H]), S.n);
          const int64_t j1 =
              min(l0[kk] + (int64_t)__builtin_amdgcn_readfirstlane(rs[(h + 1) * H]), S.n);
          nk[kk] = j1 > j0[kk] ? j1 - j0[kk] : 0;
        }
        const int64_t nt = nk[0] + nk[1];
        const int64_t nch = (nt + 63) >> 6;
        const Codec cd = codec_of<V>(S);
        int64_t c = ((int64_t)w - cbase) % NWK;
        if (c < 0) c += NWK;
        int jmn = 65536, jmx = -1;
        for (; c < nch; c += NWK) {
          const int64_t q = 64 * c + lane;  // position in the two slices, one after the other
          if (q < nt) {
            k = q >= nk[0];
            const int64_t j = k ? j0[1] + (q - nk[0]) : j0[0] + q;
            // brick b0 + 1 is brick b0's neighbour along x (b0 even)
            const uint32_t bc[3] = {bc0[0] + (uint32_t)(k * B), bc0[1], bc0[2]};
            const int sl = k * MAXSP + s;
            kick_lane<FAST, P, V>(S, A, g, cd, j, (uint32_t)(j - (k ? l0[1] : l0[0])),
                                  rel + sl * L, h * H, (h + 1) * H, bc, run + sl * L, &mvc[sl],
                                  jmn, jmx, bad, gather);
          }
        }
        ext.fold(s, jmn, jmx);
        cbase += nch;
      }
    }
  };
  stage(0, std::integral_constant<int, Z1>{});
  if (fast) pass(std::true_type{}, 0);
  else pass(std::false_type{}, 0);
#pragma nounroll
  for (int h = 1; h < NZ; ++h) {
    stage(h, std::integral_constant<int, Z1 - 1>{});
    if (fast) pass(std::true_type{}, h);
    else pass(std::false_type{}, h);
  }
  ext.flush(n_sp, smm);
  __syncthreads();
  for (int i = threadIdx.x; i < 2 * MAXSP * L; i += KB) {
    const int k = i / (MAXSP * L), rem = i - k * (MAXSP * L);
    const int s = rem / L, l = rem - s * L;
    if (s < n_sp && l < B3) A.sp[s].cnt[kb0 + k * B3 + l] = (uint64_t)run[i];
  }
  if ((int)threadIdx.x < 2 * n_sp) {
    const int k = threadIdx.x / n_sp, s = threadIdx.x - k * n_sp;
    A.sp[s].mcnt[b0 + k] = mvc[k * MAXSP + s];
    A.sp[s].pmn[b0 + k] = smm[2 * s];
    A.sp[s].pmx[b0 + k] = smm[2 * s + 1];
  }
  if (bad) latch_error(err, ERRBIT_RANGE);
}

__device__ inline int64_t lower_bound_u32(const uint32_t* a, int64_t lo, int64_t hi, uint32_t v) {
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (a[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// astart[b] = first sorted mover whose new cell lies in brick b or later, b in [0, nbrick]:
// the arrivals of brick b are the sorted movers [astart[b], astart[b + 1]).
// The mover count nm is read on the device (*nmd): the host never waits for it.
__global__ __launch_bounds__(KT) void k_brick_arrivals(const uint32_t* skey, const int64_t* nmd,
                                                      int B3, int64_t nbrick, int64_t* astart) {
  const int64_t b = (int64_t)blockIdx.x * KT + threadIdx.x;
  if (b > nbrick) return;
  astart[b] = lower_bound_u32(skey, 0, *nmd, (uint32_t)(b * B3));
}

// per group of sorted movers with the same new cell: add arrivals (low 32 bits) and
// arrivals from earlier bricks (high 32 bits) to the cell's count. A fixed grid strides
// over the nm sorted movers.
__global__ __launch_bounds__(KT) void k_arrivals(const uint32_t* skey, const uint32_t* sidx,
                                                const int64_t* nmd, const int64_t* off_in,
                                                int B3, uint64_t* cnt) {
  const int64_t nm = *nmd;
  for (int64_t s = (int64_t)blockIdx.x * KT + threadIdx.x; s < nm;
       s += (int64_t)gridDim.x * KT) {
    const uint32_t k = skey[s];
    if (s > 0 && skey[s - 1] == k) continue;  // group leader only
    const int64_t ge = lower_bound_u32(skey, s, nm, k + 1);
    const int64_t bstart = off_in[(int64_t)(k / (uint32_t)B3) * B3];  // first old index of the cell's brick
    const int64_t nb = lower_bound_u32(sidx, s, ge, (uint32_t)bstart) - s;
    atomicAdd((unsigned long long*)&cnt[k],
              (unsigned long long)(((uint64_t)nb << 32) | (uint64_t)(ge - s)));
  }
}

// The two re-sort kernels below give each brick one wave (WB bricks per workgroup) and
// take its particles in chunks of 64, PU chunks' loads issued together; ranks come from
// ballots and a running count per wave, so no kernel has a barrier.
constexpr int WB = 4;
constexpr int PU = 4;

// Movers of brick b, in old stream order, to [moff[b], moff[b] + mcnt[b]).
__global__ __launch_bounds__(64 * WB) void k_compact_movers(
    const int64_t* off, const uint32_t* mcnt, const int64_t* moff, int B3, int64_t nbrick,
    int64_t n, const uint16_t* tdig, const uint32_t* mkey, uint32_t* okey, uint32_t* oidx) {
  const int lane = threadIdx.x & 63;
  const int64_t b = (int64_t)blockIdx.x * WB + (threadIdx.x >> 6);
  if (b >= nbrick || mcnt[b] == 0) return;  // the whole wave
  const uint64_t lt = lane ? ((~0ull) >> (64 - lane)) : 0ull;
  const int64_t j0 = min(off[b * B3], n), j1 = min(off[b * B3 + B3], n);
  int64_t dst = moff[b];
  for (int64_t base = j0; base < j1; base += 64 * PU) {
    uint32_t d[PU];
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int64_t j = base + 64 * u + lane;
      d[u] = j < j1 ? tdig[j] : 0u;
    }
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int64_t j = base + 64 * u + lane;
      const bool m = j < j1 && d[u] == (uint32_t)B3;
      const uint64_t bal = __ballot(m);
      if (m) {
        const int64_t o = dst + __popcll(bal & lt);
        okey[o] = mkey[j];
        oidx[o] = (uint32_t)j;
      }
      dst += __popcll(bal);
    }
  }
}

// Stayers of brick b to their final stream positions: the first position of the
// brick's stayers in each new cell (cell offset + arrivals from earlier bricks), plus
// the stayer's rank among the brick's stayers of that cell in old stream order (a
// stable multi-split of each chunk by digit and a running count per cell).
template <int P = 1, int V = 2>  // code widths
__global__ __launch_bounds__(64 * WB) void k_place_stayers(
    const int64_t* off_in, const uint16_t* tdig, const void* tpos_, const void* tvel_,
    const uint64_t* cnt, const int64_t* bstart, int B3, int nbits, int64_t nbrick,
    const uint32_t* skey, const uint32_t* sidx, const int64_t* astart,
    void* pos_, void* vel_, int64_t* perm, int64_t n, DevErr* err) {
  using PC = typename PosCode<P>::T;
  using VC = typename VelCode<V>::T;
  const PC* tpos = (const PC*)tpos_;
  const VC* tvel = (const VC*)tvel_;
  PC* pos = (PC*)pos_;
  VC* vel = (VC*)vel_;
  extern __shared__ int64_t lds[];  // dbase [WB][B3], then run [WB][B3] (uint32)
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int64_t* dbase = lds + (int64_t)wv * B3;
  uint32_t* run = (uint32_t*)(lds + (int64_t)WB * B3) + (int64_t)wv * B3;
  const int64_t b = (int64_t)blockIdx.x * WB + wv;
  if (b >= nbrick) return;  // the whole wave
  const uint64_t lt = lane ? ((~0ull) >> (64 - lane)) : 0ull;
  const int64_t kbase = b * B3;
  // new cell offsets of the brick: its first new position bstart[b] plus the exclusive
  // prefix of its cells' new counts (low 32 bits of cnt); stayers of a cell follow its
  // arrivals from earlier bricks (high 32 bits)
  int64_t carry = bstart[b];
  for (int l0 = 0; l0 < B3; l0 += 64) {
    const int l = l0 + lane;
    const uint64_t cv = l < B3 ? cnt[kbase + l] : 0ull;
    const uint32_t x = (uint32_t)cv;
    uint32_t inc = x;  // inclusive prefix over the 64 lanes
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(inc, d, 64);
      if (lane >= d) inc += y;
    }
    if (l < B3) {
      dbase[l] = carry + (int64_t)(inc - x) + (int64_t)(cv >> 32);
      run[l] = 0;
    }
    carry += (int64_t)__shfl(inc, 63, 64);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int64_t j0 = min(off_in[kbase], n), j1 = min(off_in[kbase + B3], n);
  for (int64_t base = j0; base < j1; base += 64 * PU) {
    uint32_t d[PU], p[PU][3], v[PU][3];
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int64_t j = base + 64 * u + lane;
      const bool h = j < j1;
      const int64_t jj = h ? j : j0;
      d[u] = h ? tdig[jj] : (uint32_t)B3;  // past the end: not a stayer
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        p[u][a] = tpos[3 * jj + a];
        v[u][a] = tvel[3 * jj + a];
      }
    }
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const uint32_t du = d[u];
      const bool stay = du < (uint32_t)B3;
      uint64_t match = __ballot(stay);
      for (int bit = 0; bit < nbits; ++bit) {
        const uint64_t mbit = __ballot(stay && ((du >> bit) & 1u));
        match &= ((du >> bit) & 1u) ? mbit : ~mbit;
      }
      const uint32_t rk = (uint32_t)__popcll(match & lt);
      uint32_t before = 0;
      if (stay) before = run[du];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (stay && rk == 0) run[du] = before + (uint32_t)__popcll(match);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (stay) {
        const int64_t dst = dbase[du] + (int64_t)(before + rk);
        const int64_t j = base + 64 * u + lane;
        if (dst < 0 || dst >= n) {
          latch_error(err, ERRBIT_CORRUPT);
        } else {
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            pos[3 * dst + a] = (PC)p[u][a];
            vel[3 * dst + a] = (VC)v[u][a];
          }
          if (perm) perm[dst] = j;
        }
      }
    }
  }
  // the brick's arrivals, placed by the same wave so that every line of the brick's
  // output range is written by one wave: arrivals from earlier bricks precede the
  // stayers of their new cell, the others follow them
  if (astart) {
    const int64_t ms = astart[b], me = astart[b + 1];
    for (int64_t s = ms + lane; s < me; s += 64) {
      const uint32_t k = skey[s];
      const int64_t gs = lower_bound_u32(skey, ms, s, k);
      const int64_t ge = lower_bound_u32(skey, s, me, k + 1);
      const uint64_t cv = cnt[k];
      const int64_t before = (int64_t)(cv >> 32), total = (int64_t)(cv & 0xffffffffull);
      const int64_t stay = total - (ge - gs);
      const int64_t jg = s - gs;
      // the cell's new offset is its stayers' base less the arrivals that precede them
      const int64_t dst = dbase[k - kbase] - before + (jg < before ? jg : stay + jg);
      const int64_t j = sidx[s];
      if (dst < 0 || dst >= n || j < 0 || j >= n) {
        latch_error(err, ERRBIT_CORRUPT);
        continue;
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        pos[3 * dst + a] = tpos[3 * j + a];
        vel[3 * dst + a] = tvel[3 * j + a];
      }
      if (perm) perm[dst] = j;
    }
  }
}

__global__ void k_read_total(const int64_t* moff, int64_t nb, int64_t* out) { *out = moff[nb]; }

// New particles of each brick: its old particles less its movers, plus its arrivals (the
// brick's run [astart[b], astart[b + 1]) of the sorted movers); their scan gives each
// brick's first new stream position, so that no scan over all cells is needed.
__global__ __launch_bounds__(KT) void k_brick_totals(const int64_t* off_in, const uint32_t* mcnt,
                                                    const int64_t* astart, int B3,
                                                    int64_t nbrick, int64_t n, uint32_t* tot) {
  const int64_t b = (int64_t)blockIdx.x * KT + threadIdx.x;
  if (b >= nbrick) return;
  const int64_t j0 = min(off_in[b * B3], n), j1 = min(off_in[(b + 1) * B3], n);
  const int64_t t = (j1 > j0 ? j1 - j0 : 0) - (int64_t)mcnt[b] + (astart[b + 1] - astart[b]);
  tot[b] = (uint32_t)(t > 0 ? t : 0);
}

}  // namespace

pm_status run_kick_float(pm_context* c, const pm_species* in, pm_species* out,
                         const float* acc, double ck, double cd) {
  if (in->n == 0) return PM_OK;
  ProfScope ps(c, ST_KICK);
  hipLaunchKernelGGL(k_kick_float, dim3((unsigned)cdiv(in->n, KT)), dim3(KT), 0, c->stream,
                     in->x, in->v, out->x, out->v, in->n, acc, c->g.ng, c->g.ngL,
                     (float)c->g.box, (float)ck, (float)cd);
  PM_LAUNCH_CHECK();
  return PM_OK;
}

// All species of a compressed state: one brick kernel launch, then the re-sort of each
// species. offs[s]: input cell offsets; perm[s] (device int64 [n], nullable): new stream
// position -> old stream position. P, V: the species' code widths.
template <int P, int V>
static pm_status kick_compressed_t(pm_context* c, const pm_species* in, pm_species* out,
                                   int n_sp, int64_t* const* offs, const float* acc,
                                   const float* amax, double ck, double cd,
                                   int64_t* const* perm, const float* const* app) {
  const Geom& g = c->g;
  if (n_sp <= 0 || n_sp > MAXSP) return PM_ERR_ARG;
  const int B3 = g.B * g.B * g.B;
  int64_t ntot = 0, nbase[MAXSP + 1];
  for (int s = 0; s < n_sp; ++s) {
    nbase[s] = ntot;
    ntot += in[s].n;
  }
  nbase[n_sp] = ntot;
  const size_t nn = (size_t)(ntot > 0 ? ntot : 1);
  uint64_t* cnt = (uint64_t*)scratch(c, SC_CNT, (size_t)g.ncell3 * 8 * n_sp);
  int64_t* bstart = (int64_t*)scratch(c, SC_OFF2, (size_t)(g.nbrick + 1) * 8);
  uint32_t* btot = (uint32_t*)scratch(c, SC_BTOT, (size_t)g.nbrick * 4);
  char* tpos = (char*)scratch(c, SC_TPOS, nn * 3 * P);
  char* tvel = (char*)scratch(c, SC_TVEL, nn * 3 * V);
  uint16_t* tdig = (uint16_t*)scratch(c, SC_TDST, nn * 2);
  uint32_t* mkey = (uint32_t*)scratch(c, SC_KEYA, nn * 4);
  uint32_t* midx = (uint32_t*)scratch(c, SC_VALA, nn * 4);
  uint32_t* skey = (uint32_t*)scratch(c, SC_KEYB, nn * 4);
  uint32_t* sidx = (uint32_t*)scratch(c, SC_VALB, nn * 4);
  uint32_t* mcnt = (uint32_t*)scratch(c, SC_MCNT, (size_t)g.nbrick * 4 * n_sp);
  int64_t* moff = (int64_t*)scratch(c, SC_MOFF, (size_t)(g.nbrick + 1) * 8);
  int32_t* part = (int32_t*)scratch(c, SC_PARTS, (size_t)g.nbrick * 8 * n_sp);
  if (!cnt || !bstart || !btot || !tpos || !tvel || !tdig || !mkey || !midx || !skey || !sidx ||
      !mcnt || !moff || !part)
    return PM_ERR_NOMEM;
  KickArgs A{};
  A.n_sp = n_sp;
  A.acc = acc;
  A.ck = (float)ck;
  A.cdS = cd * g.SL * (P == 1 ? 1.0 : 256.0);
  for (int s = 0; s < n_sp; ++s) {
    KickSpecies& S = A.sp[s];
    S.n = in[s].n;
    S.pos = in[s].pos;
    S.vel = in[s].vel;
    S.hin = in[s].hdr;
    S.hout = out[s].hdr;
    S.off = offs[s];
    S.tpos = tpos + 3 * P * nbase[s];
    S.tvel = tvel + 3 * V * nbase[s];
    S.tdig = tdig + nbase[s];
    S.cnt = cnt + (int64_t)s * g.ncell3;
    S.mkey = mkey + nbase[s];
    S.mcnt = mcnt + (int64_t)s * g.nbrick;
    S.pmn = part + (int64_t)2 * s * g.nbrick;
    S.pmx = S.pmn + g.nbrick;
    S.app = app ? app[s] : nullptr;
  }
  {
    pm_status st0;
    for (int s = 0; s < n_sp; ++s)
      hipLaunchKernelGGL(k_vmax_next<V>, dim3(1), dim3(1), 0, c->stream, in[s].hdr,
                         out[s].hdr, amax, ck, in[s].n);
    ProfScope ps(c, ST_KICK);
    const int R = g.B * g.r;
    const size_t tail = (size_t)MAXSP * (B3 + 1) * 4 * 2;
    // two bricks per workgroup: R = 16, an even number of bricks per side, z quarters of
    // whole cells
    const size_t pbytes = (size_t)3 * (2 * PR + 1) * (PR + 1) * (PR / 4 + 1) * 4 + 2 * tail;
    const size_t fbytes = (size_t)3 * (R + 1) * (R + 1) * (R + 1) * 4;
    if (R == PR && g.lgnb >= 1 && (g.B % 4) == 0 && pbytes <= 48 * 1024)
      hipLaunchKernelGGL((k_kick_pair<256, 4, P, V>), dim3((unsigned)(g.nbrick / 2)),
                         dim3(256), pbytes, c->stream, A, g, c->err);
    else if (R == 16 && fbytes + tail <= 96 * 1024)
      hipLaunchKernelGGL((k_kick_brick<16, P, V>), dim3((unsigned)g.nbrick), dim3(KB),
                         fbytes + tail, c->stream, A, g, c->err);
    else if (R == 8)
      hipLaunchKernelGGL((k_kick_brick<8, P, V>), dim3((unsigned)g.nbrick), dim3(KB),
                         fbytes + tail, c->stream, A, g, c->err);
    else
      hipLaunchKernelGGL((k_kick_brick<0, P, V>), dim3((unsigned)g.nbrick), dim3(KB), tail,
                         c->stream, A, g, c->err);
    PM_LAUNCH_CHECK();
    prof_end(c);  // the scope covers the brick kernel only
    for (int s = 0; s < n_sp; ++s)
      if ((st0 = fold_minmax_to_header(c, A.sp[s].pmn, A.sp[s].pmx, g.nbrick, out[s].hdr)) !=
          PM_OK)
        return st0;
  }
  const size_t place_lds = (size_t)WB * B3 * 12;
  int64_t* nmov = (int64_t*)scratch(c, SC_NMOV, (size_t)MAXSP * 8);
  if (!nmov) return PM_ERR_NOMEM;
  for (int s = 0; s < n_sp; ++s) {
    const int64_t n = in[s].n;
    const KickSpecies& S = A.sp[s];
    ProfScope ps(c, ST_RESORT);
    pm_status st = scan_u32(c, S.mcnt, g.nbrick, moff);
    if (st != PM_OK) return st;
    // the mover count stays on the device; the kernels below read it there and are
    // launched for the worst case (every particle a mover), so nothing waits on the host
    int64_t* nmd = nmov + s;
    hipLaunchKernelGGL(k_read_total, dim3(1), dim3(1), 0, c->stream, moff, g.nbrick, nmd);
    uint32_t* sk = skey + nbase[s];
    uint32_t* si = sidx + nbase[s];
    if (n > 0) {
      hipLaunchKernelGGL(k_compact_movers, dim3((unsigned)cdiv(g.nbrick, WB)), dim3(64 * WB),
                         0, c->stream, S.off, S.mcnt, moff, B3, g.nbrick, n, S.tdig, S.mkey,
                         sk, si);
      PM_LAUNCH_CHECK();
      // stable sort (old order preserved inside each new cell)
      uint32_t *k1 = sk, *v1 = si, *k2 = S.mkey, *v2 = midx + nbase[s];
      st = radix_sort_pairs_dev(c, &k1, &v1, &k2, &v2, n, nmd, 3 * (g.lgB + g.lgnb));
      if (st != PM_OK) return st;
      sk = k1;
      si = v1;
      const int64_t ag = std::min<int64_t>(cdiv(n, KT), 2048);
      hipLaunchKernelGGL(k_arrivals, dim3((unsigned)ag), dim3(KT), 0, c->stream, sk, si, nmd,
                         S.off, B3, S.cnt);
      PM_LAUNCH_CHECK();
    }
    // the mover offsets are spent: moff now takes each brick's run of arrivals
    hipLaunchKernelGGL(k_brick_arrivals, dim3((unsigned)cdiv(g.nbrick + 1, KT)), dim3(KT), 0,
                       c->stream, sk, nmd, B3, g.nbrick, moff);
    PM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_brick_totals, dim3((unsigned)cdiv(g.nbrick, KT)), dim3(KT), 0,
                       c->stream, S.off, S.mcnt, moff, B3, g.nbrick, n, btot);
    PM_LAUNCH_CHECK();
    st = scan_u32(c, btot, g.nbrick, bstart);
    if (st != PM_OK) return st;
    int64_t* pm = perm ? perm[s] : nullptr;
    hipLaunchKernelGGL((k_place_stayers<P, V>), dim3((unsigned)cdiv(g.nbrick, WB)),
                       dim3(64 * WB), place_lds, c->stream, S.off, S.tdig,
                       (const void*)S.tpos, (const void*)S.tvel, S.cnt, bstart, B3,
                       3 * g.lgB, g.nbrick, sk, si, moff, (void*)out[s].pos,
                       (void*)out[s].vel, pm, n, c->err);
    PM_LAUNCH_CHECK();
    st = run_finalize_counts(c, nullptr, S.cnt, &out[s]);
    if (st != PM_OK) return st;
  }
  return PM_OK;
}

pm_status run_kick_compressed_all(pm_context* c, const pm_species* in, pm_species* out,
                                  int n_sp, int64_t* const* offs, const float* acc,
                                  const float* amax, double ck, double cd,
                                  int64_t* const* perm, const float* const* app) {
  if (n_sp <= 0 || n_sp > MAXSP) return PM_ERR_ARG;
  const int kind = common_width_kind(in, n_sp);
  if (kind < 0) return PM_ERR_ARG;
  return width_dispatch(kind, [&](auto P_, auto V_) {
    return kick_compressed_t<decltype(P_)::value, decltype(V_)::value>(
        c, in, out, n_sp, offs, acc, amax, ck, cd, perm, app);
  });
}

pm_status run_kick_compressed(pm_context* c, const pm_species* in, pm_species* out,
                              const float* acc, const float* amax, double ck, double cd,
                              uint32_t* /*unused*/) {
  int64_t* off = (int64_t*)scratch(c, SC_SPOFF0, (size_t)(c->g.ncell3 + 1) * 8);
  if (!off) return PM_ERR_NOMEM;
  pm_status s = run_cell_offsets(c, in, off);
  if (s != PM_OK) return s;
  int64_t* offs[1] = {off};
  return run_kick_compressed_all(c, in, out, 1, offs, acc, amax, ck, cd, nullptr);
}

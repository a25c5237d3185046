// CIC force interpolation (Fig. 2 "inverse_force_interpolation"), kick and drift, fused
// with the re-encode of compressed particles and the stable re-sort of the stream into
// cell order (Sec. 2.4: particles are written cell by cell).
//
// Compressed path, per species:
//   k_vmax_next     v_max' = smallest power of two >= V + |c_k| A_max (V: largest
//                   decoded |v| of the input, from its extreme velocity codes; A_max:
//                   largest |a| on the mesh). Interpolation is a convex combination of
//                   mesh values, so no kicked component exceeds the bound.
//   k_kick_brick    one workgroup per brick of B^3 cells, particles in stream order:
//                   decode, gather a from the 8 CIC nodes, v' = v + c_k a, fixed-point
//                   drift u' = u + floor(v' c_d S + 1/2), new codes. Particles that
//                   stay inside the brick get their stable rank inside their new cell;
//                   the others ("movers") are listed with (new cell, old index).
//   movers          compacted in old order, stably radix-sorted by new cell.
//   k_arrivals      per new cell: arrivals, and how many of them come from earlier
//                   bricks (they precede the cell's stayers in stream order).
//   scan            new cell offsets.
//   k_place_*       stayers and movers written at their final stream positions
//                   (per brick, the stayers' per-cell destinations staged in LDS).
#include <type_traits>

#include "pm_codec.h"
#include "pm_scan.h"

namespace {

constexpr int KT = 256;  // threads per workgroup
constexpr uint32_t MOVER = 0xffffffffu;
constexpr uint32_t RANK_BITS = 23;
constexpr uint32_t RANK_LIMIT = (1u << RANK_BITS) - 1;

// ------------------------------------------------------------ float layout --
__global__ __launch_bounds__(KT) void k_kick_float(const float* x, const float* v, float* xo,
                                                  float* vo, int64_t n, const float* acc,
                                                  int64_t ng, float ck, float cd) {
  int64_t p = (int64_t)blockIdx.x * KT + threadIdx.x;
  if (p >= n) return;
  const int64_t n3 = ng * ng * ng;
  int64_t i[3];
  float f[3], xv[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    xv[a] = x[3 * p + a];
    float u = xv[a] * (float)ng;  // exact (ng a power of two)
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
    x1 -= floorf(x1);
    if (x1 >= 1.f) x1 = 0.f;
    vo[3 * p + a] = v1;
    xo[3 * p + a] = x1;
  }
}

// ------------------------------------------------------- compressed layout --
__global__ void k_vmax_next(const pm_shdr* hin, pm_shdr* hout, const float* amax, double ck,
                            int64_t n) {
  double V = 0.0;
  if (n > 0 && hin->j_max >= 0) {
    double a = fabs((double)vel_decode((uint32_t)hin->j_min, hin->v_max));
    double b = fabs((double)vel_decode((uint32_t)hin->j_max, hin->v_max));
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

constexpr int KB = 512;       // threads per workgroup of the brick kick
constexpr int MAXSP = 4;

struct KickSpecies {
  int64_t n;
  const uint8_t* pos;
  const uint16_t* vel;
  const pm_shdr* hin;
  pm_shdr* hout;
  const int64_t* off;   // input cell offsets [ncell3 + 1]
  uint8_t* tpos;        // new codes, old stream order
  uint16_t* tvel;
  uint32_t* tdst;       // (new local cell << 23) | rank, or MOVER
  uint64_t* cnt;        // per cell: stayers (low 32 bits)
  uint32_t* mkey;       // movers: new cell key, at [brick start + mover rank]
  uint32_t* midx;       // movers: old stream index
  uint32_t* mcnt;       // movers per brick
  int32_t* pmn;         // per-brick extreme new velocity codes, folded into hout
  int32_t* pmx;
};
struct KickArgs {
  KickSpecies sp[MAXSP];
  int n_sp;
  const float* acc;     // [3][ng^3]
  float ck;
  double cdS;           // c_d * S (position codes per unit velocity)
};

// One workgroup per brick, all species. With STAGE the brick's force nodes
// [b R, b R + R]^3 (R = B r) are first copied to LDS with coalesced loads and every
// particle gathers its 8 CIC nodes from there; the mesh is then read once per step
// for all species. The global reads of a workgroup form two rounds: (1) the force
// tile, every species' cell offsets and velocity headers; (2) the codes of the first
// chunk of every species. Only species with more than KB particles in the brick load
// later chunks on the way.
template <int RS>  // staged tile side in nodes (compile time), or 0: gather from HBM
__global__ __launch_bounds__(KB) void k_kick_brick(KickArgs A, Geom g, DevErr* err) {
  constexpr bool STAGE = RS > 0;
  const int B = g.B, B3 = B * B * B;
  constexpr int R1 = RS + 1;
  const int r = g.r;
  extern __shared__ unsigned char smem[];
  float* F = (float*)smem;                                     // [3][R1^3] when STAGE
  const int fsz = STAGE ? 3 * R1 * R1 * R1 : 0;
  int64_t* loffs = (int64_t*)(smem + ((fsz * 4 + 7) / 8) * 8);  // [MAXSP][B3 + 1]
  uint32_t* run = (uint32_t*)(loffs + MAXSP * (B3 + 1));       // [B3 + 1] (B3 = movers)
  uint32_t* wcnt = run + (B3 + 1);  // [2][KB/64][B3 + 1], then rel [B3 + 1]
  constexpr int NW = KB / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t lt = lane ? ((~0ull) >> (64 - lane)) : 0ull;
  const int64_t b = xcd_tile(blockIdx.x, g.nbrick);
  const uint32_t kbase = (uint32_t)(b * B3);
  const int64_t ng = g.ng, n3 = ng * ng * ng;
  uint32_t bcx, bcy, bcz;  // first cell of the brick
  key_cell(g, kbase, bcx, bcy, bcz);
  const int64_t ox = (int64_t)bcx * r, oy = (int64_t)bcy * r, oz = (int64_t)bcz * r;
  const int n_sp = A.n_sp;

  // ---- round 1: cell offsets of every species, velocity headers, force tile
  const int NL = n_sp * (B3 + 1);
  int64_t lof[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int i = threadIdx.x + k * KB;
    if (i < NL) {
      const int s = i / (B3 + 1);
      lof[k] = A.sp[s].off[kbase + (i - s * (B3 + 1))];
    }
  }
  for (int i = threadIdx.x + 2 * KB; i < NL; i += KB) {  // more than 2 KB entries
    const int s = i / (B3 + 1);
    loffs[i] = A.sp[s].off[kbase + (i - s * (B3 + 1))];
  }
  float vin[MAXSP], vout[MAXSP];
#pragma unroll
  for (int s = 0; s < MAXSP; ++s) {
    vin[s] = s < n_sp ? A.sp[s].hin->v_max : 0.f;
    vout[s] = s < n_sp ? A.sp[s].hout->v_max : 0.f;
  }
  if constexpr (STAGE) {
    // rows of RS nodes (x) as float4 loads, then the x = RS halo column; node (lz, ly)
    // of component c is row (c R1 + lz) R1 + ly. Indexes past the end are clamped to
    // the last element (a duplicate load, not stored), so no load sits behind a branch.
    static_assert(RS % 4 == 0, "staged tile side must be a multiple of 4");
    constexpr int ROWS = 3 * R1 * R1;
    constexpr int Q = RS / 4;  // float4 per row
    constexpr int NQ = ROWS * Q;
    constexpr int PQ = (NQ + KB - 1) / KB;    // float4 loads per thread
    constexpr int PH = (ROWS + KB - 1) / KB;  // halo loads per thread
    const int64_t m = ng - 1;                 // ng is a power of two
    const int64_t hx = (ox + RS) & m;
    float4 vq[PQ];
    float vh[PH];
    // row index (c R1 + lz) R1 + ly advanced by KB / Q rows per load without divisions
    constexpr int RR = R1 * R1;
    constexpr int DR = KB / Q;
    constexpr int DC = DR / RR, DLZ = (DR % RR) / R1, DLY = DR % R1;
    static_assert(KB % Q == 0, "a workgroup covers whole rows");
    const float* pc0 = A.acc;
    const float* pc1 = A.acc + n3;
    const float* pc2 = A.acc + 2 * n3;
    const uint32_t mu = (uint32_t)m, ngu = (uint32_t)ng;
    const uint32_t oxq = (uint32_t)ox + 4 * (threadIdx.x % Q);
    const int row0 = threadIdx.x / Q;
    {
      int c = row0 / RR, lz = (row0 % RR) / R1, ly = row0 % R1;
#pragma unroll
      for (int k = 0; k < PQ; ++k) {
        const bool over = c >= 3;  // past the end: load the last row again (not stored)
        const int cc = over ? 2 : c, zz = over ? R1 - 1 : lz, yy = over ? R1 - 1 : ly;
        const float* pc = cc == 0 ? pc0 : (cc == 1 ? pc1 : pc2);
        const uint32_t gz = ((uint32_t)oz + zz) & mu, gy = ((uint32_t)oy + yy) & mu;
        vq[k] = *(const float4*)(pc + ((uint64_t)(gz * ngu + gy) * ngu + oxq));
        ly += DLY;
        lz += DLZ;
        c += DC;
        if (ly >= R1) {
          ly -= R1;
          ++lz;
        }
        if (lz >= R1) {
          lz -= R1;
          ++c;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < PH; ++k) {
      const int row = min((int)threadIdx.x + k * KB, ROWS - 1);
      const int c = row / RR, rem = row - c * RR;
      const int lz = rem / R1, ly = rem - lz * R1;
      const float* pc = c == 0 ? pc0 : (c == 1 ? pc1 : pc2);
      const uint32_t gz = ((uint32_t)oz + lz) & mu, gy = ((uint32_t)oy + ly) & mu;
      vh[k] = pc[(uint64_t)(gz * ngu + gy) * ngu + (uint32_t)hx];
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
        if (ly >= R1) {
          ly -= R1;
          ++lz;
        }
        if (lz >= R1) {
          lz -= R1;
          ++c;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < PH; ++k) {
      const int row = threadIdx.x + k * KB;
      if (row < ROWS) F[row * R1 + RS] = vh[k];
    }
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int i = threadIdx.x + k * KB;
    if (i < NL) loffs[i] = lof[k];
  }
  __syncthreads();

  // ---- round 2: codes of the first chunk of every species
  uint32_t pre_pb[MAXSP][3], pre_vc[MAXSP][3];
#pragma unroll
  for (int s = 0; s < MAXSP; ++s) {
    const int64_t* lo = loffs + s * (B3 + 1);
    const bool have = s < n_sp;
    const int64_t n = have ? A.sp[s].n : 0;
    const int64_t j0 = have ? min(lo[0], n) : 0, j1 = have ? min(lo[B3], n) : 0;
    const int64_t j = j0 + threadIdx.x;
    const int64_t jj = j < j1 ? j : 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      pre_pb[s][a] = j < j1 ? A.sp[s].pos[3 * jj + a] : 0u;
      pre_vc[s][a] = j < j1 ? A.sp[s].vel[3 * jj + a] : 0u;
    }
  }

  const int nbits = 3 * g.lgB + 1;  // local cell bits + mover flag
  const uint32_t mB = (uint32_t)B - 1;
  const uint32_t bc[3] = {bcx, bcy, bcz};
  const uint32_t Sm = (uint32_t)g.S - 1;
  const double Sd = (double)g.S, invS = 1.0 / Sd;  // powers of two
  bool bad = false;
  __shared__ int mm[2 * NW];  // per-wave extreme velocity codes
  // Rounds of KB particles in stream order. Per round: (1) new codes and digits, stable
  // multi-split inside each wave, per-wave digit counts into wcnt[round & 1]; barrier;
  // (2) rank = running count + counts of earlier waves + rank in the wave, outputs,
  // and the other count buffer cleared for the next round; barrier; (3) running counts
  // advanced (overlaps the next round's step 1, which uses the other buffer).
  const int WS = NW * (B3 + 1);
  uint32_t* rel = wcnt + 2 * WS;  // [B3 + 1]: cell offsets relative to the brick's first
#pragma unroll
  for (int s = 0; s < MAXSP; ++s) {
    if (s >= n_sp) break;
    const KickSpecies& S = A.sp[s];
    const int64_t* loff = loffs + s * (B3 + 1);
    __syncthreads();  // previous species done with run, rel and wcnt
    const int64_t l0 = loff[0];
    for (int i = threadIdx.x; i <= B3; i += KB) {
      run[i] = 0;
      rel[i] = (uint32_t)(loff[i] - l0);
    }
    for (int i = threadIdx.x; i < 2 * WS; i += KB) wcnt[i] = 0;
    __syncthreads();
    const int64_t j0 = min(l0, S.n), j1 = min(loff[B3], S.n);
    // float32 forms of the velocity codec where they give the same codes (uniform)
    const float vmax_in = vin[s];
    const float vmax_out = vout[s];
    const bool fdec = vmax_in >= 0x1p-90f && vmax_in <= 0x1p90f;
    const uint32_t ob = __float_as_uint(vmax_out);
    const bool fenc = vmax_out >= 0x1p-90f && vmax_out <= 0x1p90f && (ob & 0x7fffffu) == 0;
    const float wdec = vmax_in * 0x1p-15f;
    const float cenc = __uint_as_float((269u - (ob >> 23)) << 23);  // 2^15 / v_max
    int jmin = 65536, jmax = -1;
    // the round loop, compiled once with the float32 codec forms and once without
    auto rounds = [&](auto fast) {
      constexpr bool FAST = decltype(fast)::value;
      int rnd = 0;
      for (int64_t base = j0; base < j1; base += KB, ++rnd) {
        uint32_t* wc = wcnt + (rnd & 1) * WS;
        uint32_t* wo = wcnt + ((rnd & 1) ^ 1) * WS;
        const int64_t j = base + threadIdx.x;
        const bool valid = j < j1;
        const uint32_t t3 = 3 * threadIdx.x;
        uint32_t digit = 0, un[3] = {0, 0, 0};
        if (valid) {
          // the particle's codes: prefetched for the first round
          uint32_t pb[3], vc[3];
          if (base == j0) {
  #pragma unroll
            for (int a = 0; a < 3; ++a) {
              pb[a] = pre_pb[s][a];
              vc[a] = pre_vc[s][a];
            }
          } else {
            const uint8_t* pp = S.pos + 3 * base;
            const uint16_t* vp = S.vel + 3 * base;
  #pragma unroll
            for (int a = 0; a < 3; ++a) {
              pb[a] = pp[t3 + a];
              vc[a] = vp[t3 + a];
            }
          }
          const uint32_t jr = (uint32_t)(base - l0) + threadIdx.x;
          int lo = 0, hi = B3;  // local cell: largest l with rel[l] <= jr
          while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (rel[mid] <= jr) lo = mid; else hi = mid;
          }
          const uint32_t lc[3] = {(uint32_t)lo & mB, ((uint32_t)lo >> g.lgB) & mB,
                                  (uint32_t)lo >> (2 * g.lgB)};
          int li[3];
          float f[3];
  #pragma unroll
          for (int a = 0; a < 3; ++a) {
            // position in 1/512 mesh cells from the brick's corner node: (2 u + 1) r
            const uint32_t gl = (2 * ((lc[a] << 8) | pb[a]) + 1) * (uint32_t)r;
            li[a] = (int)(gl >> 9);
            f[a] = (float)(gl & 511u) * (1.0f / 512.0f);
          }
          float acc3[3] = {0.f, 0.f, 0.f};
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
          uint8_t* tp = S.tpos + 3 * base;
          uint16_t* tv = S.tvel + 3 * base;
          uint32_t nl[3];
  #pragma unroll
          for (int a = 0; a < 3; ++a) {
            const float v0 = FAST ? vel_decode_w(vc[a], wdec) : vel_decode(vc[a], vmax_in);
            const float v1 = v0 + A.ck * acc3[a];
            const double d = floor((double)v1 * A.cdS + 0.5);
            const bool okd = fabs(d) < 4.0e15;
            bad |= !okd;
            // d mod S, exact in float64 (d is an integer below 2^52, S a power of two)
            const double dm = okd ? d - Sd * floor(d * invS) : 0.0;
            un[a] = ((((bc[a] + lc[a]) << 8) | pb[a]) + (uint32_t)dm) & Sm;
            nl[a] = (un[a] >> 8) - bc[a];  // new local cell (wraps above B when outside)
            const int jc = FAST ? vel_code_p2(v1, cenc) : vel_code(v1, vmax_out);
            tp[t3 + a] = (uint8_t)(un[a] & 255u);
            tv[t3 + a] = (uint16_t)jc;
            jmin = min(jmin, jc);
            jmax = max(jmax, jc);
          }
          digit = (nl[0] <= mB && nl[1] <= mB && nl[2] <= mB)
                      ? (((nl[2] << g.lgB) | nl[1]) << g.lgB) | nl[0]
                      : (uint32_t)B3;
        }
        // stable multi-split of this round by digit (new local cell, or B3 for movers)
        uint64_t match = __ballot(valid);
        for (int bit = 0; bit < nbits; ++bit) {
          uint64_t mbit = __ballot(valid && ((digit >> bit) & 1u));
          match &= ((digit >> bit) & 1u) ? mbit : ~mbit;
        }
        const uint32_t rk = (uint32_t)__popcll(match & lt);
        if (valid && rk == 0) wc[w * (B3 + 1) + digit] = (uint32_t)__popcll(match);
        __syncthreads();
        if (valid) {
          uint32_t pre = run[digit];
          for (int q = 0; q < w; ++q) pre += wc[q * (B3 + 1) + digit];
          const uint32_t rank = pre + rk;
          if (digit < (uint32_t)B3) {
            if (rank >= RANK_LIMIT) bad = true;
            S.tdst[j] = (digit << RANK_BITS) | (rank & RANK_LIMIT);
          } else {
            S.tdst[j] = MOVER;
            S.mkey[j0 + rank] = cell_key(g, un[0] >> 8, un[1] >> 8, un[2] >> 8);
            S.midx[j0 + rank] = (uint32_t)j;
          }
        }
        for (int i = threadIdx.x; i < WS; i += KB) wo[i] = 0;
        __syncthreads();
        for (int i = threadIdx.x; i <= B3; i += KB) {
          uint32_t add = 0;
          for (int q = 0; q < NW; ++q) add += wc[q * (B3 + 1) + i];
          run[i] += add;
        }
      }
    };
    if (fdec && fenc) rounds(std::true_type{});
    else rounds(std::false_type{});
    // the thread that advanced run[i] writes it out
    for (int i = threadIdx.x; i <= B3; i += KB) {
      if (i < B3) S.cnt[kbase + i] = (uint64_t)run[i];
      else S.mcnt[b] = run[B3];
    }
    // block min / max of the new velocity codes, stored per brick (no atomics)
    for (int d = 32; d >= 1; d >>= 1) {
      jmin = min(jmin, __shfl_xor(jmin, d, 64));
      jmax = max(jmax, __shfl_xor(jmax, d, 64));
    }
    if (lane == 0) {
      mm[2 * w] = jmin;
      mm[2 * w + 1] = jmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int q = 1; q < NW; ++q) {
        jmin = min(jmin, mm[2 * q]);
        jmax = max(jmax, mm[2 * q + 1]);
      }
      S.pmn[b] = jmin;
      S.pmx[b] = jmax;
    }
  }
  if (bad) latch_error(err, ERRBIT_RANGE);
}

// movers of brick b sit at [off[b B^3], off[b B^3] + mcnt[b]); gather them in old order
__global__ __launch_bounds__(KT) void k_compact_movers(const int64_t* off, const uint32_t* mcnt,
                                                      const int64_t* moff, int B3,
                                                      const uint32_t* mkey, const uint32_t* midx,
                                                      uint32_t* okey, uint32_t* oidx) {
  const int64_t b = blockIdx.x;
  const int64_t src = off[b * B3], dst = moff[b];
  const uint32_t m = mcnt[b];
  for (uint32_t i = threadIdx.x; i < m; i += KT) {
    okey[dst + i] = mkey[src + i];
    oidx[dst + i] = midx[src + i];
  }
}

__device__ inline int64_t lower_bound_u32(const uint32_t* a, int64_t lo, int64_t hi, uint32_t v) {
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (a[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// per group of sorted movers with the same new cell: add arrivals (low 32 bits) and
// arrivals from earlier bricks (high 32 bits) to the cell's count
__global__ __launch_bounds__(KT) void k_arrivals(const uint32_t* skey, const uint32_t* sidx,
                                                int64_t nm, const int64_t* off_in, int B3,
                                                uint64_t* cnt) {
  int64_t s = (int64_t)blockIdx.x * KT + threadIdx.x;
  if (s >= nm) return;
  const uint32_t k = skey[s];
  if (s > 0 && skey[s - 1] == k) return;  // group leader only
  const int64_t ge = lower_bound_u32(skey, s, nm, k + 1);
  const int64_t bstart = off_in[(int64_t)(k / (uint32_t)B3) * B3];  // first old index of the cell's brick
  const int64_t nb = lower_bound_u32(sidx, s, ge, (uint32_t)bstart) - s;
  atomicAdd((unsigned long long*)&cnt[k], (unsigned long long)(((uint64_t)nb << 32) | (uint64_t)(ge - s)));
}

// One workgroup per brick. The first stream position of the brick's stayers in each
// new cell (cell offset + arrivals from earlier bricks) is staged in LDS, so a stayer
// needs its own coalesced loads only; each thread takes U particles per pass with all
// their loads issued before any store.
__global__ __launch_bounds__(KT) void k_place_stayers(const int64_t* off_in, const uint32_t* tdst,
                                                     const uint8_t* tpos, const uint16_t* tvel,
                                                     const uint64_t* cnt, const int64_t* off_new,
                                                     int B3, uint8_t* pos, uint16_t* vel,
                                                     int64_t* perm, int64_t n, DevErr* err) {
  extern __shared__ int64_t dbase[];  // [B3]
  constexpr int U = 2;
  const int64_t b = blockIdx.x;
  const int64_t kbase = b * B3;
  for (int l = threadIdx.x; l < B3; l += KT)
    dbase[l] = off_new[kbase + l] + (int64_t)(cnt[kbase + l] >> 32);
  const int64_t j0 = min(off_in[kbase], n), j1 = min(off_in[kbase + B3], n);
  __syncthreads();
  for (int64_t j = j0 + threadIdx.x; j < j1; j += U * KT) {
    uint32_t d[U], p[U][3], v[U][3];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t ju = j + u * KT;
      const bool h = ju < j1;
      const int64_t jj = h ? ju : j;
      d[u] = h ? tdst[jj] : MOVER;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        p[u][a] = tpos[3 * jj + a];
        v[u][a] = tvel[3 * jj + a];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (d[u] == MOVER) continue;
      const int64_t dst = dbase[d[u] >> RANK_BITS] + (int64_t)(d[u] & RANK_LIMIT);
      if (dst < 0 || dst >= n) {
        latch_error(err, ERRBIT_CORRUPT);
        continue;
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        pos[3 * dst + a] = (uint8_t)p[u][a];
        vel[3 * dst + a] = (uint16_t)v[u][a];
      }
      if (perm) perm[dst] = j + u * KT;
    }
  }
}

__global__ __launch_bounds__(KT) void k_place_movers(const uint32_t* skey, const uint32_t* sidx,
                                                    int64_t nm, const uint8_t* tpos,
                                                    const uint16_t* tvel, const uint64_t* cnt,
                                                    const int64_t* off_new, uint8_t* pos,
                                                    uint16_t* vel, int64_t* perm, int64_t n,
                                                    DevErr* err) {
  int64_t s = (int64_t)blockIdx.x * KT + threadIdx.x;
  if (s >= nm) return;
  const uint32_t k = skey[s];
  const int64_t gs = lower_bound_u32(skey, 0, s, k);
  const int64_t ge = lower_bound_u32(skey, s, nm, k + 1);
  const uint64_t cv = cnt[k];
  const int64_t before = (int64_t)(cv >> 32), total = (int64_t)(cv & 0xffffffffull);
  const int64_t stay = total - (ge - gs);
  const int64_t jg = s - gs;
  const int64_t dst = off_new[k] + (jg < before ? jg : stay + jg);
  const int64_t j = sidx[s];
  if (dst < 0 || dst >= n || j >= n) {
    latch_error(err, ERRBIT_CORRUPT);
    return;
  }
  pos[3 * dst] = tpos[3 * j];
  pos[3 * dst + 1] = tpos[3 * j + 1];
  pos[3 * dst + 2] = tpos[3 * j + 2];
  vel[3 * dst] = tvel[3 * j];
  vel[3 * dst + 1] = tvel[3 * j + 1];
  vel[3 * dst + 2] = tvel[3 * j + 2];
  if (perm) perm[dst] = j;
}

__global__ void k_read_total(const int64_t* moff, int64_t nb, int64_t* out) { *out = moff[nb]; }

}  // namespace

pm_status run_kick_float(pm_context* c, const pm_species* in, pm_species* out,
                         const float* acc, double ck, double cd) {
  if (in->n == 0) return PM_OK;
  ProfScope ps(c, ST_KICK);
  hipLaunchKernelGGL(k_kick_float, dim3((unsigned)cdiv(in->n, KT)), dim3(KT), 0, c->stream,
                     in->x, in->v, out->x, out->v, in->n, acc, c->g.ng, (float)ck, (float)cd);
  PM_LAUNCH_CHECK();
  return PM_OK;
}

// All species of a compressed state: one brick kernel launch, then the re-sort of each
// species. offs[s]: input cell offsets; perm[s] (device int64 [n], nullable): new stream
// position -> old stream position.
pm_status run_kick_compressed_all(pm_context* c, const pm_species* in, pm_species* out,
                                  int n_sp, int64_t* const* offs, const float* acc,
                                  const float* amax, double ck, double cd,
                                  int64_t* const* perm) {
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
  int64_t* off_new = (int64_t*)scratch(c, SC_OFF2, (size_t)(g.ncell3 + 1) * 8);
  uint8_t* tpos = (uint8_t*)scratch(c, SC_TPOS, nn * 3);
  uint16_t* tvel = (uint16_t*)scratch(c, SC_TVEL, nn * 6);
  uint32_t* tdst = (uint32_t*)scratch(c, SC_TDST, nn * 4);
  uint32_t* mkey = (uint32_t*)scratch(c, SC_KEYA, nn * 4);
  uint32_t* midx = (uint32_t*)scratch(c, SC_VALA, nn * 4);
  uint32_t* skey = (uint32_t*)scratch(c, SC_KEYB, nn * 4);
  uint32_t* sidx = (uint32_t*)scratch(c, SC_VALB, nn * 4);
  uint32_t* mcnt = (uint32_t*)scratch(c, SC_MCNT, (size_t)g.nbrick * 4 * n_sp);
  int64_t* moff = (int64_t*)scratch(c, SC_MOFF, (size_t)(g.nbrick + 1) * 8);
  int32_t* part = (int32_t*)scratch(c, SC_PARTS, (size_t)g.nbrick * 8 * n_sp);
  if (!cnt || !off_new || !tpos || !tvel || !tdst || !mkey || !midx || !skey || !sidx ||
      !mcnt || !moff || !part)
    return PM_ERR_NOMEM;
  KickArgs A{};
  A.n_sp = n_sp;
  A.acc = acc;
  A.ck = (float)ck;
  A.cdS = cd * (double)g.S;
  for (int s = 0; s < n_sp; ++s) {
    KickSpecies& S = A.sp[s];
    S.n = in[s].n;
    S.pos = in[s].pos;
    S.vel = in[s].vel;
    S.hin = in[s].hdr;
    S.hout = out[s].hdr;
    S.off = offs[s];
    S.tpos = tpos + 3 * nbase[s];
    S.tvel = tvel + 3 * nbase[s];
    S.tdst = tdst + nbase[s];
    S.cnt = cnt + (int64_t)s * g.ncell3;
    S.mkey = mkey + nbase[s];
    S.midx = midx + nbase[s];
    S.mcnt = mcnt + (int64_t)s * g.nbrick;
    S.pmn = part + (int64_t)2 * s * g.nbrick;
    S.pmx = S.pmn + g.nbrick;
  }
  {
    pm_status st0;
    for (int s = 0; s < n_sp; ++s)
      hipLaunchKernelGGL(k_vmax_next, dim3(1), dim3(1), 0, c->stream, in[s].hdr, out[s].hdr,
                         amax, ck, in[s].n);
    ProfScope ps(c, ST_KICK);
    const int R1 = g.B * g.r + 1;
    const size_t fbytes = (size_t)3 * R1 * R1 * R1 * 4;
    const size_t tail =
        (size_t)MAXSP * (B3 + 1) * 8 + (size_t)(B3 + 1) * 4 * (2 + 2 * (KB / 64));
    const int R = g.B * g.r;
    if (R == 16 && fbytes + tail <= 96 * 1024)
      hipLaunchKernelGGL(k_kick_brick<16>, dim3((unsigned)g.nbrick), dim3(KB),
                         ((fbytes + 7) / 8) * 8 + tail, c->stream, A, g, c->err);
    else if (R == 8)
      hipLaunchKernelGGL(k_kick_brick<8>, dim3((unsigned)g.nbrick), dim3(KB),
                         ((fbytes + 7) / 8) * 8 + tail, c->stream, A, g, c->err);
    else
      hipLaunchKernelGGL(k_kick_brick<0>, dim3((unsigned)g.nbrick), dim3(KB), tail,
                         c->stream, A, g, c->err);
    PM_LAUNCH_CHECK();
    prof_end(c);  // the scope covers the brick kernel only
    for (int s = 0; s < n_sp; ++s)
      if ((st0 = fold_minmax_to_header(c, A.sp[s].pmn, A.sp[s].pmx, g.nbrick, out[s].hdr)) !=
          PM_OK)
        return st0;
  }
  for (int s = 0; s < n_sp; ++s) {
    const int64_t n = in[s].n;
    const KickSpecies& S = A.sp[s];
    ProfScope ps(c, ST_RESORT);
    pm_status st = scan_u32(c, S.mcnt, g.nbrick, moff);
    if (st != PM_OK) return st;
    // the mover count is data dependent: read it back (one small synchronisation)
    int64_t nm = 0;
    PM_HIP_CHECK(hipMemcpyAsync(&nm, moff + g.nbrick, 8, hipMemcpyDeviceToHost, c->stream));
    PM_HIP_CHECK(hipStreamSynchronize(c->stream));
    uint32_t* sk = skey + nbase[s];
    uint32_t* si = sidx + nbase[s];
    if (nm > 0) {
      hipLaunchKernelGGL(k_compact_movers, dim3((unsigned)g.nbrick), dim3(KT), 0, c->stream,
                         S.off, S.mcnt, moff, B3, S.mkey, S.midx, sk, si);
      PM_LAUNCH_CHECK();
      // stable sort (old order preserved inside each new cell)
      uint32_t *k1 = sk, *v1 = si, *k2 = S.mkey, *v2 = S.midx;
      st = radix_sort_pairs(c, &k1, &v1, &k2, &v2, nm, 3 * (g.lgB + g.lgnb));
      if (st != PM_OK) return st;
      sk = k1;
      si = v1;
      hipLaunchKernelGGL(k_arrivals, dim3((unsigned)cdiv(nm, KT)), dim3(KT), 0, c->stream, sk,
                         si, nm, S.off, B3, S.cnt);
      PM_LAUNCH_CHECK();
    }
    st = scan_u64lo(c, S.cnt, g.ncell3, off_new);
    if (st != PM_OK) return st;
    int64_t* pm = perm ? perm[s] : nullptr;
    hipLaunchKernelGGL(k_place_stayers, dim3((unsigned)g.nbrick), dim3(KT),
                       (size_t)B3 * 8, c->stream,
                       S.off, S.tdst, S.tpos, S.tvel, S.cnt, off_new, B3, out[s].pos,
                       out[s].vel, pm, n, c->err);
    PM_LAUNCH_CHECK();
    if (nm > 0) {
      hipLaunchKernelGGL(k_place_movers, dim3((unsigned)cdiv(nm, KT)), dim3(KT), 0, c->stream,
                         sk, si, nm, S.tpos, S.tvel, S.cnt, off_new, out[s].pos, out[s].vel,
                         pm, n, c->err);
      PM_LAUNCH_CHECK();
    }
    st = run_finalize_counts(c, nullptr, S.cnt, &out[s]);
    if (st != PM_OK) return st;
  }
  return PM_OK;
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

// FFT solution of the Poisson equation (Sec. 2.1, eqs. (1)-(3)) on a periodic mesh.
//
// The paper transforms each tile with three threaded 1-D FFTW calls, one per
// dimension (Sec. 2.3). Here every axis pass is one HBM pass over the mesh, and the
// kernel multiply is fused into the z pass; the potential of a step takes these sweeps:
//   X  r2c      rho(x) -> rho~(kx)                     rows; Nyquist column kx = n/2
//                                                      kept in a side plane
//   Y  fwd      -> rho~(kx, ky)                        columns, in place
//   Z  fused    forward z FFT, multiply by G(|k|^2) (softened kernel table), inverse z
//               FFT, in place
//   Y  inv      columns, in place
//   X  c2r      phi(x), real
// and the force a = -D phi (eq. (3)), D the fourth-order central difference, is one
// stencil pass over phi (k_grad4) that also takes max |a| for the velocity bound of the
// re-encode: 6 launches moving 52 n^3 bytes. The stencil is the exact real-space form of
// the spectral factor -i D(k_a), D(k) its symbol (which is zero on the Nyquist index).
// The transposed force (adjoint) applies that factor in the spectrum, in the y and z
// passes. The 1/n^3 of the inverse transform is folded into the kernel table.
//
// A line of N points is transformed as N = T x E (four-step): each of T threads holds
// E points strided by T, does an E-point DFT in registers, multiplies by twiddles,
// exchanges through LDS, and finishes with T-point DFTs in registers. Column passes
// give each workgroup W adjacent columns so that every global access is a W x 8 byte
// run; row passes give each workgroup several whole rows.
#include <type_traits>

#include "pm_common.h"

namespace {

// ------------------------------------------------------ compile-time twiddles --
constexpr double kPi = 3.141592653589793238462643383279502884;

constexpr double taylor_sin(double y) {
  double term = y, s = y;
  for (int i = 1; i < 30; ++i) {
    term *= -y * y / ((2.0 * i) * (2.0 * i + 1.0));
    s += term;
  }
  return s;
}
constexpr double taylor_cos(double y) {
  double term = 1.0, s = 1.0;
  for (int i = 1; i < 30; ++i) {
    term *= -y * y / ((2.0 * i - 1.0) * (2.0 * i));
    s += term;
  }
  return s;
}
// cos and sin of the angle 2 pi k / m, exact at multiples of pi/2.
constexpr double turn_cos(long k, long m) {
  k %= m;
  if (k < 0) k += m;
  long q = (4 * k) / m, rem = 4 * k - q * m;
  double y = (kPi / 2) * (double)rem / (double)m;
  double s = taylor_sin(y), c = taylor_cos(y);
  return q == 0 ? c : q == 1 ? -s : q == 2 ? -c : s;
}
constexpr double turn_sin(long k, long m) {
  k %= m;
  if (k < 0) k += m;
  long q = (4 * k) / m, rem = 4 * k - q * m;
  double y = (kPi / 2) * (double)rem / (double)m;
  double s = taylor_sin(y), c = taylor_cos(y);
  return q == 0 ? s : q == 1 ? c : q == 2 ? -s : -c;
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }
constexpr int bitrev(int i, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
  return r;
}

template <int I, int N>
struct SFor {
  template <typename F>
  __device__ __forceinline__ static void run(F&& f) {
    if constexpr (I < N) {
      f(std::integral_constant<int, I>{});
      SFor<I + 1, N>::run(f);
    }
  }
};

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// In-register DFT of M points (natural order in and out); SIGN = -1 forward,
// +1 inverse (unnormalised). Radix-2 decimation in frequency, twiddles are
// compile-time constants.
template <int M, int SIGN>
__device__ __forceinline__ void dft_reg(float2* a) {
  if constexpr (M > 1) {
    constexpr int L = ilog2(M);
    SFor<0, L>::run([&](auto s_) {
      constexpr int s = decltype(s_)::value;
      constexpr int len = M >> s, half = len >> 1;
      SFor<0, M / 2>::run([&](auto b_) {
        constexpr int b = decltype(b_)::value;
        constexpr int blk = b / half, j = b % half;
        constexpr int i0 = blk * len + j, i1 = i0 + half;
        float2 u = a[i0], w = a[i1];
        a[i0] = make_float2(u.x + w.x, u.y + w.y);
        float dx = u.x - w.x, dy = u.y - w.y;
        if constexpr (j == 0) {
          a[i1] = make_float2(dx, dy);
        } else if constexpr (4 * j == len) {
          // exp(SIGN 2 pi i / 4) = SIGN i: a swap, no multiply (the products by the
          // table's 0 and 1 are kept by IEEE rules otherwise)
          a[i1] = SIGN < 0 ? make_float2(dy, -dx) : make_float2(-dy, dx);
        } else if constexpr (8 * j == len || 8 * j == 3 * len) {
          // w = exp(SIGN 2 pi i j / len) = h (1 + SIGN i) at 45 degrees, h (-1 + SIGN i)
          // at 135, h = 1/sqrt(2): (dx + i dy) w from p = dx - SIGN dy, q = dy + SIGN dx
          constexpr float h = (float)turn_sin(1, 8);
          const float p = SIGN < 0 ? dx + dy : dx - dy, q = SIGN < 0 ? dy - dx : dy + dx;
          if constexpr (8 * j == len) a[i1] = make_float2(h * p, h * q);
          else a[i1] = SIGN < 0 ? make_float2(h * q, -h * p) : make_float2(-h * q, h * p);
        } else {
          constexpr float wr = (float)turn_cos(j, len);
          constexpr float wi = (float)(SIGN * turn_sin(j, len));
          a[i1] = make_float2(dx * wr - dy * wi, dx * wi + dy * wr);
        }
      });
    });
    float2 t[M];
    SFor<0, M>::run([&](auto i_) {
      constexpr int i = decltype(i_)::value;
      t[i] = a[bitrev(i, L)];
    });
    SFor<0, M>::run([&](auto i_) {
      constexpr int i = decltype(i_)::value;
      a[i] = t[i];
    });
  }
}

template <int N>
struct Plan {
  static constexpr int LG = ilog2(N);
  static constexpr int T = 1 << (LG / 2);  // threads per line
  static constexpr int E = N / T;          // points per thread in the natural layout
  static constexpr int V = E / T;          // virtual threads per thread (1 or 2)
  static constexpr int TP = T + 1;         // padded LDS row
};

// LDS exchange buffer accessor for one line: element (k1, t) at base + k1*TP + t.
// Natural layout: thread t holds a[n1] = x[t + T n1], n1 < E.
// Transposed layout: thread t holds b[v*T + k2] = X[(t + T v) + E k2], v < V, k2 < T.
//
// nat_to_tr: N-point DFT (SIGN) of a line held in natural layout, result in transposed
// layout. tw: table exp(-2 pi i j / n) with stride `tws` = n / N.
template <int N, int SIGN>
__device__ __forceinline__ void nat_to_tr(float2 (&a)[Plan<N>::E], int t, float* lds,
                                          const float2* __restrict__ tw, int tws,
                                          int twmask) {
  using P = Plan<N>;
  // scheduling fences: without them the fully unrolled passes hoist every twiddle load
  // of the kernel to its start and run out of registers
  __builtin_amdgcn_sched_barrier(0);
  dft_reg<P::E, SIGN>(a);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int k1 = 1; k1 < P::E; ++k1) {
    float2 w = tw[((t * k1) * tws) & twmask];
    a[k1] = (SIGN < 0) ? cmul(a[k1], w) : cmulc(a[k1], w);
  }
  // exchange real parts, then imaginary parts (halves the LDS footprint); the array is
  // reused in place: a part is dead once it is in LDS
#pragma unroll
  for (int part = 0; part < 2; ++part) {
#pragma unroll
    for (int k1 = 0; k1 < P::E; ++k1) lds[k1 * P::TP + t] = part ? a[k1].y : a[k1].x;
    __syncthreads();
#pragma unroll
    for (int v = 0; v < P::V; ++v)
#pragma unroll
      for (int k2 = 0; k2 < P::T; ++k2) {
        float q = lds[(t + P::T * v) * P::TP + k2];
        if (part) a[v * P::T + k2].y = q; else a[v * P::T + k2].x = q;
      }
    __syncthreads();
  }
#pragma unroll
  for (int v = 0; v < P::V; ++v) dft_reg<P::T, SIGN>(&a[v * P::T]);
}

// tr_to_nat: N-point DFT (SIGN) of a line held in transposed layout, result in natural
// layout.
template <int N, int SIGN>
__device__ __forceinline__ void tr_to_nat(float2 (&b)[Plan<N>::E], int t, float* lds,
                                          const float2* __restrict__ tw, int tws,
                                          int twmask) {
  using P = Plan<N>;
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int v = 0; v < P::V; ++v) {
    dft_reg<P::T, SIGN>(&b[v * P::T]);
    __builtin_amdgcn_sched_barrier(0);
    const int k1 = t + P::T * v;
#pragma unroll
    for (int n1 = 1; n1 < P::T; ++n1) {
      float2 w = tw[((n1 * k1) * tws) & twmask];
      b[v * P::T + n1] = (SIGN < 0) ? cmul(b[v * P::T + n1], w) : cmulc(b[v * P::T + n1], w);
    }
  }
#pragma unroll
  for (int part = 0; part < 2; ++part) {
#pragma unroll
    for (int v = 0; v < P::V; ++v)
#pragma unroll
      for (int n1 = 0; n1 < P::T; ++n1) {
        float2 q = b[v * P::T + n1];
        lds[(t + P::T * v) * P::TP + n1] = part ? q.y : q.x;
      }
    __syncthreads();
#pragma unroll
    for (int k1 = 0; k1 < P::E; ++k1) {
      float q = lds[k1 * P::TP + t];
      if (part) b[k1].y = q; else b[k1].x = q;
    }
    __syncthreads();
  }
  dft_reg<P::E, SIGN>(b);
}

// ------------------------------------------------------------ spectrum layout --
// The half spectrum (kx < n/2, M = n/2 complex per row) is stored z-blocked:
//   index(kx, y, z) = ((z / ZB) n + y) ZB M + (z % ZB) M + kx,   ZB = min(16, T(n)),
// and ZB = 64 for split lines (2048 points, where a line's natural point stride is 64),
// so that a z line visits n / ZB address blocks of ZB consecutive rows instead of n
// blocks 4 n M bytes apart (one address translation per ZB points), while y lines keep
// runs of W kx at a stride of ZB M. The Nyquist plane kx = n/2 is a separate [z][y]
// array. T(n) is the four-step split of an n-point line, so ZB divides T and E.
__host__ __device__ constexpr int zblk(int n) {
  if (n >= 2048) return 64;  // split lines: the natural point stride H T = 64
  int t = 1 << (ilog2(n) / 2);
  return t < 16 ? t : 16;
}

// ------------------------------------------------------------- column passes --
// Lines l = (l1, l2): element e of line l at
//   base = l1 s1 + (l2 >> sh2) s2h + (l2 & (2^sh2 - 1)) s2l
//   element e: e es, or for z-blocked lines (e / ZB) es + (e % ZB) esl
// (complex units). A workgroup takes W consecutive l1 (s1 = 1 gives W*8-byte runs) and
// one l2.
struct Lines {
  int64_t s1, s2h, s2l;
  int sh2;
  int64_t es, esl;
  int64_t L1;      // number of l1 values
  int kx_mode;     // 0: kx = l1; 1: kx = kx_fixed
  int ky_mode;     // 0: ky = l2; 1: ky = l1
  int kx_fixed;
};

__device__ __forceinline__ int64_t line_base(const Lines& d, int64_t l1, int64_t l2) {
  return l1 * d.s1 + (l2 >> d.sh2) * d.s2h + (l2 & ((1 << d.sh2) - 1)) * d.s2l;
}

template <int W>
constexpr int col_cs(int per_col) {  // padded per-column stride, spreads LDS banks
  int want = 32 / W;
  int r = per_col % 32;
  return per_col + ((want - r) % 32 + 32) % 32;
}

__device__ __forceinline__ int signed_k(int k, int n) { return k < n / 2 ? k : k - n; }
// The gradient symbol of eq. (3) on the mesh: D(k) = (8 sin(k Delta) - sin(2 k Delta)) /
// (6 Delta), the fourth-order central difference (zero on the Nyquist index), from the
// context's table gk[k], k < n (built in float64 on the host).
__device__ __forceinline__ float grad_k(const float* __restrict__ gk, int k) { return gk[k]; }

// ------------------------------------------------------------- line plans --
// A column line of N points is held by H groups of T threads: H = 1 below 2048 points
// (the four-step engine above on the whole line), H = 2 at 2048 points, where the even
// and odd points are two lines of N/2 on their own thread groups (half the registers per
// thread), joined by one radix-2 step through LDS. Natural layout: thread (t, h) holds
// point H (t + T n1) + h, n1 < E; transposed layout: value v T + k2 is frequency
// (t + T v) + E k2 + h N/2.
template <int N>
struct LP {
  static constexpr int H = N >= 2048 ? 2 : 1;
  static constexpr int NH = N / H;
  using P = Plan<NH>;
  static constexpr int T = P::T, E = P::E, V = P::V, TP = P::TP;
  static constexpr int TL = H * T;          // threads per line
  static constexpr int LF = H * E * TP;     // LDS floats per line
};

// Radix-2 step of a split line (H = 2). After the half-length transforms thread (t, h)
// holds values of its half's spectrum at frequencies k = (t + T v) + E k2; the partner
// (t, 1 - h) holds the same k of the other half. Real parts, then imaginary parts, go
// through the line's LDS; w = exp(SIGN 2 pi i k / N).
//   DIF = false (forward, after the half transforms): X[k] = Y0 + w Y1 on h = 0,
//                X[k + N/2] = Y0 - w Y1 on h = 1;
//   DIF = true  (before the half inverse transforms): Y0 = X[k] + X[k + N/2] on h = 0,
//                Y1 = (X[k] - X[k + N/2]) w on h = 1.
template <int N, int SIGN, bool DIF>
__device__ __forceinline__ void split_radix2(float2 (&a)[LP<N>::E], int t, int h, float* my,
                                             const float2* __restrict__ tw, int tws,
                                             int twmask) {
  using L = LP<N>;
  float* mine = my + h * (L::E * L::TP);
  const float* other = my + (1 - h) * (L::E * L::TP);
  float pre[L::E];
#pragma unroll
  for (int q = 0; q < L::E; ++q) mine[q * L::TP + t] = a[q].x;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < L::E; ++q) pre[q] = other[q * L::TP + t];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < L::E; ++q) mine[q * L::TP + t] = a[q].y;
  __syncthreads();
#pragma unroll
  for (int v = 0; v < L::V; ++v)
#pragma unroll
    for (int k2 = 0; k2 < L::T; ++k2) {
      const int q = v * L::T + k2;
      const int k = (t + L::T * v) + L::E * k2;
      const float2 pp = make_float2(pre[q], other[q * L::TP + t]);
      float2 w = tw[(k * tws) & twmask];  // exp(-2 pi i k / N)
      if (SIGN > 0) w.y = -w.y;
      if (!DIF) {
        if (h == 0) {
          const float2 z = cmul(w, pp);
          a[q] = make_float2(a[q].x + z.x, a[q].y + z.y);
        } else {
          const float2 z = cmul(w, a[q]);
          a[q] = make_float2(pp.x - z.x, pp.y - z.y);
        }
      } else {
        if (h == 0) a[q] = make_float2(a[q].x + pp.x, a[q].y + pp.y);
        else a[q] = cmul(make_float2(pp.x - a[q].x, pp.y - a[q].y), w);
      }
    }
  __syncthreads();
}

// Thread (c, t, h) of a column workgroup: column c < W, line thread t < T, half h:
// c = tid mod W, (t, h) = (tl mod T, tl / T) for tl = tid / W.
template <int N, int W>
__device__ __forceinline__ void col_thread(int& c, int& t, int& h) {
  using L = LP<N>;
  c = threadIdx.x % W;
  const int tl = threadIdx.x / W;
  t = tl % L::T;
  h = tl / L::T;
}

// Line transforms on the plan: natural -> transposed (forward or inverse) and
// transposed -> natural. tw: table exp(-2 pi i j / n) of the full line, stride tws.
template <int N, int SIGN>
__device__ __forceinline__ void line_nat_to_tr(float2 (&a)[LP<N>::E], int t, int h, float* my,
                                               const float2* __restrict__ tw, int tws,
                                               int twmask) {
  using L = LP<N>;
  if constexpr (L::H == 1) {
    nat_to_tr<N, SIGN>(a, t, my, tw, tws, twmask);
  } else {
    nat_to_tr<L::NH, SIGN>(a, t, my + h * (L::E * L::TP), tw, 2 * tws, twmask);
    split_radix2<N, SIGN, false>(a, t, h, my, tw, tws, twmask);
  }
}
template <int N, int SIGN>
__device__ __forceinline__ void line_tr_to_nat(float2 (&a)[LP<N>::E], int t, int h, float* my,
                                               const float2* __restrict__ tw, int tws,
                                               int twmask) {
  using L = LP<N>;
  if constexpr (L::H == 1) {
    tr_to_nat<N, SIGN>(a, t, my, tw, tws, twmask);
  } else {
    split_radix2<N, SIGN, true>(a, t, h, my, tw, tws, twmask);
    tr_to_nat<L::NH, SIGN>(a, t, my + h * (L::E * L::TP), tw, 2 * tws, twmask);
  }
}

// Workgroups go round-robin over the chip's 8 XCDs (each with its own L2). A workgroup of
// W < 16 split-line columns reads and writes 8W-byte parts of 128-byte runs; the tile
// order below gives the G = 16 / W tiles Gi .. Gi + G - 1 of a run to the blocks
// 8Ga + 8b + r, b < G (r = i mod 8, a = i / 8), which run on the same XCD at about the
// same time, so that one L2 serves the whole run. A bijection of [0, gx) when 8G divides
// gx (else the identity).
template <int G>
__device__ __forceinline__ unsigned xcd_group(unsigned x, unsigned gx) {
  if (G == 1 || gx % (8u * G)) return x;
  const unsigned a = x / (8u * G), b = (x / 8u) % G, r = x % 8u;
  return (8u * G) * a + G * r + b;
}
template <int N, int W>
constexpr int col_group() { return LP<N>::H == 2 && W < 16 ? 16 / W : 1; }

// Generic c2c column FFT. OUT 0: out0 = FFT_SIGN(in). OUT 3 (y lines of the transposed
// force): out0 = +i k_x FFT_SIGN(in) + i k(e) FFT_SIGN(in1), k(e) the line's own wave
// number, k_x constant along a y line. With two lines per thread the twiddles are staged
// in LDS (32-bit addresses), which keeps both line arrays in registers without spilling.
template <int N, int W, int SIGN, int OUT>
__global__ __launch_bounds__(W * LP<N>::TL) void k_col_fft(const float2* in,
                                                           const float2* in1, float2* out0,
                                                           float2* out1, Lines d,
                                                           const float2* __restrict__ tw,
                                                           int tws, int twmask, int n,
                                                           const float* __restrict__ gk) {
  using L = LP<N>;
  constexpr int CS = col_cs<W>(L::LF);
  __shared__ float lds[W * CS];
  constexpr bool TWO = OUT == 3;
  // Split lines stage their twiddles as well: at 1024 threads (128 VGPRs) the compiler
  // issues the global twiddle loads one at a time, each waited for (y passes at 2048^3)
  constexpr bool STW = TWO || L::H == 2;
  __shared__ float2 stw[STW ? N : 1];
  if constexpr (STW) {
    for (int i = threadIdx.x; i < N; i += W * L::TL) stw[i] = tw[(i * tws) & twmask];
    __syncthreads();
  }
  const unsigned bx = xcd_group<col_group<N, W>()>(blockIdx.x, gridDim.x);
  // the grid covers the lines exactly (W divides the line count; checked on the host)
  int c, t, h;
  col_thread<N, W>(c, t, h);
  // addresses: a workgroup-uniform 64-bit part plus a 32-bit per-thread offset
  const int64_t ubase = line_base(d, (int64_t)bx * W, blockIdx.y);
  const int e0 = L::H * t + h;  // natural point of n1 = 0; point n1 is e0 + H T n1
  const uint32_t lo_in = (uint32_t)(c * d.s1 + (int64_t)e0 * d.es);
  // transposed frequency (t + T v) + E k2 + h N/2: per-thread part and k2 stride
  auto lo_out = [&](int v) {
    return (uint32_t)(c * d.s1 + (int64_t)((t + L::T * v) + h * L::NH) * d.es);
  };
  float* my = lds + c * CS;
  float2 a[L::E];
#pragma unroll
  for (int n1 = 0; n1 < L::E; ++n1)
    a[n1] = (in + (ubase + (int64_t)L::H * L::T * n1 * d.es))[lo_in];
  if constexpr (OUT == 3) {
    float2 b[L::E];
#pragma unroll
    for (int n1 = 0; n1 < L::E; ++n1)
      b[n1] = (in1 + (ubase + (int64_t)L::H * L::T * n1 * d.es))[lo_in];
    line_nat_to_tr<N, SIGN>(a, t, h, my, stw, 1, N - 1);
    line_nat_to_tr<N, SIGN>(b, t, h, my, stw, 1, N - 1);
    const float kxg = grad_k(gk, d.kx_mode ? d.kx_fixed : (int)(bx * W) + c);
#pragma unroll
    for (int v = 0; v < L::V; ++v)
#pragma unroll
      for (int k2 = 0; k2 < L::T; ++k2) {
        const float kyg = grad_k(gk, (t + L::T * v) + L::E * k2 + h * L::NH);
        const float2 q = a[v * L::T + k2], p = b[v * L::T + k2];
        // + i (k_x q + k_y p)
        a[v * L::T + k2] = make_float2(-(kxg * q.y + kyg * p.y), kxg * q.x + kyg * p.x);
      }
#pragma unroll
    for (int v = 0; v < L::V; ++v)
#pragma unroll
      for (int k2 = 0; k2 < L::T; ++k2)
        (out0 + (ubase + (int64_t)L::E * k2 * d.es))[lo_out(v)] = a[v * L::T + k2];
  } else {
    if constexpr (STW) line_nat_to_tr<N, SIGN>(a, t, h, my, stw, 1, N - 1);
    else line_nat_to_tr<N, SIGN>(a, t, h, my, tw, tws, twmask);
#pragma unroll
    for (int v = 0; v < L::V; ++v)
#pragma unroll
      for (int k2 = 0; k2 < L::T; ++k2)
        (out0 + (ubase + (int64_t)L::E * k2 * d.es))[lo_out(v)] = a[v * L::T + k2];
  }
}

// ---------------------------------------------------------------- fused z pass --
// F = FFT_z(in0) per line, then MODE 0: out0 = IFFT_z(G F) (the potential's spectrum);
// MODE 1 (transpose of the force): out0 = IFFT_z(G (FFT_z(in0) + i k_z FFT_z(in2))),
// where in0 already holds the x and y terms +i (k_x mu_x + k_y mu_y) from the y pass. BLK: the
// lines are z-blocked (main spectrum) or plain strided (Nyquist plane).
template <int N, int W, int MODE, bool BLK>
__global__ __launch_bounds__(W * LP<N>::TL) void k_col_zconv(
    const float2* in0, const float2* in1, const float2* in2, float2* out0, float2* out1,
    Lines d,
    const float2* __restrict__ tw, int tws, int twmask, int n,
    const float* __restrict__ gtab, const float* __restrict__ gk) {
  using L = LP<N>;
  constexpr int ZB = zblk(N), LZB = ilog2(ZB);
  static_assert((L::H * L::T) % ZB == 0, "z blocks must divide the thread stride");
  constexpr int CS = col_cs<W>(L::LF);
  __shared__ float lds[W * CS];
  // the line's twiddles exp(-2 pi i j / N) in LDS: 32-bit LDS addresses instead of
  // 64-bit global pointers per twiddle, which the two line arrays of MODE 1 would
  // otherwise keep live together
  __shared__ float2 stw[N];
  for (int i = threadIdx.x; i < N; i += W * L::TL) stw[i] = tw[(i * tws) & twmask];
  // the gradient symbol too (shared by the workgroup's lines): loaded from global memory
  // next to the kernel values, the compiler waits for its loads one by one
  __shared__ float sgk[N];
  for (int i = threadIdx.x; i < N; i += W * L::TL) sgk[i] = gk[i];
  __syncthreads();
  const unsigned bx = xcd_group<col_group<N, W>()>(blockIdx.x, gridDim.x);
  int c, t, h;
  col_thread<N, W>(c, t, h);
  const int64_t l1 = (int64_t)bx * W + c;
  // point e0 + H T n1 of the line (e0 = H t + h): z-blocked lines split it as (block,
  // row in block). Addresses are a workgroup-uniform 64-bit part (scalar registers) plus
  // a 32-bit per-thread offset, so that no 64-bit address per point stays live in VGPRs.
  const int64_t ubase = line_base(d, (int64_t)bx * W, blockIdx.y);
  const int e0 = L::H * t + h;
  const uint32_t toff =
      (uint32_t)(c * d.s1 + (BLK ? (int64_t)(e0 >> LZB) * d.es + (int64_t)(e0 & (ZB - 1)) * d.esl
                                 : (int64_t)e0 * d.es));
  const int64_t step = BLK ? (int64_t)((L::H * L::T) >> LZB) * d.es
                           : (int64_t)L::H * L::T * d.es;
  float* my = lds + c * CS;
  const int kx = d.kx_mode ? d.kx_fixed : (int)l1;
  const int ky = d.ky_mode ? (int)l1 : (int)blockIdx.y;
  const int sx = signed_k(kx, n), sy = signed_k(ky, n);
  // kernel values of this line: gtab row (|kx|, |ky|), indexed by |kz|
  const int h1 = n / 2 + 1;
  const float* __restrict__ grow =
      gtab + ((int64_t)(sx < 0 ? -sx : sx) * h1 + (sy < 0 ? -sy : sy)) * h1;
  float2 acc[L::E];
  if constexpr (MODE == 0) {
#pragma unroll
    for (int n1 = 0; n1 < L::E; ++n1) acc[n1] = (in0 + (ubase + n1 * step))[toff];
    line_nat_to_tr<N, -1>(acc, t, h, my, stw, 1, N - 1);
#pragma unroll
    for (int v = 0; v < L::V; ++v)
#pragma unroll
      for (int k2 = 0; k2 < L::T; ++k2) {
        const int kz = (t + L::T * v) + L::E * k2 + h * L::NH;
        const int sz = signed_k(kz, n);
        const float G = grow[sz < 0 ? -sz : sz];
        const float2 f = acc[v * L::T + k2];
        acc[v * L::T + k2] = make_float2(G * f.x, G * f.y);
      }
    line_tr_to_nat<N, +1>(acc, t, h, my, stw, 1, N - 1);
#pragma unroll
    for (int n1 = 0; n1 < L::E; ++n1) (out0 + (ubase + n1 * step))[toff] = acc[n1];
  } else {
    // sum_a (+i k_a) FFT_z(in_a): the x and y terms arrive summed in in0; k_z multiplies
    // after FFT_z(in2)
#pragma unroll
    for (int n1 = 0; n1 < L::E; ++n1) acc[n1] = (in2 + (ubase + n1 * step))[toff];
    line_nat_to_tr<N, -1>(acc, t, h, my, stw, 1, N - 1);
#pragma unroll
    for (int v = 0; v < L::V; ++v)
#pragma unroll
      for (int k2 = 0; k2 < L::T; ++k2) {
        const float k = sgk[(t + L::T * v) + L::E * k2 + h * L::NH];
        const float2 q = acc[v * L::T + k2];
        acc[v * L::T + k2] = make_float2(-k * q.y, k * q.x);  // + i k (x + i y)
      }
    float2 f[L::E];
#pragma unroll
    for (int n1 = 0; n1 < L::E; ++n1) f[n1] = (in0 + (ubase + n1 * step))[toff];
    line_nat_to_tr<N, -1>(f, t, h, my, stw, 1, N - 1);
#pragma unroll
    for (int v = 0; v < L::V; ++v)
#pragma unroll
      for (int k2 = 0; k2 < L::T; ++k2) {
        const int kz = (t + L::T * v) + L::E * k2 + h * L::NH;
        const int sz = signed_k(kz, n);
        const float G = grow[sz < 0 ? -sz : sz];
        const float2 q = acc[v * L::T + k2], p = f[v * L::T + k2];
        acc[v * L::T + k2] = make_float2(G * (q.x + p.x), G * (q.y + p.y));
      }
    line_tr_to_nat<N, +1>(acc, t, h, my, stw, 1, N - 1);
#pragma unroll
    for (int n1 = 0; n1 < L::E; ++n1) (out0 + (ubase + n1 * step))[toff] = acc[n1];
  }
}

// ----------------------------------------------------------------- row passes --
// A real row of n = 2M floats is the complex row z[m] = x[2m] + i x[2m+1] of M points.
// Workgroup: R rows x T threads, threads of a row consecutive (coalesced rows). Real
// rows are in natural order (row = z n + y); spectrum rows are z-blocked.
template <int M>
__device__ __forceinline__ int64_t spec_row(int64_t row) {
  constexpr int n = 2 * M, ZB = zblk(n), LZB = ilog2(ZB), LN = ilog2(n);
  const int64_t z = row >> LN, y = row & (n - 1);
  return (((z >> LZB) << LN) + y) * ((int64_t)ZB * M) + (z & (ZB - 1)) * M;
}
// The inverse row pass visits rows in the spectrum's storage order: index s = ((z / ZB)
// n + y) ZB + z % ZB, so the spectrum rows of consecutive workgroups are one contiguous
// run and their real rows a few runs in each of ZB planes (instead of rows ZB M complex
// apart across a whole z block of the spectrum): 17.9 -> 17.5 ms per launch at 2048^3.
// The forward pass keeps the natural order (its spectrum writes are not slowed by the
// stride, and the planes' runs slowed it 15.0 -> 16.4 ms). Returns the natural row
// z n + y of s.
template <int M>
__device__ __forceinline__ int64_t row_of(int64_t s) {
  constexpr int n = 2 * M, ZB = zblk(n), LZB = ilog2(ZB), LN = ilog2(n);
  const int64_t zl = s & (ZB - 1), t2 = s >> LZB;
  const int64_t y = t2 & (n - 1), zb = t2 >> LN;
  return ((zb << LZB) + zl) * n + y;
}

// rows per workgroup of the row passes: up to 256 threads, and LDS for the FFT exchange
// only (the pairing of k with M - k goes through lane shuffles)
template <int M>
constexpr int rows_per_wg() {
  constexpr int T = Plan<M>::T;
  int r = 256 / T;
  if (r > 16) r = 16;
  int lim = 20480 / (Plan<M>::E * Plan<M>::TP);
  if (r > lim) r = lim;
  return r < 1 ? 1 : r;
}

// X r2c: in real rows (nrows x n floats) -> out main rows (M complex) + nyq[row]. The
// spectrum is written in the transposed order the FFT leaves it in (runs of T complex),
// and the post-process pairs Z[k] with Z[M - k] by lane shuffles, so that the LDS holds
// only the FFT exchange.
template <int M>
__global__ __launch_bounds__(rows_per_wg<M>() * Plan<M>::T) void k_row_r2c(
    const float* in, float2* out, float2* nyq, int64_t nrows, const float2* __restrict__ tw,
    int twmask) {
  using P = Plan<M>;
  constexpr int R = rows_per_wg<M>();
  constexpr int LF = P::E * P::TP;
  __shared__ float lds[R * LF];
  // the twiddles in LDS: from global memory the compiler issues most of them one at a
  // time, each waited for (13.2 against 14.5 ms at 2048^3)
  __shared__ float2 stw[2 * M];
  for (int i = threadIdx.x; i < 2 * M; i += R * P::T) stw[i] = tw[i];
  __syncthreads();
  // R divides the row count (checked on the host): no bounds guards
  const int t = threadIdx.x % P::T, rr = threadIdx.x / P::T;
  const int64_t row = (int64_t)blockIdx.x * R + rr;  // natural order (faster here)
  float* my = lds + rr * LF;
  const float2* zin = (const float2*)(in + row * 2 * M);
  float2 a[P::E];
#pragma unroll
  for (int n1 = 0; n1 < P::E; ++n1) a[n1] = zin[t + P::T * n1];
  // M-point DFT: tw table is for n = 2M points, stride 2
  nat_to_tr<M, -1>(a, t, my, stw, 2, twmask);
  // a[v T + k2] = Z[k], k = (t + T v) + E k2. Z[M - k] is held by lane (T - t) of the
  // row's lane group at index (V - 1 - v) T + (T - 1 - k2); lane t = 0 holds it itself,
  // at index (V - v) T + (T - 1 - k2) for v >= 1 and (T - k2) mod T for v = 0 (Z[M] =
  // Z[0]).
  const int src = ((int)(threadIdx.x & 63) & ~(P::T - 1)) | ((P::T - t) & (P::T - 1));
  float2* o = out + spec_row<M>(row);
  const float2 z0 = a[0];
#pragma unroll
  for (int v = 0; v < P::V; ++v)
#pragma unroll
    for (int k2 = 0; k2 < P::T; ++k2) {
      const int k = (t + P::T * v) + P::E * k2;
      const float2 zk = a[v * P::T + k2];
      const int ip = (P::V - 1 - v) * P::T + (P::T - 1 - k2);
      float2 zm = make_float2(__shfl(a[ip].x, src, 64), __shfl(a[ip].y, src, 64));
      if (t == 0) zm = v == 0 ? a[(P::T - k2) % P::T] : a[(P::V - v) * P::T + (P::T - 1 - k2)];
      // A = (Z[k] + conj Z[M-k]) / 2, B = -i (Z[k] - conj Z[M-k]) / 2, X = A + W^k B
      float2 A = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
      float2 B = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
      float2 w = stw[k];
      float2 wb = cmul(w, B);
      float2 X = make_float2(A.x + wb.x, A.y + wb.y);
      if (k == 0) X = make_float2(zk.x + zk.y, 0.f);
      o[k] = X;
    }
  if (t == 0) nyq[row] = make_float2(z0.x - z0.y, 0.f);
}

// X c2r: in main rows (M complex) + nyq[row] -> out real rows.
template <int M>
constexpr bool c2r_stw() { return M >= 1024; }
template <int M>
__global__ __launch_bounds__(rows_per_wg<M>() * Plan<M>::T) void k_row_c2r(
    const float2* in, const float2* nyq, float* out, int64_t nrows,
    const float2* __restrict__ tw, int twmask) {
  using P = Plan<M>;
  constexpr int R = rows_per_wg<M>();
  constexpr int LF = P::E * P::TP;
  __shared__ float lds[R * LF];
  // 2048-point rows: twiddles in LDS, as in the forward pass (14.3 -> 12.9 ms per launch
  // at 2048^3; smaller rows keep four workgroups per CU without them)
  constexpr bool STW = c2r_stw<M>();
  __shared__ float2 stw[STW ? 2 * M : 1];
  if constexpr (STW)
    for (int i = threadIdx.x; i < 2 * M; i += R * P::T) stw[i] = tw[i];
  const float2* __restrict__ twr = STW ? stw : tw;
  const int t = threadIdx.x % P::T, rr = threadIdx.x / P::T;
  const int64_t row = row_of<M>((int64_t)blockIdx.x * R + rr);
  float* my = lds + rr * LF;
  const float2* xi = in + spec_row<M>(row);
  const int n = 2 * M;
  float2 xr[P::E];
#pragma unroll
  for (int j = 0; j < P::E; ++j) xr[j] = xi[t + P::T * j];
  if constexpr (STW) __syncthreads();  // the staged twiddles
  float2 xn = make_float2(0.f, 0.f);  // X[M], held by lane t = 0
  if (t == 0) xn = nyq[row];
  // X[M - k] for k = t + T j: lane (T - t) of the row's lane group holds it at index
  // E - 1 - j; lane t = 0 holds it itself, at index E - j (X[M] for j = 0). The row's T
  // lanes are consecutive and T divides 64, so the partner is in the same wave.
  const int src = ((int)(threadIdx.x & 63) & ~(P::T - 1)) | ((P::T - t) & (P::T - 1));
  float2 a[P::E];
#pragma unroll
  for (int n1 = 0; n1 < P::E; ++n1) {
    const int k = t + P::T * n1;
    const float2 xk = xr[n1];
    float2 xm = make_float2(__shfl(xr[P::E - 1 - n1].x, src, 64),
                            __shfl(xr[P::E - 1 - n1].y, src, 64));
    if (t == 0) xm = n1 == 0 ? xn : xr[(P::E - n1) % P::E];
    // Z = (X[k] + conj X[M-k]) + i W^{-k} (X[k] - conj X[M-k])
    float2 s = make_float2(xk.x + xm.x, xk.y - xm.y);
    float2 dd = make_float2(xk.x - xm.x, xk.y + xm.y);
    float2 wd = cmulc(dd, twr[k]);  // W^{-k} d
    a[n1] = make_float2(s.x - wd.y, s.y + wd.x);
  }
  nat_to_tr<M, +1>(a, t, my, twr, 2, twmask);
  float2* zo = (float2*)(out + row * 2 * M);
#pragma unroll
  for (int v = 0; v < P::V; ++v)
#pragma unroll
    for (int k2 = 0; k2 < P::T; ++k2) zo[(t + P::T * v) + P::E * k2] = a[v * P::T + k2];
}

// ------------------------------------------------------------- force gradient --
// a_c = -D_c phi for the three axes c, D the fourth-order central difference of eq. (3)'s
// gradient: D f(x) = n (8 (f(x + 1) - f(x - 1)) - (f(x + 2) - f(x - 2))) / 12 (mesh
// spacing 1/n, periodic). Its Fourier symbol is i D(k) with the D(k) of the spectral
// form, so the components equal the three inverse transforms of -i D(k_c) G rho but take
// one transform of G rho and this pass. A workgroup owns a tile of GX x GY nodes of the
// (x, y) plane and walks GZ planes along z: each thread keeps a window of five z values
// of its RPT rows in registers (the z difference), and the current plane, with a halo of
// two nodes in x and y, is staged in LDS (the x and y differences). Writes the per-block
// max |a| (float bits) to part[block].
constexpr int GRAD_T = 256;
__global__ __launch_bounds__(GRAD_T) void k_grad4(const float* __restrict__ phi, float* ax,
                                                  float* ay, float* az, int lgn, int GX,
                                                  int GY, int GZ, float scale,
                                                  unsigned int* part) {
  constexpr int RPT = 8;  // rows of the tile per thread
  __shared__ float tile[(32 + 4) * (64 + 4)];
  __shared__ float wmax[GRAD_T / 64];
  const int64_t n = (int64_t)1 << lgn, n2 = n * n;
  const uint32_t m = (uint32_t)n - 1u;
  const int LX = GX + 4;                       // staged row length
  const int nty = (int)(n / GY), ntx = (int)(n / GX);
  const int bx = blockIdx.x % ntx, by = (blockIdx.x / ntx) % nty;
  const int bz = blockIdx.x / (ntx * nty);
  const int x0 = bx * GX, y0 = by * GY, z0 = bz * GZ;
  const int nthr = GX * GY / RPT;
  const int tid = threadIdx.x;
  const bool act = tid < nthr;
  const int lx = tid % GX, ly0 = tid / GX;     // rows ly0 + (GY / RPT) r
  const int ystep = GY / RPT;
  const uint32_t gx = (uint32_t)(x0 + lx);
  float w[RPT][5];  // phi at z - 2 .. z + 2 of the thread's rows
  auto at = [&](uint32_t x, uint32_t y, uint32_t z) {
    return phi[((int64_t)(z & m) * n + (y & m)) * n + (x & m)];
  };
  if (act) {
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
      for (int k = 0; k < 4; ++k)
        w[r][k + 1] = at(gx, (uint32_t)(y0 + ly0 + ystep * r), (uint32_t)(z0 - 2 + k));
  }
  float amx = 0.f;
  for (int dz = 0; dz < GZ; ++dz) {
    const uint32_t z = (uint32_t)(z0 + dz);
    // the window moves on by one plane: z + 2 comes in
    if (act) {
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
#pragma unroll
        for (int k = 0; k < 4; ++k) w[r][k] = w[r][k + 1];
        w[r][4] = at(gx, (uint32_t)(y0 + ly0 + ystep * r), z + 2);
      }
    }
    __syncthreads();  // the previous plane's tile has been read
    // plane z into LDS: the tile's own nodes from the windows, the halo from memory
    if (act) {
#pragma unroll
      for (int r = 0; r < RPT; ++r) tile[(ly0 + ystep * r + 2) * LX + lx + 2] = w[r][2];
    }
    const int nh = 4 * LX + 4 * GY;  // halo rows (2 above, 2 below) and halo columns
    for (int i = tid; i < nh; i += GRAD_T) {
      int ty, tx;
      if (i < 4 * LX) {
        const int hr = i / LX;
        ty = hr < 2 ? hr : GY + hr;  // rows 0, 1 and GY + 2, GY + 3
        tx = i % LX;
      } else {
        const int j = i - 4 * LX;
        ty = 2 + j / 4;
        const int hc = j % 4;
        tx = hc < 2 ? hc : GX + hc;  // columns 0, 1 and GX + 2, GX + 3
      }
      tile[ty * LX + tx] = at((uint32_t)(x0 - 2 + tx), (uint32_t)(y0 - 2 + ty), z);
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int ty = ly0 + ystep * r + 2, tx = lx + 2;
        const float* c = tile + ty * LX + tx;
        const float gxv = 8.f * (c[1] - c[-1]) - (c[2] - c[-2]);
        const float gyv = 8.f * (c[LX] - c[-LX]) - (c[2 * LX] - c[-2 * LX]);
        const float gzv = 8.f * (w[r][3] - w[r][1]) - (w[r][4] - w[r][0]);
        const float a0 = -scale * gxv, a1 = -scale * gyv, a2 = -scale * gzv;
        const int64_t o = (int64_t)z * n2 + (int64_t)(y0 + ly0 + ystep * r) * n + gx;
        ax[o] = a0;
        ay[o] = a1;
        az[o] = a2;
        amx = fmaxf(amx, fmaxf(fabsf(a0), fmaxf(fabsf(a1), fabsf(a2))));
      }
    }
  }
  for (int d = 32; d >= 1; d >>= 1) amx = fmaxf(amx, __shfl_xor(amx, d, 64));
  if ((tid & 63) == 0) wmax[tid >> 6] = amx;
  __syncthreads();
  if (tid == 0) {
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q) amx = fmaxf(amx, wmax[q]);
    part[blockIdx.x] = __float_as_uint(amx);
  }
}

// tile of the gradient pass at mesh side n: GX x GY nodes, GZ planes per workgroup
struct GradTile {
  int gx, gy, gz;
  int64_t blocks;
};
GradTile grad_tile(int64_t n) {
  GradTile t;
  t.gx = (int)std::min<int64_t>(n, 64);
  t.gy = (int)std::min<int64_t>(n, 32);
  t.gz = (int)std::min<int64_t>(n, 64);
  t.blocks = (n / t.gx) * (n / t.gy) * (n / t.gz);
  return t;
}

// ---------------------------------------------------------------- kernel table --
// K1(x) = int_0^inf exp(-x cosh s) cosh s ds by the trapezoidal rule, which converges
// exponentially fast for this analytic, doubly-exponentially decaying integrand.
__device__ double bessel_k1(double x) {
  const double h = 0.0625;
  double sum = 0.5 * exp(-x);
  for (int j = 1; j < 20000; ++j) {
    double s = j * h;
    double ch = cosh(s);
    double term = exp(-x * ch) * ch;
    sum += term;
    if (term < 1e-19 * sum) break;
  }
  return sum * h;
}

// Kernel of |n|^2 = q in the unit box (k = 2 pi sqrt(q)), times the split factor of the
// two-level force (Sec. 2.1): exp(-k^2 rs^2) for the long-range part, 1 - exp(-k^2 rs^2)
// for the short-range part, rs = r_split / L.
__global__ void k_build_ktab(float* ktab, int64_t nent, int64_t n, double G, double eps,
                             double box, int kernel, double rs) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nent) return;
  double val = 0.0;
  if (q > 0) {
    double k = 2.0 * 3.141592653589793238462643 * sqrt((double)q);
    double g;
    if (eps > 0) g = -4.0 * 3.141592653589793238462643 * G * eps * bessel_k1(k * eps) / k;
    else g = -4.0 * 3.141592653589793238462643 * G / (k * k);
    if (kernel == PM_KERNEL_LONG) g *= exp(-(k * rs) * (k * rs));
    else if (kernel == PM_KERNEL_SHORT) g *= -expm1(-(k * rs) * (k * rs));
    // the 1/n^3 of the inverse transform, and the box: a density in mass per unit volume
    // of a box of side L has the force L a_1 of the same mesh values in the unit box
    val = g * box / ((double)n * (double)n * (double)n);
  }
  ktab[q] = (float)val;
}

// sinc(t)^4 = (sin(pi t) / (pi t))^4, 1 at t = 0: one axis of the CIC deposit window
// times the CIC interpolation window at wave number t n
__device__ inline double sinc4(double t) {
  if (t == 0.0) return 1.0;
  const double a = 3.141592653589793238462643 * t;
  const double s = sin(a) / a;
  return (s * s) * (s * s);
}

// Octant copy of the kernel table: gtab[(kx (h+1) + ay) (h+1) + az] = ktab[kx^2 + ay^2 +
// az^2] for kx, ay, az in [0, h], h = n/2. A z line at fixed (kx, ky) then reads its
// kernel values as one contiguous run. The long-range part of the two-level split is
// also divided by the mesh's CIC windows (a function of the three components, even in
// each), in float64 from the float64 kernel value.
__global__ void k_build_gtab(const float* ktab, float* gtab, int64_t h, int kernel,
                             double G, double eps, double box, double rs) {
  const int64_t h1 = h + 1, tot = h1 * h1 * h1;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= tot) return;
  const int64_t az = q % h1, ay = (q / h1) % h1, kx = q / (h1 * h1);
  const int64_t n2 = kx * kx + ay * ay + az * az;
  if (kernel != PM_KERNEL_LONG || n2 == 0) {
    gtab[q] = ktab[n2];
    return;
  }
  const double n = (double)(2 * h);
  const double k = 2.0 * 3.141592653589793238462643 * sqrt((double)n2);
  double g;
  if (eps > 0) g = -4.0 * 3.141592653589793238462643 * G * eps * bessel_k1(k * eps) / k;
  else g = -4.0 * 3.141592653589793238462643 * G / (k * k);
  g *= exp(-(k * rs) * (k * rs));
  g /= sinc4((double)kx / n) * sinc4((double)ay / n) * sinc4((double)az / n);
  gtab[q] = (float)(g * box / (n * n * n));
}

// ------------------------------------------------------------------ dispatch --
// columns per workgroup: at most 16 and at most half the line length (the number of kx
// lines is N/2, so W always divides the line count), W runs of 8-byte points per global
// access; LDS per workgroup (the exchange tiles, plus staged twiddles for two-input
// passes) within what one gfx950 workgroup may hold. Split lines (2048 points) take 16
// columns (1024 threads: 128-byte runs) in one-line passes and 8 in the two-input y pass
// of the transposed force, whose two register arrays do not fit 1024 threads (its z
// pass takes 4, zconv_w); narrower workgroups read their parts of 128-byte runs in tile
// order xcd_group.
template <int N, bool TWO>
constexpr int col_w() {
  int w = 16384 / N;
  if (LP<N>::H == 2 && !TWO) w = 16;
  if (w > 16) w = 16;
  if (w > N / 2) w = N / 2;
  if (w < 1) w = 1;
  return w;
}
// the two-input z pass with split lines (two line arrays per thread, 225 VGPRs) takes 4
// columns: 256 threads and 58 KB of LDS, two workgroups per CU
template <int N, bool TWO>
constexpr int zconv_w() {
  return LP<N>::H == 2 && TWO ? 4 : col_w<N, TWO>();
}

struct FftCtx {
  pm_context* c;
  int n;
  int twmask;
};

// out 0: plain, o0 = FFT(in); in1 (forward only): the two-input pass OUT 3 into o0; o1
// must be null
template <int N>
pm_status col_fft(const FftCtx& f, const float2* in, const float2* in1, float2* o0, float2* o1,
                  const Lines& d, int64_t L2, int sign) {
  constexpr int W1 = col_w<N, false>(), W2 = col_w<N, true>();
  const int out = in1 ? 3 : 0;
  if (o1 || !o0 || (out == 3 && sign > 0)) return PM_ERR_ARG;
  const int W = out == 3 ? W2 : W1;
  if (d.L1 % W) return PM_ERR_SHAPE;
  dim3 grid((unsigned)(d.L1 / W), (unsigned)L2);
  dim3 block(W * LP<N>::TL);
#define CLAUNCH(S, O)                                                                     \
  hipLaunchKernelGGL((k_col_fft<N, O == 3 ? W2 : W1, S, O>), grid, block, 0,             \
                     f.c->stream, in, in1, o0, o1, d, f.c->tw, 1, f.twmask, f.n, f.c->gk)
  if (sign < 0) {
    if (out == 3) CLAUNCH(-1, 3);
    else CLAUNCH(-1, 0);
  } else {
    CLAUNCH(1, 0);
  }
#undef CLAUNCH
  PM_LAUNCH_CHECK();
  return PM_OK;
}

template <int N>
pm_status col_zconv(const FftCtx& f, int mode, bool blk, const float2* i0, const float2* i1,
                    const float2* i2, float2* o0, float2* o1, const Lines& d, int64_t L2) {
  // every z pass stages its twiddles; MODE 1 holds two line arrays
  if (mode != 0 && mode != 1) return PM_ERR_ARG;
  constexpr int W1 = zconv_w<N, false>(), W2 = zconv_w<N, true>();
  const int W = mode == 1 ? W2 : W1;
  if (d.L1 % W) return PM_ERR_SHAPE;
  dim3 grid((unsigned)(d.L1 / W), (unsigned)L2);
  dim3 block(W * LP<N>::TL);
#define ZLAUNCH(MODE, BLK)                                                                  \
  hipLaunchKernelGGL((k_col_zconv<N, MODE == 1 ? W2 : W1, MODE, BLK>), grid,              \
                     block, 0, f.c->stream, i0, i1, i2, o0, o1, d, f.c->tw, 1, f.twmask,    \
                     f.n, f.c->gtab, f.c->gk)
  if (blk) {
    if (mode == 0) ZLAUNCH(0, true);
    else ZLAUNCH(1, true);
  } else {
    if (mode == 0) ZLAUNCH(0, false);
    else ZLAUNCH(1, false);
  }
#undef ZLAUNCH
  PM_LAUNCH_CHECK();
  return PM_OK;
}

template <int M>
pm_status row_r2c(const FftCtx& f, const float* in, float2* out, float2* nyq) {
  constexpr int R = rows_per_wg<M>();
  int64_t nrows = (int64_t)f.n * f.n;
  if (nrows % R) return PM_ERR_SHAPE;
  hipLaunchKernelGGL(k_row_r2c<M>, dim3((unsigned)cdiv(nrows, R)), dim3(R * Plan<M>::T), 0,
                     f.c->stream, in, out, nyq, nrows, f.c->tw, f.twmask);
  PM_LAUNCH_CHECK();
  return PM_OK;
}

template <int M>
pm_status row_c2r(const FftCtx& f, const float2* in, const float2* nyq, float* out) {
  constexpr int R = rows_per_wg<M>();
  int64_t nrows = (int64_t)f.n * f.n;
  if (nrows % R) return PM_ERR_SHAPE;
  hipLaunchKernelGGL(k_row_c2r<M>, dim3((unsigned)cdiv(nrows, R)), dim3(R * Plan<M>::T), 0,
                     f.c->stream, in, nyq, out, nrows, f.c->tw, f.twmask);
  PM_LAUNCH_CHECK();
  return PM_OK;
}

// Size dispatch: the column length is n, the row length (complex) n/2.
#define PM_FFT_SIZES(X) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048)

pm_status d_col_fft(const FftCtx& f, const float2* in, float2* o0, float2* o1, const Lines& d,
                    int64_t L2, int sign) {
  switch (f.n) {
#define CASE(N) \
  case N: return col_fft<N>(f, in, nullptr, o0, o1, d, L2, sign);
    PM_FFT_SIZES(CASE)
#undef CASE
  }
  return PM_ERR_SHAPE;
}
// forward y transform of two spectra into one: o = +i k_x FFT_y(in0) + i k_y FFT_y(in1)
pm_status d_col_fft_grad2(const FftCtx& f, const float2* in0, const float2* in1, float2* o,
                          const Lines& d, int64_t L2) {
  switch (f.n) {
#define CASE(N) \
  case N: return col_fft<N>(f, in0, in1, o, nullptr, d, L2, -1);
    PM_FFT_SIZES(CASE)
#undef CASE
  }
  return PM_ERR_SHAPE;
}
pm_status d_col_zconv(const FftCtx& f, int mode, bool blk, const float2* i0,
                      const float2* i1, const float2* i2, float2* o0, float2* o1,
                      const Lines& d, int64_t L2) {
  switch (f.n) {
#define CASE(N) \
  case N: return col_zconv<N>(f, mode, blk, i0, i1, i2, o0, o1, d, L2);
    PM_FFT_SIZES(CASE)
#undef CASE
  }
  return PM_ERR_SHAPE;
}
pm_status d_row_r2c(const FftCtx& f, const float* in, float2* out, float2* nyq) {
  switch (f.n) {
#define CASE(N) \
  case N: return row_r2c<N / 2>(f, in, out, nyq);
    PM_FFT_SIZES(CASE)
#undef CASE
  }
  return PM_ERR_SHAPE;
}
pm_status d_row_c2r(const FftCtx& f, const float2* in, const float2* nyq, float* out) {
  switch (f.n) {
#define CASE(N) \
  case N: return row_c2r<N / 2>(f, in, nyq, out);
    PM_FFT_SIZES(CASE)
#undef CASE
  }
  return PM_ERR_SHAPE;
}

int64_t d_row_blocks(int n) {
  switch (n) {
#define CASE(N) \
  case N: return cdiv((int64_t)N * N, rows_per_wg<N / 2>());
    PM_FFT_SIZES(CASE)
#undef CASE
  }
  return 0;
}

// Line descriptors of the z-blocked half spectrum (main, [z/ZB][y][z%ZB][kx < n/2]) and
// of the Nyquist plane nyq[z][y] (kx = n/2).
Lines lines_y_main(int n) {  // l1 = kx, l2 = z, element = y
  const int64_t M = n / 2, ZB = zblk(n);
  return Lines{1, (int64_t)n * ZB * M, M, ilog2(ZB), ZB * M, 0, M, 0, 1, 0};
}
Lines lines_y_nyq(int n) {  // l1 = z, element = y
  return Lines{n, 0, 0, 0, 1, 0, n, 1, 1, n / 2};
}
Lines lines_z_main(int n) {  // l1 = kx, l2 = y, element = z (blocked)
  const int64_t M = n / 2, ZB = zblk(n);
  return Lines{1, ZB * M, 0, 0, (int64_t)n * ZB * M, M, M, 0, 0, 0};
}
Lines lines_z_nyq(int n) {  // l1 = y, element = z
  return Lines{1, 0, 0, 0, n, 0, n, 1, 1, n / 2};
}

}  // namespace

pm_status build_kernel_table(pm_context* c) {
  const int64_t n = c->g.ng;
  c->ktab_n = 3 * (n / 2) * (n / 2) + 1;
  PM_HIP_CHECK(hipMalloc(&c->ktab, (size_t)c->ktab_n * sizeof(float)));
  double eps = c->cfg.soft_cells / (double)n;
  const int kernel = c->cfg.kernel;
  const double rs = kernel == PM_KERNEL_FULL ? 0.0 : c->cfg.r_split / c->cfg.box;
  hipLaunchKernelGGL(k_build_ktab, dim3((unsigned)cdiv(c->ktab_n, 256)), dim3(256), 0,
                     c->stream, c->ktab, c->ktab_n, n, c->cfg.G, eps, c->cfg.box, kernel, rs);
  PM_LAUNCH_CHECK();
  const int64_t h1 = n / 2 + 1, ng3 = h1 * h1 * h1;
  PM_HIP_CHECK(hipMalloc(&c->gtab, (size_t)ng3 * sizeof(float)));
  hipLaunchKernelGGL(k_build_gtab, dim3((unsigned)cdiv(ng3, 256)), dim3(256), 0, c->stream,
                     c->ktab, c->gtab, n / 2, kernel, c->cfg.G, eps, c->cfg.box, rs);
  PM_LAUNCH_CHECK();
  // twiddles exp(-2 pi i k / n), k < n, built in float64 on the host
  float2* h = (float2*)malloc(sizeof(float2) * n);
  if (!h) return PM_ERR_NOMEM;
  for (int64_t k = 0; k < n; ++k) {
    double a = -2.0 * 3.141592653589793238462643 * (double)k / (double)n;
    h[k] = make_float2((float)cos(a), (float)sin(a));
  }
  hipError_t e = hipMalloc(&c->tw, sizeof(float2) * n);
  if (e == hipSuccess) e = hipMemcpy(c->tw, h, sizeof(float2) * n, hipMemcpyHostToDevice);
  free(h);
  if (e != hipSuccess) return PM_ERR_DEVICE;
  // gradient symbol D(k) = n (8 sin(2 pi k/n) - sin(4 pi k/n)) / 6, k < n; both sines
  // vanish exactly where 4 k is a multiple of n or 2 k is (sin(pi j) = 0)
  std::vector<float> gk((size_t)n);
  for (int64_t k = 0; k < n; ++k) {
    auto sin_turn = [](int64_t j, int64_t m) {  // sin(2 pi j / m)
      j %= m;
      return (2 * j) % m == 0 ? 0.0 : std::sin(2.0 * 3.141592653589793238462643 * (double)j / (double)m);
    };
    gk[(size_t)k] = (float)((double)n * (8.0 * sin_turn(k, n) - sin_turn(2 * k, n)) / 6.0);
  }
  e = hipMalloc(&c->gk, sizeof(float) * n);
  if (e == hipSuccess) e = hipMemcpy(c->gk, gk.data(), sizeof(float) * n, hipMemcpyHostToDevice);
  if (e != hipSuccess) return PM_ERR_DEVICE;
  return PM_OK;
}

// Buffers: A0, A1, A2 are the three force meshes (acc), S one scratch mesh; N0 the
// Nyquist plane. Spectra are z-blocked, real meshes natural, so the x passes are out of
// place. The components of eq. (3) are the inverse transforms of -i D(k_a) G rho; D is
// the symbol of the fourth-order difference, so they are -D phi of the potential phi,
// which takes one inverse transform:
//   r2c    rho -> A1                       (rho may be A0)
//   Y      A1 in place
//   Z      G F: A1 in place
//   Y^-1   A1 in place
//   c2r    phi: A1 -> S
//   k_grad4  a = -D phi: S -> A0, A1, A2, and the per-block max |a|
pm_status run_force(pm_context* c, const float* rho, float* acc, float2* nyq, float* amax) {
  const int n = (int)c->g.ng;
  const int64_t n3 = (int64_t)n * n * n;
  FftCtx f{c, n, n - 1};
  float2* A1 = (float2*)(acc + n3);
  float* phi = (float*)scratch(c, SC_SPEC, (size_t)n3 * sizeof(float));
  if (!phi) return PM_ERR_NOMEM;
  float2* N0 = nyq;
  pm_status s;
  const GradTile gt = grad_tile(n);
  unsigned int* part = nullptr;
  if (amax) {
    part = (unsigned int*)scratch(c, SC_PARTS, (size_t)gt.blocks * 4);
    if (!part) return PM_ERR_NOMEM;
  }
  {
    ProfScope ps(c, ST_FFT_R2C);
    if ((s = d_row_r2c(f, rho, A1, N0)) != PM_OK) return s;
  }
  const Lines ym = lines_y_main(n), yn = lines_y_nyq(n);
  const Lines zm = lines_z_main(n), zn = lines_z_nyq(n);
  {
    ProfScope ps(c, ST_FFT_YF);
    if ((s = d_col_fft(f, A1, A1, nullptr, ym, n, -1)) != PM_OK) return s;
  }
  if ((s = d_col_fft(f, N0, N0, nullptr, yn, 1, -1)) != PM_OK) return s;
  // the potential's spectrum G rho, in place
  {
    ProfScope ps(c, ST_FFT_Z);
    if ((s = d_col_zconv(f, 0, true, A1, nullptr, nullptr, A1, nullptr, zm, n)) != PM_OK)
      return s;
  }
  if ((s = d_col_zconv(f, 0, false, N0, nullptr, nullptr, N0, nullptr, zn, 1)) != PM_OK)
    return s;
  {
    ProfScope ps(c, ST_FFT_YI);
    if ((s = d_col_fft(f, A1, A1, nullptr, ym, n, +1)) != PM_OK) return s;
  }
  if ((s = d_col_fft(f, N0, N0, nullptr, yn, 1, +1)) != PM_OK) return s;
  {
    ProfScope ps(c, ST_FFT_C2R);
    if ((s = d_row_c2r(f, A1, N0, phi)) != PM_OK) return s;
  }
  // the three components from the potential by the difference stencil
  {
    ProfScope ps(c, ST_GRAD);
    hipLaunchKernelGGL(k_grad4, dim3((unsigned)gt.blocks), dim3(GRAD_T), 0, c->stream,
                       (const float*)phi, acc, acc + n3, acc + 2 * n3, ilog2(n), gt.gx, gt.gy,
                       gt.gz, (float)((double)n / 12.0), part);
    PM_LAUNCH_CHECK();
  }
  if (amax) return fold_max_u32(c, part, gt.blocks, (uint32_t*)amax);
  return PM_OK;
}
pm_status run_force_transpose(pm_context* c, float* acc, float2* nyq) {
  const int n = (int)c->g.ng;
  const int64_t n3 = (int64_t)n * n * n, n2 = (int64_t)n * n;
  FftCtx f{c, n, n - 1};
  float2* A[3] = {(float2*)acc, (float2*)(acc + n3), (float2*)(acc + 2 * n3)};
  float2* S = (float2*)scratch(c, SC_SPEC, (size_t)n3 * sizeof(float));
  if (!S) return PM_ERR_NOMEM;
  float2* Nq[3] = {nyq, nyq + n2, nyq + 2 * n2};
  pm_status s;
  const Lines ym = lines_y_main(n), yn = lines_y_nyq(n);
  const Lines zm = lines_z_main(n), zn = lines_z_nyq(n);
  float2* spec[3] = {A[1], A[2], S};  // spectrum of mu_x, mu_y, mu_z
  for (int ax = 2; ax >= 0; --ax)
    if ((s = d_row_r2c(f, (const float*)A[ax], spec[ax], Nq[ax])) != PM_OK) return s;
  if ((s = d_col_fft(f, spec[2], spec[2], nullptr, ym, n, -1)) != PM_OK) return s;
  if ((s = d_col_fft(f, Nq[2], Nq[2], nullptr, yn, 1, -1)) != PM_OK) return s;
  if ((s = d_col_fft_grad2(f, spec[0], spec[1], spec[0], ym, n)) != PM_OK) return s;
  if ((s = d_col_fft_grad2(f, Nq[0], Nq[1], Nq[0], yn, 1)) != PM_OK) return s;
  if ((s = d_col_zconv(f, 1, true, spec[0], nullptr, spec[2], spec[0], nullptr, zm, n)) !=
      PM_OK)
    return s;
  if ((s = d_col_zconv(f, 1, false, Nq[0], nullptr, Nq[2], Nq[0], nullptr, zn, 1)) != PM_OK)
    return s;
  if ((s = d_col_fft(f, spec[0], spec[0], nullptr, ym, n, +1)) != PM_OK) return s;
  if ((s = d_col_fft(f, Nq[0], Nq[0], nullptr, yn, 1, +1)) != PM_OK) return s;
  return d_row_c2r(f, spec[0], Nq[0], (float*)A[0]);
}

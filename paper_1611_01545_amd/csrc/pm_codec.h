// Exact integer definitions of the compressed format's codes (Sec. 2.4), shared by
// the encode, decode, kick-drift and stream kernels. Each is an exact function of
// its inputs on any IEEE machine: products by powers of two are exact, and the one
// inexact product in the velocity code is a single correctly rounded float64
// operation with contraction disabled.
#pragma once
#include <type_traits>

#include "pm_common.h"

#define PM_STREAM_HEADER 64

// u = floor(x (S / L)) mod S (S = 256 n_c, a power of two; SL = S / L rounded once to
// float64, exact when L is a power of two). Returns false for non-finite or absurdly
// large input (u is then 0).
__device__ inline bool pos_code(float x, double SL, int64_t S, uint32_t& u) {
  double t = (double)x * SL;
  if (!(fabs(t) < 4.0e15)) {
    u = 0;
    return false;
  }
  int64_t k = (int64_t)floor(t);
  k %= S;
  if (k < 0) k += S;
  u = (uint32_t)k;
  return true;
}

// Bin centre (u + 1/2) L / S with LS = L / S rounded to float32 (exact when L is a power
// of two; u + 1/2 is exact, u < 2^19).
__device__ inline float pos_decode(uint32_t u, float LS) {
  return ((float)u + 0.5f) * LS;
}

// j = clamp(floor(v C + 32768), 0, 65535), C = 32768 / v_max, in float64 with the
// product and the sum rounded separately; v_max = 0 gives the centre bin 32768.
__device__ inline int vel_code(float v, float vmax) {
#pragma clang fp contract(off)
  if (vmax == 0.f) return 32768;
  double C = 32768.0 / (double)vmax;
  double t = (double)v * C;
  t = t + 32768.0;
  if (!(t >= 0.0)) return 0;
  if (t >= 65535.0) return 65535;
  return (int)floor(t);
}

// Bin centre (j - 32767.5) v_max / 32768: exact in float64, rounded once to float32.
__device__ inline float vel_decode(uint32_t j, float vmax) {
#pragma clang fp contract(off)
  double w = (double)vmax * 0x1p-15;
  return (float)(((double)j - 32767.5) * w);
}

// vel_code for a power-of-two v_max in [2^-90, 2^90], in float32 with the same result
// on every input. x = v C is exact (C a power of two; an overflow to +-inf or an
// underflow of a value below 2^-126 cannot change the outcome), and x + 32768 is exact
// in float64 except for |x| < 2^-15, where the float64 sum rounds up to 32768 exactly
// when -2^-39 <= x < 0 (ties to even). C is passed in as 2^15 / v_max.
__device__ inline int vel_code_p2(float v, float C) {
#pragma clang fp contract(off)
  const float x = v * C;
  float fl = floorf(x);
  if (x < 0.f && x >= -0x1p-39f) fl = 0.f;
  if (!(fl >= -32768.f)) return 0;  // also NaN
  if (fl >= 32767.f) return 65535;
  return (int)fl + 32768;
}

// vel_decode for v_max in [2^-90, 2^90], in float32 with the same result: j - 32767.5
// and w = v_max 2^-15 are exact in float32, so the one product is the same correctly
// rounded value as the float64 product rounded to float32. w is passed in.
__device__ inline float vel_decode_w(uint32_t j, float w) {
#pragma clang fp contract(off)
  return ((float)j - 32767.5f) * w;
}

// ---------------------------------------------------------------- code widths --
// Adjustable widths (Sec. 2.4, closing remark): P position bytes per axis (offset inside
// the cell in units of 1/(256^P n_c), S = 256^P n_c) and V velocity bytes per axis
// (2^(8V) bins, half range H = 2^(8V - 1)). P = 1, V = 2 is the paper's format; the
// functions below reduce to the ones above there.
template <int P> struct PosCode;
template <> struct PosCode<1> { using T = uint8_t; };
template <> struct PosCode<2> { using T = uint16_t; };
template <int V> struct VelCode;
template <> struct VelCode<1> { using T = uint8_t; };
template <> struct VelCode<2> { using T = uint16_t; };

// j = clamp(floor(v C + H), 0, 2H - 1), C = H / v_max, as vel_code
template <int V>
__device__ inline int vel_code_v(float v, float vmax) {
#pragma clang fp contract(off)
  constexpr double H = (double)(1 << (8 * V - 1));
  if (vmax == 0.f) return (int)H;
  double C = H / (double)vmax;
  double t = (double)v * C;
  t = t + H;
  if (!(t >= 0.0)) return 0;
  if (t >= 2.0 * H - 1.0) return (int)(2.0 * H - 1.0);
  return (int)floor(t);
}

// Bin centre (j - H + 1/2) v_max / H, as vel_decode
template <int V>
__device__ inline float vel_decode_v(uint32_t j, float vmax) {
#pragma clang fp contract(off)
  constexpr double H = (double)(1 << (8 * V - 1));
  double w = (double)vmax / H;
  return (float)(((double)j - (H - 0.5)) * w);
}

// vel_code_v for a power-of-two v_max in [2^-90, 2^90] in float32, as vel_code_p2: the
// float64 sum x + H rounds up to H exactly when -2^(log2 H - 54) <= x < 0. C = H / v_max.
template <int V>
__device__ inline int vel_code_p2_v(float v, float C) {
#pragma clang fp contract(off)
  constexpr float H = (float)(1 << (8 * V - 1));
  constexpr float TIE = V == 2 ? 0x1p-39f : 0x1p-47f;
  const float x = v * C;
  float fl = floorf(x);
  if (x < 0.f && x >= -TIE) fl = 0.f;
  if (!(fl >= -H)) return 0;  // also NaN
  if (fl >= H - 1.f) return (int)(2.f * H - 1.f);
  return (int)fl + (int)H;
}

// vel_decode_v for v_max in [2^-90, 2^90] in float32, as vel_decode_w: w = v_max / H.
template <int V>
__device__ inline float vel_decode_w_v(uint32_t j, float w) {
#pragma clang fp contract(off)
  constexpr float H = (float)(1 << (8 * V - 1));
  return ((float)j - (H - 0.5f)) * w;
}

// Call f(integral_constant P, integral_constant V) for the widths kind k.
template <int N> using IC = std::integral_constant<int, N>;
template <typename F>
inline pm_status width_dispatch(int k, F&& f) {
  switch (k) {
    case 0: return f(IC<1>{}, IC<2>{});
    case 1: return f(IC<2>{}, IC<2>{});
    case 2: return f(IC<1>{}, IC<1>{});
    case 3: return f(IC<2>{}, IC<1>{});
  }
  return PM_ERR_ARG;
}

// exclusive prefix of the stream bytes of each cell (count byte, escape, rb-byte records)
pm_status scan_generic_pack(pm_context* c, const int64_t* off, int64_t n, int64_t* out,
                            int64_t rb = 9);

// Exact integer definitions of the compressed format's codes (Sec. 2.4), shared by
// the encode, decode, kick-drift and stream kernels. Each is an exact function of
// its inputs on any IEEE machine: products by powers of two are exact, and the one
// inexact product in the velocity code is a single correctly rounded float64
// operation with contraction disabled.
#pragma once
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

pm_status scan_generic_pack(pm_context* c, const int64_t* off, int64_t n, int64_t* out);

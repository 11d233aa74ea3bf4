// Device-side helpers shared by the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rt_internal.h"

#define RT_PI 3.14159265358979323846

// Half-face record type of a precision.
template <typename T> struct rt_vec4;
template <> struct rt_vec4<double> { using type = double4; };
template <> struct rt_vec4<float> { using type = float4; };

// MI355X has 8 XCDs, each with its own L2; consecutive workgroups are dispatched
// round-robin over them.  The grid is padded to a multiple of 8 and workgroup b
// takes logical tile (b % 8) * per + b / 8, so every XCD sweeps one contiguous
// range of cells (cells are numbered along a space-filling curve, so its
// neighbour rows stay in that XCD's L2).  Returns -1 for padding workgroups.
__device__ __forceinline__ int64_t rt_logical_block(int64_t nblk) {
  const int64_t per = (nblk + 7) / 8;
  const int64_t b = blockIdx.x;
  const int64_t L = (b % 8) * per + b / 8;
  return L < nblk ? L : -1;
}

static inline int64_t rt_grid_for(int64_t nblk) { return ((nblk + 7) / 8) * 8; }

// A double from another lane of the same row of 16 by a DPP lane permutation (both
// halves moved by v_mov_dpp; no LDS round trip).  Controls used below (gfx9 encodings):
// quad_perm [1,0,3,2] = lane ^ 1, quad_perm [2,3,0,1] = lane ^ 2, row_half_mirror =
// lane 7 - i within each 8, row_mirror = lane 15 - i within each 16.
// Every source lane of these patterns is an active lane of the same group, so no lane
// keeps an old value and the move needs no initialised destination.
template <int CTRL> __device__ __forceinline__ double rt_dpp(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over the LPC lanes of a cell group (groups are aligned runs of LPC lanes, all
// active).  Each step adds the value of a partner lane whose own step adds this lane's
// value (pairs by lane ^ 1, lane ^ 2, then the mirrored quad and half-row), so every
// lane of the group ends with the bit-identical total (each pairwise add is
// commutative).  Groups wider than 16 lanes use the xor butterfly through LDS.
template <int LPC> __device__ __forceinline__ double rt_group_sum(double v) {
  if constexpr (LPC <= 16) {
    if constexpr (LPC >= 2) v += rt_dpp<0xB1>(v);
    if constexpr (LPC >= 4) v += rt_dpp<0x4E>(v);
    if constexpr (LPC >= 8) v += rt_dpp<0x141>(v);
    if constexpr (LPC >= 16) v += rt_dpp<0x140>(v);
  } else {
#pragma unroll
    for (int o = LPC / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, LPC);
  }
  return v;
}
template <int LPC> __device__ __forceinline__ double rt_group_min(double v) {
  if constexpr (LPC <= 16) {
    if constexpr (LPC >= 2) v = fmin(v, rt_dpp<0xB1>(v));
    if constexpr (LPC >= 4) v = fmin(v, rt_dpp<0x4E>(v));
    if constexpr (LPC >= 8) v = fmin(v, rt_dpp<0x141>(v));
    if constexpr (LPC >= 16) v = fmin(v, rt_dpp<0x140>(v));
  } else {
#pragma unroll
    for (int o = LPC / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, LPC));
  }
  return v;
}

// Unique positive root of A T^4 + B T - C = 0 (A >= 0; B, C > 0).  Newton from
// T0 = min((C/A)^(1/4), C/B): f(T0) >= 0 and f is convex and increasing for
// T > 0, so the iterates fall monotonically; stop at the first one that does not.
__device__ __forceinline__ double rt_quartic_root(double A, double B, double C) {
  if (!(A > 0.0)) return C / B;
  double T = fmin(sqrt(sqrt(C / A)), C / B);
  for (int it = 0; it < 100; ++it) {
    const double T3 = T * T * T;
    const double Tn = T - (A * T3 * T + B * T - C) / (4.0 * A * T3 + B);
    if (!(Tn < T)) break;
    T = Tn;
  }
  return T;
}

// Same root, warm-started: a previous temperature Tw with f(Tw) >= 0 lies right of
// the root, where the Newton iterates also fall monotonically, so it replaces the
// cold start when it qualifies.  Steps use the refined reciprocal.
__device__ __forceinline__ double rt_rcp(double x);
__device__ __forceinline__ double rt_quartic_root_from(double A, double B, double C, double Tw) {
  if (!(A > 0.0)) return C / B;
  double T;
  if (Tw > 0.0 && A * Tw * Tw * Tw * Tw + B * Tw - C >= 0.0) {
    T = Tw;
  } else {
    const double iA = rt_rcp(A), iB = rt_rcp(B);
    T = fmin(sqrt(sqrt(C * iA)), C * iB);
  }
  for (int it = 0; it < 100; ++it) {
    const double T3 = T * T * T;
    const double Tn = T - (A * T3 * T + B * T - C) * rt_rcp(4.0 * A * T3 + B);
    if (!(Tn < T)) break;
    T = Tn;
  }
  return T;
}

// Reciprocals for per-angle arithmetic.  FP64: the hardware estimate refined by
// two Newton steps (within an ulp of 1/x); FP32: the hardware estimate (1 ulp).
__device__ __forceinline__ double rt_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float rt_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
// The end-of-step volume V' = V + dt D of the volume update (section 2.2), formed by every
// kernel as one fused multiply-add: left to the compiler, the sum is contracted in some
// kernels and not in others, and a step and its reverse then disagree in the last bit.
__device__ __forceinline__ double rt_vol_next(double V, double dt, double D) { return fma(dt, D, V); }
// Reciprocal within an ulp in either precision (FP32: the estimate refined by one
// Newton step), for ratios that decide a limiter.
__device__ __forceinline__ double rt_rcp_refined(double x) { return rt_rcp(x); }
__device__ __forceinline__ float rt_rcp_refined(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// Angles of a lane: k = l + LPC * q for q < APL; ok[q] false past K.  With FULL
// (K == LPC * APL) every angle is live and k needs no clamping.
template <typename T, int LPC, int APL, bool FULL = false> struct rt_lane_angles {
  T dx[APL], dy[APL], dz[APL];
  double w[APL];
  int k[APL];
  bool ok[APL];
  __device__ __forceinline__ void load(const double *dirs, const double *W, int K, int l) {
#pragma unroll
    for (int q = 0; q < APL; ++q) {
      const int kk = l + LPC * q;
      ok[q] = FULL || kk < K;
      // angles past K alias angle 0: loads stay in bounds, their weight is 0 and they are never stored
      k[q] = ok[q] ? kk : 0;
      dx[q] = (T)dirs[3 * k[q]];
      dy[q] = (T)dirs[3 * k[q] + 1];
      dz[q] = (T)dirs[3 * k[q] + 2];
      w[q] = ok[q] ? W[k[q]] : 0.0;
    }
  }
};

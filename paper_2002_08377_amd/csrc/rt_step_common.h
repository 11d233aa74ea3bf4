// Pieces shared by the step kernels: the lane-to-angle layouts and the implicit
// source update of one cell held by a group of LPC lanes.
#pragma once

#include "rt_device.h"

// Angles held by one lane.
//  General layout: k_q = l + LPC q for q < APL; past K (only when !FULL) the slot
//    aliases angle 0 with weight 0 and is never stored.
//  Paired layouts (needs K = LPC APL): the lane holds P = APL/2 angles and their
//    antipodes (same weight) in slots q + P, so one stored direction serves both and
//    one dot product per face serves both fluxes.  Pair p is angles p and p + K/2 when
//    PAIRED = 1 (antipode K/2 on) and angles 2p and 2p + 1 when PAIRED = 2 (antipode
//    beside its angle, so a pair's two elements move with one wider access).
//    TWOS false: slot q holds pair l + LPC q.
//    TWOS true: pairs are dealt to the lanes two at a time: slot q < P2 = 2 floor(P/2)
//      holds pair 2 (l + LPC floor(q/2)) + q mod 2, and when P is odd the last slot holds
//      pair 2 LPC floor(P/2) + l.  A lane's pairs then come in runs of two consecutive
//      pairs, which read_lane / write_lane move together (with PAIRED = 2, four
//      consecutive elements: one 16-byte access in FP32).
//  Both orders deal the same pairs to the same slots, so a step gives the same bits in
//  either order.
template <typename T, int LPC, int APL, bool FULL, int PAIRED, bool TWOS = false> struct rt_step_angles {
  static constexpr int P = PAIRED ? APL / 2 : APL;
  static constexpr bool RUNS = TWOS && PAIRED;
  static constexpr int P2 = RUNS ? 2 * (P / 2) : 0;     // slots holding runs of two pairs
  static constexpr bool SINGLE = RUNS && P % 2 == 1;    // the last pair slot is a lone pair
  static constexpr bool PAIRED_LAYOUT = PAIRED != 0;
  static constexpr bool ADJACENT = PAIRED == 2;
  T x[P], y[P], z[P];
  double w[P];
  int k[APL];
  bool ok[APL];
  __device__ __forceinline__ void load(const double *dirs, const double *W, int K, int l) {
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const int pr = !RUNS ? l + LPC * q
                     : q < P2 ? 2 * (l + LPC * (q / 2)) + q % 2 : 2 * LPC * (P / 2) + l;  // pair of slot q
      const int kk = PAIRED == 2 ? 2 * pr : pr;
      ok[q] = FULL || PAIRED || kk < K;
      k[q] = ok[q] ? kk : 0;
      x[q] = (T)dirs[3 * k[q]];
      y[q] = (T)dirs[3 * k[q] + 1];
      z[q] = (T)dirs[3 * k[q] + 2];
      w[q] = ok[q] ? W[k[q]] : 0.0;
      if (PAIRED) {
        k[q + P] = k[q] + (PAIRED == 2 ? 1 : K / 2);
        ok[q + P] = true;
      }
    }
  }
  // direction and weight of slot q (q is a compile-time constant after unrolling)
  __device__ __forceinline__ T dx(int q) const { return PAIRED && q >= P ? -x[q - P] : x[q]; }
  __device__ __forceinline__ T dy(int q) const { return PAIRED && q >= P ? -y[q - P] : y[q]; }
  __device__ __forceinline__ T dz(int q) const { return PAIRED && q >= P ? -z[q - P] : z[q]; }
  __device__ __forceinline__ double wt(int q) const { return PAIRED && q >= P ? w[q - P] : w[q]; }
  // the lane's elements of the row starting at p (in the adjacent layout the two elements
  // of a pair are consecutive, and the compiler moves them with one wider access: the
  // arrays are only element-aligned, which the target's unaligned access mode allows)
  __device__ __forceinline__ void read_row(const T *p, T (&v)[APL]) const {
#pragma unroll
    for (int q = 0; q < APL; ++q) v[q] = p[k[q]];
  }
  // Whether slot q holds the lone pair (its angle or its antipode).
  static constexpr bool is_single(int q) { return SINGLE && (q == P - 1 || q == 2 * P - 1); }
  // Offset of slot q from the lane's first angle k[0] (from k[P - 1] for the lone pair's
  // slots); the same for every lane of a full layout (K = LPC APL), where the antipodes
  // of PAIRED 1 sit K/2 = LPC P further on.
  static constexpr int slot_offset(int q) {
    const int qq = q < P ? q : q - P;
    if (PAIRED == 1 && RUNS) return (is_single(q) ? 0 : 2 * LPC * (qq / 2) + qq % 2) + (q < P ? 0 : LPC * P);
    if (PAIRED == 2 && RUNS) return (is_single(q) ? 0 : 4 * LPC * (qq / 2) + 2 * (qq % 2)) + (q < P ? 0 : 1);
    if (PAIRED == 1) return LPC * qq + (q < P ? 0 : LPC * P);
    if (PAIRED == 2) return 2 * LPC * qq + (q < P ? 0 : 1);
    return LPC * q;
  }
  // The lane's elements of the row `r` of an [N][K] array: the lane's base pointers (row 0
  // plus k[0], and plus k[P - 1] for a lone pair) move by a row stride (one 32 x 32 -> 64-bit
  // multiply-add per row), and in a full layout every element sits at a compile-time offset
  // from one of them.
  __device__ __forceinline__ const T *lane_row(const T *lane_base, uint32_t r, uint32_t row_bytes) const {
    return (const T *)((const char *)lane_base + (uint64_t)r * row_bytes);
  }
  __device__ __forceinline__ void read_lane(const T *pl, const T *ps, T (&v)[APL]) const {
    if constexpr (FULL) {
#pragma unroll
      for (int q = 0; q < APL; ++q) v[q] = is_single(q) ? ps[slot_offset(q)] : pl[slot_offset(q)];
    } else {
#pragma unroll
      for (int q = 0; q < APL; ++q) v[q] = pl[k[q] - k[0]];
    }
  }
  __device__ __forceinline__ void write_lane(T *pl, T *ps, const T (&v)[APL]) const {
    if constexpr (FULL) {
#pragma unroll
      for (int q = 0; q < APL; ++q) {
        if (is_single(q)) ps[slot_offset(q)] = v[q];
        else pl[slot_offset(q)] = v[q];
      }
    } else {
#pragma unroll
      for (int q = 0; q < APL; ++q)
        if (ok[q]) pl[k[q] - k[0]] = v[q];
    }
  }
  __device__ __forceinline__ void write_row(T *p, const T (&v)[APL]) const {
#pragma unroll
    for (int q = 0; q < APL; ++q)
      if (ok[q]) p[k[q]] = v[q];
  }
};

// Implicit source update (section 2.3, the four-step algorithm) of the cell `cell`,
// whose LPC lanes hold the transported intensities Ic of their angles (updated in
// place).  Gas energy and momentum are written by lane 0 when a.write_gas is set.
template <typename T, int LPC, int APL, typename Ang>
__device__ __forceinline__ void rt_source_cell(const rt_step_args &a, const Ang &ang, int64_t cell, int l,
                                               T (&Ic)[APL]) {
  constexpr int P = Ang::P;
  constexpr bool PAIRED = Ang::PAIRED_LAYOUT;

    // ---- implicit source (section 2.3): 1-2. comoving sums and the temperature ----------
    const double rho = a.rho[cell];
    const double m0 = a.mom[3 * cell], m1 = a.mom[3 * cell + 1], m2 = a.mom[3 * cell + 2];
    const double Eg = a.etot[cell];
    const double kP = a.kP[cell], kJ = a.kJ[cell], ks = a.ks[cell];
    const double c = a.c_light;
    const double irho = rt_rcp(rho);
    const double vx = m0 * irho, vy = m1 * irho, vz = m2 * irho;
    const double ic = a.inv_c;
    const double gam = rsqrt(1.0 - (vx * vx + vy * vy + vz * vz) * (ic * ic));
    const double y = a.dt * a.c_red * rho;
    const double chi = kJ + ks;
    const T tg = (T)gam, tvx = (T)(vx * ic), tvy = (T)(vy * ic), tvz = (T)(vz * ic), tyc = (T)(y * chi);
    // The four sums have positive terms only.  A lane adds its own angles' terms in the
    // intensities' type (within APL rounding steps of the exact partial in FP32) and the
    // lanes' partials meet in FP64.
    T sQ_ = 0, s1_ = 0, sG_ = 0, sI_ = 0;
    // Per angle, with r = 1/(1 + y chi Gamma): the update of eq. 28 boosted back is
    // I' = (Gamma^4 I + y Gamma S) r / Gamma^4 = I r + (r / Gamma^3) y S.  FP32: I r and
    // r / Gamma^3 are kept from the sums to the update (Ic, Br), with the incoming I (I0) for
    // the bookkeeping of step 4.  FP64 (LIGHT, to stay within three waves per SIMD): only the
    // incoming I is held through the temperature solve; Gamma, r and r / Gamma^3 are formed
    // again in the update by the same expressions (their inputs pass an empty asm, so the
    // compiler cannot reuse the first values and no value changes), and the weights are read
    // again here rather than held through the caller's face loop.
    constexpr bool LIGHT = sizeof(T) == 8;
    T I0[LIGHT ? 1 : APL], Br[LIGHT ? 1 : APL];
    double wq[P];
    if constexpr (LIGHT) {
      const double *W_again = a.W;
      asm volatile("" : "+s"(W_again));
#pragma unroll
      for (int q = 0; q < P; ++q) wq[q] = ang.ok[q] ? W_again[ang.k[q]] : 0.0;
    } else {
#pragma unroll
      for (int q = 0; q < P; ++q) wq[q] = ang.w[q];
    }
    auto pass1 = [&](int q, T G) {
      if constexpr (!LIGHT) I0[q] = Ic[q];
      const T iG = rt_rcp(G);
      const T iG2 = iG * iG;
      const T G2 = G * G;
      const T r = rt_rcp(T(1) + tyc * G);
      const T qk = (T)wq[q < P ? q : q - P] * iG2;
      sQ_ += qk;
      s1_ += qk * r;
      sG_ += qk * (G * r);
      sI_ += qk * (G2 * G2 * Ic[q] * r);
      if constexpr (!LIGHT) {
        Ic[q] *= r;
        Br[q] = r * iG2 * iG;
      }
    };
#pragma unroll
    for (int q = 0; q < P; ++q) {
      // Gamma = gamma (1 - v.n/c); the antipode has gamma (1 + v.n/c)
      const T vn = tvx * ang.x[q] + tvy * ang.y[q] + tvz * ang.z[q];
      pass1(q, tg * (T(1) - vn));
      if (PAIRED) pass1(q + P, tg * (T(1) + vn));
    }
    const double sQ = rt_group_sum<LPC>((double)sQ_);
    const double s1 = rt_group_sum<LPC>((double)s1_);
    const double sG = rt_group_sum<LPC>((double)sG_);
    const double sI = rt_group_sum<LPC>((double)sI_);
    const double iQ = rt_rcp(sQ);
    const double S1 = s1 * iQ, SG = sG * iQ, SI = sI * iQ;
    const double Dd = S1 + y * kJ * SG;
    const double iD = rt_rcp(Dd);
    const double rcv = rho * a.cv;
    const double Tn = (Eg - 0.5 * (m0 * m0 + m1 * m1 + m2 * m2) * irho) * rt_rcp(rcv);
    const double fourpi = 4.0 * RT_PI;
    const double Aq = a.dt * c * rho * kP * a.a_rad * S1 * iD;
    const double Cq = rcv * Tn + a.dt * c * rho * fourpi * kJ * SI * iD;
    const double Tnew = rt_quartic_root_from(Aq, rcv, Cq, Tn);
    const double T4 = Tnew * Tnew * Tnew * Tnew;
    const double planck = a.a_4pi * T4;
    const double Jc = (SI + y * kP * SG * planck) * iD;
    const T ySrc = (T)(y * (kP * planck + ks * Jc));
    // ---- 3. per-angle implicit update, boost back; 4. radiation energy and momentum lost
    //         by the stored values, handed to the gas (eqs. 35-36) ------------------------
    double dE = 0, dFx = 0, dFy = 0, dFz = 0;
    T tg3 = tg, tvx3 = tvx, tvy3 = tvy, tvz3 = tvz, tyc3 = tyc;
    if constexpr (LIGHT) asm volatile("" : "+v"(tg3), "+v"(tvx3), "+v"(tvy3), "+v"(tvz3), "+v"(tyc3));
    // the updated value of slot q (boost factor G) and, through I_in, its incoming value
    auto update = [&](int q, T G, T &I_in) {
      if constexpr (LIGHT) {
        const T iG = rt_rcp(G);
        const T iG2 = iG * iG;
        const T r = rt_rcp(T(1) + tyc3 * G);
        const T Ir = Ic[q] * r;
        const T B = r * iG2 * iG;
        I_in = Ic[q];
        return Ir + B * ySrc;
      } else {
        I_in = I0[q];
        return Ic[q] + Br[q] * ySrc;
      }
    };
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const T vn = LIGHT ? tvx3 * ang.x[q] + tvy3 * ang.y[q] + tvz3 * ang.z[q] : T(0);
      T in1;
      const T out = update(q, tg3 * (T(1) - vn), in1);
      Ic[q] = out;
      double wd = wq[q] * ((double)in1 - (double)out);
      dE += wd;
      if (PAIRED) {
        T in2;
        const T out2 = update(q + P, tg3 * (T(1) + vn), in2);
        Ic[q + P] = out2;
        const double wd2 = wq[q] * ((double)in2 - (double)out2);
        dE += wd2;
        wd -= wd2;  // the antipode's direction is -n
      }
      dFx += wd * (double)ang.x[q];
      dFy += wd * (double)ang.y[q];
      dFz += wd * (double)ang.z[q];
    }
    dE = rt_group_sum<LPC>(dE);
    dFx = rt_group_sum<LPC>(dFx);
    dFy = rt_group_sum<LPC>(dFy);
    dFz = rt_group_sum<LPC>(dFz);
    if (l == 0) {
      if (a.write_gas) {
        a.etot[cell] = Eg + a.e_gain * dE;
        a.mom[3 * cell] = m0 + a.m_gain * dFx;
        a.mom[3 * cell + 1] = m1 + a.m_gain * dFy;
        a.mom[3 * cell + 2] = m2 + a.m_gain * dFz;
      }
      if (a.T_out) a.T_out[cell] = Tnew;
      if (a.src_tape_out) {
        double *tp = a.src_tape_out + RT_SRC_TAPE * cell;
        tp[RT_TAPE_IQ] = iQ;
        tp[RT_TAPE_S1] = S1;
        tp[RT_TAPE_SG] = SG;
        tp[RT_TAPE_SI] = SI;
        tp[RT_TAPE_ID] = iD;
        tp[RT_TAPE_T] = Tnew;
        tp[RT_TAPE_M] = m0;  // the start-of-step momentum (the volume is written by the caller)
        tp[RT_TAPE_M + 1] = m1;
        tp[RT_TAPE_M + 2] = m2;
      }
    }
  }

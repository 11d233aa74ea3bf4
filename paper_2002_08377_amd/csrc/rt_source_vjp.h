// Reverse of the implicit source update (section 2.3) of one cell held by a group of LPC
// lanes, in the step kernel's lane layouts, for the fused adjoint modes of the step kernel.
//
// Forward (per cell, with Gamma_k = gamma (1 - v.n_k / c), weights W_k):
//   comoving intensity I0_k = Gamma_k^4 I*_k, Wt_k = W_k Gamma_k^-2 / sum_j W_j Gamma_j^-2,
//   r_k = 1 / (1 + y chi Gamma_k), sums S1 = sum Wt r, SG = sum Wt Gamma r, SI = sum Wt I0 r,
//   the temperature root of A T^4 + B T = C (eq. 33 form; A, C from the sums, B = rho cv),
//   source S = kP a T^4 / 4 pi + ks J, per angle I'_k = (I0_k + y Gamma_k S) r_k Gamma_k^-4,
//   then the gas takes the radiation energy and momentum the update removed (eqs. 35-36).
// The taped forward step stores each cell's 1/sum W Gamma^-2, S1, SG, SI, 1/D and T^{n+1}
// (D = S1 + y kJ SG) with its start-of-step volume and momentum, so the reverse needs no
// sums, no root and no gas state of its own; through the root
// it uses the implicit function theorem, dT = -(T^4 dA + T dB - dC) / (4 A T^3 + B).
//
// The intensities the reverse reads are the step's output I' (which the recompute of a
// segment keeps anyway, one buffer per step) rather than the transported I*: the update
// inverts to Gamma^4 I* + y Gamma S = I' Gamma^4 / r, so the forward need not store I*.
//
// Per-angle arithmetic runs in the intensities' type T, sums over angles and per-cell
// values in FP64, as in the forward source.  On return lam holds dL/dI* divided by the
// cell's end-of-step volume V', the input of the transpose of the upwind charge update.
#pragma once

#include "rt_device.h"

template <typename T, int LPC, int APL, typename Ang>
__device__ __forceinline__ void rt_source_vjp_cell(const rt_step_args &a, const Ang &ang, int64_t cell, int l,
                                                   const T (&Io)[APL], T (&lam)[APL], double Vp) {
  constexpr int P = Ang::P;
  constexpr bool PAIRED = Ang::PAIRED_LAYOUT;
  const double rho = a.rho[cell];
  const double kP = a.kP[cell], kJ = a.kJ[cell], ks = a.ks[cell];
  const double *tp = a.src_tape + RT_SRC_TAPE * cell;
  const double m0 = tp[RT_TAPE_M], m1 = tp[RT_TAPE_M + 1], m2 = tp[RT_TAPE_M + 2];
  const double iQ = tp[RT_TAPE_IQ], S1 = tp[RT_TAPE_S1], SG = tp[RT_TAPE_SG], SI = tp[RT_TAPE_SI];
  const double iD = tp[RT_TAPE_ID], Tq = tp[RT_TAPE_T];
  const double c = a.c_light, ic = a.inv_c, dt = a.dt;
  const double irho = rt_rcp(rho);
  const double vx = m0 * irho, vy = m1 * irho, vz = m2 * irho;
  const double gam = rsqrt(1.0 - (vx * vx + vy * vy + vz * vz) * (ic * ic));
  const double y = dt * a.c_red * rho;
  const double chi = kJ + ks;
  const double rcv = rho * a.cv;
  const double T3 = Tq * Tq * Tq, T4 = T3 * Tq;
  const double planck = a.a_4pi * T4;
  const double Jc = (SI + y * kP * SG * planck) * iD;
  const double Ssrc = kP * planck + ks * Jc;
  const double fourpi = 4.0 * RT_PI;
  const double Aq = dt * c * rho * kP * a.a_rad * S1 * iD;

  const T tg = (T)gam, tvx = (T)(vx * ic), tvy = (T)(vy * ic), tvz = (T)(vz * ic);
  const T yA = (T)y, ychiA = (T)(y * chi), SsA = (T)Ssrc, iQA = (T)iQ;
  // the gas bookkeeping hands I* - I' to the gas: the energy and momentum adjoints reach
  // each angle as 4 pi W (c lamE + n.lamM) / cbar
  const double lEp = a.lamE[cell];
  const double lmp0 = a.lamM[3 * cell], lmp1 = a.lamM[3 * cell + 1], lmp2 = a.lamM[3 * cell + 2];
  const T clE = (T)(c * lEp), lm0 = (T)lmp0, lm1 = (T)lmp1, lm2 = (T)lmp2, mg = (T)a.m_gain;

  // Between the passes a lane keeps only I', the adjoint (dL/dI' net of the bookkeeping
  // after the first pass, dL/dI* at the end), v.n / c per direction, and 1 / Gamma and r
  // per slot; each pass rebuilds the other forward quantities from them.  Empty register
  // barriers on the kept values make the rebuild real: without them the compiler holds
  // every intermediate across the group sums.  At 96^3 x 80 with antipodes side by side
  // (transpose of transport fused in front): FP32 222 registers per lane, two waves per
  // SIMD, 0.83 ms per launch; with the barriers 160 registers, three waves, 0.65 ms (FP64
  // 350 -> 256 registers, 1.64 -> 1.08 ms).  Forcing a fourth FP32 wave spills: 0.71 ms.
  struct Fw {
    T G, iG, iG2, iG4, r, I0, X;
  };
  T iGk[APL], rk[APL];  // 1 / Gamma and r per slot, kept from the first pass
  auto fw = [&](int s, T vn, bool first) {  // slot s, v.n / c along the slot's own direction
    Fw f;
    f.G = tg * (T(1) - vn);
    f.iG = first ? rt_rcp(f.G) : iGk[s];
    f.iG2 = f.iG * f.iG;
    f.iG4 = f.iG2 * f.iG2;
    const T den = T(1) + ychiA * f.G;  // 1 / r
    f.r = first ? rt_rcp(den) : rk[s];
    iGk[s] = f.iG;
    rk[s] = f.r;
    const T G2 = f.G * f.G;
    // X = Gamma^4 I* + y Gamma S from the step's output I' = X r / Gamma^4; Gamma^4 I* = X - y
    // Gamma S cancels where the cell is optically thick (r << 1), but every use of it below is
    // scaled by r again, so its absolute error stays at the rounding of I'
    f.X = Io[s] * (G2 * G2) * den;
    f.I0 = f.X - yA * f.G * SsA;
    return f;
  };
  auto through = [&](int s, T nl) { return (T)ang.wt(s) * mg * (clE + nl); };
  constexpr int H = PAIRED ? 2 : 1;  // slots per stored direction
  T vnp[P];

  // ---- first pass: dL/dI' net of the bookkeeping, and dL/dS ------------------------------
  double lS = 0.0;
#pragma unroll
  for (int q = 0; q < P; ++q) {
    const T vn = tvx * ang.dx(q) + tvy * ang.dy(q) + tvz * ang.dz(q);
    const T nl = ang.dx(q) * lm0 + ang.dy(q) * lm1 + ang.dz(q) * lm2;
    vnp[q] = vn;
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const int s = q + h * P;
      const Fw f = fw(s, h ? -vn : vn, true);  // the antipode has direction -n
      // a slot past K (general layout) holds no angle: its weight is zero, and so must be
      // its adjoint, whatever the slot's row entry holds
      const T ell = (ang.ok[s] ? lam[s] : T(0)) - through(s, h ? -nl : nl);
      lam[s] = ell;
      lS += (double)(ell * f.iG4 * yA * f.G * f.r);
    }
  }
  lS = rt_group_sum<LPC>(lS);

  // ---- per cell: S -> J, T -> the root's A and C -> the sums, kappas, gas state ----------
  double lkP = lS * planck, lkJ = 0.0;
  double lplanck = lS * kP;
  const double lJc = lS * ks;
  double lSI = lJc * iD;
  lkP += lJc * y * SG * planck * iD;
  double lSG = lJc * y * kP * planck * iD;
  lplanck += lJc * y * kP * SG * iD;
  double lD = -lJc * Jc * iD;
  const double lT = lplanck * a.a_rad * T3 * (4.0 / fourpi);
  const double iFp = rt_rcp(4.0 * Aq * T3 + rcv);
  const double lA = -lT * T4 * iFp;
  const double lC = lT * iFp;
  lkP += lA * dt * c * rho * a.a_rad * S1 * iD;
  double lS1 = lA * dt * c * rho * kP * a.a_rad * iD;
  lD -= lA * Aq * iD;
  // C = rho cv T^n + dt c rho 4 pi kJ SI / D, with T^n = (E_g - |m|^2 / 2 rho) / (rho cv):
  // dL/dE_g gains lC and dL/dm gains -lC v
  lkJ += lC * dt * c * rho * fourpi * SI * iD;
  lSI += lC * dt * c * rho * fourpi * kJ * iD;
  lD -= lC * dt * c * rho * fourpi * kJ * SI * (iD * iD);
  lS1 += lD;
  lkJ += lD * y * SG;
  lSG += lD * y * kJ;
  const T lS1A = (T)lS1, lSGA = (T)lSG, lSIA = (T)lSI;

  // The adjoints of the sums' weights Wt and of r = 1 / (1 + y chi Gamma), per slot, from
  // the first pass's dL/dI' (ell): dL/d(X r) = ell Gamma^-4, dL/dr = that X plus the sums'.
  struct Bw {
    T Wt, lWt, lden;
  };
  auto bw = [&](int s, const Fw &f, T ell) {
    Bw b;
    b.Wt = (T)ang.wt(s) * f.iG2 * iQA;
    const T Z = lS1A + lSGA * f.G + lSIA * f.I0;
    b.lWt = Z * f.r;
    const T lr = ell * f.iG4 * f.X + Z * b.Wt;
    b.lden = -lr * f.r * f.r;
    return b;
  };

  // ---- second pass: dL/dchi through r and the weights' normalisation ---------------------
#pragma unroll
  for (int q = 0; q < P; ++q) asm volatile("" : "+v"(vnp[q]));
#pragma unroll
  for (int q = 0; q < APL; ++q) asm volatile("" : "+v"(iGk[q]), "+v"(rk[q]));
  double lchi = 0.0, sw = 0.0;
#pragma unroll
  for (int q = 0; q < P; ++q) {
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const int s = q + h * P;
      const Fw f = fw(s, h ? -vnp[q] : vnp[q], false);
      const Bw b = bw(s, f, lam[s]);
      lchi += (double)(b.lden * yA * f.G);
      sw += (double)(b.lWt * b.Wt);
    }
  }
  lchi = rt_group_sum<LPC>(lchi);
  sw = rt_group_sum<LPC>(sw);
  lkJ += lchi;

  // ---- third pass: Wt through Gamma^-2, I0 = Gamma^4 I*, Gamma through gamma and v --------
#pragma unroll
  for (int q = 0; q < P; ++q) asm volatile("" : "+v"(vnp[q]));
#pragma unroll
  for (int q = 0; q < APL; ++q) asm volatile("" : "+v"(iGk[q]), "+v"(rk[q]));
  const T swA = (T)sw, igamA = (T)(1.0 / gam), glc = (T)(gam * ic);
  double lgam = 0.0, lvx = 0.0, lvy = 0.0, lvz = 0.0;
#pragma unroll
  for (int q = 0; q < P; ++q) {
    const T nl = ang.dx(q) * lm0 + ang.dy(q) * lm1 + ang.dz(q) * lm2;
    double gs = 0.0;  // sum of dL/dGamma * dGamma/d(v.n) along +n over the slots
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const int s = q + h * P;
      const Fw f = fw(s, h ? -vnp[q] : vnp[q], false);
      const T ell = lam[s];
      const Bw b = bw(s, f, ell);
      const T lIn = ell * f.iG4;
      const T lIco = lIn * f.r + lSIA * b.Wt * f.r;
      const T lq = (b.lWt - swA) * iQA;
      const T qv = (T)ang.wt(s) * f.iG2;  // W Gamma^-2, the sums' unnormalised weight
      const T lg = T(-4) * ell * f.X * f.r * f.iG4 * f.iG + lIn * yA * SsA * f.r + lSGA * b.Wt * f.r +
                   b.lden * ychiA + lq * (T(-2) * qv * f.iG) + lIco * T(4) * f.I0 * f.iG;
      const T G2 = f.G * f.G;
      lam[s] = through(s, h ? -nl : nl) + lIco * G2 * G2;
      lgam += (double)(lg * f.G * igamA);
      // Gamma = gamma (1 -+ v.n / c): dGamma/dv = -+ gamma n / c
      gs += (double)(h == 0 ? -(lg * glc) : lg * glc);
    }
    lvx += gs * (double)ang.dx(q);
    lvy += gs * (double)ang.dy(q);
    lvz += gs * (double)ang.dz(q);
  }
  lgam = rt_group_sum<LPC>(lgam);
  lvx = rt_group_sum<LPC>(lvx);
  lvy = rt_group_sum<LPC>(lvy);
  lvz = rt_group_sum<LPC>(lvz);
  const T iVp = (T)rt_rcp(Vp);
#pragma unroll
  for (int q = 0; q < APL; ++q) lam[q] *= iVp;
  if (l == 0) {
    // v = m / rho and gamma(v): dL/dm = (dL/dv + dL/dgamma gamma^3 v / c^2) / rho
    const double g3 = gam * gam * gam * (ic * ic);
    a.lamE[cell] = lEp + lC;
    a.lamM[3 * cell] = lmp0 - lC * vx + (lvx + lgam * g3 * vx) * irho;
    a.lamM[3 * cell + 1] = lmp1 - lC * vy + (lvy + lgam * g3 * vy) * irho;
    a.lamM[3 * cell + 2] = lmp2 - lC * vz + (lvz + lgam * g3 * vz) * irho;
    if (a.dkP) a.dkP[cell] += lkP;
    if (a.dkJ) a.dkJ[cell] += lkJ;
  }
}

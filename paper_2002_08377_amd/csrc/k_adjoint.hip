// Reverse mode of one first-order radiation step, for gradients of a scalar loss.
//
// k_source_vjp: per cell, recompute the forward source update (section 2.3) and
// push the output adjoints back through it: the lab bookkeeping of eqs. 35-36,
// the boost back, the implicit per-angle update of eq. 28, the temperature root
// (implicit function theorem: dT = -(T^4 dA + T dB - dC)/(4 A T^3 + B)), the
// comoving sums and weights, the Lorentz factors and the gas velocity.
//
// It writes lam*/V' (dL/dI* per unit of charge) for the transpose of the upwind
// charge update, which is the step kernel's adjoint-transport mode (k_step.hip):
//   lam_i = (V_i/V'_i) lam*_i + sum_{faces, g>0} g (lam*_j/V'_j - lam*_i/V'_i).
#include "rt_device.h"

namespace {

template <typename T, int LPC, int APL>
__global__ __launch_bounds__(RT_BLOCK) void k_source_vjp(rt_adj_args a, int64_t nblk) {
  const int64_t lb = rt_logical_block(nblk);
  if (lb < 0) return;
  constexpr int CPB = RT_BLOCK / LPC;
  const int64_t cell = lb * CPB + threadIdx.x / LPC;
  if (cell >= a.N) return;
  const int l = threadIdx.x % LPC;
  const int K = a.K;
  // Per-angle arithmetic is done in the intensities' type A (FP32 in the FP32 form, as the
  // forward source does); every sum over angles and every per-cell quantity stays FP64.
  using A = T;
  rt_lane_angles<A, LPC, APL> ang;
  ang.load(a.dirs, a.W, K, l);
  const T *Is = (const T *)a.I_star;
  const T *LI = (const T *)a.lamI;
  const int64_t row = cell * (int64_t)K;

  const double rho = a.rho[cell];
  const double mom[3] = {a.mom[3 * cell], a.mom[3 * cell + 1], a.mom[3 * cell + 2]};
  const double etot = a.etot[cell];
  const double kP = a.kP[cell], kJ = a.kJ[cell], ks = a.ks[cell];
  const double c = a.c_light, cb = a.c_red, dt = a.dt;
  const double fourpi = 4.0 * RT_PI;
  const double irho = rt_rcp(rho), ic = rt_rcp(c), icb = rt_rcp(cb);
  const double v[3] = {mom[0] * irho, mom[1] * irho, mom[2] * irho};
  const double gam = rsqrt(1.0 - (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) * (ic * ic));
  const double y = dt * cb * rho;
  const double chi = kJ + ks;

  // forward recompute (reciprocals instead of divisions; the same root as the forward step)
  const A vA[3] = {(A)v[0], (A)v[1], (A)v[2]}, icA = (A)ic, gamA = (A)gam, yA = (A)y, chiA = (A)chi;
  const A ychiA = (A)(y * chi);
  A Gm[APL], iGm[APL], Ico[APL], rr[APL], qv[APL], Iout[APL];
  double sQ = 0, s1 = 0, sG = 0, sI = 0;
#pragma unroll
  for (int q = 0; q < APL; ++q) {
    const A I = ang.ok[q] ? (A)Is[row + ang.k[q]] : A(0);
    const A G = gamA * (A(1) - (vA[0] * ang.dx[q] + vA[1] * ang.dy[q] + vA[2] * ang.dz[q]) * icA);
    const A iG = rt_rcp(G);
    const A G2 = G * G;
    Gm[q] = G;
    iGm[q] = iG;
    Ico[q] = G2 * G2 * I;
    qv[q] = (A)ang.w[q] * (iG * iG);
    rr[q] = rt_rcp(A(1) + ychiA * G);
    sQ += (double)qv[q];
    s1 += (double)(qv[q] * rr[q]);
    sG += (double)(qv[q] * G * rr[q]);
    sI += (double)(qv[q] * Ico[q] * rr[q]);
  }
  sQ = rt_group_sum<LPC>(sQ);
  s1 = rt_group_sum<LPC>(s1);
  sG = rt_group_sum<LPC>(sG);
  sI = rt_group_sum<LPC>(sI);
  const double iQ = rt_rcp(sQ);
  const double S1 = s1 * iQ, SG = sG * iQ, SI = sI * iQ;
  const double D = S1 + y * kJ * SG;
  const double iD = rt_rcp(D);
  const double rcv = rho * a.cv, ircv = rt_rcp(rcv);
  const double m2 = mom[0] * mom[0] + mom[1] * mom[1] + mom[2] * mom[2];
  const double Tn = (etot - 0.5 * m2 * irho) * ircv;
  const double Aq = dt * c * rho * kP * a.a_rad * S1 * iD;
  const double Bq = rcv;
  const double Cq = rcv * Tn + dt * c * rho * fourpi * kJ * SI * iD;
  const double Tq = rt_quartic_root_from(Aq, Bq, Cq, Tn);
  const double T3 = Tq * Tq * Tq, T4 = T3 * Tq;
  const double planck = a.a_rad * T4 * (1.0 / fourpi);
  const double Jc = (SI + y * kP * SG * planck) * iD;
  const double Ssrc = kP * planck + ks * Jc;
  const A SsA = (A)Ssrc;
#pragma unroll
  for (int q = 0; q < APL; ++q) {
    const A iG2 = iGm[q] * iGm[q];
    Iout[q] = (Ico[q] + yA * Gm[q] * SsA) * rr[q] * (iG2 * iG2);
  }

  // reverse
  const double lEp = a.lamE[cell];
  const double lmp[3] = {a.lamM[3 * cell], a.lamM[3 * cell + 1], a.lamM[3 * cell + 2]};
  const A lmA[3] = {(A)lmp[0], (A)lmp[1], (A)lmp[2]}, clEA = (A)(c * lEp), icbA = (A)icb;
  A lIn[APL], lGam[APL], lIco[APL], lr[APL], lam[APL];
  double lS = 0.0;
#pragma unroll
  for (int q = 0; q < APL; ++q) {
    const A iG2 = iGm[q] * iGm[q];
    const A nl = ang.dx[q] * lmA[0] + ang.dy[q] * lmA[1] + ang.dz[q] * lmA[2];
    const A through = (A)(fourpi * ang.w[q]) * ((clEA + nl) * icbA);
    const A lin = ang.ok[q] ? (A)LI[row + ang.k[q]] : A(0);
    const A ell = lin - through;
    lam[q] = through;
    lIn[q] = ell * (iG2 * iG2);
    lGam[q] = A(-4) * ell * Iout[q] * iGm[q];
    lIco[q] = lIn[q] * rr[q];
    lS += (double)(lIn[q] * yA * Gm[q] * rr[q]);
    lGam[q] += lIn[q] * yA * SsA * rr[q];
    lr[q] = lIn[q] * (Ico[q] + yA * Gm[q] * SsA);
  }
  lS = rt_group_sum<LPC>(lS);
  double lkP = lS * planck, lkJ = 0.0;
  double lplanck = lS * kP;
  const double lJc = lS * ks;
  double lSI = lJc * iD;
  lkP += lJc * y * SG * planck * iD;
  double lSG = lJc * y * kP * planck * iD;
  lplanck += lJc * y * kP * SG * iD;
  double lD = -lJc * Jc * iD;
  const double lT = lplanck * a.a_rad * T3 * (4.0 / fourpi);
  const double iFp = rt_rcp(4.0 * Aq * T3 + Bq);
  const double lA = -lT * T4 * iFp;
  const double lC = lT * iFp;
  lkP += lA * dt * c * rho * a.a_rad * S1 * iD;
  double lS1 = lA * dt * c * rho * kP * a.a_rad * iD;
  lD -= lA * Aq * iD;
  const double lTn = lC * rcv;
  lkJ += lC * dt * c * rho * fourpi * SI * iD;
  lSI += lC * dt * c * rho * fourpi * kJ * iD;
  lD -= lC * dt * c * rho * fourpi * kJ * SI * (iD * iD);
  const double lE = lEp + lTn * ircv;
  double lm[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) lm[d] = lmp[d] - lTn * mom[d] * (irho * irho) * (1.0 / a.cv);
  lS1 += lD;
  lkJ += lD * y * SG;
  lSG += lD * y * kJ;
  const A lS1A = (A)lS1, lSGA = (A)lSG, lSIA = (A)lSI, iQA = (A)iQ;
  double lchi = 0.0, sw = 0.0;
  A lWt[APL];
#pragma unroll
  for (int q = 0; q < APL; ++q) {
    const A Wt = qv[q] * iQA;
    lWt[q] = lS1A * rr[q] + lSGA * Gm[q] * rr[q] + lSIA * Ico[q] * rr[q];
    lr[q] += lS1A * Wt + lSGA * Wt * Gm[q] + lSIA * Wt * Ico[q];
    lGam[q] += lSGA * Wt * rr[q];
    lIco[q] += lSIA * Wt * rr[q];
    const A lden = -lr[q] * rr[q] * rr[q];
    lchi += (double)(lden * yA * Gm[q]);
    lGam[q] += lden * yA * chiA;
    sw += (double)(lWt[q] * Wt);
  }
  lchi = rt_group_sum<LPC>(lchi);
  sw = rt_group_sum<LPC>(sw);
  lkJ += lchi;
  const double igam = rt_rcp(gam);
  const A swA = (A)sw, igamA = (A)igam;
  double lgam = 0.0, lv[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < APL; ++q) {
    const A G2 = Gm[q] * Gm[q];
    const A lq = (lWt[q] - swA) * iQA;
    lGam[q] += lq * (A(-2) * qv[q] * iGm[q]);
    lam[q] += lIco[q] * G2 * G2;
    lGam[q] += lIco[q] * A(4) * Ico[q] * iGm[q];
    lgam += (double)(lGam[q] * Gm[q] * igamA);
    const A gl = lGam[q] * gamA * icA;
    lv[0] -= (double)(gl * ang.dx[q]);
    lv[1] -= (double)(gl * ang.dy[q]);
    lv[2] -= (double)(gl * ang.dz[q]);
  }
  lgam = rt_group_sum<LPC>(lgam);
  lv[0] = rt_group_sum<LPC>(lv[0]);
  lv[1] = rt_group_sum<LPC>(lv[1]);
  lv[2] = rt_group_sum<LPC>(lv[2]);
  // the transport adjoint takes dL/dI* per unit of charge: lam* / V'
  const double iVp = rt_rcp(rt_vol_next(a.vol_n[cell], dt, a.D[cell]));
  T *LS = (T *)a.lam_star;
#pragma unroll
  for (int q = 0; q < APL; ++q)
    if (ang.ok[q]) LS[row + ang.k[q]] = (T)((double)lam[q] * iVp);
  if (l == 0) {
    const double g3 = gam * gam * gam * (ic * ic);
    a.lamE[cell] = lE;
#pragma unroll
    for (int d = 0; d < 3; ++d) a.lamM[3 * cell + d] = lm[d] + (lv[d] + lgam * g3 * v[d]) * irho;
    if (a.dkP) a.dkP[cell] += lkP;
    if (a.dkJ) a.dkJ[cell] += lkJ;
  }
}

template <typename T, int LPC, int APL> hipError_t launch(const rt_adj_args &a, hipStream_t s) {
  const int64_t cpb = RT_BLOCK / LPC;
  const int64_t nblk = (a.N + cpb - 1) / cpb;
  const dim3 grid((unsigned)rt_grid_for(nblk));
  hipLaunchKernelGGL((k_source_vjp<T, LPC, APL>), grid, dim3(RT_BLOCK), 0, s, a, nblk);
  return hipGetLastError();
}

template <typename T> hipError_t dispatch(const rt_adj_args &a, hipStream_t s) {
  const int K = a.K;
  if (K % 16 == 0 || K > 64) {
    switch ((K + 15) / 16) {
      case 1: return launch<T, 16, 1>(a, s);
      case 2: return launch<T, 16, 2>(a, s);
      case 3: return launch<T, 16, 3>(a, s);
      case 4: return launch<T, 16, 4>(a, s);
      case 5: return launch<T, 16, 5>(a, s);
      case 6: return launch<T, 16, 6>(a, s);
      case 7: return launch<T, 16, 7>(a, s);
      case 8: return launch<T, 16, 8>(a, s);
    }
  } else {
    switch ((K + 7) / 8) {
      case 1: return launch<T, 8, 1>(a, s);
      case 2: return launch<T, 8, 2>(a, s);
      case 3: return launch<T, 8, 3>(a, s);
      case 4: return launch<T, 8, 4>(a, s);
      case 5: return launch<T, 8, 5>(a, s);
      case 6: return launch<T, 8, 6>(a, s);
      case 7: return launch<T, 8, 7>(a, s);
      case 8: return launch<T, 8, 8>(a, s);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t rt_launch_adjoint(const rt_adj_args &a, int dtype, hipStream_t s) {
  return dtype == RT_F32 ? dispatch<float>(a, s) : dispatch<double>(a, s);
}

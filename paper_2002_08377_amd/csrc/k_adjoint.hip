// Reverse mode of one first-order radiation step, for gradients of a scalar loss.
//
// k_source_vjp: per cell, recompute the forward source update (section 2.3) and
// push the output adjoints back through it: the lab bookkeeping of eqs. 35-36,
// the boost back, the implicit per-angle update of eq. 28, the temperature root
// (implicit function theorem: dT = -(T^4 dA + T dB - dC)/(4 A T^3 + B)), the
// comoving sums and weights, the Lorentz factors and the gas velocity.
//
// k_transport_vjp: the exact transpose of the upwind charge update, gathered per
// cell over the faces it is upwind of:
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
  rt_lane_angles<double, LPC, APL> ang;
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
  const double v[3] = {mom[0] / rho, mom[1] / rho, mom[2] / rho};
  const double gam = 1.0 / sqrt(1.0 - (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) / (c * c));
  const double y = dt * cb * rho;
  const double chi = kJ + ks;

  // forward recompute
  double Gm[APL], Ico[APL], rr[APL], qv[APL], Iout[APL];
  double sQ = 0, s1 = 0, sG = 0, sI = 0;
#pragma unroll
  for (int q = 0; q < APL; ++q) {
    const double I = ang.ok[q] ? (double)Is[row + ang.k[q]] : 0.0;
    const double G = gam * (1.0 - (v[0] * ang.dx[q] + v[1] * ang.dy[q] + v[2] * ang.dz[q]) / c);
    const double G2 = G * G;
    Gm[q] = G;
    Ico[q] = G2 * G2 * I;
    qv[q] = ang.w[q] / G2;
    rr[q] = 1.0 / (1.0 + y * chi * G);
    sQ += qv[q];
    s1 += qv[q] * rr[q];
    sG += qv[q] * G * rr[q];
    sI += qv[q] * Ico[q] * rr[q];
  }
  sQ = rt_group_sum<LPC>(sQ);
  s1 = rt_group_sum<LPC>(s1);
  sG = rt_group_sum<LPC>(sG);
  sI = rt_group_sum<LPC>(sI);
  const double Qn = sQ, S1 = s1 / Qn, SG = sG / Qn, SI = sI / Qn;
  const double D = S1 + y * kJ * SG;
  const double m2 = mom[0] * mom[0] + mom[1] * mom[1] + mom[2] * mom[2];
  const double Tn = (etot - 0.5 * m2 / rho) / (rho * a.cv);
  const double Aq = dt * c * rho * kP * a.a_rad * S1 / D;
  const double Bq = rho * a.cv;
  const double Cq = rho * a.cv * Tn + dt * c * rho * fourpi * kJ * SI / D;
  const double Tq = rt_quartic_root(Aq, Bq, Cq);
  const double T3 = Tq * Tq * Tq, T4 = T3 * Tq;
  const double planck = a.a_rad * T4 / fourpi;
  const double Jc = (SI + y * kP * SG * planck) / D;
  const double Ssrc = kP * planck + ks * Jc;
#pragma unroll
  for (int q = 0; q < APL; ++q) {
    const double G2 = Gm[q] * Gm[q];
    Iout[q] = (Ico[q] + y * Gm[q] * Ssrc) * rr[q] / (G2 * G2);
  }

  // reverse
  const double lEp = a.lamE[cell];
  const double lmp[3] = {a.lamM[3 * cell], a.lamM[3 * cell + 1], a.lamM[3 * cell + 2]};
  double lIn[APL], lGam[APL], lIco[APL], lr[APL], lam[APL];
  double lS = 0.0;
#pragma unroll
  for (int q = 0; q < APL; ++q) {
    const double G2 = Gm[q] * Gm[q];
    const double nl = ang.dx[q] * lmp[0] + ang.dy[q] * lmp[1] + ang.dz[q] * lmp[2];
    const double through = fourpi * ang.w[q] * ((c / cb) * lEp + nl / cb);
    const double lin = ang.ok[q] ? (double)LI[row + ang.k[q]] : 0.0;
    const double ell = lin - through;
    lam[q] = through;
    lIn[q] = ell / (G2 * G2);
    lGam[q] = -4.0 * ell * Iout[q] / Gm[q];
    lIco[q] = lIn[q] * rr[q];
    lS += lIn[q] * y * Gm[q] * rr[q];
    lGam[q] += lIn[q] * y * Ssrc * rr[q];
    lr[q] = lIn[q] * (Ico[q] + y * Gm[q] * Ssrc);
  }
  lS = rt_group_sum<LPC>(lS);
  double lkP = lS * planck, lkJ = 0.0;
  double lplanck = lS * kP;
  const double lJc = lS * ks;
  double lSI = lJc / D;
  lkP += lJc * y * SG * planck / D;
  double lSG = lJc * y * kP * planck / D;
  lplanck += lJc * y * kP * SG / D;
  double lD = -lJc * Jc / D;
  const double lT = lplanck * a.a_rad * T3 / RT_PI;
  const double Fp = 4.0 * Aq * T3 + Bq;
  const double lA = -lT * T4 / Fp;
  const double lC = lT / Fp;
  lkP += lA * dt * c * rho * a.a_rad * S1 / D;
  double lS1 = lA * dt * c * rho * kP * a.a_rad / D;
  lD -= lA * Aq / D;
  const double lTn = lC * rho * a.cv;
  lkJ += lC * dt * c * rho * fourpi * SI / D;
  lSI += lC * dt * c * rho * fourpi * kJ / D;
  lD -= lC * dt * c * rho * fourpi * kJ * SI / (D * D);
  const double lE = lEp + lTn / (rho * a.cv);
  double lm[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) lm[d] = lmp[d] - lTn * mom[d] / (rho * rho * a.cv);
  lS1 += lD;
  lkJ += lD * y * SG;
  lSG += lD * y * kJ;
  double lchi = 0.0, sw = 0.0;
  double lWt[APL];
#pragma unroll
  for (int q = 0; q < APL; ++q) {
    const double Wt = qv[q] / Qn;
    lWt[q] = lS1 * rr[q] + lSG * Gm[q] * rr[q] + lSI * Ico[q] * rr[q];
    lr[q] += lS1 * Wt + lSG * Wt * Gm[q] + lSI * Wt * Ico[q];
    lGam[q] += lSG * Wt * rr[q];
    lIco[q] += lSI * Wt * rr[q];
    const double lden = -lr[q] * rr[q] * rr[q];
    lchi += lden * y * Gm[q];
    lGam[q] += lden * y * chi;
    sw += lWt[q] * Wt;
  }
  lchi = rt_group_sum<LPC>(lchi);
  sw = rt_group_sum<LPC>(sw);
  lkJ += lchi;
  double lgam = 0.0, lv[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < APL; ++q) {
    const double G2 = Gm[q] * Gm[q];
    const double lq = (lWt[q] - sw) / Qn;
    lGam[q] += lq * (-2.0 * qv[q] / Gm[q]);
    lam[q] += lIco[q] * G2 * G2;
    lGam[q] += lIco[q] * 4.0 * Ico[q] / Gm[q];
    lgam += lGam[q] * Gm[q] / gam;
    lv[0] -= lGam[q] * gam * ang.dx[q] / c;
    lv[1] -= lGam[q] * gam * ang.dy[q] / c;
    lv[2] -= lGam[q] * gam * ang.dz[q] / c;
  }
  lgam = rt_group_sum<LPC>(lgam);
  lv[0] = rt_group_sum<LPC>(lv[0]);
  lv[1] = rt_group_sum<LPC>(lv[1]);
  lv[2] = rt_group_sum<LPC>(lv[2]);
  T *LS = (T *)a.lam_star;
#pragma unroll
  for (int q = 0; q < APL; ++q)
    if (ang.ok[q]) LS[row + ang.k[q]] = (T)lam[q];
  if (l == 0) {
    const double g3 = gam * gam * gam / (c * c);
    a.lamE[cell] = lE;
#pragma unroll
    for (int d = 0; d < 3; ++d) a.lamM[3 * cell + d] = lm[d] + (lv[d] + lgam * g3 * v[d]) / rho;
    if (a.dkP) a.dkP[cell] += lkP;
    if (a.dkJ) a.dkJ[cell] += lkJ;
  }
}

template <typename T, int LPC, int APL>
__global__ __launch_bounds__(RT_BLOCK) void k_transport_vjp(rt_adj_args a, int64_t nblk) {
  using V4 = typename rt_vec4<T>::type;
  const int64_t lb = rt_logical_block(nblk);
  if (lb < 0) return;
  constexpr int CPB = RT_BLOCK / LPC;
  const int64_t cell = lb * CPB + threadIdx.x / LPC;
  if (cell >= a.N) return;
  const int l = threadIdx.x % LPC;
  const int K = a.K;
  rt_lane_angles<T, LPC, APL> ang;
  ang.load(a.dirs, a.W, K, l);
  const T *LS = (const T *)a.lam_star;
  const int64_t row = cell * (int64_t)K;
  const double Vn = a.vol_n[cell];
  const double Vp = Vn + a.dt * a.D[cell];
  const T ivs = (T)(1.0 / Vp);
  T ls[APL], acc[APL];
#pragma unroll
  for (int q = 0; q < APL; ++q) {
    ls[q] = ang.ok[q] ? LS[row + ang.k[q]] : T(0);
    acc[q] = (T)(Vn / Vp) * ls[q];
  }
  const T sc = (T)(a.dt * a.c_red), sd = (T)a.dt;
  const V4 *an = (const V4 *)a.hf_an;
  const int h0 = a.row_ptr[cell], h1 = a.row_ptr[cell + 1];
  for (int h = h0; h < h1; ++h) {
    const int64_t j = a.hf_nbr[h];
    const V4 r = an[h];
    const T ax = sc * r.x, ay = sc * r.y, az = sc * r.z, b = sd * r.w;
    const T ivj = (T)(1.0 / (a.vol_n[j] + a.dt * a.D[j]));
    const T *Lj = LS + j * K;
#pragma unroll
    for (int q = 0; q < APL; ++q) {
      const T g = ax * ang.dx[q] + ay * ang.dy[q] + az * ang.dz[q] - b;
      const T lj = ang.ok[q] ? Lj[ang.k[q]] : T(0);
      if (g > T(0)) acc[q] += g * (lj * ivj - ls[q] * ivs);
    }
  }
  T *LI = (T *)a.lamI;
#pragma unroll
  for (int q = 0; q < APL; ++q)
    if (ang.ok[q]) LI[row + ang.k[q]] = acc[q];
}

template <typename T, int LPC, int APL> hipError_t launch(const rt_adj_args &a, hipStream_t s) {
  const int64_t cpb = RT_BLOCK / LPC;
  const int64_t nblk = (a.N + cpb - 1) / cpb;
  const dim3 grid((unsigned)rt_grid_for(nblk));
  hipLaunchKernelGGL((k_source_vjp<T, LPC, APL>), grid, dim3(RT_BLOCK), 0, s, a, nblk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_transport_vjp<T, LPC, APL>), grid, dim3(RT_BLOCK), 0, s, a, nblk);
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

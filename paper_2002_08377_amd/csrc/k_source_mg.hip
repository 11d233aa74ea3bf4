// Multigroup implicit source update (section 2.3 with frequency groups coupled only
// through the gas temperature).  Intensities are group-major, I[g][N][K]; opacities
// kP, kJ, ks are [g][N]; group g carries the weight Wg[g] in the moments and the gas
// equation.  One cell per group of LPC lanes, each lane holding APL angles:
//  pass 1, per group: the comoving sums S1, SG, SI (the weights W~ and Gamma are the
//    same for every group), reduced over the lanes and kept in LDS; they add
//    Wg kP S1 / D and Wg kJ SI / D to the quartic's coefficients;
//  the temperature: A T^4 + B T - C = 0 in FP64, as in the grey update;
//  pass 2, per group: the row is read again and updated, I' = I r + (r / Gamma^3) y S_g
//    with S_g = kP_g a T^4/4pi + ks_g J~_g, and the radiation energy and momentum lost
//    by the stored values (weighted by Wg) go to the gas.
#include "rt_step_common.h"

namespace {

template <typename T, int LPC, int APL, bool FULL, int PAIRED>
__global__ __launch_bounds__(RT_BLOCK) void k_source_mg(rt_mg_args a, int64_t nblk) {
  using Ang = rt_step_angles<T, LPC, APL, FULL, PAIRED>;
  constexpr int P = Ang::P;
  constexpr int CPB = RT_BLOCK / LPC;
  extern __shared__ __align__(16) unsigned char rt_smem[];
  double *s_grp = (double *)rt_smem;  // [CPB][G][4]: S1, SG, SI, 1/D
  const int64_t lb = rt_logical_block(nblk);
  if (lb < 0) return;
  const int g = threadIdx.x / LPC;
  const int64_t cell = lb * CPB + g;
  if (cell >= a.N) return;
  const int l = threadIdx.x % LPC;
  const int K = a.K, G = a.G;
  const int64_t N = a.N;
  Ang ang;
  ang.load(a.dirs, a.W, K, l);
  double *sg = s_grp + (int64_t)g * G * 4;

  const double rho = a.rho[cell];
  const double m0 = a.mom[3 * cell], m1 = a.mom[3 * cell + 1], m2 = a.mom[3 * cell + 2];
  const double Eg = a.etot[cell];
  const double irho = rt_rcp(rho);
  const double vx = m0 * irho, vy = m1 * irho, vz = m2 * irho;
  const double ic = a.inv_c;
  const double gam = rsqrt(1.0 - (vx * vx + vy * vy + vz * vz) * (ic * ic));
  const double y = a.dt * a.c_red * rho;
  const T tg = (T)gam, tvx = (T)(vx * ic), tvy = (T)(vy * ic), tvz = (T)(vz * ic);
  // group-independent per angle: Gamma and 1/Gamma^2 (the comoving weight W / Gamma^2 is
  // formed again where it is used, which holds fewer registers than keeping it)
  T Gm[APL], iG2[APL];
  double sQ = 0;
#pragma unroll
  for (int q = 0; q < P; ++q) {
    const T vn = tvx * ang.x[q] + tvy * ang.y[q] + tvz * ang.z[q];
    Gm[q] = tg * (T(1) - vn);
    if (PAIRED) Gm[q + P] = tg * (T(1) + vn);
  }
#pragma unroll
  for (int q = 0; q < APL; ++q) {
    const T iG = rt_rcp(Gm[q]);
    iG2[q] = iG * iG;
    sQ += ang.wt(q) * (double)iG2[q];
  }
  sQ = rt_group_sum<LPC>(sQ);
  const double iQ = rt_rcp(sQ);

  // A group's row (and in the FP64 form its opacities) is loaded one group ahead in both
  // passes, so that its memory latency overlaps the previous group's arithmetic.  The FP32
  // form loads the opacities at the top of each group instead: held ahead, their registers
  // would cost a wave per SIMD (174 registers against 160; 1.82 against 1.70 ms at 128^3 x 80,
  // 4 groups), while the FP64 form is 3% faster with them ahead.
  constexpr bool KAPPA_AHEAD = sizeof(T) == 8;
  struct grp {
    T I[APL];
    double kJ, ks, kP;
  };
  auto fetch = [&](int j, grp &o) {
    const int64_t gc = (int64_t)j * N + cell;
    const T *Ir = (const T *)a.I + gc * K;
#pragma unroll
    for (int q = 0; q < APL; ++q) o.I[q] = Ir[ang.k[q]];
    if constexpr (KAPPA_AHEAD) {
      o.kJ = a.kJ[gc];
      o.ks = a.ks[gc];
      o.kP = a.kP[gc];
    }
  };
  auto kappa = [&](int j, const grp &g, double &kJ, double &ks, double &kP) {
    if constexpr (KAPPA_AHEAD) {
      kJ = g.kJ;
      ks = g.ks;
      kP = g.kP;
    } else {
      const int64_t gc = (int64_t)j * N + cell;
      kJ = a.kJ[gc];
      ks = a.ks[gc];
      kP = a.kP[gc];
    }
  };

  // pass 1: per-group comoving sums and the quartic's coefficients
  double Asum = 0, Csum = 0;
  grp cur, nxt;
  fetch(0, cur);
  nxt = cur;  // defined when the last group rotates it in
  for (int j = 0; j < G; ++j) {
    if (j + 1 < G) fetch(j + 1, nxt);
    double kJ, ks, kP;
    kappa(j, cur, kJ, ks, kP);
    const T tyc = (T)(y * (kJ + ks));
    double s1 = 0, sG = 0, sI = 0;
#pragma unroll
    for (int q = 0; q < APL; ++q) {
      const T I = cur.I[q];
      const T r = rt_rcp(T(1) + tyc * Gm[q]);
      const T G2 = Gm[q] * Gm[q];
      const double qk = ang.wt(q) * (double)iG2[q];
      s1 += qk * (double)r;
      sG += qk * (double)(Gm[q] * r);
      sI += qk * (double)(G2 * G2 * I * r);
    }
    s1 = rt_group_sum<LPC>(s1) * iQ;
    sG = rt_group_sum<LPC>(sG) * iQ;
    sI = rt_group_sum<LPC>(sI) * iQ;
    const double iD = rt_rcp(s1 + y * kJ * sG);
    Asum += a.Wg[j] * kP * s1 * iD;
    Csum += a.Wg[j] * kJ * sI * iD;
    if (l == 0) {
      sg[4 * j] = s1;
      sg[4 * j + 1] = sG;
      sg[4 * j + 2] = sI;
      sg[4 * j + 3] = iD;
    }
    cur = nxt;
  }
  const double rcv = rho * a.cv;
  const double Tn = (Eg - 0.5 * (m0 * m0 + m1 * m1 + m2 * m2) * irho) * rt_rcp(rcv);
  const double fourpi = 4.0 * RT_PI;
  const double Aq = a.dt * a.c_light * rho * a.a_rad * Asum;
  const double Cq = rcv * Tn + a.dt * a.c_light * rho * fourpi * Csum;
  const double Tnew = rt_quartic_root_from(Aq, rcv, Cq, Tn);
  const double T4 = Tnew * Tnew * Tnew * Tnew;
  const double planck = a.a_4pi * T4;
  // lane 0's LDS writes are read by the group's other lanes (same wave): release them to the
  // wave, meet, then acquire
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

  // pass 2: per group, update the row and book the energy and momentum handed over
  double dE = 0, dFx = 0, dFy = 0, dFz = 0;
  fetch(0, cur);
  nxt = cur;
  for (int j = 0; j < G; ++j) {
    // the next group's row is another array than this group's, so reading it ahead of
    // this group's stores is safe
    if (j + 1 < G) fetch(j + 1, nxt);
    T *Ir = (T *)a.I + ((int64_t)j * N + cell) * K;
    double kJ, ks, kP;
    kappa(j, cur, kJ, ks, kP);
    const T tyc = (T)(y * (kJ + ks));
    const double Jc = (sg[4 * j + 2] + y * kP * sg[4 * j + 1] * planck) * sg[4 * j + 3];
    const T ySrc = (T)(y * (kP * planck + ks * Jc));
    const double wg = a.Wg[j];
#pragma unroll
    for (int q = 0; q < P; ++q) {
      auto upd = [&](int qq) -> double {
        const T I0 = cur.I[qq];
        const T r = rt_rcp(T(1) + tyc * Gm[qq]);
        const T out = I0 * r + r * iG2[qq] * rt_rcp(Gm[qq]) * ySrc;
        if (ang.ok[qq]) Ir[ang.k[qq]] = out;
        return wg * ang.wt(qq) * ((double)I0 - (double)out);
      };
      double wd = upd(q);
      dE += wd;
      if (PAIRED) {
        const double wd2 = upd(q + P);
        dE += wd2;
        wd -= wd2;  // the antipode's direction is -n
      }
      dFx += wd * (double)ang.x[q];
      dFy += wd * (double)ang.y[q];
      dFz += wd * (double)ang.z[q];
    }
    cur = nxt;
  }
  dE = rt_group_sum<LPC>(dE);
  dFx = rt_group_sum<LPC>(dFx);
  dFy = rt_group_sum<LPC>(dFy);
  dFz = rt_group_sum<LPC>(dFz);
  if (l == 0) {
    a.etot[cell] = Eg + a.e_gain * dE;
    a.mom[3 * cell] = m0 + a.m_gain * dFx;
    a.mom[3 * cell + 1] = m1 + a.m_gain * dFy;
    a.mom[3 * cell + 2] = m2 + a.m_gain * dFz;
    if (a.T_out) a.T_out[cell] = Tnew;
  }
}

template <typename T, int LPC, int APL, bool FULL, int PAIRED>
hipError_t launch(const rt_mg_args &a, hipStream_t s) {
  const int64_t cpb = RT_BLOCK / LPC;
  const int64_t nblk = (a.N + cpb - 1) / cpb;
  const size_t smem = sizeof(double) * 4 * (size_t)a.G * cpb;
  if (smem > 65536) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_source_mg<T, LPC, APL, FULL, PAIRED>), dim3((unsigned)rt_grid_for(nblk)), dim3(RT_BLOCK),
                     smem, s, a, nblk);
  return hipGetLastError();
}

template <typename T, int PAIRED> hipError_t dispatch_paired(const rt_mg_args &a, hipStream_t s) {
  switch (rt_paired_lanes(a.K)) {  // 0 (no paired layout for K) matches no case
    case 0x0802: return launch<T, 8, 2, true, PAIRED>(a, s);
    case 0x0804: return launch<T, 8, 4, true, PAIRED>(a, s);
    case 0x0806: return launch<T, 8, 6, true, PAIRED>(a, s);
    case 0x0808: return launch<T, 8, 8, true, PAIRED>(a, s);
    case 0x080a: return launch<T, 8, 10, true, PAIRED>(a, s);
    case 0x080c: return launch<T, 8, 12, true, PAIRED>(a, s);
    case 0x0402: return launch<T, 4, 2, true, PAIRED>(a, s);
    case 0x0406: return launch<T, 4, 6, true, PAIRED>(a, s);
    case 0x040a: return launch<T, 4, 10, true, PAIRED>(a, s);
  }
  return hipErrorInvalidConfiguration;
}

template <typename T> hipError_t dispatch(const rt_mg_args &a, hipStream_t s) {
  if (a.paired) {
    const hipError_t e = a.paired == 2 ? dispatch_paired<T, 2>(a, s) : dispatch_paired<T, 1>(a, s);
    if (e != hipErrorInvalidConfiguration) return e;
  }
  switch (rt_step_lanes(a.K, 0)) {
    case 0x1001: return launch<T, 16, 1, false, 0>(a, s);
    case 0x1002: return launch<T, 16, 2, false, 0>(a, s);
    case 0x1003: return launch<T, 16, 3, false, 0>(a, s);
    case 0x1004: return launch<T, 16, 4, false, 0>(a, s);
    case 0x1005: return launch<T, 16, 5, false, 0>(a, s);
    case 0x1006: return launch<T, 16, 6, false, 0>(a, s);
    case 0x1007: return launch<T, 16, 7, false, 0>(a, s);
    case 0x1008: return launch<T, 16, 8, false, 0>(a, s);
    case 0x0801: return launch<T, 8, 1, false, 0>(a, s);
    case 0x0802: return launch<T, 8, 2, false, 0>(a, s);
    case 0x0803: return launch<T, 8, 3, false, 0>(a, s);
    case 0x0804: return launch<T, 8, 4, false, 0>(a, s);
    case 0x0805: return launch<T, 8, 5, false, 0>(a, s);
    case 0x0806: return launch<T, 8, 6, false, 0>(a, s);
    case 0x0807: return launch<T, 8, 7, false, 0>(a, s);
    case 0x0808: return launch<T, 8, 8, false, 0>(a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t rt_launch_source_mg(const rt_mg_args &a, int dtype, hipStream_t s) {
  return dtype == RT_F32 ? dispatch<float>(a, s) : dispatch<double>(a, s);
}

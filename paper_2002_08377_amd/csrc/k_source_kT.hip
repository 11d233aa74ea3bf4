// Implicit source update with temperature-dependent opacities (section 2.3: the
// temperature equation solved by Newton-Raphson iteration), one cell per group of LPC
// lanes.  kP(T) = kP0 (T/T_ref)^bP, kJ(T) = kJ0 (T/T_ref)^bJ at T^{n+1}; ks constant.
// With J~ eliminated the temperature equation is
//   f(T) = rho cv (T - T^n) + dt c rho [kP a T^4 S1 - 4 pi kJ SI] / D,
// whose comoving sums depend on T through chi = kJ(T) + ks; every evaluation sums the
// angles again (S1, SG, SI and their chi-derivatives) and reduces over the lanes, so
// all lanes of a cell take the same steps.  The bracket's far end is found from T^n
// (doubling upward while f < 0, halving downward while f > 0); Newton steps start at T^n,
// the bracket's near end from the first step on, and are kept inside [T^n, hi] (or
// [lo, T^n]; bisection when a step leaves it) until a step changes T by at most 1e-14 T
// (such a step is taken as it is); at most 200 evaluations, about 5 in practice.  Where f
// has several roots this gives the first met from T^n in the direction of f's sign.
// Per-angle arithmetic is FP64 in both precision forms; the update and the bookkeeping
// are those of the grey source.
#include "rt_step_common.h"

namespace {

struct kT_eval {
  double kP, kJ, S1, SG, SI, D, f, fp;
};

// Left to itself the compiler gives the larger paired instantiations all 256 registers plus
// accumulation registers, one wave per SIMD; held to two waves the 10-angle ones spill 160
// bytes per lane and still run faster (128^3 x 80: 3.09 -> 2.78 ms FP32, 3.20 -> 3.09 ms
// FP64).  The other layouts keep the compiler's choice.
template <int APL, int PAIRED> struct rt_kT_waves { static constexpr int value = PAIRED && APL <= 10 ? 2 : 1; };
template <typename T, int LPC, int APL, bool FULL, int PAIRED>
__global__ __launch_bounds__(RT_BLOCK) __attribute__((amdgpu_waves_per_eu(rt_kT_waves<APL, PAIRED>::value))) void
k_source_kT(rt_kT_args a, int64_t nblk) {
  using Ang = rt_step_angles<double, LPC, APL, FULL, PAIRED>;
  constexpr int CPB = RT_BLOCK / LPC;
  const int64_t lb = rt_logical_block(nblk);
  if (lb < 0) return;
  const int64_t cell = lb * CPB + threadIdx.x / LPC;
  if (cell >= a.N) return;
  const int l = threadIdx.x % LPC;
  const int K = a.K;
  Ang ang;
  ang.load(a.dirs, a.W, K, l);
  T *Ir = (T *)a.I + cell * (int64_t)K;

  const double rho = a.rho[cell];
  const double m0 = a.mom[3 * cell], m1 = a.mom[3 * cell + 1], m2 = a.mom[3 * cell + 2];
  const double Eg = a.etot[cell];
  const double c = a.c_light, fourpi = 4.0 * RT_PI;
  // reciprocals (within an ulp) and products instead of FP64 divisions
  const double irho = rt_rcp(rho), ic = rt_rcp(c);
  const double vx = m0 * irho, vy = m1 * irho, vz = m2 * irho;
  const double gam = rsqrt(1.0 - (vx * vx + vy * vy + vz * vz) * (ic * ic));
  double Gm[APL], Wt[APL], Ic[APL];
  double norm = 0.0;
#pragma unroll
  for (int q = 0; q < APL; ++q) {
    const double I0 = (double)Ir[ang.k[q]];
    const double vn = vx * ang.dx(q) + vy * ang.dy(q) + vz * ang.dz(q);
    Gm[q] = gam * (1.0 - vn * ic);
    const double G2 = Gm[q] * Gm[q];
    const double iG = rt_rcp(Gm[q]);
    Ic[q] = G2 * G2 * I0;
    Wt[q] = ang.wt(q) * (iG * iG);
    norm += Wt[q];
  }
  norm = rt_group_sum<LPC>(norm);
  const double inorm = rt_rcp(norm);
#pragma unroll
  for (int q = 0; q < APL; ++q) Wt[q] *= inorm;
  const double y = a.dt * a.c_red * rho;
  const double rcv = rho * a.cv;
  const double Tn = (Eg - 0.5 * (m0 * m0 + m1 * m1 + m2 * m2) * irho) * rt_rcp(rcv);
  const double iTref = rt_rcp(a.T_ref);
  const double kP0 = a.kP0[cell], kJ0 = a.kJ0[cell], ks = a.ks[cell];

  auto evaluate = [&](double Tq) {
    kT_eval e;
    // (T/T_ref)^b as exp(b ln(T/T_ref)): within (|b ln(T/T_ref)| + 2) ulp, and far cheaper
    // than pow (whose code alone, even on a branch not taken, costs this kernel registers).
    // The error stays below the Newton stopping tolerance (1e-14 T) while |b ln| < ~40;
    // beyond that the bracketed iteration still ends, through its bisection steps.
    const double lt = log(Tq * iTref);
    const double pP = exp(a.bP * lt);
    e.kP = kP0 * pP;
    e.kJ = kJ0 * (a.bJ == a.bP ? pP : exp(a.bJ * lt));
    const double chi = e.kJ + ks;
    double s1 = 0, sG = 0, sI = 0, p1 = 0, pG = 0, pI = 0;
#pragma unroll
    for (int q = 0; q < APL; ++q) {
      const double r = rt_rcp(1.0 + y * chi * Gm[q]);
      s1 += Wt[q] * r;
      sG += Wt[q] * Gm[q] * r;
      sI += Wt[q] * Ic[q] * r;
      p1 += Wt[q] * Gm[q] * r * r;
      pG += Wt[q] * Gm[q] * Gm[q] * r * r;
      pI += Wt[q] * Ic[q] * Gm[q] * r * r;
    }
    e.S1 = rt_group_sum<LPC>(s1);
    e.SG = rt_group_sum<LPC>(sG);
    e.SI = rt_group_sum<LPC>(sI);
    p1 = rt_group_sum<LPC>(p1);
    pG = rt_group_sum<LPC>(pG);
    pI = rt_group_sum<LPC>(pI);
    e.D = e.S1 + y * e.kJ * e.SG;
    const double T3 = Tq * Tq * Tq, T4 = T3 * Tq;
    const double Nn = e.kP * a.a_rad * T4 * e.S1 - fourpi * e.kJ * e.SI;
    const double iD = rt_rcp(e.D), iTq = rt_rcp(Tq);
    e.f = rcv * (Tq - Tn) + a.dt * c * rho * Nn * iD;
    const double dkP = a.bP * e.kP * iTq, dkJ = a.bJ * e.kJ * iTq;
    const double dS1 = -y * p1 * dkJ, dSG = -y * pG * dkJ, dSI = -y * pI * dkJ;
    const double dD = dS1 + y * (dkJ * e.SG + e.kJ * dSG);
    const double dN = dkP * a.a_rad * T4 * e.S1 + e.kP * a.a_rad * 4.0 * T3 * e.S1 + e.kP * a.a_rad * T4 * dS1 -
                      fourpi * (dkJ * e.SI + e.kJ * dSI);
    e.fp = rcv + a.dt * c * rho * (dN * e.D - Nn * dD) * (iD * iD);
    return e;
  };

  // Bracket the root from T^n, then safeguarded Newton inside the bracket.  One loop with a
  // single evaluation site (mode 0: at T^n; 1: doubling hi while f < 0; 2: halving lo while
  // f > 0; 3: Newton), taking the same steps in the same order as the two bracket loops and
  // the Newton loop it replaces, so the kernel holds one copy of the evaluation.
  double Tq = Tn, lo = Tn, hi = Tn, x = Tn;
  int mode = 0;
  bool done = false;
  kT_eval e;
  for (int nev = 1;; ++nev) {
    const kT_eval r = evaluate(x);
    if (mode == 0) {
      e = r;
      mode = r.f < 0.0 ? 1 : r.f > 0.0 ? 2 : 3;
    } else if (mode == 1) {
      if (!(r.f < 0.0)) mode = 3;
    } else if (mode == 2) {
      if (!(r.f > 0.0)) mode = 3;
    } else {
      Tq = x;
      e = r;
      if (done) break;
    }
    if (nev >= 200) break;
    if (mode == 1) {
      lo = hi;
      hi *= 2.0;
      x = hi;
      continue;
    }
    if (mode == 2) {
      hi = lo;
      lo *= 0.5;
      x = lo;
      continue;
    }
    if (e.f == 0.0) break;
    if (e.f < 0.0) lo = Tq;
    else hi = Tq;
    double Tx = Tq - e.f * rt_rcp(e.fp);
    // a step within the tolerance has converged and is taken as it is; a larger one that
    // leaves the bracket is replaced by bisection
    done = fabs(Tx - Tq) <= 1e-14 * Tq;
    if (!done && !(Tx > lo && Tx < hi)) Tx = 0.5 * (lo + hi);
    x = Tx;
  }

  // The directions and weights are needed before the iteration and after it, not in it: read
  // them again here (through a pointer the compiler cannot prove unchanged, so it does not keep
  // the first copy live through the iteration) instead of holding them in registers.
  const double *dirs_again = a.dirs, *W_again = a.W;
  asm volatile("" : "+s"(dirs_again), "+s"(W_again));
  ang.load(dirs_again, W_again, K, l);
  const double T4 = Tq * Tq * Tq * Tq;
  const double planck = a.a_rad * T4 * (1.0 / fourpi);
  const double Jc = (e.SI + y * e.kP * e.SG * planck) * rt_rcp(e.D);
  const double chi = e.kJ + ks;
  double dE = 0, dFx = 0, dFy = 0, dFz = 0;
#pragma unroll
  for (int q = 0; q < APL; ++q) {
    const double Inew = (Ic[q] + y * Gm[q] * (e.kP * planck + ks * Jc)) * rt_rcp(1.0 + y * chi * Gm[q]);
    const double iG = rt_rcp(Gm[q]);
    const double iG2 = iG * iG;
    const T out = (T)(Inew * (iG2 * iG2));
    // the incoming value is read again here rather than held through the iteration
    const double wd = ang.wt(q) * ((double)Ir[ang.k[q]] - (double)out);
    if (ang.ok[q]) Ir[ang.k[q]] = out;
    dE += wd;
    dFx += wd * ang.dx(q);
    dFy += wd * ang.dy(q);
    dFz += wd * ang.dz(q);
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
    if (a.T_out) a.T_out[cell] = Tq;
  }
}

template <typename T, int LPC, int APL, bool FULL, int PAIRED>
hipError_t launch(const rt_kT_args &a, hipStream_t s) {
  const int64_t cpb = RT_BLOCK / LPC;
  const int64_t nblk = (a.N + cpb - 1) / cpb;
  hipLaunchKernelGGL((k_source_kT<T, LPC, APL, FULL, PAIRED>), dim3((unsigned)rt_grid_for(nblk)), dim3(RT_BLOCK),
                     0, s, a, nblk);
  return hipGetLastError();
}

template <typename T, int PAIRED> hipError_t dispatch_paired(const rt_kT_args &a, hipStream_t s) {
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

// Antipodal sets with a paired layout put 4 or 8 lanes on a cell (more cells per wave, so the
// per-cell scalar work of each evaluation is shared by fewer lanes); others the general one.
template <typename T> hipError_t dispatch(const rt_kT_args &a, hipStream_t s) {
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

hipError_t rt_launch_source_kT(const rt_kT_args &a, int dtype, hipStream_t s) {
  return dtype == RT_F32 ? dispatch<float>(a, s) : dispatch<double>(a, s);
}

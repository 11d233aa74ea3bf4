// The radiation step kernel: transport (section 2.2) and the implicit source
// update (section 2.3) of one cell per group of LPC lanes, each lane holding
// APL angles k = l + LPC q.  One pass reads the cell's intensity row, gathers the
// neighbour rows of its faces through the half-face index (no atomics), updates
// the charges, runs the source on the transported row while it is in registers,
// and writes the row once.
#include "rt_device.h"

namespace {

template <typename T, int LPC, int APL>
__global__ __launch_bounds__(RT_BLOCK) void k_step(rt_step_args a, int64_t nblk) {
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

  const T *Iin = (const T *)a.I_in;
  const int64_t row = cell * (int64_t)K;
  T Ic[APL];
#pragma unroll
  for (int q = 0; q < APL; ++q) Ic[q] = ang.ok[q] ? Iin[row + ang.k[q]] : T(0);

  double Vnew = 0.0;
  if (a.do_transport) {
    // ---- transport: charges V I minus the upwind charge through every face -------------
    const double Vn = a.vol_in[cell];
    Vnew = Vn + a.dt * a.D[cell];
    T acc[APL];
#pragma unroll
    for (int q = 0; q < APL; ++q) acc[q] = (T)Vn * Ic[q];
    const T sc = (T)(a.dt * a.c_red), sd = (T)a.dt;
    const V4 *an = (const V4 *)a.hf_an;
    const int h0 = a.row_ptr[cell], h1 = a.row_ptr[cell + 1];
    if (a.do_transport == 1) {
      for (int h = h0; h < h1; ++h) {
        const int64_t j = a.hf_nbr[h];
        const V4 r = an[h];
        // g = dt (cbar (A n_out).n_k - A (w~.n)_out): charge leaving through the face per unit I_up
        const T ax = sc * r.x, ay = sc * r.y, az = sc * r.z, b = sd * r.w;
        const T *Ij = Iin + j * K;
#pragma unroll
        for (int q = 0; q < APL; ++q) {
          const T g = ax * ang.dx[q] + ay * ang.dy[q] + az * ang.dz[q] - b;
          const T vj = ang.ok[q] ? Ij[ang.k[q]] : T(0);
          acc[q] -= g * (g > T(0) ? Ic[q] : vj);
        }
      }
    } else {
      // reconstructed face states of the half-step intensities (PLM stage 2)
      const T *Ih = (const T *)a.I_half;
      const T *G = (const T *)a.grad;
      const V4 *rel = (const V4 *)a.hf_rel;
      T hs[APL], gsx[APL], gsy[APL], gsz[APL];
#pragma unroll
      for (int q = 0; q < APL; ++q) {
        const int k = ang.k[q];
        hs[q] = Ih[row + k];
        gsx[q] = G[(cell * 3 + 0) * K + k];
        gsy[q] = G[(cell * 3 + 1) * K + k];
        gsz[q] = G[(cell * 3 + 2) * K + k];
      }
      for (int h = h0; h < h1; ++h) {
        const int64_t j = a.hf_nbr[h];
        const V4 r = an[h];
        const V4 r0 = rel[2 * h], r1 = rel[2 * h + 1];
        const T ax = sc * r.x, ay = sc * r.y, az = sc * r.z, b = sd * r.w;
        const T *Hj = Ih + j * K;
        const T *Gj = G + j * 3 * K;
#pragma unroll
        for (int q = 0; q < APL; ++q) {
          const int k = ang.k[q];
          const T g = ax * ang.dx[q] + ay * ang.dy[q] + az * ang.dz[q] - b;
          const T fs = hs[q] + gsx[q] * r0.x + gsy[q] * r0.y + gsz[q] * r0.z;
          const T fn = Hj[k] + Gj[k] * r0.w + Gj[K + k] * r1.x + Gj[2 * K + k] * r1.y;
          acc[q] -= g * (g > T(0) ? fs : fn);
        }
      }
    }
    const T inv = (T)(1.0 / Vnew);
#pragma unroll
    for (int q = 0; q < APL; ++q) Ic[q] = acc[q] * inv;
  }

  if (a.do_source) {
    // ---- implicit source (section 2.3): 1. lab moments; 2. comoving sums and T ----------
    const double rho = a.rho[cell];
    const double m0 = a.mom[3 * cell], m1 = a.mom[3 * cell + 1], m2 = a.mom[3 * cell + 2];
    const double Eg = a.etot[cell];
    const double kP = a.kP[cell], kJ = a.kJ[cell], ks = a.ks[cell];
    const double c = a.c_light;
    const double vx = m0 / rho, vy = m1 / rho, vz = m2 / rho;
    const double gam = 1.0 / sqrt(1.0 - (vx * vx + vy * vy + vz * vz) / (c * c));
    const double y = a.dt * a.c_red * rho;
    const double chi = kJ + ks;
    const T tg = (T)gam, tvx = (T)(vx / c), tvy = (T)(vy / c), tvz = (T)(vz / c), tyc = (T)(y * chi);
    double sE = 0, sFx = 0, sFy = 0, sFz = 0, sQ = 0, s1 = 0, sG = 0, sI = 0;
    T Gm[APL], Ico[APL], rr[APL];
#pragma unroll
    for (int q = 0; q < APL; ++q) {
      const double Id = (double)Ic[q];
      const double wq = ang.w[q];
      sE += wq * Id;
      sFx += wq * (double)ang.dx[q] * Id;
      sFy += wq * (double)ang.dy[q] * Id;
      sFz += wq * (double)ang.dz[q] * Id;
      const T G = tg * (T(1) - (tvx * ang.dx[q] + tvy * ang.dy[q] + tvz * ang.dz[q]));
      const T G2 = G * G;
      Gm[q] = G;
      Ico[q] = G2 * G2 * Ic[q];
      rr[q] = T(1) / (T(1) + tyc * G);
      const double qk = wq / (double)G2;
      sQ += qk;
      s1 += qk * (double)rr[q];
      sG += qk * (double)(G * rr[q]);
      sI += qk * (double)(Ico[q] * rr[q]);
    }
    sE = rt_group_sum<LPC>(sE);
    sFx = rt_group_sum<LPC>(sFx);
    sFy = rt_group_sum<LPC>(sFy);
    sFz = rt_group_sum<LPC>(sFz);
    sQ = rt_group_sum<LPC>(sQ);
    s1 = rt_group_sum<LPC>(s1);
    sG = rt_group_sum<LPC>(sG);
    sI = rt_group_sum<LPC>(sI);
    const double S1 = s1 / sQ, SG = sG / sQ, SI = sI / sQ;
    const double Dd = S1 + y * kJ * SG;
    const double Tn = (Eg - 0.5 * (m0 * m0 + m1 * m1 + m2 * m2) / rho) / (rho * a.cv);
    const double fourpi = 4.0 * RT_PI;
    const double Aq = a.dt * c * rho * kP * a.a_rad * S1 / Dd;
    const double Bq = rho * a.cv;
    const double Cq = rho * a.cv * Tn + a.dt * c * rho * fourpi * kJ * SI / Dd;
    const double Tnew = rt_quartic_root(Aq, Bq, Cq);
    const double T4 = Tnew * Tnew * Tnew * Tnew;
    const double planck = a.a_rad * T4 / fourpi;
    const double Jc = (SI + y * kP * SG * planck) / Dd;
    const T ySrc = (T)(y * (kP * planck + ks * Jc));
    // ---- 3. per-angle implicit update, boost back; 4. moments of the stored values ------
    double tE = 0, tFx = 0, tFy = 0, tFz = 0;
#pragma unroll
    for (int q = 0; q < APL; ++q) {
      const T G2 = Gm[q] * Gm[q];
      const T out = ang.ok[q] ? (Ico[q] + Gm[q] * ySrc) * rr[q] / (G2 * G2) : T(0);
      Ic[q] = out;
      const double od = (double)out;
      const double wq = ang.w[q];
      tE += wq * od;
      tFx += wq * (double)ang.dx[q] * od;
      tFy += wq * (double)ang.dy[q] * od;
      tFz += wq * (double)ang.dz[q] * od;
    }
    tE = rt_group_sum<LPC>(tE);
    tFx = rt_group_sum<LPC>(tFx);
    tFy = rt_group_sum<LPC>(tFy);
    tFz = rt_group_sum<LPC>(tFz);
    if (l == 0) {
      if (a.write_gas) {
        a.etot[cell] = Eg + (c / a.c_red) * fourpi * (sE - tE);
        const double f = fourpi / a.c_red;
        a.mom[3 * cell] = m0 + f * (sFx - tFx);
        a.mom[3 * cell + 1] = m1 + f * (sFy - tFy);
        a.mom[3 * cell + 2] = m2 + f * (sFz - tFz);
      }
      if (a.T_out) a.T_out[cell] = Tnew;
    }
  }

  T *Iout = (T *)a.I_out;
#pragma unroll
  for (int q = 0; q < APL; ++q)
    if (ang.ok[q]) Iout[row + ang.k[q]] = Ic[q];
  if (a.do_transport && l == 0 && a.vol_out) a.vol_out[cell] = Vnew;
}

template <typename T, int LPC, int APL> hipError_t launch(const rt_step_args &a, hipStream_t s) {
  const int64_t cpb = RT_BLOCK / LPC;
  const int64_t nblk = (a.N + cpb - 1) / cpb;
  hipLaunchKernelGGL((k_step<T, LPC, APL>), dim3((unsigned)rt_grid_for(nblk)), dim3(RT_BLOCK), 0, s, a, nblk);
  return hipGetLastError();
}

template <typename T> hipError_t dispatch(const rt_step_args &a, hipStream_t s) {
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

hipError_t rt_launch_step(const rt_step_args &a, int dtype, hipStream_t s) {
  return dtype == RT_F32 ? dispatch<float>(a, s) : dispatch<double>(a, s);
}

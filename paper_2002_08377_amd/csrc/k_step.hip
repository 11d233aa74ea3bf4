// The radiation step kernel: transport (section 2.2) and the implicit source
// update (section 2.3) of one cell per group of LPC lanes, each lane holding APL
// angles.  One pass reads the cell's intensity row, gathers the neighbour rows of
// its faces through the half-face index (no atomics), updates the charges, runs the
// source on the transported row while it is in registers, and writes the row once.
#include "rt_device.h"

namespace {

// Faces gathered per batch: all their neighbour-row loads are issued before any is
// used, so one memory round trip serves U faces.
template <typename T> struct rt_batch { static constexpr int U = 4; };
template <> struct rt_batch<double> { static constexpr int U = 2; };

// Angles held by one lane.
//  General layout: k_q = l + LPC q for q < APL; past K (only when !FULL) the slot
//    aliases angle 0 with weight 0 and is never stored.
//  Paired layout (angle k + K/2 is the antipode of angle k and has its weight; needs
//    K = LPC APL): the lane holds P = APL/2 angles k_q = l + LPC q and their
//    antipodes k_q + K/2 in slots q + P, so one stored direction serves both and
//    one dot product per face serves both fluxes.
template <typename T, int LPC, int APL, bool FULL, bool PAIRED> struct rt_step_angles {
  static constexpr int P = PAIRED ? APL / 2 : APL;
  T x[P], y[P], z[P];
  double w[P];
  int k[APL];
  bool ok[APL];
  __device__ __forceinline__ void load(const double *dirs, const double *W, int K, int l) {
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const int kk = l + LPC * q;
      ok[q] = FULL || PAIRED || kk < K;
      k[q] = ok[q] ? kk : 0;
      x[q] = (T)dirs[3 * k[q]];
      y[q] = (T)dirs[3 * k[q] + 1];
      z[q] = (T)dirs[3 * k[q] + 2];
      w[q] = ok[q] ? W[k[q]] : 0.0;
      if (PAIRED) {
        k[q + P] = k[q] + K / 2;
        ok[q + P] = true;
      }
    }
  }
  // direction and weight of slot q (q is a compile-time constant after unrolling)
  __device__ __forceinline__ T dx(int q) const { return PAIRED && q >= P ? -x[q - P] : x[q]; }
  __device__ __forceinline__ T dy(int q) const { return PAIRED && q >= P ? -y[q - P] : y[q]; }
  __device__ __forceinline__ T dz(int q) const { return PAIRED && q >= P ? -z[q - P] : z[q]; }
  __device__ __forceinline__ double wt(int q) const { return PAIRED && q >= P ? w[q - P] : w[q]; }
};

// MODE 0: source only (in place); 1: upwind transport (+ source); 2: reconstructed
// transport of PLM stage 2 (+ source).  Separate instantiations keep each one's
// registers to what its own loop needs.
//
// The cells of a workgroup are consecutive, so their half-faces form one contiguous
// range; it is staged in LDS (dynamic size: the largest range of any workgroup,
// found at upload) and the face loops read their records from there.
template <typename T, int LPC, int APL, int MODE, bool FULL, bool PAIRED>
__global__ __launch_bounds__(RT_BLOCK) void k_step(rt_step_args a, int64_t nblk) {
  using V4 = typename rt_vec4<T>::type;
  using Ang = rt_step_angles<T, LPC, APL, FULL, PAIRED>;
  constexpr int P = Ang::P;
  constexpr int U = rt_batch<T>::U;
  constexpr int CPB = RT_BLOCK / LPC;
  extern __shared__ __align__(16) unsigned char rt_smem[];
  V4 *s_an = (V4 *)rt_smem;
  V4 *s_rel = s_an + a.hf_cap;
  int32_t *s_nbr = (int32_t *)(s_an + (MODE == 2 ? 3 : 1) * a.hf_cap);
  const int64_t lb = rt_logical_block(nblk);
  if (lb < 0) return;  // whole padding workgroup
  const int64_t c0 = lb * CPB;
  const int64_t cell = c0 + threadIdx.x / LPC;
  const bool live = cell < a.N;
  const int l = threadIdx.x % LPC;
  const int K = a.K;
  int H0 = 0;
  if (MODE != 0) {
    const V4 *an = (const V4 *)a.hf_an;
    const V4 *rel = (const V4 *)a.hf_rel;
    const int64_t c1 = c0 + CPB < a.N ? c0 + CPB : a.N;
    H0 = a.row_ptr[c0];
    const int nH = a.row_ptr[c1] - H0;  // <= hf_cap by construction
    for (int i = threadIdx.x; i < nH; i += RT_BLOCK) {
      s_nbr[i] = a.hf_nbr[H0 + i];
      s_an[i] = an[H0 + i];
      if (MODE == 2) {
        s_rel[2 * i] = rel[2 * (H0 + i)];
        s_rel[2 * i + 1] = rel[2 * (H0 + i) + 1];
      }
    }
    __syncthreads();
  }
  if (!live) return;
  Ang ang;
  ang.load(a.dirs, a.W, K, l);

  const T *Iin = (const T *)a.I_in;
  const int64_t row = cell * (int64_t)K;
  T Ic[APL];
#pragma unroll
  for (int q = 0; q < APL; ++q) Ic[q] = Iin[row + ang.k[q]];

  double Vnew = 0.0;
  if (MODE != 0) {
    // ---- transport: charges V I minus the upwind charge through every face -------------
    const double Vn = a.vol_in[cell];
    Vnew = Vn + a.dt * a.D[cell];
    T acc[APL];
#pragma unroll
    for (int q = 0; q < APL; ++q) acc[q] = (T)Vn * Ic[q];
    const T sc = (T)(a.dt * a.c_red), sd = (T)a.dt;
    const int h0 = a.row_ptr[cell], h1 = a.row_ptr[cell + 1];
    if (MODE == 1) {
      for (int h = h0; h < h1; h += U) {
        // batch metadata; slots past the cell's last face reuse face h0 with a zero record
        int64_t j[U];
        V4 r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const bool v = h + u < h1;
          const int i = (v ? h + u : h0) - H0;
          j[u] = s_nbr[i];
          r[u] = s_an[i];
          if (!v) r[u] = V4{T(0), T(0), T(0), T(0)};
        }
        T xn[U][APL];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int q = 0; q < APL; ++q) xn[u][q] = Iin[j[u] * K + ang.k[q]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          // g = dt (cbar (A n_out).n_k - A (w~.n)_out): charge leaving per unit upwind intensity
          const T ax = sc * r[u].x, ay = sc * r[u].y, az = sc * r[u].z, b = sd * r[u].w;
#pragma unroll
          for (int q = 0; q < P; ++q) {
            const T dot = ax * ang.x[q] + ay * ang.y[q] + az * ang.z[q];
            const T g = dot - b;
            acc[q] -= g * (g > T(0) ? Ic[q] : xn[u][q]);
            if (PAIRED) {
              const T g2 = -dot - b;  // the antipodal angle
              acc[q + P] -= g2 * (g2 > T(0) ? Ic[q + P] : xn[u][q + P]);
            }
          }
        }
      }
    } else {
      // reconstructed face states of the half-step intensities (PLM stage 2)
      const T *Ih = (const T *)a.I_half;
      const T *G = (const T *)a.grad;
      T hs[APL], gsx[APL], gsy[APL], gsz[APL];
#pragma unroll
      for (int q = 0; q < APL; ++q) {
        const int k = ang.k[q];
        hs[q] = Ih[row + k];
        gsx[q] = G[(cell * 3 + 0) * K + k];
        gsy[q] = G[(cell * 3 + 1) * K + k];
        gsz[q] = G[(cell * 3 + 2) * K + k];
      }
      constexpr int UP = sizeof(T) == 4 ? 2 : 1;
      for (int h = h0; h < h1; h += UP) {
        int64_t j[UP];
        V4 r[UP], r0[UP], r1[UP];
#pragma unroll
        for (int u = 0; u < UP; ++u) {
          const bool v = h + u < h1;
          const int i = (v ? h + u : h0) - H0;
          j[u] = s_nbr[i];
          r[u] = s_an[i];
          r0[u] = s_rel[2 * i];
          r1[u] = s_rel[2 * i + 1];
          if (!v) r[u] = V4{T(0), T(0), T(0), T(0)};
        }
        T xh[UP][APL], xg0[UP][APL], xg1[UP][APL], xg2[UP][APL];
#pragma unroll
        for (int u = 0; u < UP; ++u) {
          const T *Hj = Ih + j[u] * K;
          const T *Gj = G + j[u] * 3 * K;
#pragma unroll
          for (int q = 0; q < APL; ++q) {
            const int k = ang.k[q];
            xh[u][q] = Hj[k];
            xg0[u][q] = Gj[k];
            xg1[u][q] = Gj[K + k];
            xg2[u][q] = Gj[2 * K + k];
          }
        }
#pragma unroll
        for (int u = 0; u < UP; ++u) {
          const T ax = sc * r[u].x, ay = sc * r[u].y, az = sc * r[u].z, b = sd * r[u].w;
#pragma unroll
          for (int q = 0; q < APL; ++q) {
            const T g = ax * ang.dx(q) + ay * ang.dy(q) + az * ang.dz(q) - b;
            const T fs = hs[q] + gsx[q] * r0[u].x + gsy[q] * r0[u].y + gsz[q] * r0[u].z;
            const T fn = xh[u][q] + xg0[u][q] * r0[u].w + xg1[u][q] * r1[u].x + xg2[u][q] * r1[u].y;
            acc[q] -= g * (g > T(0) ? fs : fn);
          }
        }
      }
    }
    const T inv = (T)rt_rcp(Vnew);
#pragma unroll
    for (int q = 0; q < APL; ++q) Ic[q] = acc[q] * inv;
  }

  if (a.do_source) {
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
    double sQ = 0, s1 = 0, sG = 0, sI = 0;
    // Per angle, with r = 1/(1 + y chi Gamma): the update of eq. 28 boosted back is
    // I' = (Gamma^4 I + y Gamma S) r / Gamma^4 = I r + (r / Gamma^3) y S, so pass 2 keeps
    // only I r and r / Gamma^3 (and the incoming I for the bookkeeping of step 4).
    T I0[APL], Br[APL];
    auto pass1 = [&](int q, T G) {
      I0[q] = Ic[q];
      const T iG = rt_rcp(G);
      const T iG2 = iG * iG;
      const T G2 = G * G;
      const T r = rt_rcp(T(1) + tyc * G);
      const double qk = ang.wt(q) * (double)iG2;
      sQ += qk;
      s1 += qk * (double)r;
      sG += qk * (double)(G * r);
      sI += qk * (double)(G2 * G2 * Ic[q] * r);
      Ic[q] *= r;
      Br[q] = r * iG2 * iG;
    };
#pragma unroll
    for (int q = 0; q < P; ++q) {
      // Gamma = gamma (1 - v.n/c); the antipode has gamma (1 + v.n/c)
      const T vn = tvx * ang.x[q] + tvy * ang.y[q] + tvz * ang.z[q];
      pass1(q, tg * (T(1) - vn));
      if (PAIRED) pass1(q + P, tg * (T(1) + vn));
    }
    sQ = rt_group_sum<LPC>(sQ);
    s1 = rt_group_sum<LPC>(s1);
    sG = rt_group_sum<LPC>(sG);
    sI = rt_group_sum<LPC>(sI);
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
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const T out = Ic[q] + Br[q] * ySrc;
      Ic[q] = out;
      double wd = ang.w[q] * ((double)I0[q] - (double)out);
      dE += wd;
      if (PAIRED) {
        const T out2 = Ic[q + P] + Br[q + P] * ySrc;
        Ic[q + P] = out2;
        const double wd2 = ang.w[q] * ((double)I0[q + P] - (double)out2);
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
    }
  }

  T *Iout = (T *)a.I_out;
#pragma unroll
  for (int q = 0; q < APL; ++q)
    if (ang.ok[q]) Iout[row + ang.k[q]] = Ic[q];
  if (MODE != 0 && l == 0 && a.vol_out) a.vol_out[cell] = Vnew;
}

// Staging needs (records per half-face) x (half-faces of the largest range of the
// workgroup's cells) bytes of LDS; a layout that would need more than 64 KiB is
// refused with hipErrorInvalidConfiguration (the dispatch then tries another).
template <typename T, int LPC, int APL, bool FULL, bool PAIRED>
hipError_t launch_mode(const rt_step_args &args, hipStream_t s) {
  using V4 = typename rt_vec4<T>::type;
  rt_step_args a = args;
  a.hf_cap = LPC == 16 ? a.hf_cap16 : LPC == 8 ? a.hf_cap32 : a.hf_cap64;
  const int64_t cpb = RT_BLOCK / LPC;
  const int64_t nblk = (a.N + cpb - 1) / cpb;
  const dim3 grid((unsigned)rt_grid_for(nblk)), block(RT_BLOCK);
  const size_t per = (a.do_transport == 2 ? 3 : 1) * sizeof(V4) + sizeof(int32_t);
  const size_t smem = a.do_transport ? per * (size_t)a.hf_cap : 0;
  if (smem > 65536) return hipErrorInvalidConfiguration;
  switch (a.do_transport) {
    case 0: hipLaunchKernelGGL((k_step<T, LPC, APL, 0, FULL, PAIRED>), grid, block, smem, s, a, nblk); break;
    case 1: hipLaunchKernelGGL((k_step<T, LPC, APL, 1, FULL, PAIRED>), grid, block, smem, s, a, nblk); break;
    case 2: hipLaunchKernelGGL((k_step<T, LPC, APL, 2, FULL, PAIRED>), grid, block, smem, s, a, nblk); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int LPC, int APL> hipError_t launch(const rt_step_args &a, hipStream_t s) {
  return a.K == LPC * APL ? launch_mode<T, LPC, APL, true, false>(a, s)
                          : launch_mode<T, LPC, APL, false, false>(a, s);
}

template <typename T> hipError_t dispatch_paired(const rt_step_args &a, hipStream_t s) {
  switch (rt_step_lanes(a.K, 1)) {
    case 0x0802: return launch_mode<T, 8, 2, true, true>(a, s);
    case 0x0804: return launch_mode<T, 8, 4, true, true>(a, s);
    case 0x0806: return launch_mode<T, 8, 6, true, true>(a, s);
    case 0x0808: return launch_mode<T, 8, 8, true, true>(a, s);
    case 0x080a: return launch_mode<T, 8, 10, true, true>(a, s);
    case 0x080c: return launch_mode<T, 8, 12, true, true>(a, s);
    case 0x0402: return launch_mode<T, 4, 2, true, true>(a, s);
    case 0x0406: return launch_mode<T, 4, 6, true, true>(a, s);
    case 0x040a: return launch_mode<T, 4, 10, true, true>(a, s);
  }
  return hipErrorInvalidConfiguration;
}

template <typename T> hipError_t dispatch_general(const rt_step_args &a, hipStream_t s) {
  switch (rt_step_lanes(a.K, 0)) {
    case 0x1001: return launch<T, 16, 1>(a, s);
    case 0x1002: return launch<T, 16, 2>(a, s);
    case 0x1003: return launch<T, 16, 3>(a, s);
    case 0x1004: return launch<T, 16, 4>(a, s);
    case 0x1005: return launch<T, 16, 5>(a, s);
    case 0x1006: return launch<T, 16, 6>(a, s);
    case 0x1007: return launch<T, 16, 7>(a, s);
    case 0x1008: return launch<T, 16, 8>(a, s);
    case 0x0801: return launch<T, 8, 1>(a, s);
    case 0x0802: return launch<T, 8, 2>(a, s);
    case 0x0803: return launch<T, 8, 3>(a, s);
    case 0x0804: return launch<T, 8, 4>(a, s);
    case 0x0805: return launch<T, 8, 5>(a, s);
    case 0x0806: return launch<T, 8, 6>(a, s);
    case 0x0807: return launch<T, 8, 7>(a, s);
    case 0x0808: return launch<T, 8, 8>(a, s);
  }
  return hipErrorInvalidValue;
}

// Antipodal sets take the paired kernel when it has a lane layout for K and its staging
// fits in LDS; everything else (and that fallback) the general kernel.
template <typename T> hipError_t dispatch(const rt_step_args &a, hipStream_t s) {
  if (a.paired) {
    const hipError_t e = dispatch_paired<T>(a, s);
    if (e != hipErrorInvalidConfiguration) return e;
  }
  return dispatch_general<T>(a, s);
}

}  // namespace

hipError_t rt_launch_step(const rt_step_args &a, int dtype, hipStream_t s) {
  return dtype == RT_F32 ? dispatch<float>(a, s) : dispatch<double>(a, s);
}

// Boundary and emitter cells (sections 2.4 and 2.5), applied after a step: one group
// of LPC lanes per marked cell, each lane holding APL angles.
//  Boundary: I_k <- I_k - (I_k - I0_k) f with f = min(dt/tau, 1) and I0_k = S in the
//    cell's directions of interest (n_k . dir >= cos_open), 0 elsewhere; rho v <- rho v
//    (1 - f), the kinetic energy that goes with it leaving the total gas energy.
//  Emitter: in the directions of interest, the comoving emission-absorption term at
//    T_eff integrated implicitly: I~' = (I~ + x S)/(1 + x), I~ = Gamma^4 I,
//    x = dt Gamma cbar rho kP, Gamma = gamma (1 - v.n/c); the gas is unchanged.
// S = a T_eff^4 / 4 pi.  The marked cells are distinct (checked at upload), so no two
// groups touch the same cell.
#include "rt_device.h"

namespace {

template <typename T, int LPC, int APL>
__global__ __launch_bounds__(RT_BLOCK) void k_marked(rt_marked_args a, int64_t nblk) {
  const int64_t lb = rt_logical_block(nblk);
  if (lb < 0) return;
  constexpr int CPB = RT_BLOCK / LPC;
  const int64_t m = lb * CPB + threadIdx.x / LPC;
  if (m >= a.n) return;
  const int l = threadIdx.x % LPC;
  const int K = a.K;
  rt_lane_angles<double, LPC, APL> ang;
  ang.load(a.dirs, a.W, K, l);
  const int64_t i = a.cell[m];
  const int kind = a.kind[m];
  const double Te2 = a.T_eff[m] * a.T_eff[m];
  const double S = a.a_rad * Te2 * Te2 / (4.0 * RT_PI);
  const double d0 = a.dir[3 * m], d1 = a.dir[3 * m + 1], d2 = a.dir[3 * m + 2];
  const double co = a.cos_open[m];
  T *Ii = (T *)a.I + i * (int64_t)K;
  if (kind == RT_CELL_BOUNDARY) {
#pragma unroll
    for (int q = 0; q < APL; ++q) {
      if (!ang.ok[q]) continue;
      const double nd = ang.dx[q] * d0 + ang.dy[q] * d1 + ang.dz[q] * d2;
      const double I0 = nd >= co ? S : 0.0;
      const double x = (double)Ii[ang.k[q]];
      Ii[ang.k[q]] = (T)(x - (x - I0) * a.f);
    }
    if (l == 0) {
      double *p = a.mom + 3 * i;
      const double rho = a.rho[i];
      const double p0 = p[0], p1 = p[1], p2 = p[2];
      const double ke0 = 0.5 * (p0 * p0 + p1 * p1 + p2 * p2) / rho;
      const double q0 = p0 * (1.0 - a.f), q1 = p1 * (1.0 - a.f), q2 = p2 * (1.0 - a.f);
      const double ke1 = 0.5 * (q0 * q0 + q1 * q1 + q2 * q2) / rho;
      p[0] = q0;
      p[1] = q1;
      p[2] = q2;
      a.etot[i] -= ke0 - ke1;
    }
  } else if (kind == RT_CELL_EMITTER) {
    const double rho = a.rho[i];
    const double vx = a.mom[3 * i] / rho, vy = a.mom[3 * i + 1] / rho, vz = a.mom[3 * i + 2] / rho;
    const double c = a.c_light;
    const double gam = 1.0 / sqrt(1.0 - (vx * vx + vy * vy + vz * vz) / (c * c));
    const double xr = a.dt * a.c_red * rho * a.kP[i];
#pragma unroll
    for (int q = 0; q < APL; ++q) {
      if (!ang.ok[q]) continue;
      const double nd = ang.dx[q] * d0 + ang.dy[q] * d1 + ang.dz[q] * d2;
      if (!(nd >= co)) continue;
      const double vn = vx * ang.dx[q] + vy * ang.dy[q] + vz * ang.dz[q];
      const double G = gam * (1.0 - vn / c);
      const double G2 = G * G, G4 = G2 * G2;
      const double x = xr * G;
      const double Icom = (G4 * (double)Ii[ang.k[q]] + x * S) / (1.0 + x);
      Ii[ang.k[q]] = (T)(Icom / G4);
    }
  }
}

template <typename T, int LPC, int APL> hipError_t launch(const rt_marked_args &a, hipStream_t s) {
  const int64_t cpb = RT_BLOCK / LPC;
  const int64_t nblk = (a.n + cpb - 1) / cpb;
  hipLaunchKernelGGL((k_marked<T, LPC, APL>), dim3((unsigned)rt_grid_for(nblk)), dim3(RT_BLOCK), 0, s, a, nblk);
  return hipGetLastError();
}

template <typename T> hipError_t dispatch(const rt_marked_args &a, hipStream_t s) {
  switch ((a.K + 15) / 16) {
    case 1: return launch<T, 16, 1>(a, s);
    case 2: return launch<T, 16, 2>(a, s);
    case 3: return launch<T, 16, 3>(a, s);
    case 4: return launch<T, 16, 4>(a, s);
    case 5: return launch<T, 16, 5>(a, s);
    case 6: return launch<T, 16, 6>(a, s);
    case 7: return launch<T, 16, 7>(a, s);
    case 8: return launch<T, 16, 8>(a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t rt_launch_marked(const rt_marked_args &a, int dtype, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  return dtype == RT_F32 ? dispatch<float>(a, s) : dispatch<double>(a, s);
}

// Limited linear reconstruction of every angle (section 2.2 item ii): the S10
// Voronoi gradient estimator
//   V_i grad phi_i = sum_faces [ (phi_j - phi_i) A c/d + (phi_i + phi_j) A n_out / 2 ]
// (c = face centroid minus the generators' midpoint, d = generator distance),
// then the Barth-Jespersen factor alpha = min(1, (max - phi)/max_f delta_f,
// (min - phi)/min_f delta_f) over the extrapolations delta_f = grad.(r~_f - s_i),
// with max/min over the cell and its face neighbours.  Taking the largest and
// smallest delta is exact: IEEE division is monotone in the divisor.
#include "rt_device.h"

namespace {

template <typename T, int LPC, int APL>
__global__ __launch_bounds__(RT_BLOCK) void k_gradient(int64_t N, int K, const int32_t *__restrict__ row_ptr,
                                                       const int32_t *__restrict__ hf_nbr, const void *hf_gp,
                                                       const void *hf_rel, const double *__restrict__ vol0,
                                                       const T *__restrict__ I, T *__restrict__ G, int64_t nblk) {
  using V4 = typename rt_vec4<T>::type;
  const int64_t lb = rt_logical_block(nblk);
  if (lb < 0) return;
  constexpr int CPB = RT_BLOCK / LPC;
  const int64_t cell = lb * CPB + threadIdx.x / LPC;
  if (cell >= N) return;
  const int l = threadIdx.x % LPC;
  int kk[APL];
  bool ok[APL];
  T s[APL], gx[APL], gy[APL], gz[APL], lo[APL], hi[APL];
  const int64_t row = cell * (int64_t)K;
#pragma unroll
  for (int q = 0; q < APL; ++q) {
    const int k = l + LPC * q;
    ok[q] = k < K;
    kk[q] = ok[q] ? k : 0;
    s[q] = I[row + kk[q]];
    gx[q] = gy[q] = gz[q] = T(0);
    lo[q] = hi[q] = s[q];
  }
  const V4 *gp = (const V4 *)hf_gp;
  const V4 *rel = (const V4 *)hf_rel;
  const int h0 = row_ptr[cell], h1 = row_ptr[cell + 1];
  for (int h = h0; h < h1; ++h) {
    const int64_t j = hf_nbr[h];
    const V4 p0 = gp[2 * h], p1 = gp[2 * h + 1];
    const T *Ij = I + j * K;
#pragma unroll
    for (int q = 0; q < APL; ++q) {
      const T o = Ij[kk[q]];
      const T d = o - s[q], t = s[q] + o;
      gx[q] += d * p0.x + t * p0.w;
      gy[q] += d * p0.y + t * p1.x;
      gz[q] += d * p0.z + t * p1.y;
      lo[q] = fmin(lo[q], o);
      hi[q] = fmax(hi[q], o);
    }
  }
  const T iv = (T)(1.0 / vol0[cell]);
  T dmax[APL], dmin[APL];
#pragma unroll
  for (int q = 0; q < APL; ++q) {
    gx[q] *= iv;
    gy[q] *= iv;
    gz[q] *= iv;
    dmax[q] = dmin[q] = T(0);
  }
  for (int h = h0; h < h1; ++h) {
    const V4 r0 = rel[2 * h];
#pragma unroll
    for (int q = 0; q < APL; ++q) {
      const T dl = gx[q] * r0.x + gy[q] * r0.y + gz[q] * r0.z;
      dmax[q] = fmax(dmax[q], dl);
      dmin[q] = fmin(dmin[q], dl);
    }
  }
#pragma unroll
  for (int q = 0; q < APL; ++q) {
    if (!ok[q]) continue;
    T al = T(1);
    if (dmax[q] > T(0)) al = fmin(al, (hi[q] - s[q]) / dmax[q]);
    if (dmin[q] < T(0)) al = fmin(al, (lo[q] - s[q]) / dmin[q]);
    const int k = kk[q];
    G[(cell * 3 + 0) * K + k] = al * gx[q];
    G[(cell * 3 + 1) * K + k] = al * gy[q];
    G[(cell * 3 + 2) * K + k] = al * gz[q];
  }
}

template <typename T, int LPC, int APL>
hipError_t launch(const rt_mesh *m, int K, const void *I, void *G, hipStream_t s) {
  const int64_t cpb = RT_BLOCK / LPC;
  const int64_t nblk = (m->N + cpb - 1) / cpb;
  const void *gp = std::is_same<T, double>::value ? (const void *)m->hf_gp64 : (const void *)m->hf_gp32;
  const void *rel = std::is_same<T, double>::value ? (const void *)m->hf_rel64 : (const void *)m->hf_rel32;
  hipLaunchKernelGGL((k_gradient<T, LPC, APL>), dim3((unsigned)rt_grid_for(nblk)), dim3(RT_BLOCK), 0, s, m->N, K,
                     m->row_ptr, m->hf_nbr, gp, rel, m->vol0, (const T *)I, (T *)G, nblk);
  return hipGetLastError();
}

template <typename T> hipError_t dispatch(const rt_mesh *m, int K, const void *I, void *G, hipStream_t s) {
  if (K % 16 == 0 || K > 64) {
    switch ((K + 15) / 16) {
      case 1: return launch<T, 16, 1>(m, K, I, G, s);
      case 2: return launch<T, 16, 2>(m, K, I, G, s);
      case 3: return launch<T, 16, 3>(m, K, I, G, s);
      case 4: return launch<T, 16, 4>(m, K, I, G, s);
      case 5: return launch<T, 16, 5>(m, K, I, G, s);
      case 6: return launch<T, 16, 6>(m, K, I, G, s);
      case 7: return launch<T, 16, 7>(m, K, I, G, s);
      case 8: return launch<T, 16, 8>(m, K, I, G, s);
    }
  } else {
    switch ((K + 7) / 8) {
      case 1: return launch<T, 8, 1>(m, K, I, G, s);
      case 2: return launch<T, 8, 2>(m, K, I, G, s);
      case 3: return launch<T, 8, 3>(m, K, I, G, s);
      case 4: return launch<T, 8, 4>(m, K, I, G, s);
      case 5: return launch<T, 8, 5>(m, K, I, G, s);
      case 6: return launch<T, 8, 6>(m, K, I, G, s);
      case 7: return launch<T, 8, 7>(m, K, I, G, s);
      case 8: return launch<T, 8, 8>(m, K, I, G, s);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t rt_launch_gradient(const rt_mesh *m, int K, const void *I, void *grad, int dtype, hipStream_t s) {
  return dtype == RT_F32 ? dispatch<float>(m, K, I, grad, s) : dispatch<double>(m, K, I, grad, s);
}

// Limited linear reconstruction of every angle (section 2.2 item ii): the S10
// Voronoi gradient estimator
//   V_i grad phi_i = sum_faces [ (phi_j - phi_i) A c/d + (phi_i + phi_j) A n_out / 2 ]
// (c = face centroid minus the generators' midpoint, d = generator distance), gathered as
//   V_i grad phi_i = sum_faces phi_j e_f + phi_i b_i,
//   e_f = A c/d + A n_out / 2,  b_i = sum_faces (A n_out / 2 - A c/d)
// (the same sum regrouped; e_f and b_i are formed once per mesh in FP64), so each face
// costs three multiply-adds per angle instead of eleven operations;
// then the Barth-Jespersen factor alpha = min(1, (max - phi)/max_f delta_f,
// (min - phi)/min_f delta_f) over the extrapolations delta_f = grad.(r~_f - s_i),
// with max/min over the cell and its face neighbours.  Taking the largest and
// smallest delta and dividing once matches taking the minimum of the per-face
// ratios (division is monotone in the divisor; the reciprocal here is refined to
// within an ulp).
#include "rt_device.h"

namespace {

// The workgroup's cells are consecutive, so their half-faces form one contiguous range;
// its records (the neighbour's weight e_f, the extrapolation offset and the neighbour)
// are staged in LDS once and every lane group reads them from there.  Neighbour rows
// are gathered two faces per batch, all loads of a batch issued before any is used.
// Output: the limited gradient as [N][3][K] (PACKED false), or, for the PLM step's own
// stage 2, each cell and angle's (phi, alpha grad phi) as one 4-vector, [N][K][4]
// (PACKED true), so stage 2 gathers a neighbour's face state with one access per angle.
template <typename T, int LPC, int APL, bool PACKED>
__global__ __launch_bounds__(RT_BLOCK) void k_gradient(int64_t N, int K, const int32_t *__restrict__ row_ptr,
                                                       const int32_t *__restrict__ hf_nbr, const void *hf_gp,
                                                       const void *hf_rel, const void *cell_gb,
                                                       const double *__restrict__ vol0,
                                                       const T *__restrict__ I, T *__restrict__ G, int hf_cap,
                                                       int64_t nblk) {
  using V4 = typename rt_vec4<T>::type;
  constexpr int U = 2;
  constexpr int CPB = RT_BLOCK / LPC;
  extern __shared__ __align__(16) unsigned char rt_smem[];
  V4 *s_gp = (V4 *)rt_smem;        // [hf_cap]: e_f
  V4 *s_rel = s_gp + hf_cap;       // [hf_cap]: r~_f - s_i
  int32_t *s_nbr = (int32_t *)(s_rel + hf_cap);
  const int64_t lb = rt_logical_block(nblk);
  if (lb < 0) return;
  const int64_t c0 = lb * CPB;
  const int64_t c1 = c0 + CPB < N ? c0 + CPB : N;
  const int H0 = row_ptr[c0];
  {
    const V4 *gp = (const V4 *)hf_gp;
    const V4 *rel = (const V4 *)hf_rel;
    const int nH = row_ptr[c1] - H0;  // <= hf_cap by construction
    for (int i = threadIdx.x; i < nH; i += RT_BLOCK) {
      s_gp[i] = gp[H0 + i];
      s_rel[i] = rel[2 * (H0 + i)];
      s_nbr[i] = hf_nbr[H0 + i];
    }
  }
  __syncthreads();
  const int64_t cell = c0 + threadIdx.x / LPC;
  if (cell >= N) return;
  const int l = threadIdx.x % LPC;
  int kk[APL];
  bool ok[APL];
  T s[APL], gx[APL], gy[APL], gz[APL], lo[APL], hi[APL];
  const int64_t row = cell * (int64_t)K;
  const V4 b = ((const V4 *)cell_gb)[cell];
#pragma unroll
  for (int q = 0; q < APL; ++q) {
    const int k = l + LPC * q;
    ok[q] = k < K;
    kk[q] = ok[q] ? k : 0;
    s[q] = I[row + kk[q]];
    gx[q] = s[q] * b.x;
    gy[q] = s[q] * b.y;
    gz[q] = s[q] * b.z;
    lo[q] = hi[q] = s[q];
  }
  const int h0 = row_ptr[cell], h1 = row_ptr[cell + 1];
  for (int h = h0; h < h1; h += U) {
    // slots past the cell's last face repeat its first face with zero weights; they
    // leave the sums unchanged and re-read a neighbour already in the min/max
    int64_t j[U];
    V4 e[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool v = h + u < h1;
      const int i = (v ? h + u : h0) - H0;
      j[u] = s_nbr[i];
      e[u] = s_gp[i];
      if (!v) e[u] = V4{T(0), T(0), T(0), T(0)};
    }
    T o[U][APL];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int q = 0; q < APL; ++q) o[u][q] = I[j[u] * K + kk[q]];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int q = 0; q < APL; ++q) {
        gx[q] += o[u][q] * e[u].x;
        gy[q] += o[u][q] * e[u].y;
        gz[q] += o[u][q] * e[u].z;
        lo[q] = fmin(lo[q], o[u][q]);
        hi[q] = fmax(hi[q], o[u][q]);
      }
  }
  const T iv = (T)rt_rcp(vol0[cell]);
  T dmax[APL], dmin[APL];
#pragma unroll
  for (int q = 0; q < APL; ++q) {
    gx[q] *= iv;
    gy[q] *= iv;
    gz[q] *= iv;
    dmax[q] = dmin[q] = T(0);
  }
  for (int h = h0; h < h1; ++h) {
    const V4 r0 = s_rel[h - H0];
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
    if (dmax[q] > T(0)) al = fmin(al, (hi[q] - s[q]) * rt_rcp_refined(dmax[q]));
    if (dmin[q] < T(0)) al = fmin(al, (lo[q] - s[q]) * rt_rcp_refined(dmin[q]));
    const int k = kk[q];
    if constexpr (PACKED) {
      using V4 = typename rt_vec4<T>::type;
      ((V4 *)G)[cell * K + k] = V4{s[q], al * gx[q], al * gy[q], al * gz[q]};
    } else {
      G[(cell * 3 + 0) * K + k] = al * gx[q];
      G[(cell * 3 + 1) * K + k] = al * gy[q];
      G[(cell * 3 + 2) * K + k] = al * gz[q];
    }
  }
}

template <typename T, int LPC, int APL, bool PACKED>
hipError_t launch(const rt_mesh *m, int K, const void *I, void *G, hipStream_t s) {
  using V4 = typename rt_vec4<T>::type;
  const int64_t cpb = RT_BLOCK / LPC;
  const int64_t nblk = (m->N + cpb - 1) / cpb;
  const void *gp = std::is_same<T, double>::value ? (const void *)m->hf_gp64 : (const void *)m->hf_gp32;
  const void *rel = std::is_same<T, double>::value ? (const void *)m->hf_rel64 : (const void *)m->hf_rel32;
  const void *gb = std::is_same<T, double>::value ? (const void *)m->gb64 : (const void *)m->gb32;
  const int cap = cpb == 16 ? m->hf_cap16 : m->hf_cap32;
  const size_t smem = (2 * sizeof(V4) + sizeof(int32_t)) * (size_t)cap;
  if (smem > (size_t)m->lds_max) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_gradient<T, LPC, APL, PACKED>), dim3((unsigned)rt_grid_for(nblk)), dim3(RT_BLOCK), smem, s,
                     m->N, K, m->row_ptr, m->hf_nbr, gp, rel, gb, m->vol0, (const T *)I, (T *)G, cap, nblk);
  return hipGetLastError();
}

template <typename T, bool PACKED>
hipError_t dispatch16(const rt_mesh *m, int K, const void *I, void *G, hipStream_t s) {
  switch ((K + 15) / 16) {
    case 1: return launch<T, 16, 1, PACKED>(m, K, I, G, s);
    case 2: return launch<T, 16, 2, PACKED>(m, K, I, G, s);
    case 3: return launch<T, 16, 3, PACKED>(m, K, I, G, s);
    case 4: return launch<T, 16, 4, PACKED>(m, K, I, G, s);
    case 5: return launch<T, 16, 5, PACKED>(m, K, I, G, s);
    case 6: return launch<T, 16, 6, PACKED>(m, K, I, G, s);
    case 7: return launch<T, 16, 7, PACKED>(m, K, I, G, s);
    case 8: return launch<T, 16, 8, PACKED>(m, K, I, G, s);
  }
  return hipErrorInvalidValue;
}

// Small angle sets take 8 lanes per cell (32-cell workgroups); if their half-face
// records do not fit in LDS, 16 lanes (16-cell workgroups) halve the staging.
template <typename T, bool PACKED>
hipError_t dispatch(const rt_mesh *m, int K, const void *I, void *G, hipStream_t s) {
  if (K % 16 == 0 || K > 64) return dispatch16<T, PACKED>(m, K, I, G, s);
  hipError_t e = hipErrorInvalidValue;
  switch ((K + 7) / 8) {
    case 1: e = launch<T, 8, 1, PACKED>(m, K, I, G, s); break;
    case 2: e = launch<T, 8, 2, PACKED>(m, K, I, G, s); break;
    case 3: e = launch<T, 8, 3, PACKED>(m, K, I, G, s); break;
    case 4: e = launch<T, 8, 4, PACKED>(m, K, I, G, s); break;
    case 5: e = launch<T, 8, 5, PACKED>(m, K, I, G, s); break;
    case 6: e = launch<T, 8, 6, PACKED>(m, K, I, G, s); break;
    case 7: e = launch<T, 8, 7, PACKED>(m, K, I, G, s); break;
    case 8: e = launch<T, 8, 8, PACKED>(m, K, I, G, s); break;
  }
  return e == hipErrorInvalidConfiguration ? dispatch16<T, PACKED>(m, K, I, G, s) : e;
}

}  // namespace

hipError_t rt_launch_gradient(const rt_mesh *m, int K, const void *I, void *grad, int dtype, bool packed,
                              hipStream_t s) {
  if (packed)
    return dtype == RT_F32 ? dispatch<float, true>(m, K, I, grad, s) : dispatch<double, true>(m, K, I, grad, s);
  return dtype == RT_F32 ? dispatch<float, false>(m, K, I, grad, s) : dispatch<double, false>(m, K, I, grad, s);
}

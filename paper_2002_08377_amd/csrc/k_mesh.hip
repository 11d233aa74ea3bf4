// Mesh preparation, run once at upload: face normal speeds (eq. 9), the half-face
// records each cell gathers from, and the rate of change of the cell volumes.
#include "rt_device.h"

namespace {

// Face velocity of S10 (eq. 9): the mean generator velocity plus the correction
// [(w_i - w_j).(r~ - (r_i + r_j)/2) / |r_j - r_i|] (r_j - r_i)/|r_j - r_i|; only
// its component along the face normal enters the face-frame flux (section 2.2).
__global__ void k_face_speed(const double *gen, const double *w, const int32_t *fc, const int8_t *shift,
                             const double *nrm, const double *cen, double box, int64_t F, double *wn) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  const int64_t i = fc[2 * f], j = fc[2 * f + 1];
  double d[3], mid[3], dw[3], wb[3];
  for (int c = 0; c < 3; ++c) {
    const double rj = gen[3 * j + c] + shift[3 * f + c] * box;
    d[c] = rj - gen[3 * i + c];
    mid[c] = 0.5 * (rj + gen[3 * i + c]);
    dw[c] = w[3 * i + c] - w[3 * j + c];
    wb[c] = 0.5 * (w[3 * i + c] + w[3 * j + c]);
  }
  const double dist = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  double corr = 0.0;
  for (int c = 0; c < 3; ++c) corr += dw[c] * (cen[3 * f + c] - mid[c]);
  corr /= dist;
  double s = 0.0;
  for (int c = 0; c < 3; ++c) s += (corr * d[c] / dist + wb[c]) * nrm[3 * f + c];
  wn[f] = s;
}

// Gradient-estimator weights of half-face h seen from its own cell: cw = A c/d and
// nw = A/2 n_g, with c the face centroid minus the generators' midpoint, d the generator
// distance and n_g = (r_other - r_self)/d.  Geometry in the frame of the face's first cell a
// (b's image is gen[b] + shift * box).
struct rt_gp_weights {
  double cw[3], nw[3];
};
__device__ rt_gp_weights rt_half_face_gp(int64_t f, bool second, const int32_t *fc, const int8_t *shift,
                                         const double *area, const double *cen, const double *gen, double box) {
  const int64_t a = fc[2 * f], b = fc[2 * f + 1];
  const double A = area[f];
  double rab[3], cf[3];
  for (int c = 0; c < 3; ++c) {
    const double rb = gen[3 * b + c] + shift[3 * f + c] * box;
    rab[c] = gen[3 * a + c] - rb;
    cf[c] = cen[3 * f + c] - 0.5 * (gen[3 * a + c] + rb);
  }
  const double dist = sqrt(rab[0] * rab[0] + rab[1] * rab[1] + rab[2] * rab[2]);
  // self = a: n_g = -rab/d; self = b: n_g = +rab/d
  const double hq = second ? 0.5 * A / dist : -0.5 * A / dist;
  rt_gp_weights g;
  for (int c = 0; c < 3; ++c) {
    g.cw[c] = A * cf[c] / dist;
    g.nw[c] = hq * rab[c];
  }
  return g;
}

// One record per half-face h (face f seen from one of its cells, the "self" cell):
//   an  = (A n_out, A (w~.n)_out)            n_out = +n_f on the face's first cell, -n_f on its second
//   gp  = (A c/d + A/2 n_g, 0)               the neighbour's weight in the gradient estimator
//   rel = (r~ - s_self, r~ - s_other)         reconstruction offsets, each in its own cell's frame
// The estimator's sum over faces of (phi_j - phi_i) A c/d + (phi_i + phi_j) A/2 n_g is
// gathered as sum_j phi_j gp_j + phi_i b_i, with b_i = sum_faces (A/2 n_g - A c/d) per cell.
__global__ void k_half_faces(int64_t H, const int32_t *hf_face, const int32_t *fc, const int8_t *shift,
                             const double *area, const double *nrm, const double *cen, const double *wn,
                             const double *gen, const double *com, double box, int32_t *hf_nbr, double4 *an64,
                             float4 *an32, double4 *gp64, float4 *gp32, double4 *rel64, float4 *rel32) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= H) return;
  const int32_t code = hf_face[h];
  const bool second = code < 0;
  const int64_t f = second ? -(int64_t)code - 1 : code;
  const int64_t a = fc[2 * f], b = fc[2 * f + 1];
  const int64_t self = second ? b : a, other = second ? a : b;
  hf_nbr[h] = (int32_t)other;
  const double A = area[f];
  const double sg = second ? -1.0 : 1.0;
  const double4 r = make_double4(sg * A * nrm[3 * f], sg * A * nrm[3 * f + 1], sg * A * nrm[3 * f + 2],
                                 sg * A * wn[f]);
  an64[h] = r;
  an32[h] = make_float4((float)r.x, (float)r.y, (float)r.z, (float)r.w);
  if (!gp64) return;
  const rt_gp_weights g = rt_half_face_gp(f, second, fc, shift, area, cen, gen, box);
  const double4 e = make_double4(g.cw[0] + g.nw[0], g.cw[1] + g.nw[1], g.cw[2] + g.nw[2], 0.0);
  gp64[h] = e;
  gp32[h] = make_float4((float)e.x, (float)e.y, (float)e.z, 0.f);
  double cs[3], co[3];
  for (int c = 0; c < 3; ++c) {
    const double sh = shift[3 * f + c] * box;
    const double ca = cen[3 * f + c] - com[3 * a + c];
    const double cb = cen[3 * f + c] - sh - com[3 * b + c];
    cs[c] = second ? cb : ca;
    co[c] = second ? ca : cb;
  }
  const double4 q0 = make_double4(cs[0], cs[1], cs[2], co[0]);
  const double4 q1 = make_double4(co[1], co[2], 0.0, 0.0);
  rel64[2 * h] = q0;
  rel64[2 * h + 1] = q1;
  rel32[2 * h] = make_float4((float)q0.x, (float)q0.y, (float)q0.z, (float)q0.w);
  rel32[2 * h + 1] = make_float4((float)q1.x, (float)q1.y, 0.f, 0.f);
}

// b_i = sum over the cell's half-faces, in their order, of A/2 n_g - A c/d (FP64).
__global__ void k_gradient_base(int64_t N, const int32_t *row_ptr, const int32_t *hf_face, const int32_t *fc,
                                const int8_t *shift, const double *area, const double *cen, const double *gen,
                                double box, double4 *gb64, float4 *gb32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double s[3] = {0.0, 0.0, 0.0};
  for (int h = row_ptr[i]; h < row_ptr[i + 1]; ++h) {
    const int32_t code = hf_face[h];
    const bool second = code < 0;
    const int64_t f = second ? -(int64_t)code - 1 : code;
    const rt_gp_weights g = rt_half_face_gp(f, second, fc, shift, area, cen, gen, box);
    for (int c = 0; c < 3; ++c) s[c] += g.nw[c] - g.cw[c];
  }
  gb64[i] = make_double4(s[0], s[1], s[2], 0.0);
  gb32[i] = make_float4((float)s[0], (float)s[1], (float)s[2], 0.f);
}

// D_i = sum over the cell's half-faces of A (w~.n)_out.
__global__ void k_volume_rate(int64_t N, const int32_t *row_ptr, const double4 *an, double *D) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double s = 0.0;
  for (int h = row_ptr[i]; h < row_ptr[i + 1]; ++h) s += an[h].w;
  D[i] = s;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + RT_BLOCK - 1) / RT_BLOCK); }

}  // namespace

hipError_t rt_launch_face_speed(const double *gen, const double *mesh_vel, const int32_t *face_cells,
                                const int8_t *face_shift, const double *face_normal, const double *face_centroid,
                                double box, int64_t F, double *wn, hipStream_t s) {
  hipLaunchKernelGGL(k_face_speed, dim3(blocks_for(F)), dim3(RT_BLOCK), 0, s, gen, mesh_vel, face_cells, face_shift,
                     face_normal, face_centroid, box, F, wn);
  return hipGetLastError();
}

hipError_t rt_launch_half_faces(rt_mesh *m, const int32_t *face_cells, const double *face_area,
                                const double *face_normal, const double *face_centroid, const double *gen,
                                const double *com, const int8_t *face_shift, hipStream_t s) {
  hipLaunchKernelGGL(k_half_faces, dim3(blocks_for(m->H)), dim3(RT_BLOCK), 0, s, m->H, m->hf_face, face_cells,
                     face_shift, face_area, face_normal, face_centroid, m->wn, gen, com,
                     m->box, m->hf_nbr, m->hf_an64, m->hf_an32, m->hf_gp64, m->hf_gp32, m->hf_rel64, m->hf_rel32);
  return hipGetLastError();
}

hipError_t rt_launch_gradient_base(rt_mesh *m, const int32_t *face_cells, const double *face_area,
                                   const double *face_centroid, const double *gen, const int8_t *face_shift,
                                   hipStream_t s) {
  hipLaunchKernelGGL(k_gradient_base, dim3(blocks_for(m->N)), dim3(RT_BLOCK), 0, s, m->N, m->row_ptr, m->hf_face,
                     face_cells, face_shift, face_area, face_centroid, gen, m->box, m->gb64, m->gb32);
  return hipGetLastError();
}

hipError_t rt_launch_volume_rate(rt_mesh *m, hipStream_t s) {
  hipLaunchKernelGGL(k_volume_rate, dim3(blocks_for(m->N)), dim3(RT_BLOCK), 0, s, m->N, m->row_ptr, m->hf_an64,
                     m->D);
  return hipGetLastError();
}

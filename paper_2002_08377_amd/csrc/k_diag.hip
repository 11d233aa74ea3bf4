// Grid reductions: conservation diagnostics (section 2.3.1) and the emergent-flux
// loss with its seed; and the per-cell angle moments (section 2.1), reduced over each
// cell's lanes only.  Each cell group reduces over its angles, each workgroup
// over its cells through LDS, then two folds over the per-workgroup partials in a
// fixed order, so results are deterministic (no atomics).
#include <mutex>

#include "rt_device.h"

// Scratch of the loss that allocates nothing: the per-workgroup partial sums in its first
// RT_NOALLOC_PARTIALS doubles, the first fold in the last RT_BLOCK.  Each device holds
// its own copy for the life of the process.
static __device__ __align__(256) double rt_noalloc_scratch[RT_NOALLOC_PARTIALS + RT_BLOCK];

namespace {

constexpr int ND = RT_NDIAG;

// Block reduction of NV values held by lane 0 of each cell group; kinds: 0 sum, 1 min.
template <int NV, int LPC>
__device__ __forceinline__ void block_reduce_store(double (&v)[NV], const int (&kind)[NV], double *out_blk) {
  __shared__ double sh[RT_BLOCK / LPC][NV];
  constexpr int CPB = RT_BLOCK / LPC;
  const int g = threadIdx.x / LPC, l = threadIdx.x % LPC;
  if (l == 0)
    for (int i = 0; i < NV; ++i) sh[g][i] = v[i];
  __syncthreads();
  if (threadIdx.x < NV) {
    const int i = threadIdx.x;
    double acc = sh[0][i];
    for (int c = 1; c < CPB; ++c) acc = kind[i] ? fmin(acc, sh[c][i]) : acc + sh[c][i];
    out_blk[i] = acc;
  }
}

template <typename T, int LPC, int APL>
__global__ __launch_bounds__(RT_BLOCK) void k_diag(int64_t N, int K, const double *dirs, const double *W,
                                                   double c_red, double c_light, const T *I, const double *vol,
                                                   const double *etot, const double *mom, double *partial,
                                                   int64_t nblk) {
  const int64_t lb = rt_logical_block(nblk);
  if (lb < 0) return;
  constexpr int CPB = RT_BLOCK / LPC;
  const int64_t cell = lb * CPB + threadIdx.x / LPC;
  const int l = threadIdx.x % LPC;
  double v[ND] = {0, 0, 0, 0, 0, 0, 0, 0, INFINITY, 0};
  const int kind[ND] = {0, 0, 0, 0, 0, 0, 0, 0, 1, 0};
  if (cell < N) {
    rt_lane_angles<double, LPC, APL> ang;
    ang.load(dirs, W, K, l);
    double E = 0, Fx = 0, Fy = 0, Fz = 0, mn = INFINITY, bad = 0;
    for (int q = 0; q < APL; ++q) {
      if (!ang.ok[q]) continue;
      const double x = (double)I[cell * (int64_t)K + ang.k[q]];
      if (!isfinite(x)) bad += 1;
      mn = fmin(mn, x);
      E += ang.w[q] * x;
      Fx += ang.w[q] * ang.dx[q] * x;
      Fy += ang.w[q] * ang.dy[q] * x;
      Fz += ang.w[q] * ang.dz[q] * x;
    }
    E = rt_group_sum<LPC>(E);
    Fx = rt_group_sum<LPC>(Fx);
    Fy = rt_group_sum<LPC>(Fy);
    Fz = rt_group_sum<LPC>(Fz);
    bad = rt_group_sum<LPC>(bad);
    mn = rt_group_min<LPC>(mn);
    const double V = vol[cell], fp = 4.0 * RT_PI;
    const double eg = etot[cell];
    const double m[3] = {mom[3 * cell], mom[3 * cell + 1], mom[3 * cell + 2]};
    bad += !isfinite(eg) + !isfinite(m[0]) + !isfinite(m[1]) + !isfinite(m[2]);
    v[0] = V * eg;
    v[1] = V * (c_light / c_red) * fp * E;
    v[2] = V * m[0];
    v[3] = V * m[1];
    v[4] = V * m[2];
    v[5] = V * fp * Fx / c_red;
    v[6] = V * fp * Fy / c_red;
    v[7] = V * fp * Fz / c_red;
    v[8] = mn;
    v[9] = bad;
  }
  block_reduce_store<ND, LPC>(v, kind, partial + lb * ND);
}

// Fold rows [blockIdx.x * chunk, +chunk) of an [nrows][nv] table into row blockIdx.x of
// `out`: for column i, thread t folds rows t, t + 256, ... of the chunk in order, then a
// fixed tree in LDS.  The chunking depends on nrows only, so results are deterministic.
__global__ __launch_bounds__(RT_BLOCK) void k_fold(const double *partial, int64_t nrows, int nv,
                                                   unsigned min_mask, int64_t chunk, double *out) {
  __shared__ double sh[RT_BLOCK];
  const int t = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = r0 + chunk < nrows ? r0 + chunk : nrows;
  for (int i = 0; i < nv; ++i) {
    const bool is_min = (min_mask >> i) & 1u;
    double acc = is_min ? INFINITY : 0.0;
    for (int64_t b = r0 + t; b < r1; b += RT_BLOCK) {
      const double x = partial[b * nv + i];
      acc = is_min ? fmin(acc, x) : acc + x;
    }
    sh[t] = acc;
    __syncthreads();
    for (int o = RT_BLOCK / 2; o > 0; o >>= 1) {
      if (t < o) sh[t] = is_min ? fmin(sh[t], sh[t + o]) : sh[t] + sh[t + o];
      __syncthreads();
    }
    if (t == 0) out[blockIdx.x * nv + i] = sh[0];
    __syncthreads();
  }
}

// Two folds: up to RT_BLOCK workgroups over contiguous chunks of the per-workgroup
// partials into `mid` ([RT_BLOCK][nv]), then one workgroup over those into `out`.
hipError_t reduce_partials(const double *partial, int64_t nrows, int nv, unsigned min_mask, double *mid,
                           double *out, hipStream_t s) {
  const int64_t g = nrows < RT_BLOCK ? nrows : RT_BLOCK;
  const int64_t chunk = (nrows + g - 1) / g;
  hipLaunchKernelGGL(k_fold, dim3((unsigned)g), dim3(RT_BLOCK), 0, s, partial, nrows, nv, min_mask, chunk, mid);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fold, dim3(1), dim3(RT_BLOCK), 0, s, (const double *)mid, g, nv, min_mask, g, out);
  return hipGetLastError();
}

// Loss: each (face, angle) belongs to its upwind cell (A n_out . n_k > 0), which adds
// u_f sigma 4 pi c W_k (A n_out . n_k) I to its partial loss and that coefficient to
// its seed; sigma = -1 on a face's second cell since n_out = -n_f there.
template <typename T, int LPC, int APL>
__global__ __launch_bounds__(RT_BLOCK) void k_loss(int64_t N, int K, const int32_t *row_ptr, const int32_t *hf_face,
                                                   const double4 *hf_an, const double *dirs, const double *W,
                                                   double c_light, const T *I, const double *face_weight,
                                                   T *seed, double *partial, int64_t nblk) {
  const int64_t lb = rt_logical_block(nblk);
  if (lb < 0) return;
  constexpr int CPB = RT_BLOCK / LPC;
  const int64_t cell = lb * CPB + threadIdx.x / LPC;
  const int l = threadIdx.x % LPC;
  double v[1] = {0.0};
  const int kind[1] = {0};
  if (cell < N) {
    rt_lane_angles<double, LPC, APL> ang;
    ang.load(dirs, W, K, l);
    const int64_t row = cell * (int64_t)K;
    double sd[APL], Iv[APL];
    for (int q = 0; q < APL; ++q) sd[q] = Iv[q] = 0.0;
    bool have_row = false;  // the row is read only by cells with a weighted face (few)
    const double fpc = 4.0 * RT_PI * c_light;
    double part = 0.0;
    const int h0 = row_ptr[cell], h1 = row_ptr[cell + 1];
    constexpr int B = 4;  // faces whose ids and weights are fetched together
    for (int hb = h0; hb < h1; hb += B) {
      int32_t fc[B];
      double u[B];
#pragma unroll
      for (int b = 0; b < B; ++b) fc[b] = hb + b < h1 ? hf_face[hb + b] : 0;
#pragma unroll
      for (int b = 0; b < B; ++b) u[b] = hb + b < h1 ? face_weight[fc[b] >= 0 ? fc[b] : -(int64_t)fc[b] - 1] : 0.0;
#pragma unroll
      for (int b = 0; b < B; ++b) {
        if (u[b] == 0.0) continue;
        if (!have_row) {
          for (int q = 0; q < APL; ++q) Iv[q] = ang.ok[q] ? (double)I[row + ang.k[q]] : 0.0;
          have_row = true;
        }
        const double sg = fc[b] >= 0 ? u[b] : -u[b];
        const double4 r = hf_an[hb + b];
        for (int q = 0; q < APL; ++q) {
          const double m = r.x * ang.dx[q] + r.y * ang.dy[q] + r.z * ang.dz[q];
          if (m > 0.0) {
            const double coef = sg * fpc * ang.w[q] * m;
            part += coef * Iv[q];
            sd[q] += coef;
          }
        }
      }
    }
    if (seed)
      for (int q = 0; q < APL; ++q)
        if (ang.ok[q] && sd[q] != 0.0) seed[row + ang.k[q]] = (T)((double)seed[row + ang.k[q]] + sd[q]);
    v[0] = rt_group_sum<LPC>(part);
  }
  block_reduce_store<1, LPC>(v, kind, partial + lb);
}

// Angle moments of every cell (section 2.1): with intensities in energy-density units,
// E_r = 4 pi sum W I, F_r = 4 pi c sum W n I, P_r = 4 pi sum W n n I.  The LPC lanes of a
// cell sum their angles; the group sums (DPP) leave the totals in every lane, and lane c
// writes component c (two rounds when LPC = 8), so a cell's 80 bytes go out together.
// Each lane group takes RT_MOM_CELLS cells (CPB apart, so every round of a workgroup reads
// consecutive rows): the lane's directions and weights are loaded once for all of them,
// and all their intensity loads are issued before any is used.
#define RT_MOM_CELLS 4
template <typename T, int LPC, int APL>
__global__ __launch_bounds__(RT_BLOCK) void k_moments(int64_t N, int K, const double *dirs, const double *W,
                                                      double c_light, const T *I, double *out, int64_t nblk) {
  const int64_t lb = rt_logical_block(nblk);
  if (lb < 0) return;
  constexpr int CPB = RT_BLOCK / LPC;
  constexpr int R = RT_MOM_CELLS;
  const int64_t c0 = lb * CPB * R + threadIdx.x / LPC;
  if (c0 >= N) return;  // whole lane groups
  const int l = threadIdx.x % LPC;
  rt_lane_angles<double, LPC, APL> ang;
  ang.load(dirs, W, K, l);
  T x[R][APL];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t cell = c0 + (int64_t)CPB * r;
#pragma unroll
    for (int q = 0; q < APL; ++q) x[r][q] = cell < N && ang.ok[q] ? I[cell * (int64_t)K + ang.k[q]] : T(0);
  }
  const double fourpi = 4.0 * RT_PI;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t cell = c0 + (int64_t)CPB * r;
    if (cell >= N) break;  // the same for all lanes of the group
    double m[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < APL; ++q) {
      const double wI = ang.w[q] * (double)x[r][q];
      const double nx = ang.dx[q], ny = ang.dy[q], nz = ang.dz[q];
      m[0] += wI;
      m[1] += wI * nx;
      m[2] += wI * ny;
      m[3] += wI * nz;
      m[4] += wI * nx * nx;
      m[5] += wI * ny * ny;
      m[6] += wI * nz * nz;
      m[7] += wI * nx * ny;
      m[8] += wI * nx * nz;
      m[9] += wI * ny * nz;
    }
    double v[10];
#pragma unroll
    for (int c = 0; c < 10; ++c) v[c] = rt_group_sum<LPC>(m[c]) * (c >= 1 && c <= 3 ? fourpi * c_light : fourpi);
#pragma unroll
    for (int b = 0; b < 10; b += LPC) {
      // lane l writes component b + l
      double o = v[b];
#pragma unroll
      for (int c = b + 1; c < b + LPC && c < 10; ++c)
        if (l == c - b) o = v[c];
      if (b + l < 10) out[10 * cell + b + l] = o;
    }
  }
}

// Angle moments with 16-byte row chunks: 4 lanes per cell, lane l reading chunks
// l, l + 4, ... (CPL of them) of its cell's row, so a wave's loads cover 16 rows 64 bytes
// at a time (the cheapest access pattern for these rows).  Each angle's (W, n) comes from
// LDS, where every lane at one position reads the same entry; the 4 lanes' moments are
// summed by DPP quad permutations.  Needs rows of whole 16-byte chunks, 16-byte aligned.
template <typename T, int CPL>
__global__ __launch_bounds__(RT_BLOCK) void k_moments16(int64_t N, int K, const double *dirs, const double *W,
                                                        double c_light, const T *I, double *out, int64_t nblk) {
  constexpr int EPC = 16 / sizeof(T);  // elements per chunk
  __shared__ double4 s_dw[RT_K_MAX];   // (W, n_x, n_y, n_z) per angle
  for (int k = threadIdx.x; k < K; k += RT_BLOCK) s_dw[k] = double4{W[k], dirs[3 * k], dirs[3 * k + 1], dirs[3 * k + 2]};
  __syncthreads();
  const int64_t lb = rt_logical_block(nblk);
  if (lb < 0) return;
  const int64_t cell = lb * (RT_BLOCK / 4) + threadIdx.x / 4;
  if (cell >= N) return;  // whole lane groups
  const int l = threadIdx.x % 4;
  const int nch = K / EPC;  // chunks per row
  // the lane's chunks, all loads issued before any is used
  const char *row = (const char *)(I + cell * (int64_t)K);
  T x[CPL][EPC];
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    const int ch = l + 4 * c;
    if (ch < nch) {
      if constexpr (EPC == 4) {
        const float4 v = *(const float4 *)(row + 16 * ch);
        x[c][0] = v.x; x[c][1] = v.y; x[c][2] = v.z; x[c][3] = v.w;
      } else {
        const double2 v = *(const double2 *)(row + 16 * ch);
        x[c][0] = v.x; x[c][1] = v.y;
      }
    } else {
#pragma unroll
      for (int e = 0; e < EPC; ++e) x[c][e] = T(0);
    }
  }
  double m[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    const int ch = l + 4 * c;
    if (ch >= nch) continue;
#pragma unroll
    for (int e = 0; e < EPC; ++e) {
      const double4 d = s_dw[EPC * ch + e];
      const double t = d.x * (double)x[c][e];
      const double tx = t * d.y, ty = t * d.z, tz = t * d.w;
      m[0] += t;
      m[1] += tx;
      m[2] += ty;
      m[3] += tz;
      m[4] += tx * d.y;
      m[5] += ty * d.z;
      m[6] += tz * d.w;
      m[7] += tx * d.z;
      m[8] += tx * d.w;
      m[9] += ty * d.w;
    }
  }
  const double fourpi = 4.0 * RT_PI;
  double v[10];
#pragma unroll
  for (int c = 0; c < 10; ++c) v[c] = rt_group_sum<4>(m[c]) * (c >= 1 && c <= 3 ? fourpi * c_light : fourpi);
  // lane l writes components l, l + 4 and (l < 2) l + 8
#pragma unroll
  for (int b = 0; b < 10; b += 4) {
    double o = v[b];
#pragma unroll
    for (int c = b + 1; c < b + 4 && c < 10; ++c)
      if (l == c - b) o = v[c];
    if (b + l < 10) out[10 * cell + b + l] = o;
  }
}

// The same moments for an antipodal set (pair kind 1: angle k's antipode at k + K/2; 2: at
// k + 1 for even k).  Each pair (k, k'), n_k' = -n_k and W_k' = W_k, adds W (I_k + I_k') to
// the energy and the pressure and W (I_k - I_k') n_k to the flux: one direction read and
// half the multiply-adds per angle.  Lane l of a cell's 4 takes chunks l, l + 4, ... of the
// first half of the row with their antipodes' chunks (kind 1), or whole chunks holding
// EPC / 2 pairs (kind 2).  Needs what the chunked kernel needs, and K / 2 a multiple of
// EPC for kind 1.
template <typename T, int CPL, int PAIRED>
__global__ __launch_bounds__(RT_BLOCK) void k_moments16p(int64_t N, int K, const double *dirs, const double *W,
                                                         double c_light, const T *I, double *out, int64_t nblk) {
  constexpr int EPC = 16 / sizeof(T);          // elements per chunk
  constexpr int PPC = PAIRED == 1 ? EPC : EPC / 2;  // pairs per chunk (kind 1: with its antipode chunk)
  __shared__ double4 s_dw[RT_K_MAX];           // (W, n_x, n_y, n_z) per angle
  for (int k = threadIdx.x; k < K; k += RT_BLOCK) s_dw[k] = double4{W[k], dirs[3 * k], dirs[3 * k + 1], dirs[3 * k + 2]};
  __syncthreads();
  const int64_t lb = rt_logical_block(nblk);
  if (lb < 0) return;
  const int64_t cell = lb * (RT_BLOCK / 4) + threadIdx.x / 4;
  if (cell >= N) return;  // whole lane groups
  const int l = threadIdx.x % 4;
  const int nc = PAIRED == 1 ? K / (2 * EPC) : K / EPC;  // chunks the lanes walk
  const char *row = (const char *)(I + cell * (int64_t)K);
  T x[CPL][EPC], y[CPL][EPC];
  auto load = [&](T(&v)[EPC], int ch) {
    if constexpr (EPC == 4) {
      const float4 a = *(const float4 *)(row + 16 * ch);
      v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    } else {
      const double2 a = *(const double2 *)(row + 16 * ch);
      v[0] = a.x; v[1] = a.y;
    }
  };
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    const int ch = l + 4 * c;
    if (ch < nc) {
      load(x[c], ch);
      if (PAIRED == 1) load(y[c], ch + nc);
    }
  }
  double m[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    const int ch = l + 4 * c;
    if (ch >= nc) continue;
#pragma unroll
    for (int e = 0; e < PPC; ++e) {
      const double a = (double)(PAIRED == 1 ? x[c][e] : x[c][2 * e]);
      const double b = (double)(PAIRED == 1 ? y[c][e] : x[c][2 * e + 1]);
      const double4 d = s_dw[EPC * ch + (PAIRED == 1 ? e : 2 * e)];
      const double t = d.x * (a + b), u = d.x * (a - b);
      const double tx = t * d.y, ty = t * d.z, tz = t * d.w;
      m[0] += t;
      m[1] += u * d.y;
      m[2] += u * d.z;
      m[3] += u * d.w;
      m[4] += tx * d.y;
      m[5] += ty * d.z;
      m[6] += tz * d.w;
      m[7] += tx * d.z;
      m[8] += tx * d.w;
      m[9] += ty * d.w;
    }
  }
  const double fourpi = 4.0 * RT_PI;
  double v[10];
#pragma unroll
  for (int c = 0; c < 10; ++c) v[c] = rt_group_sum<4>(m[c]) * (c >= 1 && c <= 3 ? fourpi * c_light : fourpi);
  // lane l writes components l, l + 4 and (l < 2) l + 8
#pragma unroll
  for (int b = 0; b < 10; b += 4) {
    double o = v[b];
#pragma unroll
    for (int c = b + 1; c < b + 4 && c < 10; ++c)
      if (l == c - b) o = v[c];
    if (b + l < 10) out[10 * cell + b + l] = o;
  }
}

template <typename T, int CPL, int PAIRED>
hipError_t launch_moments16p(const rt_mesh *m, int K, const double *dirs, const double *W, double c_light,
                             const void *I, double *out, hipStream_t s) {
  const int64_t nblk = (m->N + RT_BLOCK / 4 - 1) / (RT_BLOCK / 4);
  hipLaunchKernelGGL((k_moments16p<T, CPL, PAIRED>), dim3((unsigned)rt_grid_for(nblk)), dim3(RT_BLOCK), 0, s, m->N,
                     K, dirs, W, c_light, (const T *)I, out, nblk);
  return hipGetLastError();
}

template <typename T, int PAIRED>
hipError_t dispatch_moments16p(const rt_mesh *m, int K, const double *dirs, const double *W, double c_light,
                               const void *I, double *out, hipStream_t s) {
  constexpr int EPC = 16 / sizeof(T);
  const int nc = PAIRED == 1 ? K / (2 * EPC) : K / EPC;
  switch ((nc + 3) / 4) {  // chunks (kind 1: chunk pairs) per lane
    case 1: return launch_moments16p<T, 1, PAIRED>(m, K, dirs, W, c_light, I, out, s);
    case 2: return launch_moments16p<T, 2, PAIRED>(m, K, dirs, W, c_light, I, out, s);
    case 3: return launch_moments16p<T, 3, PAIRED>(m, K, dirs, W, c_light, I, out, s);
    case 4: return launch_moments16p<T, 4, PAIRED>(m, K, dirs, W, c_light, I, out, s);
    case 5: return launch_moments16p<T, 5, PAIRED>(m, K, dirs, W, c_light, I, out, s);
    case 6: return launch_moments16p<T, 6, PAIRED>(m, K, dirs, W, c_light, I, out, s);
    case 7: return launch_moments16p<T, 7, PAIRED>(m, K, dirs, W, c_light, I, out, s);
    case 8: return launch_moments16p<T, 8, PAIRED>(m, K, dirs, W, c_light, I, out, s);
  }
  return hipErrorInvalidValue;
}

template <typename T, int CPL>
hipError_t launch_moments16(const rt_mesh *m, int K, const double *dirs, const double *W, double c_light,
                            const void *I, double *out, hipStream_t s) {
  const int64_t nblk = (m->N + RT_BLOCK / 4 - 1) / (RT_BLOCK / 4);
  hipLaunchKernelGGL((k_moments16<T, CPL>), dim3((unsigned)rt_grid_for(nblk)), dim3(RT_BLOCK), 0, s, m->N, K, dirs,
                     W, c_light, (const T *)I, out, nblk);
  return hipGetLastError();
}

template <typename T, int LPC, int APL>
hipError_t launch_moments(const rt_mesh *m, int K, const double *dirs, const double *W, double c_light, const void *I,
                          double *out, hipStream_t s) {
  const int64_t cpc = (int64_t)(RT_BLOCK / LPC) * RT_MOM_CELLS;  // cells per workgroup
  const int64_t nblk = (m->N + cpc - 1) / cpc;
  hipLaunchKernelGGL((k_moments<T, LPC, APL>), dim3((unsigned)rt_grid_for(nblk)), dim3(RT_BLOCK), 0, s, m->N, K,
                     dirs, W, c_light, (const T *)I, out, nblk);
  return hipGetLastError();
}

template <typename T, int LPC, int APL>
hipError_t launch_diag(const rt_mesh *m, int K, const double *dirs, const double *W, double c_red, double c_light,
                       const void *I, const double *vol, const double *etot, const double *mom, double *out,
                       hipStream_t s) {
  const int64_t cpb = RT_BLOCK / LPC;
  const int64_t nblk = (m->N + cpb - 1) / cpb;
  if (nblk > m->n_red_blocks) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_diag<T, LPC, APL>), dim3((unsigned)rt_grid_for(nblk)), dim3(RT_BLOCK), 0, s, m->N, K, dirs,
                     W, c_red, c_light, (const T *)I, vol, etot, mom, m->red, nblk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return reduce_partials(m->red, nblk, ND, 1u << 8, m->red_mid, out, s);
}

// The loss into `partial` (one row per workgroup, at most `cap` rows), folded through `mid`
// ([RT_BLOCK] rows) into *loss.
template <typename T, int LPC, int APL>
hipError_t launch_loss(const rt_mesh *m, int K, const double *dirs, const double *W, double c_light, const void *I,
                       const double *fw, double *loss, void *seed, double *partial, double *mid, int64_t cap,
                       hipStream_t s) {
  const int64_t cpb = RT_BLOCK / LPC;
  const int64_t nblk = (m->N + cpb - 1) / cpb;
  if (nblk > cap) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_loss<T, LPC, APL>), dim3((unsigned)rt_grid_for(nblk)), dim3(RT_BLOCK), 0, s, m->N, K,
                     m->row_ptr, m->hf_face, m->hf_an64, dirs, W, c_light, (const T *)I, fw, (T *)seed, partial,
                     nblk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return reduce_partials(partial, nblk, 1, 0u, mid, loss, s);
}

#define RT_DISPATCH(FN, T, ...)                                   \
  do {                                                            \
    if (K % 16 == 0 || K > 64) {                                  \
      switch ((K + 15) / 16) {                                    \
        case 1: return FN<T, 16, 1>(__VA_ARGS__);                 \
        case 2: return FN<T, 16, 2>(__VA_ARGS__);                 \
        case 3: return FN<T, 16, 3>(__VA_ARGS__);                 \
        case 4: return FN<T, 16, 4>(__VA_ARGS__);                 \
        case 5: return FN<T, 16, 5>(__VA_ARGS__);                 \
        case 6: return FN<T, 16, 6>(__VA_ARGS__);                 \
        case 7: return FN<T, 16, 7>(__VA_ARGS__);                 \
        case 8: return FN<T, 16, 8>(__VA_ARGS__);                 \
      }                                                           \
    } else {                                                      \
      switch ((K + 7) / 8) {                                      \
        case 1: return FN<T, 8, 1>(__VA_ARGS__);                  \
        case 2: return FN<T, 8, 2>(__VA_ARGS__);                  \
        case 3: return FN<T, 8, 3>(__VA_ARGS__);                  \
        case 4: return FN<T, 8, 4>(__VA_ARGS__);                  \
        case 5: return FN<T, 8, 5>(__VA_ARGS__);                  \
        case 6: return FN<T, 8, 6>(__VA_ARGS__);                  \
        case 7: return FN<T, 8, 7>(__VA_ARGS__);                  \
        case 8: return FN<T, 8, 8>(__VA_ARGS__);                  \
      }                                                           \
    }                                                             \
    return hipErrorInvalidValue;                                  \
  } while (0)

template <typename T>
hipError_t diag_t(const rt_mesh *m, int K, const double *dirs, const double *W, double c_red, double c_light,
                  const void *I, const double *vol, const double *etot, const double *mom, double *out,
                  hipStream_t s) {
  RT_DISPATCH(launch_diag, T, m, K, dirs, W, c_red, c_light, I, vol, etot, mom, out, s);
}

template <typename T>
hipError_t moments_t(const rt_mesh *m, int K, const double *dirs, const double *W, double c_light, const void *I,
                     double *out, int paired, hipStream_t s) {
  // rows of whole 16-byte chunks starting 16-byte aligned: the chunked kernel, 4 lanes per cell
  constexpr int EPC = 16 / sizeof(T);
  const bool chunked = K % EPC == 0 && ((uintptr_t)I & 15u) == 0;
  // antipodal sets whose pairs sit whole in the chunks (kind 2) or fill whole chunks in each
  // half of the row (kind 1): the paired form
  if (chunked && paired == 2 && EPC % 2 == 0 && K <= 32 * EPC)
    return dispatch_moments16p<T, 2>(m, K, dirs, W, c_light, I, out, s);
  if (chunked && paired == 1 && K % (2 * EPC) == 0 && K <= 64 * EPC)
    return dispatch_moments16p<T, 1>(m, K, dirs, W, c_light, I, out, s);
  if (chunked) {
    switch ((K / EPC + 3) / 4) {  // chunks per lane
      case 1: return launch_moments16<T, 1>(m, K, dirs, W, c_light, I, out, s);
      case 2: return launch_moments16<T, 2>(m, K, dirs, W, c_light, I, out, s);
      case 3: return launch_moments16<T, 3>(m, K, dirs, W, c_light, I, out, s);
      case 4: return launch_moments16<T, 4>(m, K, dirs, W, c_light, I, out, s);
      case 5: return launch_moments16<T, 5>(m, K, dirs, W, c_light, I, out, s);
      case 6: return launch_moments16<T, 6>(m, K, dirs, W, c_light, I, out, s);
      case 7: return launch_moments16<T, 7>(m, K, dirs, W, c_light, I, out, s);
      case 8: return launch_moments16<T, 8>(m, K, dirs, W, c_light, I, out, s);
      case 9: return launch_moments16<T, 9>(m, K, dirs, W, c_light, I, out, s);
      case 10: return launch_moments16<T, 10>(m, K, dirs, W, c_light, I, out, s);
      case 11: return launch_moments16<T, 11>(m, K, dirs, W, c_light, I, out, s);
      case 12: return launch_moments16<T, 12>(m, K, dirs, W, c_light, I, out, s);
      case 13: return launch_moments16<T, 13>(m, K, dirs, W, c_light, I, out, s);
      case 14: return launch_moments16<T, 14>(m, K, dirs, W, c_light, I, out, s);
      case 15: return launch_moments16<T, 15>(m, K, dirs, W, c_light, I, out, s);
      case 16: return launch_moments16<T, 16>(m, K, dirs, W, c_light, I, out, s);
    }
  }
  RT_DISPATCH(launch_moments, T, m, K, dirs, W, c_light, I, out, s);
}

template <typename T>
hipError_t loss_t(const rt_mesh *m, int K, const double *dirs, const double *W, double c_light, const void *I,
                  const double *fw, double *loss, void *seed, double *partial, double *mid, int64_t cap,
                  hipStream_t s) {
  RT_DISPATCH(launch_loss, T, m, K, dirs, W, c_light, I, fw, loss, seed, partial, mid, cap, s);
}

// Device address of the scratch on each device, looked up once per device with that
// device current (host code must never use the array's own name as a device pointer).
std::mutex g_scratch_mu;
double *g_scratch_ptr[RT_MAX_DEVICES] = {};

hipError_t noalloc_scratch(int device, double **out) {
  if (device < 0 || device >= RT_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(rt_noalloc_scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = (double *)p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

}  // namespace

hipError_t rt_launch_diagnostics(const rt_mesh *m, int K, const double *dirs, const double *W, double c_red,
                                 double c_light, const void *I, const double *vol, const double *etot,
                                 const double *mom, double *out_dev, int dtype, hipStream_t s) {
  return dtype == RT_F32 ? diag_t<float>(m, K, dirs, W, c_red, c_light, I, vol, etot, mom, out_dev, s)
                         : diag_t<double>(m, K, dirs, W, c_red, c_light, I, vol, etot, mom, out_dev, s);
}

hipError_t rt_launch_flux_loss(const rt_mesh *m, int K, const double *dirs, const double *W, double c_light,
                               const void *I, const double *face_weight, double *loss, void *seed, int dtype,
                               hipStream_t s) {
  return dtype == RT_F32
             ? loss_t<float>(m, K, dirs, W, c_light, I, face_weight, loss, seed, m->red, m->red_mid, m->n_red_blocks, s)
             : loss_t<double>(m, K, dirs, W, c_light, I, face_weight, loss, seed, m->red, m->red_mid, m->n_red_blocks,
                              s);
}

int64_t rt_loss_blocks(int64_t N, int K) {
  const int64_t cpb = (K % 16 == 0 || K > 64) ? RT_BLOCK / 16 : RT_BLOCK / 8;  // the lane layout of RT_DISPATCH
  return (N + cpb - 1) / cpb;
}

hipError_t rt_launch_flux_loss_noalloc(const rt_mesh *m, int K, const double *dirs, const double *W, double c_light,
                                       const void *I, const double *face_weight, double *loss, void *seed, int dtype,
                                       hipStream_t s) {
  double *scratch = nullptr;
  const hipError_t e = noalloc_scratch(m->device, &scratch);
  if (e != hipSuccess) return e;
  double *mid = scratch + RT_NOALLOC_PARTIALS;
  return dtype == RT_F32
             ? loss_t<float>(m, K, dirs, W, c_light, I, face_weight, loss, seed, scratch, mid, RT_NOALLOC_PARTIALS, s)
             : loss_t<double>(m, K, dirs, W, c_light, I, face_weight, loss, seed, scratch, mid, RT_NOALLOC_PARTIALS,
                              s);
}

hipError_t rt_launch_moments(const rt_mesh *m, int K, const double *dirs, const double *W, double c_light,
                             const void *I, double *out, int dtype, int paired, hipStream_t s) {
  return dtype == RT_F32 ? moments_t<float>(m, K, dirs, W, c_light, I, out, paired, s)
                         : moments_t<double>(m, K, dirs, W, c_light, I, out, paired, s);
}

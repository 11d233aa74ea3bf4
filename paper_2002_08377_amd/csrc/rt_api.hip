// Host side of the C ABI declared in rtmm.h: argument checks, mesh upload (the
// half-face index every cell gathers through), scratch management and the launch
// sequence of each call.  All arithmetic of the method runs in the kernels.
#include <math.h>

#include <cmath>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "rt_internal.h"
#include "rt_mesh_host.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(RT_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define RT_HIP(call, what)                     \
  do {                                         \
    hipError_t e_ = (call);                    \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

template <typename P> hipError_t dmalloc(P **p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) return hipSuccess;
  return hipMalloc((void **)p, bytes);
}

void free_mesh_arrays(rt_mesh *m) {
  void *ptrs[] = {m->vol0,     m->D,       m->wn,      m->row_ptr,    m->hf_nbr,     m->hf_face,
                  m->hf_an64,   m->hf_an32, m->hf_gp64, m->hf_rel64,   m->hf_gp32,    m->hf_rel32,
                  m->gb64,      m->gb32,    m->I_half,  m->grad,       m->lam_star,   m->red,
                  m->red_mid,   m->wg_order16, m->wg_order32, m->wg_order64};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
}

bool aligned8(const void *p) { return ((uintptr_t)p & 7u) == 0; }

// Antipodal layout claims verified by rt_angles_check against the device arrays they name.
// A claim of RT_ANGLES_ANTIPODAL or RT_ANGLES_ANTIPODAL_ADJACENT reaches the paired
// kernels (which take the antipode's direction as -n and its weight as the angle's)
// only if it is recorded here.
struct checked_claim {
  const double *dir, *weight;
  int32_t K, layout;
};
std::mutex g_claims_mu;
std::vector<checked_claim> g_claims;

bool claim_checked(const rt_angles *a) {
  std::lock_guard<std::mutex> lk(g_claims_mu);
  for (const checked_claim &c : g_claims)
    if (c.dir == a->dir && c.weight == a->weight && c.K == a->K && c.layout == a->layout) return true;
  return false;
}

int check_call(const rt_mesh *m, const rt_params *p, const rt_angles *a) {
  if (!m) return fail(RT_EINVAL, "mesh is NULL");
  if (!p) return fail(RT_EINVAL, "params is NULL");
  if (!a) return fail(RT_EINVAL, "angles is NULL");
  if (a->K < 1 || a->K > m->k_max || a->K > RT_K_MAX)
    return fail(RT_EINVAL, "K=%d outside [1, k_max=%d]", a->K, m->k_max);
  if (!a->dir || !a->weight) return fail(RT_EINVAL, "angle arrays are NULL");
  if (a->layout != RT_ANGLES_GENERAL &&
      !((a->layout == RT_ANGLES_ANTIPODAL || a->layout == RT_ANGLES_ANTIPODAL_ADJACENT) && a->K % 2 == 0))
    return fail(RT_EINVAL, "invalid angle layout %d for K=%d", a->layout, a->K);
  if (a->layout != RT_ANGLES_GENERAL && !claim_checked(a))
    return fail(RT_EINVAL, "angle layout %d (K=%d) was not verified by rt_angles_check", a->layout, a->K);
  if (!(p->dt > 0.0) || !isfinite(p->dt)) return fail(RT_EINVAL, "dt must be positive and finite");
  if (!(p->c_red > 0.0) || !isfinite(p->c_red)) return fail(RT_EINVAL, "c_red must be positive");
  if (!(p->c_light >= p->c_red) || !isfinite(p->c_light)) return fail(RT_EINVAL, "c_light must be >= c_red");
  if (!(p->a_rad >= 0.0) || !isfinite(p->a_rad)) return fail(RT_EINVAL, "a_rad must be >= 0");
  if (!(p->cv > 0.0) || !isfinite(p->cv)) return fail(RT_EINVAL, "cv must be positive");
  if (p->dtype != RT_F64 && p->dtype != RT_F32) return fail(RT_EINVAL, "unknown dtype %d", p->dtype);
  if (p->scheme != RT_UPWIND1 && p->scheme != RT_PLM_VL2) return fail(RT_EINVAL, "unknown scheme %d", p->scheme);
  return RT_OK;
}

int check_ptrs(std::initializer_list<const void *> ps) {
  for (const void *q : ps) {
    if (!q) return fail(RT_EINVAL, "a required device pointer is NULL");
    if (!aligned8(q)) return fail(RT_EINVAL, "a device pointer is not 8-byte aligned");
  }
  return RT_OK;
}

size_t elem(int dtype) { return dtype == RT_F32 ? sizeof(float) : sizeof(double); }

bool overlap(const void *a, const void *b, size_t bytes) {
  const char *x = (const char *)a, *y = (const char *)b;
  return x < y + bytes && y < x + bytes;
}

rt_step_args base_args(const rt_mesh *m, const rt_params *p, const rt_angles *a) {
  rt_step_args s;
  memset(&s, 0, sizeof s);
  s.N = m->N;
  s.K = a->K;
  s.row_ptr = m->row_ptr;
  s.hf_nbr = m->hf_nbr;
  s.hf_an = p->dtype == RT_F32 ? (const void *)m->hf_an32 : (const void *)m->hf_an64;
  s.hf_rel = p->dtype == RT_F32 ? (const void *)m->hf_rel32 : (const void *)m->hf_rel64;
  s.D = m->D;
  s.dirs = a->dir;
  s.W = a->weight;
  s.c_red = p->c_red;
  s.c_light = p->c_light;
  s.a_rad = p->a_rad;
  s.cv = p->cv;
  s.dt = p->dt;
  s.inv_c = 1.0 / p->c_light;
  s.e_gain = 4.0 * M_PI * p->c_light / p->c_red;
  s.m_gain = 4.0 * M_PI / p->c_red;
  s.a_4pi = p->a_rad / (4.0 * M_PI);
  s.paired = rt_pair_kind(a->layout);
  s.lds_max = m->lds_max;
  s.hf_cap16 = m->hf_cap16;
  s.hf_cap32 = m->hf_cap32;
  s.hf_cap64 = m->hf_cap64;
  s.wg_order16 = m->wg_order16;
  s.wg_order32 = m->wg_order32;
  s.wg_order64 = m->wg_order64;
  return s;
}

// The transport part of a step; with `src` set, the source follows each stage.
int run_step(rt_mesh *m, const rt_params *p, const rt_angles *a, const void *I_in, void *I_out, double *vol,
             const double *rho, double *mom, double *etot, const double *kP, const double *kJ, const double *ks,
             double *T_new, bool src, hipStream_t st, void *I_star = nullptr, double *src_tape = nullptr) {
  rt_step_args s = base_args(m, p, a);
  s.rho = rho;
  s.mom = mom;
  s.etot = etot;
  s.kP = kP;
  s.kJ = kJ;
  s.ks = ks;
  if (p->scheme == RT_UPWIND1) {
    s.I_in = I_in;
    s.I_out = I_out;
    s.I_star_out = I_star;
    s.src_tape_out = src_tape;
    s.vol_in = vol;
    s.vol_out = vol;
    s.T_out = T_new;
    s.do_transport = 1;
    s.do_source = src;
    s.write_gas = 1;
    hipError_t e = rt_launch_step(s, p->dtype, st);
    if (e != hipSuccess) return hip_fail(e, "step kernel launch");
    return RT_OK;
  }
  if (!(m->flags & RT_MESH_PLM)) return fail(RT_ESTATE, "RT_PLM_VL2 needs a mesh uploaded with RT_MESH_PLM");
  // stage 1: first-order transport and source over dt/2 into the half-step state; gas untouched
  rt_step_args s1 = s;
  s1.dt = 0.5 * p->dt;
  s1.I_in = I_in;
  s1.I_out = m->I_half;
  s1.vol_in = vol;
  s1.vol_out = nullptr;
  s1.do_transport = 1;
  s1.do_source = src;
  s1.write_gas = 0;
  hipError_t e = rt_launch_step(s1, p->dtype, st);
  if (e != hipSuccess) return hip_fail(e, "stage-1 kernel launch");
  // FP32: (I_half, gradient) packed per cell and angle for stage 2; FP64: the gradient alone
  e = rt_launch_gradient(m, a->K, m->I_half, m->grad, p->dtype, p->dtype == RT_F32, st);
  if (e != hipSuccess) return hip_fail(e, "gradient kernel launch");
  // stage 2: reconstructed fluxes of the half-step state on the start-of-step charges, source on gas^n
  rt_step_args s2 = s;
  s2.I_in = I_in;
  s2.I_half = m->I_half;
  s2.grad = m->grad;
  s2.I_out = I_out;
  s2.vol_in = vol;
  s2.vol_out = vol;
  s2.T_out = T_new;
  s2.do_transport = 2;
  s2.do_source = src;
  s2.write_gas = 1;
  e = rt_launch_step(s2, p->dtype, st);
  if (e != hipSuccess) return hip_fail(e, "stage-2 kernel launch");
  return RT_OK;
}

}  // namespace

extern "C" {

const char *rt_strerror(int code) {
  switch (code) {
    case RT_OK: return "ok";
    case RT_EINVAL: return "invalid argument";
    case RT_ENOMEM: return "out of device memory";
    case RT_EHIP: return "HIP runtime error";
    case RT_ENONFINITE: return "non-finite values";
    case RT_ESTATE: return "mesh not prepared for this call";
  }
  return "unknown error";
}

const char *rt_last_error(void) { return g_last_error.c_str(); }

int rt_version(void) { return RTMM_VERSION; }

int rt_angles_layout(int32_t K, const double *dir, const double *weight, int32_t *layout) {
  if (!dir || !weight || !layout) return fail(RT_EINVAL, "NULL argument");
  if (K < 1 || K > RT_K_MAX) return fail(RT_EINVAL, "K=%d outside [1, %d]", K, RT_K_MAX);
  *layout = RT_ANGLES_GENERAL;
  if (K % 2) return RT_OK;
  // is angle b(k) the exact antipode of angle a(k), with its weight, for every k < K/2?
  auto pairs = [&](auto a, auto b) {
    for (int k = 0; k < K / 2; ++k) {
      if (weight[b(k)] != weight[a(k)]) return false;
      for (int c = 0; c < 3; ++c)
        if (dir[3 * b(k) + c] != -dir[3 * a(k) + c]) return false;
    }
    return true;
  };
  if (pairs([](int k) { return k; }, [K](int k) { return k + K / 2; }))
    *layout = RT_ANGLES_ANTIPODAL;
  else if (pairs([](int k) { return 2 * k; }, [](int k) { return 2 * k + 1; }))
    *layout = RT_ANGLES_ANTIPODAL_ADJACENT;
  return RT_OK;
}

int rt_angles_check(const rt_angles *a, void *stream) {
  if (!a) return fail(RT_EINVAL, "angles is NULL");
  if (a->K < 1 || a->K > RT_K_MAX) return fail(RT_EINVAL, "K=%d outside [1, %d]", a->K, RT_K_MAX);
  if (!a->dir || !a->weight) return fail(RT_EINVAL, "angle arrays are NULL");
  if (a->layout != RT_ANGLES_GENERAL && a->layout != RT_ANGLES_ANTIPODAL && a->layout != RT_ANGLES_ANTIPODAL_ADJACENT)
    return fail(RT_EINVAL, "unknown angle layout %d", a->layout);
  hipStream_t st = (hipStream_t)stream;
  std::vector<double> d(3 * (size_t)a->K), w((size_t)a->K);
  RT_HIP(hipMemcpyAsync(d.data(), a->dir, sizeof(double) * d.size(), hipMemcpyDeviceToHost, st), "copy directions");
  RT_HIP(hipMemcpyAsync(w.data(), a->weight, sizeof(double) * w.size(), hipMemcpyDeviceToHost, st), "copy weights");
  RT_HIP(hipStreamSynchronize(st), "angle copy");
  // the discrete ordinates of section 2.1: unit directions, non-negative weights summing to one
  double wsum = 0.0;
  for (int k = 0; k < a->K; ++k) {
    const double *n = &d[3 * (size_t)k];
    const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    if (!(fabs(nn - 1.0) < 1e-10)) return fail(RT_EINVAL, "direction %d is not a unit vector", k);
    if (!(w[k] >= 0.0) || !isfinite(w[k])) return fail(RT_EINVAL, "weight %d is negative or not finite", k);
    wsum += w[k];
  }
  if (!(fabs(wsum - 1.0) <= 1e-10)) return fail(RT_EINVAL, "the weights sum to %.17g, not one", wsum);
  if (a->layout == RT_ANGLES_GENERAL) return RT_OK;  // the general kernels hold for any such set
  int32_t found = RT_ANGLES_GENERAL;
  int rc = rt_angles_layout(a->K, d.data(), w.data(), &found);
  if (rc) return rc;
  if (found != a->layout)
    return fail(RT_EINVAL, "angle set claims layout %d but its arrays have layout %d", a->layout, found);
  std::lock_guard<std::mutex> lk(g_claims_mu);
  for (const checked_claim &c : g_claims)
    if (c.dir == a->dir && c.weight == a->weight && c.K == a->K && c.layout == a->layout) return RT_OK;
  g_claims.push_back(checked_claim{a->dir, a->weight, a->K, a->layout});
  return RT_OK;
}

int rt_angles_release(const rt_angles *a) {
  if (!a) return fail(RT_EINVAL, "angles is NULL");
  std::lock_guard<std::mutex> lk(g_claims_mu);
  g_claims.erase(std::remove_if(g_claims.begin(), g_claims.end(),
                                [a](const checked_claim &c) { return c.dir == a->dir && c.weight == a->weight; }),
                 g_claims.end());
  return RT_OK;
}

int rt_mesh_upload(rt_mesh **out, int64_t N, int64_t F, int32_t k_max, int32_t flags, const double *gen,
                   const double *com, const double *vol, const double *mesh_vel, const int32_t *face_cells,
                   const int8_t *face_shift, const double *face_area, const double *face_normal,
                   const double *face_centroid, double box, void *stream) {
  if (!out) return fail(RT_EINVAL, "out is NULL");
  *out = nullptr;
  if (N < 1 || F < 1) return fail(RT_EINVAL, "need n_cells >= 1 and n_faces >= 1");
  if (N >= (int64_t)1 << 31 || 2 * F >= (int64_t)1 << 31) return fail(RT_EINVAL, "mesh too large for int32 indices");
  if (k_max < 1 || k_max > RT_K_MAX) return fail(RT_EINVAL, "k_max=%d outside [1, %d]", k_max, RT_K_MAX);
  if (flags & ~(RT_MESH_PLM | RT_MESH_ADJOINT)) return fail(RT_EINVAL, "unknown flags 0x%x", flags);
  if (!gen || !com || !vol || !mesh_vel || !face_cells || !face_shift || !face_area || !face_normal ||
      !face_centroid)
    return fail(RT_EINVAL, "a mesh array is NULL");
  if (!(box > 0.0) || !isfinite(box)) return fail(RT_EINVAL, "box must be positive");
  {
    // positions, centres of mass, velocities and centroids enter the face speeds and the
    // reconstruction offsets: a non-finite entry would give non-finite intensities later
    const struct {
      const double *p;
      int64_t n;
      const char *what;
    } arrs[] = {{gen, 3 * N, "gen_pos"}, {com, 3 * N, "com"}, {mesh_vel, 3 * N, "mesh_vel"},
                {face_centroid, 3 * F, "face_centroid"}};
    for (const auto &a : arrs)
      for (int64_t k = 0; k < a.n; ++k)
        if (!isfinite(a.p[k])) return fail(RT_EINVAL, "%s has a non-finite entry (index %lld)", a.what, (long long)k);
  }
  rt_host_mesh hm;
  {
    const std::string why = rt_build_host_mesh(N, F, vol, face_cells, face_shift, face_area, face_normal, hm);
    if (!why.empty()) return fail(RT_EINVAL, "%s", why.c_str());
  }
  const int64_t H = 2 * F;
  const std::vector<int32_t> &row_ptr = hm.row_ptr;
  const std::vector<int32_t> &hf_face = hm.hf_face;

  rt_mesh *m = new rt_mesh;
  memset(m, 0, sizeof *m);
  m->hf_cap16 = hm.hf_cap16;
  m->hf_cap32 = hm.hf_cap32;
  m->hf_cap64 = hm.hf_cap64;
  const std::vector<uint8_t> &order16 = hm.order16, &order32 = hm.order32, &order64 = hm.order64;
  (void)hipGetDevice(&m->device);
  {
    // Every cell-parallel kernel that reads face records stages a workgroup's records in
    // LDS; the general layouts (16 cells per workgroup) must fit, the others fall back to them.
    int lds = 0;
    hipError_t ea = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, m->device);
    if (ea != hipSuccess || lds <= 0) {
      delete m;
      return hip_fail(ea != hipSuccess ? ea : hipErrorInvalidValue, "LDS size query");
    }
    m->lds_max = lds;
    // bytes per half-face: FP64 upwind 36, FP64 PLM stage 2 and gradient 100
    const size_t per = (flags & RT_MESH_PLM) ? 3 * sizeof(double4) + sizeof(int32_t) : sizeof(double4) + sizeof(int32_t);
    if (per * (size_t)m->hf_cap16 > (size_t)lds) {
      const int cap = m->hf_cap16;
      delete m;
      return fail(RT_EINVAL, "16 consecutive cells have %d half-faces; their face records (%zu bytes) exceed the %d bytes of LDS a workgroup may use",
                  cap, per * (size_t)cap, lds);
    }
  }
  m->N = N;
  m->F = F;
  m->H = H;
  m->k_max = k_max;
  m->flags = flags;
  m->box = box;
  hipStream_t st = (hipStream_t)stream;
  const bool plm = flags & RT_MESH_PLM;
  const int64_t nred = (N + 7) / 8 + 8;  // >= blocks of any cell-parallel kernel (>= 8 cells per block)
  m->n_red_blocks = nred;
  hipError_t e = hipSuccess;
#define RT_ALLOC(ptr, bytes)                         \
  do {                                               \
    if (e == hipSuccess) e = dmalloc(&(ptr), bytes); \
  } while (0)
  RT_ALLOC(m->vol0, sizeof(double) * N);
  RT_ALLOC(m->D, sizeof(double) * N);
  RT_ALLOC(m->wn, sizeof(double) * F);
  RT_ALLOC(m->row_ptr, sizeof(int32_t) * (N + 1));
  RT_ALLOC(m->hf_nbr, sizeof(int32_t) * H);
  RT_ALLOC(m->hf_face, sizeof(int32_t) * H);
  RT_ALLOC(m->hf_an64, sizeof(double4) * H);
  RT_ALLOC(m->hf_an32, sizeof(float4) * H);
  if (plm) {
    RT_ALLOC(m->hf_gp64, sizeof(double4) * H);
    RT_ALLOC(m->hf_rel64, sizeof(double4) * 2 * H);
    RT_ALLOC(m->hf_gp32, sizeof(float4) * H);
    RT_ALLOC(m->hf_rel32, sizeof(float4) * 2 * H);
    RT_ALLOC(m->gb64, sizeof(double4) * N);
    RT_ALLOC(m->gb32, sizeof(float4) * N);
    RT_ALLOC(m->I_half, sizeof(double) * N * k_max);
    RT_ALLOC(m->grad, sizeof(double) * 4 * N * k_max);
  }
  if (flags & RT_MESH_ADJOINT) RT_ALLOC(m->lam_star, sizeof(double) * N * k_max);
  RT_ALLOC(m->red, sizeof(double) * RT_NDIAG * nred);
  RT_ALLOC(m->red_mid, sizeof(double) * RT_NDIAG * RT_BLOCK);
  RT_ALLOC(m->wg_order16, N);
  RT_ALLOC(m->wg_order32, N);
  RT_ALLOC(m->wg_order64, N);
  // temporaries of the upload
  double *d_gen = nullptr, *d_com = nullptr, *d_w = nullptr, *d_area = nullptr, *d_nrm = nullptr, *d_cen = nullptr;
  int32_t *d_fc = nullptr;
  int8_t *d_shift = nullptr;
  RT_ALLOC(d_gen, sizeof(double) * 3 * N);
  RT_ALLOC(d_com, sizeof(double) * 3 * N);
  RT_ALLOC(d_w, sizeof(double) * 3 * N);
  RT_ALLOC(d_area, sizeof(double) * F);
  RT_ALLOC(d_nrm, sizeof(double) * 3 * F);
  RT_ALLOC(d_cen, sizeof(double) * 3 * F);
  RT_ALLOC(d_fc, sizeof(int32_t) * 2 * F);
  RT_ALLOC(d_shift, 3 * F);
#undef RT_ALLOC
  auto cleanup_tmp = [&]() {
    void *t[] = {d_gen, d_com, d_w, d_area, d_nrm, d_cen, d_fc, d_shift};
    for (void *p : t)
      if (p) (void)hipFree(p);
  };
  if (e != hipSuccess) {
    cleanup_tmp();
    free_mesh_arrays(m);
    delete m;
    return fail(RT_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
  }
  auto H2D = [&](void *dst, const void *src, size_t bytes) {
    if (e == hipSuccess) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
  };
  H2D(m->vol0, vol, sizeof(double) * N);
  H2D(m->row_ptr, row_ptr.data(), sizeof(int32_t) * (N + 1));
  H2D(m->hf_face, hf_face.data(), sizeof(int32_t) * H);
  H2D(m->wg_order16, order16.data(), N);
  H2D(m->wg_order32, order32.data(), N);
  H2D(m->wg_order64, order64.data(), N);
  H2D(d_gen, gen, sizeof(double) * 3 * N);
  H2D(d_com, com, sizeof(double) * 3 * N);
  H2D(d_w, mesh_vel, sizeof(double) * 3 * N);
  H2D(d_area, face_area, sizeof(double) * F);
  H2D(d_nrm, face_normal, sizeof(double) * 3 * F);
  H2D(d_cen, face_centroid, sizeof(double) * 3 * F);
  H2D(d_fc, face_cells, sizeof(int32_t) * 2 * F);
  H2D(d_shift, face_shift, 3 * F);
  if (e == hipSuccess) e = rt_launch_face_speed(d_gen, d_w, d_fc, d_shift, d_nrm, d_cen, box, F, m->wn, st);
  if (e == hipSuccess) e = rt_launch_half_faces(m, d_fc, d_area, d_nrm, d_cen, d_gen, d_com, d_shift, st);
  if (e == hipSuccess && plm) e = rt_launch_gradient_base(m, d_fc, d_area, d_cen, d_gen, d_shift, st);
  if (e == hipSuccess) e = rt_launch_volume_rate(m, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  cleanup_tmp();
  if (e != hipSuccess) {
    free_mesh_arrays(m);
    delete m;
    return hip_fail(e, "mesh upload");
  }
  *out = m;
  return RT_OK;
}

int rt_mesh_free(rt_mesh *m) {
  if (!m) return RT_OK;
  (void)hipDeviceSynchronize();
  free_mesh_arrays(m);
  delete m;
  return RT_OK;
}

int rt_mesh_info(const rt_mesh *m, int64_t *n_cells, int64_t *n_faces, int64_t *n_half, int32_t *k_max,
                 int32_t *flags) {
  if (!m) return fail(RT_EINVAL, "mesh is NULL");
  if (n_cells) *n_cells = m->N;
  if (n_faces) *n_faces = m->F;
  if (n_half) *n_half = m->H;
  if (k_max) *k_max = m->k_max;
  if (flags) *flags = m->flags;
  return RT_OK;
}

int rt_mesh_geometry(const rt_mesh *m, double *face_speed, double *vol_rate, void *stream) {
  if (!m) return fail(RT_EINVAL, "mesh is NULL");
  hipStream_t st = (hipStream_t)stream;
  if (face_speed)
    RT_HIP(hipMemcpyAsync(face_speed, m->wn, sizeof(double) * m->F, hipMemcpyDeviceToDevice, st), "copy wn");
  if (vol_rate)
    RT_HIP(hipMemcpyAsync(vol_rate, m->D, sizeof(double) * m->N, hipMemcpyDeviceToDevice, st), "copy D");
  return RT_OK;
}

int rt_transport_step(rt_mesh *m, const rt_params *p, const rt_angles *a, const void *I_in, void *I_out,
                      double *vol, void *stream) {
  int rc = check_call(m, p, a);
  if (rc) return rc;
  if ((rc = check_ptrs({I_in, I_out, vol}))) return rc;
  if (overlap(I_in, I_out, elem(p->dtype) * m->N * a->K)) return fail(RT_EINVAL, "I_in and I_out overlap");
  return run_step(m, p, a, I_in, I_out, vol, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, false,
                  (hipStream_t)stream);
}

int rt_source_implicit(rt_mesh *m, const rt_params *p, const rt_angles *a, void *I, const double *rho,
                       double *mom, double *etot, const double *kP, const double *kJ, const double *ks,
                       double *T_new, void *stream) {
  int rc = check_call(m, p, a);
  if (rc) return rc;
  if ((rc = check_ptrs({I, rho, mom, etot, kP, kJ, ks}))) return rc;
  rt_step_args s = base_args(m, p, a);
  s.I_in = I;
  s.I_out = I;
  s.rho = rho;
  s.mom = mom;
  s.etot = etot;
  s.kP = kP;
  s.kJ = kJ;
  s.ks = ks;
  s.T_out = T_new;
  s.do_transport = 0;
  s.do_source = 1;
  s.write_gas = 1;
  hipError_t e = rt_launch_step(s, p->dtype, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "source kernel launch");
  return RT_OK;
}

int rt_step(rt_mesh *m, const rt_params *p, const rt_angles *a, const void *I_in, void *I_out, double *vol,
            const double *rho, double *mom, double *etot, const double *kP, const double *kJ, const double *ks,
            double *T_new, void *stream) {
  int rc = check_call(m, p, a);
  if (rc) return rc;
  if ((rc = check_ptrs({I_in, I_out, vol, rho, mom, etot, kP, kJ, ks}))) return rc;
  if (overlap(I_in, I_out, elem(p->dtype) * m->N * a->K)) return fail(RT_EINVAL, "I_in and I_out overlap");
  return run_step(m, p, a, I_in, I_out, vol, rho, mom, etot, kP, kJ, ks, T_new, true, (hipStream_t)stream);
}

int rt_step_taped(rt_mesh *m, const rt_params *p, const rt_angles *a, const void *I_in, void *I_out, void *I_star,
                  double *vol, const double *rho, double *mom, double *etot, const double *kP, const double *kJ,
                  const double *ks, double *T_new, double *src_tape, void *stream) {
  int rc = check_call(m, p, a);
  if (rc) return rc;
  if ((rc = check_ptrs({I_in, I_out, vol, rho, mom, etot, kP, kJ, ks}))) return rc;
  if (p->scheme != RT_UPWIND1) return fail(RT_EINVAL, "rt_step_taped covers RT_UPWIND1 steps only");
  if (!I_star && !src_tape) return fail(RT_EINVAL, "rt_step_taped needs I_star or src_tape");
  if (I_star && !aligned8(I_star)) return fail(RT_EINVAL, "I_star is not 8-byte aligned");
  if (src_tape && !aligned8(src_tape)) return fail(RT_EINVAL, "src_tape is not 8-byte aligned");
  const size_t bytes = elem(p->dtype) * m->N * a->K;
  if (overlap(I_in, I_out, bytes) || (I_star && (overlap(I_in, I_star, bytes) || overlap(I_out, I_star, bytes))))
    return fail(RT_EINVAL, "I_in, I_out and I_star must not overlap");
  return run_step(m, p, a, I_in, I_out, vol, rho, mom, etot, kP, kJ, ks, T_new, true, (hipStream_t)stream, I_star,
                  src_tape);
}

int rt_gradient(rt_mesh *m, const rt_params *p, const rt_angles *a, const void *I, void *grad, void *stream) {
  int rc = check_call(m, p, a);
  if (rc) return rc;
  if ((rc = check_ptrs({I, grad}))) return rc;
  if (!(m->flags & RT_MESH_PLM)) return fail(RT_ESTATE, "rt_gradient needs a mesh uploaded with RT_MESH_PLM");
  hipError_t e = rt_launch_gradient(m, a->K, I, grad, p->dtype, false, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "gradient kernel launch");
  return RT_OK;
}

int rt_step_adjoint(rt_mesh *m, const rt_params *p, const rt_angles *a, const void *I_star, const double *vol_n,
                    const double *rho, const double *mom_n, const double *etot_n, const double *kP,
                    const double *kJ, const double *ks, void *lamI, double *lamE, double *lamM, double *dkP,
                    double *dkJ, void *stream) {
  int rc = check_call(m, p, a);
  if (rc) return rc;
  if ((rc = check_ptrs({I_star, vol_n, rho, mom_n, etot_n, kP, kJ, ks, lamI, lamE, lamM}))) return rc;
  if (p->scheme != RT_UPWIND1) return fail(RT_EINVAL, "the adjoint covers RT_UPWIND1 steps only");
  if (!(m->flags & RT_MESH_ADJOINT)) return fail(RT_ESTATE, "rt_step_adjoint needs RT_MESH_ADJOINT");
  rt_adj_args s;
  memset(&s, 0, sizeof s);
  s.N = m->N;
  s.K = a->K;
  s.row_ptr = m->row_ptr;
  s.hf_nbr = m->hf_nbr;
  s.hf_an = p->dtype == RT_F32 ? (const void *)m->hf_an32 : (const void *)m->hf_an64;
  s.D = m->D;
  s.dirs = a->dir;
  s.W = a->weight;
  s.I_star = I_star;
  s.vol_n = vol_n;
  s.rho = rho;
  s.mom = mom_n;
  s.etot = etot_n;
  s.kP = kP;
  s.kJ = kJ;
  s.ks = ks;
  s.lamI = lamI;
  s.lam_star = m->lam_star;
  s.lamE = lamE;
  s.lamM = lamM;
  s.dkP = dkP;
  s.dkJ = dkJ;
  s.c_red = p->c_red;
  s.c_light = p->c_light;
  s.a_rad = p->a_rad;
  s.cv = p->cv;
  s.dt = p->dt;
  hipError_t e = rt_launch_adjoint(s, p->dtype, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "adjoint kernel launch");
  // transpose of the upwind transport: lam*/V' (written by the source adjoint) in, lam out
  rt_step_args t = base_args(m, p, a);
  t.I_in = m->lam_star;
  t.I_out = lamI;
  t.vol_in = vol_n;
  t.vol_out = nullptr;
  t.do_transport = 3;
  t.do_source = 0;
  t.write_gas = 0;
  e = rt_launch_step(t, p->dtype, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "adjoint transport kernel launch");
  return RT_OK;
}

int rt_step_adjoint_run(rt_mesh *m, const rt_params *p, const rt_angles *a, int32_t n_steps,
                        const void *const *I_next, const double *const *src_tape, const double *rho,
                        const double *kP, const double *kJ, const double *ks, void *lamI, double *lamE,
                        double *lamM, double *dkP, double *dkJ, void *stream) {
  int rc = check_call(m, p, a);
  if (rc) return rc;
  if (n_steps < 0) return fail(RT_EINVAL, "n_steps < 0");
  if (n_steps == 0) return RT_OK;
  if ((rc = check_ptrs({rho, kP, kJ, ks, lamI, lamE, lamM}))) return rc;
  if (!I_next || !src_tape) return fail(RT_EINVAL, "a per-step pointer array is NULL");
  for (int32_t i = 0; i < n_steps; ++i) {
    if ((rc = check_ptrs({I_next[i], src_tape[i]}))) return rc;
    if (!aligned8(src_tape[i])) return fail(RT_EINVAL, "src_tape[%d] is not 8-byte aligned", i);
  }
  if (p->scheme != RT_UPWIND1) return fail(RT_EINVAL, "the adjoint covers RT_UPWIND1 steps only");
  if (!(m->flags & RT_MESH_ADJOINT)) return fail(RT_ESTATE, "rt_step_adjoint_run needs RT_MESH_ADJOINT");
  const size_t bytes = elem(p->dtype) * m->N * a->K;
  for (int32_t i = 0; i < n_steps; ++i)
    if (overlap(I_next[i], lamI, bytes) || overlap(I_next[i], m->lam_star, bytes))
      return fail(RT_EINVAL, "I_next[%d] overlaps lamI or the mesh's adjoint buffer", i);
  const hipStream_t st = (hipStream_t)stream;
  // The reverse chain alternates between lamI and the mesh's adjoint buffer: every launch
  // after the first gathers its neighbours' rows from the previous launch's output, so it
  // writes the other buffer.  The first launch (per cell, in place allowed) picks its
  // buffer so that the last one, the transpose of step 0, writes lamI.
  void *buf[2] = {lamI, m->lam_star};
  int out = n_steps % 2;  // the buffer the first launch writes (lamI in place when 0)
  rt_step_args s = base_args(m, p, a);
  s.rho = rho;
  s.kP = kP;
  s.kJ = kJ;
  s.ks = ks;
  s.lamE = lamE;
  s.lamM = lamM;
  s.dkP = dkP;
  s.dkJ = dkJ;
  s.do_source = 0;
  s.write_gas = 0;
  for (int32_t n = n_steps - 1; n >= 0; --n) {
    // n = n_steps - 1: the source reverse of the last step; below it, the transpose of step
    // n + 1 fused with the source reverse of step n
    const bool first = n == n_steps - 1;
    rt_step_args t = s;
    t.I_in = first ? lamI : buf[out];
    if (!first) out = 1 - out;
    t.I_out = buf[out];
    t.I_next = I_next[n];
    t.src_tape = src_tape[n];
    t.do_transport = first ? 5 : 4;
    hipError_t e = rt_launch_step(t, p->dtype, st);
    if (e != hipSuccess) return hip_fail(e, first ? "source reverse launch" : "fused adjoint launch");
  }
  // the transpose of step 0 (start-of-step volume V^0, from its tape) into lamI
  rt_step_args t = s;
  t.I_in = buf[out];
  t.I_out = lamI;
  t.src_tape = src_tape[0];
  t.do_transport = 3;
  hipError_t e = rt_launch_step(t, p->dtype, st);
  if (e != hipSuccess) return hip_fail(e, "adjoint transport kernel launch");
  return RT_OK;
}

int rt_flux_loss(rt_mesh *m, const rt_params *p, const rt_angles *a, const void *I, const double *face_weight,
                 double *loss, void *seed, void *stream) {
  int rc = check_call(m, p, a);
  if (rc) return rc;
  if ((rc = check_ptrs({I, face_weight, loss}))) return rc;
  if (seed && !aligned8(seed)) return fail(RT_EINVAL, "seed is not 8-byte aligned");
  hipError_t e = rt_launch_flux_loss(m, a->K, a->dir, a->weight, p->c_light, I, face_weight, loss, seed, p->dtype,
                                     (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "loss kernel launch");
  return RT_OK;
}

int rt_flux_loss_noalloc(rt_mesh *m, const rt_params *p, const rt_angles *a, const void *I,
                         const double *face_weight, double *loss, void *seed, void *stream) {
  int rc = check_call(m, p, a);
  if (rc) return rc;
  if ((rc = check_ptrs({I, face_weight, loss}))) return rc;
  if (seed && !aligned8(seed)) return fail(RT_EINVAL, "seed is not 8-byte aligned");
  int dev = -1;
  RT_HIP(hipGetDevice(&dev), "current device");
  if (dev != m->device) return fail(RT_EINVAL, "the mesh lives on device %d but device %d is current", m->device, dev);
  const int64_t nblk = rt_loss_blocks(m->N, a->K);
  if (nblk > RT_NOALLOC_PARTIALS)
    return fail(RT_EINVAL, "%lld cells at K=%d need %lld partial sums; the static scratch holds %d",
                (long long)m->N, a->K, (long long)nblk, RT_NOALLOC_PARTIALS);
  hipError_t e = rt_launch_flux_loss_noalloc(m, a->K, a->dir, a->weight, p->c_light, I, face_weight, loss, seed,
                                             p->dtype, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "loss kernel launch (static scratch)");
  return RT_OK;
}

int rt_source_implicit_mg(rt_mesh *m, const rt_params *p, const rt_angles *a, int32_t G, const double *group_weight,
                          void *I, const double *rho, double *mom, double *etot, const double *kP, const double *kJ,
                          const double *ks, double *T_new, void *stream) {
  int rc = check_call(m, p, a);
  if (rc) return rc;
  if (G < 1 || G > RT_G_MAX) return fail(RT_EINVAL, "G=%d outside [1, %d]", G, RT_G_MAX);
  if ((rc = check_ptrs({group_weight, I, rho, mom, etot, kP, kJ, ks}))) return rc;
  rt_mg_args g;
  memset(&g, 0, sizeof g);
  g.N = m->N;
  g.K = a->K;
  g.G = G;
  g.paired = rt_pair_kind(a->layout);
  g.dirs = a->dir;
  g.W = a->weight;
  g.Wg = group_weight;
  g.I = I;
  g.rho = rho;
  g.mom = mom;
  g.etot = etot;
  g.kP = kP;
  g.kJ = kJ;
  g.ks = ks;
  g.T_out = T_new;
  g.c_red = p->c_red;
  g.c_light = p->c_light;
  g.a_rad = p->a_rad;
  g.cv = p->cv;
  g.dt = p->dt;
  g.inv_c = 1.0 / p->c_light;
  g.e_gain = 4.0 * M_PI * p->c_light / p->c_red;
  g.m_gain = 4.0 * M_PI / p->c_red;
  g.a_4pi = p->a_rad / (4.0 * M_PI);
  hipError_t e = rt_launch_source_mg(g, p->dtype, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "multigroup source kernel launch");
  return RT_OK;
}

int rt_step_mg(rt_mesh *m, const rt_params *p, const rt_angles *a, int32_t G, const double *group_weight,
               const void *I_in, void *I_out, double *vol, const double *rho, double *mom, double *etot,
               const double *kP, const double *kJ, const double *ks, double *T_new, void *stream) {
  int rc = check_call(m, p, a);
  if (rc) return rc;
  if (p->scheme != RT_UPWIND1) return fail(RT_EINVAL, "multigroup steps cover RT_UPWIND1 only");
  if (G < 1 || G > RT_G_MAX) return fail(RT_EINVAL, "G=%d outside [1, %d]", G, RT_G_MAX);
  if ((rc = check_ptrs({group_weight, I_in, I_out, vol, rho, mom, etot, kP, kJ, ks}))) return rc;
  const size_t slab = elem(p->dtype) * m->N * a->K;
  if (overlap(I_in, I_out, slab * G)) return fail(RT_EINVAL, "I_in and I_out overlap");
  hipStream_t st = (hipStream_t)stream;
  // every group's slab is transported by the upwind kernel; the volume advances once
  for (int32_t j = 0; j < G; ++j) {
    rt_step_args s = base_args(m, p, a);
    s.I_in = (const char *)I_in + slab * j;
    s.I_out = (char *)I_out + slab * j;
    s.vol_in = vol;
    s.vol_out = j == G - 1 ? vol : nullptr;
    s.do_transport = 1;
    s.do_source = 0;
    s.write_gas = 0;
    hipError_t e = rt_launch_step(s, p->dtype, st);
    if (e != hipSuccess) return hip_fail(e, "multigroup transport kernel launch");
  }
  return rt_source_implicit_mg(m, p, a, G, group_weight, I_out, rho, mom, etot, kP, kJ, ks, T_new, stream);
}

int rt_source_implicit_kT(rt_mesh *m, const rt_params *p, const rt_angles *a, void *I, const double *rho,
                          double *mom, double *etot, const double *kP0, const double *kJ0, const double *ks,
                          double T_ref, double bP, double bJ, double *T_new, void *stream) {
  int rc = check_call(m, p, a);
  if (rc) return rc;
  if (!(T_ref > 0.0) || !std::isfinite(T_ref)) return fail(RT_EINVAL, "T_ref=%g must be positive and finite", T_ref);
  if (!(fabs(bP) <= 20.0) || !(fabs(bJ) <= 20.0))
    return fail(RT_EINVAL, "opacity exponents (%g, %g) outside [-20, 20]", bP, bJ);
  if ((rc = check_ptrs({I, rho, mom, etot, kP0, kJ0, ks}))) return rc;
  rt_kT_args g;
  memset(&g, 0, sizeof g);
  g.N = m->N;
  g.K = a->K;
  g.dirs = a->dir;
  g.W = a->weight;
  g.I = I;
  g.rho = rho;
  g.mom = mom;
  g.etot = etot;
  g.kP0 = kP0;
  g.kJ0 = kJ0;
  g.ks = ks;
  g.T_out = T_new;
  g.T_ref = T_ref;
  g.bP = bP;
  g.bJ = bJ;
  g.c_red = p->c_red;
  g.c_light = p->c_light;
  g.a_rad = p->a_rad;
  g.cv = p->cv;
  g.dt = p->dt;
  g.e_gain = 4.0 * M_PI * p->c_light / p->c_red;
  g.m_gain = 4.0 * M_PI / p->c_red;
  g.paired = rt_pair_kind(a->layout);
  hipError_t e = rt_launch_source_kT(g, p->dtype, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "temperature-dependent-opacity source kernel launch");
  return RT_OK;
}

int rt_step_kT(rt_mesh *m, const rt_params *p, const rt_angles *a, const void *I_in, void *I_out, double *vol,
               const double *rho, double *mom, double *etot, const double *kP0, const double *kJ0, const double *ks,
               double T_ref, double bP, double bJ, double *T_new, void *stream) {
  int rc = check_call(m, p, a);
  if (rc) return rc;
  if (p->scheme != RT_UPWIND1) return fail(RT_EINVAL, "steps with T-dependent opacities cover RT_UPWIND1 only");
  if ((rc = check_ptrs({I_in, I_out, vol}))) return rc;
  if (overlap(I_in, I_out, elem(p->dtype) * m->N * a->K)) return fail(RT_EINVAL, "I_in and I_out overlap");
  if ((rc = run_step(m, p, a, I_in, I_out, vol, rho, mom, etot, kP0, kJ0, ks, nullptr, false, (hipStream_t)stream)))
    return rc;
  return rt_source_implicit_kT(m, p, a, I_out, rho, mom, etot, kP0, kJ0, ks, T_ref, bP, bJ, T_new, stream);
}

int rt_marked_free(rt_marked *set) {
  if (!set) return RT_OK;
  (void)hipDeviceSynchronize();
  void *ptrs[] = {set->cell, set->kind, set->T_eff, set->dir, set->cos_open};
  for (void *q : ptrs)
    if (q) (void)hipFree(q);
  delete set;
  return RT_OK;
}

int rt_marked_upload(rt_marked **out, int64_t n_cells, int64_t n, const int32_t *cell, const int32_t *kind,
                     const double *T_eff, const double *dir, const double *cos_open, double tau, void *stream) {
  if (!out) return fail(RT_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_cells <= 0) return fail(RT_EINVAL, "n_cells=%lld must be positive", (long long)n_cells);
  if (n < 0 || n > n_cells) return fail(RT_EINVAL, "n=%lld outside [0, n_cells]", (long long)n);
  if (n > 0 && (!cell || !kind || !T_eff || !dir || !cos_open)) return fail(RT_EINVAL, "a marked-cell array is NULL");
  if (!(tau > 0.0) || !std::isfinite(tau)) return fail(RT_EINVAL, "tau=%g must be positive and finite", tau);
  std::vector<uint8_t> seen((size_t)n_cells, 0);
  for (int64_t m = 0; m < n; ++m) {
    const int64_t c = cell[m];
    if (c < 0 || c >= n_cells) return fail(RT_EINVAL, "entry %lld: cell %lld out of range", (long long)m, (long long)c);
    if (seen[(size_t)c]) return fail(RT_EINVAL, "entry %lld: cell %lld marked twice", (long long)m, (long long)c);
    seen[(size_t)c] = 1;
    if (kind[m] != RT_CELL_BOUNDARY && kind[m] != RT_CELL_EMITTER)
      return fail(RT_EINVAL, "entry %lld: kind %d is neither boundary nor emitter", (long long)m, kind[m]);
    if (!(T_eff[m] >= 0.0) || !std::isfinite(T_eff[m]))
      return fail(RT_EINVAL, "entry %lld: T_eff=%g must be finite and >= 0", (long long)m, T_eff[m]);
    const double *d = dir + 3 * m;
    const double nn = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (!(fabs(nn - 1.0) <= 1e-12)) return fail(RT_EINVAL, "entry %lld: dir is not a unit vector", (long long)m);
    if (std::isnan(cos_open[m])) return fail(RT_EINVAL, "entry %lld: cos_open is NaN", (long long)m);
  }
  rt_marked *set = new rt_marked;
  memset(set, 0, sizeof *set);
  set->n_cells = n_cells;
  set->n = n;
  set->tau = tau;
  hipError_t e = hipSuccess;
  if (n > 0) {
    if (e == hipSuccess) e = dmalloc(&set->cell, sizeof(int32_t) * n);
    if (e == hipSuccess) e = dmalloc(&set->kind, sizeof(int32_t) * n);
    if (e == hipSuccess) e = dmalloc(&set->T_eff, sizeof(double) * n);
    if (e == hipSuccess) e = dmalloc(&set->dir, sizeof(double) * 3 * n);
    if (e == hipSuccess) e = dmalloc(&set->cos_open, sizeof(double) * n);
    if (e != hipSuccess) {
      rt_marked_free(set);
      return fail(RT_ENOMEM, "device allocation of %lld marked cells failed", (long long)n);
    }
    hipStream_t st = (hipStream_t)stream;
    const struct {
      void *dst;
      const void *src;
      size_t bytes;
    } cp[] = {{set->cell, cell, sizeof(int32_t) * n},   {set->kind, kind, sizeof(int32_t) * n},
              {set->T_eff, T_eff, sizeof(double) * n}, {set->dir, dir, sizeof(double) * 3 * n},
              {set->cos_open, cos_open, sizeof(double) * n}};
    for (const auto &c : cp)
      if (e == hipSuccess) e = hipMemcpyAsync(c.dst, c.src, c.bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      rt_marked_free(set);
      return hip_fail(e, "marked-cell upload");
    }
  }
  *out = set;
  return RT_OK;
}

int rt_marked_apply(rt_mesh *m, const rt_params *p, const rt_angles *a, const rt_marked *set, void *I,
                    const double *rho, double *mom, double *etot, const double *kP, void *stream) {
  int rc = check_call(m, p, a);
  if (rc) return rc;
  if (!set) return fail(RT_EINVAL, "marked-cell set is NULL");
  if (set->n_cells != m->N)
    return fail(RT_EINVAL, "marked cells were uploaded for %lld cells, the mesh has %lld", (long long)set->n_cells,
                (long long)m->N);
  if ((rc = check_ptrs({I, rho, mom, etot, kP}))) return rc;
  rt_marked_args g;
  memset(&g, 0, sizeof g);
  g.n = set->n;
  g.K = a->K;
  g.cell = set->cell;
  g.kind = set->kind;
  g.T_eff = set->T_eff;
  g.dir = set->dir;
  g.cos_open = set->cos_open;
  g.dirs = a->dir;
  g.W = a->weight;
  g.I = I;
  g.rho = rho;
  g.mom = mom;
  g.etot = etot;
  g.kP = kP;
  g.f = p->dt / set->tau < 1.0 ? p->dt / set->tau : 1.0;
  g.dt = p->dt;
  g.a_rad = p->a_rad;
  g.c_red = p->c_red;
  g.c_light = p->c_light;
  hipError_t e = rt_launch_marked(g, p->dtype, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "marked-cell kernel launch");
  return RT_OK;
}

int rt_moments(rt_mesh *m, const rt_params *p, const rt_angles *a, const void *I, double *moments, void *stream) {
  int rc = check_call(m, p, a);
  if (rc) return rc;
  if ((rc = check_ptrs({I, moments}))) return rc;
  {
    const char *i0 = (const char *)I, *i1 = i0 + elem(p->dtype) * (size_t)m->N * (size_t)a->K;
    const char *o0 = (const char *)moments, *o1 = o0 + sizeof(double) * 10 * (size_t)m->N;
    if (i0 < o1 && o0 < i1) return fail(RT_EINVAL, "I and moments overlap");
  }
  hipError_t e = rt_launch_moments(m, a->K, a->dir, a->weight, p->c_light, I, moments, p->dtype,
                                   rt_pair_kind(a->layout), (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "moments kernel launch");
  return RT_OK;
}

int rt_diagnostics(rt_mesh *m, const rt_params *p, const rt_angles *a, const void *I, const double *vol,
                   const double *etot, const double *mom, double *out, void *stream) {
  int rc = check_call(m, p, a);
  if (rc) return rc;
  if ((rc = check_ptrs({I, vol, etot, mom}))) return rc;
  if (!out) return fail(RT_EINVAL, "out is NULL");
  hipStream_t st = (hipStream_t)stream;
  double *dout = m->red + (m->n_red_blocks - 1) * RT_NDIAG;  // last row of the partials, unused by the kernels
  hipError_t e = rt_launch_diagnostics(m, a->K, a->dir, a->weight, p->c_red, p->c_light, I, vol, etot, mom, dout,
                                       p->dtype, st);
  if (e != hipSuccess) return hip_fail(e, "diagnostics kernel launch");
  RT_HIP(hipMemcpyAsync(out, dout, sizeof(double) * RT_NDIAG, hipMemcpyDeviceToHost, st), "copy diagnostics");
  RT_HIP(hipStreamSynchronize(st), "synchronise diagnostics");
  if (out[9] != 0.0) return fail(RT_ENONFINITE, "%g non-finite values", out[9]);
  return RT_OK;
}

}  // extern "C"

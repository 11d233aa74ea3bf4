/*
 * sanitize_driver.c -- TEST INFRASTRUCTURE: drives the FP64 oracle (oracle/rt_oracle.c,
 * built real and complex) and the input mesh builder (inputs/voronoi.c) through every
 * exported routine on a small jittered periodic mesh, so that a build with
 * -fsanitize=address,undefined reports any out-of-bounds access, leak or undefined
 * behaviour.  It also checks a few invariants on the way (volumes tile the box, charges
 * are conserved by transport, the source conserves energy per cell), and exits non-zero
 * on any failure.  Nothing here is product code.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#undef I

#define DRV_PI 3.14159265358979323846

typedef struct {
  int64_t n_cells, n_faces;
  const double *gen, *com, *vol, *mesh_vel;
  const int32_t *face_cells;
  const int8_t *face_shift;
  const double *face_area, *face_normal, *face_centroid;
  double box;
} or_mesh;

int vor_count(int n, double L, double jitter, const double *gen, const int32_t *cell_lat, const int32_t *lat_cell,
              int mode, int64_t *face_count, double *vol, double *com, int64_t *bad_cell);
int vor_faces(int n, double L, double jitter, const double *gen, const int32_t *cell_lat, const int32_t *lat_cell,
              int mode, const int64_t *face_off, int32_t *fcells, int8_t *fshift, double *farea, double *fnormal,
              double *fcent);
void or_face_speed(const or_mesh *m, double *wn);
void or_volume_rate(const or_mesh *m, const double *wn, double *D);
void or_advance_volume(int64_t N, const double *D, double dt, const double *vol_in, double *vol_out);
void or_transport_upwind(const or_mesh *m, const double *wn, int K, const double *dirs, double c_red, double dt,
                         const double *I_in, const double *vol_in, const double *vol_out, double *I_out);
void or_gradient_limited(const or_mesh *m, int K, const double *I, double *grad);
void or_transport_plm(const or_mesh *m, const double *wn, int K, const double *dirs, double c_red, double dt,
                      const double *I_base, const double *I_half, const double *grad, const double *vol_in,
                      const double *vol_out, double *I_out);
void or_source(int64_t N, int K, const double *dirs, const double *W, double c_red, double c_light, double a_rad,
               double cv, double dt, double *I, const double *rho, double *mom, double *etot, const double *kP,
               const double *kJ, const double *ks, double *T_out);
void or_source_cs(int64_t N, int K, const double *dirs, const double *W, double c_red, double c_light, double a_rad,
                  double cv, double dt, double _Complex *I, const double *rho, double _Complex *mom,
                  double _Complex *etot, const double _Complex *kP, const double _Complex *kJ, const double *ks,
                  double _Complex *T_out);
void or_transport_upwind_cs(const or_mesh *m, const double *wn, int K, const double *dirs, double c_red, double dt,
                            const double _Complex *I_in, const double *vol_in, const double *vol_out,
                            double _Complex *I_out);
void or_flux_loss(const or_mesh *m, int K, const double *dirs, const double *W, double c_light, const double *I,
                  const double *face_weight, double *seed, double *L_out);
void or_moments(int64_t N, int K, const double *dirs, const double *W, double c_light, const double *I, double *out);
void or_diagnostics(int64_t N, int K, const double *dirs, const double *W, double c_red, double c_light,
                    const double *I, const double *vol, const double *etot, const double *mom, double *out);
void or_transport_upwind_vjp(const or_mesh *m, const double *wn, int K, const double *dirs, double c_red, double dt,
                             const double *vol_in, const double *vol_out, const double *lam_out, double *lam_in);
void or_source_vjp(int64_t N, int K, const double *dirs, const double *W, double c_red, double c_light, double a_rad,
                   double cv, double dt, const double *I, const double *rho, const double *mom, const double *etot,
                   const double *kP, const double *kJ, const double *ks, double *lamI, double *lamE, double *lamM,
                   double *dkP, double *dkJ);
void or_marked_cells(int64_t n, const int32_t *cell, const int32_t *kind, const double *T_eff, const double *dir,
                     const double *cos_open, double tau, int K, const double *dirs, double c_red, double c_light,
                     double a_rad, double dt, double *I, const double *rho, double *mom, double *etot,
                     const double *kP);
void or_source_mg(int64_t N, int K, int G, const double *dirs, const double *W, const double *Wg, double c_red,
                  double c_light, double a_rad, double cv, double dt, double *I, const double *rho, double *mom,
                  double *etot, const double *kP, const double *kJ, const double *ks, double *T_out);
void or_source_kT(int64_t N, int K, const double *dirs, const double *W, double c_red, double c_light, double a_rad,
                  double cv, double dt, double *I, const double *rho, double *mom, double *etot, const double *kP0,
                  const double *kJ0, const double *ks, double T_ref, double bP, double bJ, double *T_out);
double or_quartic_root(double A, double B, double C);

static int failures = 0;
#define CHECK(cond, ...)                      \
  do {                                        \
    if (!(cond)) {                            \
      fprintf(stderr, "FAIL: " __VA_ARGS__);  \
      fprintf(stderr, "\n");                  \
      ++failures;                             \
    }                                         \
  } while (0)

/* deterministic uniform draws in [0, 1) (a 64-bit linear congruential generator) */
static uint64_t lcg_state = 0x9E3779B97F4A7C15ull;
static double uniform01(void) {
  lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(lcg_state >> 11) * (1.0 / 9007199254740992.0);
}

static void *xcalloc(size_t n, size_t size) {
  void *p = calloc(n, size);
  if (!p) {
    fprintf(stderr, "out of memory\n");
    exit(2);
  }
  return p;
}

int main(void) {
  const int n = 6, K = 8, G = 2;
  const double L = 1.0, jitter = 0.2, h = L / n;
  const int64_t N = (int64_t)n * n * n;
  double *gen = xcalloc(3 * N, sizeof(double));
  int32_t *lat = xcalloc(3 * N, sizeof(int32_t)), *lat_cell = xcalloc(N, sizeof(int32_t));
  for (int64_t i = 0; i < N; ++i) {
    const int a = (int)(i % n), b = (int)((i / n) % n), c = (int)(i / (n * n));
    lat[3 * i] = a; lat[3 * i + 1] = b; lat[3 * i + 2] = c;
    lat_cell[i] = (int32_t)i;
    const int s[3] = {a, b, c};
    for (int d = 0; d < 3; ++d) gen[3 * i + d] = (s[d] + 0.5 + jitter * (2.0 * uniform01() - 1.0)) * h;
  }
  int64_t *cnt = xcalloc(N, sizeof(int64_t)), *off = xcalloc(N + 1, sizeof(int64_t)), bad = -1;
  double *vol = xcalloc(N, sizeof(double)), *com = xcalloc(3 * N, sizeof(double));
  int rc = vor_count(n, L, jitter, gen, lat, lat_cell, 0, cnt, vol, com, &bad);
  CHECK(rc == 0, "vor_count returned %d (cell %lld)", rc, (long long)bad);
  for (int64_t i = 0; i < N; ++i) off[i + 1] = off[i] + cnt[i];
  const int64_t F = off[N];
  int32_t *fc = xcalloc(2 * F, sizeof(int32_t));
  int8_t *fs = xcalloc(3 * F, 1);
  double *fa = xcalloc(F, sizeof(double)), *fn = xcalloc(3 * F, sizeof(double)), *fcen = xcalloc(3 * F, sizeof(double));
  rc = vor_faces(n, L, jitter, gen, lat, lat_cell, 0, off, fc, fs, fa, fn, fcen);
  CHECK(rc == 0, "vor_faces returned %d", rc);
  double vsum = 0.0;
  for (int64_t i = 0; i < N; ++i) vsum += vol[i];
  CHECK(fabs(vsum - 1.0) < 1e-12, "volumes sum to %.17g", vsum);
  /* an invalid jitter is refused */
  CHECK(vor_count(n, L, 0.6, gen, lat, lat_cell, 0, cnt, vol, com, &bad) != 0, "jitter 0.6 accepted");

  double *w = xcalloc(3 * N, sizeof(double));
  for (int64_t i = 0; i < 3 * N; ++i) w[i] = 0.2 * (uniform01() - 0.5);
  or_mesh m = {N, F, gen, com, vol, w, fc, fs, fa, fn, fcen, L};
  double *wn = xcalloc(F, sizeof(double)), *D = xcalloc(N, sizeof(double));
  or_face_speed(&m, wn);
  or_volume_rate(&m, wn, D);

  /* one direction per octant, equal weights */
  double dirs[3 * 8], W[8];
  for (int k = 0; k < K; ++k) {
    for (int d = 0; d < 3; ++d) dirs[3 * k + d] = ((k >> d) & 1 ? -1.0 : 1.0) / sqrt(3.0);
    W[k] = 1.0 / K;
  }
  const double c_red = 10.0, c_light = 100.0, a_rad = 1.0, cv = 1.5, dt = 0.3 * h / c_red;
  double *I0 = xcalloc(N * K, sizeof(double)), *I1 = xcalloc(N * K, sizeof(double)), *I2 = xcalloc(N * K, sizeof(double));
  double *rho = xcalloc(N, sizeof(double)), *mom = xcalloc(3 * N, sizeof(double)), *etot = xcalloc(N, sizeof(double));
  double *kP = xcalloc(N, sizeof(double)), *kJ = xcalloc(N, sizeof(double)), *ks = xcalloc(N, sizeof(double));
  double *T = xcalloc(N, sizeof(double));
  for (int64_t i = 0; i < N; ++i) {
    rho[i] = 0.5 + uniform01();
    const double Tg = 0.5 + 1.5 * uniform01();
    double v2 = 0.0;
    for (int d = 0; d < 3; ++d) {
      mom[3 * i + d] = rho[i] * w[3 * i + d];
      v2 += w[3 * i + d] * w[3 * i + d];
    }
    etot[i] = rho[i] * cv * Tg + 0.5 * rho[i] * v2;
    kP[i] = kJ[i] = pow(10.0, 2.0 * uniform01() - 1.0);
    ks[i] = 0.1;
    for (int k = 0; k < K; ++k) I0[i * K + k] = Tg * Tg * Tg * Tg / (4.0 * DRV_PI) * (0.9 + 0.2 * uniform01());
  }

  /* transport: charges V I of every angle are conserved */
  double *vol1 = xcalloc(N, sizeof(double));
  or_advance_volume(N, D, dt, vol, vol1);
  or_transport_upwind(&m, wn, K, dirs, c_red, dt, I0, vol, vol1, I1);
  for (int k = 0; k < K; ++k) {
    double q0 = 0.0, q1 = 0.0;
    for (int64_t i = 0; i < N; ++i) {
      q0 += vol[i] * I0[i * K + k];
      q1 += vol1[i] * I1[i * K + k];
    }
    CHECK(fabs(q1 - q0) <= 1e-13 * fabs(q0), "angle %d charge %.17g -> %.17g", k, q0, q1);
  }
  /* PLM pieces */
  double *grad = xcalloc(3 * N * K, sizeof(double));
  or_gradient_limited(&m, K, I1, grad);
  or_transport_plm(&m, wn, K, dirs, c_red, dt, I0, I1, grad, vol, vol1, I2);
  for (int64_t i = 0; i < N * K; ++i) CHECK(isfinite(I2[i]), "PLM value %lld not finite", (long long)i);

  /* source: E_g + (4 pi c / cbar) sum W I of every cell is unchanged */
  double *Eb = xcalloc(N, sizeof(double));
  for (int64_t i = 0; i < N; ++i) {
    double e = 0.0;
    for (int k = 0; k < K; ++k) e += W[k] * I1[i * K + k];
    Eb[i] = etot[i] + 4.0 * DRV_PI * c_light / c_red * e;
  }
  double *mom1 = xcalloc(3 * N, sizeof(double)), *etot1 = xcalloc(N, sizeof(double));
  memcpy(I2, I1, sizeof(double) * N * K);
  memcpy(mom1, mom, sizeof(double) * 3 * N);
  memcpy(etot1, etot, sizeof(double) * N);
  or_source(N, K, dirs, W, c_red, c_light, a_rad, cv, dt, I2, rho, mom1, etot1, kP, kJ, ks, T);
  for (int64_t i = 0; i < N; ++i) {
    double e = 0.0;
    for (int k = 0; k < K; ++k) e += W[k] * I2[i * K + k];
    const double Ea = etot1[i] + 4.0 * DRV_PI * c_light / c_red * e;
    CHECK(fabs(Ea - Eb[i]) <= 1e-13 * fabs(Eb[i]), "cell %lld energy %.17g -> %.17g", (long long)i, Eb[i], Ea);
    CHECK(T[i] > 0.0 && isfinite(T[i]), "cell %lld temperature %g", (long long)i, T[i]);
  }
  CHECK(fabs(or_quartic_root(2.0, 3.0, 5.0) - 1.0) < 1e-15, "quartic root of 2T^4 + 3T = 5");

  /* complex builds */
  double _Complex *Ic = xcalloc(N * K, sizeof(double _Complex)), *Ic2 = xcalloc(N * K, sizeof(double _Complex));
  double _Complex *mc = xcalloc(3 * N, sizeof(double _Complex)), *ec = xcalloc(N, sizeof(double _Complex));
  double _Complex *kPc = xcalloc(N, sizeof(double _Complex)), *kJc = xcalloc(N, sizeof(double _Complex));
  double _Complex *Tc = xcalloc(N, sizeof(double _Complex));
  for (int64_t i = 0; i < N * K; ++i) Ic[i] = I1[i] + 1e-30 * _Complex_I;
  for (int64_t i = 0; i < 3 * N; ++i) mc[i] = mom[i];
  for (int64_t i = 0; i < N; ++i) {
    ec[i] = etot[i];
    kPc[i] = kP[i];
    kJc[i] = kJ[i];
  }
  or_transport_upwind_cs(&m, wn, K, dirs, c_red, dt, Ic, vol, vol1, Ic2);
  or_source_cs(N, K, dirs, W, c_red, c_light, a_rad, cv, dt, Ic, rho, mc, ec, kPc, kJc, ks, Tc);
  for (int64_t i = 0; i < N; ++i) CHECK(fabs(creal(Tc[i]) - T[i]) <= 1e-12 * T[i], "complex T of cell %lld", (long long)i);

  /* loss and seed, moments, diagnostics */
  double *u = xcalloc(F, sizeof(double)), *seed = xcalloc(N * K, sizeof(double));
  for (int64_t f = 0; f < F; f += 3) u[f] = uniform01();
  double loss = 0.0, m10[10 * 216], diag[10];
  or_flux_loss(&m, K, dirs, W, c_light, I2, u, seed, &loss);
  double dot = 0.0;
  for (int64_t i = 0; i < N * K; ++i) dot += seed[i] * I2[i];
  CHECK(fabs(dot - loss) <= 1e-12 * (fabs(loss) + 1.0), "loss %.17g vs <seed, I> %.17g", loss, dot);
  or_moments(N, K, dirs, W, c_light, I2, m10);
  or_diagnostics(N, K, dirs, W, c_red, c_light, I2, vol1, etot1, mom1, diag);
  CHECK(diag[9] == 0.0, "non-finite values counted: %g", diag[9]);

  /* reverse mode */
  double *lam = xcalloc(N * K, sizeof(double)), *lam_in = xcalloc(N * K, sizeof(double));
  double *lE = xcalloc(N, sizeof(double)), *lM = xcalloc(3 * N, sizeof(double));
  double *dkP = xcalloc(N, sizeof(double)), *dkJ = xcalloc(N, sizeof(double));
  for (int64_t i = 0; i < N * K; ++i) lam[i] = uniform01() - 0.5;
  or_source_vjp(N, K, dirs, W, c_red, c_light, a_rad, cv, dt, I1, rho, mom, etot, kP, kJ, ks, lam, lE, lM, dkP, dkJ);
  or_transport_upwind_vjp(&m, wn, K, dirs, c_red, dt, vol, vol1, lam, lam_in);

  /* boundary and emitter cells */
  int32_t mcell[3] = {0, 5, 17}, mkind[3] = {1, 2, 1};
  double mT[3] = {1.0, 2.0, 0.5}, mdir[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, mco[3] = {0.5, -0.2, 2.0};
  or_marked_cells(3, mcell, mkind, mT, mdir, mco, 2.0 * dt, K, dirs, c_red, c_light, a_rad, dt, I2, rho, mom1, etot1,
                  kP);

  /* multigroup and kappa(T) sources */
  double *Ig = xcalloc((size_t)G * N * K, sizeof(double)), Wg[2] = {0.3, 0.7};
  double *kPg = xcalloc((size_t)G * N, sizeof(double)), *kJg = xcalloc((size_t)G * N, sizeof(double));
  double *ksg = xcalloc((size_t)G * N, sizeof(double));
  for (int g = 0; g < G; ++g)
    for (int64_t i = 0; i < N; ++i) {
      kPg[g * N + i] = kP[i] * (g + 1);
      kJg[g * N + i] = kJ[i];
      ksg[g * N + i] = ks[i];
      for (int k = 0; k < K; ++k) Ig[(g * N + i) * K + k] = I1[i * K + k];
    }
  memcpy(mom1, mom, sizeof(double) * 3 * N);
  memcpy(etot1, etot, sizeof(double) * N);
  or_source_mg(N, K, G, dirs, W, Wg, c_red, c_light, a_rad, cv, dt, Ig, rho, mom1, etot1, kPg, kJg, ksg, T);
  memcpy(I2, I1, sizeof(double) * N * K);
  memcpy(mom1, mom, sizeof(double) * 3 * N);
  memcpy(etot1, etot, sizeof(double) * N);
  or_source_kT(N, K, dirs, W, c_red, c_light, a_rad, cv, dt, I2, rho, mom1, etot1, kP, kJ, ks, 1.2, -3.5, 1.0, T);
  for (int64_t i = 0; i < N; ++i) CHECK(T[i] > 0.0 && isfinite(T[i]), "kappa(T) temperature of cell %lld", (long long)i);

  free(gen); free(lat); free(lat_cell); free(cnt); free(off); free(vol); free(com); free(fc); free(fs); free(fa);
  free(fn); free(fcen); free(w); free(wn); free(D); free(I0); free(I1); free(I2); free(rho); free(mom); free(etot);
  free(kP); free(kJ); free(ks); free(T); free(vol1); free(grad); free(Eb); free(mom1); free(etot1); free(Ic);
  free(Ic2); free(mc); free(ec); free(kPc); free(kJc); free(Tc); free(u); free(seed); free(lam); free(lam_in);
  free(lE); free(lM); free(dkP); free(dkJ); free(Ig); free(kPg); free(kJg); free(ksg);
  if (failures) {
    fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  printf("sanitize driver OK: %lld cells, %lld faces\n", (long long)N, (long long)F);
  return 0;
}

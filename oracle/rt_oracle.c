/*
 * rt_oracle.c -- TEST INFRASTRUCTURE, not part of the product path.
 *
 * A plain, slow, FP64 CPU oracle of the radiation step of Chang, Davis & Jiang,
 * "Time Dependent Radiation Hydrodynamics on a Moving Mesh" (MNRAS).  Only the
 * tests, the smoke check and the benchmark's CPU-baseline leg may call it.  It
 * shares no source, header, table or helper with the HIP library.
 *
 * Every function states the passage it follows.  Readings of passages the paper
 * leaves silent or prints with errors are marked READING.
 *
 * Units (READING of the two normalisations the paper mixes, sections 2.1 and
 * 2.3): intensities are carried in energy-density units, I = I_std / c, so
 * that the equilibrium intensity is a T^4 / 4 pi as in eqs. 19, 25 and 26.
 * Then E_r = 4 pi sum_k W_k I_k and F_r = 4 pi c sum_k W_k n_k I_k, and the
 * gas updates of eqs. 35-36 become dE = (4 pi c / cbar) sum W (I - I') and
 * d(rho v) = (4 pi / cbar) sum W n (I - I').
 *
 * The file is compiled twice: once with REAL = double, once with
 * REAL = double _Complex (-DOR_COMPLEX, symbols suffixed _cs) so that tests can
 * take complex-step derivatives of exactly this forward code.  Branches and
 * min/max act on real parts only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef OR_COMPLEX
#include <complex.h>
#undef I /* the imaginary-unit macro would clash with intensity names */
typedef double _Complex REAL;
#define RE(x) creal(x)
#define SFX(name) name##_cs
#define RSQRT(x) csqrt(x)
#else
typedef double REAL;
#define RE(x) (x)
#define SFX(name) name
#define RSQRT(x) sqrt(x)
#endif

#define OR_PI 3.14159265358979323846

/* Mesh as plain arrays.  Faces are listed once with cell0 = i, cell1 = j;
 * the image of j adjacent to i is gen[j] + shift * box; normal points i -> j;
 * the face centroid is given in the frame of i. */
typedef struct {
  int64_t n_cells, n_faces;
  const double *gen;      /* [N][3] generator positions r_i */
  const double *com;      /* [N][3] centres of mass s_i */
  const double *vol;      /* [N] geometric cell volumes */
  const double *mesh_vel; /* [N][3] generator velocities w_i */
  const int32_t *face_cells;
  const int8_t *face_shift;
  const double *face_area;
  const double *face_normal;
  const double *face_centroid;
  double box;
} or_mesh;

static REAL rmin(REAL a, REAL b) { return RE(a) <= RE(b) ? a : b; }
static REAL rmax(REAL a, REAL b) { return RE(a) >= RE(b) ? a : b; }

#ifndef OR_COMPLEX
/* ------------------------------------------------------------------------------------------
 * Geometry-only steps (real arithmetic; compiled once).
 * ------------------------------------------------------------------------------------------ */

/* Image of generator j adjacent to i for face f. */
static void image_of_j(const or_mesh *m, int64_t f, double rj[3]) {
  const int32_t j = m->face_cells[2 * f + 1];
  for (int c = 0; c < 3; ++c) rj[c] = m->gen[3 * j + c] + m->face_shift[3 * f + c] * m->box;
}

/*
 * Normal speed of each face, w~_ij . n_ij, with w~_ij from eq. 9 (section 2,
 * face velocity of S10): the mean generator velocity plus the correction
 * [(w_i - w_j).(r~_ij - (r_i+r_j)/2) / |r_j - r_i|] (r_j - r_i)/|r_j - r_i|.
 * The transport step only needs its component along the face normal
 * (section 2.2 item iii, flux (cbar n - w~) I through a face of normal n_ij).
 */
void or_face_speed(const or_mesh *m, double *wn) {
#pragma omp parallel for schedule(static)
  for (int64_t f = 0; f < m->n_faces; ++f) {
    const int32_t i = m->face_cells[2 * f], j = m->face_cells[2 * f + 1];
    double rj[3];
    image_of_j(m, f, rj);
    double d[3], mid[3], dw[3], wbar[3];
    for (int c = 0; c < 3; ++c) {
      d[c] = rj[c] - m->gen[3 * i + c];
      mid[c] = 0.5 * (rj[c] + m->gen[3 * i + c]);
      dw[c] = m->mesh_vel[3 * i + c] - m->mesh_vel[3 * j + c];
      wbar[c] = 0.5 * (m->mesh_vel[3 * i + c] + m->mesh_vel[3 * j + c]);
    }
    const double dist = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double corr = 0.0;
    for (int c = 0; c < 3; ++c) corr += dw[c] * (m->face_centroid[3 * f + c] - mid[c]);
    corr /= dist;
    double wface[3];
    for (int c = 0; c < 3; ++c) wface[c] = corr * d[c] / dist + wbar[c];
    const double *n = &m->face_normal[3 * f];
    wn[f] = wface[0] * n[0] + wface[1] * n[1] + wface[2] * n[2];
  }
}

/*
 * Rate of change of each cell volume from the motion of its faces,
 * D_i = sum_faces (+-) A_f (w~.n)_f, outward normal positive.
 * READING: the paper re-tessellates each step (section 2, steps 3-5); with the
 * tessellation frozen over the radiation step (section 4, subcycling remark),
 * the cell volume is advanced as V^{n+1} = V^n + dt D_i so that the moving-face
 * term of the flux (section 2.2 item iii) keeps a uniform field uniform.
 */
void or_volume_rate(const or_mesh *m, const double *wn, double *D) {
  for (int64_t i = 0; i < m->n_cells; ++i) D[i] = 0.0;
  for (int64_t f = 0; f < m->n_faces; ++f) {
    const int32_t i = m->face_cells[2 * f], j = m->face_cells[2 * f + 1];
    const double q = m->face_area[f] * wn[f];
    D[i] += q;
    D[j] -= q;
  }
}

/* Advance volumes: V_out = V_in + dt * D. */
void or_advance_volume(int64_t N, const double *D, double dt, const double *vol_in, double *vol_out) {
  for (int64_t i = 0; i < N; ++i) vol_out[i] = vol_in[i] + dt * D[i];
}
#endif /* !OR_COMPLEX */

/* ------------------------------------------------------------------------------------------
 * Transport (section 2.2) as the finite-volume charge update of eq. 8.
 * ------------------------------------------------------------------------------------------ */

/*
 * First-order upwind transport of every angle over dt (section 2.2 items i, iii,
 * iv; eq. 8 with the charges U = V I of eq. 5).
 * Per face f (i -> j, area A) and angle k: face-frame normal speed
 * s = cbar n_k . n_f - (w~.n)_f; the upwind intensity is I_i if s > 0 else I_j;
 * the charge leaving i into j is Phi = dt A s I_up.
 * READING: eq. 8 is printed with "+ dt sum F A"; a flux along the outward
 * normal of i removes charge from i, so Phi is subtracted from i, added to j.
 * Then I_out = (V_in I_in - sum Phi) / V_out with V_out = V_in + dt D.
 * Angles never mix in transport, so the loop runs angle by angle.
 */
void SFX(or_transport_upwind)(const or_mesh *m, const double *wn, int K, const double *dirs, double c_red,
                              double dt, const REAL *I_in, const double *vol_in, const double *vol_out,
                              REAL *I_out) {
  const int64_t N = m->n_cells, F = m->n_faces;
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < K; ++k) {
    REAL *Q = (REAL *)malloc(sizeof(REAL) * (size_t)N);
    for (int64_t i = 0; i < N; ++i) Q[i] = vol_in[i] * I_in[i * K + k];
    const double *nk = &dirs[3 * k];
    for (int64_t f = 0; f < F; ++f) {
      const int32_t i = m->face_cells[2 * f], j = m->face_cells[2 * f + 1];
      const double *nf = &m->face_normal[3 * f];
      const double s = c_red * (nk[0] * nf[0] + nk[1] * nf[1] + nk[2] * nf[2]) - wn[f];
      const REAL Iup = (s > 0.0) ? I_in[(int64_t)i * K + k] : I_in[(int64_t)j * K + k];
      const REAL Phi = dt * m->face_area[f] * s * Iup;
      Q[i] -= Phi;
      Q[j] += Phi;
    }
    for (int64_t i = 0; i < N; ++i) I_out[i * K + k] = Q[i] / vol_out[i];
    free(Q);
  }
}

/*
 * Linear reconstruction for the full step (section 2.2 item ii, "same limiter
 * as Chang+17").  READING (the limiter paper is not part of this one): the
 * gradient is the Voronoi estimator of S10,
 *   grad phi_i = (1/V_i) sum_j A_ij [ (phi_j - phi_i) c_ij/|r_ij|
 *                                     - (phi_i + phi_j)/2 r_ij/|r_ij| ],
 * r_ij = r_i - r_j, c_ij = face centroid minus the midpoint of r_i and r_j,
 * with V_i the geometric volume of the frozen tessellation; the limiter is
 * Barth-Jespersen at the face centroids: alpha_i = min over faces of
 * psi_f = (max(phi) - phi_i)/delta_f if delta_f > 0, (min(phi) - phi_i)/delta_f
 * if delta_f < 0, 1 if delta_f = 0, capped at 1, where delta_f =
 * grad phi_i . (r~_f - s_i) extrapolates from the centre of mass s_i and the
 * extrema run over i and its face neighbours.  Output: limited gradient
 * alpha_i grad phi_i, layout [N][3][K].
 */
void SFX(or_gradient_limited)(const or_mesh *m, int K, const REAL *I, REAL *grad) {
  const int64_t N = m->n_cells, F = m->n_faces;
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < K; ++k) {
    REAL *g = (REAL *)malloc(sizeof(REAL) * 3 * (size_t)N);
    REAL *lo = (REAL *)malloc(sizeof(REAL) * (size_t)N);
    REAL *hi = (REAL *)malloc(sizeof(REAL) * (size_t)N);
    REAL *alpha = (REAL *)malloc(sizeof(REAL) * (size_t)N);
    for (int64_t i = 0; i < N; ++i) {
      g[3 * i] = g[3 * i + 1] = g[3 * i + 2] = 0.0;
      lo[i] = hi[i] = I[i * K + k];
      alpha[i] = 1.0;
    }
    for (int64_t f = 0; f < F; ++f) {
      const int32_t a = m->face_cells[2 * f], b = m->face_cells[2 * f + 1];
      double rb[3], rab[3], cf[3];
      for (int c = 0; c < 3; ++c) {
        rb[c] = m->gen[3 * b + c] + m->face_shift[3 * f + c] * m->box;
        rab[c] = m->gen[3 * a + c] - rb[c];
        cf[c] = m->face_centroid[3 * f + c] - 0.5 * (m->gen[3 * a + c] + rb[c]);
      }
      const double dist = sqrt(rab[0] * rab[0] + rab[1] * rab[1] + rab[2] * rab[2]);
      const double A = m->face_area[f];
      const REAL pa = I[(int64_t)a * K + k], pb = I[(int64_t)b * K + k];
      for (int c = 0; c < 3; ++c) {
        /* side a: r_ab = r_a - r_b; side b: r_ba = -r_ab; c_ij is the same vector */
        g[3 * a + c] += A * ((pb - pa) * cf[c] / dist - 0.5 * (pa + pb) * rab[c] / dist);
        g[3 * b + c] += A * ((pa - pb) * cf[c] / dist + 0.5 * (pa + pb) * rab[c] / dist);
      }
      lo[a] = rmin(lo[a], pb); hi[a] = rmax(hi[a], pb);
      lo[b] = rmin(lo[b], pa); hi[b] = rmax(hi[b], pa);
    }
    for (int64_t i = 0; i < N; ++i)
      for (int c = 0; c < 3; ++c) g[3 * i + c] /= m->vol[i];
    for (int64_t f = 0; f < F; ++f) {
      const int32_t a = m->face_cells[2 * f], b = m->face_cells[2 * f + 1];
      for (int side = 0; side < 2; ++side) {
        const int32_t i = side ? b : a;
        double rel[3];
        for (int c = 0; c < 3; ++c) {
          const double cen = m->face_centroid[3 * f + c] - (side ? m->face_shift[3 * f + c] * m->box : 0.0);
          rel[c] = cen - m->com[3 * i + c];
        }
        const REAL delta = g[3 * i] * rel[0] + g[3 * i + 1] * rel[1] + g[3 * i + 2] * rel[2];
        const REAL phi = I[(int64_t)i * K + k];
        REAL psi = 1.0;
        if (RE(delta) > 0.0) psi = (hi[i] - phi) / delta;
        else if (RE(delta) < 0.0) psi = (lo[i] - phi) / delta;
        alpha[i] = rmin(alpha[i], psi);
      }
    }
    for (int64_t i = 0; i < N; ++i)
      for (int c = 0; c < 3; ++c) grad[(i * 3 + c) * K + k] = alpha[i] * g[3 * i + c];
    free(g); free(lo); free(hi); free(alpha);
  }
}

/*
 * Full-step transport with reconstructed face states (section 2.2 item ii;
 * section 2 steps 2b and 4, the van Leer predictor-corrector): fluxes are built
 * from the half-step state I_half extrapolated from the upwind cell's centre of
 * mass to the face centroid with the limited gradient, and applied over dt to
 * the charges of the start-of-step state I_base:
 *   phi_face = I_half[c] + grad[c] . (r~_f - s_c),  c = upwind cell,
 *   I_out = (V_in I_base - sum dt A s phi_face) / V_out.
 */
void SFX(or_transport_plm)(const or_mesh *m, const double *wn, int K, const double *dirs, double c_red, double dt,
                           const REAL *I_base, const REAL *I_half, const REAL *grad, const double *vol_in,
                           const double *vol_out, REAL *I_out) {
  const int64_t N = m->n_cells, F = m->n_faces;
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < K; ++k) {
    REAL *Q = (REAL *)malloc(sizeof(REAL) * (size_t)N);
    for (int64_t i = 0; i < N; ++i) Q[i] = vol_in[i] * I_base[i * K + k];
    const double *nk = &dirs[3 * k];
    for (int64_t f = 0; f < F; ++f) {
      const int32_t a = m->face_cells[2 * f], b = m->face_cells[2 * f + 1];
      const double *nf = &m->face_normal[3 * f];
      const double s = c_red * (nk[0] * nf[0] + nk[1] * nf[1] + nk[2] * nf[2]) - wn[f];
      const int up_is_b = !(s > 0.0);
      const int32_t c = up_is_b ? b : a;
      double rel[3];
      for (int q = 0; q < 3; ++q) {
        const double cen = m->face_centroid[3 * f + q] - (up_is_b ? m->face_shift[3 * f + q] * m->box : 0.0);
        rel[q] = cen - m->com[3 * c + q];
      }
      const REAL phi = I_half[(int64_t)c * K + k] + grad[((int64_t)c * 3 + 0) * K + k] * rel[0] +
                       grad[((int64_t)c * 3 + 1) * K + k] * rel[1] + grad[((int64_t)c * 3 + 2) * K + k] * rel[2];
      const REAL Phi = dt * m->face_area[f] * s * phi;
      Q[a] -= Phi;
      Q[b] += Phi;
    }
    for (int64_t i = 0; i < N; ++i) I_out[i * K + k] = Q[i] / vol_out[i];
    free(Q);
  }
}

/* ------------------------------------------------------------------------------------------
 * Implicit source step (section 2.3), per cell, in the order of the paper's
 * four-step algorithm.
 * ------------------------------------------------------------------------------------------ */

/*
 * Unique positive root of A T^4 + B T - C = 0 (A >= 0, B, C > 0): the
 * temperature equation after eliminating J~ (section 2.3, eq. 32 with eq. 29).
 * The paper solves the quartic analytically; READING: Newton's method from
 * T0 = min((C/A)^(1/4), C/B), where f(T0) >= 0 and f is convex and increasing
 * on T > 0, so the iterates decrease monotonically to the root; stop at the
 * first iterate that does not decrease.
 */
static REAL quartic_root(REAL A, REAL B, REAL C) {
  if (RE(A) <= 0.0) return C / B;
  REAL T = rmin(RSQRT(RSQRT(C / A)), C / B);
  for (int it = 0; it < 100; ++it) {
    const REAL T3 = T * T * T;
    const REAL Tn = T - (A * T3 * T + B * T - C) / (4.0 * A * T3 + B);
    if (!(RE(Tn) < RE(T))) break;
    T = Tn;
  }
#ifdef OR_COMPLEX
  /* converge the derivative (imaginary) part as well */
  for (int it = 0; it < 3; ++it) {
    const REAL T3 = T * T * T;
    T = T - (A * T3 * T + B * T - C) / (4.0 * A * T3 + B);
  }
#endif
  return T;
}

#ifndef OR_COMPLEX
#ifdef _OPENMP
#include <omp.h>
#endif
/* Number of threads the oracle's parallel loops use. */
int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads for the OpenMP loops that follow (timing on one core, say); n >= 1. */
void or_set_num_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* The temperature root alone, exported for the tests. */
double or_quartic_root(double A, double B, double C) { return quartic_root(A, B, C); }
#endif

/*
 * Source update of one cell (section 2.3, the four-step algorithm):
 *  1. lab-frame moments E^n, F^n (eqs. 33-34, energy-density units);
 *  2. boost every angle to the comoving frame, Gamma_k = gamma (1 - v.n_k/c)
 *     (eq. 20, real c), I~_k = Gamma_k^4 I_k (eq. 23), comoving weights
 *     W~_k = N W_k / Gamma_k^2 with sum W~ = 1 (eq. 24); form the sums of
 *     eqs. 30-31 and eliminate J~ to solve eq. 32 for T^{n+1};
 *  3. per angle, I~^{n+1} from eq. 28, then I^{n+1} = I~^{n+1} / Gamma^4;
 *  4. new moments, and the gas energy and momentum changes of eqs. 35-36.
 * READINGS:
 *  - eq. 29 as printed drops rho from the numerator and puts (kJ + ks) in the
 *    denominator; summing eq. 28 with W~ gives instead
 *      J~ = (S_I + y kP S_G a T^4/4pi) / (1 - y ks S_G),  y = dt cbar rho,
 *    and eqs. 30-31 also need rho: x_k = y (kJ + ks) Gamma_k in 1 + x_k.
 *  - since sum W~ = 1, 1 - y (kJ+ks) S_G = S_1 = sum W~/(1+x); so the
 *    denominator is written D = S_1 + y kJ S_G and the T^4 coefficient
 *    A = dt c rho kP a S_1 / D, sums of positive terms only (the direct
 *    difference cancels catastrophically when x >> 1).
 *  - gas temperature T^n = (E_g - |rho v|^2 / 2 rho) / (rho cv); the updates
 *    of step 4 apply to the total gas energy E_g.
 *  - v is the gas velocity (rho v)/rho at the start of the step.
 */
static void source_cell(int K, const double *dirs, const double *W, double c_red, double c_light, double a_rad,
                        double cv, double dt, REAL *I, double rho, REAL *mom, REAL *etot, REAL kP, REAL kJ,
                        double ks, REAL *T_out, REAL *Gam, REAL *Wt, REAL *Icom) {
  const double fourpi = 4.0 * OR_PI;
  /* step 1: lab-frame moments */
  REAL E0 = 0.0, F0[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < K; ++k) {
    E0 += fourpi * W[k] * I[k];
    for (int c = 0; c < 3; ++c) F0[c] += fourpi * c_light * W[k] * dirs[3 * k + c] * I[k];
  }
  /* step 2: comoving quantities and the temperature */
  REAL v[3];
  for (int c = 0; c < 3; ++c) v[c] = mom[c] / rho;
  const REAL beta2 = (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) / (c_light * c_light);
  const REAL gam = 1.0 / RSQRT(1.0 - beta2);
  REAL norm = 0.0;
  for (int k = 0; k < K; ++k) {
    const REAL vn = v[0] * dirs[3 * k] + v[1] * dirs[3 * k + 1] + v[2] * dirs[3 * k + 2];
    Gam[k] = gam * (1.0 - vn / c_light);
    const REAL G2 = Gam[k] * Gam[k];
    Icom[k] = G2 * G2 * I[k];
    Wt[k] = W[k] / G2;
    norm += Wt[k];
  }
  for (int k = 0; k < K; ++k) Wt[k] /= norm;
  const double y = dt * c_red * rho;
  const REAL chi = kJ + ks;
  REAL S1 = 0.0, SG = 0.0, SI = 0.0;
  for (int k = 0; k < K; ++k) {
    const REAL den = 1.0 + y * chi * Gam[k];
    S1 += Wt[k] / den;
    SG += Wt[k] * Gam[k] / den;
    SI += Wt[k] * Icom[k] / den;
  }
  const REAL D = S1 + y * kJ * SG;
  REAL v2 = 0.0;
  for (int c = 0; c < 3; ++c) v2 += mom[c] * mom[c];
  const REAL Tn = (*etot - 0.5 * v2 / rho) / (rho * cv);
  const REAL Aq = dt * c_light * rho * kP * a_rad * S1 / D;
  const double Bq = rho * cv;
  const REAL Cq = rho * cv * Tn + dt * c_light * rho * fourpi * kJ * SI / D;
  const REAL T = quartic_root(Aq, Bq, Cq);
  const REAL T4 = T * T * T * T;
  const REAL planck = a_rad * T4 / fourpi;
  const REAL Jc = (SI + y * kP * SG * planck) / D;
  /* step 3: per-angle implicit update and boost back to the lab frame */
  for (int k = 0; k < K; ++k) {
    const REAL x = y * chi * Gam[k];
    const REAL Inew = (Icom[k] + y * Gam[k] * (kP * planck + ks * Jc)) / (1.0 + x);
    const REAL G2 = Gam[k] * Gam[k];
    I[k] = Inew / (G2 * G2);
  }
  /* step 4: new moments and the gas updates */
  REAL E1 = 0.0, F1[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < K; ++k) {
    E1 += fourpi * W[k] * I[k];
    for (int c = 0; c < 3; ++c) F1[c] += fourpi * c_light * W[k] * dirs[3 * k + c] * I[k];
  }
  *etot += (c_light / c_red) * (E0 - E1);
  for (int c = 0; c < 3; ++c) mom[c] += (F0[c] - F1[c]) / (c_light * c_red);
  if (T_out) *T_out = T;
}

void SFX(or_source)(int64_t N, int K, const double *dirs, const double *W, double c_red, double c_light,
                    double a_rad, double cv, double dt, REAL *I, const double *rho, REAL *mom, REAL *etot,
                    const REAL *kP, const REAL *kJ, const double *ks, REAL *T_out) {
#pragma omp parallel
  {
    REAL *Gam = (REAL *)malloc(sizeof(REAL) * (size_t)K);
    REAL *Wt = (REAL *)malloc(sizeof(REAL) * (size_t)K);
    REAL *Icom = (REAL *)malloc(sizeof(REAL) * (size_t)K);
#pragma omp for schedule(static)
    for (int64_t i = 0; i < N; ++i)
      source_cell(K, dirs, W, c_red, c_light, a_rad, cv, dt, &I[i * K], rho[i], &mom[3 * i], &etot[i], kP[i],
                  kJ[i], ks[i], T_out ? &T_out[i] : NULL, Gam, Wt, Icom);
    free(Gam); free(Wt); free(Icom);
  }
}

/*
 * Loss on the emergent flux through a set of faces: for face f with signed
 * weight u_f (orientation times a weight) the radiative flux F_r . n_f A_f with
 * F_r = 4 pi c sum_k W_k n_k I_k (section 2.1, eq. 34 in energy-density
 * units), each angle taking the intensity of its upwind cell by the sign of
 * n_k . n_f.  L = sum_f u_f A_f 4 pi c sum_k W_k (n_k . n_f) I_up.
 * When seed != NULL, dL/dI is accumulated into it; L is written to *L_out.
 */
void SFX(or_flux_loss)(const or_mesh *m, int K, const double *dirs, const double *W, double c_light,
                       const REAL *I, const double *face_weight, REAL *seed, REAL *L_out) {
  REAL L = 0.0;
  for (int64_t f = 0; f < m->n_faces; ++f) {
    const double u = face_weight[f];
    if (u == 0.0) continue;
    const int32_t a = m->face_cells[2 * f], b = m->face_cells[2 * f + 1];
    const double *nf = &m->face_normal[3 * f];
    for (int k = 0; k < K; ++k) {
      const double mu = dirs[3 * k] * nf[0] + dirs[3 * k + 1] * nf[1] + dirs[3 * k + 2] * nf[2];
      const int32_t up = (mu > 0.0) ? a : b;
      const double coef = u * m->face_area[f] * 4.0 * OR_PI * c_light * W[k] * mu;
      L += coef * I[(int64_t)up * K + k];
      if (seed) seed[(int64_t)up * K + k] += coef;
    }
  }
  *L_out = L;
}

/*
 * Angle moments per cell (section 2.1: the zeroth, first and second moments J, H, K of
 * the intensity and E_r = 4 pi J / c, F_r = 4 pi H, P_r = 4 pi K / c).  With the
 * intensities carried as I = I_std / c (energy-density units) they are
 *   E_r = 4 pi sum_k W_k I_k,  F_r = 4 pi c sum_k W_k n_k I_k,  P_r = 4 pi sum_k W_k n_k n_k I_k.
 * out[N][10] = (E_r, F_x, F_y, F_z, P_xx, P_yy, P_zz, P_xy, P_xz, P_yz).
 */
#ifndef OR_COMPLEX
void or_moments(int64_t N, int K, const double *dirs, const double *W, double c_light, const double *I,
                double *out) {
  const double fourpi = 4.0 * OR_PI;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    double m[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = 0; k < K; ++k) {
      const double wI = W[k] * I[i * K + k];
      const double *n = dirs + 3 * k;
      m[0] += wI;
      for (int c = 0; c < 3; ++c) m[1 + c] += wI * n[c];
      m[4] += wI * n[0] * n[0];
      m[5] += wI * n[1] * n[1];
      m[6] += wI * n[2] * n[2];
      m[7] += wI * n[0] * n[1];
      m[8] += wI * n[0] * n[2];
      m[9] += wI * n[1] * n[2];
    }
    out[10 * i] = fourpi * m[0];
    for (int c = 1; c < 4; ++c) out[10 * i + c] = fourpi * c_light * m[c];
    for (int c = 4; c < 10; ++c) out[10 * i + c] = fourpi * m[c];
  }
}
#endif

/*
 * Conservation diagnostics (section 2.3.1, eqs. 37-38): out[0] = sum V E_g,
 * out[1] = sum V (c/cbar) E_r, out[2..4] = sum V rho v, out[5..7] =
 * sum V F_r/(c cbar), out[8] = min I, out[9] = number of non-finite values in
 * I, E_g and rho v.
 */
#ifndef OR_COMPLEX
void or_diagnostics(int64_t N, int K, const double *dirs, const double *W, double c_red, double c_light,
                    const double *I, const double *vol, const double *etot, const double *mom, double *out) {
  const double fourpi = 4.0 * OR_PI;
  double eg = 0, er = 0, pg[3] = {0, 0, 0}, pr[3] = {0, 0, 0}, mn = INFINITY, bad = 0;
  for (int64_t i = 0; i < N; ++i) {
    double E = 0.0, Fx = 0.0, Fy = 0.0, Fz = 0.0;
    for (int k = 0; k < K; ++k) {
      const double v = I[i * K + k];
      if (!isfinite(v)) bad += 1;
      if (v < mn) mn = v;
      E += fourpi * W[k] * v;
      Fx += fourpi * c_light * W[k] * dirs[3 * k] * v;
      Fy += fourpi * c_light * W[k] * dirs[3 * k + 1] * v;
      Fz += fourpi * c_light * W[k] * dirs[3 * k + 2] * v;
    }
    if (!isfinite(etot[i])) bad += 1;
    for (int c = 0; c < 3; ++c)
      if (!isfinite(mom[3 * i + c])) bad += 1;
    eg += vol[i] * etot[i];
    er += vol[i] * (c_light / c_red) * E;
    for (int c = 0; c < 3; ++c) pg[c] += vol[i] * mom[3 * i + c];
    pr[0] += vol[i] * Fx / (c_light * c_red);
    pr[1] += vol[i] * Fy / (c_light * c_red);
    pr[2] += vol[i] * Fz / (c_light * c_red);
  }
  out[0] = eg; out[1] = er;
  for (int c = 0; c < 3; ++c) { out[2 + c] = pg[c]; out[5 + c] = pr[c]; }
  out[8] = mn; out[9] = bad;
}
#endif

#ifndef OR_COMPLEX
/* ------------------------------------------------------------------------------------------
 * Reverse mode (vector-Jacobian products) of the forward steps above, written
 * by hand.  Used to check the library's adjoint; pinned in the tests against
 * complex-step derivatives of the forward code and a transpose identity.
 * ------------------------------------------------------------------------------------------ */

/*
 * Transpose of or_transport_upwind for fixed geometry: given lam_out = dL/dI_out
 * returns lam_in = dL/dI_in.  I_out = (V_in I_in - sum Phi)/V_out is linear in
 * I_in; each Phi = dt A s I_up feeds -Phi/V_out[a] and +Phi/V_out[b].
 */
void or_transport_upwind_vjp(const or_mesh *m, const double *wn, int K, const double *dirs, double c_red,
                             double dt, const double *vol_in, const double *vol_out, const double *lam_out,
                             double *lam_in) {
  const int64_t N = m->n_cells, F = m->n_faces;
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < K; ++k) {
    double *L = (double *)malloc(sizeof(double) * (size_t)N);
    for (int64_t i = 0; i < N; ++i) L[i] = vol_in[i] / vol_out[i] * lam_out[i * K + k];
    const double *nk = &dirs[3 * k];
    for (int64_t f = 0; f < F; ++f) {
      const int32_t a = m->face_cells[2 * f], b = m->face_cells[2 * f + 1];
      const double *nf = &m->face_normal[3 * f];
      const double s = c_red * (nk[0] * nf[0] + nk[1] * nf[1] + nk[2] * nf[2]) - wn[f];
      const double dPhi = -lam_out[(int64_t)a * K + k] / vol_out[a] + lam_out[(int64_t)b * K + k] / vol_out[b];
      const int32_t up = (s > 0.0) ? a : b;
      L[up] += dt * m->face_area[f] * s * dPhi;
    }
    for (int64_t i = 0; i < N; ++i) lam_in[i * K + k] = L[i];
    free(L);
  }
}

/*
 * Reverse of source_cell.  Inputs: the source-step inputs (I = intensities
 * entering the source, gas state before it, opacities) and the adjoints of its
 * outputs (lamI for I', lamE for E_g', lamM for rho v').  On return lamI,
 * lamE, lamM hold the adjoints of the inputs, and dkP, dkJ are incremented by
 * dL/dkP, dL/dkJ of this cell.  The temperature root enters through the
 * implicit function theorem: dT = -(T^4 dA + T dB - dC) / (4 A T^3 + B).
 */
static void source_cell_vjp(int K, const double *dirs, const double *W, double c_red, double c_light,
                            double a_rad, double cv, double dt, const double *I, double rho, const double *mom,
                            double etot, double kP, double kJ, double ks, double *lamI, double *lamE, double *lamM,
                            double *dkP, double *dkJ, double *ws) {
  const double fourpi = 4.0 * OR_PI;
  double *Gam = ws, *Wt = ws + K, *Icom = ws + 2 * K, *r = ws + 3 * K, *Iout = ws + 4 * K, *q = ws + 5 * K;
  double *lGam = ws + 6 * K, *lr = ws + 7 * K, *lIcom = ws + 8 * K, *lInew = ws + 9 * K;
  /* forward recompute */
  double v[3];
  for (int c = 0; c < 3; ++c) v[c] = mom[c] / rho;
  const double beta2 = (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) / (c_light * c_light);
  const double gam = 1.0 / sqrt(1.0 - beta2);
  double Qn = 0.0;
  for (int k = 0; k < K; ++k) {
    const double vn = v[0] * dirs[3 * k] + v[1] * dirs[3 * k + 1] + v[2] * dirs[3 * k + 2];
    Gam[k] = gam * (1.0 - vn / c_light);
    const double G2 = Gam[k] * Gam[k];
    Icom[k] = G2 * G2 * I[k];
    q[k] = W[k] / G2;
    Qn += q[k];
  }
  for (int k = 0; k < K; ++k) Wt[k] = q[k] / Qn;
  const double y = dt * c_red * rho;
  const double chi = kJ + ks;
  double S1 = 0.0, SG = 0.0, SI = 0.0;
  for (int k = 0; k < K; ++k) {
    r[k] = 1.0 / (1.0 + y * chi * Gam[k]);
    S1 += Wt[k] * r[k];
    SG += Wt[k] * Gam[k] * r[k];
    SI += Wt[k] * Icom[k] * r[k];
  }
  const double D = S1 + y * kJ * SG;
  const double m2 = mom[0] * mom[0] + mom[1] * mom[1] + mom[2] * mom[2];
  const double Tn = (etot - 0.5 * m2 / rho) / (rho * cv);
  const double Aq = dt * c_light * rho * kP * a_rad * S1 / D;
  const double Bq = rho * cv;
  const double Cq = rho * cv * Tn + dt * c_light * rho * fourpi * kJ * SI / D;
  const double T = quartic_root(Aq, Bq, Cq);
  const double T3 = T * T * T, T4 = T3 * T;
  const double planck = a_rad * T4 / fourpi;
  const double Jc = (SI + y * kP * SG * planck) / D;
  const double Ssrc = kP * planck + ks * Jc;
  for (int k = 0; k < K; ++k) {
    const double G2 = Gam[k] * Gam[k];
    Iout[k] = (Icom[k] + y * Gam[k] * Ssrc) * r[k] / (G2 * G2);
  }
  /* reverse */
  const double lEp = *lamE;
  const double lmp[3] = {lamM[0], lamM[1], lamM[2]};
  double lS = 0.0;
  for (int k = 0; k < K; ++k) {
    const double G2 = Gam[k] * Gam[k];
    const double nl = dirs[3 * k] * lmp[0] + dirs[3 * k + 1] * lmp[1] + dirs[3 * k + 2] * lmp[2];
    const double through = fourpi * W[k] * ((c_light / c_red) * lEp + nl / c_red);
    const double ell = lamI[k] - through;  /* adjoint of I'_k */
    lamI[k] = through;                     /* direct part of the adjoint of I_k (step 4) */
    lInew[k] = ell / (G2 * G2);
    lGam[k] = -4.0 * ell * Iout[k] / Gam[k];
    lIcom[k] = lInew[k] * r[k];
    lS += lInew[k] * y * Gam[k] * r[k];
    lGam[k] += lInew[k] * y * Ssrc * r[k];
    lr[k] = lInew[k] * (Icom[k] + y * Gam[k] * Ssrc);
  }
  double lkP = 0.0, lkJ = 0.0, lplanck = 0.0, lJc = 0.0, lSI = 0.0, lSG = 0.0, lS1 = 0.0, lD = 0.0;
  lkP += lS * planck;
  lplanck += lS * kP;
  lJc += lS * ks;
  lSI += lJc / D;
  lkP += lJc * y * SG * planck / D;
  lSG += lJc * y * kP * planck / D;
  lplanck += lJc * y * kP * SG / D;
  lD -= lJc * Jc / D;
  const double lT = lplanck * a_rad * T3 / OR_PI;
  const double Fp = 4.0 * Aq * T3 + Bq;
  const double lA = -lT * T4 / Fp;
  const double lC = lT / Fp;
  lkP += lA * dt * c_light * rho * a_rad * S1 / D;
  lS1 += lA * dt * c_light * rho * kP * a_rad / D;
  lD -= lA * Aq / D;
  const double lTn = lC * rho * cv;
  lkJ += lC * dt * c_light * rho * fourpi * SI / D;
  lSI += lC * dt * c_light * rho * fourpi * kJ / D;
  lD -= lC * dt * c_light * rho * fourpi * kJ * SI / (D * D);
  double lE = lEp + lTn / (rho * cv);
  double lm[3];
  for (int c = 0; c < 3; ++c) lm[c] = lmp[c] - lTn * mom[c] / (rho * rho * cv);
  lS1 += lD;
  lkJ += lD * y * SG;
  lSG += lD * y * kJ;
  double lchi = 0.0, sw = 0.0;
  for (int k = 0; k < K; ++k) {
    const double lWt = lS1 * r[k] + lSG * Gam[k] * r[k] + lSI * Icom[k] * r[k];
    lr[k] += lS1 * Wt[k] + lSG * Wt[k] * Gam[k] + lSI * Wt[k] * Icom[k];
    lGam[k] += lSG * Wt[k] * r[k];
    lIcom[k] += lSI * Wt[k] * r[k];
    const double lden = -lr[k] * r[k] * r[k];
    lchi += lden * y * Gam[k];
    lGam[k] += lden * y * chi;
    q[k] = lWt; /* reuse: adjoint of Wt */
    sw += lWt * Wt[k];
  }
  lkJ += lchi;
  double lgam = 0.0, lv[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < K; ++k) {
    const double G2 = Gam[k] * Gam[k];
    const double qk = W[k] / G2;
    const double lq = (q[k] - sw) / Qn;
    lGam[k] += lq * (-2.0 * qk / Gam[k]);
    lamI[k] += lIcom[k] * G2 * G2;
    lGam[k] += lIcom[k] * 4.0 * Icom[k] / Gam[k];
    lgam += lGam[k] * Gam[k] / gam;
    for (int c = 0; c < 3; ++c) lv[c] -= lGam[k] * gam * dirs[3 * k + c] / c_light;
  }
  for (int c = 0; c < 3; ++c) lv[c] += lgam * gam * gam * gam * v[c] / (c_light * c_light);
  for (int c = 0; c < 3; ++c) lm[c] += lv[c] / rho;
  *lamE = lE;
  for (int c = 0; c < 3; ++c) lamM[c] = lm[c];
  *dkP += lkP;
  *dkJ += lkJ;
}

void or_source_vjp(int64_t N, int K, const double *dirs, const double *W, double c_red, double c_light,
                   double a_rad, double cv, double dt, const double *I, const double *rho, const double *mom,
                   const double *etot, const double *kP, const double *kJ, const double *ks, double *lamI,
                   double *lamE, double *lamM, double *dkP, double *dkJ) {
#pragma omp parallel
  {
    double *ws = (double *)malloc(sizeof(double) * 10 * (size_t)K);
#pragma omp for schedule(static)
    for (int64_t i = 0; i < N; ++i)
      source_cell_vjp(K, dirs, W, c_red, c_light, a_rad, cv, dt, &I[i * K], rho[i], &mom[3 * i], etot[i], kP[i],
                      kJ[i], ks[i], &lamI[i * K], &lamE[i], &lamM[3 * i], &dkP[i], &dkJ[i], ws);
    free(ws);
  }
}
#endif

#ifndef OR_COMPLEX
/*
 * Marked cells (sections 2.4 and 2.5), applied after a step.  Marked cell m is
 * cell[m] of kind[m] with radiation temperature T_eff[m], a unit direction dir[m]
 * and an opening cosine cos_open[m]; its directions "of interest" are the angles
 * with n_k . dir >= cos_open (READING: the paper selects the directions of a source
 * by an opening angle around a user direction).  S = a T_eff^4 / 4 pi.
 *  kind 1, boundary (section 2.4, the discretised relaxation with f = min(dt/tau, 1)):
 *    I_k <- I_k - (I_k - I0_k) f, with I0_k = S for the directions of interest and 0
 *    otherwise (an absorbing boundary when no direction is of interest);
 *    rho v <- rho v (1 - f), and the gas total energy loses the kinetic energy that
 *    goes with it (READING: the energy term the paper leaves to the reader; the
 *    density is not evolved by the radiation step, so its relaxation is not applied).
 *  kind 2, emitter (section 2.5): for the directions of interest only, the comoving
 *    emission-absorption term at T_eff, integrated implicitly over dt like eq. 28
 *    (READING: the paper gives the continuous form only):
 *      Gamma = gamma (1 - v.n/c), I~ = Gamma^4 I, x = dt Gamma cbar rho kP,
 *      I~' = (I~ + x S) / (1 + x), I' = I~' / Gamma^4;
 *    the gas is not changed (the source is external).
 * Cells are distinct; the others are untouched.
 */
void or_marked_cells(int64_t n, const int32_t *cell, const int32_t *kind, const double *T_eff, const double *dir,
                     const double *cos_open, double tau, int K, const double *dirs, double c_red, double c_light,
                     double a_rad, double dt, double *I, const double *rho, double *mom, double *etot,
                     const double *kP) {
  const double f = dt / tau < 1.0 ? dt / tau : 1.0;
  for (int64_t m = 0; m < n; ++m) {
    const int64_t i = cell[m];
    const double T2 = T_eff[m] * T_eff[m];
    const double S = a_rad * T2 * T2 / (4.0 * OR_PI);
    const double *d = dir + 3 * m;
    double *Ii = I + i * K;
    if (kind[m] == 1) {
      for (int k = 0; k < K; ++k) {
        const double nd = dirs[3 * k] * d[0] + dirs[3 * k + 1] * d[1] + dirs[3 * k + 2] * d[2];
        const double I0 = nd >= cos_open[m] ? S : 0.0;
        Ii[k] -= (Ii[k] - I0) * f;
      }
      double *p = mom + 3 * i;
      const double ke0 = 0.5 * (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]) / rho[i];
      for (int c = 0; c < 3; ++c) p[c] *= 1.0 - f;
      const double ke1 = 0.5 * (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]) / rho[i];
      etot[i] -= ke0 - ke1;
    } else if (kind[m] == 2) {
      double v[3];
      for (int c = 0; c < 3; ++c) v[c] = mom[3 * i + c] / rho[i];
      const double gam = 1.0 / sqrt(1.0 - (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) / (c_light * c_light));
      for (int k = 0; k < K; ++k) {
        const double nd = dirs[3 * k] * d[0] + dirs[3 * k + 1] * d[1] + dirs[3 * k + 2] * d[2];
        if (!(nd >= cos_open[m])) continue;
        const double vn = v[0] * dirs[3 * k] + v[1] * dirs[3 * k + 1] + v[2] * dirs[3 * k + 2];
        const double G = gam * (1.0 - vn / c_light);
        const double G2 = G * G, G4 = G2 * G2;
        const double x = dt * G * c_red * rho[i] * kP[i];
        const double Icom = (G4 * Ii[k] + x * S) / (1.0 + x);
        Ii[k] = Icom / G4;
      }
    }
  }
}
#endif

#ifndef OR_COMPLEX
/*
 * Multigroup source update (section 2.3, the implicit form generalised to
 * frequency groups): groups j = 0..G-1 with weights Wg[j], intensities
 * I[j][N][K] (group-major), opacities kP[j][N], kJ[j][N], ks[j][N].  Groups couple
 * only through (T^{n+1})^4.  Per group, as in the grey update: r_kj =
 * 1/(1 + y chi_j Gamma_k), S1_j, SG_j, SI_j, D_j = S1_j + y kJ_j SG_j and
 * J~_j = (SI_j + y kP_j SG_j a T^4/4pi) / D_j.  Summing the gas energy equation
 * over the groups with their weights gives again A T^4 + B T - C = 0 with
 *   A = dt c rho a sum_j Wg_j kP_j S1_j / D_j,
 *   C = rho cv T^n + dt c rho 4 pi sum_j Wg_j kJ_j SI_j / D_j,
 * solved as in the grey case.  The gas receives (c/cbar) sum_j Wg_j (E_j^n - E_j^{n+1})
 * and sum_j Wg_j (F_j^n - F_j^{n+1}) / (c cbar).  (READING: the emission of group j is
 * kP_j a T^4/4pi as printed, so a Planck split over groups is carried by kP_j; the
 * group weights enter the moments and the gas equation as printed.)
 */
void or_source_mg(int64_t N, int K, int G, const double *dirs, const double *W, const double *Wg, double c_red,
                  double c_light, double a_rad, double cv, double dt, double *I, const double *rho, double *mom,
                  double *etot, const double *kP, const double *kJ, const double *ks, double *T_out) {
  const double fourpi = 4.0 * OR_PI;
#pragma omp parallel
  {
    double *Gam = (double *)malloc(sizeof(double) * (size_t)K);
    double *Wt = (double *)malloc(sizeof(double) * (size_t)K);
    double *S1 = (double *)malloc(sizeof(double) * (size_t)G);
    double *SG = (double *)malloc(sizeof(double) * (size_t)G);
    double *SI = (double *)malloc(sizeof(double) * (size_t)G);
    double *D = (double *)malloc(sizeof(double) * (size_t)G);
#pragma omp for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
      double *p = mom + 3 * i;
      double v[3];
      for (int c = 0; c < 3; ++c) v[c] = p[c] / rho[i];
      const double gam = 1.0 / sqrt(1.0 - (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) / (c_light * c_light));
      double norm = 0.0;
      for (int k = 0; k < K; ++k) {
        const double vn = v[0] * dirs[3 * k] + v[1] * dirs[3 * k + 1] + v[2] * dirs[3 * k + 2];
        Gam[k] = gam * (1.0 - vn / c_light);
        Wt[k] = W[k] / (Gam[k] * Gam[k]);
        norm += Wt[k];
      }
      for (int k = 0; k < K; ++k) Wt[k] /= norm;
      const double y = dt * c_red * rho[i];
      /* lab moments before the update, and the comoving sums of every group */
      double E0 = 0.0, F0[3] = {0.0, 0.0, 0.0};
      double A = 0.0, Cs = 0.0;
      for (int j = 0; j < G; ++j) {
        const double *Ij = I + ((int64_t)j * N + i) * K;
        const double kPj = kP[(int64_t)j * N + i], kJj = kJ[(int64_t)j * N + i], ksj = ks[(int64_t)j * N + i];
        const double chi = kJj + ksj;
        S1[j] = SG[j] = SI[j] = 0.0;
        for (int k = 0; k < K; ++k) {
          E0 += Wg[j] * fourpi * W[k] * Ij[k];
          for (int c = 0; c < 3; ++c) F0[c] += Wg[j] * fourpi * c_light * W[k] * dirs[3 * k + c] * Ij[k];
          const double G2 = Gam[k] * Gam[k];
          const double den = 1.0 + y * chi * Gam[k];
          S1[j] += Wt[k] / den;
          SG[j] += Wt[k] * Gam[k] / den;
          SI[j] += Wt[k] * G2 * G2 * Ij[k] / den;
        }
        D[j] = S1[j] + y * kJj * SG[j];
        A += Wg[j] * kPj * S1[j] / D[j];
        Cs += Wg[j] * kJj * SI[j] / D[j];
      }
      const double v2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
      const double Tn = (etot[i] - 0.5 * v2 / rho[i]) / (rho[i] * cv);
      const double Aq = dt * c_light * rho[i] * a_rad * A;
      const double Bq = rho[i] * cv;
      const double Cq = rho[i] * cv * Tn + dt * c_light * rho[i] * fourpi * Cs;
      const double T = quartic_root(Aq, Bq, Cq);
      const double T4 = T * T * T * T;
      const double planck = a_rad * T4 / fourpi;
      /* per group and angle: the implicit update, boosted back; the new moments */
      double E1 = 0.0, F1[3] = {0.0, 0.0, 0.0};
      for (int j = 0; j < G; ++j) {
        double *Ij = I + ((int64_t)j * N + i) * K;
        const double kPj = kP[(int64_t)j * N + i], kJj = kJ[(int64_t)j * N + i], ksj = ks[(int64_t)j * N + i];
        const double chi = kJj + ksj;
        const double Jc = (SI[j] + y * kPj * SG[j] * planck) / D[j];
        for (int k = 0; k < K; ++k) {
          const double G2 = Gam[k] * Gam[k];
          const double Icom = G2 * G2 * Ij[k];
          const double Inew = (Icom + y * Gam[k] * (kPj * planck + ksj * Jc)) / (1.0 + y * chi * Gam[k]);
          Ij[k] = Inew / (G2 * G2);
          E1 += Wg[j] * fourpi * W[k] * Ij[k];
          for (int c = 0; c < 3; ++c) F1[c] += Wg[j] * fourpi * c_light * W[k] * dirs[3 * k + c] * Ij[k];
        }
      }
      etot[i] += (c_light / c_red) * (E0 - E1);
      for (int c = 0; c < 3; ++c) p[c] += (F0[c] - F1[c]) / (c_light * c_red);
      if (T_out) T_out[i] = T;
    }
    free(Gam); free(Wt); free(S1); free(SG); free(SI); free(D);
  }
}
#endif

#ifndef OR_COMPLEX
/*
 * Source update with temperature-dependent opacities (section 2.3: the temperature
 * equation solved by Newton-Raphson iteration).  READING: the opacities follow power
 * laws, kP(T) = kP0 (T/T_ref)^bP and kJ(T) = kJ0 (T/T_ref)^bJ, evaluated at
 * T^{n+1} (the implicit time level of eqs. 27-32); ks is constant.  With J~
 * eliminated as in the grey update the temperature equation is
 *   f(T) = rho cv (T - T^n) + dt c rho [kP a T^4 S1 - 4 pi kJ SI] / D = 0,
 * where S1, SG, SI and D = S1 + y kJ SG depend on T through chi = kJ(T) + ks
 * (r_k = 1/(1 + y chi Gamma_k)); f' follows from dS/dchi = -y sum W~ Gamma r^2 (.)
 * and dk/dT = b k / T.  f is negative as T -> 0 and grows like rho cv T, but it
 * need not be monotone, so plain Newton can fail (READING: the paper names the
 * method, not its safeguards).  The far end of a bracket is found from T^n (doubling
 * upward while f < 0, halving downward while f > 0); Newton steps then start at T^n,
 * which becomes the bracket's near end at the first step, so the bracket is [T^n, hi]
 * (or [lo, T^n]), and a bisection replaces any larger step that leaves it, until a
 * step changes T by at most 1e-14 T; that converged step is taken as it is, even when
 * rounding puts it on the bracket's end (at most 200 evaluations in all).  Where f has
 * several roots the iteration is meant to give the first one met from T^n in the
 * direction of f's sign (the smallest above T^n, or the largest below it); the tests
 * check that by a scan of f written apart from this code.  The comoving
 * sums are then evaluated at the final T, and the per-angle update and the
 * bookkeeping are those of the grey update with the opacities at T^{n+1}.
 */
typedef struct {
  double kP, kJ, S1, SG, SI, D, f, fp;
} kT_eval;

static kT_eval kT_evaluate(double T, int K, const double *Gam, const double *Wt, const double *Icom, double y,
                           double rho, double cv, double Tn, double dt, double c_light, double a_rad, double kP0,
                           double kJ0, double ks, double T_ref, double bP, double bJ) {
  kT_eval e;
  e.kP = kP0 * pow(T / T_ref, bP);
  e.kJ = kJ0 * pow(T / T_ref, bJ);
  const double chi = e.kJ + ks;
  double S1p = 0, SGp = 0, SIp = 0;
  e.S1 = e.SG = e.SI = 0;
  for (int k = 0; k < K; ++k) {
    const double r = 1.0 / (1.0 + y * chi * Gam[k]);
    e.S1 += Wt[k] * r;
    e.SG += Wt[k] * Gam[k] * r;
    e.SI += Wt[k] * Icom[k] * r;
    S1p += Wt[k] * Gam[k] * r * r;
    SGp += Wt[k] * Gam[k] * Gam[k] * r * r;
    SIp += Wt[k] * Icom[k] * Gam[k] * r * r;
  }
  e.D = e.S1 + y * e.kJ * e.SG;
  const double fourpi = 4.0 * OR_PI;
  const double T3 = T * T * T, T4 = T3 * T;
  const double Nn = e.kP * a_rad * T4 * e.S1 - fourpi * e.kJ * e.SI;
  e.f = rho * cv * (T - Tn) + dt * c_light * rho * Nn / e.D;
  const double dkP = bP * e.kP / T, dkJ = bJ * e.kJ / T;
  const double dS1 = -y * S1p * dkJ, dSG = -y * SGp * dkJ, dSI = -y * SIp * dkJ;
  const double dD = dS1 + y * (dkJ * e.SG + e.kJ * dSG);
  const double dN = dkP * a_rad * T4 * e.S1 + e.kP * a_rad * 4.0 * T3 * e.S1 + e.kP * a_rad * T4 * dS1 -
                    fourpi * (dkJ * e.SI + e.kJ * dSI);
  e.fp = rho * cv + dt * c_light * rho * (dN * e.D - Nn * dD) / (e.D * e.D);
  return e;
}

void or_source_kT(int64_t N, int K, const double *dirs, const double *W, double c_red, double c_light,
                  double a_rad, double cv, double dt, double *I, const double *rho, double *mom, double *etot,
                  const double *kP0, const double *kJ0, const double *ks, double T_ref, double bP, double bJ,
                  double *T_out) {
  const double fourpi = 4.0 * OR_PI;
#pragma omp parallel
  {
    double *Gam = (double *)malloc(sizeof(double) * (size_t)K);
    double *Wt = (double *)malloc(sizeof(double) * (size_t)K);
    double *Icom = (double *)malloc(sizeof(double) * (size_t)K);
#pragma omp for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
      double *Ii = I + i * K;
      double *p = mom + 3 * i;
      double E0 = 0.0, F0[3] = {0.0, 0.0, 0.0};
      for (int k = 0; k < K; ++k) {
        E0 += fourpi * W[k] * Ii[k];
        for (int c = 0; c < 3; ++c) F0[c] += fourpi * c_light * W[k] * dirs[3 * k + c] * Ii[k];
      }
      double v[3];
      for (int c = 0; c < 3; ++c) v[c] = p[c] / rho[i];
      const double gam = 1.0 / sqrt(1.0 - (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) / (c_light * c_light));
      double norm = 0.0;
      for (int k = 0; k < K; ++k) {
        const double vn = v[0] * dirs[3 * k] + v[1] * dirs[3 * k + 1] + v[2] * dirs[3 * k + 2];
        Gam[k] = gam * (1.0 - vn / c_light);
        const double G2 = Gam[k] * Gam[k];
        Icom[k] = G2 * G2 * Ii[k];
        Wt[k] = W[k] / G2;
        norm += Wt[k];
      }
      for (int k = 0; k < K; ++k) Wt[k] /= norm;
      const double y = dt * c_red * rho[i];
      const double v2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
      const double Tn = (etot[i] - 0.5 * v2 / rho[i]) / (rho[i] * cv);
#define KT_EVAL(T) kT_evaluate((T), K, Gam, Wt, Icom, y, rho[i], cv, Tn, dt, c_light, a_rad, kP0[i], kJ0[i], ks[i], \
                               T_ref, bP, bJ)
      /* bracket the root from T^n */
      double T = Tn, lo = Tn, hi = Tn;
      kT_eval e = KT_EVAL(T);
      int nev = 1;
      if (e.f < 0.0) {
        for (kT_eval eh = e; eh.f < 0.0 && nev < 200; ++nev) {
          lo = hi;
          hi *= 2.0;
          eh = KT_EVAL(hi);
        }
      } else if (e.f > 0.0) {
        for (kT_eval el = e; el.f > 0.0 && nev < 200; ++nev) {
          hi = lo;
          lo *= 0.5;
          el = KT_EVAL(lo);
        }
      }
      /* safeguarded Newton from T^n inside [lo, hi] */
      while (e.f != 0.0 && nev < 200) {
        if (e.f < 0.0) lo = T;
        else hi = T;
        double Tq = T - e.f / e.fp;
        /* a step within the tolerance has converged and is taken as it is; a larger one that
           leaves the bracket is replaced by bisection */
        const int done = fabs(Tq - T) <= 1e-14 * T;
        if (!done && !(Tq > lo && Tq < hi)) Tq = 0.5 * (lo + hi);
        T = Tq;
        e = KT_EVAL(T);
        ++nev;
        if (done) break;
      }
#undef KT_EVAL
      const double T4 = T * T * T * T;
      const double planck = a_rad * T4 / fourpi;
      const double Jc = (e.SI + y * e.kP * e.SG * planck) / e.D;
      const double chi = e.kJ + ks[i];
      double E1 = 0.0, F1[3] = {0.0, 0.0, 0.0};
      for (int k = 0; k < K; ++k) {
        const double Inew = (Icom[k] + y * Gam[k] * (e.kP * planck + ks[i] * Jc)) / (1.0 + y * chi * Gam[k]);
        const double G2 = Gam[k] * Gam[k];
        Ii[k] = Inew / (G2 * G2);
        E1 += fourpi * W[k] * Ii[k];
        for (int c = 0; c < 3; ++c) F1[c] += fourpi * c_light * W[k] * dirs[3 * k + c] * Ii[k];
      }
      etot[i] += (c_light / c_red) * (E0 - E1);
      for (int c = 0; c < 3; ++c) p[c] += (F0[c] - F1[c]) / (c_light * c_red);
      if (T_out) T_out[i] = T;
    }
    free(Gam); free(Wt); free(Icom);
  }
}
#endif

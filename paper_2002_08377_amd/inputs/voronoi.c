/*
 * voronoi.c -- periodic Voronoi tessellation of generators on a jittered cubic
 * lattice, used only to generate the synthetic meshes the radiation step runs
 * on.  It produces, for every cell, its volume and centre of mass, and for
 * every face its cell pair, periodic image shift, area, unit normal and
 * centroid: the quantities the finite-volume charge update of the paper's
 * section 2 (the Voronoi cell charges and face fluxes) needs as geometry.
 *
 * It holds none of the radiation method's arithmetic: no face velocity, no
 * flux, no source term.  Both the HIP library and the CPU oracle consume its
 * output as plain input arrays.
 *
 * Method: each cell starts as a large cube around its generator and is clipped
 * by the bisector half-space of every candidate neighbour in the lattice
 * stencil of offsets [-2,2]^3, nearest first.  Clipping stops once the next
 * candidate lies farther than twice the cell's circumradius (no farther
 * generator can cut the cell).  A generator outside the stencil is at least
 * (3 - 2*jitter) spacings away; the builder fails loudly if the cell's
 * circumradius does not prove the stencil sufficient.
 *
 * Coordinates are local to the generator while clipping, so periodic images
 * never need wrapping.  Face normal = unit vector from generator i to the
 * image of generator j (exact for a Voronoi face).  Centroids are returned in
 * the frame of the cell that emitted the face.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define VOR_MAXV 320
#define VOR_MAXF 96
#define VOR_MAXFV 64
#define VOR_NCAND 124

enum { VOR_OK = 0, VOR_EOVERFLOW = 1, VOR_EOPEN = 2, VOR_ESTENCIL = 3, VOR_EDEGEN = 4, VOR_EARG = 5 };

typedef struct {
  int nv;
  double v[VOR_MAXV][3];
  int nf;
  int fnv[VOR_MAXF];
  int fv[VOR_MAXF][VOR_MAXFV];
  int ftag[VOR_MAXF];
} vor_poly;

typedef struct {
  double u[3];
  double d2;
  int32_t cell;
  int8_t shift[3];
} vor_cand;

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void init_cube(vor_poly *P, double hw) {
  static const int sgn[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                                {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};
  /* faces listed counter-clockwise seen from outside */
  static const int faces[6][4] = {{0, 3, 2, 1}, {4, 5, 6, 7}, {0, 1, 5, 4},
                                  {2, 3, 7, 6}, {1, 2, 6, 5}, {0, 4, 7, 3}};
  P->nv = 8;
  for (int v = 0; v < 8; ++v)
    for (int c = 0; c < 3; ++c) P->v[v][c] = hw * sgn[v][c];
  P->nf = 6;
  for (int f = 0; f < 6; ++f) {
    P->fnv[f] = 4;
    for (int e = 0; e < 4; ++e) P->fv[f][e] = faces[f][e];
    P->ftag[f] = -1;
  }
}

/* Keep the part of P with x.u <= |u|^2/2.  Returns VOR_OK or an error code. */
static int clip(vor_poly *P, const double u[3], int tag, double eps) {
  double d[VOR_MAXV];
  const double half = 0.5 * dot3(u, u);
  int any_out = 0;
  for (int v = 0; v < P->nv; ++v) {
    double dv = dot3(P->v[v], u) - half;
    if (fabs(dv) < eps) dv = 0.0;
    d[v] = dv;
    if (dv > 0.0) any_out = 1;
  }
  if (!any_out) return VOR_OK;

  /* new vertices created on cut edges: keyed by (inside, outside) vertex pair */
  int ek_in[VOR_MAXV], ek_out[VOR_MAXV], ek_id[VOR_MAXV];
  int ne = 0;
  int nv = P->nv;
  static _Thread_local int cap_next[2 * VOR_MAXV];
  for (int v = 0; v < 2 * VOR_MAXV; ++v) cap_next[v] = -1;

  static _Thread_local int nfv[VOR_MAXF][VOR_MAXFV];
  static _Thread_local int nfn[VOR_MAXF];
  static _Thread_local int nft[VOR_MAXF];
  int nf = 0;
  int ncut = 0;

  for (int f = 0; f < P->nf; ++f) {
    const int m = P->fnv[f];
    int cnt = 0;
    int exit_pt = -1, entry_pt = -1;
    for (int e = 0; e < m; ++e) {
      const int a = P->fv[f][e];
      const int b = P->fv[f][(e + 1) % m];
      const int ina = d[a] <= 0.0, inb = d[b] <= 0.0;
      if (ina) {
        if (cnt >= VOR_MAXFV) return VOR_EOVERFLOW;
        nfv[nf][cnt++] = a;
      }
      if (ina != inb) {
        const int vin = ina ? a : b, vout = ina ? b : a;
        int p;
        if (d[vin] == 0.0) {
          p = vin;
        } else {
          p = -1;
          for (int q = 0; q < ne; ++q)
            if (ek_in[q] == vin && ek_out[q] == vout) { p = ek_id[q]; break; }
          if (p < 0) {
            if (nv >= VOR_MAXV || ne >= VOR_MAXV) return VOR_EOVERFLOW;
            const double t = d[vin] / (d[vin] - d[vout]);
            for (int c = 0; c < 3; ++c) P->v[nv][c] = P->v[vin][c] + t * (P->v[vout][c] - P->v[vin][c]);
            d[nv] = 0.0;
            ek_in[ne] = vin; ek_out[ne] = vout; ek_id[ne] = nv; ++ne;
            p = nv++;
          }
          if (cnt >= VOR_MAXFV) return VOR_EOVERFLOW;
          nfv[nf][cnt++] = p;
        }
        if (ina) exit_pt = p; else entry_pt = p;
      }
    }
    if (exit_pt >= 0 || entry_pt >= 0) {
      if (exit_pt < 0 || entry_pt < 0) return VOR_EDEGEN;
      if (exit_pt != entry_pt) { /* a face touching the plane at one vertex adds no cap edge */
        cap_next[entry_pt] = exit_pt;
        ++ncut;
      }
    }
    if (cnt >= 3) {
      nfn[nf] = cnt;
      nft[nf] = P->ftag[f];
      ++nf;
    }
  }
  if (ncut < 3) return VOR_EDEGEN;
  /* walk the cap cycle */
  int start = -1;
  for (int v = 0; v < nv; ++v)
    if (cap_next[v] >= 0) { start = v; break; }
  if (start < 0) return VOR_EDEGEN;
  if (nf >= VOR_MAXF) return VOR_EOVERFLOW;
  int cnt = 0, cur = start;
  do {
    if (cnt >= VOR_MAXFV) return VOR_EOVERFLOW;
    nfv[nf][cnt++] = cur;
    cur = cap_next[cur];
    if (cur < 0) return VOR_EDEGEN;
  } while (cur != start);
  if (cnt != ncut) return VOR_EDEGEN;
  nfn[nf] = cnt;
  nft[nf] = tag;
  ++nf;

  /* compact vertices: keep those referenced by faces */
  int remap[VOR_MAXV];
  for (int v = 0; v < nv; ++v) remap[v] = -1;
  int nk = 0;
  static _Thread_local double nvtx[VOR_MAXV][3];
  for (int f = 0; f < nf; ++f)
    for (int e = 0; e < nfn[f]; ++e) {
      const int v = nfv[f][e];
      if (remap[v] < 0) {
        remap[v] = nk;
        nvtx[nk][0] = P->v[v][0]; nvtx[nk][1] = P->v[v][1]; nvtx[nk][2] = P->v[v][2];
        ++nk;
      }
      nfv[f][e] = remap[v];
    }
  P->nv = nk;
  memcpy(P->v, nvtx, sizeof(double) * 3 * (size_t)nk);
  P->nf = nf;
  for (int f = 0; f < nf; ++f) {
    P->fnv[f] = nfn[f];
    P->ftag[f] = nft[f];
    memcpy(P->fv[f], nfv[f], sizeof(int) * (size_t)nfn[f]);
  }
  return VOR_OK;
}

static double max_r2(const vor_poly *P) {
  double r2 = 0.0;
  for (int v = 0; v < P->nv; ++v) {
    const double q = dot3(P->v[v], P->v[v]);
    if (q > r2) r2 = q;
  }
  return r2;
}

static int cand_cmp(const void *a, const void *b) {
  const vor_cand *x = (const vor_cand *)a, *y = (const vor_cand *)b;
  if (x->d2 < y->d2) return -1;
  if (x->d2 > y->d2) return 1;
  return (x->cell > y->cell) - (x->cell < y->cell);
}

/* Build the cell of generator i.  Fills P and the candidate table; returns an error code. */
static int build_cell(int64_t i, int n, double L, double jitter, const double *gen, const int32_t *cell_lat,
                      const int32_t *lat_cell, vor_poly *P, vor_cand *cand) {
  const double h = L / n;
  const int a0 = cell_lat[3 * i], b0 = cell_lat[3 * i + 1], c0 = cell_lat[3 * i + 2];
  int nc = 0;
  for (int dz = -2; dz <= 2; ++dz)
    for (int dy = -2; dy <= 2; ++dy)
      for (int dx = -2; dx <= 2; ++dx) {
        if (!dx && !dy && !dz) continue;
        int a = a0 + dx, b = b0 + dy, c = c0 + dz;
        int sa = 0, sb = 0, sc = 0;
        if (a < 0) { a += n; sa = -1; } else if (a >= n) { a -= n; sa = 1; }
        if (b < 0) { b += n; sb = -1; } else if (b >= n) { b -= n; sb = 1; }
        if (c < 0) { c += n; sc = -1; } else if (c >= n) { c -= n; sc = 1; }
        const int32_t j = lat_cell[((int64_t)c * n + b) * n + a];
        vor_cand *q = &cand[nc++];
        q->cell = j;
        q->shift[0] = (int8_t)sa; q->shift[1] = (int8_t)sb; q->shift[2] = (int8_t)sc;
        q->u[0] = gen[3 * j] + sa * L - gen[3 * i];
        q->u[1] = gen[3 * j + 1] + sb * L - gen[3 * i + 1];
        q->u[2] = gen[3 * j + 2] + sc * L - gen[3 * i + 2];
        q->d2 = dot3(q->u, q->u);
      }
  qsort(cand, (size_t)nc, sizeof(vor_cand), cand_cmp);
  init_cube(P, 3.0 * h);
  const double eps = 1e-13 * h * h;
  int done = 0;
  for (int k = 0; k < nc; ++k) {
    if (cand[k].d2 > 4.0 * max_r2(P)) { done = 1; break; }
    const int rc = clip(P, cand[k].u, k, eps);
    if (rc) return rc;
  }
  for (int f = 0; f < P->nf; ++f)
    if (P->ftag[f] < 0) return VOR_EOPEN;
  if (!done) {
    const double excl = (3.0 - 2.0 * jitter) * h;
    if (4.0 * max_r2(P) >= excl * excl) return VOR_ESTENCIL;
  }
  return VOR_OK;
}

/* Area (projected on the exact normal), centroid (local), plane distance. */
static void face_props(const vor_poly *P, int f, const double nrm[3], double *area, double cen[3], double *vol,
                       double vcen[3]) {
  const int m = P->fnv[f];
  double c0[3] = {0, 0, 0};
  for (int e = 0; e < m; ++e)
    for (int c = 0; c < 3; ++c) c0[c] += P->v[P->fv[f][e]][c];
  for (int c = 0; c < 3; ++c) c0[c] /= m;
  double A = 0.0, C[3] = {0, 0, 0}, V = 0.0, VC[3] = {0, 0, 0};
  for (int e = 0; e < m; ++e) {
    const double *p = P->v[P->fv[f][e]], *q = P->v[P->fv[f][(e + 1) % m]];
    const double x[3] = {p[0] - c0[0], p[1] - c0[1], p[2] - c0[2]};
    const double y[3] = {q[0] - c0[0], q[1] - c0[1], q[2] - c0[2]};
    const double cr[3] = {x[1] * y[2] - x[2] * y[1], x[2] * y[0] - x[0] * y[2], x[0] * y[1] - x[1] * y[0]};
    const double a = 0.5 * dot3(cr, nrm);
    A += a;
    for (int c = 0; c < 3; ++c) C[c] += a * (c0[c] + p[c] + q[c]) / 3.0;
    /* tetrahedron (generator at origin, c0, p, q) */
    const double tv = (c0[0] * (p[1] * q[2] - p[2] * q[1]) - c0[1] * (p[0] * q[2] - p[2] * q[0]) +
                       c0[2] * (p[0] * q[1] - p[1] * q[0])) / 6.0;
    V += tv;
    for (int c = 0; c < 3; ++c) VC[c] += tv * (c0[c] + p[c] + q[c]) / 4.0;
  }
  *area = A;
  for (int c = 0; c < 3; ++c) cen[c] = (A != 0.0) ? C[c] / A : c0[c];
  *vol = V;
  for (int c = 0; c < 3; ++c) vcen[c] = VC[c];
}

/*
 * Pass 1: per-cell face count, volume and centre of mass.
 * mode 0 counts faces whose neighbour id is larger (each face once);
 * mode 1 counts every face of the cell (both sides of each face appear).
 * Returns VOR_OK, or the first error code met (cell index in *bad_cell).
 */
int vor_count(int n, double L, double jitter, const double *gen, const int32_t *cell_lat,
              const int32_t *lat_cell, int mode, int64_t *face_count, double *vol, double *com,
              int64_t *bad_cell) {
  if (n < 5 || L <= 0 || jitter < 0 || jitter >= 0.5) return VOR_EARG;
  const int64_t N = (int64_t)n * n * n;
  int err = VOR_OK;
  int64_t bad = -1;
#pragma omp parallel
  {
    vor_poly *P = (vor_poly *)malloc(sizeof(vor_poly));
    vor_cand *cand = (vor_cand *)malloc(sizeof(vor_cand) * VOR_NCAND);
#pragma omp for schedule(dynamic, 256)
    for (int64_t i = 0; i < N; ++i) {
      const int rc = build_cell(i, n, L, jitter, gen, cell_lat, lat_cell, P, cand);
      if (rc) {
#pragma omp critical
        { if (!err) { err = rc; bad = i; } }
        face_count[i] = 0;
        continue;
      }
      int64_t cnt = 0;
      double V = 0.0, VC[3] = {0, 0, 0};
      for (int f = 0; f < P->nf; ++f) {
        const vor_cand *q = &cand[P->ftag[f]];
        const double du = sqrt(q->d2);
        const double nrm[3] = {q->u[0] / du, q->u[1] / du, q->u[2] / du};
        double A, cen[3], tv, tvc[3];
        face_props(P, f, nrm, &A, cen, &tv, tvc);
        V += tv;
        for (int c = 0; c < 3; ++c) VC[c] += tvc[c];
        if (mode == 1 || q->cell > i) ++cnt;
      }
      face_count[i] = cnt;
      vol[i] = V;
      for (int c = 0; c < 3; ++c) com[3 * i + c] = gen[3 * i + c] + VC[c] / V;
    }
    free(P);
    free(cand);
  }
  if (bad_cell) *bad_cell = bad;
  return err;
}

/* Pass 2: write faces at the offsets face_off (exclusive prefix sum of pass-1 counts). */
int vor_faces(int n, double L, double jitter, const double *gen, const int32_t *cell_lat, const int32_t *lat_cell,
              int mode, const int64_t *face_off, int32_t *fcells, int8_t *fshift, double *farea, double *fnormal,
              double *fcent) {
  if (n < 5 || L <= 0 || jitter < 0 || jitter >= 0.5) return VOR_EARG;
  const int64_t N = (int64_t)n * n * n;
  int err = VOR_OK;
#pragma omp parallel
  {
    vor_poly *P = (vor_poly *)malloc(sizeof(vor_poly));
    vor_cand *cand = (vor_cand *)malloc(sizeof(vor_cand) * VOR_NCAND);
#pragma omp for schedule(dynamic, 256)
    for (int64_t i = 0; i < N; ++i) {
      const int rc = build_cell(i, n, L, jitter, gen, cell_lat, lat_cell, P, cand);
      if (rc) {
#pragma omp critical
        { if (!err) err = rc; }
        continue;
      }
      int64_t o = face_off[i];
      for (int f = 0; f < P->nf; ++f) {
        const vor_cand *q = &cand[P->ftag[f]];
        if (!(mode == 1 || q->cell > i)) continue;
        const double du = sqrt(q->d2);
        const double nrm[3] = {q->u[0] / du, q->u[1] / du, q->u[2] / du};
        double A, cen[3], tv, tvc[3];
        face_props(P, f, nrm, &A, cen, &tv, tvc);
        fcells[2 * o] = (int32_t)i;
        fcells[2 * o + 1] = q->cell;
        for (int c = 0; c < 3; ++c) {
          fshift[3 * o + c] = q->shift[c];
          fnormal[3 * o + c] = nrm[c];
          fcent[3 * o + c] = gen[3 * i + c] + cen[c];
        }
        farea[o] = A;
        ++o;
      }
      if (o != face_off[i + 1]) {
#pragma omp critical
        { if (!err) err = VOR_EDEGEN; }
      }
    }
    free(P);
    free(cand);
  }
  return err;
}

// Host half of the mesh upload (section 2: cells and faces of the tessellation): the
// checks of the input tessellation, the half-face index grouped by cell that every cell
// gathers its fluxes through, and the per-workgroup staging sizes and cell orders of the
// kernels.  Plain C++17 with no HIP, so that a host-only build can run it under sanitizers.
#pragma once

#include <math.h>
#include <stdint.h>
#include <stdio.h>

#include <algorithm>
#include <string>
#include <vector>

struct rt_host_mesh {
  std::vector<int32_t> row_ptr;  // [N+1]: half-faces of cell i are [row_ptr[i], row_ptr[i+1])
  std::vector<int32_t> hf_face;  // [2F]: face f for its first cell, -(f+1) for its second, in input order
  int32_t hf_cap16 = 0;          // most half-faces of any 16 / 32 / 64 consecutive cells
  int32_t hf_cap32 = 0;
  int32_t hf_cap64 = 0;
  // within every run of 16 / 32 / 64 consecutive cells, position g holds the offset of the
  // cell with the g-th smallest face count (a stable order), so each wave's cells pad alike
  std::vector<uint8_t> order16, order32, order64;
};

// Checks the tessellation and fills `out`.  Returns "" on success, else the reason (the
// first bad cell or face): volume <= 0, face cells out of range or equal, area <= 0,
// non-unit normal, periodic shift outside {-1, 0, 1}, a cell whose faces do not close
// (|sum A n| > 1e-8 V^(2/3)).  N, F >= 1 and 2F < 2^31 are the caller's to check.
inline std::string rt_build_host_mesh(int64_t N, int64_t F, const double *vol, const int32_t *face_cells,
                                      const int8_t *face_shift, const double *face_area, const double *face_normal,
                                      rt_host_mesh &out) {
  char buf[256];
  for (int64_t i = 0; i < N; ++i)
    if (!(vol[i] > 0.0) || !isfinite(vol[i])) {
      snprintf(buf, sizeof buf, "cell %lld has volume <= 0", (long long)i);
      return buf;
    }
  // faces: indices, areas, normals; closure of every cell
  std::vector<double> clo(3 * (size_t)N, 0.0);
  std::vector<int32_t> cnt((size_t)N + 1, 0);
  for (int64_t f = 0; f < F; ++f) {
    const int32_t i = face_cells[2 * f], j = face_cells[2 * f + 1];
    if (i < 0 || j < 0 || i >= N || j >= N || i == j) {
      snprintf(buf, sizeof buf, "face %lld has invalid cells (%d, %d)", (long long)f, i, j);
      return buf;
    }
    const double A = face_area[f];
    if (!(A > 0.0) || !isfinite(A)) {
      snprintf(buf, sizeof buf, "face %lld has area <= 0", (long long)f);
      return buf;
    }
    const double *n = &face_normal[3 * f];
    const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    if (!(fabs(nn - 1.0) < 1e-10)) {
      snprintf(buf, sizeof buf, "face %lld normal is not unit", (long long)f);
      return buf;
    }
    for (int c = 0; c < 3; ++c) {
      if (face_shift[3 * f + c] < -1 || face_shift[3 * f + c] > 1) {
        snprintf(buf, sizeof buf, "face %lld shift outside {-1,0,1}", (long long)f);
        return buf;
      }
      clo[3 * (size_t)i + c] += A * n[c];
      clo[3 * (size_t)j + c] -= A * n[c];
    }
    cnt[(size_t)i + 1]++;
    cnt[(size_t)j + 1]++;
  }
  for (int64_t i = 0; i < N; ++i) {
    const double *c = &clo[3 * (size_t)i];
    const double r = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    if (!(r <= 1e-8 * pow(vol[i], 2.0 / 3.0))) {
      snprintf(buf, sizeof buf, "cell %lld is not closed: |sum A n| = %g", (long long)i, r);
      return buf;
    }
  }
  // half-face index grouped by cell, faces in input order within a cell
  out.row_ptr.assign((size_t)N + 1, 0);
  for (int64_t i = 0; i < N; ++i) out.row_ptr[(size_t)i + 1] = out.row_ptr[(size_t)i] + cnt[(size_t)i + 1];
  out.hf_face.assign(2 * (size_t)F, 0);
  {
    std::vector<int32_t> fill(out.row_ptr.begin(), out.row_ptr.end() - 1);
    for (int64_t f = 0; f < F; ++f) {
      const int32_t i = face_cells[2 * f], j = face_cells[2 * f + 1];
      out.hf_face[(size_t)fill[(size_t)i]++] = (int32_t)f;
      out.hf_face[(size_t)fill[(size_t)j]++] = (int32_t)(-f - 1);
    }
  }
  // staging sizes and cell orders of the workgroups of 16 / 32 / 64 consecutive cells
  auto cap = [&](int cpb) {
    int32_t best = 0;
    for (int64_t c = 0; c < N; c += cpb) {
      const int64_t e = c + cpb < N ? c + cpb : N;
      best = std::max<int32_t>(best, out.row_ptr[(size_t)e] - out.row_ptr[(size_t)c]);
    }
    return best;
  };
  out.hf_cap16 = cap(16);
  out.hf_cap32 = cap(32);
  out.hf_cap64 = cap(64);
  std::vector<int> idx;
  auto fill_order = [&](int cpb, std::vector<uint8_t> &ord) {
    ord.assign((size_t)N, 0);
    for (int64_t c = 0; c < N; c += cpb) {
      const int n = (int)std::min<int64_t>(cpb, N - c);
      idx.resize((size_t)n);
      for (int g = 0; g < n; ++g) idx[(size_t)g] = g;
      std::stable_sort(idx.begin(), idx.end(),
                       [&](int x, int y) { return cnt[(size_t)(c + x) + 1] < cnt[(size_t)(c + y) + 1]; });
      for (int g = 0; g < n; ++g) ord[(size_t)(c + g)] = (uint8_t)idx[(size_t)g];
    }
  };
  fill_order(16, out.order16);
  fill_order(32, out.order32);
  fill_order(64, out.order64);
  return std::string();
}

// sanitize_host_mesh.cpp -- TEST INFRASTRUCTURE: runs the host half of the mesh upload
// (paper_2002_08377_amd/csrc/rt_mesh_host.h: tessellation checks, the half-face index,
// staging sizes, workgroup cell orders) on valid and invalid meshes, in a build with
// -fsanitize=address,undefined, and checks its output against brute-force recomputation.
// Exits non-zero on any failure.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <string>
#include <vector>

#include "rt_mesh_host.h"

static int failures = 0;
#define CHECK(cond, ...)                     \
  do {                                       \
    if (!(cond)) {                           \
      fprintf(stderr, "FAIL: " __VA_ARGS__); \
      fprintf(stderr, "\n");                 \
      ++failures;                            \
    }                                        \
  } while (0)

struct Mesh {
  int64_t N = 0;
  std::vector<double> vol, area, normal;
  std::vector<int32_t> cells;
  std::vector<int8_t> shift;
  int64_t F() const { return (int64_t)area.size(); }
};

// Periodic n^3 cubic lattice of unit box; faces +x, +y, +z of every cell, each face of a cell
// with lattice x below `split_below` cut into m x m coplanar sub-faces (face counts vary).
static Mesh lattice(int n, int m, int split_below) {
  Mesh M;
  M.N = (int64_t)n * n * n;
  const double h = 1.0 / n;
  M.vol.assign((size_t)M.N, h * h * h);
  for (int64_t i = 0; i < M.N; ++i) {
    const int s[3] = {(int)(i % n), (int)((i / n) % n), (int)(i / ((int64_t)n * n))};
    for (int ax = 0; ax < 3; ++ax) {
      int t[3] = {s[0], s[1], s[2]};
      t[ax] = (t[ax] + 1) % n;
      const int64_t j = t[0] + (int64_t)n * t[1] + (int64_t)n * n * t[2];
      const int parts = (s[0] < split_below || t[0] < split_below) ? m : 1;
      for (int p = 0; p < parts * parts; ++p) {
        M.cells.push_back((int32_t)i);
        M.cells.push_back((int32_t)j);
        for (int c = 0; c < 3; ++c) {
          M.normal.push_back(c == ax ? 1.0 : 0.0);
          M.shift.push_back((int8_t)(c == ax && s[ax] == n - 1 ? 1 : 0));
        }
        M.area.push_back(h * h / (parts * parts));
      }
    }
  }
  return M;
}

static std::string build(const Mesh &M, rt_host_mesh &out) {
  return rt_build_host_mesh(M.N, M.F(), M.vol.data(), M.cells.data(), M.shift.data(), M.area.data(), M.normal.data(),
                            out);
}

static void check_valid(const Mesh &M, const char *name) {
  rt_host_mesh hm;
  const std::string why = build(M, hm);
  CHECK(why.empty(), "%s refused: %s", name, why.c_str());
  if (!why.empty()) return;
  const int64_t N = M.N, F = M.F();
  CHECK((int64_t)hm.row_ptr.size() == N + 1 && hm.row_ptr[0] == 0 && hm.row_ptr[(size_t)N] == 2 * F, "%s row_ptr",
        name);
  // every face once from each of its cells, with the sign of the side, in input order
  std::vector<int> seen((size_t)F, 0);
  for (int64_t i = 0; i < N; ++i) {
    int32_t last = -1;
    for (int32_t h = hm.row_ptr[(size_t)i]; h < hm.row_ptr[(size_t)i + 1]; ++h) {
      const int32_t e = hm.hf_face[(size_t)h];
      const int32_t f = e >= 0 ? e : -e - 1;
      CHECK(f >= 0 && f < F, "%s half-face %d names face %d", name, h, f);
      if (f < 0 || f >= F) continue;
      CHECK(M.cells[2 * (size_t)f + (e >= 0 ? 0 : 1)] == i, "%s half-face %d is not cell %lld's", name, h, (long long)i);
      CHECK(f > last, "%s cell %lld faces out of input order", name, (long long)i);
      last = f;
      seen[(size_t)f] += e >= 0 ? 1 : 2;
    }
  }
  for (int64_t f = 0; f < F; ++f) CHECK(seen[(size_t)f] == 3, "%s face %lld listed %d", name, (long long)f, seen[(size_t)f]);
  // staging sizes and orders against brute force
  const int cpbs[3] = {16, 32, 64};
  const int32_t caps[3] = {hm.hf_cap16, hm.hf_cap32, hm.hf_cap64};
  const std::vector<uint8_t> *ords[3] = {&hm.order16, &hm.order32, &hm.order64};
  for (int b = 0; b < 3; ++b) {
    const int cpb = cpbs[b];
    int32_t best = 0;
    for (int64_t c = 0; c < N; c += cpb) {
      const int64_t e = std::min<int64_t>(c + cpb, N);
      int32_t s = 0;
      std::vector<int> used((size_t)cpb, 0);
      int prev = -1;
      int64_t prev_off = -1;
      for (int64_t g = c; g < e; ++g) {
        s += hm.row_ptr[(size_t)g + 1] - hm.row_ptr[(size_t)g];
        const int o = (*ords[b])[(size_t)g];
        CHECK(o < e - c, "%s order %d out of its block", name, o);
        if (o >= e - c) continue;
        used[(size_t)o]++;
        const int cntg = hm.row_ptr[(size_t)(c + o) + 1] - hm.row_ptr[(size_t)(c + o)];
        CHECK(cntg > prev || (cntg == prev && o > prev_off), "%s order not sorted stably", name);
        prev = cntg;
        prev_off = o;
      }
      for (int64_t g = 0; g < e - c; ++g) CHECK(used[(size_t)g] == 1, "%s order is not a permutation", name);
      best = std::max(best, s);
    }
    CHECK(best == caps[b], "%s cap of %d cells %d, brute force %d", name, cpb, caps[b], best);
  }
}

static void check_refused(const Mesh &M, const char *expect, const char *name) {
  rt_host_mesh hm;
  const std::string why = build(M, hm);
  CHECK(why.find(expect) != std::string::npos, "%s: expected '%s', got '%s'", name, expect, why.c_str());
}

int main() {
  check_valid(lattice(5, 1, 0), "lattice 5^3");
  check_valid(lattice(6, 3, 3), "split lattice 6^3");
  check_valid(lattice(7, 2, 4), "split lattice 7^3 (ragged blocks)");
  const Mesh base = lattice(5, 1, 0);
  Mesh m = base;
  m.vol[7] = 0.0;
  check_refused(m, "cell 7 has volume <= 0", "zero volume");
  m = base;
  m.cells[2 * 10 + 1] = (int32_t)m.N;
  check_refused(m, "face 10 has invalid cells", "cell out of range");
  m = base;
  m.cells[2 * 11 + 1] = m.cells[2 * 11];
  check_refused(m, "face 11 has invalid cells", "self face");
  m = base;
  m.area[12] = -1.0;
  check_refused(m, "face 12 has area <= 0", "negative area");
  m = base;
  for (int c = 0; c < 3; ++c) m.normal[3 * 13 + c] *= 1.1;
  check_refused(m, "face 13 normal is not unit", "long normal");
  m = base;
  m.shift[3 * 14 + 2] = 2;
  check_refused(m, "face 14 shift outside", "shift 2");
  m = base;
  m.area[15] *= 1.5;
  check_refused(m, "is not closed", "open cell");
  // random face lists: never crash, refuse what is not a closed tessellation
  srand(12345);
  for (int trial = 0; trial < 200; ++trial) {
    Mesh r;
    r.N = 1 + rand() % 40;
    r.vol.assign((size_t)r.N, 1.0);
    const int F = 1 + rand() % 120;
    for (int f = 0; f < F; ++f) {
      r.cells.push_back((int32_t)(rand() % (r.N + 2)) - 1);
      r.cells.push_back((int32_t)(rand() % (r.N + 2)) - 1);
      const double a = rand() / (double)RAND_MAX - 0.1;
      r.area.push_back(a);
      double n[3] = {rand() / (double)RAND_MAX - 0.5, rand() / (double)RAND_MAX - 0.5, rand() / (double)RAND_MAX - 0.5};
      const double l = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]) + 1e-300;
      for (int c = 0; c < 3; ++c) {
        r.normal.push_back(rand() % 4 ? n[c] / l : n[c]);
        r.shift.push_back((int8_t)(rand() % 4 - 1));
      }
    }
    rt_host_mesh hm;
    (void)build(r, hm);
  }
  if (failures) {
    fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  printf("host mesh driver OK\n");
  return 0;
}

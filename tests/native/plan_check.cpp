// Host-table checks of plan.cpp, built with g++ and the address and
// undefined-behaviour sanitizers by tests/test_abi_host.py (no GPU, no HIP).
// It builds the offset-array tables of spheres and ellipsoids on several
// grids (Section 3.3: the xy-projection of the sphere, z compressed), feeds
// the validator malformed maps, and checks the radix plans and twiddle
// tables; any out-of-bounds access or undefined behaviour aborts the run.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../paper_2406_05577_amd/csrc/plan.hpp"

using namespace fftb;

static int failures = 0;
#define CHECK(c)                                                 \
  do {                                                           \
    if (!(c)) {                                                  \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      ++failures;                                                \
    }                                                            \
  } while (0)

// wrapped linear indices of the integer points of an ellipsoid around -k
static std::vector<int32_t> ellipsoid(int nx, int ny, int nz, double ax, double ay, double az,
                                      double kx, double ky, double kz) {
  std::vector<int32_t> out;
  const int rx = static_cast<int>(ax) + 2, ry = static_cast<int>(ay) + 2, rz = static_cast<int>(az) + 2;
  for (int mx = -rx; mx <= rx; ++mx)
    for (int my = -ry; my <= ry; ++my)
      for (int mz = -rz; mz <= rz; ++mz) {
        const double t = ((mx + kx) / ax) * ((mx + kx) / ax) + ((my + ky) / ay) * ((my + ky) / ay) +
                         ((mz + kz) / az) * ((mz + kz) / az);
        if (t > 1.0) continue;
        const int x = ((mx % nx) + nx) % nx, y = ((my % ny) + ny) % ny, z = ((mz % nz) + nz) % nz;
        out.push_back(x + nx * (y + ny * z));
      }
  return out;
}

static void check_tables(int nx, int ny, int nz, const std::vector<int32_t>& map) {
  SphereTables t;
  std::string err;
  const int rc = build_sphere_tables(nx, ny, nz, map.data(), static_cast<int64_t>(map.size()), 3, t, err);
  CHECK(rc == 0);
  if (rc != 0) return;
  CHECK(t.ns == static_cast<int64_t>(map.size()));
  CHECK(static_cast<int>(t.col_x.size()) == t.ncol);
  CHECK(static_cast<int>(t.slabstart.size()) == t.nslab + 1);
  CHECK(static_cast<int64_t>(t.gidx.size()) == static_cast<int64_t>(t.ncol) * nz);
  int64_t hits = 0;
  for (int c = 0; c < t.ncol; ++c)
    for (int z = 0; z < nz; ++z) {
      const int g = t.gidx[static_cast<size_t>(c) * nz + z];
      if (g < 0) continue;
      ++hits;
      CHECK(map[g] == t.col_x[c] + nx * (t.col_y[c] + ny * z));
    }
  CHECK(hits == t.ns);
  for (int xi = 0; xi < t.nslab; ++xi)
    for (int c = t.slabstart[xi]; c < t.slabstart[xi + 1]; ++c) {
      CHECK(t.col_xi[c] == xi);
      CHECK(t.colidx[static_cast<size_t>(xi) * ny + t.col_y[c]] == c);
      CHECK(t.xinv[t.col_x[c]] == xi);
    }
}

static void expect_invalid(int nx, int ny, int nz, const std::vector<int32_t>& map) {
  SphereTables t;
  std::string err;
  CHECK(build_sphere_tables(nx, ny, nz, map.data(), static_cast<int64_t>(map.size()), 2, t, err) != 0);
  CHECK(!err.empty());
}

int main() {
  const int dims[][3] = {{6, 5, 4}, {32, 32, 32}, {30, 24, 36}, {96, 96, 96}, {144, 160, 180}};
  const double semi[][3] = {{1.6, 1.3, 1.1}, {8, 8, 8}, {7.1, 5.9, 8.8}, {24, 24, 24}, {36, 40, 45}};
  for (int i = 0; i < 5; ++i) {
    const int nx = dims[i][0], ny = dims[i][1], nz = dims[i][2];
    std::vector<int32_t> m = ellipsoid(nx, ny, nz, semi[i][0], semi[i][1], semi[i][2], 0.21, -0.33, 0.1);
    check_tables(nx, ny, nz, m);
    // reversed order: any permutation of the map is accepted
    std::vector<int32_t> r(m.rbegin(), m.rend());
    check_tables(nx, ny, nz, r);
    // malformed maps: a duplicate, an index past the grid, a negative index
    std::vector<int32_t> dup = m;
    dup.push_back(m[m.size() / 2]);
    expect_invalid(nx, ny, nz, dup);
    std::vector<int32_t> big = m;
    big.back() = nx * ny * nz;
    expect_invalid(nx, ny, nz, big);
    std::vector<int32_t> neg = m;
    neg.front() = -1;
    expect_invalid(nx, ny, nz, neg);
  }
  // a single coefficient and the whole grid
  check_tables(12, 10, 8, std::vector<int32_t>{0});
  std::vector<int32_t> all(12 * 10 * 8);
  for (size_t i = 0; i < all.size(); ++i) all[i] = static_cast<int32_t>(i);
  check_tables(12, 10, 8, all);
  // radix plans and twiddles of every 2,3,5-smooth length up to 400
  for (int n = 1; n <= 400; ++n) {
    std::vector<int> rad;
    int k = n;
    for (int p : {2, 3, 5})
      while (k % p == 0) k /= p;
    const bool smooth = k == 1;
    CHECK(plan_radices(n, rad) == smooth);
    if (!smooth) continue;
    AxisPlan ap;
    make_axis_plan(n, rad, ap);
    int prod = 1;
    for (int s = 0; s < ap.nst; ++s) prod *= ap.R[s];
    CHECK(prod == n);
    const std::vector<double> tw = axis_twiddles(ap);
    for (double v : tw) CHECK(std::fabs(v) <= 1.0 + 1e-15);
    const std::vector<double> rt = root_table(n);
    CHECK(rt.size() == static_cast<size_t>(2 * n));
    for (int j = 0; j < n; ++j) {
      const double re = rt[2 * j], im = rt[2 * j + 1];
      CHECK(std::fabs(re * re + im * im - 1.0) < 1e-14);
    }
  }
  if (failures) {
    std::fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  std::printf("plan_check OK\n");
  return 0;
}

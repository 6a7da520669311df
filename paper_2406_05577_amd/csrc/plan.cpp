// Host-side plan: validation, column tables, radix plans, twiddle tables.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <numeric>

namespace fftb {

namespace {

const int kRadices[] = {16, 15, 12, 10, 9, 8, 6, 5, 4, 3, 2};

bool only_235(int n) {
  if (n < 1) return false;
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

// Fewest-stage factorisation; among those, maximise the smallest radix.
void search(int n, int depth, int maxdepth, std::vector<int>& cur, std::vector<int>& best) {
  if (n == 1) {
    if (best.empty() || cur.size() < best.size() ||
        (cur.size() == best.size() &&
         *std::min_element(cur.begin(), cur.end()) > *std::min_element(best.begin(), best.end())))
      best = cur;
    return;
  }
  if (depth == maxdepth) return;
  for (int r : kRadices) {
    if (n % r) continue;
    if (!cur.empty() && r > cur.back()) continue;  // non-increasing order
    cur.push_back(r);
    search(n / r, depth + 1, maxdepth, cur, best);
    cur.pop_back();
  }
}

}  // namespace

bool plan_radices(int n, std::vector<int>& radices) {
  radices.clear();
  if (!only_235(n)) return false;
  if (n == 1) {
    radices.push_back(1);
    return true;
  }
  std::vector<int> cur, best;
  for (int d = 1; d <= kMaxStages && best.empty(); ++d) search(n, 0, d, cur, best);
  if (best.empty()) return false;
  radices = best;
  return true;
}

void make_axis_plan(int n, const std::vector<int>& radices, AxisPlan& ap) {
  ap = AxisPlan();
  ap.n = n;
  ap.nst = static_cast<int>(radices.size());
  int p = 1, off = 0;
  for (int s = 0; s < ap.nst; ++s) {
    ap.R[s] = radices[s];
    ap.p[s] = p;
    ap.twoff[s] = off;
    off += p * radices[s];
    p *= radices[s];
  }
  ap.twlen = off;
}

static void root(int64_t num, int64_t den, double& c, double& s) {
  // exp(-2*pi*i*num/den) with num already reduced to [0, den)
  const double ang = 2.0 * M_PI * static_cast<double>(num) / static_cast<double>(den);
  c = std::cos(ang);
  s = -std::sin(ang);
}

std::vector<double> axis_twiddles(const AxisPlan& ap) {
  std::vector<double> t(2 * static_cast<size_t>(ap.twlen), 0.0);
  for (int s = 0; s < ap.nst; ++s) {
    const int R = ap.R[s], p = ap.p[s];
    const int64_t L = static_cast<int64_t>(p) * R;
    for (int k = 0; k < p; ++k)
      for (int q = 0; q < R; ++q) {
        double c, sn;
        root((static_cast<int64_t>(q) * k) % L, L, c, sn);
        const size_t idx = static_cast<size_t>(ap.twoff[s] + k * R + q);
        t[2 * idx] = c;
        t[2 * idx + 1] = sn;
      }
  }
  return t;
}

std::vector<double> root_table(int n) {
  std::vector<double> t(2 * static_cast<size_t>(n));
  for (int j = 0; j < n; ++j) root(j, n, t[2 * j], t[2 * j + 1]);
  return t;
}

int build_sphere_tables(int nx, int ny, int nz, const int32_t* map, int64_t ns, int nb,
                        SphereTables& st, std::string& err) {
  st = SphereTables();
  if (!map) { err = "null map pointer"; return -1; }
  if (ns < 1) { err = "sphere has no coefficients"; return -1; }
  if (nb < 1) { err = "nbands must be >= 1"; return -1; }
  const int64_t N = static_cast<int64_t>(nx) * ny * nz;
  if (ns > N) { err = "more coefficients than grid points"; return -1; }
  st.ns = ns;
  st.nb = nb;
  // range and uniqueness
  std::vector<int32_t> sorted(map, map + ns);
  for (int64_t g = 0; g < ns; ++g)
    if (map[g] < 0 || map[g] >= N) {
      char buf[128];
      std::snprintf(buf, sizeof buf, "map entry %lld = %d outside [0, %lld)", (long long)g, map[g],
                    (long long)N);
      err = buf;
      return -1;
    }
  std::sort(sorted.begin(), sorted.end());
  for (int64_t g = 1; g < ns; ++g)
    if (sorted[g] == sorted[g - 1]) {
      char buf[96];
      std::snprintf(buf, sizeof buf, "duplicate map entry %d", sorted[g]);
      err = buf;
      return -1;
    }
  // columns: distinct (x, y), ordered by (x, y)
  std::vector<int32_t> colkey(static_cast<size_t>(nx) * ny, -1);
  std::vector<char> xocc(nx, 0);
  for (int64_t g = 0; g < ns; ++g) {
    const int32_t v = map[g];
    const int x = v % nx, y = (v / nx) % ny;
    colkey[static_cast<size_t>(x) * ny + y] = 0;
    xocc[x] = 1;
  }
  st.xinv.assign(nx, -1);
  for (int x = 0; x < nx; ++x)
    if (xocc[x]) {
      st.xinv[x] = static_cast<int32_t>(st.xs.size());
      st.xs.push_back(x);
    }
  st.nslab = static_cast<int>(st.xs.size());
  int ncol = 0;
  for (int x = 0; x < nx; ++x)
    for (int y = 0; y < ny; ++y) {
      int32_t& k = colkey[static_cast<size_t>(x) * ny + y];
      if (k < 0) continue;
      k = ncol++;
      st.col_x.push_back(x);
      st.col_y.push_back(y);
      st.col_xi.push_back(st.xinv[x]);
    }
  st.ncol = ncol;
  st.slabstart.assign(st.nslab + 1, ncol);
  for (int c = ncol - 1; c >= 0; --c) st.slabstart[st.col_xi[c]] = c;
  st.colidx.assign(static_cast<size_t>(st.nslab) * ny, -1);
  for (int c = 0; c < ncol; ++c)
    st.colidx[static_cast<size_t>(st.col_xi[c]) * ny + st.col_y[c]] = c;
  st.slab_order.resize(st.nslab);
  for (int xi = 0; xi < st.nslab; ++xi) st.slab_order[xi] = xi;
  std::stable_sort(st.slab_order.begin(), st.slab_order.end(), [&st](int p, int q) {
    return st.slabstart[p + 1] - st.slabstart[p] > st.slabstart[q + 1] - st.slabstart[q];
  });
  st.gidx.assign(static_cast<size_t>(ncol) * nz, -1);
  st.entry_col.resize(ns);
  st.entry_z.resize(ns);
  for (int64_t g = 0; g < ns; ++g) {
    const int32_t v = map[g];
    const int x = v % nx, y = (v / nx) % ny, z = v / (nx * ny);
    const int c = colkey[static_cast<size_t>(x) * ny + y];
    st.gidx[static_cast<size_t>(c) * nz + z] = static_cast<int32_t>(g);
    st.entry_col[g] = c;
    st.entry_z[g] = z;
  }
  return 0;
}

}  // namespace fftb

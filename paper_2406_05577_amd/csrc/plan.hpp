// Host-side plan for the sphere<->grid transform: validation, column tables,
// radix plans and twiddle tables. Plain C++17, no HIP dependency, so the same
// code is compiled into the library and into host-only unit tests.
//
// The column table is the offset array of Section 3.3: the sphere projected
// on the xy-plane, z compressed, x and y dense. Every occupied (x,y) pair is a
// column; every occupied x is a slab. The plane kernel's y-transform runs only
// over the slabs and its x-transform over the full grid (staged padding of
// Section 2.2).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace fftb {

constexpr int kMaxStages = 8;
constexpr int kMaxRadix = 16;

// Radix plan of one axis (Stockham stages; stage s has radix R[s] and
// sub-transform length p[s] = R[0]*...*R[s-1]).
struct AxisPlan {
  int n = 1;
  int nst = 0;
  int R[kMaxStages] = {0};
  int p[kMaxStages] = {0};
  int twoff[kMaxStages] = {0};  // offset of stage s in the axis twiddle table
  int twlen = 0;                // total twiddle entries of the axis
};

// Factorise n (prime factors 2, 3, 5 only) into radices <= 16 with the fewest
// stages; returns false if n has another prime factor. `prefer` optionally
// fixes the order (largest radix first by default).
bool plan_radices(int n, std::vector<int>& radices);
void make_axis_plan(int n, const std::vector<int>& radices, AxisPlan& ap);

// Forward-sign twiddles exp(-2*pi*i*q*k/(p*R)) for every stage, k < p, q < R,
// laid out stage by stage as [k*R + q]; the angle is formed from (q*k) mod
// (p*R) reduced in integers. Returned as (re, im) pairs of double.
std::vector<double> axis_twiddles(const AxisPlan& ap);
// exp(-2*pi*i*j/n), j < n.
std::vector<double> root_table(int n);

struct SphereTables {
  int64_t ns = 0;
  int nb = 0;
  double kpt[3] = {0, 0, 0};
  int ncol = 0, nslab = 0;
  std::vector<int32_t> col_x, col_y;   // per column, grid coordinates
  std::vector<int32_t> col_xi;         // slab index of each column
  std::vector<int32_t> xs;             // occupied x, ascending (nslab)
  std::vector<int32_t> xinv;           // nx entries: slab index or -1
  std::vector<int32_t> slabstart;      // nslab+1 entries: first column of each slab
  std::vector<int32_t> colidx;         // nslab*ny: column index or -1
  std::vector<int32_t> slab_order;     // slab indices by descending column count
  std::vector<int32_t> gidx;           // ncol*nz: coefficient index or -1
  std::vector<int32_t> entry_col, entry_z;  // per coefficient
};

// Validate one map and build its tables. Returns 0 on success, -1 (invalid)
// with a message in err.
int build_sphere_tables(int nx, int ny, int nz, const int32_t* map, int64_t ns, int nb,
                        SphereTables& st, std::string& err);

}  // namespace fftb

// C ABI of the sphere<->grid transform: plan creation (validation, tables,
// tiling, device uploads), execution, introspection and clean-up.
//
// The plan object mirrors the create / execute / clean-up model of the
// paper's transform object (Section 3.1); an input the library has no stage
// pattern for is rejected with FFTB_ERR_UNSUPPORTED, the analog of the
// exception the paper's framework raises for patterns outside its predefined
// list (Section 3.1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/fftb.h"
#include "kargs.hpp"
#include "plan.hpp"

namespace fftb {
hipError_t prepare_kernels(bool fp64, size_t lds1, size_t lds2);
hipError_t launch_reset(unsigned int* counters, hipStream_t st);
hipError_t launch_kernel(int which, const KArgs& a, bool inverse, bool fp64, int grid, int threads,
                         size_t lds, hipStream_t st);
bool reg_shape_supported(bool fp64, int E, int H);
hipError_t launch_reg(int which, const KArgs& a, bool inverse, bool fp64, int E, int H, int grid,
                      int threads, size_t lds, hipStream_t st, bool mfma, int fold_m);
hipError_t prepare_reg(bool fp64, int E, int H, size_t lds, bool mfma);
bool mfma_shape_supported(bool fp64, int E, int H);
bool fold_m_supported(int H, int m);
hipError_t launch_combine(const KArgs& a, bool fp64, int grid, int threads, hipStream_t st);
hipError_t static_scratch_ptr(void** out);
bool bil_shape_supported(bool fp64, bool zaxis, int E, int H);
bool bil_narrow_supported(bool fp64, int E, int H);
hipError_t launch_bil(int which, const KArgs& a, bool inverse, bool fp64, int E, int H, int grid,
                      int threads, size_t lds, hipStream_t st, int fold_m);
hipError_t prepare_bil(bool fp64, int E, int H, size_t lds, bool narrow);
hipError_t launch_zero_scratch(void* p, size_t bytes, hipStream_t st);
}  // namespace fftb

using namespace fftb;

extern "C" fftb_status fftb_plan_create(fftb_plan*, const int32_t[3], const fftb_sphere*, int32_t,
                                        fftb_dtype, uint32_t, const fftb_tuning*, void*);

namespace {

thread_local std::string g_last_error;

fftb_status fail(fftb_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

// Column scratch shared by the autotuner's trial plans: set while the trials
// run on this thread, so that each trial borrows it (growing it when a trial
// needs more) instead of allocating and freeing its own.
struct TuneScratch {
  void* p = nullptr;
  size_t bytes = 0;
};
thread_local TuneScratch* g_tune_scratch = nullptr;

// Upper bound on the device memory one plan may hold (FFTB_MAX_DEVICE_BYTES,
// bytes; unset or 0 = no bound). A plan that would exceed it fails with
// FFTB_ERR_NOMEM before any device call.
size_t device_byte_cap() {
  const char* v = std::getenv("FFTB_MAX_DEVICE_BYTES");
  if (!v || !*v) return 0;
  return static_cast<size_t>(std::strtoull(v, nullptr, 10));
}

constexpr size_t kLdsMax = 160 * 1024 - 1024;  // leave room for static LDS

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// Tiling and task decomposition of one direction.
struct DirCfg {
  int bc = 8, n1 = 1, m = 1, lx = 1, lc = 1, threads = 256;
  int bc2 = 0;                      // plane kernel's band chunk when it differs (0 = bc)
  bool narrow = false;              // band-inner inverse plane kernel on half pieces
  int qc = 1;                       // inverse band-inner: y classes per plane task (2: pairs)
  int ovf_lines = 0;                // class pairs: lines per task held in the overflow scratch
  int64_t ovf_off = 0;              // class pairs: overflow scratch offset in the column region
  bool reg1 = false, reg2 = false;  // register path for the column / plane kernel
  bool mf1 = false, mf2 = false;    // DFT_16 stages on the matrix cores
  bool bil1 = false, bil2 = false;  // band-inner lines (column / plane kernel)
  int lds_twx = 0, zline = 0;       // band-inner plane kernel: twiddle table (bytes), spare line
  int e1 = 0, h1 = 0, e2 = 0, h2 = 0;
  bool class_par = false;           // plane tasks include the y class
  bool acc_lds = false;             // forward accumulators in LDS
  bool fwd_cls = false;             // forward class partials, combined by the column kernel
  int fold_m = 0;                   // inverse: compile-time class length of the fold (0 = generic)
  int nsplit = 1;                   // forward plane tasks per (plane, chunk)
  std::vector<int32_t> splits;      // per sphere nsplit+1 slab boundaries
  int sx = 0;
  size_t lds1 = 0, lds2 = 0;
  int lds_P = 0, lds_X0 = 0, lds_X1 = 0, lds_acc = 0, lds_tab = 0;
  AxisPlan ay;                      // y plan of length m
  std::vector<SphereDesc> desc;
  int k1_tasks = 0, k2_tasks = 0, k3_tasks = 0;
  int64_t col_elems = 0;
  SphereDesc* d_desc = nullptr;
  int32_t* d_splits = nullptr;
  void* d_twy = nullptr;
  void* d_twy_lo = nullptr;
};

}  // namespace

struct fftb_plan_s {
  int nx = 0, ny = 0, nz = 0;
  fftb_dtype dtype = FFTB_C128;
  uint32_t flags = 0;
  std::vector<SphereTables> sph;
  AxisPlan ax, az;
  DirCfg dir[2];  // 0 = inverse (sphere_to_grid), 1 = forward
  fftb_tuning tun = {};
  int64_t sphere_elems = 0, grid_elems = 0;
  int64_t total_coeffs = 0, total_columns = 0;
  int max_ncol = 0, max_nslab = 0;
  int autotuned = 0;
  bool device = false;
  int num_cus = 256;
  // device memory
  std::vector<DevBuf> bufs;
  int32_t *d_gidx = nullptr, *d_colidx = nullptr, *d_colxi = nullptr, *d_coly = nullptr,
          *d_xinv = nullptr, *d_slabstart = nullptr, *d_colslot = nullptr, *d_slabblk = nullptr,
          *d_slabnblk = nullptr, *d_slaborder = nullptr;
  // column scratch slots: with pad_m > 0 every slab's columns sit in zero-padded
  // blocks of pad_m consecutive y (the inverse fold reads whole blocks)
  int pad_m = 0;
  std::vector<int32_t> col_slot, slab_blk, slab_nblk, colidx_slot;  // concatenated over spheres
  std::vector<int32_t> npcol;                            // per sphere
  void *d_twx = nullptr, *d_twz = nullptr, *d_twf = nullptr;
  void *d_twx_lo = nullptr, *d_twz_lo = nullptr, *d_twf_lo = nullptr;
  void *d_rootx = nullptr, *d_rootx_lo = nullptr, *d_rootz = nullptr, *d_rootz_lo = nullptr;
  void* d_col = nullptr;
  unsigned int* d_counters = nullptr;
  size_t dev_bytes = 0;
  // graph cache per direction
  struct GraphCache {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    const void* in = nullptr;
    void* out = nullptr;
    const void* pot = nullptr;
  } gc[2];
  hipStream_t cap_stream = nullptr;
  // per-kernel timing
  bool profiling = false;
  struct ProfRec {
    int kid;
    hipEvent_t a, b;
  };
  std::vector<ProfRec> prof_pending;
  std::vector<hipEvent_t> ev_pool;
  int64_t prof_launches[5] = {0, 0, 0, 0, 0};
  double prof_ms[5] = {0, 0, 0, 0, 0};

  ~fftb_plan_s() {
    for (auto& r : prof_pending) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (auto e : ev_pool) (void)hipEventDestroy(e);
    for (auto& g : gc) {
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
      if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (auto& b : bufs)
      if (b.p) (void)hipFree(b.p);
  }
};

namespace {

int es_of(fftb_dtype dt) { return dt == FFTB_C128 ? 16 : 8; }
int nbuf_of(int nst) { return nst >= 3 ? 2 : (nst == 2 ? 1 : 0); }
int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}
bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
bool single_codelet(int m) {
  switch (m) {
    case 1: case 2: case 3: case 4: case 5: case 6: case 8: case 9: case 10: case 12: case 15:
    case 16:
      return true;
  }
  return false;
}
// class counts the forward combine has a codelet for
bool combine_codelet(int c) { return c == 18 || c == 20 || single_codelet(c); }

// Register shape (E values per lane, H lanes per line) for a line of length n:
// the most lanes with a compiled shape, or exactly `lanes` if given. Lines of
// 12 lanes (a radix-3 step across lane groups) serve the column kernel only and
// only on request (allow12 = the lanes knob asks for 12): their bands are spread
// over four waves, which measured slower than 4-lane lines at 180 points.
bool reg_shape(int n, bool fp64, int& E, int& H, int lanes = 0, bool allow12 = false) {
  for (int h : {16, 12, 8, 4, 2, 1}) {
    if (h == 12 && !(allow12 && lanes == 12)) continue;
    if (lanes && h != lanes) continue;
    if (n % h) continue;
    if (reg_shape_supported(fp64, n / h, h)) {
      E = n / h;
      H = h;
      return true;
    }
  }
  return false;
}

// LDS bytes of the LDS-stage plane kernel for class count n1 and x batch lx.
bool plane_lds_generic(const fftb_plan_s& P, int n1, int bc, int lx, size_t& bytes, int& offP,
                       int& offX0, int& offX1, AxisPlan& aym) {
  const int m = P.ny / n1;
  std::vector<int> rad;
  if (!plan_radices(m, rad)) return false;
  make_axis_plan(m, rad, aym);
  const int64_t S = static_cast<int64_t>(P.max_nslab) * m * bc;
  const int64_t Pn = aym.nst >= 2 ? S : 0;
  const int nbx = nbuf_of(P.ax.nst);
  const int64_t X = static_cast<int64_t>(lx) * P.nx * bc;
  offP = static_cast<int>(S);
  offX0 = static_cast<int>(S + Pn);
  offX1 = static_cast<int>(S + Pn + (nbx >= 1 ? X : 0));
  bytes = static_cast<size_t>(S + Pn + nbx * X) * es_of(P.dtype);
  return true;
}

// LDS of the register-path plane kernel: the class slab (nslab lines of m
// values for bc bands, line stride padded by one element) plus, in the forward
// direction with accumulators in LDS, ncol x bc accumulators.
size_t plane_lds_reg(const fftb_plan_s& P, int m, int bc, bool acc, int& sx, int& off_acc) {
  sx = m * bc + 1;
  const int64_t S = static_cast<int64_t>(P.max_nslab) * sx;
  off_acc = static_cast<int>(S);
  const int64_t A = acc ? static_cast<int64_t>(P.max_ncol) * bc : 0;
  return static_cast<size_t>(S + A) * es_of(P.dtype);
}

// Element stride between band vectors in the column scratch and the class
// partials: the band chunks of all bands, plus one 128-byte line when the
// stride is a multiple of 256 bytes (runs of equal stride then spread over the
// L2 channels instead of landing on one; measured 5 % per round trip at C2).
int64_t band_stride(int64_t nb, int bc, int es) {
  const int64_t n = (nb + bc - 1) / bc * bc;
  return (n * es) % 256 == 0 ? n + 128 / es : n;
}

// Slots of the padded layout stay below 2^21 (they are packed with the block
// index), and one plane of the column scratch below 2 GiB (the fold addresses
// it with 32-bit buffer offsets).
int64_t padded_slots(const SphereTables& s, int M);

bool fold_slots_fit(const fftb_plan_s& P, int M, int bc) {
  for (auto& s : P.sph) {
    const int64_t slots = padded_slots(s, M);
    if (slots >= (int64_t{1} << 21)) return false;
    const int64_t nbp = band_stride(s.nb, bc, es_of(P.dtype));
    if (slots * nbp * es_of(P.dtype) >= (int64_t{1} << 31)) return false;
  }
  return true;
}

// LDS of the inverse fold's staged tables: per slab n1 block entries, a count
// and the slab order, then n1 roots (hi and lo) of the class and its m
// twiddles (FP32: hi and lo).
size_t fold_table_bytes(const fftb_plan_s& P, int n1, bool pair = false) {
  const size_t ints = ((static_cast<size_t>(P.max_nslab) * n1 + 3) & ~size_t{3}) +
                      2 * ((P.max_nslab + 3) & ~3);
  // class pairs: the second class's twiddles too
  return ints * 4 + static_cast<size_t>(2 * n1 + (pair ? 4 : 2) * (P.ny / n1)) * es_of(P.dtype);
}

// Band-inner shape of a line of length n: H = 4 positions (complex64) or 8
// (complex128), so that one line fills a wavefront; complex128 z lines may
// also take 4 positions (two lines per wavefront, e.g. 180 = 45 x 4).
bool bil_shape(int n, bool fp64, bool zaxis, int& E, int& H) {
  for (int h : {fp64 ? 8 : 4, (fp64 && zaxis) ? 4 : 0}) {
    if (!h || n % h || !bil_shape_supported(fp64, zaxis, n / h, h)) continue;
    E = n / h;
    H = h;
    return true;
  }
  return false;
}

// Column slots of one plane of a sphere when its columns sit in zero-padded
// blocks of M consecutive y (M = 16 bounds every layout the plans use).
int64_t padded_slots(const SphereTables& s, int M) {
  int64_t slots = 0;
  for (int xi = 0; xi < s.nslab; ++xi) {
    int cur = -1;
    for (int c = s.slabstart[xi]; c < s.slabstart[xi + 1]; ++c)
      if (s.col_y[c] / M != cur) {
        cur = s.col_y[c] / M;
        slots += M;
      }
  }
  return slots;
}

// The band-inner kernels address every grid plane, column plane and class
// partial plane with 32-bit offsets (below 2 GiB) and every sphere's
// coefficients and column region below 4 GiB (columns in padded blocks of at
// most M consecutive y).
bool bil_regions_fit(const fftb_plan_s& P, int bw, int M = 16) {
  const int64_t es = es_of(P.dtype);
  for (const auto& sp : P.sph) {
    const int64_t nbp = band_stride(sp.nb, bw, es);
    const int64_t colplane = padded_slots(sp, M) * nbp * es;
    const int64_t zplane = static_cast<int64_t>(sp.nslab) * P.ny * nbp * es;
    const int64_t gplane = static_cast<int64_t>(P.nx) * P.ny * sp.nb * es;
    if (std::max(colplane, std::max(zplane, gplane)) >= (int64_t{1} << 31)) return false;
    if (sp.ns * sp.nb * es >= 0xffffffffLL || colplane * P.nz >= 0xffffffffLL) return false;
  }
  return true;
}

// LDS of the band-inner plane kernel with class length m: the class slab
// (max_nslab lines of m x bw values, plus the spare line), then (inverse) the
// fold tables, then the E x H twiddle table of the x lines.
size_t plane_lds_bil(const fftb_plan_s& P, int n1, int bw, int e2, int h2, bool inverse,
                     int& sx, int& tab_at, int& tw_at, bool pair = false) {
  const int m = P.ny / n1;
  sx = m * bw;
  size_t b = static_cast<size_t>(P.max_nslab + 1) * sx * es_of(P.dtype);
  b = (b + 15) & ~size_t{15};
  tab_at = static_cast<int>(b);
  // inverse: the fold tables; forward: the class twiddles (FP32 hi and lo)
  if (inverse) b = (b + fold_table_bytes(P, n1, pair) + 15) & ~size_t{15};
  else b = (b + static_cast<size_t>(2 * m) * es_of(P.dtype) + 15) & ~size_t{15};
  tw_at = static_cast<int>(b);
  // the twiddle table (lines of more than one position), then the slab-line
  // offsets of the nx x positions
  return b + (h2 > 1 ? static_cast<size_t>(tw_row_stride(e2)) * h2 * 16 : 0) + static_cast<size_t>(P.nx) * 4;
}

// Cut a sphere's slabs into Q contiguous ranges with about equal column counts.
void split_slabs(const SphereTables& sp, int Q, std::vector<int32_t>& cuts) {
  cuts.assign(Q + 1, sp.nslab);
  cuts[0] = 0;
  int q = 1;
  for (int xi = 0; xi < sp.nslab && q < Q; ++xi) {
    // cut after slab xi once the columns so far reach q/Q of the total
    if (static_cast<int64_t>(sp.slabstart[xi + 1]) * Q >= static_cast<int64_t>(sp.ncol) * q) {
      cuts[q++] = xi + 1;
    }
  }
  for (; q < Q; ++q) cuts[q] = sp.nslab;
}

int default_bc(const fftb_plan_s& P, int want) {
  int maxnb = 1;
  for (auto& s : P.sph) maxnb = std::max(maxnb, s.nb);
  int cap = 1;
  while (cap < maxnb) cap <<= 1;
  return std::min(want, cap);
}

fftb_status choose_dir(fftb_plan_s& P, int d, const fftb_dir_tuning& t) {
  DirCfg& D = P.dir[d];
  const bool fp64 = P.dtype == FFTB_C128;
  const bool inverse = d == 0;
  const int es = es_of(P.dtype);
  int bc = t.band_chunk;
  int n1 = t.y_classes;
  if (bc == 0) bc = default_bc(P, fp64 ? 8 : 16);
  if (!is_pow2(bc) || bc > 64)
    return fail(FFTB_ERR_INVALID, "band_chunk must be a power of two in [1, 64]");
  int threads = t.threads ? t.threads : 256;
  if (threads != 64 && threads != 128 && threads != 256 && threads != 512)
    return fail(FFTB_ERR_INVALID, "threads must be 64, 128, 256 or 512");
  if (n1 != 0 && (n1 < 1 || P.ny % n1)) return fail(FFTB_ERR_INVALID, "y_classes must divide ny");
  if (t.path < 0 || t.path > 3) return fail(FFTB_ERR_INVALID, "path must be 0, 1, 2 or 3");
  if (t.acc < 0 || t.acc > 3) return fail(FFTB_ERR_INVALID, "acc must be 0, 1, 2 or 3");
  if (t.splits < 0 || t.splits > 8) return fail(FFTB_ERR_INVALID, "splits must be in [1, 8]");
  if (t.col_tile < 0) return fail(FFTB_ERR_INVALID, "col_tile must be >= 1");
  if (t.x_rows < 0) return fail(FFTB_ERR_INVALID, "x_rows must be >= 1");
  D.bc = bc;
  D.bc2 = 0;
  D.narrow = false;
  D.qc = 1;
  D.threads = threads;
  D.bil1 = D.bil2 = false;
  D.mf1 = D.mf2 = false;
  // ---- band-inner lines (path 3, and the default where the shapes exist):
  // the band chunk is one 128-byte piece; the complex64 inverse plane kernel
  // may take half of one (band_chunk = 8: x lines over twice the positions,
  // the fold over classes of 16 or 32; the column kernel keeps whole pieces)
  const int bw = fp64 ? 8 : 16;
  const bool narrow = inverse && t.band_chunk == bw / 2;
  const bool mfma = (P.flags & FFTB_PLAN_MFMA) != 0;
  const bool bil_ok = (t.path == 0 || t.path == 3) &&
                      (t.band_chunk == 0 || t.band_chunk == bw || narrow) && (t.lanes == 0) &&
                      !(mfma && fp64) && bil_regions_fit(P, bw);
  if (bil_ok) {
    int e1 = 0, h1 = 0, e2 = 0, h2 = 0;
    // the column kernel takes the band-inner shape of z, else a register shape
    const bool z_bil = bil_shape(P.nz, fp64, true, e1, h1);
    const bool z_ok = z_bil || reg_shape(P.nz, fp64, e1, h1, 0, true);
    bool x_ok;
    if (narrow) {
      h2 = 8;
      e2 = P.nx / h2;
      x_ok = P.nx % h2 == 0 && bil_narrow_supported(fp64, e2, h2);
    } else {
      x_ok = bil_shape(P.nx, fp64, false, e2, h2);
    }
    const int bwp = narrow ? bw / 2 : bw;  // the plane kernel's band chunk
    if (z_ok && x_ok) {
      // inverse: the fewest classes whose slab fits (every class re-reads the
      // plane's columns) with a register fold of length 8 or 16 (narrow: 16
      // or 32); forward: the fewest classes with a combine codelet, two
      // workgroups per CU if possible
      int best_n1 = 0, sx = 0, tab_at = 0, tw_at = 0;
      size_t best_b = 0;
      for (size_t cap : {(n1 || inverse) ? kLdsMax : kLdsMax / 2, kLdsMax}) {
        for (int c = 1; c <= P.ny && !best_n1; ++c) {
          if (P.ny % c || (n1 && c != n1)) continue;
          const int m = P.ny / c;
          const bool fold_ok = narrow ? (m == 16 || m == 32) : (m == 8 || m == 16);
          if (inverse ? !fold_ok || !fold_slots_fit(P, m, bw) || !bil_regions_fit(P, bw, m)
                      : !single_codelet(m) || !combine_codelet(c))
            continue;
          const size_t b = plane_lds_bil(P, c, bwp, e2, h2, inverse, sx, tab_at, tw_at);
          if (b > cap) continue;
          best_n1 = c;
          best_b = b;
        }
        if (best_n1) break;
      }
      // with FFTB_PLAN_MFMA the inverse takes band-inner lines only with its
      // fold of length 16 on the matrix cores, the forward only where the
      // register lines have no matrix-core stage
      const bool mf_fold = mfma && inverse && !narrow && best_n1 && P.ny / best_n1 == 16;
      if (mfma && inverse && !mf_fold) best_n1 = 0;
      if (mfma && !inverse) {
        int er = 0, hr = 0;
        if (reg_shape(P.nx, fp64, er, hr, 8, false) && mfma_shape_supported(fp64, er, hr)) best_n1 = 0;
      }
      if (best_n1) {
        // inverse class pairs (r, r + n1/2 per task: one read of the plane's
        // columns serves both) where the fold has length 16 and the second
        // class's twiddles fit
        bool pair = false;
        if (inverse && !narrow && t.acc != 1 && best_n1 % 2 == 0 && P.ny / best_n1 == 16) {
          int sx2 = 0, tab2 = 0, tw2 = 0;
          pair = plane_lds_bil(P, best_n1, bwp, e2, h2, true, sx2, tab2, tw2, true) <= kLdsMax;
        }
        if (inverse && t.acc == 2 && !pair)
          return fail(FFTB_ERR_UNSUPPORTED, "class pairs need an even class count with classes of 16");
        best_b = plane_lds_bil(P, best_n1, bwp, e2, h2, inverse, sx, tab_at, tw_at, pair);
        D.qc = pair ? 2 : 1;
        D.mf1 = false;
        D.mf2 = mf_fold;
        D.bc = bw;
        D.bc2 = bwp;
        D.narrow = narrow;
        D.bil1 = z_bil;
        D.bil2 = D.reg1 = D.reg2 = true;
        D.e1 = e1;
        D.h1 = h1;
        D.e2 = e2;
        D.h2 = h2;
        D.lc = t.col_tile ? t.col_tile
                          : z_bil ? 8 * std::max(1, 64 / (bw * h1))
                                  : std::max(1, 512 / (bw * (h1 == 12 ? 16 : h1)));
        D.lds1 = 0;
        D.n1 = best_n1;
        D.m = P.ny / best_n1;
        D.sx = sx;
        D.lds2 = best_b;
        D.lds_tab = tab_at;
        D.lds_twx = tw_at;
        D.zline = P.max_nslab * sx;
        D.class_par = true;
        D.fwd_cls = !inverse;
        // inverse: the fold's class length; forward: the y transform's, where
        // compiled (8, 12, 16)
        D.fold_m = (inverse || D.m == 8 || D.m == 12 || D.m == 16) ? D.m : 0;
        D.acc_lds = false;
        D.nsplit = 1;
        std::vector<int> rad;
        plan_radices(D.m, rad);
        make_axis_plan(D.m, rad, D.ay);
        if (!t.threads && D.lds2 > kLdsMax / 2) D.threads = 512;
        // the complex64 forward kernel stays within 128 registers per lane:
        // two workgroups of 512 threads per CU (measured 5 % faster per round
        // trip on the 144x160x180 workload than two of 256)
        if (!t.threads && !inverse && !fp64) D.threads = 512;
        return FFTB_OK;
      }
    }
    if (t.path == 3)
      return fail(FFTB_ERR_UNSUPPORTED, mfma ? "no band-inner plan with a matrix-core stage fits"
                                             : "no band-inner line shape or class split fits");
  }
  // ---- column kernel
  int e1 = 0, h1 = 0;
  if (t.lanes != 0 && t.lanes != 1 && t.lanes != 4 && t.lanes != 8 && t.lanes != 12 &&
      t.lanes != 16)
    return fail(FFTB_ERR_INVALID, "lanes must be 0, 1, 4, 8, 12 or 16");
  // the matrix-core DFT_16 runs on lines of 16 values per lane over 8 lanes
  const int lanes = t.lanes ? t.lanes : ((P.flags & FFTB_PLAN_MFMA) && !fp64 ? 8 : 0);
  D.reg1 = t.path != 1 && (reg_shape(P.nz, fp64, e1, h1, lanes, true) ||
                           reg_shape(P.nz, fp64, e1, h1, 0, true));
  D.e1 = e1;
  D.h1 = h1;
  if (D.reg1) {
    D.lc = t.col_tile ? t.col_tile : std::max(1, 512 / (bc * (h1 == 12 ? 16 : h1)));
    D.lds1 = 0;
  } else {
    const int nbz = nbuf_of(P.az.nst);
    int lc = t.col_tile;
    if (lc == 0) {
      if (nbz == 0) {
        lc = 16;
      } else {
        const int64_t per = static_cast<int64_t>(nbz) * P.nz * bc * es;
        lc = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(16, (64 * 1024) / per)));
      }
    }
    D.lc = lc;
    D.lds1 = static_cast<size_t>(nbz) * lc * P.nz * bc * es;
  }
  if (D.lds1 > kLdsMax) return fail(FFTB_ERR_UNSUPPORTED, "column kernel tile does not fit in LDS");
  // ---- plane kernel, register path
  int e2 = 0, h2 = 0;
  D.reg2 = false;
  // class-parallel tasks (plane, chunk, class): the class slab must fit (aim for
  // two workgroups per CU unless the class count is fixed)
  // want_fold_m: only class lengths with a compiled inverse fold; want_codelet:
  // only class counts with a DFT codelet (the forward combine)
  // (inverse: the fewest classes that fit, since every class re-reads the
  // plane's columns; forward: fit two workgroups per CU where possible)
  auto pick_classes = [&](bool want_fold_m, bool want_codelet) {
    for (size_t cap : {(n1 || inverse) ? kLdsMax : kLdsMax / 2, kLdsMax}) {
      for (int c = 1; c <= P.ny; ++c) {
        if (P.ny % c || (n1 && c != n1)) continue;
        const int m = P.ny / c;
        if (!single_codelet(m)) continue;
        if (want_fold_m && !fold_m_supported(h2, m)) continue;
        if (want_codelet && !single_codelet(c)) continue;
        int sx, oa;
        size_t b = plane_lds_reg(P, m, bc, false, sx, oa);
        const size_t tab_at = (b + 15) & ~size_t{15};
        if (want_fold_m) b = tab_at + fold_table_bytes(P, c);
        if (b > cap) continue;
        D.reg2 = true;
        D.n1 = c;
        D.m = m;
        D.lds2 = b;
        D.lds_tab = static_cast<int>(tab_at);
        D.sx = sx;
        D.class_par = true;
        return;
      }
    }
  };
  D.fwd_cls = false;
  D.fold_m = 0;
  if (t.path != 1 && (reg_shape(P.nx, fp64, e2, h2, lanes) || reg_shape(P.nx, fp64, e2, h2))) {
    if (inverse) {
      // prefer a class length with a compiled register fold
      pick_classes(true, false);
      if (!D.reg2) pick_classes(false, false);
      D.fold_m = D.reg2 && fold_m_supported(h2, D.m) && D.n1 <= 1024 && fold_slots_fit(P, D.m, D.bc)
                     ? D.m : 0;
      if (D.reg2 && !D.fold_m) {
        // the generic fold needs no staged tables
        pick_classes(false, false);
      }
    } else if ((t.acc == 0 || t.acc == 3) && t.splits <= 1) {
      // class partials combined by a separate kernel: no accumulators; a class
      // count with a DFT codelet for the combine, halving the band chunk once
      // if none fits
      pick_classes(false, true);
      if (!D.reg2 && !t.band_chunk && bc > 1) {
        bc /= 2;
        D.bc = bc;
        pick_classes(false, true);
        if (!D.reg2) {
          bc *= 2;
          D.bc = bc;
        }
      }
      if (!D.reg2) pick_classes(false, false);
      D.fwd_cls = D.reg2;
      if (!D.reg2 && t.acc == 3)
        return fail(FFTB_ERR_UNSUPPORTED, "no class slab fits in LDS");
    } else if (t.acc == 3) {
      return fail(FFTB_ERR_UNSUPPORTED, "class partials take one column split");
    }
    if (!inverse && !D.reg2) {
      // forward: the plane's columns are split into nsplit slab ranges whose
      // accumulators (LDS) and class slab fit; each split redoes the x transform of
      // the class rows. Cost model: HBM segment efficiency x redundant x work x
      // occupancy; global accumulators (no split) are the fallback.
      double best = 1e30;
      const int bc_lo = t.band_chunk ? bc : std::max(1, bc / 2);
      for (int b = bc; b >= bc_lo; b >>= 1) {
        const int seg = b * es;
        const double eff = seg >= 128 ? 1.0 : seg >= 64 ? 1.1 : seg >= 32 ? 1.5 : 3.0;
        for (int c = 1; c <= P.ny; ++c) {
          if (P.ny % c || (n1 && c != n1)) continue;
          const int m = P.ny / c;
          if (!single_codelet(m)) continue;
          for (int Q = t.splits ? t.splits : 1; Q <= 8; ++Q) {
            if (t.acc == 2 && Q > 1) break;
            int max_sl = 0, max_cl = 0;
            for (auto& sp : P.sph) {
              std::vector<int32_t> cuts;
              split_slabs(sp, Q, cuts);
              for (int q = 0; q < Q; ++q) {
                max_sl = std::max(max_sl, cuts[q + 1] - cuts[q]);
                max_cl = std::max(max_cl, sp.slabstart[cuts[q + 1]] - sp.slabstart[cuts[q]]);
              }
            }
            const int sx = m * b + 1;
            const bool acc = t.acc != 2;
            const size_t bytes = (static_cast<size_t>(max_sl) * sx +
                                  (acc ? static_cast<size_t>(max_cl) * b : 0)) * es;
            if (bytes > kLdsMax) continue;
            // each class costs a pass over the split's accumulators and two barriers
            const double cost = eff * (1.0 + 0.12 * (Q - 1)) * (1.0 + 0.03 * c) *
                                (bytes > kLdsMax / 2 ? 1.15 : 1.0) * (acc ? 1.0 : 4.0);
            if (cost < best) {
              best = cost;
              D.reg2 = true;
              D.bc = b;
              D.n1 = c;
              D.m = m;
              D.nsplit = Q;
              D.acc_lds = acc;
              D.sx = sx;
              D.lds_acc = max_sl * sx;
              D.lds2 = bytes;
              D.class_par = false;
            }
            break;  // larger Q only adds work once this one fits
          }
        }
      }
      if (D.reg2) bc = D.bc;
    }
    if (D.reg2) {
      D.e2 = e2;
      D.h2 = h2;
      std::vector<int> rad;
      plan_radices(D.m, rad);
      make_axis_plan(D.m, rad, D.ay);
      if (D.reg1 && !t.col_tile) D.lc = std::max(1, 512 / (bc * (h1 == 12 ? 16 : h1)));
    } else if (t.path == 2) {
      return fail(FFTB_ERR_UNSUPPORTED, "no register-path class split fits in LDS");
    }
  } else if (t.path == 2) {
    return fail(FFTB_ERR_UNSUPPORTED, "x length has no register-path shape");
  }
  if (t.path == 2 && !D.reg1) return fail(FFTB_ERR_UNSUPPORTED, "z length has no register-path shape");
  if (P.flags & FFTB_PLAN_MFMA) {
    if (fp64) return fail(FFTB_ERR_UNSUPPORTED, "matrix-core DFT_16 stages are FP32 only");
    D.mf1 = D.reg1 && mfma_shape_supported(fp64, D.e1, D.h1);
    D.mf2 = D.reg2 && mfma_shape_supported(fp64, D.e2, D.h2);
    if (!D.mf1 && !D.mf2)
      return fail(FFTB_ERR_UNSUPPORTED, "no in-lane DFT_16 stage for the matrix cores in this plan");
  }
  if (D.reg2) {
    // a class slab that leaves room for one workgroup per CU: twice the waves
    // per workgroup (measured faster for the inverse of the FP32
    // configurations and the 96^3 FP64 one, and picked by the autotuner for
    // both directions of the 144x160x180 one)
    if (!t.threads && D.lds2 > kLdsMax / 2) D.threads = 512;
    return FFTB_OK;
  }
  // ---- plane kernel, LDS-stage path
  int lx = t.x_rows;
  AxisPlan aym;
  size_t bytes = 0;
  int offP = 0, offX0 = 0, offX1 = 0;
  if (n1 == 0) {
    n1 = -1;
    for (int c = 1; c <= P.ny; ++c) {
      if (P.ny % c) continue;
      const int m = P.ny / c;
      const int want = std::min(m, lx ? lx : 2);
      if (!plane_lds_generic(P, c, bc, want, bytes, offP, offX0, offX1, aym)) continue;
      if (bytes <= kLdsMax) {
        n1 = c;
        break;
      }
    }
    if (n1 < 0) return fail(FFTB_ERR_UNSUPPORTED, "no y-class split fits the plane in LDS");
  }
  const int m = P.ny / n1;
  if (lx == 0) {
    lx = 1;
    for (int c = m; c >= 1; --c) {
      if (!plane_lds_generic(P, n1, bc, c, bytes, offP, offX0, offX1, aym)) break;
      if (bytes <= kLdsMax / 2 || c == 1) {
        lx = c;
        break;
      }
    }
  }
  lx = std::min(lx, m);
  if (!plane_lds_generic(P, n1, bc, lx, bytes, offP, offX0, offX1, aym))
    return fail(FFTB_ERR_UNSUPPORTED, "class length has an unsupported factor");
  if (bytes > kLdsMax) return fail(FFTB_ERR_UNSUPPORTED, "plane kernel tile does not fit in LDS");
  D.n1 = n1;
  D.m = m;
  D.lx = lx;
  // the LDS-stage kernels are compiled for at most 256 threads per workgroup
  D.threads = std::min(D.threads, 256);
  D.ay = aym;
  D.lds2 = bytes;
  D.lds_P = offP;
  D.lds_X0 = offX0;
  D.lds_X1 = offX1;
  D.class_par = false;
  D.acc_lds = false;
  return FFTB_OK;
}

void fill_axis(const AxisPlan& a, AxisDev& d) {
  std::memset(&d, 0, sizeof d);
  d.n = a.n;
  d.nst = a.nst;
  for (int s = 0; s < a.nst; ++s) {
    d.R[s] = a.R[s];
    d.p[s] = a.p[s];
    d.twoff[s] = a.twoff[s];
  }
}

// Column scratch slots. With M = pad_m > 0, slab xi's columns occupy blocks of
// M slots, one block per M-aligned run of y (y = tb*M .. tb*M + M - 1) that
// holds a column, in ascending y; slots of absent y stay zero (the scratch is
// cleared once at plan creation and no kernel writes them). slab_blk gives the
// per slab the list of its blocks as (first slot << 10 | tb) and their count.
// M = 0: slot = column.
void build_slots(fftb_plan_s& P) {
  const int M = P.pad_m;
  const int nblk = M > 0 ? P.ny / M : 0;
  P.col_slot.clear();
  P.slab_blk.clear();
  P.slab_nblk.clear();
  P.colidx_slot.clear();
  P.npcol.clear();
  for (auto& s : P.sph) {
    std::vector<int32_t> slot(s.ncol);
    int next = 0;
    if (M > 0) {
      // per slab: the blocks holding columns, ascending, as (first slot << 10 | tb)
      std::vector<int32_t> list(static_cast<size_t>(s.nslab) * nblk, -1);
      for (int xi = 0; xi < s.nslab; ++xi) {
        int n = 0, cur_tb = -1, cur_slot = 0;
        for (int c = s.slabstart[xi]; c < s.slabstart[xi + 1]; ++c) {
          const int tb = s.col_y[c] / M;
          if (tb != cur_tb) {
            cur_tb = tb;
            cur_slot = next;
            next += M;
            list[static_cast<size_t>(xi) * nblk + n++] = (cur_slot << 10) | tb;
          }
          slot[c] = cur_slot + (s.col_y[c] - tb * M);
        }
        P.slab_nblk.push_back(n);
      }
      P.slab_blk.insert(P.slab_blk.end(), list.begin(), list.end());
    } else {
      for (int c = 0; c < s.ncol; ++c) slot[c] = c;
      next = s.ncol;
    }
    P.npcol.push_back(next);
    P.col_slot.insert(P.col_slot.end(), slot.begin(), slot.end());
    for (int32_t c : s.colidx) P.colidx_slot.push_back(c >= 0 ? slot[c] : -1);
  }
}

// Per-sphere descriptors and task ranges of one direction.
void build_descs(fftb_plan_s& P, DirCfg& D) {
  const int bc = D.bc;
  const int bc2 = D.bc2 ? D.bc2 : D.bc;  // plane kernel (band-inner: may be narrower)
  const int64_t N = static_cast<int64_t>(P.nx) * P.ny * P.nz;
  D.desc.clear();
  D.splits.clear();
  int64_t soff = 0, goff = 0, coff = 0;
  int32_t gi = 0, ci = 0, cm = 0, xo = 0, so = 0, sl = 0;
  int k1 = 0, k2 = 0, k3 = 0;
  int64_t zoff = 0;
  for (auto& s : P.sph) {
    SphereDesc d = {};
    d.sph_off = soff;
    d.grid_off = goff;
    d.col_off = coff;
    d.gidx_off = gi;
    d.colidx_off = ci;
    d.colmeta_off = cm;
    d.xinv_off = xo;
    d.slab_off = so;
    d.sl_off = sl;
    d.ncol = s.ncol;
    d.npcol = P.npcol[&s - P.sph.data()];
    d.nslab = s.nslab;
    d.nb = s.nb;
    d.nchunk = (s.nb + bc - 1) / bc;
    d.nchunk2 = (s.nb + bc2 - 1) / bc2;
    d.nbp = static_cast<int32_t>(band_stride(s.nb, bc, es_of(P.dtype)));
    d.k1_start = k1;
    k1 += ((s.ncol + D.lc - 1) / D.lc) * d.nchunk;
    d.k1_end = k1;
    d.k2_start = k2;
    k2 += P.nz * d.nchunk2 * (D.class_par ? D.n1 / D.qc : D.nsplit);
    d.split_off = static_cast<int32_t>(D.splits.size());
    std::vector<int32_t> cuts;
    split_slabs(s, D.nsplit, cuts);
    D.splits.insert(D.splits.end(), cuts.begin(), cuts.end());
    d.k2_end = k2;
    d.k3_start = k3;
    if (D.fwd_cls) k3 += P.nz * d.nchunk;
    d.k3_end = k3;
    d.zp_off = zoff;  // relative to the end of the column region, fixed up below
    soff += s.ns * s.nb;
    goff += N * s.nb;
    coff += static_cast<int64_t>(d.nbp) * P.nz * d.npcol;
    if (D.fwd_cls) zoff += static_cast<int64_t>(d.nbp) * P.nz * s.nslab * P.ny;
    gi += s.ncol * P.nz;
    ci += s.nslab * P.ny;
    cm += s.ncol;
    xo += P.nx;
    so += s.nslab + 1;
    sl += s.nslab;
    D.desc.push_back(d);
  }
  // the forward class partials follow the column region
  for (auto& d : D.desc) d.zp_off += coff;
  D.k1_tasks = k1;
  D.k2_tasks = k2;
  D.k3_tasks = k3;
  D.col_elems = coff + zoff;
  // inverse class pairs: (slab, band) lines past the kPairRegLines per
  // thread whose second class waits in registers keep it in an overflow
  // region, m values per line, one region per plane task
  D.ovf_lines = 0;
  D.ovf_off = 0;
  if (D.qc == 2) {
    for (auto& s : P.sph)
      D.ovf_lines = std::max(D.ovf_lines, s.nslab * bc2 - (P.dtype == FFTB_C64 ? kPairRegLines<float>
                                                                              : kPairRegLines<double>) *
                                                                 D.threads);
    D.ovf_off = D.col_elems;
    D.col_elems += static_cast<int64_t>(k2) * D.m * D.ovf_lines;
  }
}

fftb_status dev_alloc(fftb_plan_s& P, size_t bytes, void** out) {
  const size_t cap = device_byte_cap();
  if (cap && P.dev_bytes + bytes > cap)
    return fail(FFTB_ERR_NOMEM, "plan would exceed FFTB_MAX_DEVICE_BYTES");
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, std::max<size_t>(bytes, 256));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(e == hipErrorOutOfMemory ? FFTB_ERR_NOMEM : FFTB_ERR_HIP,
                std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  P.bufs.push_back({p, bytes});
  P.dev_bytes += bytes;
  *out = p;
  return FFTB_OK;
}

template <typename V>
fftb_status upload(fftb_plan_s& P, const std::vector<V>& v, void** out, hipStream_t st) {
  fftb_status s = dev_alloc(P, v.size() * sizeof(V), out);
  if (s != FFTB_OK) return s;
  if (v.empty()) return FFTB_OK;
  hipError_t e = hipMemcpyAsync(*out, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return fail(FFTB_ERR_HIP, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
  return FFTB_OK;
}

// FP64 twiddles as-is, or split into FP32 hi = fl(w), lo = fl(w - hi).
fftb_status upload_tw(fftb_plan_s& P, const std::vector<double>& w, void** hi, void** lo,
                      hipStream_t st) {
  if (P.dtype == FFTB_C128) {
    *lo = nullptr;
    return upload(P, w, hi, st);
  }
  std::vector<float> h(w.size()), l(w.size());
  for (size_t i = 0; i < w.size(); ++i) {
    h[i] = static_cast<float>(w[i]);
    l[i] = static_cast<float>(w[i] - static_cast<double>(h[i]));
  }
  fftb_status s = upload(P, h, hi, st);
  if (s != FFTB_OK) return s;
  return upload(P, l, lo, st);
}

fftb_status device_setup(fftb_plan_s& P, hipStream_t st) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(FFTB_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess)
    return fail(FFTB_ERR_HIP, std::string("hipGetDeviceProperties: ") + hipGetErrorString(e));
  P.num_cus = prop.multiProcessorCount;
  std::vector<int32_t> gidx, colxi, coly, xinv, slabstart, slaborder;
  for (auto& s : P.sph) {
    slaborder.insert(slaborder.end(), s.slab_order.begin(), s.slab_order.end());
    gidx.insert(gidx.end(), s.gidx.begin(), s.gidx.end());
    colxi.insert(colxi.end(), s.col_xi.begin(), s.col_xi.end());
    coly.insert(coly.end(), s.col_y.begin(), s.col_y.end());
    xinv.insert(xinv.end(), s.xinv.begin(), s.xinv.end());
    slabstart.insert(slabstart.end(), s.slabstart.begin(), s.slabstart.end());
  }
  fftb_status s;
  void* p;
  for (auto& D : P.dir) {
    if ((s = upload(P, D.desc, &p, st)) != FFTB_OK) return s;
    D.d_desc = static_cast<SphereDesc*>(p);
    if ((s = upload(P, D.splits, &p, st)) != FFTB_OK) return s;
    D.d_splits = static_cast<int32_t*>(p);
    if ((s = upload_tw(P, axis_twiddles(D.ay), &D.d_twy, &D.d_twy_lo, st)) != FFTB_OK) return s;
  }
  if ((s = upload(P, gidx, &p, st)) != FFTB_OK) return s;
  P.d_gidx = static_cast<int32_t*>(p);
  if ((s = upload(P, P.colidx_slot, &p, st)) != FFTB_OK) return s;
  P.d_colidx = static_cast<int32_t*>(p);
  if ((s = upload(P, colxi, &p, st)) != FFTB_OK) return s;
  P.d_colxi = static_cast<int32_t*>(p);
  if ((s = upload(P, coly, &p, st)) != FFTB_OK) return s;
  P.d_coly = static_cast<int32_t*>(p);
  if ((s = upload(P, xinv, &p, st)) != FFTB_OK) return s;
  P.d_xinv = static_cast<int32_t*>(p);
  if ((s = upload(P, slabstart, &p, st)) != FFTB_OK) return s;
  P.d_slabstart = static_cast<int32_t*>(p);
  if ((s = upload(P, P.col_slot, &p, st)) != FFTB_OK) return s;
  P.d_colslot = static_cast<int32_t*>(p);
  if ((s = upload(P, P.slab_blk, &p, st)) != FFTB_OK) return s;
  P.d_slabblk = static_cast<int32_t*>(p);
  if ((s = upload(P, P.slab_nblk, &p, st)) != FFTB_OK) return s;
  P.d_slabnblk = static_cast<int32_t*>(p);
  if ((s = upload(P, slaborder, &p, st)) != FFTB_OK) return s;
  P.d_slaborder = static_cast<int32_t*>(p);
  if ((s = upload_tw(P, axis_twiddles(P.ax), &P.d_twx, &P.d_twx_lo, st)) != FFTB_OK) return s;
  if ((s = upload_tw(P, axis_twiddles(P.az), &P.d_twz, &P.d_twz_lo, st)) != FFTB_OK) return s;
  if ((s = upload_tw(P, root_table(P.ny), &P.d_twf, &P.d_twf_lo, st)) != FFTB_OK) return s;
  if ((s = upload_tw(P, root_table(P.nx), &P.d_rootx, &P.d_rootx_lo, st)) != FFTB_OK) return s;
  if ((s = upload_tw(P, root_table(P.nz), &P.d_rootz, &P.d_rootz_lo, st)) != FFTB_OK) return s;
  const int64_t col_elems = P.dir[0].col_elems + P.dir[1].col_elems;
  const size_t col_bytes = static_cast<size_t>(col_elems) * es_of(P.dtype);
  if (g_tune_scratch) {
    // an autotuning trial: borrow the tuner's scratch (the previous trial has
    // completed; the tuner synchronises after every trial)
    TuneScratch& ts = *g_tune_scratch;
    if (ts.bytes < col_bytes) {
      if (ts.p) (void)hipFree(ts.p);
      ts.p = nullptr;
      ts.bytes = 0;
      e = hipMalloc(&ts.p, std::max<size_t>(col_bytes, 256));
      if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(FFTB_ERR_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
      }
      ts.bytes = col_bytes;
    }
    P.d_col = ts.p;
  } else if ((s = dev_alloc(P, col_bytes, &P.d_col)) != FFTB_OK) {
    return s;
  }
  // the padding slots of the inverse's column region must read as zero (no
  // kernel writes them); every other scratch value is written before it is read
  e = hipMemsetAsync(P.d_col, 0, static_cast<size_t>(P.dir[0].col_elems) * es_of(P.dtype), st);
  if (e != hipSuccess) return fail(FFTB_ERR_HIP, std::string("hipMemsetAsync: ") + hipGetErrorString(e));
  if ((s = dev_alloc(P, 24 * sizeof(unsigned int), &p)) != FFTB_OK) return s;
  P.d_counters = static_cast<unsigned int*>(p);
  e = hipMemsetAsync(P.d_counters, 0, 24 * sizeof(unsigned int), st);
  if (e != hipSuccess) return fail(FFTB_ERR_HIP, std::string("hipMemsetAsync: ") + hipGetErrorString(e));
  const bool fp64 = P.dtype == FFTB_C128;
  size_t g1 = 4, g2 = 4, r2 = 4;
  for (auto& D : P.dir) {
    if (!D.reg1) g1 = std::max(g1, D.lds1);
    if (!D.reg2) g2 = std::max(g2, D.lds2);
    else r2 = std::max(r2, D.lds2);
  }
  e = prepare_kernels(fp64, g1, g2);
  if (e != hipSuccess)
    return fail(FFTB_ERR_HIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
  for (auto& D : P.dir) {
    if (!D.reg2) continue;
    e = D.bil2 ? prepare_bil(fp64, D.e2, D.h2, r2, D.narrow)
               : prepare_reg(fp64, D.e2, D.h2, r2, D.mf2);
    if (e != hipSuccess)
      return fail(FFTB_ERR_HIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
  }
  e = hipStreamSynchronize(st);
  if (e != hipSuccess)
    return fail(FFTB_ERR_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
  P.device = true;
  return FFTB_OK;
}

KArgs make_args(const fftb_plan_s& P, const DirCfg& D, const void* in, void* out, bool inverse,
                const void* pot) {
  KArgs a;
  std::memset(&a, 0, sizeof a);
  a.nx = P.nx;
  a.ny = P.ny;
  a.nz = P.nz;
  a.bcl = ilog2(D.bc);
  a.bcl2 = ilog2(D.bc2 ? D.bc2 : D.bc);
  a.n1 = D.n1;
  a.m = D.m;
  a.lx = D.lx;
  a.lc = D.lc;
  a.nsph = static_cast<int>(P.sph.size());
  a.k1_tasks = D.k1_tasks;
  a.k2_tasks = D.k2_tasks;
  a.k3_tasks = D.k3_tasks;
  a.persistent = (P.flags & FFTB_PLAN_BATCHED) ? 1 : 0;
  a.lds_P = D.lds_P;
  a.lds_X0 = D.lds_X0;
  a.lds_X1 = D.lds_X1;
  a.lds_acc = D.lds_acc;
  a.acc_lds = D.acc_lds ? 1 : 0;
  a.sx = D.sx;
  a.nsplit = D.nsplit;
  a.fwd_cls = D.fwd_cls ? 1 : 0;
  a.g2 = D.reg2 ? (D.class_par ? D.n1 / D.qc : D.nsplit) : 1;
  a.qc = D.qc;
  a.mfma = (D.bil2 && D.mf2) ? 1 : 0;
  a.ovf_lines = D.ovf_lines;
  a.ovf_off = D.ovf_off;
  // 32-bit buffer addressing where every region it covers allows it
  a.plane32 = 1;
  a.k1buf = 1;
  const int64_t es = es_of(P.dtype);
  for (size_t i = 0; i < P.sph.size(); ++i) {
    const auto& sp = P.sph[i];
    const int64_t nbp = D.desc[i].nbp;
    const int64_t colplane = static_cast<int64_t>(D.desc[i].npcol) * nbp * es;
    const int64_t zplane = static_cast<int64_t>(sp.nslab) * P.ny * nbp * es;
    const int64_t gplane = static_cast<int64_t>(P.nx) * P.ny * sp.nb * es;
    if (std::max(colplane, std::max(zplane, gplane)) >= (int64_t{1} << 31)) a.plane32 = 0;
    if (sp.ns * sp.nb * es >= 0xffffffffLL || colplane * P.nz >= 0xffffffffLL) a.k1buf = 0;
  }
  a.splits = D.d_splits;
  fill_axis(P.ax, a.ax);
  fill_axis(D.ay, a.ay);
  fill_axis(P.az, a.az);
  a.sph = D.d_desc;
  a.gidx = P.d_gidx;
  a.colidx = P.d_colidx;
  a.col_xi = P.d_colxi;
  a.col_y = P.d_coly;
  a.xinv = P.d_xinv;
  a.slabstart = P.d_slabstart;
  a.col_slot = P.d_colslot;
  a.slab_blk = P.d_slabblk;
  a.slab_nblk = P.d_slabnblk;
  a.lds_tab = D.lds_tab;
  a.lds_twx = D.lds_twx;
  a.zline = D.zline;
  a.slab_order = P.d_slaborder;
  a.twx = P.d_twx;
  a.twy = D.d_twy;
  a.twz = P.d_twz;
  a.twf = P.d_twf;
  a.twx_lo = P.d_twx_lo;
  a.twy_lo = D.d_twy_lo;
  a.twz_lo = P.d_twz_lo;
  a.twf_lo = P.d_twf_lo;
  a.rootx = P.d_rootx;
  a.rootx_lo = P.d_rootx_lo;
  a.rootz = P.d_rootz;
  a.rootz_lo = P.d_rootz_lo;
  a.in = in;
  a.out = out;
  a.pot = inverse ? pot : nullptr;
  a.col = P.d_col;
  a.scale = inverse ? 1.0 : 1.0 / (static_cast<double>(P.nx) * P.ny * P.nz);
  a.counters = P.d_counters;
  return a;
}

int occupancy(size_t lds) {
  const int by_lds = lds > 0 ? std::max<int>(1, static_cast<int>(kLdsMax / lds)) : 8;
  return std::min(by_lds, 8);
}

// Static grids cover every task under the group-interleaved XCD mapping:
// ceil(groups / 8) groups per XCD.
void grids(const fftb_plan_s& P, const DirCfg& D, int& g1, int& g2, int& g3) {
  const int G = D.reg2 ? (D.class_par ? D.n1 / D.qc : D.nsplit) : 1;
  g1 = ((D.k1_tasks + 7) / 8) * 8;
  g2 = ((D.k2_tasks / G + 7) / 8) * 8 * G;
  g3 = ((D.k3_tasks + 7) / 8) * 8;
  if (P.flags & FFTB_PLAN_BATCHED) {
    // persistent: enough blocks to fill the chip, at least one per XCD queue
    const int c1 = P.num_cus * occupancy(D.lds1);
    const int c2 = P.num_cus * occupancy(D.lds2);
    const int c3 = P.num_cus * occupancy(0);
    g1 = std::max(8, std::min(c1, g1));
    g2 = std::max(8, std::min(c2, g2));
    g3 = std::max(8, std::min(c3, g3));
    g1 = (g1 + 7) / 8 * 8;
    g2 = (g2 + 7) / 8 * 8;
    g3 = (g3 + 7) / 8 * 8;
  }
}

hipError_t get_event(fftb_plan_s* P, hipEvent_t* e) {
  if (!P->ev_pool.empty()) {
    *e = P->ev_pool.back();
    P->ev_pool.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(e);
}

// Enqueue one direction: inverse = column kernel then plane kernel; forward =
// plane kernel then column kernel. Persistent kernels first reset their work
// counters with a kernel (graph-safe, no memset node).
hipError_t enqueue(fftb_plan_s* P, const KArgs& a, const DirCfg& D, bool inverse, int g1, int g2,
                   int g3, hipStream_t st, bool profile) {
  const bool fp64 = P->dtype == FFTB_C128;
  hipError_t e = hipSuccess;
  if (a.persistent) {
    e = launch_reset(a.counters, st);
    if (e != hipSuccess) return e;
  }
  // which: 1 column kernel, 2 plane kernel, 3 forward class combine
  int order[3] = {inverse ? 1 : 2, inverse ? 2 : 1, 0};
  if (!inverse && D.fwd_cls) {
    order[1] = 3;
    order[2] = 1;
  }
  for (int which : order) {
    if (which == 0) continue;
    // kernel ids: 0 column inverse, 1 plane inverse, 2 plane forward, 3 column forward,
    // 4 class combine forward
    const int kid = which == 3 ? 4 : inverse ? (which == 1 ? 0 : 1) : (which == 2 ? 2 : 3);
    hipEvent_t ea = nullptr, eb = nullptr;
    if (profile) {
      if ((e = get_event(P, &ea)) != hipSuccess) return e;
      if ((e = get_event(P, &eb)) != hipSuccess) return e;
      if ((e = hipEventRecord(ea, st)) != hipSuccess) return e;
    }
    const bool reg = which == 1 ? D.reg1 : D.reg2;
    if (which == 3) {
      e = launch_combine(a, fp64, g3, 256, st);
    } else if (which == 1 ? D.bil1 : D.bil2) {
      e = launch_bil(which == 2 && D.narrow ? 3 : which, a, inverse, fp64,
                     which == 1 ? D.e1 : D.e2, which == 1 ? D.h1 : D.h2,
                     which == 1 ? g1 : g2, which == 1 ? 256 : D.threads, which == 1 ? 0 : D.lds2, st,
                     which == 1 ? 0 : D.fold_m);
    } else if (reg) {
      e = launch_reg(which, a, inverse, fp64, which == 1 ? D.e1 : D.e2, which == 1 ? D.h1 : D.h2,
                     which == 1 ? g1 : g2, which == 1 ? std::min(D.threads, 256) : D.threads,
                     which == 1 ? 0 : D.lds2, st, which == 1 ? D.mf1 : D.mf2,
                     which == 1 ? 0 : D.fold_m);
    } else {
      e = launch_kernel(which, a, inverse, fp64, which == 1 ? g1 : g2, std::min(D.threads, 256),
                        which == 1 ? D.lds1 : D.lds2, st);
    }
    if (e != hipSuccess) return e;
    if (profile) {
      if ((e = hipEventRecord(eb, st)) != hipSuccess) return e;
      P->prof_pending.push_back({kid, ea, eb});
    }
  }
  return hipSuccess;
}

fftb_status run(fftb_plan_s* P, const void* in, void* out, void* stream, bool inverse,
                const void* pot = nullptr) {
  if (!P) return fail(FFTB_ERR_INVALID, "null plan");
  if (!P->device) return fail(FFTB_ERR_INVALID, "plan was created host-only");
  if (!in || !out) return fail(FFTB_ERR_INVALID, "null data pointer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const DirCfg& D = P->dir[inverse ? 0 : 1];
  int g1, g2, g3;
  grids(*P, D, g1, g2, g3);
  KArgs a = make_args(*P, D, in, out, inverse, pot);
  if (P->flags & FFTB_PLAN_GRAPH) {
    auto& gc = P->gc[inverse ? 0 : 1];
    if (!gc.exec || gc.in != in || gc.out != out || gc.pot != a.pot) {
      if (gc.exec) { (void)hipGraphExecDestroy(gc.exec); gc.exec = nullptr; }
      if (gc.graph) { (void)hipGraphDestroy(gc.graph); gc.graph = nullptr; }
      if (!P->cap_stream) {
        hipError_t e = hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return fail(FFTB_ERR_HIP, std::string("hipStreamCreate: ") + hipGetErrorString(e));
      }
      hipError_t e = hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return fail(FFTB_ERR_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
      hipError_t el = enqueue(P, a, D, inverse, g1, g2, g3, P->cap_stream, false);
      e = hipStreamEndCapture(P->cap_stream, &gc.graph);
      if (el != hipSuccess) return fail(FFTB_ERR_HIP, std::string("launch during capture: ") + hipGetErrorString(el));
      if (e != hipSuccess) return fail(FFTB_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
      e = hipGraphInstantiate(&gc.exec, gc.graph, nullptr, nullptr, 0);
      if (e != hipSuccess) return fail(FFTB_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
      gc.in = in;
      gc.out = out;
      gc.pot = a.pot;
    }
    hipError_t e = hipGraphLaunch(gc.exec, st);
    if (e != hipSuccess) return fail(FFTB_ERR_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    return FFTB_OK;
  }
  hipError_t e = enqueue(P, a, D, inverse, g1, g2, g3, st, P->profiling);
  if (e != hipSuccess) return fail(FFTB_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return FFTB_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: time candidate tilings of each direction on scratch buffers of
// the plan's real size (warm-up + 3 timed executions with HIP events, never
// inside a graph capture) and keep the fastest per direction. Results are
// cached per input (FNV-1a hash of dims, dtype, persistent flag, the spheres'
// sizes and maps) in the file named by FFTB_TUNE_CACHE, if set.

// Plan summary on stderr when FFTB_LOG is set (to anything but 0).
void log_plan(const fftb_plan_s& P) {
  const char* v = std::getenv("FFTB_LOG");
  if (!v || !*v || std::strcmp(v, "0") == 0) return;
  std::fprintf(stderr,
               "fftb plan: grid %dx%dx%d, %zu sphere(s), %lld coefficients, %lld columns, %s, "
               "flags %u, %s, device %.3f GB (scratch %.3f GB)\n",
               P.nx, P.ny, P.nz, P.sph.size(), static_cast<long long>(P.total_coeffs),
               static_cast<long long>(P.total_columns), P.dtype == FFTB_C128 ? "complex128" : "complex64",
               P.flags, P.autotuned == 1 ? "autotuned" : P.autotuned == 2 ? "tuning from cache" : "default tiling",
               P.dev_bytes / 1e9,
               static_cast<double>(P.dir[0].col_elems + P.dir[1].col_elems) * es_of(P.dtype) / 1e9);
  for (int d = 0; d < 2; ++d) {
    const DirCfg& D = P.dir[d];
    std::fprintf(stderr,
                 "  %s: band chunk %d, %d y classes of %d, %d threads, column kernel %s (%dx%d, %d "
                 "columns/task, %d tasks), plane kernel %s (%dx%d, LDS %zu B, %d tasks)%s%s, "
                 "fold m %d\n",
                 d == 0 ? "inverse" : "forward", D.bc, D.n1, D.m, D.threads,
                 D.bil1 ? "band-inner" : D.reg1 ? "register" : "LDS-stage", D.e1, D.h1, D.lc, D.k1_tasks,
                 D.narrow ? "band-inner, half pieces" : D.bil2 ? "band-inner" : D.reg2 ? "register" : "LDS-stage",
                 D.e2, D.h2, D.lds2, D.k2_tasks,
                 D.fwd_cls ? ", class partials + combine" : D.qc == 2 ? ", class pairs" : "",
                 D.mf2 || D.mf1 ? ", matrix-core DFT_16" : "",
                 D.fold_m);
  }
}

uint64_t plan_key(const int32_t dims[3], const fftb_sphere* spheres, int nsph, fftb_dtype dt,
                  uint32_t flags) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&h](const void* p, size_t n) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
      h ^= c[i];
      h *= 1099511628211ull;
    }
  };
  mix(dims, 3 * sizeof(int32_t));
  const int32_t d = dt;
  mix(&d, sizeof d);
  const uint32_t f = flags & (FFTB_PLAN_BATCHED | FFTB_PLAN_MFMA);
  mix(&f, sizeof f);
  for (int s = 0; s < nsph; ++s) {
    mix(&spheres[s].n_coeffs, sizeof(int64_t));
    mix(&spheres[s].nbands, sizeof(int32_t));
    mix(spheres[s].map, sizeof(int32_t) * static_cast<size_t>(spheres[s].n_coeffs));
  }
  return h;
}

constexpr int kDirInts = static_cast<int>(sizeof(fftb_dir_tuning) / sizeof(int32_t));
constexpr int kTuneInts = 2 * kDirInts;
constexpr const char* kTuneTag = "fftb-tune-v2";

void tuning_to_ints(const fftb_tuning& t, int32_t* v) {
  std::memcpy(v, &t.inv, kDirInts * sizeof(int32_t));
  std::memcpy(v + kDirInts, &t.fwd, kDirInts * sizeof(int32_t));
}
void ints_to_tuning(const int32_t* v, fftb_tuning& t) {
  std::memcpy(&t.inv, v, kDirInts * sizeof(int32_t));
  std::memcpy(&t.fwd, v + kDirInts, kDirInts * sizeof(int32_t));
}

bool cache_lookup(uint64_t key, fftb_tuning& t) {
  const char* path = std::getenv("FFTB_TUNE_CACHE");
  if (!path || !*path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    // "<tag> <hex key> <ints>": lines of another format version are skipped
    char tag[32];
    unsigned long long k;
    int used = 0;
    if (std::sscanf(line, "%31s %llx%n", tag, &k, &used) != 2) continue;
    if (std::strcmp(tag, kTuneTag) != 0 || k != key) continue;
    int32_t v[kTuneInts];
    const char* p = line + used;
    bool ok = true;
    for (int i = 0; i < kTuneInts && ok; ++i) {
      int n = 0;
      ok = std::sscanf(p, "%d%n", &v[i], &n) == 1;
      p += n;
    }
    if (ok) {
      ints_to_tuning(v, t);
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

void cache_store(uint64_t key, const fftb_tuning& t) {
  const char* path = std::getenv("FFTB_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  int32_t v[kTuneInts];
  tuning_to_ints(t, v);
  std::fprintf(f, "%s %llx", kTuneTag, static_cast<unsigned long long>(key));
  for (int i = 0; i < kTuneInts; ++i) std::fprintf(f, " %d", v[i]);
  std::fprintf(f, "\n");
  std::fclose(f);
}

// Effective tiling of one direction as choose_dir resolves it (the fields
// that tell two candidates apart).
struct DirKey {
  int v[9];
  bool operator==(const DirKey& o) const { return std::memcmp(v, o.v, sizeof v) == 0; }
};
DirKey dir_key(const DirCfg& D, bool inverse) {
  DirKey k = {{D.narrow ? D.bc2 : D.bc, D.n1, D.threads,
               (D.reg1 ? 1 : 0) | (D.reg2 ? 2 : 0) | (D.bil1 ? 4 : 0) | (D.bil2 ? 8 : 0),
               D.reg2 ? D.h2 : D.lx,
               D.lc, inverse ? D.qc : (D.fwd_cls ? 3 : D.acc_lds ? 1 : 2), D.nsplit, D.h1}};
  return k;
}

// Candidate tilings of one direction around the library defaults, most
// promising first: band chunk (default, half, and twice for the inverse),
// class count (default, ny/16, ny/8), 256 or 512 threads, the 8-lane line
// shapes, for the inverse class pairs or one class per task, and for the
// forward the class-partial and the LDS-accumulator variants. The LDS-stage kernels are tried only where an axis has no
// register shape. Candidates that resolve to the same tiling, or that do not
// fit, are dropped; at most `cap` remain.
std::vector<fftb_dir_tuning> candidates(fftb_plan_s& P, bool inverse, const fftb_dir_tuning& base,
                                        size_t cap) {
  const bool fp64 = P.dtype == FFTB_C128;
  const int d = inverse ? 0 : 1;
  const DirCfg saved = P.dir[d];
  const std::string saved_err = g_last_error;
  std::vector<fftb_dir_tuning> raw;
  const int bc0 = default_bc(P, fp64 ? 8 : 16);
  std::vector<int> bcs = {bc0};
  if (bc0 / 2 >= 1) bcs.push_back(bc0 / 2);
  if (inverse && bc0 * 2 <= default_bc(P, 64)) bcs.push_back(bc0 * 2);
  std::vector<int> classes = {0};
  for (int m : {16, 8})
    if (P.ny % m == 0 && P.ny / m > 1) classes.push_back(P.ny / m);
  raw.push_back(base);
  for (int lanes : {0, 8}) {
    for (int bc : bcs) {
      for (int n1 : classes) {
        for (int threads : {256, 512}) {
          fftb_dir_tuning t = base;
          t.band_chunk = bc;
          t.y_classes = n1;
          t.threads = threads;
          t.path = 0;
          t.lanes = lanes;
          if (inverse) {
            // band-inner: class pairs (the default where they apply) and one
            // class per task
            for (int acc : {0, 1}) {
              t.acc = acc;
              raw.push_back(t);
            }
          } else {
            for (int acc : {3, 1}) {
              t.acc = acc;
              raw.push_back(t);
            }
          }
        }
      }
    }
  }
  // the LDS-stage kernels, only where the default has no register path
  bool reg_default = false;
  if (choose_dir(P, d, base) == FFTB_OK) reg_default = P.dir[d].reg1 && P.dir[d].reg2;
  if (!reg_default) {
    for (int bc : bcs) {
      fftb_dir_tuning g = base;
      g.band_chunk = bc;
      g.path = 1;
      raw.push_back(g);
    }
  }
  std::vector<fftb_dir_tuning> out;
  std::vector<DirKey> seen;
  for (const auto& t : raw) {
    if (out.size() >= cap) break;
    P.dir[d] = DirCfg();
    if (choose_dir(P, d, t) != FFTB_OK) continue;
    const DirKey k = dir_key(P.dir[d], inverse);
    if (std::find(seen.begin(), seen.end(), k) != seen.end()) continue;
    seen.push_back(k);
    out.push_back(t);
  }
  P.dir[d] = saved;
  g_last_error = saved_err;
  return out;
}

std::string tiling_str(const fftb_dir_tuning& t) {
  char b[160];
  std::snprintf(b, sizeof b, "bc=%d n1=%d thr=%d lanes=%d acc=%d path=%d", t.band_chunk,
                t.y_classes, t.threads, t.lanes, t.acc, t.path);
  return b;
}

double env_seconds(const char* name, double dflt) {
  const char* v = std::getenv(name);
  if (!v || !*v) return dflt;
  const double x = std::atof(v);
  return x > 0 ? x : dflt;
}

fftb_status autotune(fftb_plan_s& P, const int32_t dims[3], const fftb_sphere* spheres, int nsph,
                     fftb_dtype dtype, uint32_t flags, fftb_tuning& t, hipStream_t st) {
  const uint64_t key = plan_key(dims, spheres, nsph, dtype, flags);
  if (cache_lookup(key, t)) {
    P.autotuned = 2;
    return FFTB_OK;
  }
  const size_t cap = static_cast<size_t>(env_seconds("FFTB_TUNE_MAX_CANDIDATES", 16));
  const double budget = env_seconds("FFTB_TUNE_SECONDS", 60.0);
  const int es = es_of(dtype);
  void *sin = nullptr, *sout = nullptr, *grid = nullptr;
  if (hipMalloc(&sin, P.sphere_elems * es) != hipSuccess ||
      hipMalloc(&sout, P.sphere_elems * es) != hipSuccess ||
      hipMalloc(&grid, P.grid_elems * es) != hipSuccess) {
    (void)hipGetLastError();
    if (sin) (void)hipFree(sin);
    if (sout) (void)hipFree(sout);
    return FFTB_OK;  // not enough memory to tune: keep the defaults
  }
  (void)hipMemsetAsync(sin, 0, P.sphere_elems * es, st);
  (void)hipMemsetAsync(grid, 0, P.grid_elems * es, st);
  const std::vector<fftb_dir_tuning> ci = candidates(P, true, t.inv, cap);
  const std::vector<fftb_dir_tuning> cf = candidates(P, false, t.fwd, cap);
  const size_t n = std::max(ci.size(), cf.size());
  double best[2] = {1e30, 1e30};
  fftb_dir_tuning pick[2] = {t.inv, t.fwd};
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const std::string saved_err = g_last_error;
  TuneScratch scratch;
  g_tune_scratch = &scratch;
  const auto t_start = std::chrono::steady_clock::now();
  std::fprintf(stderr, "fftb autotune: %zu inverse and %zu forward candidates, budget %.0f s\n",
               ci.size(), cf.size(), budget);
  size_t i = 0;
  for (; i < n; ++i) {
    const double el =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    if (i > 0 && el > budget) break;  // the first trial always runs
    fftb_tuning c = t;
    c.inv = ci[std::min(i, ci.size() - 1)];
    c.fwd = cf[std::min(i, cf.size() - 1)];
    fftb_plan sub = nullptr;
    const uint32_t sflags = flags & ~(FFTB_PLAN_AUTOTUNE | FFTB_PLAN_GRAPH);
    double ms_dir[2] = {-1, -1};
    if (fftb_plan_create(&sub, dims, spheres, nsph, dtype, sflags, &c, st) == FFTB_OK) {
      for (int d = 0; d < 2; ++d) {
        const bool inv = d == 0;
        if (i >= (inv ? ci.size() : cf.size())) continue;  // this direction's list is done
        const void* in = inv ? sin : grid;
        void* out = inv ? grid : sout;
        // one warm-up; then 3 timed executions, or 1 when one takes over 50 ms
        fftb_status ok = FFTB_OK;
        float ms = 0.f;
        if (hipEventRecord(e0, st) != hipSuccess) ok = FFTB_ERR_HIP;
        if (ok == FFTB_OK) ok = run(sub, in, out, st, inv);
        if (ok == FFTB_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                              hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
          ok = FFTB_ERR_HIP;
        const int reps = ms > 50.f ? 1 : 3;
        if (ok == FFTB_OK && hipEventRecord(e0, st) != hipSuccess) ok = FFTB_ERR_HIP;
        for (int r = 0; r < reps && ok == FFTB_OK; ++r) ok = run(sub, in, out, st, inv);
        if (ok == FFTB_OK && hipEventRecord(e1, st) == hipSuccess &&
            hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) {
          ms_dir[d] = ms / reps;
          if (ms_dir[d] < best[d]) {
            best[d] = ms_dir[d];
            pick[d] = inv ? c.inv : c.fwd;
          }
        }
      }
      fftb_plan_destroy(sub);
    }
    (void)hipStreamSynchronize(st);
    std::fprintf(stderr, "fftb autotune %zu/%zu: inv [%s] %.3f ms | fwd [%s] %.3f ms\n", i + 1, n,
                 i < ci.size() ? tiling_str(c.inv).c_str() : "-", ms_dir[0],
                 i < cf.size() ? tiling_str(c.fwd).c_str() : "-", ms_dir[1]);
    std::fflush(stderr);
  }
  g_tune_scratch = nullptr;
  (void)hipStreamSynchronize(st);
  if (scratch.p) (void)hipFree(scratch.p);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(sin);
  (void)hipFree(sout);
  (void)hipFree(grid);
  (void)hipGetLastError();
  g_last_error = saved_err;
  if (best[0] < 1e30) t.inv = pick[0];
  if (best[1] < 1e30) t.fwd = pick[1];
  std::fprintf(stderr, "fftb autotune: %zu of %zu trials in %.1f s; inverse [%s] %.3f ms, forward [%s] %.3f ms\n",
               i, n, std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count(),
               tiling_str(t.inv).c_str(), best[0], tiling_str(t.fwd).c_str(), best[1]);
  P.autotuned = 1;
  cache_store(key, t);
  return FFTB_OK;
}

}  // namespace

extern "C" {

fftb_status fftb_plan_create(fftb_plan* out, const int32_t dims[3], const fftb_sphere* spheres,
                             int32_t nspheres, fftb_dtype dtype, uint32_t flags,
                             const fftb_tuning* tuning, void* stream) {
  try {
    g_last_error.clear();
    if (!out) return fail(FFTB_ERR_INVALID, "null output pointer");
    *out = nullptr;
    if (!dims) return fail(FFTB_ERR_INVALID, "null dims");
    if (!spheres) return fail(FFTB_ERR_INVALID, "null spheres");
    if (nspheres < 1) return fail(FFTB_ERR_INVALID, "nspheres must be >= 1");
    if (dtype != FFTB_C128 && dtype != FFTB_C64) return fail(FFTB_ERR_INVALID, "unknown dtype");
    for (int i = 0; i < 3; ++i)
      if (dims[i] < 1) return fail(FFTB_ERR_INVALID, "dims must be >= 1");
    const int64_t N = static_cast<int64_t>(dims[0]) * dims[1] * dims[2];
    if (N > (int64_t{1} << 31) - 1) return fail(FFTB_ERR_UNSUPPORTED, "grid larger than 2^31 points");
    std::unique_ptr<fftb_plan_s> P(new fftb_plan_s());
    P->nx = dims[0];
    P->ny = dims[1];
    P->nz = dims[2];
    P->dtype = dtype;
    P->flags = flags;
    std::vector<int> rx, ry, rz;
    if (!plan_radices(P->nx, rx) || !plan_radices(P->ny, ry) || !plan_radices(P->nz, rz))
      return fail(FFTB_ERR_UNSUPPORTED, "grid dimensions must have prime factors 2, 3, 5 only");
    make_axis_plan(P->nx, rx, P->ax);
    make_axis_plan(P->nz, rz, P->az);
    P->sph.resize(nspheres);
    for (int s = 0; s < nspheres; ++s) {
      std::string err;
      if (build_sphere_tables(P->nx, P->ny, P->nz, spheres[s].map, spheres[s].n_coeffs,
                              spheres[s].nbands, P->sph[s], err) != 0) {
        char buf[64];
        std::snprintf(buf, sizeof buf, "sphere %d: ", s);
        return fail(FFTB_ERR_INVALID, buf + err);
      }
      for (int k = 0; k < 3; ++k) P->sph[s].kpt[k] = spheres[s].kpt[k];
      P->max_ncol = std::max(P->max_ncol, P->sph[s].ncol);
      P->max_nslab = std::max(P->max_nslab, P->sph[s].nslab);
      P->total_columns += P->sph[s].ncol;
      P->total_coeffs += P->sph[s].ns;
      P->sphere_elems += P->sph[s].ns * P->sph[s].nb;
      P->grid_elems += N * P->sph[s].nb;
    }
    fftb_tuning t = {};
    if (tuning) t = *tuning;
    if ((flags & FFTB_PLAN_AUTOTUNE) && !(flags & FFTB_PLAN_HOST_ONLY)) {
      fftb_status st = autotune(*P, dims, spheres, nspheres, dtype, flags, t,
                                static_cast<hipStream_t>(stream));
      if (st != FFTB_OK) return st;
    }
    for (int d = 0; d < 2; ++d) {
      fftb_status st = choose_dir(*P, d, d == 0 ? t.inv : t.fwd);
      if (st != FFTB_OK) return st;
    }
    if ((flags & FFTB_PLAN_MFMA) && !(P->dir[0].mf1 || P->dir[0].mf2 || P->dir[1].mf1 || P->dir[1].mf2))
      return fail(FFTB_ERR_UNSUPPORTED, "no DFT_16 stage for the matrix cores in this plan");
    P->pad_m = P->dir[0].fold_m;
    build_slots(*P);
    for (int d = 0; d < 2; ++d) build_descs(*P, P->dir[d]);
    // the scratch holds the inverse's columns first, then the forward's columns
    // and class partials: the inverse fold relies on its zero padding slots,
    // which a forward with another band stride would otherwise overwrite
    for (auto& dd : P->dir[1].desc) {
      dd.col_off += P->dir[0].col_elems;
      dd.zp_off += P->dir[0].col_elems;
    }
    for (int d = 0; d < 2; ++d) {
      const DirCfg& D = P->dir[d];
      fftb_dir_tuning& o = d == 0 ? P->tun.inv : P->tun.fwd;
      o.band_chunk = D.narrow ? D.bc2 : D.bc;
      o.y_classes = D.n1;
      o.x_rows = D.lx;
      o.col_tile = D.lc;
      o.threads = D.threads;
      o.path = D.bil2 ? 3 : (D.reg1 && D.reg2) ? 2 : (D.reg1 || D.reg2) ? 0 : 1;
      o.acc = d == 0 ? ((D.bil2 && !D.narrow) ? D.qc : 0)
                     : D.fwd_cls ? 3 : (D.reg2 && D.acc_lds) ? 1 : 2;
      o.splits = D.nsplit;
      o.lanes = D.bil2 ? 0 : D.reg2 ? D.h2 : (D.reg1 ? D.h1 : 0);
    }
    if (!(flags & FFTB_PLAN_HOST_ONLY)) {
      const size_t cap = device_byte_cap();
      const size_t scratch = static_cast<size_t>(P->dir[0].col_elems + P->dir[1].col_elems) *
                             es_of(dtype);
      if (cap && !g_tune_scratch && scratch > cap)
        return fail(FFTB_ERR_NOMEM, "plan scratch of " + std::to_string(scratch) +
                                        " bytes exceeds FFTB_MAX_DEVICE_BYTES");
      fftb_status st = device_setup(*P, static_cast<hipStream_t>(stream));
      if (st != FFTB_OK) return st;
    }
    if (!g_tune_scratch) log_plan(*P);
    *out = P.release();
    return FFTB_OK;
  } catch (const std::bad_alloc&) {
    return fail(FFTB_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(FFTB_ERR_INVALID, "unexpected exception");
  }
}

fftb_status fftb_sphere_to_grid(fftb_plan plan, const void* sphere_in, void* grid_out, void* stream) {
  try {
    return run(plan, sphere_in, grid_out, stream, true);
  } catch (...) {
    return fail(FFTB_ERR_INVALID, "unexpected exception");
  }
}

fftb_status fftb_grid_to_sphere(fftb_plan plan, const void* grid_in, void* sphere_out, void* stream) {
  try {
    return run(plan, grid_in, sphere_out, stream, false);
  } catch (...) {
    return fail(FFTB_ERR_INVALID, "unexpected exception");
  }
}

fftb_status fftb_sphere_to_grid_static(fftb_plan P, const void* sphere_in, void* grid_out,
                                       void* stream) {
  try {
    if (!P) return fail(FFTB_ERR_INVALID, "null plan");
    if (!P->device) return fail(FFTB_ERR_INVALID, "plan was created host-only");
    if (!sphere_in || !grid_out) return fail(FFTB_ERR_INVALID, "null data pointer");
    const DirCfg& D = P->dir[0];
    const size_t need = static_cast<size_t>(D.col_elems) * es_of(P->dtype);
    if (need > FFTB_STATIC_SCRATCH_BYTES)
      return fail(FFTB_ERR_UNSUPPORTED,
                  "the plan's inverse column scratch (" + std::to_string(need) +
                      " bytes) exceeds the static scratch (" +
                      std::to_string(static_cast<size_t>(FFTB_STATIC_SCRATCH_BYTES)) + " bytes)");
    void* scr = nullptr;
    hipError_t e = static_scratch_ptr(&scr);
    if (e != hipSuccess)
      return fail(FFTB_ERR_HIP, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
    hipStream_t st = static_cast<hipStream_t>(stream);
    // the padding slots the inverse fold reads must be zero; the array keeps
    // the previous call's contents (col_elems * value size is a multiple of 16)
    e = launch_zero_scratch(scr, (need + 15) & ~size_t{15}, st);
    if (e != hipSuccess) return fail(FFTB_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    int g1, g2, g3;
    grids(*P, D, g1, g2, g3);
    KArgs a = make_args(*P, D, sphere_in, grid_out, true, nullptr);
    a.col = scr;
    e = enqueue(P, a, D, true, g1, g2, g3, st, false);
    if (e != hipSuccess) return fail(FFTB_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return FFTB_OK;
  } catch (...) {
    return fail(FFTB_ERR_INVALID, "unexpected exception");
  }
}

fftb_status fftb_plan_create_cuboid(fftb_plan* out, const int32_t dims[3], int32_t nbands,
                                    fftb_dtype dtype, uint32_t flags, const fftb_tuning* tuning,
                                    void* stream) {
  try {
    if (!out) return fail(FFTB_ERR_INVALID, "null output pointer");
    *out = nullptr;
    if (!dims) return fail(FFTB_ERR_INVALID, "null dims");
    for (int i = 0; i < 3; ++i)
      if (dims[i] < 1) return fail(FFTB_ERR_INVALID, "dims must be >= 1");
    const int64_t N = static_cast<int64_t>(dims[0]) * dims[1] * dims[2];
    if (N > (int64_t{1} << 31) - 1) return fail(FFTB_ERR_UNSUPPORTED, "grid larger than 2^31 points");
    // every grid point is a coefficient, in grid order
    std::vector<int32_t> map(static_cast<size_t>(N));
    for (int64_t i = 0; i < N; ++i) map[static_cast<size_t>(i)] = static_cast<int32_t>(i);
    fftb_sphere s = {};
    s.n_coeffs = N;
    s.map = map.data();
    s.nbands = nbands;
    return fftb_plan_create(out, dims, &s, 1, dtype, flags, tuning, stream);
  } catch (const std::bad_alloc&) {
    return fail(FFTB_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(FFTB_ERR_INVALID, "unexpected exception");
  }
}

fftb_status fftb_apply_potential(fftb_plan P, const void* sphere_in, const void* potential,
                                 void* grid_work, void* sphere_out, void* stream) {
  try {
    if (!P) return fail(FFTB_ERR_INVALID, "null plan");
    if (!potential) return fail(FFTB_ERR_INVALID, "null potential");
    fftb_status s = run(P, sphere_in, grid_work, stream, true, potential);
    if (s != FFTB_OK) return s;
    return run(P, grid_work, sphere_out, stream, false);
  } catch (...) {
    return fail(FFTB_ERR_INVALID, "unexpected exception");
  }
}

fftb_status fftb_plan_get_info(fftb_plan P, fftb_plan_info* info) {
  if (!P || !info) return fail(FFTB_ERR_INVALID, "null argument");
  std::memset(info, 0, sizeof *info);
  info->dims[0] = P->nx;
  info->dims[1] = P->ny;
  info->dims[2] = P->nz;
  info->nspheres = static_cast<int32_t>(P->sph.size());
  info->dtype = P->dtype;
  info->flags = P->flags;
  info->total_coeffs = P->total_coeffs;
  info->sphere_elems = P->sphere_elems;
  info->grid_elems = P->grid_elems;
  info->total_columns = P->total_columns;
  info->max_columns = P->max_ncol;
  info->max_slab = P->max_nslab;
  info->workspace_bytes = static_cast<int64_t>(P->dev_bytes);
  for (int s = 0; s < P->ax.nst && s < 8; ++s) info->radix_x[s] = P->ax.R[s];
  for (int s = 0; s < P->dir[0].ay.nst && s < 8; ++s) info->radix_y[s] = P->dir[0].ay.R[s];
  for (int s = 0; s < P->az.nst && s < 8; ++s) info->radix_z[s] = P->az.R[s];
  info->tuning = P->tun;
  info->autotuned = P->autotuned;
  return FFTB_OK;
}

fftb_status fftb_plan_workspace_size(fftb_plan P, size_t* bytes) {
  if (!P || !bytes) return fail(FFTB_ERR_INVALID, "null argument");
  *bytes = P->dev_bytes;
  return FFTB_OK;
}

fftb_status fftb_plan_sphere_stats(fftb_plan P, int32_t sphere, int32_t* ncolumns, int32_t* nslab) {
  if (!P) return fail(FFTB_ERR_INVALID, "null plan");
  if (sphere < 0 || sphere >= static_cast<int32_t>(P->sph.size()))
    return fail(FFTB_ERR_INVALID, "sphere index out of range");
  if (ncolumns) *ncolumns = P->sph[sphere].ncol;
  if (nslab) *nslab = P->sph[sphere].nslab;
  return FFTB_OK;
}

fftb_status fftb_plan_sphere_columns(fftb_plan P, int32_t sphere, int32_t* col_x, int32_t* col_y,
                                     int32_t* entry_col, int32_t* entry_z) {
  if (!P) return fail(FFTB_ERR_INVALID, "null plan");
  if (sphere < 0 || sphere >= static_cast<int32_t>(P->sph.size()))
    return fail(FFTB_ERR_INVALID, "sphere index out of range");
  const auto& s = P->sph[sphere];
  if (col_x) std::copy(s.col_x.begin(), s.col_x.end(), col_x);
  if (col_y) std::copy(s.col_y.begin(), s.col_y.end(), col_y);
  if (entry_col) std::copy(s.entry_col.begin(), s.entry_col.end(), entry_col);
  if (entry_z) std::copy(s.entry_z.begin(), s.entry_z.end(), entry_z);
  return FFTB_OK;
}

fftb_status fftb_plan_set_profiling(fftb_plan P, int32_t enable) {
  if (!P) return fail(FFTB_ERR_INVALID, "null plan");
  P->profiling = enable != 0;
  return FFTB_OK;
}

fftb_status fftb_plan_get_profile(fftb_plan P, fftb_profile* out) {
  if (!P || !out) return fail(FFTB_ERR_INVALID, "null argument");
  for (auto& r : P->prof_pending) {
    hipError_t e = hipEventSynchronize(r.b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess) return fail(FFTB_ERR_HIP, std::string("hipEventElapsedTime: ") + hipGetErrorString(e));
    P->prof_launches[r.kid] += 1;
    P->prof_ms[r.kid] += ms;
    P->ev_pool.push_back(r.a);
    P->ev_pool.push_back(r.b);
  }
  P->prof_pending.clear();
  for (int k = 0; k < 5; ++k) {
    out->launches[k] = P->prof_launches[k];
    out->total_ms[k] = P->prof_ms[k];
    P->prof_launches[k] = 0;
    P->prof_ms[k] = 0;
  }
  return FFTB_OK;
}

fftb_status fftb_plan_destroy(fftb_plan P) {
  delete P;
  return FFTB_OK;
}

const char* fftb_status_string(fftb_status s) {
  switch (s) {
    case FFTB_OK: return "ok";
    case FFTB_ERR_INVALID: return "invalid argument";
    case FFTB_ERR_UNSUPPORTED: return "unsupported pattern";
    case FFTB_ERR_NOMEM: return "out of device memory";
    case FFTB_ERR_HIP: return "HIP runtime error";
  }
  return "unknown status";
}

const char* fftb_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

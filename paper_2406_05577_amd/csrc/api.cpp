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
}  // namespace fftb

using namespace fftb;

namespace {

thread_local std::string g_last_error;

fftb_status fail(fftb_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

constexpr size_t kLdsMax = 160 * 1024 - 1024;  // leave room for static LDS

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct fftb_plan_s {
  int nx = 0, ny = 0, nz = 0;
  fftb_dtype dtype = FFTB_C128;
  uint32_t flags = 0;
  std::vector<SphereTables> sph;
  std::vector<SphereDesc> desc;
  AxisPlan ax, ay, az;  // ay is the plan of the class length m
  fftb_tuning tun = {};
  int k1_tasks = 0, k2_tasks = 0;
  size_t lds1 = 0, lds2 = 0;
  int lds_P = 0, lds_X0 = 0, lds_X1 = 0;
  int64_t sphere_elems = 0, grid_elems = 0, col_elems = 0;
  int64_t total_coeffs = 0, total_columns = 0;
  int max_ncol = 0, max_nslab = 0;
  bool device = false;
  int num_cus = 256;
  // device memory
  std::vector<DevBuf> bufs;
  SphereDesc* d_desc = nullptr;
  int32_t *d_gidx = nullptr, *d_colidx = nullptr, *d_colxi = nullptr, *d_coly = nullptr,
          *d_xinv = nullptr;
  void *d_twx = nullptr, *d_twy = nullptr, *d_twz = nullptr, *d_twf = nullptr;
  void *d_twx_lo = nullptr, *d_twy_lo = nullptr, *d_twz_lo = nullptr, *d_twf_lo = nullptr;
  void* d_col = nullptr;
  unsigned int* d_counters = nullptr;
  size_t dev_bytes = 0;
  // graph cache per direction
  struct GraphCache {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    const void* in = nullptr;
    void* out = nullptr;
  } gc[2];
  hipStream_t cap_stream = nullptr;
  // per-kernel timing (FFTB profiling)
  bool profiling = false;
  struct ProfRec {
    int kid;
    hipEvent_t a, b;
  };
  std::vector<ProfRec> prof_pending;
  std::vector<hipEvent_t> ev_pool;
  int64_t prof_launches[4] = {0, 0, 0, 0};
  double prof_ms[4] = {0, 0, 0, 0};

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

// LDS bytes of the plane kernel for a given class count n1 and x batch lx.
bool plane_lds(const fftb_plan_s& P, int n1, int bc, int lx, size_t& bytes, int& offP, int& offX0,
               int& offX1, AxisPlan& aym) {
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
  const int64_t tot = S + Pn + nbx * X;
  bytes = static_cast<size_t>(tot) * es_of(P.dtype);
  return true;
}

fftb_status choose_tiling(fftb_plan_s& P, const fftb_tuning* user) {
  const int es = es_of(P.dtype);
  int maxnb = 1;
  for (auto& s : P.sph) maxnb = std::max(maxnb, s.nb);
  fftb_tuning t = {};
  if (user) t = *user;
  // band chunk
  int bc = t.band_chunk;
  if (bc == 0) {
    bc = (P.dtype == FFTB_C128) ? 8 : 16;
    int cap = 1;
    while (cap < maxnb) cap <<= 1;
    bc = std::min(bc, cap);
  }
  if (!is_pow2(bc) || bc > 64)
    return fail(FFTB_ERR_INVALID, "band_chunk must be a power of two in [1, 64]");
  int threads = t.threads ? t.threads : 256;
  if (threads != 64 && threads != 128 && threads != 256)
    return fail(FFTB_ERR_INVALID, "threads must be 64, 128 or 256");
  // column kernel tile
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
  if (lc < 1) return fail(FFTB_ERR_INVALID, "col_tile must be >= 1");
  P.lds1 = static_cast<size_t>(nbz) * lc * P.nz * bc * es;
  if (P.lds1 > kLdsMax)
    return fail(FFTB_ERR_UNSUPPORTED, "column kernel tile does not fit in LDS");
  // plane kernel: residue classes and x batch
  int n1 = t.y_classes, lx = t.x_rows;
  AxisPlan aym;
  size_t bytes = 0;
  int offP = 0, offX0 = 0, offX1 = 0;
  if (n1 == 0) {
    n1 = -1;
    for (int c = 1; c <= P.ny; ++c) {
      if (P.ny % c) continue;
      const int m = P.ny / c;
      const int want = std::min(m, lx ? lx : 2);
      if (!plane_lds(P, c, bc, want, bytes, offP, offX0, offX1, aym)) continue;
      if (bytes <= kLdsMax) {
        n1 = c;
        break;
      }
    }
    if (n1 < 0) return fail(FFTB_ERR_UNSUPPORTED, "no y-class split fits the plane in LDS");
  }
  if (n1 < 1 || P.ny % n1) return fail(FFTB_ERR_INVALID, "y_classes must divide ny");
  const int m = P.ny / n1;
  if (lx == 0) {
    // as many rows per batch as fit (all rows if the x plan is one stage)
    lx = 1;
    for (int c = m; c >= 1; --c) {
      if (!plane_lds(P, n1, bc, c, bytes, offP, offX0, offX1, aym)) break;
      if (bytes <= kLdsMax / 2 || c == 1) {
        lx = c;
        break;
      }
    }
  }
  if (lx < 1) return fail(FFTB_ERR_INVALID, "x_rows must be >= 1");
  lx = std::min(lx, m);
  if (!plane_lds(P, n1, bc, lx, bytes, offP, offX0, offX1, aym))
    return fail(FFTB_ERR_UNSUPPORTED, "class length has an unsupported factor");
  if (bytes > kLdsMax) return fail(FFTB_ERR_UNSUPPORTED, "plane kernel tile does not fit in LDS");
  P.ay = aym;
  P.lds2 = bytes;
  P.lds_P = offP;
  P.lds_X0 = offX0;
  P.lds_X1 = offX1;
  P.tun.band_chunk = bc;
  P.tun.y_classes = n1;
  P.tun.x_rows = lx;
  P.tun.col_tile = lc;
  P.tun.threads = threads;
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

// Build the per-sphere descriptors and task ranges for the current tiling.
void build_descs(fftb_plan_s& P) {
  const int bc = P.tun.band_chunk;
  const int64_t N = static_cast<int64_t>(P.nx) * P.ny * P.nz;
  P.desc.clear();
  int64_t soff = 0, goff = 0, coff = 0;
  int32_t gi = 0, ci = 0, cm = 0, xo = 0;
  int k1 = 0, k2 = 0;
  for (auto& s : P.sph) {
    SphereDesc d = {};
    d.sph_off = soff;
    d.grid_off = goff;
    d.col_off = coff;
    d.gidx_off = gi;
    d.colidx_off = ci;
    d.colmeta_off = cm;
    d.xinv_off = xo;
    d.ncol = s.ncol;
    d.nslab = s.nslab;
    d.nb = s.nb;
    d.nchunk = (s.nb + bc - 1) / bc;
    d.k1_start = k1;
    k1 += ((s.ncol + P.tun.col_tile - 1) / P.tun.col_tile) * d.nchunk;
    d.k1_end = k1;
    d.k2_start = k2;
    k2 += P.nz * d.nchunk;
    d.k2_end = k2;
    soff += s.ns * s.nb;
    goff += N * s.nb;
    coff += static_cast<int64_t>(d.nchunk) * bc * P.nz * s.ncol;
    gi += s.ncol * P.nz;
    ci += s.nslab * P.ny;
    cm += s.ncol;
    xo += P.nx;
    P.desc.push_back(d);
  }
  P.k1_tasks = k1;
  P.k2_tasks = k2;
  P.col_elems = coff;
}

fftb_status dev_alloc(fftb_plan_s& P, size_t bytes, void** out) {
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
  std::vector<int32_t> gidx, colidx, colxi, coly, xinv;
  for (auto& s : P.sph) {
    gidx.insert(gidx.end(), s.gidx.begin(), s.gidx.end());
    colidx.insert(colidx.end(), s.colidx.begin(), s.colidx.end());
    colxi.insert(colxi.end(), s.col_xi.begin(), s.col_xi.end());
    coly.insert(coly.end(), s.col_y.begin(), s.col_y.end());
    xinv.insert(xinv.end(), s.xinv.begin(), s.xinv.end());
  }
  fftb_status s;
  void* p;
  if ((s = upload(P, P.desc, &p, st)) != FFTB_OK) return s;
  P.d_desc = static_cast<SphereDesc*>(p);
  if ((s = upload(P, gidx, &p, st)) != FFTB_OK) return s;
  P.d_gidx = static_cast<int32_t*>(p);
  if ((s = upload(P, colidx, &p, st)) != FFTB_OK) return s;
  P.d_colidx = static_cast<int32_t*>(p);
  if ((s = upload(P, colxi, &p, st)) != FFTB_OK) return s;
  P.d_colxi = static_cast<int32_t*>(p);
  if ((s = upload(P, coly, &p, st)) != FFTB_OK) return s;
  P.d_coly = static_cast<int32_t*>(p);
  if ((s = upload(P, xinv, &p, st)) != FFTB_OK) return s;
  P.d_xinv = static_cast<int32_t*>(p);
  if ((s = upload_tw(P, axis_twiddles(P.ax), &P.d_twx, &P.d_twx_lo, st)) != FFTB_OK) return s;
  if ((s = upload_tw(P, axis_twiddles(P.ay), &P.d_twy, &P.d_twy_lo, st)) != FFTB_OK) return s;
  if ((s = upload_tw(P, axis_twiddles(P.az), &P.d_twz, &P.d_twz_lo, st)) != FFTB_OK) return s;
  if ((s = upload_tw(P, root_table(P.ny), &P.d_twf, &P.d_twf_lo, st)) != FFTB_OK) return s;
  if ((s = dev_alloc(P, static_cast<size_t>(P.col_elems) * es_of(P.dtype), &P.d_col)) != FFTB_OK)
    return s;
  if ((s = dev_alloc(P, 16 * sizeof(unsigned int), &p)) != FFTB_OK) return s;
  P.d_counters = static_cast<unsigned int*>(p);
  e = hipMemsetAsync(P.d_counters, 0, 16 * sizeof(unsigned int), st);
  if (e != hipSuccess) return fail(FFTB_ERR_HIP, std::string("hipMemsetAsync: ") + hipGetErrorString(e));
  e = prepare_kernels(P.dtype == FFTB_C128, std::max<size_t>(P.lds1, 4), std::max<size_t>(P.lds2, 4));
  if (e != hipSuccess)
    return fail(FFTB_ERR_HIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
  e = hipStreamSynchronize(st);
  if (e != hipSuccess)
    return fail(FFTB_ERR_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
  P.device = true;
  return FFTB_OK;
}

KArgs make_args(const fftb_plan_s& P, const void* in, void* out, bool inverse) {
  KArgs a;
  std::memset(&a, 0, sizeof a);
  a.nx = P.nx;
  a.ny = P.ny;
  a.nz = P.nz;
  a.bcl = ilog2(P.tun.band_chunk);
  a.n1 = P.tun.y_classes;
  a.m = P.ny / P.tun.y_classes;
  a.lx = P.tun.x_rows;
  a.lc = P.tun.col_tile;
  a.nsph = static_cast<int>(P.sph.size());
  a.k1_tasks = P.k1_tasks;
  a.k2_tasks = P.k2_tasks;
  a.persistent = (P.flags & FFTB_PLAN_BATCHED) ? 1 : 0;
  a.lds_P = P.lds_P;
  a.lds_X0 = P.lds_X0;
  a.lds_X1 = P.lds_X1;
  fill_axis(P.ax, a.ax);
  fill_axis(P.ay, a.ay);
  fill_axis(P.az, a.az);
  a.sph = P.d_desc;
  a.gidx = P.d_gidx;
  a.colidx = P.d_colidx;
  a.col_xi = P.d_colxi;
  a.col_y = P.d_coly;
  a.xinv = P.d_xinv;
  a.twx = P.d_twx;
  a.twy = P.d_twy;
  a.twz = P.d_twz;
  a.twf = P.d_twf;
  a.twx_lo = P.d_twx_lo;
  a.twy_lo = P.d_twy_lo;
  a.twz_lo = P.d_twz_lo;
  a.twf_lo = P.d_twf_lo;
  a.in = in;
  a.out = out;
  a.col = P.d_col;
  a.scale = inverse ? 1.0 : 1.0 / (static_cast<double>(P.nx) * P.ny * P.nz);
  a.counters = P.d_counters;
  (void)inverse;
  return a;
}

void grids(const fftb_plan_s& P, int& g1, int& g2) {
  if (P.flags & FFTB_PLAN_BATCHED) {
    // persistent: enough blocks to fill the chip, at least one per XCD queue
    const int occ1 = P.lds1 > 0 ? std::max<int>(1, static_cast<int>(kLdsMax / P.lds1)) : 8;
    const int occ2 = P.lds2 > 0 ? std::max<int>(1, static_cast<int>(kLdsMax / P.lds2)) : 8;
    g1 = std::max(8, std::min(P.num_cus * std::min(occ1, 8), ((P.k1_tasks + 7) / 8) * 8));
    g2 = std::max(8, std::min(P.num_cus * std::min(occ2, 8), ((P.k2_tasks + 7) / 8) * 8));
    g1 = (g1 + 7) / 8 * 8;
    g2 = (g2 + 7) / 8 * 8;
  } else {
    g1 = ((P.k1_tasks + 7) / 8) * 8;
    g2 = ((P.k2_tasks + 7) / 8) * 8;
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
hipError_t enqueue(fftb_plan_s* P, const KArgs& a, bool inverse, int g1, int g2, hipStream_t st,
                   bool profile) {
  const bool fp64 = P->dtype == FFTB_C128;
  hipError_t e = hipSuccess;
  if (a.persistent) {
    e = launch_reset(a.counters, st);
    if (e != hipSuccess) return e;
  }
  const int order[2] = {inverse ? 1 : 2, inverse ? 2 : 1};
  for (int which : order) {
    // kernel ids: 0 column inverse, 1 plane inverse, 2 plane forward, 3 column forward
    const int kid = inverse ? (which == 1 ? 0 : 1) : (which == 2 ? 2 : 3);
    hipEvent_t ea = nullptr, eb = nullptr;
    if (profile) {
      if ((e = get_event(P, &ea)) != hipSuccess) return e;
      if ((e = get_event(P, &eb)) != hipSuccess) return e;
      if ((e = hipEventRecord(ea, st)) != hipSuccess) return e;
    }
    e = launch_kernel(which, a, inverse, fp64, which == 1 ? g1 : g2, P->tun.threads,
                      which == 1 ? P->lds1 : P->lds2, st);
    if (e != hipSuccess) return e;
    if (profile) {
      if ((e = hipEventRecord(eb, st)) != hipSuccess) return e;
      P->prof_pending.push_back({kid, ea, eb});
    }
  }
  return hipSuccess;
}

fftb_status run(fftb_plan_s* P, const void* in, void* out, void* stream, bool inverse) {
  if (!P) return fail(FFTB_ERR_INVALID, "null plan");
  if (!P->device) return fail(FFTB_ERR_INVALID, "plan was created host-only");
  if (!in || !out) return fail(FFTB_ERR_INVALID, "null data pointer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int g1, g2;
  grids(*P, g1, g2);
  KArgs a = make_args(*P, in, out, inverse);
  if (P->flags & FFTB_PLAN_GRAPH) {
    auto& gc = P->gc[inverse ? 0 : 1];
    if (!gc.exec || gc.in != in || gc.out != out) {
      if (gc.exec) { (void)hipGraphExecDestroy(gc.exec); gc.exec = nullptr; }
      if (gc.graph) { (void)hipGraphDestroy(gc.graph); gc.graph = nullptr; }
      if (!P->cap_stream) {
        hipError_t e = hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return fail(FFTB_ERR_HIP, std::string("hipStreamCreate: ") + hipGetErrorString(e));
      }
      hipError_t e = hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return fail(FFTB_ERR_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
      hipError_t el = enqueue(P, a, inverse, g1, g2, P->cap_stream, false);
      e = hipStreamEndCapture(P->cap_stream, &gc.graph);
      if (el != hipSuccess) return fail(FFTB_ERR_HIP, std::string("launch during capture: ") + hipGetErrorString(el));
      if (e != hipSuccess) return fail(FFTB_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
      e = hipGraphInstantiate(&gc.exec, gc.graph, nullptr, nullptr, 0);
      if (e != hipSuccess) return fail(FFTB_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
      gc.in = in;
      gc.out = out;
    }
    hipError_t e = hipGraphLaunch(gc.exec, st);
    if (e != hipSuccess) return fail(FFTB_ERR_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    return FFTB_OK;
  }
  hipError_t e = enqueue(P, a, inverse, g1, g2, st, P->profiling);
  if (e != hipSuccess) return fail(FFTB_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
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
    fftb_status st = choose_tiling(*P, tuning);
    if (st != FFTB_OK) return st;
    build_descs(*P);
    if (!(flags & FFTB_PLAN_HOST_ONLY)) {
      st = device_setup(*P, static_cast<hipStream_t>(stream));
      if (st != FFTB_OK) return st;
    }
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
  for (int s = 0; s < P->ay.nst && s < 8; ++s) info->radix_y[s] = P->ay.R[s];
  for (int s = 0; s < P->az.nst && s < 8; ++s) info->radix_z[s] = P->az.R[s];
  info->tuning = P->tun;
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
  for (int k = 0; k < 4; ++k) {
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

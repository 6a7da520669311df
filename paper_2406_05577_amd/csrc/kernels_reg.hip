// Register-path kernels for gfx950. Each 1D transform line lives in the
// registers of H adjacent lanes (E = n/H values per lane, DFT_E in registers,
// DFT_H across the lanes), so the column kernel needs no LDS at all and the
// plane kernel uses LDS only for the y-class slab (and, in the forward
// direction, optionally for the column accumulators).
//
// Column kernel: z-transforms on the occupied (x,y) columns only (the padding
// along z is fused with the transform, Section 2.2).
// Plane kernel, inverse: task = (plane z, band chunk, y class r). The columns
// of each occupied slab x are folded into the class (one decimation-in-
// frequency stage evaluated for the single output class r), transformed along
// y with length m = ny/n1, then every row y = r + n1*k2 is transformed along x
// over the full grid and written. The n1 tasks of one (plane, chunk) are
// consecutive, so the blocks on one XCD read the same column data from L2.
// Plane kernel, forward: task = (plane z, band chunk); for each class r the
// rows y = r + n1*k2 are transformed along x keeping the occupied x only, then
// along y with length m, and the class's contribution w_ny^{-y*r} * Y[xi][y mod m]
// is accumulated into each column (a decimation-in-time combination over the
// classes, each column owned by one thread).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.hpp"

namespace fftb {


__device__ __forceinline__ int find_sphere_k1r(const KArgs& a, int t) {
  int s = 0;
  while (s + 1 < a.nsph && t >= a.sph[s].k1_end) ++s;
  return s;
}
__device__ __forceinline__ int find_sphere_k2r(const KArgs& a, int t) {
  int s = 0;
  while (s + 1 < a.nsph && t >= a.sph[s].k2_end) ++s;
  return s;
}

__device__ __forceinline__ int static_task_r(int total) {
  const int per = (total + 7) >> 3;
  const int t = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  return t < total ? t : -1;
}
__device__ __forceinline__ int dynamic_task_r(unsigned int* counters, int total) {
  const int per = (total + 7) >> 3;
  const int q = blockIdx.x & 7;
  const unsigned int idx = atomicAdd(&counters[q], 1u);
  const long t = static_cast<long>(q) * per + idx;
  return (static_cast<int>(idx) < per && t < total) ? static_cast<int>(t) : -1;
}

// ---------------------------------------------------------------------------
template <int S, typename T, int E, int H, bool MF>
__device__ void k1r_task(const KArgs& a, int t) {
  constexpr int L = log2_const<H>();
  const int s = find_sphere_k1r(a, t);
  const SphereDesc d = a.sph[s];
  const int lt = t - d.k1_start;
  const int ncb = (d.ncol + a.lc - 1) / a.lc;
  const int cb = lt % ncb, chunk = lt / ncb;
  const int c0 = cb * a.lc;
  const int nl = min(a.lc, d.ncol - c0);
  const int bcl = a.bcl, bmask = (1 << bcl) - 1;
  const int b0 = chunk << bcl;
  const int nz = a.nz, nb = d.nb, ncol = d.ncol;
  const int32_t* __restrict__ gidx = a.gidx + d.gidx_off;
  cpx<T>* __restrict__ colbuf = reinterpret_cast<cpx<T>*>(a.col) + d.col_off +
                                ((static_cast<int64_t>(chunk) * nz * ncol) << bcl);
  const cpx<T>* rootz = reinterpret_cast<const cpx<T>*>(a.rootz);
  const cpx<T>* rootz_lo = reinterpret_cast<const cpx<T>*>(a.rootz_lo);
  const int items = (nl << bcl) * H;
  // with the matrix-core codelet whole waves take part: pad to 64 lanes
  const int iters = MF ? ((items + 63) & ~63) : items;
  for (int it = threadIdx.x; it < iters; it += blockDim.x) {
    const bool valid = !MF || it < items;
    const int iv = valid ? it : 0;
    const int h = iv % H;
    const int rest = iv / H;
    const int bl = rest & bmask;
    const int c = c0 + (rest >> bcl);
    const int b = b0 + bl;
    cpx<T> v[E];
    if constexpr (S > 0) {
      const cpx<T>* __restrict__ in = reinterpret_cast<const cpx<T>*>(a.in) + d.sph_off;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int g = gidx[c * nz + h + H * j];
        v[j] = (valid && g >= 0 && b < nb) ? in[static_cast<int64_t>(g) * nb + b] : cpx<T>{0, 0};
      }
    } else {
#pragma unroll
      for (int j = 0; j < E; ++j)
        v[j] = valid ? colbuf[((static_cast<int64_t>(h + H * j) * ncol + c) << bcl) + bl]
                     : cpx<T>{0, 0};
    }
    line_fft<E, H, S, T, MF>(v, h, rootz, rootz_lo);
    const int q = bitrev_bits(h, L);
    if (!valid) continue;
    if constexpr (S > 0) {
#pragma unroll
      for (int k = 0; k < E; ++k)
        colbuf[((static_cast<int64_t>(k + E * q) * ncol + c) << bcl) + bl] = v[k];
    } else {
      cpx<T>* __restrict__ out = reinterpret_cast<cpx<T>*>(a.out) + d.sph_off;
      const T sc = static_cast<T>(a.scale);
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const int g = gidx[c * nz + k + E * q];
        if (g >= 0 && b < nb) out[static_cast<int64_t>(g) * nb + b] = cscale(v[k], sc);
      }
    }
  }
}

// ---------------------------------------------------------------------------
template <typename T, int E, int H, bool MF>
__device__ void k2r_inv_task(const KArgs& a, int t, cpx<T>* S) {
  constexpr int L = log2_const<H>();
  const int s = find_sphere_k2r(a, t);
  const SphereDesc d = a.sph[s];
  const int lt = t - d.k2_start;
  const int n1 = a.n1, m = a.m;
  const int r = lt % n1;
  const int rest0 = lt / n1;
  const int chunk = rest0 % d.nchunk, z = rest0 / d.nchunk;
  const int bcl = a.bcl, bmask = (1 << bcl) - 1;
  const int b0 = chunk << bcl;
  const int nx = a.nx, ny = a.ny, sx = a.sx;
  const int nb = d.nb, ncol = d.ncol, nslab = d.nslab;
  const int32_t* __restrict__ xinv = a.xinv + d.xinv_off;
  const int32_t* __restrict__ cy = a.col_y + d.colmeta_off;
  const int32_t* __restrict__ sst = a.slabstart + d.slab_off;
  const cpx<T>* __restrict__ colp = reinterpret_cast<const cpx<T>*>(a.col) + d.col_off +
                                    (((static_cast<int64_t>(chunk) * a.nz + z) * ncol) << bcl);
  const cpx<T>* twf = reinterpret_cast<const cpx<T>*>(a.twf);
  const cpx<T>* twfl = reinterpret_cast<const cpx<T>*>(a.twf_lo);
  const cpx<T>* rootx = reinterpret_cast<const cpx<T>*>(a.rootx);
  const cpx<T>* rootx_lo = reinterpret_cast<const cpx<T>*>(a.rootx_lo);

  // fold the slab's columns into class r, then y-IFFT of length m (one thread per line)
  const int nlines = nslab << bcl;
  for (int it = threadIdx.x; it < nlines; it += blockDim.x) {
    const int bl = it & bmask, xi = it >> bcl;
    cpx<T>* line = S + xi * sx + bl;
    for (int j = 0; j < m; ++j) line[j << bcl] = cpx<T>{0, 0};
    const int ce = sst[xi + 1];
    int c = sst[xi];
    // batches of FB columns: all loads in flight before the LDS updates
    constexpr int FB = sizeof(T) == 8 ? 8 : 16;
    for (; c + FB <= ce; c += FB) {
      cpx<T> v[FB];
      int yy[FB];
#pragma unroll
      for (int u = 0; u < FB; ++u) {
        yy[u] = cy[c + u];
        v[u] = colp[((c + u) << bcl) + bl];
      }
#pragma unroll
      for (int u = 0; u < FB; ++u) {
        cpx<T>* p = line + ((yy[u] % m) << bcl);
        *p = cadd(*p, twmul<+1>(v[u], twf, twfl, (yy[u] * r) % ny));
      }
    }
    for (; c < ce; ++c) {
      const int y = cy[c];
      const cpx<T> v = colp[(c << bcl) + bl];
      cpx<T>* p = line + ((y % m) << bcl);
      *p = cadd(*p, twmul<+1>(v, twf, twfl, (y * r) % ny));
    }
    cpx<T> u[kMaxRadixDev];
#pragma unroll
    for (int j = 0; j < kMaxRadixDev; ++j)
      if (j < m) u[j] = line[j << bcl];
    butterfly<+1>(m, u);
#pragma unroll
    for (int j = 0; j < kMaxRadixDev; ++j)
      if (j < m) line[j << bcl] = u[j];
  }
  __syncthreads();
  // x-IFFT of the class's rows, written to the grid
  cpx<T>* __restrict__ gout = reinterpret_cast<cpx<T>*>(a.out) + d.grid_off;
  const int items = (m << bcl) * H;
  const int iters = MF ? ((items + 63) & ~63) : items;
  for (int it = threadIdx.x; it < iters; it += blockDim.x) {
    const bool valid = !MF || it < items;
    const int iv = valid ? it : 0;
    const int h = iv % H;
    const int rest = iv / H;
    const int bl = rest & bmask, k2 = rest >> bcl;
    cpx<T> v[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int xi = xinv[h + H * j];
      v[j] = (valid && xi >= 0) ? S[xi * sx + (k2 << bcl) + bl] : cpx<T>{0, 0};
    }
    line_fft<E, H, +1, T, MF>(v, h, rootx, rootx_lo);
    const int q = bitrev_bits(h, L);
    const int y = r + n1 * k2;
    const int b = b0 + bl;
    if (valid && b < nb) {
      cpx<T>* row = gout + static_cast<int64_t>(z * ny + y) * nx * nb + b;
#pragma unroll
      for (int k = 0; k < E; ++k) row[static_cast<int64_t>(k + E * q) * nb] = v[k];
    }
  }
}

// ---------------------------------------------------------------------------
template <typename T, int E, int H, bool MF>
__device__ void k2r_fwd_task(const KArgs& a, int t, cpx<T>* S) {
  constexpr int L = log2_const<H>();
  const int s = find_sphere_k2r(a, t);
  const SphereDesc d = a.sph[s];
  const int lt = t - d.k2_start;
  // task = (plane, chunk, split): split q owns the slabs [x_lo, x_hi) and their columns
  const int q_split = lt % a.nsplit;
  const int rest0 = lt / a.nsplit;
  const int chunk = rest0 % d.nchunk, z = rest0 / d.nchunk;
  const int x_lo = a.splits[d.split_off + q_split], x_hi = a.splits[d.split_off + q_split + 1];
  const int bcl = a.bcl, bmask = (1 << bcl) - 1;
  const int b0 = chunk << bcl;
  const int nx = a.nx, ny = a.ny, n1 = a.n1, m = a.m, sx = a.sx;
  const int nb = d.nb, ncol = d.ncol, nslab = d.nslab;
  const int32_t* __restrict__ xinv = a.xinv + d.xinv_off;
  const int32_t* __restrict__ cy = a.col_y + d.colmeta_off;
  const int32_t* __restrict__ cxi = a.col_xi + d.colmeta_off;
  const int32_t* __restrict__ sst = a.slabstart + d.slab_off;
  cpx<T>* __restrict__ colp = reinterpret_cast<cpx<T>*>(a.col) + d.col_off +
                              (((static_cast<int64_t>(chunk) * a.nz + z) * ncol) << bcl);
  const cpx<T>* __restrict__ gin = reinterpret_cast<const cpx<T>*>(a.in) + d.grid_off;
  const cpx<T>* twf = reinterpret_cast<const cpx<T>*>(a.twf);
  const cpx<T>* twfl = reinterpret_cast<const cpx<T>*>(a.twf_lo);
  const cpx<T>* rootx = reinterpret_cast<const cpx<T>*>(a.rootx);
  const cpx<T>* rootx_lo = reinterpret_cast<const cpx<T>*>(a.rootx_lo);
  cpx<T>* acc = S + a.lds_acc;
  const bool acc_lds = a.acc_lds != 0;
  const int c_lo = sst[x_lo];
  (void)nslab;

  for (int r = 0; r < n1; ++r) {
    // x-FFT of the class's rows, keeping the occupied x
    const int items = (m << bcl) * H;
    const int iters = MF ? ((items + 63) & ~63) : items;
    for (int it = threadIdx.x; it < iters; it += blockDim.x) {
      const bool valid = !MF || it < items;
      const int iv = valid ? it : 0;
      const int h = iv % H;
      const int rest = iv / H;
      const int bl = rest & bmask, k2 = rest >> bcl;
      const int y = r + n1 * k2;
      const int b = b0 + bl;
      cpx<T> v[E];
      const cpx<T>* row = gin + static_cast<int64_t>(z * ny + y) * nx * nb + b;
#pragma unroll
      for (int j = 0; j < E; ++j)
        v[j] = (valid && b < nb) ? row[static_cast<int64_t>(h + H * j) * nb] : cpx<T>{0, 0};
      line_fft<E, H, -1, T, MF>(v, h, rootx, rootx_lo);
      const int q = bitrev_bits(h, L);
      if (!valid) continue;
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const int xi = xinv[k + E * q] - x_lo;
        if (xi >= 0 && xi < x_hi - x_lo) S[xi * sx + (k2 << bcl) + bl] = v[k];
      }
    }
    __syncthreads();
    // y-FFT of length m per occupied x of the split, in place
    const int nlines = (x_hi - x_lo) << bcl;
    for (int it = threadIdx.x; it < nlines; it += blockDim.x) {
      const int bl = it & bmask, xl = it >> bcl;
      cpx<T>* line = S + xl * sx + bl;
      cpx<T> u[kMaxRadixDev];
#pragma unroll
      for (int j = 0; j < kMaxRadixDev; ++j)
        if (j < m) u[j] = line[j << bcl];
      butterfly<-1>(m, u);
#pragma unroll
      for (int j = 0; j < kMaxRadixDev; ++j)
        if (j < m) line[j << bcl] = u[j];
    }
    __syncthreads();
    // the class's contribution w_ny^{-y*r} * Y[xi][y mod m] to each column of the
    // split, one (column, band) item per thread
    const int c_hi = sst[x_hi];
    const int nitems = (c_hi - c_lo) << bcl;
    for (int it = threadIdx.x; it < nitems; it += blockDim.x) {
      const int bl = it & bmask, cl = it >> bcl, c = c_lo + cl;
      const int y = cy[c];
      const cpx<T> val =
          twmul<-1>(S[(cxi[c] - x_lo) * sx + ((y % m) << bcl) + bl], twf, twfl, (y * r) % ny);
      cpx<T>* g = colp + (c << bcl) + bl;
      if (acc_lds) {
        cpx<T>* p = acc + it;
        if (n1 == 1) *g = val;
        else if (r == 0) *p = val;
        else if (r < n1 - 1) *p = cadd(*p, val);
        else *g = cadd(*p, val);
      } else {
        *g = (r == 0) ? val : cadd(*g, val);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
template <int S, typename T, int E, int H, bool MF>
__global__ void __launch_bounds__(256) k1r_kernel(const KArgs a) {
  if (!a.persistent) {
    const int t = static_task_r(a.k1_tasks);
    if (t >= 0) k1r_task<S, T, E, H, MF>(a, t);
    return;
  }
  __shared__ int sh_task;
  for (;;) {
    if (threadIdx.x == 0) sh_task = dynamic_task_r(a.counters, a.k1_tasks);
    __syncthreads();
    const int t = sh_task;
    __syncthreads();
    if (t < 0) break;
    k1r_task<S, T, E, H, MF>(a, t);
  }
}

template <int S, typename T, int E, int H, bool MF>
__global__ void __launch_bounds__(512) k2r_kernel(const KArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  if (!a.persistent) {
    const int t = static_task_r(a.k2_tasks);
    if (t >= 0) {
      if constexpr (S > 0) k2r_inv_task<T, E, H, MF>(a, t, lds);
      else k2r_fwd_task<T, E, H, MF>(a, t, lds);
    }
    return;
  }
  __shared__ int sh_task;
  for (;;) {
    if (threadIdx.x == 0) sh_task = dynamic_task_r(a.counters + 8, a.k2_tasks);
    __syncthreads();
    const int t = sh_task;
    __syncthreads();
    if (t < 0) break;
    if constexpr (S > 0) k2r_inv_task<T, E, H, MF>(a, t, lds);
    else k2r_fwd_task<T, E, H, MF>(a, t, lds);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// (E, H) pairs compiled for each precision; the host picks one per axis.
#define FFTB_REG_SHAPES_F64(X) \
  X(4, 1) X(5, 1) X(6, 1) X(8, 1) X(9, 1) X(10, 1) X(12, 1) X(15, 1) X(16, 1) \
  X(5, 4) X(6, 4) X(4, 8) X(12, 8) X(16, 8) X(18, 8) X(20, 8) X(45, 4)
#define FFTB_REG_SHAPES_F32(X) \
  X(4, 1) X(5, 1) X(6, 1) X(8, 1) X(9, 1) X(10, 1) X(12, 1) X(15, 1) X(16, 1) \
  X(5, 4) X(6, 4) X(4, 8) X(12, 8) X(16, 8) X(18, 8) X(20, 8) X(45, 4)

bool reg_shape_supported(bool fp64, int E, int H) {
#define FFTB_CHK(e, h) if (E == e && H == h) return true;
  if (fp64) {
    FFTB_REG_SHAPES_F64(FFTB_CHK)
  } else {
    FFTB_REG_SHAPES_F32(FFTB_CHK)
  }
#undef FFTB_CHK
  return false;
}

template <int S, typename T, int E, int H, bool MF>
static hipError_t launch_one(int which, const KArgs& a, int grid, int threads, size_t lds,
                             hipStream_t st) {
  if (which == 1)
    hipLaunchKernelGGL((k1r_kernel<S, T, E, H, MF>), dim3(grid), dim3(threads), 0, st, a);
  else
    hipLaunchKernelGGL((k2r_kernel<S, T, E, H, MF>), dim3(grid), dim3(threads), lds, st, a);
  return hipGetLastError();
}

template <int S, typename T, int E, int H, bool MF>
static hipError_t attr_one(size_t lds) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k2r_kernel<S, T, E, H, MF>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

// the FP32 DFT_16 on the matrix cores is compiled for lines of 16 values per lane
bool mfma_shape_supported(bool fp64, int E, int H) { return !fp64 && E == 16 && H == 8; }

// which: 1 = column kernel (E, H of the z axis), 2 = plane kernel (E, H of x)
hipError_t launch_reg(int which, const KArgs& a, bool inverse, bool fp64, int E, int H, int grid,
                      int threads, size_t lds, hipStream_t st, bool mfma) {
  if (mfma) {
    if (fp64 || E != 16 || H != 8) return hipErrorInvalidValue;
    return inverse ? launch_one<+1, float, 16, 8, true>(which, a, grid, threads, lds, st)
                   : launch_one<-1, float, 16, 8, true>(which, a, grid, threads, lds, st);
  }
#define FFTB_L64(e, h)                                                                     \
  if (E == e && H == h)                                                                    \
    return inverse ? launch_one<+1, double, e, h, false>(which, a, grid, threads, lds, st) \
                   : launch_one<-1, double, e, h, false>(which, a, grid, threads, lds, st);
#define FFTB_L32(e, h)                                                                     \
  if (E == e && H == h)                                                                    \
    return inverse ? launch_one<+1, float, e, h, false>(which, a, grid, threads, lds, st)  \
                   : launch_one<-1, float, e, h, false>(which, a, grid, threads, lds, st);
  if (fp64) {
    FFTB_REG_SHAPES_F64(FFTB_L64)
  } else {
    FFTB_REG_SHAPES_F32(FFTB_L32)
  }
#undef FFTB_L64
#undef FFTB_L32
  return hipErrorInvalidValue;
}

hipError_t prepare_reg(bool fp64, int E, int H, size_t lds, bool mfma) {
  if (mfma) {
    if (fp64 || E != 16 || H != 8) return hipErrorInvalidValue;
    hipError_t err = attr_one<+1, float, 16, 8, true>(lds);
    return err != hipSuccess ? err : attr_one<-1, float, 16, 8, true>(lds);
  }
#define FFTB_A64(e, h)                                                      \
  if (E == e && H == h) {                                                   \
    hipError_t err = attr_one<+1, double, e, h, false>(lds);                \
    return err != hipSuccess ? err : attr_one<-1, double, e, h, false>(lds); \
  }
#define FFTB_A32(e, h)                                                     \
  if (E == e && H == h) {                                                  \
    hipError_t err = attr_one<+1, float, e, h, false>(lds);                \
    return err != hipSuccess ? err : attr_one<-1, float, e, h, false>(lds); \
  }
  if (fp64) {
    FFTB_REG_SHAPES_F64(FFTB_A64)
  } else {
    FFTB_REG_SHAPES_F32(FFTB_A32)
  }
#undef FFTB_A64
#undef FFTB_A32
  return hipErrorInvalidValue;
}

}  // namespace fftb

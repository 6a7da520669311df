// HIP kernels for gfx950: the column kernel (z-transforms on the occupied
// columns) and the plane kernel (y-transforms on the occupied slab, then
// x-transforms on every row of the plane), both directions, FP64 and FP32.
//
// Method (paper, Section 2.2): the sphere is zero-padded one axis at a time and
// each padding step is fused with the 1D transforms on that axis, so the z pass
// touches only the columns of the xy-projection (the offset array of Section
// 3.3), the y pass only the occupied x planes, and only the x pass the full grid.
// Each 1D transform is a mixed-radix Cooley-Tukey FFT (Section 2.1) executed as
// Stockham stages with radices 2..16 in registers and LDS exchanges between
// stages.
//
// Data layout: band index fastest everywhere (Section 3.3). A workgroup tile
// holds a chunk of 2^bcl consecutive bands; lanes map to bands first, so every
// global access of a wavefront covers contiguous band segments and every LDS
// access is bank-linear.
#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace fftb {

// One Stockham stage over `nlines` lines of length n (radix R, sub-transform
// length p): item (line, i, band) reads x[i + q*n/R], twiddles by
// w_{pR}^{q*(i mod p)}, applies DFT_R and writes y[(i - i mod p)*R + i mod p + q*p].
template <int S, typename T, class Src, class Dst>
__device__ __forceinline__ void stage_run(int nlines, int n, int R, int p, const cpx<T>* tw,
                                          const cpx<T>* twlo, int bcl, Src src, Dst dst) {
  const int nq = n / R;
  const int bmask = (1 << bcl) - 1;
  const int total = (nlines * nq) << bcl;
  for (int it = threadIdx.x; it < total; it += blockDim.x) {
    const int bl = it & bmask;
    const int rest = it >> bcl;
    const int line = rest / nq;
    const int i = rest - line * nq;
    const int k = i % p;
    cpx<T> v[kMaxRadixDev];
#pragma unroll
    for (int q = 0; q < kMaxRadixDev; ++q)
      if (q < R) v[q] = src(line, i + q * nq, bl);
    if (p > 1) {
#pragma unroll
      for (int q = 1; q < kMaxRadixDev; ++q)
        if (q < R) v[q] = twmul<S>(v[q], tw, twlo, k * R + q);
    }
    butterfly<S>(R, v);
    const int j = (i - k) * R + k;
#pragma unroll
    for (int q = 0; q < kMaxRadixDev; ++q)
      if (q < R) dst(line, j + q * p, bl, v[q]);
  }
}

template <typename T>
struct LdsSrc {
  const cpx<T>* buf;
  int n, bcl;
  __device__ __forceinline__ cpx<T> operator()(int line, int pos, int bl) const {
    return buf[((line * n + pos) << bcl) + bl];
  }
};
template <typename T>
struct LdsDst {
  cpx<T>* buf;
  int n, bcl;
  __device__ __forceinline__ void operator()(int line, int pos, int bl, cpx<T> v) const {
    buf[((line * n + pos) << bcl) + bl] = v;
  }
};

// Run every stage of an axis plan: the first stage reads through `gsrc`, the
// last writes through `gdst`, intermediate results ping-pong between LDS
// buffers b0 and b1 (each nlines*n*2^bcl elements).
template <int S, typename T, class GSrc, class GDst>
__device__ __forceinline__ void axis_run(const AxisDev& ap, int nlines, const cpx<T>* tw,
                                         const cpx<T>* twlo, int bcl, cpx<T>* b0, cpx<T>* b1,
                                         GSrc gsrc, GDst gdst) {
  const int n = ap.n, nst = ap.nst;
  if (nst == 1) {
    stage_run<S, T>(nlines, n, ap.R[0], ap.p[0], tw + ap.twoff[0], twlo ? twlo + ap.twoff[0] : twlo,
                    bcl, gsrc, gdst);
    return;
  }
  stage_run<S, T>(nlines, n, ap.R[0], ap.p[0], tw + ap.twoff[0], twlo ? twlo + ap.twoff[0] : twlo,
                  bcl, gsrc, LdsDst<T>{b0, n, bcl});
  __syncthreads();
  for (int s = 1; s < nst - 1; ++s) {
    cpx<T>* from = (s & 1) ? b0 : b1;
    cpx<T>* to = (s & 1) ? b1 : b0;
    stage_run<S, T>(nlines, n, ap.R[s], ap.p[s], tw + ap.twoff[s], twlo ? twlo + ap.twoff[s] : twlo,
                    bcl, LdsSrc<T>{from, n, bcl}, LdsDst<T>{to, n, bcl});
    __syncthreads();
  }
  const int s = nst - 1;
  const cpx<T>* from = (s & 1) ? b0 : b1;
  stage_run<S, T>(nlines, n, ap.R[s], ap.p[s], tw + ap.twoff[s], twlo ? twlo + ap.twoff[s] : twlo,
                  bcl, LdsSrc<T>{from, n, bcl}, gdst);
}

__device__ __forceinline__ int find_sphere_k1(const KArgs& a, int t) {
  int s = 0;
  while (s + 1 < a.nsph && t >= a.sph[s].k1_end) ++s;
  return s;
}
__device__ __forceinline__ int find_sphere_k2(const KArgs& a, int t) {
  int s = 0;
  while (s + 1 < a.nsph && t >= a.sph[s].k2_end) ++s;
  return s;
}

// ---------------------------------------------------------------------------
// Column kernel task: LC columns x one band chunk, z-transform of length nz.
// S > 0: sphere -> (pad z) -> z-IFFT -> column scratch.
// S < 0: column scratch -> z-FFT -> gather the sphere's z values, scale 1/N.
template <int S, typename T>
__device__ void k1_task(const KArgs& a, int t, cpx<T>* lds) {
  const int s = find_sphere_k1(a, t);
  const SphereDesc d = a.sph[s];
  const int lt = t - d.k1_start;
  const int chunk = lt % d.nchunk, cb = lt / d.nchunk;
  const int c0 = cb * a.lc;
  const int nl = min(a.lc, d.ncol - c0);
  const int bcl = a.bcl, bc = 1 << bcl;
  const int b0 = chunk << bcl;
  const int nz = a.nz, nb = d.nb, npcol = d.npcol;
  const int32_t* __restrict__ cslot = a.col_slot + d.colmeta_off;
  const int32_t* __restrict__ gidx = a.gidx + d.gidx_off;
  cpx<T>* colbuf = reinterpret_cast<cpx<T>*>(a.col) + d.col_off;
  const cpx<T>* tw = reinterpret_cast<const cpx<T>*>(a.twz);
  const cpx<T>* twlo = reinterpret_cast<const cpx<T>*>(a.twz_lo);
  cpx<T>* b_0 = lds;
  cpx<T>* b_1 = lds + ((a.lc * nz) << bcl);
  const int64_t nbp = d.nbp;  // band vector stride per (z, column)
  if constexpr (S > 0) {
    const cpx<T>* __restrict__ in = reinterpret_cast<const cpx<T>*>(a.in) + d.sph_off;
    auto gsrc = [=](int line, int z, int bl) -> cpx<T> {
      const int g = gidx[(c0 + line) * nz + z];
      const int b = b0 + bl;
      if (g >= 0 && b < nb) return in[static_cast<int64_t>(g) * nb + b];
      return cpx<T>{0, 0};
    };
    auto gdst = [=](int line, int z, int bl, cpx<T> v) {
      colbuf[(static_cast<int64_t>(z) * npcol + cslot[c0 + line]) * nbp + b0 + bl] = v;
    };
    axis_run<S, T>(a.az, nl, tw, twlo, bcl, b_0, b_1, gsrc, gdst);
  } else {
    cpx<T>* __restrict__ out = reinterpret_cast<cpx<T>*>(a.out) + d.sph_off;
    const T sc = static_cast<T>(a.scale);
    auto gsrc = [=](int line, int z, int bl) -> cpx<T> {
      return colbuf[(static_cast<int64_t>(z) * npcol + cslot[c0 + line]) * nbp + b0 + bl];
    };
    auto gdst = [=](int line, int z, int bl, cpx<T> v) {
      const int g = gidx[(c0 + line) * nz + z];
      const int b = b0 + bl;
      if (g >= 0 && b < nb) out[static_cast<int64_t>(g) * nb + b] = cscale(v, sc);
    };
    axis_run<S, T>(a.az, nl, tw, twlo, bcl, b_0, b_1, gsrc, gdst);
  }
  (void)bc;
}

// Plane kernel task: one z-plane x one band chunk, looping over the n1 residue
// classes r of the y output index (y = r + n1*k2, k2 < m).
//  S > 0: fold the plane's columns into the class (S[xi][j2] = sum_t
//         col(xi, j2 + m*t) * w_ny^{+(j2+m*t)*r}), y-IFFT of length m on every
//         occupied x, then x-IFFT of every row of the class -> grid.
//  S < 0: x-FFT of the class's rows keeping the occupied x, y-FFT of length m,
//         then col(xi, y) += w_ny^{-y*r} * Y[xi][y mod m].
template <int S, typename T>
__device__ void k2_task(const KArgs& a, int t, cpx<T>* lds) {
  const int s = find_sphere_k2(a, t);
  const SphereDesc d = a.sph[s];
  const int lt = t - d.k2_start;
  const int chunk = lt % d.nchunk, z = lt / d.nchunk;
  const int bcl = a.bcl;
  const int bmask = (1 << bcl) - 1;
  const int b0 = chunk << bcl;
  const int nx = a.nx, ny = a.ny, n1 = a.n1, m = a.m;
  const int nb = d.nb, ncol = d.ncol, nslab = d.nslab, npcol = d.npcol;
  const int32_t* __restrict__ colidx = a.colidx + d.colidx_off;  // (slab, y) -> slot
  const int32_t* __restrict__ cslot = a.col_slot + d.colmeta_off;
  const int32_t* __restrict__ xinv = a.xinv + d.xinv_off;
  const int32_t* __restrict__ cxi = a.col_xi + d.colmeta_off;
  const int32_t* __restrict__ cy = a.col_y + d.colmeta_off;
  const int64_t nbp = d.nbp;
  cpx<T>* colp =
      reinterpret_cast<cpx<T>*>(a.col) + d.col_off + static_cast<int64_t>(z) * npcol * nbp + b0;
  const cpx<T>* twx = reinterpret_cast<const cpx<T>*>(a.twx);
  const cpx<T>* twxl = reinterpret_cast<const cpx<T>*>(a.twx_lo);
  const cpx<T>* twy = reinterpret_cast<const cpx<T>*>(a.twy);
  const cpx<T>* twyl = reinterpret_cast<const cpx<T>*>(a.twy_lo);
  const cpx<T>* twf = reinterpret_cast<const cpx<T>*>(a.twf);
  const cpx<T>* twfl = reinterpret_cast<const cpx<T>*>(a.twf_lo);
  cpx<T>* Sb = lds;
  cpx<T>* Pb = lds + a.lds_P;
  cpx<T>* X0 = lds + a.lds_X0;
  cpx<T>* X1 = lds + a.lds_X1;
  // result buffer of the y stages: single stage runs in place in Sb
  cpx<T>* Yb = (a.ay.nst == 1 || (a.ay.nst & 1) == 0) ? Sb : Pb;

  for (int r = 0; r < n1; ++r) {
    if constexpr (S > 0) {
      // fold
      const int total = (nslab * m) << bcl;
      for (int it = threadIdx.x; it < total; it += blockDim.x) {
        const int bl = it & bmask;
        const int rest = it >> bcl;
        const int xi = rest / m, j2 = rest - xi * m;
        cpx<T> acc = {0, 0};
        for (int tt = 0; tt < n1; ++tt) {
          const int y = j2 + m * tt;
          const int c = colidx[xi * ny + y];
          if (c >= 0) {
            const cpx<T> v = colp[static_cast<int64_t>(c) * nbp + bl];
            acc = cadd(acc, twmul<S>(v, twf, twfl, (y * r) % ny));
          }
        }
        Sb[it] = acc;
      }
      __syncthreads();
      // y stages (in place for one stage, else ping-pong Sb/Pb)
      if (a.ay.nst == 1) {
        stage_run<S, T>(nslab, m, a.ay.R[0], 1, twy, twyl, bcl, LdsSrc<T>{Sb, m, bcl},
                        LdsDst<T>{Sb, m, bcl});
      } else {
        for (int st = 0; st < a.ay.nst; ++st) {
          cpx<T>* from = (st & 1) ? Pb : Sb;
          cpx<T>* to = (st & 1) ? Sb : Pb;
          stage_run<S, T>(nslab, m, a.ay.R[st], a.ay.p[st], twy + a.ay.twoff[st],
                          twyl ? twyl + a.ay.twoff[st] : twyl, bcl, LdsSrc<T>{from, m, bcl},
                          LdsDst<T>{to, m, bcl});
          if (st + 1 < a.ay.nst) __syncthreads();
        }
      }
      __syncthreads();
      // x transforms of the class's rows, lx rows at a time
      cpx<T>* __restrict__ gout = reinterpret_cast<cpx<T>*>(a.out) + d.grid_off;
      for (int rb = 0; rb < m; rb += a.lx) {
        const int nrows = min(a.lx, m - rb);
        auto gsrc = [=](int line, int x, int bl) -> cpx<T> {
          const int xi = xinv[x];
          if (xi >= 0) return Yb[((xi * m + rb + line) << bcl) + bl];
          return cpx<T>{0, 0};
        };
        const T* __restrict__ pot = reinterpret_cast<const T*>(a.pot);
        auto gdst = [=](int line, int x, int bl, cpx<T> v) {
          const int y = r + n1 * (rb + line);
          const int b = b0 + bl;
          const int64_t p = static_cast<int64_t>(z * ny + y) * nx + x;
          if (pot) v = cscale(v, pot[p]);  // fused real-space potential
          if (b < nb) gout[p * nb + b] = v;
        };
        axis_run<S, T>(a.ax, nrows, twx, twxl, bcl, X0, X1, gsrc, gdst);
        __syncthreads();
      }
    } else {
      const cpx<T>* __restrict__ gin = reinterpret_cast<const cpx<T>*>(a.in) + d.grid_off;
      for (int rb = 0; rb < m; rb += a.lx) {
        const int nrows = min(a.lx, m - rb);
        auto gsrc = [=](int line, int x, int bl) -> cpx<T> {
          const int y = r + n1 * (rb + line);
          const int b = b0 + bl;
          if (b < nb) return gin[(static_cast<int64_t>(z * ny + y) * nx + x) * nb + b];
          return cpx<T>{0, 0};
        };
        auto gdst = [=](int line, int x, int bl, cpx<T> v) {
          const int xi = xinv[x];
          if (xi >= 0) Sb[((xi * m + rb + line) << bcl) + bl] = v;
        };
        axis_run<S, T>(a.ax, nrows, twx, twxl, bcl, X0, X1, gsrc, gdst);
        __syncthreads();
      }
      if (a.ay.nst == 1) {
        stage_run<S, T>(nslab, m, a.ay.R[0], 1, twy, twyl, bcl, LdsSrc<T>{Sb, m, bcl},
                        LdsDst<T>{Sb, m, bcl});
      } else {
        for (int st = 0; st < a.ay.nst; ++st) {
          cpx<T>* from = (st & 1) ? Pb : Sb;
          cpx<T>* to = (st & 1) ? Sb : Pb;
          stage_run<S, T>(nslab, m, a.ay.R[st], a.ay.p[st], twy + a.ay.twoff[st],
                          twyl ? twyl + a.ay.twoff[st] : twyl, bcl, LdsSrc<T>{from, m, bcl},
                          LdsDst<T>{to, m, bcl});
          if (st + 1 < a.ay.nst) __syncthreads();
        }
      }
      __syncthreads();
      // unfold into the columns
      const int total = ncol << bcl;
      for (int it = threadIdx.x; it < total; it += blockDim.x) {
        const int bl = it & bmask;
        const int c = it >> bcl;
        const int xi = cxi[c], y = cy[c];
        const int ym = y % m;
        cpx<T> v = twmul<S>(Yb[((xi * m + ym) << bcl) + bl], twf, twfl, (y * r) % ny);
        cpx<T>* p = colp + (static_cast<int64_t>(cslot[c]) * nbp + bl);
        if (r > 0) v = cadd(v, *p);
        *p = v;
      }
      __syncthreads();
    }
  }
}

template <int S, typename T>
__global__ void __launch_bounds__(256) k1_kernel(const KArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  if (!a.persistent) {
    const int t = static_task_g(a.k1_tasks, 1);
    if (t >= 0) k1_task<S, T>(a, t, lds);
    return;
  }
  __shared__ int sh_task;
  for (;;) {
    if (threadIdx.x == 0) sh_task = dynamic_task_g(a.counters, a.k1_tasks, 1);
    __syncthreads();
    const int t = sh_task;
    __syncthreads();
    if (t < 0) break;
    k1_task<S, T>(a, t, lds);
    __syncthreads();
  }
}

template <int S, typename T>
__global__ void __launch_bounds__(256) k2_kernel(const KArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  if (!a.persistent) {
    const int t = static_task_g(a.k2_tasks, 1);
    if (t >= 0) k2_task<S, T>(a, t, lds);
    return;
  }
  __shared__ int sh_task;
  for (;;) {
    if (threadIdx.x == 0) sh_task = dynamic_task_g(a.counters + 8, a.k2_tasks, 1);
    __syncthreads();
    const int t = sh_task;
    __syncthreads();
    if (t < 0) break;
    k2_task<S, T>(a, t, lds);
    __syncthreads();
  }
}

__global__ void reset_counters(unsigned int* c) {
  if (threadIdx.x < 24) c[threadIdx.x] = 0u;
}

// ---------------------------------------------------------------------------
// Host-side launchers (called from the C ABI layer).
template <int S, typename T>
static hipError_t set_attrs(size_t lds1, size_t lds2) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k1_kernel<S, T>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds1);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k2_kernel<S, T>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2);
}

hipError_t prepare_kernels(bool fp64, size_t lds1, size_t lds2) {
  hipError_t e = fp64 ? set_attrs<+1, double>(lds1, lds2) : set_attrs<+1, float>(lds1, lds2);
  if (e != hipSuccess) return e;
  return fp64 ? set_attrs<-1, double>(lds1, lds2) : set_attrs<-1, float>(lds1, lds2);
}

hipError_t launch_reset(unsigned int* counters, hipStream_t st) {
  hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, st, counters);
  return hipGetLastError();
}

// which: 1 = column kernel, 2 = plane kernel
hipError_t launch_kernel(int which, const KArgs& a, bool inverse, bool fp64, int grid, int threads,
                         size_t lds, hipStream_t st) {
  if (which == 1) {
    if (inverse) {
      if (fp64) hipLaunchKernelGGL((k1_kernel<+1, double>), dim3(grid), dim3(threads), lds, st, a);
      else hipLaunchKernelGGL((k1_kernel<+1, float>), dim3(grid), dim3(threads), lds, st, a);
    } else {
      if (fp64) hipLaunchKernelGGL((k1_kernel<-1, double>), dim3(grid), dim3(threads), lds, st, a);
      else hipLaunchKernelGGL((k1_kernel<-1, float>), dim3(grid), dim3(threads), lds, st, a);
    }
  } else {
    if (inverse) {
      if (fp64) hipLaunchKernelGGL((k2_kernel<+1, double>), dim3(grid), dim3(threads), lds, st, a);
      else hipLaunchKernelGGL((k2_kernel<+1, float>), dim3(grid), dim3(threads), lds, st, a);
    } else {
      if (fp64) hipLaunchKernelGGL((k2_kernel<-1, double>), dim3(grid), dim3(threads), lds, st, a);
      else hipLaunchKernelGGL((k2_kernel<-1, float>), dim3(grid), dim3(threads), lds, st, a);
    }
  }
  return hipGetLastError();
}

}  // namespace fftb

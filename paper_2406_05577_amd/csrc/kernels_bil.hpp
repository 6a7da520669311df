// Band-inner register-line kernels (bline.hpp): the column kernel, and the
// dispatch of the plane kernels whose x transforms run on band-inner lines
// (their fold, y transforms and class partials are those of kernels_reg.hpp).
// Instantiated in the bil_*.hip translation units.
#pragma once

#include "kernels_reg.hpp"

namespace fftb {

// Column kernel on band-inner lines. Task = `lc` columns x one band chunk (one
// 128-byte piece); one z line (one column, all bands of the chunk) per
// wavefront, or two for positions of half a wavefront.
// Inverse (S > 0): the sphere coefficients of each column are read through the
// (column, z) table (zeros elsewhere: the z padding is never stored, Section
// 2.2), transformed along z and written to the column scratch.
// Forward (S < 0): the column is read from the scratch, transformed, and only
// the sphere's z values are gathered, scaled by 1/N.
template <int S, typename T, int E, int H>
__device__ void k1b_task(const KArgs& a, int t, const TwEntry<T>* tab) {
  using Lane = BLane<T, H>;
  const Lane ln;
  const int s = find_sphere_k1r(a, t);
  const SphereDesc d = a.sph[s];
  const int lt = t - d.k1_start;
  const int chunk = lt % d.nchunk, cb = lt / d.nchunk;
  const int c0 = cb * a.lc;
  const int nl = min(a.lc, d.ncol - c0);
  const int b0 = chunk << a.bcl;
  int h = ln.h;
  asm volatile("" : "+v"(h));
  const int q = bitrev_bits(h, log2_const<H>());
  const auto ctx = bline_ctx<E, H, S, T>(h, tab);
  const int nz = a.nz, nb = d.nb, npcol = d.npcol, nbp = d.nbp;
  const int32_t* __restrict__ cslot = a.col_slot + d.colmeta_off;
  const int32_t* __restrict__ gidx = a.gidx + d.gidx_off;
  cpx<T>* __restrict__ colbuf = reinterpret_cast<cpx<T>*>(a.col) + d.col_off + b0;
  const int b = b0 + ln.bl;
  const bool bok = b < nb;
  constexpr unsigned es = sizeof(cpx<T>);
  const unsigned nbp_es = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(nbp) * es);
  const unsigned zstep_out = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(npcol) * nbp_es);
  const unsigned zstep_in = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(H * npcol) * nbp_es);
  const __amdgpu_buffer_rsrc_t rcol = buf_rsrc(colbuf);
  const cpx<T>* __restrict__ sin_ = reinterpret_cast<const cpx<T>*>(a.in) + d.sph_off;
  cpx<T>* __restrict__ sout = reinterpret_cast<cpx<T>*>(a.out) + d.sph_off;
  const __amdgpu_buffer_rsrc_t rsph = buf_rsrc(S > 0 ? sin_ : sout);
  const int wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  for (int base = wave * Lane::LPW; base < nl; base += nwave * Lane::LPW) {
    const int ci = base + ln.sub;
    const bool ok = ci < nl;
    const int c = c0 + (ok ? ci : 0);
    const int slot = cslot[c];
    cpx<T> v[E];
    // (band-inner plans keep every sphere's coefficients and column region
    // below 4 GiB: 32-bit buffer offsets)
    if constexpr (S > 0) {
      int g[E];
#pragma unroll
      for (int j = 0; j < E; ++j) g[j] = ok ? gidx[c * nz + h + H * j] : -1;
#pragma unroll
      for (int j = 0; j < E; ++j)
        v[j] = (g[j] >= 0 && bok) ? buf_load(rsph, sin_, static_cast<unsigned>(g[j] * nb + b) * es, 0)
                                  : cpx<T>{0, 0};
    } else {
      // running lane offsets: scalar offsets j*zstep would be hoisted as E
      // live scalar registers
      unsigned o = static_cast<unsigned>(h * npcol + slot) * nbp_es + ln.bl * es;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        v[j] = ok ? buf_load(rcol, colbuf, o, 0) : cpx<T>{0, 0};
        o += zstep_in;
        asm volatile("" : "+v"(o));
      }
    }
    bline_fft<E, H, S, T>(v, ctx);
    if (!ok) continue;
    if constexpr (S > 0) {
      unsigned o = static_cast<unsigned>(E * q * npcol + slot) * nbp_es + ln.bl * es;
#pragma unroll
      for (int k = 0; k < E; ++k) {
        buf_store(rcol, v[k], o, 0);
        o += zstep_out;
        asm volatile("" : "+v"(o));
      }
    } else {
      const T sc = static_cast<T>(a.scale);
      // the (column, z) lookups are all issued before the first store (the
      // compiler does not move loads across the buffer stores, so a lookup
      // per store would serialise their latencies)
      int g[E];
#pragma unroll
      for (int k = 0; k < E; ++k) g[k] = gidx[c * nz + k + E * q];
#pragma unroll
      for (int k = 0; k < E; ++k)
        if (g[k] >= 0 && bok)
          buf_store(rsph, cscale(v[k], sc), static_cast<unsigned>(g[k] * nb + b) * es, 0);
    }
  }
}

template <int S, typename T, int E, int H>
__global__ void __launch_bounds__(256) k1b_kernel(const KArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TwEntry<T>* tab = reinterpret_cast<TwEntry<T>*>(smem_raw);
  bl_fill_twiddles<S, T>(tab, reinterpret_cast<const cpx<T>*>(a.rootz),
                         reinterpret_cast<const cpx<T>*>(a.rootz_lo), E, H);
  __syncthreads();
  if (!a.persistent) {
    const int t = static_task_g(a.k1_tasks, 1);
    if (t >= 0) k1b_task<S, T, E, H>(a, t, tab);
    return;
  }
  __shared__ int sh_task;
  for (;;) {
    if (threadIdx.x == 0) sh_task = dynamic_task_g(a.counters, a.k1_tasks, 1);
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(sh_task);
    __syncthreads();
    if (t < 0) break;
    k1b_task<S, T, E, H>(a, t, tab);
  }
}

// Band-inner shapes (E values per position, H positions per line) compiled per
// precision, for z lines (column kernel) and x lines (plane kernel).
#define FFTB_BIL_Z_F32(X) X(8, 4) X(24, 4) X(32, 4) X(45, 4) X(64, 4)
#define FFTB_BIL_X_F32(X) X(8, 4) X(24, 4) X(32, 4) X(36, 4)
#define FFTB_BIL_Z_F64(X) X(4, 8) X(12, 8) X(16, 8) X(32, 8) X(45, 4)
#define FFTB_BIL_X_F64(X) X(4, 8) X(12, 8) X(16, 8) X(18, 8)
// narrow inverse x lines (complex64): half a 128-byte piece of bands (8) per
// row of lanes, twice the positions. (The complex128 form, 4 bands over 16
// positions, measured 1.5-1.9x slower than whole pieces and is not compiled.)
#define FFTB_BIL_XN_F32(X) X(4, 8) X(12, 8) X(16, 8) X(18, 8)

template <int S, typename T, int E, int H>
hipError_t bil_launch_k1(const KArgs& a, int grid, int threads, hipStream_t st) {
  const size_t lds = static_cast<size_t>(tw_row_stride(E)) * H * sizeof(TwEntry<T>);
  hipLaunchKernelGGL((k1b_kernel<S, T, E, H>), dim3(grid), dim3(threads), lds, st, a);
  return hipGetLastError();
}

// Plane kernel on band-inner x lines: inverse with the register fold of class
// length 8 or 16 (with or without the potential), forward with class partials.
// Class pairs (a.qc == 2) with the fold of length 16; complex64 folds of
// length 16 on the matrix cores (a.mfma).
template <int S, typename T, int E, int H>
hipError_t bil_plane(const KArgs& a, int grid, int threads, size_t lds, hipStream_t st, int fold_m,
                     bool attr_only) {
  if constexpr (S > 0) {
    constexpr int BW = band_width<T>();
    constexpr bool f32 = std::is_same<T, float>::value;
    if (attr_only) {
      hipError_t e = attr_k2<S, T, E, H, false, false, 8, true>(lds);
      if (e == hipSuccess) e = attr_k2<S, T, E, H, false, false, 16, true>(lds);
      if (e == hipSuccess) e = attr_k2<S, T, E, H, false, true, 8, true>(lds);
      if (e == hipSuccess) e = attr_k2<S, T, E, H, false, true, 16, true>(lds);
      if (e == hipSuccess) e = attr_k2<S, T, E, H, false, false, 16, true, BW, 2>(lds);
      if (e == hipSuccess) e = attr_k2<S, T, E, H, false, true, 16, true, BW, 2>(lds);
      if constexpr (f32) {
        if (e == hipSuccess) e = attr_k2<S, T, E, H, true, false, 16, true>(lds);
        if (e == hipSuccess) e = attr_k2<S, T, E, H, true, true, 16, true>(lds);
        if (e == hipSuccess) e = attr_k2<S, T, E, H, true, false, 16, true, BW, 2>(lds);
        if (e == hipSuccess) e = attr_k2<S, T, E, H, true, true, 16, true, BW, 2>(lds);
      }
      return e;
    }
    const bool pot = a.pot != nullptr;
    if constexpr (f32) {
      if (a.mfma) {
        if (fold_m != 16) return hipErrorInvalidValue;
        if (a.qc == 2)
          return pot ? launch_k2<S, T, E, H, true, true, 16, true, BW, 2>(a, grid, threads, lds, st)
                     : launch_k2<S, T, E, H, true, false, 16, true, BW, 2>(a, grid, threads, lds, st);
        return pot ? launch_k2<S, T, E, H, true, true, 16, true>(a, grid, threads, lds, st)
                   : launch_k2<S, T, E, H, true, false, 16, true>(a, grid, threads, lds, st);
      }
    }
    if (a.qc == 2) {
      if (fold_m != 16) return hipErrorInvalidValue;
      return pot ? launch_k2<S, T, E, H, false, true, 16, true, BW, 2>(a, grid, threads, lds, st)
                 : launch_k2<S, T, E, H, false, false, 16, true, BW, 2>(a, grid, threads, lds, st);
    }
    if (fold_m == 8)
      return pot ? launch_k2<S, T, E, H, false, true, 8, true>(a, grid, threads, lds, st)
                 : launch_k2<S, T, E, H, false, false, 8, true>(a, grid, threads, lds, st);
    if (fold_m == 16)
      return pot ? launch_k2<S, T, E, H, false, true, 16, true>(a, grid, threads, lds, st)
                 : launch_k2<S, T, E, H, false, false, 16, true>(a, grid, threads, lds, st);
    return hipErrorInvalidValue;
  } else {
    // forward: class partials, the y transform of length 8, 12 or 16 compiled
    // (0: any codelet length)
    if (attr_only) {
      hipError_t e = attr_k2<S, T, E, H, false, true, 0, true>(lds);
      if (e == hipSuccess) e = attr_k2<S, T, E, H, false, true, 8, true>(lds);
      if (e == hipSuccess) e = attr_k2<S, T, E, H, false, true, 12, true>(lds);
      if (e == hipSuccess) e = attr_k2<S, T, E, H, false, true, 16, true>(lds);
      return e;
    }
    if (fold_m == 8) return launch_k2<S, T, E, H, false, true, 8, true>(a, grid, threads, lds, st);
    if (fold_m == 12) return launch_k2<S, T, E, H, false, true, 12, true>(a, grid, threads, lds, st);
    if (fold_m == 16) return launch_k2<S, T, E, H, false, true, 16, true>(a, grid, threads, lds, st);
    return launch_k2<S, T, E, H, false, true, 0, true>(a, grid, threads, lds, st);
  }
}

// Narrow inverse plane kernel (complex64): fold of class length 16 or 32, with
// or without the potential.
template <typename T, int E, int H>
hipError_t bil_plane_narrow(const KArgs& a, int grid, int threads, size_t lds, hipStream_t st,
                            int fold_m, bool attr_only) {
  constexpr int BWN = band_width<T>() / 2;
  if (attr_only) {
    hipError_t e = attr_k2<+1, T, E, H, false, false, 16, true, BWN>(lds);
    if (e == hipSuccess) e = attr_k2<+1, T, E, H, false, true, 16, true, BWN>(lds);
    if (e == hipSuccess) e = attr_k2<+1, T, E, H, false, false, 32, true, BWN>(lds);
    if (e == hipSuccess) e = attr_k2<+1, T, E, H, false, true, 32, true, BWN>(lds);
    return e;
  }
  const bool pot = a.pot != nullptr;
  if (fold_m == 16)
    return pot ? launch_k2<+1, T, E, H, false, true, 16, true, BWN>(a, grid, threads, lds, st)
               : launch_k2<+1, T, E, H, false, false, 16, true, BWN>(a, grid, threads, lds, st);
  if (fold_m == 32)
    return pot ? launch_k2<+1, T, E, H, false, true, 32, true, BWN>(a, grid, threads, lds, st)
               : launch_k2<+1, T, E, H, false, false, 32, true, BWN>(a, grid, threads, lds, st);
  return hipErrorInvalidValue;
}

// which: 1 = column kernel (shape of z), 2 = plane kernel (shape of x),
// 3 = narrow inverse plane kernel (shape of x)
template <int S, typename T>
hipError_t bil_dispatch(int which, const KArgs& a, int E, int H, int grid, int threads, size_t lds,
                        hipStream_t st, int fold_m, bool attr_only) {
  constexpr bool f64 = std::is_same<T, double>::value;
  if (which == 3) {
    if constexpr (S > 0 && !f64) {
#define FFTB_X(e, h) \
  if (E == e && H == h) return bil_plane_narrow<T, e, h>(a, grid, threads, lds, st, fold_m, attr_only);
      FFTB_BIL_XN_F32(FFTB_X)
#undef FFTB_X
    }
    return attr_only ? hipSuccess : hipErrorInvalidValue;
  }
  if (which == 1) {
    if (attr_only) return hipSuccess;
#define FFTB_X(e, h) \
  if (E == e && H == h) return bil_launch_k1<S, T, e, h>(a, grid, threads, st);
    if constexpr (f64) {
      FFTB_BIL_Z_F64(FFTB_X)
    } else {
      FFTB_BIL_Z_F32(FFTB_X)
    }
#undef FFTB_X
    return hipErrorInvalidValue;
  }
#define FFTB_X(e, h) \
  if (E == e && H == h) return bil_plane<S, T, e, h>(a, grid, threads, lds, st, fold_m, attr_only);
  if constexpr (f64) {
    FFTB_BIL_X_F64(FFTB_X)
  } else {
    FFTB_BIL_X_F32(FFTB_X)
  }
#undef FFTB_X
  return hipErrorInvalidValue;
}

#define FFTB_BIL_DECL(EXT, S, T)                                                          \
  EXT template hipError_t bil_dispatch<S, T>(int, const KArgs&, int, int, int, int, size_t, \
                                             hipStream_t, int, bool);

}  // namespace fftb

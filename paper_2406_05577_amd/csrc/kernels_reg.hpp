// Register-path kernels for gfx950 (templates; the instantiations are split
// over the reg_*.hip translation units so that they compile in parallel). Each 1D transform line lives in the
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
// Plane kernel, forward, class-parallel (default): task = (plane z, band chunk,
// y class r). The rows y = r + n1*k2 are transformed along x keeping the
// occupied x only, then along y with length m; the result, multiplied by
// w_ny^{-j*r}, is stored as the class partial Z_r[xi][j]. The combine kernel
// then forms each column value y = j + m*t as the length-n1 DFT over the
// classes, sum_r w_n1^{-t*r} Z_r[xi][j] (a decimation-in-time split of the
// y transform), and the column kernel runs the z transforms.
// Plane kernel, forward, accumulating: task = (plane z, band chunk, column
// split); for each class r the split's columns accumulate the class's
// contribution w_ny^{-y*r} * Y[xi][y mod m] in LDS or in global memory.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "bline.hpp"
#include "device_common.hpp"

// Compile-time overrides of the memory-level parallelism (0 = the defaults
// below): blocks per round trip of the inverse fold, rows per round of the
// forward x transforms.
#ifndef FFTB_FOLD_BLOCKS
#define FFTB_FOLD_BLOCKS 0
#endif
#ifndef FFTB_FWD_ROWS
#define FFTB_FWD_ROWS 0
#endif

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

// floor(n / d) for 0 <= n < 2^22 through a float reciprocal and one correction
__device__ __forceinline__ int div_small(int n, int d, float inv_d) {
  int q = static_cast<int>(static_cast<float>(n) * inv_d);
  const int rem = n - q * d;
  q += (rem >= d) - (rem < 0);
  return q;
}

// ---------------------------------------------------------------------------
template <int S, typename T, int E, int H, bool MF>
__device__ void k1r_task(const KArgs& a, int t) {
  // lanes per line group: a line of 12 lanes takes a row of 16
  constexpr int HG = lane_group<H>();
  const int s = find_sphere_k1r(a, t);
  const SphereDesc d = a.sph[s];
  const int lt = t - d.k1_start;
  const int chunk = lt % d.nchunk, cb = lt / d.nchunk;
  const int c0 = cb * a.lc;
  const int nl = min(a.lc, d.ncol - c0);
  const int bcl = a.bcl, bmask = (1 << bcl) - 1;
  const int b0 = chunk << bcl;
  const int nz = a.nz, nb = d.nb, npcol = d.npcol;
  const int32_t* __restrict__ cslot = a.col_slot + d.colmeta_off;
  const int32_t* __restrict__ gidx = a.gidx + d.gidx_off;
  // column scratch: one padded band vector (nbp values) per (z, column slot)
  const int nbp = d.nbp;
  cpx<T>* __restrict__ colbuf = reinterpret_cast<cpx<T>*>(a.col) + d.col_off + b0;
  const cpx<T>* rootz = reinterpret_cast<const cpx<T>*>(a.rootz);
  const cpx<T>* rootz_lo = reinterpret_cast<const cpx<T>*>(a.rootz_lo);
  const int items = (nl << bcl) * HG;
  // with the matrix-core codelet whole waves take part: pad to 64 lanes
  const int iters = MF ? ((items + 63) & ~63) : items;
  // the block size is a multiple of HG: a thread keeps its lane position h;
  // lanes past H in a 16-lane row of a 12-lane line only join the exchanges
  const int h = threadIdx.x % HG;
  const bool lane_on = h < H;
  const auto ctx = line_ctx<E, H, S, T>(h, rootz, rootz_lo);
  // NP lines per thread per round (two for short lines): the table lookups and
  // loads of all of them are issued before any is used
  constexpr int NP = (E <= 10 && !MF) ? 2 : 1;
  const int q = out_block<H>(lane_on ? h : 0);
  // with a.k1buf the sphere and the column region are addressed as buffers
  // (both below 4 GiB): one offset register per line, uniform z strides
  constexpr unsigned es = sizeof(cpx<T>);
  const unsigned nbp_es = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(nbp) * es);
  const unsigned zstep_out = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(npcol) * nbp_es);
  const unsigned zstep_in = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(H * npcol) * nbp_es);
  const __amdgpu_buffer_rsrc_t rcol = buf_rsrc(colbuf);
  const __amdgpu_buffer_rsrc_t rsph =
      buf_rsrc(reinterpret_cast<const cpx<T>*>(S > 0 ? a.in : a.out) + d.sph_off);
  for (int it0 = threadIdx.x; it0 < iters; it0 += NP * blockDim.x) {
    bool ok[NP];
    int cc[NP], slot[NP], bls[NP];
    cpx<T> v[NP][E];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const int it = it0 + p * blockDim.x;
      // with the matrix-core codelet padded lanes still run the transform
      ok[p] = (MF ? it < items : it < iters) && lane_on;
      const int iv = (MF ? it < items : it < iters) ? it : h;
      const int rest = iv / HG;
      bls[p] = rest & bmask;
      cc[p] = c0 + (rest >> bcl);
      slot[p] = cslot[cc[p]];
    }
    if constexpr (S > 0) {
      const cpx<T>* __restrict__ in = reinterpret_cast<const cpx<T>*>(a.in) + d.sph_off;
      int g[NP][E];
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int j = 0; j < E; ++j) g[p][j] = ok[p] ? gidx[cc[p] * nz + h + H * j] : -1;
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const int b = b0 + bls[p];
        if (a.k1buf) {
#pragma unroll
          for (int j = 0; j < E; ++j)
            v[p][j] = (ok[p] && g[p][j] >= 0 && b < nb)
                          ? buf_load(rsph, in, static_cast<unsigned>(g[p][j] * nb + b) * es, 0)
                          : cpx<T>{0, 0};
        } else {
#pragma unroll
          for (int j = 0; j < E; ++j)
            v[p][j] = (ok[p] && g[p][j] >= 0 && b < nb) ? in[static_cast<int64_t>(g[p][j]) * nb + b]
                                                         : cpx<T>{0, 0};
        }
      }
    } else {
      if (a.k1buf) {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          const unsigned off = static_cast<unsigned>(h * npcol + slot[p]) * nbp_es + bls[p] * es;
#pragma unroll
          for (int j = 0; j < E; ++j)
            v[p][j] = ok[p] ? buf_load(rcol, colbuf, off, j * zstep_in) : cpx<T>{0, 0};
        }
      } else {
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
          for (int j = 0; j < E; ++j)
            v[p][j] = ok[p] ? colbuf[(static_cast<int64_t>(h + H * j) * npcol + slot[p]) * nbp + bls[p]]
                            : cpx<T>{0, 0};
      }
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      line_fft<E, H, S, T, MF>(v[p], ctx);
      if (!ok[p]) continue;
      if constexpr (S > 0) {
        if (a.k1buf) {
          const unsigned off =
              static_cast<unsigned>(E * q * npcol + slot[p]) * nbp_es + bls[p] * es;
#pragma unroll
          for (int k = 0; k < E; ++k) buf_store(rcol, v[p][k], off, k * zstep_out);
        } else {
#pragma unroll
          for (int k = 0; k < E; ++k)
            colbuf[(static_cast<int64_t>(k + E * q) * npcol + slot[p]) * nbp + bls[p]] = v[p][k];
        }
      } else {
        cpx<T>* __restrict__ out = reinterpret_cast<cpx<T>*>(a.out) + d.sph_off;
        const T sc = static_cast<T>(a.scale);
        const int b = b0 + bls[p];
        if (a.k1buf) {
#pragma unroll
          for (int k = 0; k < E; ++k) {
            const int g = gidx[cc[p] * nz + k + E * q];
            if (g >= 0 && b < nb)
              buf_store(rsph, cscale(v[p][k], sc), static_cast<unsigned>(g * nb + b) * es, 0);
          }
        } else {
#pragma unroll
          for (int k = 0; k < E; ++k) {
            const int g = gidx[cc[p] * nz + k + E * q];
            if (g >= 0 && b < nb) out[static_cast<int64_t>(g) * nb + b] = cscale(v[p][k], sc);
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// x transforms of the class rows y = r + n1*k2 (k2 < m) on band-inner lines:
// one line (one row, all bands of the chunk) per wavefront, or two for
// positions of half a wavefront. The band chunk is one 128-byte piece, so
// every grid access of a row of lanes is a whole piece.
//
// Inverse: the row's occupied x values come from the class slab S[xi][k2][bl]
// in LDS (zero at the other x), the line is transformed, and the whole row is
// written to plane z of the grid (times the potential with POT).
// EARLY_POT: the potential's loads are issued before the transform (their
// latency hides behind it); otherwise after it, with fewer live registers.
template <typename T, int E, int H, bool POT, int BW, bool EARLY_POT = true>
__device__ __forceinline__ void bl_inv_x(const KArgs& a, const SphereDesc& d, const cpx<T>* S,
                                         const TwEntry<T>* tab, const int* xo, int z, int r,
                                         int b0) {
  using Lane = BLane<T, H, BW>;
  const Lane ln;
  // opaque lane position: the line context is formed per task instead of being
  // hoisted out of the persistent loop, where it would stay live across the fold
  int h = ln.h;
  asm volatile("" : "+v"(h));
  const int q = bitrev_bits(h, log2_const<H>());
  const auto ctx = bline_ctx<E, H, +1, T, BW>(h, tab);
  const int nx = a.nx, ny = a.ny, nb = d.nb, n1 = a.n1, m = a.m, bcl = a.bcl2;
  cpx<T>* __restrict__ gout = reinterpret_cast<cpx<T>*>(a.out) + d.grid_off;
  const __amdgpu_buffer_rsrc_t gplane = buf_rsrc(gout + static_cast<int64_t>(z) * ny * nx * nb);
  const unsigned xstride =
      __builtin_amdgcn_readfirstlane(static_cast<unsigned>(nb) * sizeof(cpx<T>));
  const int wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  const int b = b0 + ln.bl;
  for (int base = wave * Lane::LPW; base < m; base += nwave * Lane::LPW) {
    const int k2 = base + ln.sub;
    const bool valid = k2 < m;
    const int y = r + n1 * (valid ? k2 : 0);
    T vp[E];
    const T* __restrict__ vrow =
        POT ? reinterpret_cast<const T*>(a.pot) + static_cast<int64_t>(z * ny + y) * nx : nullptr;
    if constexpr (POT && EARLY_POT) {
#pragma unroll
      for (int k = 0; k < E; ++k) vp[k] = vrow[k + E * q];
    }
    // the row's values: x = h + H*j from its slab line (the spare zero line
    // for x without a slab), in groups of eight so that the offsets read from
    // the table do not all stay live
    const cpx<T>* row = S + (k2 << bcl) + ln.bl;
    cpx<T> v[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
      v[j] = row[xo[h + H * j]];
      if ((j & 7) == 7) __builtin_amdgcn_sched_barrier(0);
    }
    bline_fft<E, H, +1, T>(v, ctx);
    if constexpr (POT) {
      if constexpr (!EARLY_POT) {
#pragma unroll
        for (int k = 0; k < E; ++k) vp[k] = vrow[k + E * q];
      }
#pragma unroll
      for (int k = 0; k < E; ++k) v[k] = cscale(v[k], vp[k]);
    }
    if (valid && b < nb) {
      // (band-inner plans keep every grid plane below 2 GiB: 32-bit offsets)
      // Non-temporal stores: the grid is not read again by this kernel, and
      // streaming it past the L2 keeps the plane's columns there for the
      // other classes' folds (measured 5 % (complex64) to 11 % (complex128)
      // faster). A running lane offset: per-store scalar offsets k*xstride would be
      // hoisted out of the row loop as E live scalar registers
      unsigned o =
          static_cast<unsigned>((y * nx + E * q) * nb + b) * static_cast<unsigned>(sizeof(cpx<T>));
#pragma unroll
      for (int k = 0; k < E; ++k) {
        buf_store_nt(gplane, v[k], o);
        o += xstride;
        asm volatile("" : "+v"(o));
      }
    }
  }
}

// Forward: the row is read from plane z of the grid, transformed, and its
// occupied x values are kept in the class slab S[xi][k2][bl] (the others land
// in the spare line).
template <typename T, int E, int H, int BW>
__device__ __forceinline__ void bl_fwd_x(const KArgs& a, const SphereDesc& d, cpx<T>* S,
                                         const TwEntry<T>* tab, const int* xo, int z, int r,
                                         int b0) {
  using Lane = BLane<T, H, BW>;
  const Lane ln;
  int h = ln.h;
  asm volatile("" : "+v"(h));
  const int q = bitrev_bits(h, log2_const<H>());
  const auto ctx = bline_ctx<E, H, -1, T, BW>(h, tab);
  const int nx = a.nx, ny = a.ny, nb = d.nb, n1 = a.n1, m = a.m, bcl = a.bcl2;
  const cpx<T>* __restrict__ gin = reinterpret_cast<const cpx<T>*>(a.in) + d.grid_off;
  const __amdgpu_buffer_rsrc_t gplane = buf_rsrc(gin + static_cast<int64_t>(z) * ny * nx * nb);
  const unsigned hstride =
      __builtin_amdgcn_readfirstlane(static_cast<unsigned>(H * nb) * sizeof(cpx<T>));
  const int wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  const int b = b0 + ln.bl;
  for (int base = wave * Lane::LPW; base < m; base += nwave * Lane::LPW) {
    const int k2 = base + ln.sub;
    const bool valid = k2 < m;
    const int y = r + n1 * (valid ? k2 : 0);
    const bool ld = valid && b < nb;
    cpx<T> v[E];
    unsigned o = static_cast<unsigned>((y * nx + h) * nb + b) * static_cast<unsigned>(sizeof(cpx<T>));
#pragma unroll
    for (int j = 0; j < E; ++j) {
      v[j] = ld ? buf_load(gplane, gin, o, 0) : cpx<T>{0, 0};
      o += hstride;
      asm volatile("" : "+v"(o));
    }
    bline_fft<E, H, -1, T>(v, ctx);
    if (valid) {
      cpx<T>* row = S + (k2 << bcl) + ln.bl;
#pragma unroll
      for (int k = 0; k < E; ++k) {
        row[xo[k + E * q]] = v[k];
        if ((k & 7) == 7) __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
}

// Stage the slab-line offsets of the x positions of sphere d in LDS:
// xo[x] = xi*sx for the slab xi of x, the spare line for x without a slab.
__device__ __forceinline__ void bl_stage_xoff(const KArgs& a, const SphereDesc& d, int* xo) {
  const int32_t* __restrict__ xinv = a.xinv + d.xinv_off;
  for (int x = threadIdx.x; x < a.nx; x += blockDim.x) {
    const int xi = xinv[x];
    xo[x] = xi >= 0 ? xi * a.sx : a.zline;
  }
}

// ---------------------------------------------------------------------------
// M > 0: the class length m = M is a compile-time constant and the column
// slots are laid out in zero-padded blocks of M consecutive y per slab; one
// thread folds and transforms a whole (slab, band) line in registers.
// M == 0: generic fold.
// QC == 2 (band-inner, M > 0): the task makes classes r and r2 = r + n1/2 from
// the same column reads, since w_n1^{tb*r2} = (-1)^tb * w_n1^{tb*r}: every
// loaded block is accumulated twice, with the sign of odd blocks flipped for
// r2. The transformed lines of r2 wait in registers (NLR lines per thread;
// the lines past NLR*blockDim in the plan's overflow scratch, one region per
// task) while the rows of class r are x-transformed, then fill the slab for
// the rows of r2. Half the tasks read the plane's columns.
template <typename T, int E, int H, bool MF, int M, bool POT, bool BL, int BWK, int QC>
__device__ void k2r_inv_task(const KArgs& a, int t, cpx<T>* S, const TwEntry<T>* tab, int* xo) {
  constexpr int L = log2_const<H>();
  constexpr bool PAIR = QC == 2;
  static_assert(QC == 1 || (QC == 2 && BL && M > 0), "class pairs: band-inner register fold only");
  const int s = find_sphere_k2r(a, t);
  const SphereDesc d = a.sph[s];
  const int lt = t - d.k2_start;
  const int n1 = a.n1, m = a.m;
  const int ncls = PAIR ? (n1 >> 1) : n1;  // tasks per (plane, chunk)
  const int r = lt % ncls;
  const int r2 = r + (n1 >> 1);            // the second class (QC == 2)
  const int rest0 = lt / ncls;
  // band-inner plane tasks may take a narrower band chunk than the column kernel
  const int nchunk = BL ? d.nchunk2 : d.nchunk;
  const int chunk = rest0 % nchunk, z = rest0 / nchunk;
  const int bcl = BL ? a.bcl2 : a.bcl, bmask = (1 << bcl) - 1;
  const int b0 = chunk << bcl;
  const int nx = a.nx, ny = a.ny, sx = a.sx;
  const int nb = d.nb, npcol = d.npcol, nslab = d.nslab;
  const int32_t* __restrict__ xinv = a.xinv + d.xinv_off;
  const int nbp = d.nbp;
  const cpx<T>* __restrict__ colp = reinterpret_cast<const cpx<T>*>(a.col) + d.col_off +
                                    static_cast<int64_t>(z) * npcol * nbp + b0;
  const cpx<T>* twf = reinterpret_cast<const cpx<T>*>(a.twf);
  const cpx<T>* twfl = reinterpret_cast<const cpx<T>*>(a.twf_lo);
  const cpx<T>* rootx = reinterpret_cast<const cpx<T>*>(a.rootx);
  const cpx<T>* rootx_lo = reinterpret_cast<const cpx<T>*>(a.rootx_lo);

  if constexpr (M > 0) {
    // per (slab, band) line, heaviest slabs first: for each block tb of M
    // consecutive y (y = k + M*tb) holding a column of the slab, u[k] +=
    // col(y) * w_n1^{+tb*r} (absent columns are zero slots); then u[k] *=
    // w_ny^{+k*r} and the length-M IFFT, written once to S. The slab's block
    // list (slot << 10 | tb) and the roots w_n1^{+tb*r} are staged in LDS.
    int32_t* tl = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(S) + a.lds_tab);
    int32_t* tn = tl + ((nslab * n1 + 3) & ~3);  // 16-byte aligned regions
    int32_t* tord = tn + ((nslab + 3) & ~3);     // the slab order
    cpx<T>* troot = reinterpret_cast<cpx<T>*>(tord + ((nslab + 3) & ~3));
    // the class twiddles w_ny^{k*r}, k < M (FP32: hi and lo of each), then
    // those of r2 (QC == 2)
    cpx<T>* ttw = troot + 2 * n1;
    cpx<T>* ttw2 = ttw + 2 * M;
    {
      const int32_t* __restrict__ blk = a.slab_blk + d.sl_off * n1;
      const int32_t* __restrict__ nblk = a.slab_nblk + d.sl_off;
      const int32_t* __restrict__ ord = a.slab_order + d.sl_off;
      for (int i = threadIdx.x; i < nslab * n1; i += blockDim.x) tl[i] = blk[i];
      for (int i = threadIdx.x; i < nslab; i += blockDim.x) {
        tn[i] = nblk[i];
        tord[i] = ord[i];
      }
      for (int tb = threadIdx.x; tb < n1; tb += blockDim.x) {
        const int idx = M * ((tb * r) % n1);  // w_n1^{tb*r} = w_ny^{M*((tb*r) mod n1)}
        cpx<T> w = twf[idx];
        w.im = -w.im;
        troot[2 * tb] = w;
        if constexpr (std::is_same<T, float>::value) {
          cpx<T> wl = twfl[idx];
          wl.im = -wl.im;
          troot[2 * tb + 1] = wl;
        }
      }
      for (int k = threadIdx.x; k < M; k += blockDim.x) {
        if constexpr (std::is_same<T, double>::value) {
          ttw[k] = twf[k * r];
          if constexpr (PAIR) ttw2[k] = twf[k * r2];
        } else {
          ttw[2 * k] = twf[k * r];
          ttw[2 * k + 1] = twfl[k * r];
          if constexpr (PAIR) {
            ttw2[2 * k] = twf[k * r2];
            ttw2[2 * k + 1] = twfl[k * r2];
          }
        }
      }
      if constexpr (BL) bl_stage_xoff(a, d, xo);
    }
    __syncthreads();
    // NBF blocks per round trip (their loads are all issued before the first
    // is accumulated; two measured best: four cost registers and time; one
    // for blocks of 32, for complex128 class pairs, for complex64 band-inner
    // folds of two bands per lane and for the matrix-core fold, whose
    // accumulators fill the registers)
    constexpr int NBF = FFTB_FOLD_BLOCKS > 0 ? FFTB_FOLD_BLOCKS
                        : (PAIR && std::is_same<T, float>::value && !MF) ? 2
                        : ((M > 16 || PAIR || (BL && std::is_same<T, float>::value)) ? 1 : 2);
    static_assert(NBF >= 1, "fold blocks per round trip");
    // the plane's column scratch as a buffer (the host keeps it below 2 GiB):
    // a block's M loads share one offset register
    const __amdgpu_buffer_rsrc_t rs = buf_rsrc(colp);
    const unsigned slot_bytes =
        __builtin_amdgcn_readfirstlane(static_cast<unsigned>(nbp) * sizeof(cpx<T>));
    // FB bands per lane: complex64 band-inner folds of blocks up to 16 take two
    // adjacent bands per lane (one 16-byte load each), halving the load
    // instructions
    constexpr int FB = (BL && std::is_same<T, float>::value && M <= 16 && !PAIR) ? 2 : 1;
    constexpr int FBL = FB == 2 ? 1 : 0;
    const int nlines = nslab << (bcl - FBL);
    // MF (band-inner, complex64, M == 16): the length-16 IFFT of the lines on
    // the matrix cores, which every lane of a wave takes part in: the line
    // loops run to whole waves, and lanes past the last line fold nothing
    constexpr bool MFB = MF && BL && M == 16 && std::is_same<T, float>::value;
    const int nlines_w = MFB ? ((nlines + 63) & ~63) : nlines;
    // fold line `it` into u (class r) and, for class pairs, u2 (class r2)
    auto fold_line = [&](int it, cpx<T> (&u)[FB][M], cpx<T> (&u2)[M]) {
      const bool live = it < nlines;
      const int bl = (it & (bmask >> FBL)) << FBL;
      const int xi = live ? tord[it >> (bcl - FBL)] : 0;
      const int nh = live ? tn[xi] : 0;
      const int32_t* lst = tl + xi * n1;
#pragma unroll
      for (int f = 0; f < FB; ++f)
#pragma unroll
        for (int k = 0; k < M; ++k) u[f][k] = cpx<T>{0, 0};
      if constexpr (PAIR) {
#pragma unroll
        for (int k = 0; k < M; ++k) u2[k] = cpx<T>{0, 0};
      }
      auto accumulate = [&](const cpx<T> (*v)[M], int tb, bool use) {
        cpx<T> w = troot[2 * tb];
        if (!use) w = cpx<T>{0, 0};
        // r2's root: the sign of odd blocks flipped
        const T sg = (tb & 1) ? static_cast<T>(-1) : static_cast<T>(1);
        if constexpr (std::is_same<T, float>::value) {
          cpx<T> wl = troot[2 * tb + 1];
          if (!use) wl = cpx<T>{0, 0};
          if constexpr (PAIR) {
            // one compensated product serves both classes (r2's root is +-r's)
#pragma unroll
            for (int k = 0; k < M; ++k) {
              const cpx<T> p = cmul_hl(v[0][k], w, wl);
              u[0][k] = cadd(u[0][k], p);
              u2[k] = {ffma(sg, p.re, u2[k].re), ffma(sg, p.im, u2[k].im)};
            }
          } else {
#pragma unroll
            for (int f = 0; f < FB; ++f)
#pragma unroll
              for (int k = 0; k < M; ++k) u[f][k] = cmac_hl(u[f][k], v[f][k], w, wl);
          }
        } else {
#pragma unroll
          for (int k = 0; k < M; ++k) u[0][k] = cmac(u[0][k], v[0][k], w);
          if constexpr (PAIR) {
            const cpx<T> w2{sg * w.re, sg * w.im};
#pragma unroll
            for (int k = 0; k < M; ++k) u2[k] = cmac(u2[k], v[0][k], w2);
          }
        }
      };
      auto off_of = [&](int e) {
        return static_cast<unsigned>((e >> 10) * nbp + bl) * static_cast<unsigned>(sizeof(cpx<T>));
      };
      for (int i = 0; i < nh; i += NBF) {
        // past the list's end the last block is loaded again (cache hits) and
        // accumulated with weight zero
        int eb[NBF];
        cpx<T> vb[NBF][FB][M];
#pragma unroll
        for (int b = 0; b < NBF; ++b) {
          eb[b] = lst[min(i + b, nh - 1)];
          const unsigned o = off_of(eb[b]);
#pragma unroll
          for (int k = 0; k < M; ++k) {
            if constexpr (FB == 2)
              buf_load2(rs, o, k * slot_bytes, vb[b][0][k], vb[b][1][k]);
            else
              vb[b][0][k] = buf_load(rs, colp, o, k * slot_bytes);
          }
        }
#pragma unroll
        for (int b = 0; b < NBF; ++b) accumulate(vb[b], eb[b] & 1023, i + b < nh);
      }
    };
    // class twiddles w_ny^{k*r} (tw = ttw) or w_ny^{k*r2} (tw = ttw2), then the
    // length-M IFFT
    auto finish = [&](cpx<T> (&u)[M], const cpx<T>* tw) {
      if constexpr (std::is_same<T, double>::value) {
#pragma unroll
        for (int k = 1; k < M; ++k) u[k] = twmul<+1>(u[k], tw, tw, k);
      } else {
#pragma unroll
        for (int k = 1; k < M; ++k) u[k] = twmul<+1>(u[k], tw, tw + 1, 2 * k);
      }
      if constexpr (MFB)
        dft16_mfma<+1>(u);
      else
        dft<M, +1>(u);
    };
    // write the M outputs of line `it` (FB adjacent bands) to the class slab
    auto store_line = [&](int it, const cpx<T> (&u)[FB][M]) {
      const int bl = (it & (bmask >> FBL)) << FBL;
      const int xi = tord[it >> (bcl - FBL)];
      cpx<T>* line = S + xi * sx + bl;
#pragma unroll
      for (int k = 0; k < M; ++k) {
        if constexpr (FB == 2) {
          typedef float v4f __attribute__((ext_vector_type(4)));
          *reinterpret_cast<v4f*>(line + (k << bcl)) = v4f{u[0][k].re, u[0][k].im, u[1][k].re, u[1][k].im};
        } else {
          line[k << bcl] = u[0][k];
        }
      }
    };
    if constexpr (!PAIR) {
      for (int it = threadIdx.x; it < nlines_w; it += blockDim.x) {
        cpx<T> u[FB][M], u2[M];  // (u2: class pairs only)
        fold_line(it, u, u2);
#pragma unroll
        for (int f = 0; f < FB; ++f) finish(u[f], ttw);
        if (it < nlines) store_line(it, u);
      }
      __syncthreads();
    } else {
      // lines past the register lines first (their r2 outputs go to the
      // overflow scratch), then the register lines, so that waiting r2 lines
      // stay live across as few folds as possible
      constexpr int NLR = kPairRegLines<T>;
      const int nreg = NLR * static_cast<int>(blockDim.x);
      const int ovl = a.ovf_lines;
      cpx<T>* __restrict__ ovf =
          reinterpret_cast<cpx<T>*>(a.col) + a.ovf_off + static_cast<int64_t>(t) * M * ovl;
      for (int it = nreg + threadIdx.x; it < nlines_w; it += blockDim.x) {
        cpx<T> u[1][M], u2[M];
        fold_line(it, u, u2);
        finish(u[0], ttw);
        finish(u2, ttw2);
        if (it < nlines) {
          store_line(it, u);
          const int j = it - nreg;
#pragma unroll
          for (int k = 0; k < M; ++k) ovf[k * ovl + j] = u2[k];
        }
      }
      cpx<T> hB[NLR][M];
#pragma unroll
      for (int li = 0; li < NLR; ++li) {
        const int it = threadIdx.x + li * static_cast<int>(blockDim.x);
        if (it < nlines_w) {
          cpx<T> u[1][M];
          fold_line(it, u, hB[li]);
          finish(u[0], ttw);
          finish(hB[li], ttw2);
          if (it < nlines) store_line(it, u);
        }
      }
      __syncthreads();
      // rows of class r, then the waiting lines of r2 into the slab and its
      // rows (one copy of the x phase: two would keep each other's constants)
#pragma unroll 1
      for (int c = 0; c < 2; ++c) {
        bl_inv_x<T, E, H, POT, BWK, false>(a, d, S, tab, xo, z, c == 0 ? r : r2, b0);
        if (c == 1) break;
        __syncthreads();
#pragma unroll
        for (int li = 0; li < NLR; ++li) {
          const int it = threadIdx.x + li * static_cast<int>(blockDim.x);
          if (it < nlines) {
            cpx<T> u[1][M];
#pragma unroll
            for (int k = 0; k < M; ++k) u[0][k] = hB[li][k];
            store_line(it, u);
          }
        }
        for (int it = nreg + threadIdx.x; it < nlines; it += blockDim.x) {
          const int j = it - nreg;
          cpx<T> u[1][M];
#pragma unroll
          for (int k = 0; k < M; ++k) u[0][k] = ovf[k * ovl + j];
          store_line(it, u);
        }
        __syncthreads();
      }
      return;
    }
  } else {
    const int32_t* __restrict__ cidx = a.colidx + d.colidx_off;

    // fold, one output per thread:
    //   F_r[xi][j] = w_ny^{+j*r} * sum_t col(xi, y = j + m*t) * w_n1^{+t*r}
    // (the first stage of a decimation-in-frequency split of the y transform,
    // evaluated for the single output class r; absent columns are zero)
    const int mr = m * r;  // w_n1^{t*r} = w_ny^{m*t*r}
    const float inv_m = 1.0f / static_cast<float>(m);
    const int nfold = (nslab * m) << bcl;
    for (int it = threadIdx.x; it < nfold; it += blockDim.x) {
      const int bl = it & bmask;
      const int jx = it >> bcl;
      const int xi = div_small(jx, m, inv_m);
      const int j = jx - xi * m;
      const int32_t* __restrict__ crow = cidx + xi * ny + j;
      cpx<T> acc{0, 0};
      int idx = 0;
  #pragma unroll 4
      for (int tt = 0; tt < n1; ++tt) {
        const int ci = crow[tt * m];
        if (ci >= 0) acc = cadd(acc, twmul<+1>(colp[static_cast<int64_t>(ci) * nbp + bl], twf, twfl, idx));
        idx += mr;
        if (idx >= ny) idx -= ny;
      }
      S[xi * sx + (j << bcl) + bl] = twmul<+1>(acc, twf, twfl, j * r);
    }
    __syncthreads();
    // y-IFFT of length m per (slab, band) line, in place
    const int nlines = nslab << bcl;
    for (int it = threadIdx.x; it < nlines; it += blockDim.x) {
      const int bl = it & bmask, xi = it >> bcl;
      cpx<T>* line = S + xi * sx + bl;
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
  }
  if constexpr (BL) {
    bl_inv_x<T, E, H, POT, BWK>(a, d, S, tab, xo, z, r, b0);
    return;
  }
  // x-IFFT of the class's rows, written to the grid. Lane h of a line keeps
  // the same h for every row, so its slab lookups are loaded once.
  cpx<T>* __restrict__ gout = reinterpret_cast<cpx<T>*>(a.out) + d.grid_off;
  // the lane position is made opaque here so that the line context below is
  // formed per task instead of being hoisted out of the persistent loop, where
  // it would stay live across the fold
  int h = threadIdx.x % H;
  asm volatile("" : "+v"(h));
  const int q = bitrev_bits(h, L);
  const auto ctx = line_ctx<E, H, +1, T>(h, rootx, rootx_lo);
  int xs[E];
#pragma unroll
  for (int j = 0; j < E; ++j) xs[j] = xinv[h + H * j];
  const int nrest = m << bcl;
  const int per_wave = 64 / H;
  const int nrest_p = MF ? (nrest + per_wave - 1) / per_wave * per_wave : nrest;
  const int rstep = blockDim.x / H;
  // plane z of the grid (below 2 GiB when a.plane32 is set)
  const __amdgpu_buffer_rsrc_t gplane = buf_rsrc(gout + static_cast<int64_t>(z) * ny * nx * nb);
  const unsigned xstride =
      __builtin_amdgcn_readfirstlane(static_cast<unsigned>(nb) * sizeof(cpx<T>));
  for (int rest = threadIdx.x / H; rest < nrest_p; rest += rstep) {
    const bool valid = rest < nrest;
    const int rv = valid ? rest : 0;
    const int bl = rv & bmask, k2 = rv >> bcl;
    const int y = r + n1 * k2;
    const int b = b0 + bl;
    // fused real-space step: the potential at the x this lane writes, requested
    // before the transform so that its latency hides behind it
    T vp[E];
    if constexpr (POT) {
      const T* __restrict__ vrow =
          reinterpret_cast<const T*>(a.pot) + static_cast<int64_t>(z * ny + y) * nx;
#pragma unroll
      for (int k = 0; k < E; ++k) vp[k] = vrow[k + E * q];
    }
    cpx<T> v[E];
#pragma unroll
    for (int j = 0; j < E; ++j)
      v[j] = (valid && xs[j] >= 0) ? S[xs[j] * sx + (k2 << bcl) + bl] : cpx<T>{0, 0};
    line_fft<E, H, +1, T, MF>(v, ctx);
    if constexpr (POT) {
      // the grid receives V(x, y, z) * psi
#pragma unroll
      for (int k = 0; k < E; ++k) v[k] = cscale(v[k], vp[k]);
    }
    if (valid && b < nb) {
      if (a.plane32) {
        // the plane as a buffer: one offset register per line, the x stride
        // in a scalar register
        const unsigned off =
            static_cast<unsigned>((y * nx + E * q) * nb + b) * static_cast<unsigned>(sizeof(cpx<T>));
#pragma unroll
        for (int k = 0; k < E; ++k) buf_store(gplane, v[k], off, k * xstride);
      } else {
        cpx<T>* row = gout + static_cast<int64_t>(z * ny + y) * nx * nb + b;
#pragma unroll
        for (int k = 0; k < E; ++k) row[static_cast<int64_t>(k + E * q) * nb] = v[k];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Forward x transform of the class rows y = r + n1*k2 (k2 < m) of plane z for
// the bands b0 + bl, keeping the occupied x of slabs [x_lo, x_hi) as
// S[xi - x_lo][k2][bl]. Lane h of a line keeps the same h for every row, so
// its slab lookups are loaded once.
template <typename T, int E, int H, bool MF>
__device__ __forceinline__ void fwd_x_rows(const KArgs& a, const cpx<T>* __restrict__ gin,
                                           const int32_t* __restrict__ xinv, cpx<T>* S, int r,
                                           int z, int b0, int nb, int x_lo, int x_hi) {
  constexpr int L = log2_const<H>();
  const int bcl = a.bcl, bmask = (1 << bcl) - 1;
  const int nx = a.nx, ny = a.ny, n1 = a.n1, sx = a.sx;
  const cpx<T>* rootx = reinterpret_cast<const cpx<T>*>(a.rootx);
  const cpx<T>* rootx_lo = reinterpret_cast<const cpx<T>*>(a.rootx_lo);
  const int h = threadIdx.x % H;
  const int q = bitrev_bits(h, L);
  const auto ctx = line_ctx<E, H, -1, T>(h, rootx, rootx_lo);
  int xs[E];
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const int xi = xinv[k + E * q] - x_lo;
    xs[k] = (xi >= 0 && xi < x_hi - x_lo) ? xi : -1;
  }
  const int nrest = a.m << bcl;
  const int per_wave = 64 / H;
  const int nrest_p = MF ? (nrest + per_wave - 1) / per_wave * per_wave : nrest;
  const int rstep = blockDim.x / H;
  // plane z of the grid as a buffer (below 2 GiB when a.plane32 is set)
  const __amdgpu_buffer_rsrc_t gplane = buf_rsrc(gin + static_cast<int64_t>(z) * ny * nx * nb);
  const unsigned hstride =
      __builtin_amdgcn_readfirstlane(static_cast<unsigned>(H * nb) * sizeof(cpx<T>));
  // RB rows per thread per round, the loads of all of them issued before the
  // first is transformed (one measured best: batching two or four rows was
  // slower at every benchmark shape)
  constexpr int RB = FFTB_FWD_ROWS > 0 ? FFTB_FWD_ROWS : 1;
  for (int rest0 = threadIdx.x / H; rest0 < nrest_p; rest0 += RB * rstep) {
    cpx<T> v[RB][E];
    int k2s[RB], bls[RB];
    bool valid[RB];
#pragma unroll
    for (int u = 0; u < RB; ++u) {
      const int rest = rest0 + u * rstep;
      valid[u] = rest < nrest;
      const int rv = valid[u] ? rest : 0;
      bls[u] = rv & bmask;
      k2s[u] = rv >> bcl;
      const int y = r + n1 * k2s[u];
      const int b = b0 + bls[u];
      const bool ld = valid[u] && b < nb;
      if (a.plane32) {
        const unsigned off =
            static_cast<unsigned>((y * nx + h) * nb + b) * static_cast<unsigned>(sizeof(cpx<T>));
#pragma unroll
        for (int j = 0; j < E; ++j)
          v[u][j] = ld ? buf_load(gplane, gin, off, j * hstride) : cpx<T>{0, 0};
      } else {
        const cpx<T>* row = gin + static_cast<int64_t>(z * ny + y) * nx * nb + b;
#pragma unroll
        for (int j = 0; j < E; ++j)
          v[u][j] = ld ? row[static_cast<int64_t>(h + H * j) * nb] : cpx<T>{0, 0};
      }
    }
#pragma unroll
    for (int u = 0; u < RB; ++u) {
      // rows past the padded count are skipped by whole waves
      if (rest0 + u * rstep >= nrest_p) continue;
      line_fft<E, H, -1, T, MF>(v[u], ctx);
      if (!valid[u]) continue;
#pragma unroll
      for (int k = 0; k < E; ++k)
        if (xs[k] >= 0) S[xs[k] * sx + (k2s[u] << bcl) + bls[u]] = v[u][k];
    }
  }
}

// ---------------------------------------------------------------------------
// Class-parallel forward task (plane z, chunk, class r): x transform of the
// class rows, y transform of length m per (slab, band) line, then the class
// partial Z_r[xi][j] = w_ny^{-j*r} * Y[xi][j] stored as Z[z][xi][j][r][band].
// M > 0 (band-inner): the class length is a compile-time constant.
template <typename T, int E, int H, bool MF, bool BL, int BWK, int M>
__device__ void k2r_fwd_cls_task(const KArgs& a, int t, cpx<T>* S, const TwEntry<T>* tab, int* xo) {
  const int s = find_sphere_k2r(a, t);
  const SphereDesc d = a.sph[s];
  const int lt = t - d.k2_start;
  const int n1 = a.n1, m = a.m;
  const int r = lt % n1;
  const int rest0 = lt / n1;
  const int nchunk = BL ? d.nchunk2 : d.nchunk;
  const int chunk = rest0 % nchunk, z = rest0 / nchunk;
  const int bcl = BL ? a.bcl2 : a.bcl, bmask = (1 << bcl) - 1;
  const int b0 = chunk << bcl;
  const int ny = a.ny, sx = a.sx;
  const int nb = d.nb, nslab = d.nslab;
  const int32_t* __restrict__ xinv = a.xinv + d.xinv_off;
  const cpx<T>* __restrict__ gin = reinterpret_cast<const cpx<T>*>(a.in) + d.grid_off;
  const cpx<T>* twf = reinterpret_cast<const cpx<T>*>(a.twf);
  const cpx<T>* twfl = reinterpret_cast<const cpx<T>*>(a.twf_lo);
  const int nbp = d.nbp;
  cpx<T>* __restrict__ zp = reinterpret_cast<cpx<T>*>(a.col) + d.zp_off +
                            (static_cast<int64_t>(z) * nslab * ny + r) * nbp + b0;

  if constexpr (BL) {
    // the slab-line offsets of the x positions and the class twiddles
    // w_ny^{-j*r}, j < m (FP32: hi and lo)
    bl_stage_xoff(a, d, xo);
    cpx<T>* ttw = reinterpret_cast<cpx<T>*>(reinterpret_cast<char*>(S) + a.lds_tab);
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
      if constexpr (std::is_same<T, double>::value) {
        ttw[j] = twf[j * r];
      } else {
        ttw[2 * j] = twf[j * r];
        ttw[2 * j + 1] = twfl[j * r];
      }
    }
    __syncthreads();
    bl_fwd_x<T, E, H, BWK>(a, d, S, tab, xo, z, r, b0);
    __syncthreads();
    // y transform of length m per (slab, band) line; the class partials are
    // written with streaming stores (the combine kernel reads them much later)
    const __amdgpu_buffer_rsrc_t rz = buf_rsrc(zp);
    const unsigned jstride = __builtin_amdgcn_readfirstlane(
        static_cast<unsigned>(n1 * nbp) * static_cast<unsigned>(sizeof(cpx<T>)));
    const int nlines = nslab << bcl;
    constexpr int MU = M > 0 ? M : kMaxRadixDev;
    for (int it = threadIdx.x; it < nlines; it += blockDim.x) {
      const int bl = it & bmask, xi = it >> bcl;
      const cpx<T>* line = S + xi * sx + bl;
      cpx<T> u[MU];
#pragma unroll
      for (int j = 0; j < MU; ++j)
        if (M > 0 || j < m) u[j] = line[j << bcl];
      if constexpr (M > 0)
        dft<M, -1>(u);
      else
        butterfly<-1>(m, u);
      unsigned o = static_cast<unsigned>(xi * ny * nbp + bl) * static_cast<unsigned>(sizeof(cpx<T>));
#pragma unroll
      for (int j = 0; j < MU; ++j) {
        if (M > 0 || j < m) {
          const cpx<T> val = std::is_same<T, double>::value ? twmul<-1>(u[j], ttw, ttw, j)
                                                           : twmul<-1>(u[j], ttw, ttw + 1, 2 * j);
          buf_store_nt(rz, val, o);
          o += jstride;
          asm volatile("" : "+v"(o));
        }
      }
    }
    return;
  }
  fwd_x_rows<T, E, H, MF>(a, gin, xinv, S, r, z, b0, nb, 0, nslab);
  __syncthreads();
  const int nlines = nslab << bcl;
  for (int it = threadIdx.x; it < nlines; it += blockDim.x) {
    const int bl = it & bmask, xi = it >> bcl;
    const cpx<T>* line = S + xi * sx + bl;
    cpx<T> u[kMaxRadixDev];
#pragma unroll
    for (int j = 0; j < kMaxRadixDev; ++j)
      if (j < m) u[j] = line[j << bcl];
    butterfly<-1>(m, u);
    cpx<T>* __restrict__ zl = zp + static_cast<int64_t>(xi) * ny * nbp + bl;
#pragma unroll
    for (int j = 0; j < kMaxRadixDev; ++j)
      if (j < m) zl[j * n1 * nbp] = twmul<-1>(u[j], twf, twfl, j * r);
  }
}

// ---------------------------------------------------------------------------
template <typename T, int E, int H, bool MF>
__device__ void k2r_fwd_task(const KArgs& a, int t, cpx<T>* S) {
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
  const int ny = a.ny, n1 = a.n1, m = a.m, sx = a.sx;
  const int nb = d.nb, npcol = d.npcol;
  const int32_t* __restrict__ xinv = a.xinv + d.xinv_off;
  const int32_t* __restrict__ cy = a.col_y + d.colmeta_off;
  const int32_t* __restrict__ cxi = a.col_xi + d.colmeta_off;
  const int32_t* __restrict__ cslot = a.col_slot + d.colmeta_off;
  const int32_t* __restrict__ sst = a.slabstart + d.slab_off;
  const int nbp = d.nbp;
  cpx<T>* __restrict__ colp = reinterpret_cast<cpx<T>*>(a.col) + d.col_off +
                              static_cast<int64_t>(z) * npcol * nbp + b0;
  const cpx<T>* __restrict__ gin = reinterpret_cast<const cpx<T>*>(a.in) + d.grid_off;
  const cpx<T>* twf = reinterpret_cast<const cpx<T>*>(a.twf);
  const cpx<T>* twfl = reinterpret_cast<const cpx<T>*>(a.twf_lo);
  cpx<T>* acc = S + a.lds_acc;
  const bool acc_lds = a.acc_lds != 0;
  const int c_lo = sst[x_lo];

  for (int r = 0; r < n1; ++r) {
    fwd_x_rows<T, E, H, MF>(a, gin, xinv, S, r, z, b0, nb, x_lo, x_hi);
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
      cpx<T>* g = colp + static_cast<int64_t>(cslot[c]) * nbp + bl;
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
// Forward class combine (task = plane z, band chunk): column (xi, y = j + m*t)
// = sum_r w_n1^{-t*r} Z_r[xi][j], the last, length-n1 stage of the
// decimation-in-time split of the y transform. One (slab, j, band) item per
// thread: its n1 class partials in, the n1 outputs t out to the columns that
// exist.
__device__ __forceinline__ int find_sphere_k3r(const KArgs& a, int t) {
  int s = 0;
  while (s + 1 < a.nsph && t >= a.sph[s].k3_end) ++s;
  return s;
}
__device__ __forceinline__ bool codelet_radix(int R) {
  return R == 1 || R == 2 || R == 3 || R == 4 || R == 5 || R == 6 || R == 8 || R == 9 ||
         R == 10 || R == 12 || R == 15 || R == 16 || R == 18 || R == 20;
}
// class counts of the combine: the codelets up to 20
constexpr int kMaxCombine = 20;
template <int S, typename T>
__device__ __forceinline__ void combine_dft(int R, cpx<T>* v) {
  if (R == 18) dft<18, S>(v);
  else if (R == 20) dft<20, S>(v);
  else butterfly<S>(R, v);
}

template <typename T>
__device__ void k3r_task(const KArgs& a, int t) {
  const int s = find_sphere_k3r(a, t);
  const SphereDesc d = a.sph[s];
  const int lt = t - d.k3_start;
  const int chunk = lt % d.nchunk, z = lt / d.nchunk;
  const int bcl = a.bcl, bmask = (1 << bcl) - 1;
  const int b0 = chunk << bcl;
  const int ny = a.ny, n1 = a.n1, m = a.m;
  const int nslab = d.nslab, npcol = d.npcol;
  const int nbp = d.nbp;
  const cpx<T>* __restrict__ zp = reinterpret_cast<const cpx<T>*>(a.col) + d.zp_off +
                                  static_cast<int64_t>(z) * nslab * ny * nbp + b0;
  cpx<T>* __restrict__ colp = reinterpret_cast<cpx<T>*>(a.col) + d.col_off +
                              static_cast<int64_t>(z) * npcol * nbp + b0;
  const int32_t* __restrict__ cidx = a.colidx + d.colidx_off;
  const cpx<T>* twf = reinterpret_cast<const cpx<T>*>(a.twf);
  const cpx<T>* twfl = reinterpret_cast<const cpx<T>*>(a.twf_lo);
  const float inv_m = 1.0f / static_cast<float>(m);
  const int items = (nslab * m) << bcl;
  if (codelet_radix(n1)) {
    // NP items per thread per round (two in FP32); the partials and the column
    // slots of all of them are requested before any of them is used
    constexpr int NP = sizeof(T) == 4 ? 2 : 1;
    // with a.plane32 the plane's partials and columns are addressed as buffers
    constexpr unsigned es = sizeof(cpx<T>);
    const unsigned nbp_es = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(nbp) * es);
    const __amdgpu_buffer_rsrc_t rz = buf_rsrc(zp);
    const __amdgpu_buffer_rsrc_t rc = buf_rsrc(colp);
    for (int it0 = threadIdx.x; it0 < items; it0 += NP * blockDim.x) {
      cpx<T> u[NP][kMaxCombine];
      int cs[NP][kMaxCombine];
      bool ok[NP];
      int bls[NP];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const int it = it0 + p * blockDim.x;
        ok[p] = it < items;
        const int iv = ok[p] ? it : it0;
        const int bl = iv & bmask;
        const int jx = iv >> bcl;
        const int xi = div_small(jx, m, inv_m);
        const int j = jx - xi * m;
        bls[p] = bl;
        const int32_t* __restrict__ crow = cidx + xi * ny + j;
        if (a.plane32) {
          const unsigned off = static_cast<unsigned>((xi * ny + j * n1) * nbp + bl) * es;
#pragma unroll
          for (int r = 0; r < kMaxCombine; ++r) {
            if (r < n1) {
              u[p][r] = buf_load(rz, zp, off, r * nbp_es);
              cs[p][r] = crow[r * m];
            }
          }
        } else {
          const cpx<T>* __restrict__ src = zp + (static_cast<int64_t>(xi) * ny + j * n1) * nbp + bl;
#pragma unroll
          for (int r = 0; r < kMaxCombine; ++r) {
            if (r < n1) {
              u[p][r] = src[r * nbp];
              cs[p][r] = crow[r * m];
            }
          }
        }
      }
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        if (!ok[p]) continue;
        combine_dft<-1>(n1, u[p]);
        if (a.plane32) {
#pragma unroll
          for (int q = 0; q < kMaxCombine; ++q)
            if (q < n1 && cs[p][q] >= 0)
              buf_store(rc, u[p][q], static_cast<unsigned>(cs[p][q] * nbp + bls[p]) * es, 0);
        } else {
#pragma unroll
          for (int q = 0; q < kMaxCombine; ++q)
            if (q < n1 && cs[p][q] >= 0) colp[static_cast<int64_t>(cs[p][q]) * nbp + bls[p]] = u[p][q];
        }
      }
    }
    return;
  }
  // class counts without a codelet: direct sums
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    const int bl = it & bmask;
    const int jx = it >> bcl;
    const int xi = div_small(jx, m, inv_m);
    const int j = jx - xi * m;
    const cpx<T>* __restrict__ src = zp + (static_cast<int64_t>(xi) * ny + j * n1) * nbp + bl;
    const int32_t* __restrict__ crow = cidx + xi * ny + j;
    for (int q = 0; q < n1; ++q) {
      const int c = crow[q * m];
      if (c < 0) continue;
      cpx<T> acc = src[0];
      const int step = m * q;  // w_n1^{q} = w_ny^{m*q}
      int idx = 0;
      for (int r = 1; r < n1; ++r) {
        idx += step;
        if (idx >= ny) idx -= ny;
        acc = cadd(acc, twmul<-1>(src[r * nbp], twf, twfl, idx));
      }
      colp[static_cast<int64_t>(c) * nbp + bl] = acc;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k3r_kernel(const KArgs a) {
  if (!a.persistent) {
    const int t = static_task_g(a.k3_tasks, 1);
    if (t >= 0) k3r_task<T>(a, t);
    return;
  }
  __shared__ int sh_task;
  for (;;) {
    if (threadIdx.x == 0) sh_task = dynamic_task_g(a.counters + 16, a.k3_tasks, 1);
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(sh_task);
    __syncthreads();
    if (t < 0) break;
    k3r_task<T>(a, t);
  }
}

// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
template <int S, typename T, int E, int H, bool MF>
__global__ void __launch_bounds__(256) k1r_kernel(const KArgs a) {
  if (!a.persistent) {
    const int t = static_task_g(a.k1_tasks, 1);
    if (t >= 0) k1r_task<S, T, E, H, MF>(a, t);
    return;
  }
  __shared__ int sh_task;
  for (;;) {
    if (threadIdx.x == 0) sh_task = dynamic_task_g(a.counters, a.k1_tasks, 1);
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(sh_task);
    __syncthreads();
    if (t < 0) break;
    k1r_task<S, T, E, H, MF>(a, t);
  }
}

// FC: forward tasks write class partials (compiled apart from the accumulating
// forward so that neither variant's register allocation limits the other);
// inverse tasks multiply by the real-space potential (compiled apart so that
// the plain transform carries no potential registers)
// BWK: bands per row of lanes of the band-inner x lines (one 128-byte piece,
// or half of one for the narrow inverse tiling)
// QC: y classes per inverse task (2: class pairs sharing the fold's reads)
template <int S, typename T, int E, int H, bool MF, bool FC, int M, bool BL,
          int BWK = band_width<T>(), int QC = 1>
__global__ void __launch_bounds__(512) k2r_kernel(const KArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  // band-inner lines: the x twiddles w_nx^{h*k} staged in LDS once per block,
  // followed by the per-task table of slab-line offsets of the x positions
  TwEntry<T>* tab = reinterpret_cast<TwEntry<T>*>(smem_raw + a.lds_twx);
  int* xo = reinterpret_cast<int*>(smem_raw + a.lds_twx + (H > 1 ? tw_row_stride(E) * H : 0) * sizeof(TwEntry<T>));
  if constexpr (BL) {
    if constexpr (H > 1)
      bl_fill_twiddles<S, T>(tab, reinterpret_cast<const cpx<T>*>(a.rootx),
                             reinterpret_cast<const cpx<T>*>(a.rootx_lo), E, H);
    // the spare slab line: zeros for the x positions without a slab (inverse;
    // no fold writes it), a sink for them (forward)
    if constexpr (S > 0)
      for (int i = threadIdx.x; i < a.sx; i += blockDim.x) lds[a.zline + i] = cpx<T>{0, 0};
    __syncthreads();
  }
  if (!a.persistent) {
    const int t = static_task_g(a.k2_tasks, a.g2);
    if (t >= 0) {
      if constexpr (S > 0) k2r_inv_task<T, E, H, MF, M, FC, BL, BWK, QC>(a, t, lds, tab, xo);
      else if constexpr (FC) k2r_fwd_cls_task<T, E, H, MF, BL, BWK, M>(a, t, lds, tab, xo);
      else k2r_fwd_task<T, E, H, MF>(a, t, lds);
    }
    return;
  }
  __shared__ int sh_task;
  for (;;) {
    if (threadIdx.x == 0) sh_task = dynamic_task_g(a.counters + 8, a.k2_tasks, a.g2);
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(sh_task);
    __syncthreads();
    if (t < 0) break;
    if constexpr (S > 0) k2r_inv_task<T, E, H, MF, M, FC, BL, BWK, QC>(a, t, lds, tab, xo);
    else if constexpr (FC) k2r_fwd_cls_task<T, E, H, MF, BL, BWK, M>(a, t, lds, tab, xo);
    else k2r_fwd_task<T, E, H, MF>(a, t, lds);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------

// Inverse plane kernels with a compile-time class length are compiled for the
// lines spread over 8 or 16 lanes (x lengths 32 .. 160) and m = 8 or 16.
constexpr bool fold_m_compiled(int H, int m) { return (H == 8 || H == 16) && (m == 8 || m == 16); }

template <int S, typename T, int E, int H, bool MF, bool FC, int M, bool BL = false,
          int BWK = band_width<T>(), int QC = 1>
hipError_t launch_k2(const KArgs& a, int grid, int threads, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL((k2r_kernel<S, T, E, H, MF, FC, M, BL, BWK, QC>), dim3(grid), dim3(threads), lds,
                     st, a);
  return hipGetLastError();
}

template <int S, typename T, int E, int H, bool MF, bool FC, int M, bool BL = false,
          int BWK = band_width<T>(), int QC = 1>
hipError_t attr_k2(size_t lds) {
  return hipFuncSetAttribute(
      reinterpret_cast<const void*>(k2r_kernel<S, T, E, H, MF, FC, M, BL, BWK, QC>),
      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <int S, typename T, int E, int H, bool MF>
hipError_t launch_one(int which, const KArgs& a, int grid, int threads, size_t lds,
                             hipStream_t st, int fold_m) {
  if (which == 1) {
    hipLaunchKernelGGL((k1r_kernel<S, T, E, H, MF>), dim3(grid), dim3(threads), 0, st, a);
    return hipGetLastError();
  }
  if constexpr (H == 12) {
    return hipErrorInvalidValue;  // 12-lane lines serve the column kernel only
  } else if constexpr (S < 0) {
    if (a.fwd_cls) return launch_k2<S, T, E, H, MF, true, 0>(a, grid, threads, lds, st);
  } else {
    const bool pot = a.pot != nullptr;
    if constexpr (fold_m_compiled(H, 8)) {
      if (fold_m == 8)
        return pot ? launch_k2<S, T, E, H, MF, true, 8>(a, grid, threads, lds, st)
                   : launch_k2<S, T, E, H, MF, false, 8>(a, grid, threads, lds, st);
      if (fold_m == 16)
        return pot ? launch_k2<S, T, E, H, MF, true, 16>(a, grid, threads, lds, st)
                   : launch_k2<S, T, E, H, MF, false, 16>(a, grid, threads, lds, st);
    }
    if (fold_m != 0) return hipErrorInvalidValue;
    if (pot) return launch_k2<S, T, E, H, MF, true, 0>(a, grid, threads, lds, st);
  }
  if constexpr (H != 12) {
    if (fold_m != 0) return hipErrorInvalidValue;
    return launch_k2<S, T, E, H, MF, false, 0>(a, grid, threads, lds, st);
  }
  return hipErrorInvalidValue;
}

template <int S, typename T, int E, int H, bool MF>
hipError_t attr_one(size_t lds) {
  if constexpr (H == 12) return hipSuccess;  // no plane kernel for 12-lane lines
  hipError_t e = attr_k2<S, T, E, H, MF, false, 0>(lds);
  if (e == hipSuccess) e = attr_k2<S, T, E, H, MF, true, 0>(lds);
  if constexpr (S > 0 && fold_m_compiled(H, 8)) {
    if (e == hipSuccess) e = attr_k2<S, T, E, H, MF, false, 8>(lds);
    if (e == hipSuccess) e = attr_k2<S, T, E, H, MF, false, 16>(lds);
    if (e == hipSuccess) e = attr_k2<S, T, E, H, MF, true, 8>(lds);
    if (e == hipSuccess) e = attr_k2<S, T, E, H, MF, true, 16>(lds);
  }
  return e;
}


// (E, H, part) triples compiled for each precision: E values per lane, H lanes
// per transform line; `part` picks the translation unit that instantiates the
// shape (the host picks one shape per axis).
#define FFTB_REG_SHAPES(X)                                                         \
  X(4, 1, 0) X(5, 1, 0) X(6, 1, 0) X(8, 1, 0) X(9, 1, 0) X(10, 1, 0) X(12, 1, 0) \
  X(15, 1, 0) X(16, 1, 0) X(5, 4, 0) X(6, 4, 0) X(45, 4, 0) X(15, 12, 0)         \
  X(4, 8, 1) X(12, 8, 1) X(16, 8, 1) X(18, 8, 1) X(20, 8, 1)                      \
  X(6, 16, 2) X(8, 16, 2) X(9, 16, 2) X(10, 16, 2) X(16, 16, 2)
constexpr int kRegParts = 3;

// Launch (or, with attr_only, set the LDS attribute of) the register-path
// kernels of one shape of part PART; *found reports whether the shape belongs
// to the part.
template <int S, typename T, int PART>
hipError_t reg_dispatch(int which, const KArgs& a, int E, int H, int grid, int threads, size_t lds,
                        hipStream_t st, int fold_m, bool attr_only, bool* found) {
  *found = false;
#define FFTB_X(e, h, p)                                                                   \
  if constexpr (p == PART) {                                                            \
    if (E == e && H == h) {                                                             \
      *found = true;                                                                    \
      return attr_only ? attr_one<S, T, e, h, false>(lds)                               \
                       : launch_one<S, T, e, h, false>(which, a, grid, threads, lds, st, \
                                                       fold_m);                         \
    }                                                                                   \
  }
  FFTB_REG_SHAPES(FFTB_X)
#undef FFTB_X
  return hipErrorInvalidValue;
}

// The FP32 DFT_16 on the matrix cores: lines of 16 values per lane over 8 lanes.
template <int S>
hipError_t reg_dispatch_mfma(int which, const KArgs& a, int grid, int threads, size_t lds,
                             hipStream_t st, int fold_m, bool attr_only) {
  return attr_only ? attr_one<S, float, 16, 8, true>(lds)
                   : launch_one<S, float, 16, 8, true>(which, a, grid, threads, lds, st, fold_m);
}

#define FFTB_REG_DECL(EXT, S, T, P)                                                         \
  EXT template hipError_t reg_dispatch<S, T, P>(int, const KArgs&, int, int, int, int, size_t, \
                                                hipStream_t, int, bool, bool*);
#define FFTB_REG_DECL_ALL(EXT)                                                          \
  FFTB_REG_DECL(EXT, +1, double, 0) FFTB_REG_DECL(EXT, +1, double, 1)                  \
  FFTB_REG_DECL(EXT, +1, double, 2) FFTB_REG_DECL(EXT, -1, double, 0)                  \
  FFTB_REG_DECL(EXT, -1, double, 1) FFTB_REG_DECL(EXT, -1, double, 2)                  \
  FFTB_REG_DECL(EXT, +1, float, 0) FFTB_REG_DECL(EXT, +1, float, 1)                    \
  FFTB_REG_DECL(EXT, +1, float, 2) FFTB_REG_DECL(EXT, -1, float, 0)                    \
  FFTB_REG_DECL(EXT, -1, float, 1) FFTB_REG_DECL(EXT, -1, float, 2)                    \
  EXT template hipError_t reg_dispatch_mfma<+1>(int, const KArgs&, int, int, size_t,     \
                                                hipStream_t, int, bool);               \
  EXT template hipError_t reg_dispatch_mfma<-1>(int, const KArgs&, int, int, size_t,     \
                                                hipStream_t, int, bool);

}  // namespace fftb

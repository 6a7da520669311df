// Band-inner transform lines for gfx950.
//
// The grid, the sphere and the column scratch all hold a band vector per point
// (band fastest). A band-inner line keeps that order in the lanes of a
// wavefront: lane = bl + BW*h (+ BW*H*i for the i-th line of a wave), with BW
// bands per row of lanes such that BW values are one 128-byte piece (16
// complex64 or 8 complex128 values). A line of length N = E*H lives in H
// positions h of E values each; every global load or store of a row of BW
// lanes is then one whole 128-byte piece, which measured 1.3x (stores) and
// 1.8x (loads) faster than pieces of 32 bytes on MI355X.
//
// The transform is the Cooley-Tukey split N = E*H (Section 2.1): DFT_E in
// registers, twiddles w_N^{h*k} read from a table in LDS (the E*H entries are
// the same for every line, and the lanes of a row read the same entry), then
// log2(H) radix-2 rounds across the positions, each lane fetching its partner's
// value through the LDS crossbar.
#pragma once

#include "device_common.hpp"

namespace fftb {

// bands per 128-byte piece
template <typename T>
constexpr int band_width() {
  return 128 / static_cast<int>(2 * sizeof(T));
}

// One twiddle of the LDS table: the FP64 value, or the FP32 hi and lo parts.
template <typename T>
struct TwEntry;
template <>
struct alignas(16) TwEntry<double> {
  double re, im;
};
template <>
struct alignas(16) TwEntry<float> {
  float re, im, lre, lim;
};

// Fill tab[h*R + k] = w_N^{S*h*k} (N = E*H, R = tw_row_stride(E)) from the
// forward-sign root table of length N (FP32: hi and lo tables).
// Block-cooperative; the caller synchronises before use.
template <int S, typename T>
__device__ void bl_fill_twiddles(TwEntry<T>* tab, const cpx<T>* __restrict__ root,
                                 const cpx<T>* __restrict__ root_lo, int E, int H) {
  for (int i = threadIdx.x; i < E * H; i += blockDim.x) {
    const int h = i / E, k = i - (i / E) * E;
    const cpx<T> w = root[h * k];
    const T sg = S > 0 ? static_cast<T>(-1) : static_cast<T>(1);
    TwEntry<T> e;
    e.re = w.re;
    e.im = sg * w.im;
    if constexpr (std::is_same<T, float>::value) {
      const cpx<T> l = root_lo[h * k];
      e.lre = l.re;
      e.lim = sg * l.im;
    }
    tab[h * tw_row_stride(E) + k] = e;
  }
}

// Ordering point between groups of a line's values: the values k0 .. k1-1 are
// complete here, and everything that reads them, or reads memory, comes after.
// (Scheduling barriers alone did not keep the groups apart: the compiler
// issued all table reads and all partner fetches of a line at once, holding a
// second copy of the line in registers.)
template <typename T>
__device__ __forceinline__ void bl_fence(cpx<T>* v, int k0, int k1) {
#pragma unroll
  for (int k = k0; k < k1; ++k) asm volatile("" : "+v"(v[k].re), "+v"(v[k].im)::"memory");
}

// Values per group of twiddle reads and partner fetches (two measured no
// better than four for the longest complex128 lines).
template <int E, typename T>
constexpr int bl_group() {
  return 4;
}
// The DPP round grouped too: only for long complex128 lines, where the
// partner copies of a whole line overflowed the registers (the 45 x 4 z lines
// of 180: 126-186 extra registers without it, 2.12 -> 2.02 ms per column
// kernel at 144x160x180; shorter lines measured better ungrouped)
template <int E, typename T>
constexpr bool bl_group_dpp() {
  return sizeof(T) == 8 && E >= 32;
}

template <int E, int H, int S, typename T, int BW = band_width<T>()>
struct BLineCtx {
  static constexpr int kBW = BW;  // bands per row of lanes
  static constexpr int kRounds = H > 1 ? log2_const<H>() : 1;
  const TwEntry<T>* tw;  // row h of the LDS table
  T sgn[kRounds];
  cpx<T> rw[kRounds];
};

// Context of the lane at position h of its line; tab is the LDS table.
template <int E, int H, int S, typename T, int BW = band_width<T>()>
__device__ __forceinline__ BLineCtx<E, H, S, T, BW> bline_ctx(int h, const TwEntry<T>* tab) {
  BLineCtx<E, H, S, T, BW> c;
  c.tw = tab + h * tw_row_stride(E);
  if constexpr (H > 1) {
    int i = 0;
#pragma unroll
    for (int hs = H / 2; hs >= 1; hs >>= 1, ++i) {
      const int b = (h / hs) & 1;
      const int hl = h % hs;
      c.sgn[i] = b ? static_cast<T>(-1) : static_cast<T>(1);
      c.rw[i] = (b && hl) ? root16<S, T>(hl * (8 / hs)) : cpx<T>{1, 0};
    }
  }
  return c;
}

// Radix-2 rounds across the positions: partner distance hs positions = BW*hs
// lanes. Each lane fetches its partner's value through the LDS crossbar
// (ds_bpermute: no LDS memory, no VALU moves; 8 lanes apart: a DPP row
// rotation), then the lower lane of a pair
// keeps own + partner, the upper one forms partner - own and multiplies it by
// the round twiddle.
template <int HS, int I, int E, int H, int S, typename T, int BW>
__device__ __forceinline__ void bl_rounds(cpx<T>* v, const BLineCtx<E, H, S, T, BW>& c) {
  if constexpr (HS >= 1) {
    constexpr int D = HS * BW;
    constexpr int G = bl_group<E, T>();
    const T sg = c.sgn[I];
    if constexpr (D <= 8) {
      // partners 4 or 8 lanes apart sit in the same row of 16: DPP moves
      // (VALU; the LDS crossbar is left to the wider rounds)
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const T pr = dpp_xor<D>(v[k].re), pi = dpp_xor<D>(v[k].im);
        v[k] = {ffma(sg, v[k].re, pr), ffma(sg, v[k].im, pi)};
        if constexpr (bl_group_dpp<E, T>())
          if (k % G == G - 1 && k + 1 < E) bl_fence(v, k - G + 1, k + 1 + G < E ? k + 1 + G : E);
      }
    } else {
      const int src = ((threadIdx.x & 63) ^ D) << 2;
      // in groups of G values, so that the fetched values do not all stay live
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const T pr = lane_read(src, v[k].re), pi = lane_read(src, v[k].im);
        v[k] = {ffma(sg, v[k].re, pr), ffma(sg, v[k].im, pi)};
        if (k % G == G - 1 && k + 1 < E) bl_fence(v, k - G + 1, k + 1 + G < E ? k + 1 + G : E);
      }
    }
    if constexpr (HS == 2) {
      // the round twiddle is 1 or w_4 = S*i: a swap of the components with
      // one sign, selected per lane
      const bool rot = c.rw[I].im != static_cast<T>(0);
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const T re = v[k].re, im = v[k].im;
        v[k] = {rot ? static_cast<T>(-S) * im : re, rot ? static_cast<T>(S) * re : im};
      }
    } else if constexpr (HS > 2) {
      const cpx<T> w = c.rw[I];
#pragma unroll
      for (int k = 0; k < E; ++k) v[k] = cmul(v[k], w);
    }
    bl_rounds<HS / 2, I + 1, E, H, S, T, BW>(v, c);
  }
}

// One band-inner line: on entry the lane at position h holds x[h + H*j] in
// v[j] (j < E); on exit it holds X[k + E*bitrev(h)] in v[k]. Every lane of the
// wavefront must take part (lanes of a line that has no data transform zeros).
template <int E, int H, int S, typename T, int BW>
__device__ __forceinline__ void bline_fft(cpx<T>* v, const BLineCtx<E, H, S, T, BW>& c) {
  dft<E, S>(v);
  if constexpr (H > 1) {
    // in groups of G: the scheduler would otherwise issue every table read at
    // once and keep all E-1 twiddles live beside the line
    constexpr int G = bl_group<E, T>();
#pragma unroll
    for (int k = 1; k < E; ++k) {
      const TwEntry<T> w = c.tw[k];
      if constexpr (std::is_same<T, float>::value)
        v[k] = cmul_hl(v[k], cpx<float>{w.re, w.im}, cpx<float>{w.lre, w.lim});
      else
        v[k] = cmul(v[k], cpx<double>{w.re, w.im});
      if (k % G == G - 1 && k + 1 < E) bl_fence(v, k - G + 1, k + 1);
    }
    bl_rounds<H / 2, 0, E, H, S, T, BW>(v, c);
  }
}

// Positions of a lane: band bl of the chunk, position h on its line, and the
// line i of the wave (when one line uses only part of the wavefront).
template <typename T, int H, int BWL = band_width<T>()>
struct BLane {
  static constexpr int BW = BWL;
  static constexpr int LPW = 64 / (BW * H);  // lines per wavefront
  int bl, h, sub;
  __device__ __forceinline__ BLane() {
    const int lane = threadIdx.x & 63;
    bl = lane & (BW - 1);
    h = (lane / BW) % H;
    sub = lane / (BW * H);
  }
};

}  // namespace fftb

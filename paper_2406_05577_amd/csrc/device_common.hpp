// Device building blocks shared by the HIP kernels: complex arithmetic,
// compile-time roots of unity, in-register DFT codelets (Cooley-Tukey
// factorisation of Section 2.1), twiddle multiplication with FP64 or
// compensated FP32 (hi+lo) tables, and cross-lane exchanges.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "kargs.hpp"

namespace fftb {

constexpr int kMaxRadixDev = 16;

// Task scheduling over the XCDs (the hardware places blocks on the 8 XCDs
// round-robin by block index). Tasks come in groups of G consecutive indices
// that read the same input through L2 (the y classes of one plane and band
// chunk); group g runs on XCD g mod 8 and every XCD walks its groups in order,
// so at any time the chip works on neighbouring groups: all band chunks of the
// same planes, whose pieces of each band vector then reach HBM together.
__device__ __forceinline__ int xcd_task(int q, int k, int G) {
  return (((k / G) << 3) + q) * G + k % G;
}
// one block per task: block b is the k = b/8 th block on XCD q = b mod 8
__device__ __forceinline__ int static_task_g(int total, int G) {
  const int t = xcd_task(blockIdx.x & 7, blockIdx.x >> 3, G);
  return t < total ? t : -1;
}
// persistent blocks: one counter per XCD; the task index grows with the
// counter, so the first index past the end ends that XCD's queue
__device__ __forceinline__ int dynamic_task_g(unsigned int* counters, int total, int G) {
  const int q = blockIdx.x & 7;
  const unsigned int idx = atomicAdd(&counters[q], 1u);
  if (idx >= static_cast<unsigned int>(total)) return -1;
  const int t = xcd_task(q, static_cast<int>(idx), G);
  return t < total ? t : -1;
}

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cpx<T> cscale(cpx<T> a, T s) { return {a.re * s, a.im * s}; }
__device__ __forceinline__ float ffma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double ffma(double a, double b, double c) { return __builtin_fma(a, b, c); }
// Raw buffer loads from a wave-uniform base: the lane supplies one 32-bit byte
// offset and each load adds a uniform byte offset held in a scalar register,
// so a strided run of loads needs a single address register instead of one
// 64-bit address per load. Reads past the 4 GiB range return zero.
// `base` must be the same in every lane of the wave (it is read from the first).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base) {
  const uint64_t pa = reinterpret_cast<uint64_t>(base);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(pa));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(pa >> 32));
  void* p = reinterpret_cast<void*>((static_cast<uint64_t>(hi) << 32) | lo);
  // gfx9 raw buffer: no stride, full 32-bit range, dword 3 = 0x00020000
  return __builtin_amdgcn_make_buffer_rsrc(p, static_cast<short>(0),
                                           static_cast<int>(0xffffffffu), 0x00020000);
}
__device__ __forceinline__ cpx<double> buf_load(__amdgpu_buffer_rsrc_t r, const cpx<double>*,
                                                unsigned voff, unsigned soff) {
  typedef int v4i __attribute__((ext_vector_type(4)));
  const v4i x = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
  return __builtin_bit_cast(cpx<double>, x);
}
__device__ __forceinline__ cpx<float> buf_load(__amdgpu_buffer_rsrc_t r, const cpx<float>*,
                                               unsigned voff, unsigned soff) {
  typedef int v2i __attribute__((ext_vector_type(2)));
  const v2i x = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
  return __builtin_bit_cast(cpx<float>, x);
}

// two adjacent complex64 values in one 16-byte load
__device__ __forceinline__ void buf_load2(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff,
                                          cpx<float>& a, cpx<float>& b) {
  typedef float v4f __attribute__((ext_vector_type(4)));
  const v4f x = __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  a = {x.x, x.y};
  b = {x.z, x.w};
}

__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, cpx<double> v, unsigned voff,
                                          unsigned soff) {
  typedef int v4i __attribute__((ext_vector_type(4)));
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4i, v), r, voff, soff, 0);
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, cpx<float> v, unsigned voff,
                                          unsigned soff) {
  typedef int v2i __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2i, v), r, voff, soff, 0);
}

// Non-temporal (streaming) stores: cache policy bit 1 (nt on gfx950).
__device__ __forceinline__ void buf_store_nt(__amdgpu_buffer_rsrc_t r, cpx<double> v, unsigned voff) {
  typedef int v4i __attribute__((ext_vector_type(4)));
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4i, v), r, voff, 0, 2);
}
__device__ __forceinline__ void buf_store_nt(__amdgpu_buffer_rsrc_t r, cpx<float> v, unsigned voff) {
  typedef int v2i __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2i, v), r, voff, 0, 2);
}

// u + v*w with fused multiply-adds
template <typename T>
__device__ __forceinline__ cpx<T> cmac(cpx<T> u, cpx<T> v, cpx<T> w) {
  T re = ffma(v.re, w.re, u.re);
  re = ffma(-v.im, w.im, re);
  T im = ffma(v.re, w.im, u.im);
  im = ffma(v.im, w.re, im);
  return {re, im};
}
// v*(hi + lo) for a compensated FP32 twiddle, the small products first
__device__ __forceinline__ cpx<float> cmul_hl(cpx<float> v, cpx<float> hi, cpx<float> lo) {
  float re = v.re * lo.re;
  re = ffma(-v.im, lo.im, re);
  re = ffma(v.re, hi.re, re);
  re = ffma(-v.im, hi.im, re);
  float im = v.re * lo.im;
  im = ffma(v.im, lo.re, im);
  im = ffma(v.re, hi.im, im);
  im = ffma(v.im, hi.re, im);
  return {re, im};
}
// u + v*(hi + lo)
__device__ __forceinline__ cpx<float> cmac_hl(cpx<float> u, cpx<float> v, cpx<float> hi,
                                              cpx<float> lo) {
  return cmac(cmac(u, v, lo), v, hi);
}
// multiply by S*i
template <int S, typename T>
__device__ __forceinline__ cpx<T> mul_si(cpx<T> a) {
  if constexpr (S > 0) return {-a.im, a.re};
  else return {a.im, -a.re};
}

// ---------------------------------------------------------------------------
// Compile-time roots of unity for the in-register codelets: cos and sin of
// 2*pi*j/R, reduced exactly in integers to the first octant, then a Taylor
// series (|x| <= pi/4, 14 terms).
constexpr double kHalfPi = 1.57079632679489661923132169163975144;

constexpr double taylor_sin(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}
// first-quadrant angle (pi/2) * r / R, 0 <= r < R
constexpr double q_sin(int r, int R) {
  return (2 * r <= R) ? taylor_sin(kHalfPi * r / R) : taylor_cos(kHalfPi * (R - r) / R);
}
constexpr double q_cos(int r, int R) {
  return (2 * r <= R) ? taylor_cos(kHalfPi * r / R) : taylor_sin(kHalfPi * (R - r) / R);
}
// cos(2*pi*j/R), sin(2*pi*j/R)
constexpr double kcos(int j, int R) {
  j = ((j % R) + R) % R;
  const int q = (4 * j) / R, r = 4 * j - q * R;
  const double c = q_cos(r, R), s = q_sin(r, R);
  return q == 0 ? c : q == 1 ? -s : q == 2 ? -c : s;
}
constexpr double ksin(int j, int R) {
  j = ((j % R) + R) % R;
  const int q = (4 * j) / R, r = 4 * j - q * R;
  const double c = q_cos(r, R), s = q_sin(r, R);
  return q == 0 ? s : q == 1 ? c : q == 2 ? -s : -c;
}

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// x * exp(S*2*pi*i*J/R), with exact quarter turns folded at compile time.
template <int J, int R, int S, typename T>
__device__ __forceinline__ cpx<T> rot(cpx<T> x) {
  constexpr int j = ((J % R) + R) % R;
  if constexpr (j == 0) {
    return x;
  } else if constexpr (4 * j == R) {
    return mul_si<S>(x);
  } else if constexpr (2 * j == R) {
    return {-x.re, -x.im};
  } else if constexpr (4 * j == 3 * R) {
    return mul_si<-S>(x);
  } else {
    constexpr T c = static_cast<T>(kcos(j, R));
    constexpr T s = static_cast<T>(S * ksin(j, R));
    return {x.re * c - x.im * s, x.re * s + x.im * c};
  }
}

// ---------------------------------------------------------------------------
// DFT codelets in registers, sign S (+1: exp(+...), -1: exp(-...)).
template <int R, int S, typename T>
__device__ __forceinline__ void dft(cpx<T>* v);

template <int S, typename T>
__device__ __forceinline__ void dft2(cpx<T>* v) {
  const cpx<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}
template <int S, typename T>
__device__ __forceinline__ void dft3(cpx<T>* v) {
  constexpr T h = static_cast<T>(0.866025403784438646763723170752936183);  // sin(2pi/3)
  const cpx<T> a = v[0], b = v[1], c = v[2];
  const cpx<T> t1 = cadd(b, c);
  const cpx<T> t2 = {a.re - static_cast<T>(0.5) * t1.re, a.im - static_cast<T>(0.5) * t1.im};
  const cpx<T> t3 = mul_si<S>(cscale(csub(b, c), h));
  v[0] = cadd(a, t1);
  v[1] = cadd(t2, t3);
  v[2] = csub(t2, t3);
}
template <int S, typename T>
__device__ __forceinline__ void dft4(cpx<T>* v) {
  const cpx<T> a = v[0], b = v[1], c = v[2], d = v[3];
  const cpx<T> s0 = cadd(a, c), s1 = csub(a, c), s2 = cadd(b, d);
  const cpx<T> s3 = mul_si<S>(csub(b, d));
  v[0] = cadd(s0, s2);
  v[2] = csub(s0, s2);
  v[1] = cadd(s1, s3);
  v[3] = csub(s1, s3);
}
template <int S, typename T>
__device__ __forceinline__ void dft5(cpx<T>* v) {
  constexpr T c1 = static_cast<T>(kcos(1, 5)), c2 = static_cast<T>(kcos(2, 5));
  constexpr T s1 = static_cast<T>(ksin(1, 5)), s2 = static_cast<T>(ksin(2, 5));
  const cpx<T> a0 = v[0];
  const cpx<T> t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
  const cpx<T> t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
  const cpx<T> r1 = {a0.re + c1 * t1.re + c2 * t2.re, a0.im + c1 * t1.im + c2 * t2.im};
  const cpx<T> r2 = {a0.re + c2 * t1.re + c1 * t2.re, a0.im + c2 * t1.im + c1 * t2.im};
  const cpx<T> i1 = mul_si<S>(cpx<T>{s1 * t3.re + s2 * t4.re, s1 * t3.im + s2 * t4.im});
  const cpx<T> i2 = mul_si<S>(cpx<T>{s2 * t3.re - s1 * t4.re, s2 * t3.im - s1 * t4.im});
  v[0] = cadd(a0, cadd(t1, t2));
  v[1] = cadd(r1, i1);
  v[4] = csub(r1, i1);
  v[2] = cadd(r2, i2);
  v[3] = csub(r2, i2);
}

// R = A*B: B sub-DFTs of length A over stride-B elements, twiddles, then A
// sub-DFTs of length B (Section 2.1, Cooley-Tukey factorisation).
template <int A, int B, int S, typename T>
__device__ __forceinline__ void dft_ab(cpx<T>* v) {
  constexpr int R = A * B;
  cpx<T> u[R];
  static_for<0, B>([&](auto bb) {
    constexpr int b = decltype(bb)::value;
    cpx<T> t[A];
#pragma unroll
    for (int a = 0; a < A; ++a) t[a] = v[b + B * a];
    dft<A, S>(t);
    static_for<0, A>([&](auto aa) {
      constexpr int ap = decltype(aa)::value;
      u[b * A + ap] = rot<b * ap, R, S>(t[ap]);
    });
  });
#pragma unroll
  for (int ap = 0; ap < A; ++ap) {
    cpx<T> t[B];
#pragma unroll
    for (int b = 0; b < B; ++b) t[b] = u[b * A + ap];
    dft<B, S>(t);
#pragma unroll
    for (int bp = 0; bp < B; ++bp) v[ap + A * bp] = t[bp];
  }
}

// R = A*B with A and B coprime: the prime-factor (Good-Thomas) split. The
// input index n = (B*n1 + A*n2) mod R and the output index k = (B*(B^-1 mod A)*k1
// + A*(A^-1 mod B)*k2) mod R turn the transform into A transforms of length B
// and B of length A with no twiddles between them (Section 2.1 factorisation,
// the index map of the Chinese remainder theorem).
constexpr int inv_mod(int a, int m) {
  for (int x = 1; x < m; ++x)
    if ((a * x) % m == 1) return x;
  return 1;
}
template <int A, int B, int S, typename T>
__device__ __forceinline__ void dft_pfa(cpx<T>* v) {
  constexpr int R = A * B;
  cpx<T> u[R];
  static_for<0, A>([&](auto i1) {
    constexpr int n1 = decltype(i1)::value;
    cpx<T> t[B];
    static_for<0, B>([&](auto i2) {
      constexpr int n2 = decltype(i2)::value;
      t[n2] = v[(B * n1 + A * n2) % R];
    });
    dft<B, S>(t);
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) u[n1 * B + k2] = t[k2];
  });
  // long codelets: keep the scheduler from interleaving the two stages (it
  // would hold both arrays live: 2R values)
  if constexpr (R >= 36) __builtin_amdgcn_sched_barrier(0);
  constexpr int cb = B * inv_mod(B % A, A), ca = A * inv_mod(A % B, B);
  static_for<0, B>([&](auto j2) {
    constexpr int k2 = decltype(j2)::value;
    cpx<T> t[A];
#pragma unroll
    for (int n1 = 0; n1 < A; ++n1) t[n1] = u[n1 * B + k2];
    dft<A, S>(t);
    static_for<0, A>([&](auto j1) {
      constexpr int k1 = decltype(j1)::value;
      v[(cb * k1 + ca * k2) % R] = t[k1];
    });
  });
}

template <int R, int S, typename T>
__device__ __forceinline__ void dft(cpx<T>* v) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2) {
    dft2<S>(v);
  } else if constexpr (R == 3) {
    dft3<S>(v);
  } else if constexpr (R == 4) {
    dft4<S>(v);
  } else if constexpr (R == 5) {
    dft5<S>(v);
  } else if constexpr (R == 6) {
    dft_pfa<2, 3, S>(v);
  } else if constexpr (R == 8) {
    dft_ab<4, 2, S>(v);
  } else if constexpr (R == 9) {
    dft_ab<3, 3, S>(v);
  } else if constexpr (R == 10) {
    dft_pfa<2, 5, S>(v);
  } else if constexpr (R == 12) {
    dft_pfa<4, 3, S>(v);
  } else if constexpr (R == 15) {
    dft_pfa<5, 3, S>(v);
  } else if constexpr (R == 16) {
    dft_ab<4, 4, S>(v);
  } else if constexpr (R == 18) {
    dft_pfa<2, 9, S>(v);
  } else if constexpr (R == 20) {
    dft_pfa<4, 5, S>(v);
  } else if constexpr (R == 24) {
    dft_pfa<8, 3, S>(v);
  } else if constexpr (R == 32) {
    dft_ab<8, 4, S>(v);
  } else if constexpr (R == 36) {
    dft_pfa<4, 9, S>(v);
  } else if constexpr (R == 40) {
    dft_pfa<8, 5, S>(v);
  } else if constexpr (R == 45) {
    dft_pfa<9, 5, S>(v);
  } else if constexpr (R == 48) {
    dft_pfa<16, 3, S>(v);
  } else if constexpr (R == 64) {
    dft_ab<8, 8, S>(v);
  } else if constexpr (R == 72) {
    dft_pfa<8, 9, S>(v);
  } else if constexpr (R == 96) {
    dft_pfa<32, 3, S>(v);
  } else if constexpr (R == 128) {
    dft_ab<16, 8, S>(v);
  } else if constexpr (R == 144) {
    dft_pfa<16, 9, S>(v);
  } else {
    static_assert(R == 1, "unsupported radix");
  }
}

template <int S, typename T>
__device__ __forceinline__ void butterfly(int R, cpx<T>* v) {
  switch (R) {
    case 2: dft<2, S>(v); break;
    case 3: dft<3, S>(v); break;
    case 4: dft<4, S>(v); break;
    case 5: dft<5, S>(v); break;
    case 6: dft<6, S>(v); break;
    case 8: dft<8, S>(v); break;
    case 9: dft<9, S>(v); break;
    case 10: dft<10, S>(v); break;
    case 12: dft<12, S>(v); break;
    case 15: dft<15, S>(v); break;
    case 16: dft<16, S>(v); break;
    default: break;
  }
}

// Twiddle multiply with a forward-sign table entry; S > 0 conjugates it.
// FP32 applies the compensated pair x*hi + x*lo.
template <int S, typename T>
__device__ __forceinline__ cpx<T> twmul(cpx<T> v, const cpx<T>* __restrict__ hi,
                                         const cpx<T>* __restrict__ lo, int idx) {
  cpx<T> w = hi[idx];
  if constexpr (S > 0) w.im = -w.im;
  if constexpr (std::is_same<T, float>::value) {
    cpx<T> l = lo[idx];
    if constexpr (S > 0) l.im = -l.im;
    return cmul_hl(v, w, l);
  } else {
    (void)lo;
    return cmul(v, w);
  }
}

// ---------------------------------------------------------------------------
__device__ __forceinline__ int bitrev_bits(int h, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) r |= ((h >> i) & 1) << (bits - 1 - i);
  return r;
}

template <int H>
constexpr int log2_const() {
  int l = 0;
  while ((1 << l) < H) ++l;
  return l;
}

// Lanes a transform line of H lanes occupies: a line of 12 lanes takes a row
// of 16 (the unit of the cross-lane moves), whose last 4 lanes idle.
template <int H>
constexpr int lane_group() {
  return H == 12 ? 16 : H;
}

// After line_fft, lane h holds the E outputs X[k + E*out_block(h)], k < E.
template <int H>
__device__ __forceinline__ int out_block(int h) {
  if constexpr (H == 12) {
    // radix-3 output c = h / 4, then the 4-point output bitrev2(h mod 4)
    return (h >> 2) + 3 * (((h & 1) << 1) | ((h >> 1) & 1));
  } else {
    return bitrev_bits(h, log2_const<H>());
  }
}

// exp(S*2*pi*i*j/12), j < 12 (the radix-3 step of 12-lane lines).
template <int S, typename T>
__device__ __forceinline__ cpx<T> root12(int j) {
  const T c[12] = {static_cast<T>(kcos(0, 12)), static_cast<T>(kcos(1, 12)),
                   static_cast<T>(kcos(2, 12)), static_cast<T>(kcos(3, 12)),
                   static_cast<T>(kcos(4, 12)), static_cast<T>(kcos(5, 12)),
                   static_cast<T>(kcos(6, 12)), static_cast<T>(kcos(7, 12)),
                   static_cast<T>(kcos(8, 12)), static_cast<T>(kcos(9, 12)),
                   static_cast<T>(kcos(10, 12)), static_cast<T>(kcos(11, 12))};
  const T sn[12] = {static_cast<T>(ksin(0, 12)), static_cast<T>(ksin(1, 12)),
                    static_cast<T>(ksin(2, 12)), static_cast<T>(ksin(3, 12)),
                    static_cast<T>(ksin(4, 12)), static_cast<T>(ksin(5, 12)),
                    static_cast<T>(ksin(6, 12)), static_cast<T>(ksin(7, 12)),
                    static_cast<T>(ksin(8, 12)), static_cast<T>(ksin(9, 12)),
                    static_cast<T>(ksin(10, 12)), static_cast<T>(ksin(11, 12))};
  const int jj = ((j % 12) + 12) % 12;
  return {c[jj], static_cast<T>(S) * sn[jj]};
}

// exp(S*2*pi*i*j/16), j < 16 (the roots needed by the cross-lane radix-2
// rounds for groups of up to 16 lanes).
template <int S, typename T>
__device__ __forceinline__ cpx<T> root16(int j) {
  constexpr T r = static_cast<T>(kcos(2, 16)), c1 = static_cast<T>(kcos(1, 16)),
              s1 = static_cast<T>(ksin(1, 16));
  const T c[16] = {1, c1, r, s1, 0, -s1, -r, -c1, -1, -c1, -r, -s1, 0, s1, r, c1};
  const T sn[16] = {0, s1, r, c1, 1, c1, r, s1, 0, -s1, -r, -c1, -1, -c1, -r, -s1};
  return {c[j & 15], static_cast<T>(S) * sn[j & 15]};
}

// ---------------------------------------------------------------------------
// DFT_16 of 64 lines at once (one per lane of the wavefront) as a dense FP32
// matrix product on the matrix cores: with v = (Re, Im) interleaved, the 16x16
// complex DFT is the real 32x32 matrix M with M[2k][2s] = M[2k+1][2s+1] =
// cos(2 pi k s/16), M[2k][2s+1] = -S sin(2 pi k s/16), M[2k+1][2s] = S sin(...).
// v_mfma_f32_32x32x2f32 multiplies 32 rows of M by 2 input components of 32
// lines per instruction, so each half of the wave's lines takes 16 steps. The
// operand halves are paired with v_permlane32_swap before the products and the
// result halves are paired back afterwards. Every lane of the wave must take
// part (callers pad their loops to whole waves).
typedef float mfma_f16v __attribute__((ext_vector_type(16)));

__constant__ float c_cos16[16] = {
    (float)kcos(0, 16), (float)kcos(1, 16), (float)kcos(2, 16), (float)kcos(3, 16),
    (float)kcos(4, 16), (float)kcos(5, 16), (float)kcos(6, 16), (float)kcos(7, 16),
    (float)kcos(8, 16), (float)kcos(9, 16), (float)kcos(10, 16), (float)kcos(11, 16),
    (float)kcos(12, 16), (float)kcos(13, 16), (float)kcos(14, 16), (float)kcos(15, 16)};
__constant__ float c_sin16[16] = {
    (float)ksin(0, 16), (float)ksin(1, 16), (float)ksin(2, 16), (float)ksin(3, 16),
    (float)ksin(4, 16), (float)ksin(5, 16), (float)ksin(6, 16), (float)ksin(7, 16),
    (float)ksin(8, 16), (float)ksin(9, 16), (float)ksin(10, 16), (float)ksin(11, 16),
    (float)ksin(12, 16), (float)ksin(13, 16), (float)ksin(14, 16), (float)ksin(15, 16)};

__device__ __forceinline__ void pair_halves(float& x, float& y) {
  // x <- (x lanes 0-31, y lanes 0-31), y <- (x lanes 32-63, y lanes 32-63)
  const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  x = __uint_as_float(p[0]);
  y = __uint_as_float(p[1]);
}

template <int S>
__device__ __forceinline__ void dft16_mfma(cpx<float>* v) {
  const int lane = threadIdx.x & 63;
  const int row = lane & 31;      // output component of M supplied by this lane
  const int kk = lane >> 5;       // which of the two input components of a step
  const int ko = row >> 1;        // output frequency
  const bool im = row & 1;
  mfma_f16v acc0 = {0}, acc1 = {0};
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    float b0 = v[s].re, b1 = v[s].im;
    pair_halves(b0, b1);  // b0: operand for lines 0-31, b1: for lines 32-63
    const int j = (ko * s) & 15;
    const float c = c_cos16[j], sn = static_cast<float>(S) * c_sin16[j];
    const float a = im ? (kk ? c : sn) : (kk ? -sn : c);
    acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b0, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b1, acc1, 0, 0, 0);
  }
  // acc[r] holds row 8*(r/4) + 4*(lane/32) + r%4 of column lane%32; pair the halves so
  // that acc0 holds rows 8*(r/4) + r%4 and acc1 rows 8*(r/4) + 4 + r%4 of the lane's line
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    float x = acc0[r], y = acc1[r];
    pair_halves(x, y);
    const int o0 = 8 * (r >> 2) + (r & 3), o1 = o0 + 4;
    if (o0 & 1) v[o0 >> 1].im = x; else v[o0 >> 1].re = x;
    if (o1 & 1) v[o1 >> 1].im = y; else v[o1 >> 1].re = y;
  }
}

// Cross-lane partner value (lane ^ M, M = 1, 2, 4 or 8) inside rows of 16
// lanes through DPP moves: quad permutations for 1 and 2, a half-row mirror
// followed by a quad reversal for 4 ((i ^ 7) ^ 3 = i ^ 4), a row rotation by 8
// for 8. Every lane of a transform line is active whenever the line is.
template <int M>
__device__ __forceinline__ int dpp_xor_i(int v) {
  if constexpr (M == 1) {
    return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);   // quad_perm [1,0,3,2]
  } else if constexpr (M == 2) {
    return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);   // quad_perm [2,3,0,1]
  } else if constexpr (M == 4) {
    const int m = __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true);  // row_half_mirror
    return __builtin_amdgcn_mov_dpp(m, 0x1B, 0xF, 0xF, true);          // quad_perm [3,2,1,0]
  } else {
    static_assert(M == 8, "partner distance 1, 2, 4 or 8");
    return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, true);  // row_ror:8
  }
}
template <int M>
__device__ __forceinline__ float dpp_xor(float x) {
  return __int_as_float(dpp_xor_i<M>(__float_as_int(x)));
}
template <int M>
__device__ __forceinline__ double dpp_xor(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = dpp_xor_i<M>(static_cast<int>(b & 0xffffffffll));
  const int hi = dpp_xor_i<M>(static_cast<int>(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              (static_cast<long long>(lo) & 0xffffffffll));
}

// Per-lane constants of a transform line of length N = E*H over H lanes (lane
// h of its group): the twiddles w_N^{h*k} (k < E; kept in registers when E is
// small, else read per line from the root table) and, per cross-lane round of
// partner distance hs, the sign of the lane's own value (+1 keeps v + p, -1
// forms p - v) and the round twiddle w_{2hs}^{h mod hs} (1 for the lanes that
// keep the sum).
template <int E, int H, int S, typename T>
struct LineCtx {
  static constexpr bool kHoist = E <= 10 || H == 12;
  // radix-2 rounds across the lanes (for 12 lanes: those of the 4-lane part)
  static constexpr int kRounds = H == 12 ? 2 : (H > 1 ? log2_const<H>() : 1);
  int h;
  const cpx<T>* rootN;
  const cpx<T>* rootN_lo;
  cpx<T> tw[kHoist ? E : 1];
  cpx<T> twl[kHoist && std::is_same<T, float>::value ? E : 1];
  T sgn[kRounds];
  cpx<T> rw[kRounds];
  // 12 lanes: the radix-3 step across the three 4-lane groups (byte
  // addresses of the two partner lanes and the weights of the lane's own value
  // and of the partners' values, the step's twiddle folded in)
  int src1, src2;
  cpx<T> a3[H == 12 ? 3 : 1];
};

template <int E, int H, int S, typename T>
__device__ __forceinline__ LineCtx<E, H, S, T> line_ctx(int h, const cpx<T>* __restrict__ rootN,
                                                        const cpx<T>* __restrict__ rootN_lo) {
  LineCtx<E, H, S, T> c;
  if constexpr (H == 12) {
    // idle lanes (12..15 of the row) compute with the position of lane 0
    if (h >= 12) h = 0;
  }
  c.h = h;
  c.rootN = rootN;
  c.rootN_lo = rootN_lo;
  if constexpr (LineCtx<E, H, S, T>::kHoist && H > 1) {
#pragma unroll
    for (int k = 0; k < E; ++k) {
      cpx<T> w = rootN[h * k];
      if constexpr (S > 0) w.im = -w.im;
      c.tw[k] = w;
      if constexpr (std::is_same<T, float>::value) {
        cpx<T> l = rootN_lo[h * k];
        if constexpr (S > 0) l.im = -l.im;
        c.twl[k] = l;
      }
    }
  }
  if constexpr (H == 12) {
    // lane h = h0 + 4g: DFT_3 over g, output c = g, then the twiddle
    // w_12^{h0*g}: Y = sum_g' x[g'] w_3^{g'*g} w_12^{h0*g}, with
    // w_3^e = w_12^{4e}; partners g+1 and g+2 (mod 3) of the same h0
    const int h0 = h & 3, g = h >> 2;
    const int g1 = g == 2 ? 0 : g + 1, g2 = g == 0 ? 2 : g - 1;
    const int row = (threadIdx.x & 63) & ~15;
    c.src1 = (row + h0 + 4 * g1) << 2;
    c.src2 = (row + h0 + 4 * g2) << 2;
    c.a3[0] = root12<S, T>(4 * g * g + h0 * g);
    c.a3[1] = root12<S, T>(4 * g1 * g + h0 * g);
    c.a3[2] = root12<S, T>(4 * g2 * g + h0 * g);
    // the 4-lane part: rounds of partner distance 2 and 1 over h0
    int i = 0;
#pragma unroll
    for (int hs = 2; hs >= 1; hs >>= 1, ++i) {
      const int b = (h0 / hs) & 1;
      const int hl = h0 % hs;
      c.sgn[i] = b ? static_cast<T>(-1) : static_cast<T>(1);
      c.rw[i] = (b && hl) ? root16<S, T>(hl * (8 / hs)) : cpx<T>{1, 0};
    }
  } else if constexpr (H > 1) {
    int i = 0;
#pragma unroll
    for (int hs = H / 2; hs >= 1; hs >>= 1, ++i) {
      const int b = (h / hs) & 1;
      const int hl = h % hs;
      c.sgn[i] = b ? static_cast<T>(-1) : static_cast<T>(1);
      // w_{2*hs}^{hl} = root16(hl * 16 / (2*hs))
      c.rw[i] = (b && hl) ? root16<S, T>(hl * (8 / hs)) : cpx<T>{1, 0};
    }
  }
  return c;
}

template <int HS, int I, int E, int H, int S, typename T>
__device__ __forceinline__ void xlane_rounds(cpx<T>* v, const LineCtx<E, H, S, T>& c) {
  if constexpr (HS >= 1) {
    const T sg = c.sgn[I];
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const T pr = dpp_xor<HS>(v[k].re), pi = dpp_xor<HS>(v[k].im);
      v[k] = {ffma(sg, v[k].re, pr), ffma(sg, v[k].im, pi)};
    }
    if constexpr (HS > 1) {
      const cpx<T> w = c.rw[I];
#pragma unroll
      for (int k = 0; k < E; ++k) v[k] = cmul(v[k], w);
    }
    xlane_rounds<HS / 2, I + 1, E, H, S, T>(v, c);
  }
}

// Value of another lane (byte address src = 4*lane) through the LDS
// crossbar; no LDS memory is used.
__device__ __forceinline__ float lane_read(int src, float x) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(x)));
}
__device__ __forceinline__ double lane_read(int src, double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_ds_bpermute(src, static_cast<int>(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_ds_bpermute(src, static_cast<int>(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              (static_cast<long long>(lo) & 0xffffffffll));
}

// The radix-3 step of a 12-lane line: every lane forms its output c = g of
// the DFT_3 over the three 4-lane groups (with the twiddle w_12^{h0*c}).
template <int E, int H, int S, typename T>
__device__ __forceinline__ void xlane_radix3(cpx<T>* v, const LineCtx<E, H, S, T>& c) {
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const cpx<T> p1 = {lane_read(c.src1, v[k].re), lane_read(c.src1, v[k].im)};
    const cpx<T> p2 = {lane_read(c.src2, v[k].re), lane_read(c.src2, v[k].im)};
    v[k] = cmac(cmac(cmul(v[k], c.a3[0]), p1, c.a3[1]), p2, c.a3[2]);
  }
}

// One transform line of length N = E*H spread over H adjacent lanes of a
// wavefront (h = position of the lane in its group). On entry lane h holds
// x[h + H*j] in v[j] (j < E); on exit it holds X[k + E*bitrev(h)] in v[k].
// Cooley-Tukey with N = E*H (Section 2.1): DFT_E in registers, twiddles
// w_N^{h*k}, then DFT_H across the lanes as log2(H) radix-2 rounds (partner
// h ^ H/2, then h ^ H/4, ...) exchanged through DPP.
template <int E, int H, int S, typename T, bool MF = false>
__device__ __forceinline__ void line_fft(cpx<T>* v, const LineCtx<E, H, S, T>& c) {
  if constexpr (MF && E == 16 && std::is_same<T, float>::value) dft16_mfma<S>(v);
  else dft<E, S>(v);
  if constexpr (H > 1) {
    if constexpr (LineCtx<E, H, S, T>::kHoist) {
#pragma unroll
      for (int k = 1; k < E; ++k) {
        if constexpr (std::is_same<T, float>::value)
          v[k] = cmul_hl(v[k], c.tw[k], c.twl[k]);
        else
          v[k] = cmul(v[k], c.tw[k]);
      }
    } else if (c.h > 0) {
#pragma unroll
      for (int k = 1; k < E; ++k) v[k] = twmul<S>(v[k], c.rootN, c.rootN_lo, c.h * k);
    }
    if constexpr (H == 12) {
      xlane_radix3(v, c);
      xlane_rounds<2, 0, E, H, S, T>(v, c);
    } else {
      xlane_rounds<H / 2, 0, E, H, S, T>(v, c);
    }
  }
}

}  // namespace fftb

// fft_core.hpp -- register/LDS building blocks of the batched inverse FFTs.
//
// Host- and device-callable so that the CPU emulator (tests) runs exactly the
// same index arithmetic and butterflies as the gfx950 kernels.
//
// Sign convention: every transform here is the un-normalised inverse DFT
//   X[j] = sum_k x[k] exp(+2 pi i k j / L),
// which turns the frequency-domain integrand into the matched-filter output at
// every coalescence sample (Sec. II.C: maximisation over t_c by FFT).
#pragma once

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define FCAS_HD __host__ __device__ __forceinline__
#else
#include <cmath>
#define FCAS_HD inline
#endif

// Address spaces of the device build.  Tables that a kernel only reads, and
// that earlier launches wrote, are read through the constant address space:
// with a uniform address the compiler then issues scalar loads, which are
// counted apart from the vector memory operations, so that reading the next
// work item's descriptors never waits for the stores and prefetches in flight.
// Segment data reached through pointers held in those tables are read through
// the global address space (vector loads rather than flat ones).  The host
// build (CPU emulator) reads plain memory.
#if defined(__HIP_DEVICE_COMPILE__)
#define FCAS_AS_CONST __attribute__((address_space(4)))
#define FCAS_AS_GLOBAL __attribute__((address_space(1)))
#else
#define FCAS_AS_CONST
#define FCAS_AS_GLOBAL
#endif

namespace fcas {

template <class T>
FCAS_HD const FCAS_AS_CONST T* const_view(const T* p) {
  return (const FCAS_AS_CONST T*)p;
}
template <class T>
FCAS_HD const FCAS_AS_GLOBAL T* global_view(const T* p) {
  return (const FCAS_AS_GLOBAL T*)p;
}

template <typename R>
struct cplx {
  R x, y;
};

template <typename R> FCAS_HD cplx<R> mk(R a, R b) { cplx<R> c; c.x = a; c.y = b; return c; }
template <typename R> FCAS_HD cplx<R> add(cplx<R> a, cplx<R> b) { return mk<R>(a.x + b.x, a.y + b.y); }
template <typename R> FCAS_HD cplx<R> sub(cplx<R> a, cplx<R> b) { return mk<R>(a.x - b.x, a.y - b.y); }
template <typename R> FCAS_HD cplx<R> mul(cplx<R> a, cplx<R> b) {
  return mk<R>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename R> FCAS_HD cplx<R> scale(cplx<R> a, R s) { return mk<R>(a.x * s, a.y * s); }
// multiply by +i
template <typename R> FCAS_HD cplx<R> mul_i(cplx<R> a) { return mk<R>(-a.y, a.x); }
// multiply by -i
template <typename R> FCAS_HD cplx<R> mul_mi(cplx<R> a) { return mk<R>(a.y, -a.x); }
template <typename R> FCAS_HD R norm2(cplx<R> a) { return a.x * a.x + a.y * a.y; }

// ---------------------------------------------------------------------------
// sin(2 pi r), cos(2 pi r) for r in revolutions, |r| <= 1/2, float.
// On gfx950 the hardware sine / cosine take their argument in revolutions
// (measured maximum absolute error 1.3e-7 on [-1/2, 1/2]).  The host build
// (CPU emulation) uses an octant reduction, exact in binary floating point,
// followed by the Taylor series of sin (to t^11) and cos (to t^10) on
// |2 pi t| <= pi/4; truncation error below 1.2e-10.
// ---------------------------------------------------------------------------
FCAS_HD void sincos_rev(float r, float* s, float* c) {
#if defined(__HIP_DEVICE_COMPILE__)
  *s = __builtin_amdgcn_sinf(r);
  *c = __builtin_amdgcn_cosf(r);
#else
  float q = rintf(4.0f * r);           // nearest quarter turn
  float t = r - 0.25f * q;             // |t| <= 1/8, exact
  float u = t * t;
  // coefficients (2 pi)^n / n! with alternating signs
  const float S1 = 6.283185307179586f, S3 = -41.341702240399755f, S5 = 81.60524927607504f,
              S7 = -76.70585975306136f, S9 = 42.058693944897634f, S11 = -15.094642576822984f;
  const float C2 = -19.739208802178716f, C4 = 64.93939402266828f, C6 = -85.45681720669371f,
              C8 = 60.24464137187664f, C10 = -26.426256783374388f;
  float sn = t * (S1 + u * (S3 + u * (S5 + u * (S7 + u * (S9 + u * S11)))));
  float cs = 1.0f + u * (C2 + u * (C4 + u * (C6 + u * (C8 + u * C10))));
  int qi = ((int)q) & 3;
  float so = sn, co = cs;
  if (qi == 1) { so = cs; co = -sn; }
  else if (qi == 2) { so = -sn; co = -cs; }
  else if (qi == 3) { so = -cs; co = sn; }
  *s = so;
  *c = co;
#endif
}

// double version for the FP64 path: sin(2 pi r), cos(2 pi r)
FCAS_HD void sincos_rev(double r, double* s, double* c) {
#if defined(__HIP_DEVICE_COMPILE__)
  sincospi(2.0 * r, s, c);
#else
  const double tp = 6.283185307179586476925286766559;
  *s = std::sin(tp * r);
  *c = std::cos(tp * r);
#endif
}

// e^{+2 pi i m / L} for integer 0 <= m < L
template <typename R>
FCAS_HD cplx<R> twiddle(int m, int L) {
  R s, c;
  R r = (R)m / (R)L;
  if (r > (R)0.5) r -= (R)1;
  sincos_rev(r, &s, &c);
  return mk<R>(c, s);
}

// Streaming (non-temporal) access to the FFT workspace: each element is
// written once by pass 1 and read once by pass 2, so it should not displace
// the segment data that every work item re-reads from L2.
template <typename R>
FCAS_HD cplx<R> stream_load(const cplx<R>* p) {
#if defined(__HIP_DEVICE_COMPILE__)
  typedef R v2 __attribute__((ext_vector_type(2)));
  const v2 t = __builtin_nontemporal_load((const v2*)p);
  return mk<R>(t.x, t.y);
#else
  return *p;
#endif
}

template <typename R>
FCAS_HD void stream_store(cplx<R>* p, cplx<R> v) {
#if defined(__HIP_DEVICE_COMPILE__)
  typedef R v2 __attribute__((ext_vector_type(2)));
  v2 t;
  t.x = v.x;
  t.y = v.y;
  __builtin_nontemporal_store(t, (v2*)p);
#else
  *p = v;
#endif
}

// Non-temporal stores into one region of the workspace through a buffer
// resource (base and size in scalar registers).  A store's byte offset is a
// per-thread part (a vector register) plus a uniform part (a scalar register
// or constant), so the stores of a thread at compile-time strides share one
// address computation instead of a 64-bit address each.  The region is at
// most 2^32 - 1 bytes; the hardware drops a store past its end.
template <typename R>
struct StreamOut {
#if defined(__HIP_DEVICE_COMPILE__)
  __amdgpu_buffer_rsrc_t rs;
  FCAS_HD StreamOut(cplx<R>* base, int64_t elems)
      : rs(__builtin_amdgcn_make_buffer_rsrc(base, 0, (int)(elems * (int64_t)sizeof(cplx<R>)), kRsrcWord3)) {}
  // element `vo + so` of the region, vo per thread, so uniform
  FCAS_HD void store(int vo, int so, cplx<R> v) const {
    if constexpr (sizeof(R) == 4) {
      typedef int i2 __attribute__((ext_vector_type(2)));
      i2 t;
      t.x = __builtin_bit_cast(int, v.x);
      t.y = __builtin_bit_cast(int, v.y);
      __builtin_amdgcn_raw_buffer_store_b64(t, rs, vo * (int)sizeof(cplx<R>), so * (int)sizeof(cplx<R>), kNt);
    } else {
      typedef int i4 __attribute__((ext_vector_type(4)));
      const long long xr = __builtin_bit_cast(long long, v.x), yr = __builtin_bit_cast(long long, v.y);
      i4 t;
      t.x = (int)xr;
      t.y = (int)(xr >> 32);
      t.z = (int)yr;
      t.w = (int)(yr >> 32);
      __builtin_amdgcn_raw_buffer_store_b128(t, rs, vo * (int)sizeof(cplx<R>), so * (int)sizeof(cplx<R>), kNt);
    }
  }
  // descriptor word 3 of an untyped gfx9 buffer (32-bit data format); cache
  // policy of the stores: non-temporal
  static constexpr int kRsrcWord3 = 0x00020000;
  static constexpr int kNt = 2;
#else
  cplx<R>* base;
  FCAS_HD StreamOut(cplx<R>* b, int64_t) : base(b) {}
  FCAS_HD void store(int vo, int so, cplx<R> v) const { base[(int64_t)vo + so] = v; }
#endif
};

// ---------------------------------------------------------------------------
// Small inverse DFTs in registers: x[0..R) -> X[0..R), X[j] = sum_p x[p] w_R^{pj}
// ---------------------------------------------------------------------------
template <typename T>
FCAS_HD void dft2(cplx<T>& a, cplx<T>& b) {
  cplx<T> t = a;
  a = add(t, b);
  b = sub(t, b);
}

template <typename T>
FCAS_HD void dft4(cplx<T>& x0, cplx<T>& x1, cplx<T>& x2, cplx<T>& x3) {
  cplx<T> a = add(x0, x2), b = sub(x0, x2), c = add(x1, x3), d = mul_i(sub(x1, x3));
  x0 = add(a, c);
  x2 = sub(a, c);
  x1 = add(b, d);
  x3 = sub(b, d);
}

template <typename T>
FCAS_HD void dft3(cplx<T>& x0, cplx<T>& x1, cplx<T>& x2) {
  // w = e^{+2 pi i/3} = -1/2 + i sqrt(3)/2
  const T h = (T)0.86602540378443864676;
  const cplx<T> s = add(x1, x2), d = sub(x1, x2);
  const cplx<T> m = mk<T>(x0.x - (T)0.5 * s.x, x0.y - (T)0.5 * s.y);
  // i h d = (-h d.y, h d.x)
  x0 = add(x0, s);
  x1 = mk<T>(m.x - h * d.y, m.y + h * d.x);
  x2 = mk<T>(m.x + h * d.y, m.y - h * d.x);
}

// w = e^{+2 pi i/5}: X[j] = x0 + sum_{p=1..4} x_p w^{pj}.  The conjugate pairs
// (x1, x4) and (x2, x3) enter through their sums (real parts of w^p) and
// differences (imaginary parts).
template <typename T>
FCAS_HD void dft5(cplx<T>* x) {
  const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;   // cos(2 pi/5), cos(4 pi/5)
  const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;    // sin(2 pi/5), sin(4 pi/5)
  const cplx<T> t1 = add(x[1], x[4]), t2 = add(x[2], x[3]), t3 = sub(x[1], x[4]), t4 = sub(x[2], x[3]);
  const cplx<T> a1 = mk<T>(x[0].x + c1 * t1.x + c2 * t2.x, x[0].y + c1 * t1.y + c2 * t2.y);
  const cplx<T> a2 = mk<T>(x[0].x + c2 * t1.x + c1 * t2.x, x[0].y + c2 * t1.y + c1 * t2.y);
  const cplx<T> b1 = mk<T>(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y);
  const cplx<T> b2 = mk<T>(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y);
  x[0] = add(x[0], add(t1, t2));
  x[1] = add(a1, mul_i(b1));
  x[4] = sub(a1, mul_i(b1));
  x[2] = add(a2, mul_i(b2));
  x[3] = sub(a2, mul_i(b2));
}

// 15 = 3 x 5 by the prime-factor (Good-Thomas) algorithm, which needs no
// twiddle factors: input n = (5 n1 + 3 n2) mod 15 and output
// k = (10 k1 + 6 k2) mod 15 (the CRT map; 10 = 1 mod 3, 6 = 1 mod 5) give
// w15^{nk} = w3^{n1 k1} w5^{n2 k2}.  Five 3-point transforms over n1, then
// three 5-point transforms over n2.
template <typename T>
FCAS_HD void dft15(cplx<T>* x) {
  cplx<T> y[5][3];
#pragma unroll
  for (int n2 = 0; n2 < 5; ++n2) {
    cplx<T> a0 = x[(3 * n2) % 15], a1 = x[(5 + 3 * n2) % 15], a2 = x[(10 + 3 * n2) % 15];
    dft3(a0, a1, a2);
    y[n2][0] = a0; y[n2][1] = a1; y[n2][2] = a2;
  }
#pragma unroll
  for (int k1 = 0; k1 < 3; ++k1) {
    cplx<T> z[5] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1], y[4][k1]};
    dft5(z);
#pragma unroll
    for (int k2 = 0; k2 < 5; ++k2) x[(10 * k1 + 6 * k2) % 15] = z[k2];
  }
}

// Last step of an 8-point DFT from the 4-point DFTs of the even (e) and odd
// (o) inputs: X[j] = e_j + w8^j o_j, X[j+4] = e_j - w8^j o_j.  The 1/sqrt2 of
// w8^1 = (1+i)/sqrt2 and w8^3 = (-1+i)/sqrt2 is applied inside the sums, each
// output component one expression (a single fused multiply-add).
template <typename T>
FCAS_HD void dft8_combine(cplx<T>* x, cplx<T> e0, cplx<T> e1, cplx<T> e2, cplx<T> e3, cplx<T> o0, cplx<T> o1,
                          cplx<T> o2, cplx<T> o3) {
  const T r = (T)0.70710678118654752440;
  const T a1 = o1.x - o1.y, b1 = o1.x + o1.y;    // (1+i) o1
  const T a3 = -o3.x - o3.y, b3 = o3.x - o3.y;   // (-1+i) o3
  const cplx<T> t2 = mul_i(o2);                  // w8^2 = i
  x[0] = add(e0, o0); x[4] = sub(e0, o0);
  x[1] = mk<T>(e1.x + r * a1, e1.y + r * b1); x[5] = mk<T>(e1.x - r * a1, e1.y - r * b1);
  x[2] = add(e2, t2); x[6] = sub(e2, t2);
  x[3] = mk<T>(e3.x + r * a3, e3.y + r * b3); x[7] = mk<T>(e3.x - r * a3, e3.y - r * b3);
}

template <typename T>
FCAS_HD void dft8(cplx<T>* x) {
  // even / odd split, then combine with w_8^j
  cplx<T> e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
  cplx<T> o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  dft8_combine(x, e0, e1, e2, e3, o0, o1, o2, o3);
}

template <typename T>
FCAS_HD void dft16(cplx<T>* x) {
  // 16 = 4 x 4: p = 4a + b, j = c + 4d.
  // inner DFT4 over a for each b, twiddle w16^{b c}, outer DFT4 over b for each c.
  cplx<T> y[16];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    cplx<T> a0 = x[b], a1 = x[b + 4], a2 = x[b + 8], a3 = x[b + 12];
    dft4(a0, a1, a2, a3);
    y[4 * b + 0] = a0; y[4 * b + 1] = a1; y[4 * b + 2] = a2; y[4 * b + 3] = a3;   // y[4b + c]
  }
  const T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173;
  const T r2 = (T)0.70710678118654752440;
  // w16^m = e^{+2 pi i m /16}
  const cplx<T> w1 = mk<T>(c1, s1), w2 = mk<T>(r2, r2), w3 = mk<T>(s1, c1);
  const cplx<T> w6 = mk<T>(-r2, r2), w9 = mk<T>(-c1, -s1);
  // b=1: c=1,2,3 -> w^1, w^2, w^3 ; b=2: w^2, w^4, w^6 ; b=3: w^3, w^6, w^9
  y[5] = mul(y[5], w1); y[6] = mul(y[6], w2); y[7] = mul(y[7], w3);
  y[9] = mul(y[9], w2); y[10] = mul_i(y[10]); y[11] = mul(y[11], w6);
  y[13] = mul(y[13], w3); y[14] = mul(y[14], w6); y[15] = mul(y[15], w9);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    cplx<T> b0 = y[c], b1 = y[4 + c], b2 = y[8 + c], b3 = y[12 + c];
    dft4(b0, b1, b2, b3);
    x[c] = b0; x[c + 4] = b1; x[c + 8] = b2; x[c + 12] = b3;
  }
}

// Inverse DFT of R points whose upper half x[R/2..R) is zero (the negative
// frequencies of the pass-1 columns).  x[R/2..R) need not be initialised.
template <typename T>
FCAS_HD void dft4_half(cplx<T>& x0, cplx<T>& x1, cplx<T>& x2, cplx<T>& x3) {
  const cplx<T> a = x0, b = x1, ib = mul_i(x1);
  x0 = add(a, b);
  x1 = add(a, ib);
  x2 = sub(a, b);
  x3 = sub(a, ib);
}

template <int R, typename T>
FCAS_HD void dft_half(cplx<T>* x) {
  if constexpr (R == 2) {
    x[1] = x[0];
  } else if constexpr (R == 4) {
    dft4_half(x[0], x[1], x[2], x[3]);
  } else if constexpr (R == 8) {
    cplx<T> e0 = x[0], e1 = x[2], e2, e3, o0 = x[1], o1 = x[3], o2, o3;
    dft4_half(e0, e1, e2, e3);
    dft4_half(o0, o1, o2, o3);
    dft8_combine(x, e0, e1, e2, e3, o0, o1, o2, o3);
  } else if constexpr (R == 16) {
    cplx<T> y[16];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      cplx<T> a0 = x[b], a1 = x[b + 4], a2, a3;
      dft4_half(a0, a1, a2, a3);
      y[4 * b + 0] = a0; y[4 * b + 1] = a1; y[4 * b + 2] = a2; y[4 * b + 3] = a3;
    }
    const T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173;
    const T r2 = (T)0.70710678118654752440;
    const cplx<T> w1 = mk<T>(c1, s1), w2 = mk<T>(r2, r2), w3 = mk<T>(s1, c1);
    const cplx<T> w6 = mk<T>(-r2, r2), w9 = mk<T>(-c1, -s1);
    y[5] = mul(y[5], w1); y[6] = mul(y[6], w2); y[7] = mul(y[7], w3);
    y[9] = mul(y[9], w2); y[10] = mul_i(y[10]); y[11] = mul(y[11], w6);
    y[13] = mul(y[13], w3); y[14] = mul(y[14], w6); y[15] = mul(y[15], w9);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      cplx<T> b0 = y[c], b1 = y[4 + c], b2 = y[8 + c], b3 = y[12 + c];
      dft4(b0, b1, b2, b3);
      x[c] = b0; x[c + 4] = b1; x[c + 8] = b2; x[c + 12] = b3;
    }
  } else {
    static_assert(R == 2 || R == 4 || R == 8 || R == 16, "unsupported half-input radix");
  }
}

template <int R, typename T>
FCAS_HD void dft(cplx<T>* x) {
  if constexpr (R == 2) {
    dft2(x[0], x[1]);
  } else if constexpr (R == 3) {
    dft3(x[0], x[1], x[2]);
  } else if constexpr (R == 4) {
    dft4(x[0], x[1], x[2], x[3]);
  } else if constexpr (R == 5) {
    dft5(x);
  } else if constexpr (R == 8) {
    dft8(x);
  } else if constexpr (R == 15) {
    dft15(x);
  } else if constexpr (R == 16) {
    dft16(x);
  } else {
    static_assert(R == 2 || R == 3 || R == 4 || R == 5 || R == 8 || R == 15 || R == 16, "unsupported radix");
  }
}

// ---------------------------------------------------------------------------
// Stockham schedule of one length-L transform spread over P = L/E threads,
// each holding E elements in registers.  Register q of thread t holds element
// t + q P both before the first stage and after the last, so the prologue
// loads and the epilogue stores are strided by P ("natural strided order").
//
// Stage s with radix R and Ns = product of the earlier radices: butterfly b of
// thread t is the virtual thread v = t + b P (0 <= v < L/R); its inputs are
// elements v + p L/R (registers b + p E/R), twiddled by w_{Ns R}^{(v mod Ns) p},
// and its outputs go to (v / Ns) Ns R + (v mod Ns) + p Ns.
// ---------------------------------------------------------------------------
template <int... Rs>
struct Radices {
  static constexpr int count = sizeof...(Rs);
  static constexpr int value[sizeof...(Rs)] = {Rs...};
  static constexpr int product() {
    int p = 1;
    for (int i = 0; i < count; ++i) p *= value[i];
    return p;
  }
};

// LDS index padding: one spare element after every 2^S (S > 0) breaks the
// power-of-two strides of the stage writes across banks; S = 0 leaves the
// buffer unpadded.  Each pass takes the S measured fastest for it.
template <int S>
FCAS_HD int lds_pad(int i) {
  if constexpr (S > 0) return i + (i >> S);
  else return i;
}
template <int S>
constexpr int lds_padded_len(int L) {
  if constexpr (S > 0) return L + (L >> S) + 1;
  else return L;
}

// position of output p of virtual thread v in stage with sub-length Ns, radix R
FCAS_HD int stockham_dst(int v, int Ns, int R, int p) { return (v / Ns) * Ns * R + (v % Ns) + p * Ns; }

// Twiddle index (into a table of w_L^m, m < L) for input p of virtual thread v.
FCAS_HD int stockham_tw(int v, int Ns, int R, int p, int L) { return (v % Ns) * p * (L / (Ns * R)); }

}  // namespace fcas

// Device building blocks for the split-step kernels (gfx950).
//
//  * cx<T>            interleaved complex in registers (T = float or double).
//  * Stockham FFT     register-resident, radix 2/3/4/8 passes with LDS exchanges.
//  * sym4_apply       spin-2 rotation of a 5-vector as the 4th symmetric power of an
//                     SU(2) element, factored L * D * R (two Taylor shifts + diagonal).
//  * nl_point         exact nonlinear flow at one grid point (Sec. 3.2, eq. solution2).
//
// Component order everywhere: index i = 0..4 <-> spin projection l = 2, 1, 0, -1, -2.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sgp {

template <typename T>
struct __align__(2 * sizeof(T)) cx {
  T re, im;
};

template <typename T> __device__ __forceinline__ cx<T> mk(T r, T i) { cx<T> z; z.re = r; z.im = i; return z; }
template <typename T> __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk<T>(a.re + b.re, a.im + b.im); }
template <typename T> __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk<T>(a.re - b.re, a.im - b.im); }
template <typename T> __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return mk<T>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T> __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return mk<T>(s * a.re, s * a.im); }
template <typename T> __device__ __forceinline__ cx<T> conj(cx<T> a) { return mk<T>(a.re, -a.im); }
template <typename T> __device__ __forceinline__ T norm2(cx<T> a) { return a.re * a.re + a.im * a.im; }
// i * a
template <typename T> __device__ __forceinline__ cx<T> mul_i(cx<T> a) { return mk<T>(-a.im, a.re); }
// conj(a) * b
template <typename T> __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return mk<T>(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
// acc + a * b
template <typename T> __device__ __forceinline__ cx<T> cfma(cx<T> a, cx<T> b, cx<T> acc) {
  return mk<T>(acc.re + a.re * b.re - a.im * b.im, acc.im + a.re * b.im + a.im * b.re);
}

// x + a x for a factor 1 + a close to 1, with the product a x formed before the sum.
// In cfma's order the small real part of a (of second order in the angle, for a
// unit-modulus factor) is added to x alone and rounds away whenever it is below half
// an ulp of x, always in the same direction, so that repeated unit-modulus factors
// let |x| grow; formed first, it is a term of a x and its rounding is unbiased.
template <typename T> __device__ __forceinline__ cx<T> inc_apply(cx<T> a, cx<T> x) {
  const cx<T> d = a * x;
  return mk<T>(x.re + d.re, x.im + d.im);
}

// 1/x.  FP32: the hardware reciprocal estimate (within 1 ulp) refined by one Newton
// step; FP64: division.  Used only on magnitudes bounded away from 0 and infinity.
template <typename T>
__device__ __forceinline__ T recip(T x) {
  if constexpr (sizeof(T) == 4) {
    const float y = __builtin_amdgcn_rcpf(x);
    return fmaf(fmaf(-x, y, 1.0f), y, y);
  } else {
    return T(1) / x;
  }
}

// Square root of x >= 0.  FP32: the hardware square root (within 1 ulp; the results
// only set small rotation angles); FP64: sqrt.
template <typename T>
__device__ __forceinline__ T sqrt_nn(T x) {
  if constexpr (sizeof(T) == 4) return __builtin_amdgcn_sqrtf(x);
  else return sqrt(x);
}


// ---------------------------------------------------------------------------
// Small DFT kernels, y_q = sum_s x_s exp(SIGN 2 pi i s q / R), in place.
// ---------------------------------------------------------------------------
template <int SIGN, typename T>
__device__ __forceinline__ cx<T> rot_quarter(cx<T> a) {  // a * exp(SIGN i pi/2)
  return SIGN < 0 ? mk<T>(a.im, -a.re) : mk<T>(-a.im, a.re);
}

template <int R, int SIGN, typename T>
struct Dft;

template <int SIGN, typename T>
struct Dft<2, SIGN, T> {
  __device__ __forceinline__ static void run(cx<T>* x) {
    cx<T> a = x[0], b = x[1];
    x[0] = a + b;
    x[1] = a - b;
  }
};

// c * z for a constant c = c_hi + c_lo (c_lo = 0 in FP64): a rounded constant would
// repeat the same relative error in every step.
template <typename T>
__device__ __forceinline__ T kmul(T hi, T lo, T z) {
  if constexpr (sizeof(T) == 4) return fmaf(hi, z, lo * z);
  else return hi * z;
}

template <int SIGN, typename T>
struct Dft<3, SIGN, T> {
  __device__ __forceinline__ static void run(cx<T>* x) {
    // sqrt(3)/2 as a float pair
    const T sh = T(0.866025388240814208984375), sl = T(sizeof(T) == 4 ? 1.5543625e-08 : 0.0);
    const T s3 = sizeof(T) == 4 ? sh : T(0.86602540378443864676372317075293618);
    cx<T> a = x[0], b = x[1], d = x[2];
    cx<T> sum = b + d, dif = b - d;
    x[0] = a + sum;
    cx<T> m = mk<T>(a.re - T(0.5) * sum.re, a.im - T(0.5) * sum.im);
    // SIGN * i * sqrt(3)/2 * dif
    cx<T> r = mk<T>(-kmul<T>(s3, sl, dif.im), kmul<T>(s3, sl, dif.re));
    if (SIGN < 0) r = mk<T>(-r.re, -r.im);
    x[1] = m + r;
    x[2] = m - r;
  }
};

template <int SIGN, typename T>
struct Dft<4, SIGN, T> {
  __device__ __forceinline__ static void run(cx<T>* x) {
    cx<T> a0 = x[0] + x[2], a1 = x[0] - x[2];
    cx<T> b0 = x[1] + x[3], b1 = rot_quarter<SIGN>(x[1] - x[3]);
    x[0] = a0 + b0;
    x[2] = a0 - b0;
    x[1] = a1 + b1;
    x[3] = a1 - b1;
  }
};

// Length 6 = 2 * 3 by the prime-factor (Good-Thomas) mapping, which needs no inner
// twiddles: input n = (3 n1 + 2 n2) mod 6, output k = (3 k1 + 4 k2) mod 6, so that
// exp(2 pi i n k / 6) = exp(2 pi i n1 k1 / 2) exp(2 pi i n2 k2 / 3).
template <int SIGN, typename T>
struct Dft<6, SIGN, T> {
  __device__ __forceinline__ static void run(cx<T>* x) {
    // length-2 transforms over n1 for n2 = 0, 1, 2 (inputs (0, 3), (2, 5), (4, 1))
    cx<T> y0[3] = {x[0] + x[3], x[2] + x[5], x[4] + x[1]};  // k1 = 0
    cx<T> y1[3] = {x[0] - x[3], x[2] - x[5], x[4] - x[1]};  // k1 = 1
    // length-3 transforms over n2; k2 = 0, 1, 2 land at (3 k1 + 4 k2) mod 6
    Dft<3, SIGN, T>::run(y0);
    Dft<3, SIGN, T>::run(y1);
    x[0] = y0[0];
    x[4] = y0[1];
    x[2] = y0[2];
    x[3] = y1[0];
    x[1] = y1[1];
    x[5] = y1[2];
  }
};

// Length 12 = 4 * 3 by the prime-factor mapping (no inner twiddles): input
// n = (3 n1 + 4 n2) mod 12, output k = (9 k1 + 4 k2) mod 12, so that
// exp(2 pi i n k / 12) = exp(2 pi i n1 k1 / 4) exp(2 pi i n2 k2 / 3).
template <int SIGN, typename T>
struct Dft<12, SIGN, T> {
  __device__ __forceinline__ static void run(cx<T>* x) {
    // length-4 transforms over n1 for n2 = 0, 1, 2
    cx<T> a[4] = {x[0], x[3], x[6], x[9]};
    cx<T> b[4] = {x[4], x[7], x[10], x[1]};
    cx<T> c[4] = {x[8], x[11], x[2], x[5]};
    Dft<4, SIGN, T>::run(a);
    Dft<4, SIGN, T>::run(b);
    Dft<4, SIGN, T>::run(c);
    // length-3 transforms over n2 for k1 = 0..3; k2 = 0, 1, 2 land at (9 k1 + 4 k2) mod 12
    cx<T> z0[3] = {a[0], b[0], c[0]};
    cx<T> z1[3] = {a[1], b[1], c[1]};
    cx<T> z2[3] = {a[2], b[2], c[2]};
    cx<T> z3[3] = {a[3], b[3], c[3]};
    Dft<3, SIGN, T>::run(z0);
    Dft<3, SIGN, T>::run(z1);
    Dft<3, SIGN, T>::run(z2);
    Dft<3, SIGN, T>::run(z3);
    x[0] = z0[0]; x[4] = z0[1]; x[8] = z0[2];
    x[9] = z1[0]; x[1] = z1[1]; x[5] = z1[2];
    x[6] = z2[0]; x[10] = z2[1]; x[2] = z2[2];
    x[3] = z3[0]; x[7] = z3[1]; x[11] = z3[2];
  }
};

// Length 16 = 4 x 4: length-4 transforms over n1 of x[4 n1 + n2], the inner
// twiddles exp(SIGN 2 pi i n2 k1 / 16) (compensated constants in FP32), then
// length-4 transforms over n2, landing at k1 + 4 k2.
template <int SIGN, typename T>
__device__ __forceinline__ cx<T> w16_mul(cx<T> z, T crh, T crl, T cih, T cil) {
  // z * (cr + SIGN i ci)
  const T a = kmul<T>(crh, crl, z.re), b = kmul<T>(cih, cil, z.im);
  const T c = kmul<T>(cih, cil, z.re), d = kmul<T>(crh, crl, z.im);
  return SIGN > 0 ? mk<T>(a - b, c + d) : mk<T>(a + b, d - c);
}

template <int SIGN, typename T>
struct Dft<16, SIGN, T> {
  __device__ __forceinline__ static void run(cx<T>* x) {
    const bool f32 = sizeof(T) == 4;
    // cos(pi/8), sin(pi/8), sqrt(2)/2 as (hi, lo) pairs in FP32
    const T ch = f32 ? T(0.92387950420379638671875) : T(0.92387953251128675612818318939678829);
    const T cl = T(f32 ? 2.830749e-08 : 0.0);
    const T sh = f32 ? T(0.3826834261417388916015625) : T(0.38268343236508977172845998403039887);
    const T sl = T(f32 ? 6.2233507e-09 : 0.0);
    const T hh = f32 ? T(0.707106769084930419921875) : T(0.70710678118654752440084436210484904);
    const T hl = T(f32 ? 1.2101617e-08 : 0.0);
    cx<T> a[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      a[n2][0] = x[n2];
      a[n2][1] = x[4 + n2];
      a[n2][2] = x[8 + n2];
      a[n2][3] = x[12 + n2];
      Dft<4, SIGN, T>::run(a[n2]);
    }
    // twiddles exp(SIGN 2 pi i j / 16), j = n2 k1
    a[1][1] = w16_mul<SIGN, T>(a[1][1], ch, cl, sh, sl);  // j = 1
    a[1][2] = w16_mul<SIGN, T>(a[1][2], hh, hl, hh, hl);  // j = 2
    a[1][3] = w16_mul<SIGN, T>(a[1][3], sh, sl, ch, cl);  // j = 3
    a[2][1] = w16_mul<SIGN, T>(a[2][1], hh, hl, hh, hl);  // j = 2
    a[2][2] = rot_quarter<SIGN>(a[2][2]);                  // j = 4
    {                                                      // j = 6: -h + SIGN i h
      const cx<T> t = w16_mul<SIGN, T>(a[2][3], hh, hl, hh, hl);
      a[2][3] = rot_quarter<SIGN>(t);
    }
    a[3][1] = w16_mul<SIGN, T>(a[3][1], sh, sl, ch, cl);  // j = 3
    {                                                      // j = 6
      const cx<T> t = w16_mul<SIGN, T>(a[3][2], hh, hl, hh, hl);
      a[3][2] = rot_quarter<SIGN>(t);
    }
    {                                                      // j = 9: -(c + SIGN i s)
      const cx<T> t = w16_mul<SIGN, T>(a[3][3], ch, cl, sh, sl);
      a[3][3] = mk<T>(-t.re, -t.im);
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      cx<T> z[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
      Dft<4, SIGN, T>::run(z);
      x[k1] = z[0];
      x[k1 + 4] = z[1];
      x[k1 + 8] = z[2];
      x[k1 + 12] = z[3];
    }
  }
};

template <int SIGN, typename T>
struct Dft<8, SIGN, T> {
  __device__ __forceinline__ static void run(cx<T>* x) {
    // sqrt(2)/2 as a float pair
    const T hh = sizeof(T) == 4 ? T(0.707106769084930419921875) : T(0.70710678118654752440084436210484904);
    const T hl = T(sizeof(T) == 4 ? 1.2101617e-08 : 0.0);
    // two length-4 DFTs on even and odd samples
    cx<T> e[4] = {x[0], x[2], x[4], x[6]};
    cx<T> o[4] = {x[1], x[3], x[5], x[7]};
    Dft<4, SIGN, T>::run(e);
    Dft<4, SIGN, T>::run(o);
    // twiddles exp(SIGN 2 pi i q / 8), q = 1, 2, 3
    cx<T> o1 = o[1], o2 = o[2], o3 = o[3];
    cx<T> t1, t2, t3;
    if (SIGN < 0) {
      t1 = mk<T>(kmul<T>(hh, hl, o1.re + o1.im), kmul<T>(hh, hl, o1.im - o1.re));
      t2 = mk<T>(o2.im, -o2.re);
      t3 = mk<T>(kmul<T>(hh, hl, o3.im - o3.re), -kmul<T>(hh, hl, o3.re + o3.im));
    } else {
      t1 = mk<T>(kmul<T>(hh, hl, o1.re - o1.im), kmul<T>(hh, hl, o1.re + o1.im));
      t2 = mk<T>(-o2.im, o2.re);
      t3 = mk<T>(-kmul<T>(hh, hl, o3.re + o3.im), kmul<T>(hh, hl, o3.re - o3.im));
    }
    x[0] = e[0] + o[0];
    x[4] = e[0] - o[0];
    x[1] = e[1] + t1;
    x[5] = e[1] - t1;
    x[2] = e[2] + t2;
    x[6] = e[2] - t2;
    x[3] = e[3] + t3;
    x[7] = e[3] - t3;
  }
};

// ---------------------------------------------------------------------------
// Register-resident Stockham FFT of length N along one line.
//
// The line is owned by TL = N / E threads; thread t holds elements t + TL*m,
// m = 0..E-1, in v[m].  A pass of radix R (sub-transform size NS before the pass)
// runs E/R butterflies per thread: butterfly j = t + TL*b takes inputs
// j + (N/R) r (registers b + (E/R) r), multiplies input r by w^(r (j mod NS)),
// w = exp(SIGN 2 pi i / (NS R)), and its output r lands at element
// (j / NS) NS R + (j mod NS) + r NS.  That position lies in another thread's
// registers except after the last pass, where it is the input position again,
// so a transform needs (passes - 1) LDS exchanges and both ends of it use the same
// register layout.  Twiddles come from a per-pass table: for each k in [0, NS)
// the R-1 values w^(r k), r = 1..R-1, each stored as a (hi, lo) pair.
//
// LDS exchange buffers are split re / im and padded by one slot every 8 entries
// (bank-conflict-free stride-8 writes).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 3); }
template <int N> struct LdsLine { static constexpr int size = N + N / 8; };

// x * (wh + wl) with the small product folded in before the large one.
template <typename T>
__device__ __forceinline__ cx<T> twmul(cx<T> x, cx<T> wh, cx<T> wl) {
  if constexpr (sizeof(T) == 4) {
    const T sr = x.re * wl.re - x.im * wl.im;
    const T si = x.re * wl.im + x.im * wl.re;
    return mk<T>(fmaf(x.re, wh.re, fmaf(-x.im, wh.im, sr)), fmaf(x.re, wh.im, fmaf(x.im, wh.re, si)));
  } else {
    return x * wh;
  }
}

// SYNC = 0: the line's threads may span several wavefronts (workgroup barrier);
// SYNC = 1: every line lies inside one wavefront (wavefront-scope ordering only).
template <int SYNC>
__device__ __forceinline__ void lds_sync() {
  if constexpr (SYNC == 0) {
    __syncthreads();
  } else {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// NBUF: how many components share one LDS exchange round (1 <= NBUF <= NC); buffer
// b of a line starts at b * lds_stride.
template <typename T, int N, int E, int R, int NS, int SIGN, bool LAST, int NC, int NBUF, int SYNC>
__device__ __forceinline__ void fft_pass(cx<T> (&v)[NC][E], cx<T>* __restrict__ lx, int t,
                                         const cx<T>* __restrict__ tw, int lds_stride) {
  constexpr int TL = N / E;
  constexpr int B = E / R;
  static_assert(E % R == 0, "radix must divide the elements per thread");
  // twiddles for this thread's butterflies (shared by all NC components), each a
  // (hi, lo) pair so that the product carries no fixed rounding of the twiddle
  cx<T> w[B][R > 1 ? R - 1 : 1], wl[B][R > 1 ? R - 1 : 1];
  if constexpr (NS > 1) {
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = t + TL * b;
      const int k = j % NS;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        // table order [r - 1][k]: adjacent lanes (adjacent k) read adjacent entries
        cx<T> z = tw[2 * ((r - 1) * NS + k)];
        cx<T> zl = tw[2 * ((r - 1) * NS + k) + 1];
        w[b][r - 1] = SIGN < 0 ? z : conj(z);
        wl[b][r - 1] = SIGN < 0 ? zl : conj(zl);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
#pragma unroll
    for (int b = 0; b < B; ++b) {
      cx<T> x[R];
#pragma unroll
      for (int r = 0; r < R; ++r) x[r] = v[c][b + B * r];
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) x[r] = twmul(x[r], w[b][r - 1], wl[b][r - 1]);
      }
      Dft<R, SIGN, T>::run(x);
      if constexpr (LAST) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[c][b + B * r] = x[r];
      } else {
        const int j = t + TL * b;
        const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int o = lds_pad(base + r * NS) + (c % NBUF) * lds_stride;
          lx[o] = x[r];
        }
      }
    }
    if constexpr (!LAST) {
      if (c % NBUF == NBUF - 1 || c == NC - 1) {
        lds_sync<SYNC>();
        const int c0 = c - (c % NBUF);
#pragma unroll
        for (int cc = c0; cc <= c; ++cc)
#pragma unroll
          for (int m = 0; m < E; ++m) {
            const int o = lds_pad(t + TL * m) + (cc % NBUF) * lds_stride;
            v[cc][m] = lx[o];
          }
        lds_sync<SYNC>();
      }
    }
  }
}

// Radix plans.  Forward passes run in the listed order, the inverse runs the
// reverse order so that the two share the register layout at both ends.
template <int... Rs> struct RadixList {};
template <int N, int E> struct Plan;
// E = 8 (defaults for powers of two)
template <> struct Plan<16, 8> { using fwd = RadixList<2, 8>; using inv = RadixList<8, 2>; };
template <> struct Plan<32, 8> { using fwd = RadixList<4, 8>; using inv = RadixList<8, 4>; };
template <> struct Plan<64, 8> { using fwd = RadixList<8, 8>; using inv = RadixList<8, 8>; };
template <> struct Plan<128, 8> { using fwd = RadixList<2, 8, 8>; using inv = RadixList<8, 8, 2>; };
template <> struct Plan<256, 8> { using fwd = RadixList<4, 8, 8>; using inv = RadixList<8, 8, 4>; };
template <> struct Plan<512, 8> { using fwd = RadixList<8, 8, 8>; using inv = RadixList<8, 8, 8>; };
// E = 4: radix 2 and 4 only, twice the threads per line
template <> struct Plan<16, 4> { using fwd = RadixList<4, 4>; using inv = RadixList<4, 4>; };
template <> struct Plan<32, 4> { using fwd = RadixList<2, 4, 4>; using inv = RadixList<4, 4, 2>; };
template <> struct Plan<64, 4> { using fwd = RadixList<4, 4, 4>; using inv = RadixList<4, 4, 4>; };
template <> struct Plan<128, 4> { using fwd = RadixList<2, 4, 4, 4>; using inv = RadixList<4, 4, 4, 2>; };
template <> struct Plan<256, 4> { using fwd = RadixList<4, 4, 4, 4>; using inv = RadixList<4, 4, 4, 4>; };
template <> struct Plan<512, 4> { using fwd = RadixList<2, 4, 4, 4, 4>; using inv = RadixList<4, 4, 4, 4, 2>; };
// E = 16: radix 16 for 128 (8.16) and 256 (16.16); for 64 and 512 the E = 8
// radices, two butterflies per thread and pass
template <> struct Plan<64, 16> { using fwd = RadixList<8, 8>; using inv = RadixList<8, 8>; };
template <> struct Plan<128, 16> { using fwd = RadixList<8, 16>; using inv = RadixList<16, 8>; };
template <> struct Plan<256, 16> { using fwd = RadixList<16, 16>; using inv = RadixList<16, 16>; };
template <> struct Plan<512, 16> { using fwd = RadixList<8, 8, 8>; using inv = RadixList<8, 8, 8>; };
// 384 = 3 * 2^7: E = 12 (default) and E = 24
template <> struct Plan<384, 12> { using fwd = RadixList<6, 4, 4, 4>; using inv = RadixList<4, 4, 4, 6>; };
template <> struct Plan<384, 24> { using fwd = RadixList<6, 8, 8>; using inv = RadixList<8, 8, 6>; };
// 192 = 3 * 2^6 and 768 = 3 * 2^8: E = 12 (default) and E = 24 (radix 12: 4 x 3)
template <> struct Plan<192, 12> { using fwd = RadixList<12, 4, 4>; using inv = RadixList<4, 4, 12>; };
template <> struct Plan<192, 24> { using fwd = RadixList<3, 8, 8>; using inv = RadixList<8, 8, 3>; };
template <> struct Plan<768, 12> { using fwd = RadixList<12, 4, 4, 4>; using inv = RadixList<4, 4, 4, 12>; };
template <> struct Plan<768, 24> { using fwd = RadixList<12, 8, 8>; using inv = RadixList<8, 8, 12>; };

// Twiddle-table entries of a plan direction: NS (R - 1) per pass with NS > 1 (each
// entry is a (hi, lo) pair of cx<T>).
template <int... Rs>
constexpr int tw_entries(RadixList<Rs...>) {
  int ns = 1, n = 0;
  ((n += (ns > 1 ? ns * (Rs - 1) : 0), ns *= Rs), ...);
  return n;
}
template <int... Rs>
constexpr int n_passes(RadixList<Rs...>) { return (int)sizeof...(Rs); }
template <int N, int E>
struct TwSize {
  static constexpr int fwd = tw_entries(typename Plan<N, E>::fwd{});
  static constexpr int inv = tw_entries(typename Plan<N, E>::inv{});
  // the first pass has no twiddles and ends with an exchange (a block barrier), so
  // tables staged in LDS before the transform are visible when first read
  static_assert(n_passes(typename Plan<N, E>::fwd{}) >= 2, "plans have at least two passes");
};

// Copy NCX cx<T> values (a whole twiddle table) from global memory to LDS with the
// NT threads of a block, in 16-byte pieces: rounds of up to four pieces per thread,
// all loads of a round issued before its stores (named registers, not an array, so
// that nothing lands in scratch memory).
template <int NT, int NCH, int B>
__device__ __forceinline__ void stage_round(const uint4* __restrict__ s, uint4* __restrict__ d, int tid) {
  uint4 t0 = {}, t1 = {}, t2 = {}, t3 = {};
  if (B + tid < NCH) t0 = s[B + tid];
  if (NCH > B + NT && B + tid + NT < NCH) t1 = s[B + tid + NT];
  if (NCH > B + 2 * NT && B + tid + 2 * NT < NCH) t2 = s[B + tid + 2 * NT];
  if (NCH > B + 3 * NT && B + tid + 3 * NT < NCH) t3 = s[B + tid + 3 * NT];
  if (B + tid < NCH) d[B + tid] = t0;
  if (NCH > B + NT && B + tid + NT < NCH) d[B + tid + NT] = t1;
  if (NCH > B + 2 * NT && B + tid + 2 * NT < NCH) d[B + tid + 2 * NT] = t2;
  if (NCH > B + 3 * NT && B + tid + 3 * NT < NCH) d[B + tid + 3 * NT] = t3;
  if constexpr (NCH > B + 4 * NT) stage_round<NT, NCH, B + 4 * NT>(s, d, tid);
}

template <typename T, int NT, int NCX>
__device__ __forceinline__ void stage_tw(cx<T>* __restrict__ dst, const void* __restrict__ src, int tid) {
  constexpr int NCH = NCX * (int)sizeof(cx<T>) / 16;
  static_assert(NCX * sizeof(cx<T>) % 16 == 0, "tables are whole 16-byte pieces");
  stage_round<NT, NCH, 0>(reinterpret_cast<const uint4*>(src), reinterpret_cast<uint4*>(dst), tid);
}

template <typename T, int N, int E, int SIGN, int NS, int NC, int NBUF, int SYNC, int R, int... Rest>
__device__ __forceinline__ void fft_passes(cx<T> (&v)[NC][E], cx<T>* lx, int t, const cx<T>* tw,
                                           int lds_stride) {
  constexpr bool last = sizeof...(Rest) == 0;
  fft_pass<T, N, E, R, NS, SIGN, last, NC, NBUF, SYNC>(v, lx, t, tw, lds_stride);
  if constexpr (!last) {
    fft_passes<T, N, E, SIGN, NS * R, NC, NBUF, SYNC, Rest...>(v, lx, t,
                                                              tw + (NS > 1 ? 2 * NS * (R - 1) : 0), lds_stride);
  }
}

template <typename T, int N, int E, int SIGN, int NC, int NBUF, int SYNC, int... Rs>
__device__ __forceinline__ void fft_run(RadixList<Rs...>, cx<T> (&v)[NC][E], cx<T>* lx, int t,
                                        const cx<T>* tw, int lds_stride) {
  fft_passes<T, N, E, SIGN, 1, NC, NBUF, SYNC, Rs...>(v, lx, t, tw, lds_stride);
}

// Forward (SIGN = -1) or inverse (SIGN = +1) unscaled transform of NC components.
// tw points at the table of the plan for this direction.
template <typename T, int N, int E, int SIGN, int NC, int NBUF, int SYNC>
__device__ __forceinline__ void fft_line(cx<T> (&v)[NC][E], cx<T>* lx, int t, const cx<T>* tw,
                                         int lds_stride) {
  if constexpr (SIGN < 0)
    fft_run<T, N, E, SIGN, NC, NBUF, SYNC>(typename Plan<N, E>::fwd{}, v, lx, t, tw, lds_stride);
  else
    fft_run<T, N, E, SIGN, NC, NBUF, SYNC>(typename Plan<N, E>::inv{}, v, lx, t, tw, lds_stride);
}

// ---------------------------------------------------------------------------
// Spin-2 rotation as the 4th symmetric power of U = [[alpha, beta], [-conj(beta),
// conj(alpha)]] (|alpha|^2 + |beta|^2 = 1), times a scalar `scale`, applied to x.
//
// A 5-vector x (order m = 2..-2) is the binary quartic form sum_k x_k sqrt(C(4,k))
// u^k v^(4-k), k = m + 2; U acts by u -> U11 u + U21 v, v -> U12 u + U22 v.
// With U = L D R, L = [[1, 0], [l, 1]], D = diag(a, det/a), R = [[1, r], [0, 1]]:
// R is a Taylor shift of the form in v by r, D scales u^k v^(4-k) by
// a^(2k-4) det^(4-k), and L is a Taylor shift in u by l.  The shifts run directly on
// the normalised components (coefficient ratios rho_j = sqrt(C(4,j+1)/C(4,j))...).
// When |beta| > |alpha| the factorisation runs on U P (P swaps u and v, i.e.
// reverses x) so that |l|, |r| <= 1.  The spin-1/2 matrices sigma/2 map to the
// spin-2 matrices f of Sec. 1 under this representation, so
// exp(i t n.sigma/2) -> exp(i t n.f).
//
// Inputs come in increment form: alpha = 1 + as, scale = 1 + ss.  Every update is
// x <- x + (small coefficient) * x, so a coefficient's rounding error scales with
// the coefficient and the near-identity maps of small time steps repeat no O(1)
// rounding error from step to step.
// ---------------------------------------------------------------------------
// The factorisation of U (or of U P) depends on alpha and beta only; the scalar
// factor enters only the diagonal.  sym4_prepare computes the factorisation once
// (for many vectors rotated by the same U, e.g. every kz of one (kx, ky) column),
// sym4_apply_prep applies it with a scale 1 + ss.
template <typename T>
struct Sym4Prep {
  cx<T> r, l;   // Taylor-shift coefficients of R and L
  cx<T> m[4];   // diagonal of D minus 1 at k = 0, 1, 3, 4 (at k = 2 it is 0)
  int pivot;    // 1: the factorisation of U P (the components are reversed first)
};

template <typename T>
__device__ __forceinline__ Sym4Prep<T> sym4_prepare(cx<T> as, cx<T> beta) {
  Sym4Prep<T> P;
  const cx<T> alpha = mk<T>(T(1) + as.re, as.im);
  const cx<T> one = mk<T>(T(1), T(0));
  P.pivot = norm2(beta) > norm2(alpha);
  if (!P.pivot) {
    const T q = recip(norm2(alpha));
    const cx<T> ia = mk<T>(alpha.re * q, -alpha.im * q);  // 1/alpha
    P.r = beta * ia;
    P.l = mk<T>(-beta.re, beta.im) * ia;  // -conj(beta)/alpha
    // a^2 - 1, a^4 - 1, a^-2 - 1, a^-4 - 1 from as = a - 1 without cancellation
    const cx<T> e2 = as * (mk<T>(T(2), T(0)) + as);
    const cx<T> e4 = e2 * (mk<T>(T(2), T(0)) + e2);
    const cx<T> one_e2 = one + e2;
    const T q2 = recip(norm2(one_e2));
    const cx<T> inv_e2 = mk<T>(one_e2.re * q2, -one_e2.im * q2);
    const cx<T> em2 = mk<T>(-e2.re, -e2.im) * inv_e2;
    const cx<T> em4 = em2 * (mk<T>(T(2), T(0)) + em2);
    P.m[0] = e4;
    P.m[1] = e2;
    P.m[2] = em2;
    P.m[3] = em4;
  } else {
    // U P = [[beta, alpha], [conj(alpha), -conj(beta)]], det -1
    const T q = recip(norm2(beta));
    const cx<T> ia = mk<T>(beta.re * q, -beta.im * q);  // 1/beta
    P.r = alpha * ia;
    P.l = conj(alpha) * ia;
    const cx<T> a2 = beta * beta, a4 = a2 * a2;
    const cx<T> ia2 = ia * ia, ia4 = ia2 * ia2;
    P.m[0] = a4 - one;
    P.m[1] = mk<T>(-a2.re, -a2.im) - one;
    P.m[2] = mk<T>(-ia2.re, -ia2.im) - one;
    P.m[3] = ia4 - one;
  }
  return P;
}

template <typename T>
__device__ __forceinline__ void sym4_apply_prep(const Sym4Prep<T>& P, cx<T> ss, cx<T> (&x)[5]) {
  const T rho0 = T(2), rho1 = T(1.22474487139158904909864203735294570), rho2 = T(0.81649658092772603273242802490196380),
          rho3 = T(0.5);
  if (P.pivot) {
    cx<T> t0 = x[0], t1 = x[1];
    x[0] = x[4];
    x[1] = x[3];
    x[3] = t1;
    x[4] = t0;
  }
  const cx<T> r = P.r, l = P.l;
  const cx<T> rr0 = rho0 * r, rr1 = rho1 * r, rr2 = rho2 * r, rr3 = rho3 * r;
  const cx<T> lr0 = rho0 * l, lr1 = rho1 * l, lr2 = rho2 * l, lr3 = rho3 * l;
  // R: Taylor shift, x_j += r rho_j x_(j+1), i = 0..3, j = 3..i
  x[3] = cfma(rr3, x[4], x[3]);
  x[2] = cfma(rr2, x[3], x[2]);
  x[1] = cfma(rr1, x[2], x[1]);
  x[0] = cfma(rr0, x[1], x[0]);
  x[3] = cfma(rr3, x[4], x[3]);
  x[2] = cfma(rr2, x[3], x[2]);
  x[1] = cfma(rr1, x[2], x[1]);
  x[3] = cfma(rr3, x[4], x[3]);
  x[2] = cfma(rr2, x[3], x[2]);
  x[3] = cfma(rr3, x[4], x[3]);
  // D: x_j += eps_j x_j with 1 + eps_j = (1 + m_j)(1 + ss) (m at k = 2 is 0)
  cx<T> eps[5];
  eps[0] = P.m[0] + ss + P.m[0] * ss;
  eps[1] = P.m[1] + ss + P.m[1] * ss;
  eps[2] = ss;
  eps[3] = P.m[2] + ss + P.m[2] * ss;
  eps[4] = P.m[3] + ss + P.m[3] * ss;
#pragma unroll
  for (int j = 0; j < 5; ++j) x[j] = inc_apply(eps[j], x[j]);
  // L: Taylor shift on the reversed vector, x_(4-k) += l rho_k x_(3-k)
  x[1] = cfma(lr3, x[0], x[1]);
  x[2] = cfma(lr2, x[1], x[2]);
  x[3] = cfma(lr1, x[2], x[3]);
  x[4] = cfma(lr0, x[3], x[4]);
  x[1] = cfma(lr3, x[0], x[1]);
  x[2] = cfma(lr2, x[1], x[2]);
  x[3] = cfma(lr1, x[2], x[3]);
  x[1] = cfma(lr3, x[0], x[1]);
  x[2] = cfma(lr2, x[1], x[2]);
  x[1] = cfma(lr3, x[0], x[1]);
}

template <typename T>
__device__ __forceinline__ void sym4_apply_inc(cx<T> as, cx<T> beta, cx<T> ss, cx<T> (&x)[5]) {
  sym4_apply_prep<T>(sym4_prepare<T>(as, beta), ss, x);
}

// cos(x) - 1 and sin(x)/x without cancellation or division by zero.
template <typename T>
__device__ __forceinline__ void cosm1_sinc(T x, T& cm1, T& sc) {
  const T x2 = x * x;
  const T small = sizeof(T) == 4 ? T(1e-2) : T(1e-4);
  if (fabs(x) < small) {
    sc = T(1) - x2 * (T(1) / T(6)) * (T(1) - x2 * T(0.05));
    cm1 = -x2 * T(0.5) * (T(1) - x2 * (T(1) / T(12)));
  } else {
    T s, c, sh, ch;
    if constexpr (sizeof(T) == 4) { sincosf(x, &s, &c); sincosf(T(0.5) * x, &sh, &ch); }
    else { sincos(x, &s, &c); sincos(T(0.5) * x, &sh, &ch); }
    sc = s / x;
    cm1 = T(-2) * sh * sh;
  }
}

// exp(-i phi) - 1 = (cos phi - 1) - i sin phi for an FP64 phase, both parts to full
// FP64 accuracy without cancellation and without a general-range sin/cos: phi is
// reduced mod 2 pi to r in [-pi, pi] (two-part 2 pi), q = r/4 lies in [-pi/4, pi/4],
// where the Taylor series of sin q (to q^15) and cos q (to q^16) truncate below
// 5e-17; then sin(r/2) = 2 sin q cos q gives
//   cos phi - 1 = -2 sin^2(r/2) = -8 sin^2 q cos^2 q,
//   sin phi = 2 sin(r/2) cos(r/2) = 4 sin q cos q (1 - 2 sin^2 q).
__device__ __forceinline__ void phase_inc(double phi, double& cm1, double& sn) {
  const double k = rint(phi * 0.15915494309189533576888376337251437);
  double r = fma(-k, 6.283185307179586231995926937088370323, phi);
  r = fma(-k, 2.449293598294706e-16, r);
  const double q = 0.25 * r, q2 = q * q;
  const double sq =
      q * fma(q2, fma(q2, fma(q2, fma(q2, fma(q2, fma(q2, fma(q2, -7.647163731819816475901131985788e-13,
                                                                 1.605904383682161459939237717015e-10),
                                                         -2.505210838544171877505210838544e-8),
                                                 2.755731922398589065255731922399e-6),
                                         -1.984126984126984126984126984127e-4),
                                 8.333333333333333333333333333333e-3),
                         -1.666666666666666666666666666667e-1),
              1.0);
  const double cq =
      fma(q2, fma(q2, fma(q2, fma(q2, fma(q2, fma(q2, fma(q2, fma(q2, 4.779477332387385297438207491118e-14,
                                                                 -1.147074559772972471385169797868e-11),
                                                         2.087675698786809897921009032120e-9),
                                                 -2.755731922398589065255731922399e-7),
                                         2.480158730158730158730158730159e-5),
                                 -1.388888888888888888888888888889e-3),
                         4.166666666666666666666666666667e-2),
                 -0.5),
          1.0);
  const double sc = sq * cq;
  cm1 = -8.0 * sc * sc;
  sn = 4.0 * sc * fma(-2.0 * sq, sq, 1.0);
}

// ---------------------------------------------------------------------------
// Exact nonlinear flow at one point for time d (Sec. 3.2, eq. solution2):
//   b = cos(c2 S d) psi + i (sin(c2 S d)/S) (rho/5 psi - A00 A conj(psi))
//   psi <- exp(-i d [V + (c0 + c2/5) rho]) exp(-i c1 d F.f) b
// S = sqrt(max(0, (rho/5)^2 - |A00|^2/5)).  The spin rotation exp(-i c1 d F.f) is
// sym4 of exp(-i c1 d F.sigma/2): alpha = cos(kappa/2) - i s F_z,
// beta = -i s F_-, s = sin(kappa/2)/|F| = (c1 d/2) sinc(kappa/2), kappa = c1 d |F|.
// The scalar phase is evaluated in FP64 (argument, its reduction mod 2 pi, and
// exp(-i phi) - 1) and folded into the rotation's diagonal.  Every factor enters
// in increment form (cos - 1, exp(-i phi) - 1, ...).
// ---------------------------------------------------------------------------
struct NLCoef {
  double d;      // substep duration
  double c0p;    // c0 + c2/5
  double c1, c2;
};

template <typename T>
__device__ __forceinline__ void nl_point(cx<T> (&p)[5], double V, const NLCoef& K) {
  const T r6 = T(2.44948974278317809819728407470589139);
  const T r5i = T(0.44721359549995793928183473374625524);
  const T n0 = norm2(p[0]), n1 = norm2(p[1]), n2 = norm2(p[2]), n3 = norm2(p[3]), n4 = norm2(p[4]);
  const T rho = n0 + n1 + n2 + n3 + n4;
  const T Fz = T(2) * (n0 - n4) + (n1 - n3);
  // F_+ = 2 (conj(psi2) psi1 + conj(psi-1) psi-2) + sqrt6 (conj(psi1) psi0 + conj(psi0) psi-1)
  const cx<T> Fp = T(2) * (cmulc(p[0], p[1]) + cmulc(p[3], p[4])) + r6 * (cmulc(p[1], p[2]) + cmulc(p[2], p[3]));
  // A00 = (2 psi2 psi-2 - 2 psi1 psi-1 + psi0^2)/sqrt5
  const cx<T> A00 = r5i * (T(2) * (p[0] * p[4] - p[1] * p[3]) + p[2] * p[2]);
  const T rho5 = rho * T(0.2);
  T S2 = rho5 * rho5 - norm2(A00) * T(0.2);
  S2 = S2 > T(0) ? S2 : T(0);
  const T S = sqrt_nn(S2);
  const T c2d = T(K.c2 * K.d);
  T cm1, snc;
  cosm1_sinc<T>(c2d * S, cm1, snc);
  const T snS = c2d * snc;  // sin(c2 S d) / S
  // b = psi + (cos - 1) psi + i snS (rho/5 psi - A00 (A conj psi)_i),
  // (A conj psi)_i = (-1)^i conj(psi_(4-i)) / sqrt5, i.e.
  // b_i = psi_i + k1 psi_i - k2 (-1)^i conj(psi_(4-i)) with k1 = (cos - 1) + i snS rho/5
  // and k2 = i snS A00 / sqrt5
  const cx<T> k1 = mk<T>(cm1, snS * rho5);
  const cx<T> k2 = mul_i((snS * r5i) * A00);
  cx<T> b[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    cx<T> ab = conj(p[4 - i]);
    if (i & 1) ab = mk<T>(-ab.re, -ab.im);
    b[i] = p[i] + (k1 * p[i] - k2 * ab);
  }
  // spin rotation: alpha - 1 = (cos(kappa/2) - 1) - i s F_z, beta = -i s F_-
  const T Fabs = sqrt_nn(norm2(Fp) + Fz * Fz);
  const T hc1d = T(0.5 * K.c1 * K.d);
  T ckm1, skc;
  cosm1_sinc<T>(hc1d * Fabs, ckm1, skc);
  const T s = hc1d * skc;  // sin(kappa/2)/|F|
  const cx<T> as = mk<T>(ckm1, -s * Fz);
  const cx<T> beta = mk<T>(-s * Fp.im, -s * Fp.re);
  // scalar phase exp(-i phi) - 1, phi = d [V + (c0 + c2/5) rho], in FP64
  double pcm1, psn;
  phase_inc(K.d * (V + K.c0p * (double)rho), pcm1, psn);
  const cx<T> phs = mk<T>((T)pcm1, (T)(-psn));  // exp(-i phi) - 1
  sym4_apply_inc<T>(as, beta, phs, b);
#pragma unroll
  for (int i = 0; i < 5; ++i) p[i] = b[i];
}

// ---------------------------------------------------------------------------
// Adjoint of the nonlinear flow at one point (real-linear, Wirtinger form).
// Convention: a gradient g of a real loss J with respect to psi is 2 dJ/d conj(psi),
// i.e. dJ = Re sum conj(g) dpsi.  With psi' = exp(-i phi) R b (see nl_point),
// h = exp(i phi) R^H g' and k = -i Sigma h (Sigma = sin(c2 S d)/S, C = cos(c2 S d)):
//   g = C h + (rho/5) k - A00 A conj(k) + 2 c_rho psi + 2 (c_F.f) psi + 2 conj(z) A conj(psi)
// where the scalar sensitivities collect the dependence through rho, F, A00, S^2:
//   q_phi = Im(g'^H psi') = Im(h^H b) (the map is unitary), m_a = Im(h^H f_a b),
//   M = J_r(omega)^T m (omega = c1 d F, J_r the right Jacobian of the rotation
//   exponential), q_C = Re(h^H psi), q_Sig = -Im(h^H w), q_w = Re(k^H psi)/5,
//   z_w = -k^H A conj(psi), q_S = C'(S^2) q_C + Sigma'(S^2) q_Sig,
//   c_rho = d c0' q_phi + q_w + q_S 2 rho/25, z = z_w - q_S (2/5) conj(A00), c_F = c1 d M.
// Parameter partials (added to acc): dJ/dOmega (through the rotated trap, dVdO),
// dJ/dc0, dJ/dc1, dJ/dc2.
// The forward output psi' itself is never formed (q_phi uses h and b), and w and
// A conj(psi) are recomputed from psi where needed, so that few values are live at
// once: the forward point (psi, b), the adjoint vector (g, turned into h in place)
// and scalars.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void nl_point_adj(const cx<T> (&p)[5], cx<T> (&g)[5], double V, double dVdO,
                                             const NLCoef& K, double (&acc)[4]) {
  const T r6 = T(2.44948974278317809819728407470589139);
  const T r5i = T(0.44721359549995793928183473374625524);
  const T w4[4] = {T(1), T(1.22474487139158904909864203735294570), T(1.22474487139158904909864203735294570), T(1)};
  const T ml[5] = {T(2), T(1), T(0), T(-1), T(-2)};
  const T n0 = norm2(p[0]), n1 = norm2(p[1]), n2 = norm2(p[2]), n3 = norm2(p[3]), n4 = norm2(p[4]);
  const T rho = n0 + n1 + n2 + n3 + n4;
  const T Fz = T(2) * (n0 - n4) + (n1 - n3);
  const cx<T> Fp = T(2) * (cmulc(p[0], p[1]) + cmulc(p[3], p[4])) + r6 * (cmulc(p[1], p[2]) + cmulc(p[2], p[3]));
  const cx<T> A00 = r5i * (T(2) * (p[0] * p[4] - p[1] * p[3]) + p[2] * p[2]);
  const T rho5 = rho * T(0.2);
  T S2 = rho5 * rho5 - norm2(A00) * T(0.2);
  S2 = S2 > T(0) ? S2 : T(0);
  const T S = sqrt_nn(S2);
  const T c2d = T(K.c2 * K.d);
  T cm1, snc;
  cosm1_sinc<T>(c2d * S, cm1, snc);
  const T C = T(1) + cm1;
  const T Sig = c2d * snc;
  // (A conj psi)_i = (-1)^i conj(psi_(4-i)) / sqrt5 and w_i = rho/5 psi_i - A00 (A conj psi)_i
  auto Ab = [&](int i) {
    cx<T> ab = conj(p[4 - i]);
    if (i & 1) ab = mk<T>(-ab.re, -ab.im);
    return r5i * ab;
  };
  auto wv = [&](int i) { return rho5 * p[i] - A00 * Ab(i); };
  cx<T> b[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) b[i] = p[i] + (cm1 * p[i] + Sig * mul_i(wv(i)));
  // rotation and phase (as in nl_point)
  const T Fabs = sqrt_nn(norm2(Fp) + Fz * Fz);
  const T hc1d = T(0.5 * K.c1 * K.d);
  T ckm1, skc;
  cosm1_sinc<T>(hc1d * Fabs, ckm1, skc);
  const T sr = hc1d * skc;
  const cx<T> as = mk<T>(ckm1, -sr * Fz);
  const cx<T> beta = mk<T>(-sr * Fp.im, -sr * Fp.re);
  double pcm1, psn;
  phase_inc(K.d * (V + K.c0p * (double)rho), pcm1, psn);
  const cx<T> phs = mk<T>((T)pcm1, (T)(-psn));
  // h = exp(i phi) R^H g', in place
  sym4_apply_inc<T>(conj(as), mk<T>(-beta.re, -beta.im), conj(phs), g);
  // q_phi = Im(h^H b); m_a = Im(h^H f_a b)
  double qphi = 0.0;
#pragma unroll
  for (int i = 0; i < 5; ++i) qphi += (double)g[i].re * b[i].im - (double)g[i].im * b[i].re;
  cx<T> up = mk<T>(T(0), T(0)), um = mk<T>(T(0), T(0)), uz = mk<T>(T(0), T(0));
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    up = up + (T(2) * w4[l]) * cmulc(g[l], b[l + 1]);
    um = um + (T(2) * w4[l]) * cmulc(g[l + 1], b[l]);
  }
#pragma unroll
  for (int l = 0; l < 5; ++l) uz = uz + ml[l] * cmulc(g[l], b[l]);
  const T mx = T(0.5) * (up.im + um.im);
  const T my = -T(0.5) * (up.re - um.re);
  const T mz = uz.im;
  // M = J_r(omega)^T m = m + a (omega x m) + bb (omega x (omega x m))
  const T c1d = T(K.c1 * K.d);
  const T ox = c1d * Fp.re, oy = c1d * Fp.im, oz = c1d * Fz;  // F_x = Re F_+, F_y = Im F_+
  const T th2 = ox * ox + oy * oy + oz * oz;
  T ja, jb;
  if (th2 < (sizeof(T) == 4 ? T(1e-4) : T(1e-8))) {
    ja = T(0.5) - th2 / T(24);
    jb = T(1) / T(6) - th2 / T(120);
  } else {
    const T th = sqrt(th2);
    T sth, cth;
    if constexpr (sizeof(T) == 4) sincosf(th, &sth, &cth);
    else sincos(th, &sth, &cth);
    const T hs = sizeof(T) == 4 ? sinf(T(0.5) * th) : sin(T(0.5) * th);
    ja = T(2) * hs * hs / th2;
    jb = (th - sth) / (th2 * th);
  }
  const T cx1 = oy * mz - oz * my, cy1 = oz * mx - ox * mz, cz1 = ox * my - oy * mx;
  const T cx2 = oy * cz1 - oz * cy1, cy2 = oz * cx1 - ox * cz1, cz2 = ox * cy1 - oy * cx1;
  const T Mx = mx + ja * cx1 + jb * cx2, My = my + ja * cy1 + jb * cy2, Mz = mz + ja * cz1 + jb * cz2;
  // sensitivities through b; k_i = -i Sigma h_i
  T qC = T(0), qSig = T(0), qw = T(0);
  cx<T> zw = mk<T>(T(0), T(0));
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const cx<T> k = mk<T>(Sig * g[i].im, -Sig * g[i].re);
    qC += cmulc(g[i], p[i]).re;
    qSig -= cmulc(g[i], wv(i)).im;
    qw += cmulc(k, p[i]).re;
    zw = zw - cmulc(k, Ab(i));
  }
  qw *= T(0.2);
  // Sigma'(S^2) = (c2 d C - Sigma)/(2 S^2), series -(c2 d)^3/6 (1 - x^2/10) for small x = c2 d S
  const T x2 = c2d * c2d * S2;
  const T Sigp = x2 < (sizeof(T) == 4 ? T(1e-3) : T(1e-6)) ? -(c2d * c2d * c2d) / T(6) * (T(1) - x2 / T(10))
                                                           : (c2d * C - Sig) / (T(2) * S2);
  const T Cp = -T(0.5) * c2d * Sig;
  const T qS = Cp * qC + Sigp * qSig;
  const T crho = T(K.d * K.c0p * qphi) + qw + qS * (T(2) * rho / T(25));
  const cx<T> z = zw - (T(0.4) * qS) * conj(A00);
  const T cFx = c1d * Mx, cFy = c1d * My, cFz = c1d * Mz;
  const cx<T> cpm = mk<T>(cFx, -cFy), cpp = mk<T>(cFx, cFy);  // c_Fx -/+ i c_Fy
  const cx<T> zc2 = T(2) * conj(z);
  cx<T> gn[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const cx<T> k = mk<T>(Sig * g[i].im, -Sig * g[i].re);
    cx<T> ak = mk<T>(Sig * g[4 - i].im, Sig * g[4 - i].re);  // conj(k_(4-i))
    if (i & 1) ak = mk<T>(-ak.re, -ak.im);
    cx<T> r = C * g[i] + rho5 * k - A00 * (r5i * ak) + (T(2) * crho) * p[i] + zc2 * Ab(i);
    cx<T> fpsi = (cFz * ml[i]) * p[i];
    if (i < 4) fpsi = fpsi + w4[i] * (cpm * p[i + 1]);
    if (i > 0) fpsi = fpsi + w4[i - 1] * (cpp * p[i - 1]);
    gn[i] = r + T(2) * fpsi;
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) g[i] = gn[i];
  acc[0] += K.d * dVdO * qphi;                                                  // Omega (trap)
  acc[1] += K.d * (double)rho * qphi;                                           // c0
  acc[2] += K.d * ((double)Fp.re * Mx + (double)Fp.im * My + (double)Fz * Mz);  // c1
  acc[3] += K.d * (double)rho5 * qphi + (double)(-(T)K.d * S2 * Sig) * qC + (double)((T)K.d * C) * qSig;  // c2
}

}  // namespace sgp

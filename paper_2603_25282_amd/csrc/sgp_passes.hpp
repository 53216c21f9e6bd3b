// Split-step kernels for the rotating SOC spin-2 GPE on gfx950.
//
// State layout: [nz][ny][nx][5] complex (components innermost).
//
// One linear substep of the compact splitting (Sec. 3.1) in 2D is two passes over
// the state; each pass reads and writes every value once:
//   X-pass (lines along x): inverse FFT along x, exact nonlinear flow per point
//                           (Sec. 3.2) with the trap at R(Omega s) x, forward FFT.
//   Y-pass (lines along y): forward FFT along y, exact linear propagator per
//                           wavevector (eq. sl1), inverse FFT along y.
// Between passes the state is held x-transformed (Fourier in x, physical in y).
// The first X-pass of a call starts from physical data (no inverse FFT) and the
// last one ends in physical data (no forward FFT).  3D: Y1 (forward y),
// Z (forward z, propagator, inverse z), Y2 (inverse y).
//
// Work split inside a block: W lines x 5 components; each (line, component) is
// transformed by TL = N/E threads holding E elements each (register Stockham FFT
// with LDS exchanges).  The pointwise stage (nonlinear flow or propagator) needs the
// 5 components of a point together: the block writes its lines into an LDS tile
// (components innermost), every thread updates whole points from the tile, and
// the FFT threads read their elements back.
#pragma once
#include <hip/hip_ext.h>

#include "sgp_device.hpp"
#include "sgp_kernels.hpp"

namespace sgp {

// LDS line stride of the FFT exchanges: N + N/8 (one pad slot per 8) plus a per-length
// extra that spreads the 5 component lines of adjacent lanes over the 32 banks
// (chosen with a bank-conflict model of every exchange pattern; complex values are
// interleaved, one 8- or 16-byte LDS access each).
template <int N> struct PadLine {
  static constexpr int extra = N == 512 ? 13 : N == 256 ? 13 : N == 128 ? 13 : N == 64 ? 5 : N == 384 ? 2
                             : N == 768 ? 13 : N == 192 ? 5 : N == 32 ? 9 : N == 16 ? 1 : 1;
  static constexpr int size = N + N / 8 + extra;
};

// Block index -> logical tile index so that the 8 XCDs (which take blocks round
// robin) each process one contiguous range of tiles and share their L2 lines.
__device__ __forceinline__ long xcd_tile(long b, long nblocks) {
  if (nblocks % 8) return b;
  return (b % 8) * (nblocks / 8) + b / 8;
}

// Trap rotation cos/sin(Omega s): from the host value (first pass of a call) or from
// the device clock, whose slots 1, 2 hold cos and sin of the current angle (written by
// whichever pass last moved the clock).
__device__ __forceinline__ void trap_angle(const PassArgs& a, double& c, double& s) {
  if (a.clock_mode == CLOCK_ARG) {
    sincos(a.Omega * a.s_arg, &s, &c);
  } else {
    c = a.clock[1];
    s = a.clock[2];
  }
}

// ---------------------------------------------------------------------------
// Generic pass.  KIND selects the line direction and the stages:
//   X_FIRST: load phys -> NL -> FFTx -> store       X_MID: iFFTx -> NL -> FFTx
//   X_LAST:  iFFTx -> NL -> store phys              X_NLONLY: NL only
//   C_PROP:  FFT -> propagator -> iFFT (column)     C_FWD / C_INV: FFT / iFFT only
// ---------------------------------------------------------------------------
template <int KIND> struct KindInfo {
  static constexpr bool XL = KIND == X_FIRST || KIND == X_MID || KIND == X_LAST || KIND == X_NLONLY ||
                             KIND == XA_FIRST || KIND == XA_MID || KIND == XA_LAST || KIND == X_SHEAR ||
                             KIND == X_FWD || KIND == X_INV;
  static constexpr bool SHEAR = KIND == X_SHEAR || KIND == C_SHEAR;
  static constexpr bool XADJ = KIND == XA_FIRST || KIND == XA_MID || KIND == XA_LAST;
  static constexpr bool ADJ = XADJ || KIND == C_ADJ;
  static constexpr bool PW = (XL && !SHEAR && KIND != X_FWD && KIND != X_INV) || KIND == C_PROP ||
                             KIND == C_ADJ || KIND == C_FSPIN;  // has a pointwise stage (on the LDS tile)
  // which transforms the pass runs (forward: exp(-i..), inverse: exp(+i..))
  static constexpr bool HF = KIND == X_FIRST || KIND == X_MID || KIND == XA_MID || KIND == XA_LAST ||
                             KIND == C_PROP || KIND == C_FWD || KIND == C_ADJ || SHEAR || KIND == X_FWD ||
                             KIND == C_FSPIN || KIND == C_KIN;
  static constexpr bool HI = KIND == X_MID || KIND == X_LAST || KIND == XA_FIRST || KIND == XA_MID ||
                             KIND == C_PROP || KIND == C_INV || KIND == C_ADJ || SHEAR || KIND == X_INV ||
                             KIND == C_KIN;
};

// LDS cx<T> values of the staged twiddle tables of a pass (forward table first).
template <int N, int E, int KIND>
constexpr int pass_tw() {
  return (KindInfo<KIND>::HF ? 2 * TwSize<N, E>::fwd : 0) + (KindInfo<KIND>::HI ? 2 * TwSize<N, E>::inv : 0);
}

// LDS elements (per re / im array) a pass needs.
template <int N, int W, int KIND>
constexpr int pass_lds() {
  constexpr int TILE = KindInfo<KIND>::PW ? W * N * 5 : 0;
  constexpr int XCH = W * 5 * PadLine<N>::size;
  return TILE > XCH ? TILE : XCH;
}

// Body of one block of a pass over `tile` (W lines), with caller-provided LDS.
template <typename T, int N, int E, int W, int KIND>
__device__ __forceinline__ void pass_body(cx<T>* __restrict__ psi, const PassArgs& a, long tile, cx<T>* lx,
                                          cx<T>* ltw, double (*gred)[NGRAD]) {
  constexpr int TL = N / E;
  constexpr int NT = W * 5 * TL;
  constexpr int LS = PadLine<N>::size;
  constexpr bool XL = KindInfo<KIND>::XL;
  constexpr bool XADJ = KindInfo<KIND>::XADJ;
  constexpr bool ADJ = KindInfo<KIND>::ADJ;
  constexpr bool PW = KindInfo<KIND>::PW;

  const int tid = threadIdx.x;
  const int c = tid % 5;
  const int rest = tid / 5;
  // x-lines: the TL threads of a line are adjacent (contiguous loads);
  // columns: the W columns are adjacent (W*5 contiguous values per row)
  const int col = XL ? rest / TL : rest % W;
  const int t = XL ? rest % TL : rest / W;

  // line geometry, in 32-bit element offsets (every supported state, up to
  // 512^3 points x 5 components, has fewer than 2^31 elements)
  int base;         // element offset of the line's first point (component 0)
  int estride;      // element stride between consecutive points of the line
  int line0 = 0;    // x-lines: first line of the block (line = z * ny + y)
  int o = 0, kx0 = 0;
  bool active;
  if constexpr (XL) {
    line0 = (int)tile * W;
    const int line = line0 + col;
    active = line < a.nlines;
    base = (active ? line : 0) * N * 5;
    estride = 5;
  } else {
    const int ncolblk = ((int)a.ncols + W - 1) / W;
    o = (int)tile / ncolblk;
    kx0 = ((int)tile % ncolblk) * W;
    const int kx = kx0 + col;
    active = kx < a.ncols;
    base = o * (int)a.outer_stride + (active ? kx : 0) * 5;
    estride = (int)a.stride;
  }

  cx<T> v[1][E];
#pragma unroll
  for (int m = 0; m < E; ++m)
    v[0][m] = active ? psi[base + (t + TL * m) * estride + c] : mk<T>(T(0), T(0));

  cx<T>* xl = lx + (col * 5 + c) * LS;
  // twiddle tables staged in LDS while the state loads are in flight
  constexpr int TWF = KindInfo<KIND>::HF ? 2 * TwSize<N, E>::fwd : 0;
  constexpr int TWI = KindInfo<KIND>::HI ? 2 * TwSize<N, E>::inv : 0;
  const cx<T>* twf = ltw;
  const cx<T>* twi = ltw + TWF;
  if constexpr (TWF > 0) stage_tw<T, NT, TWF>(ltw, a.tw_fwd, tid);
  if constexpr (TWI > 0) stage_tw<T, NT, TWI>(ltw + TWF, a.tw_inv, tid);

  if constexpr (KIND == X_MID || KIND == X_LAST || KIND == C_INV || KIND == XA_FIRST || KIND == XA_MID ||
                KIND == X_INV)
    fft_line<T, N, E, +1, 1, 1, 0>(v, xl, t, twi, 0);
  if constexpr (KIND == C_PROP || KIND == C_FWD || KIND == C_ADJ || KIND == X_FWD || KindInfo<KIND>::SHEAR ||
                KIND == C_FSPIN || KIND == C_KIN)
    fft_line<T, N, E, -1, 1, 1, 0>(v, xl, t, twf, 0);

  if constexpr (KIND == C_KIN) {
    // the kinetic phase along the line, per component: coefficient k times
    // exp(-i d nu_k^2/2), in increment form (table entry exp(..) - 1)
    const cx<T>* kin_l = reinterpret_cast<const cx<T>*>(a.kin_l);
#pragma unroll
    for (int m = 0; m < E; ++m) v[0][m] = inc_apply(kin_l[t + TL * m], v[0][m]);
    fft_line<T, N, E, +1, 1, 1, 0>(v, xl, t, twi, 0);
  }

  if constexpr (KindInfo<KIND>::SHEAR) {
    // f(.. + a w ..) along the line: coefficient k times exp(i nu_k a w) / N, w the
    // line's coordinate on the other in-plane axis; FP64 phase
    double w;
    if constexpr (XL) {
      const int line = (int)line0 + col;
      const int iy = a.dim == 3 ? line - (line / a.ny) * a.ny : line;
      w = -a.L[1] + iy * a.h[1];
    } else {
      w = -a.L[0] + (kx0 + col) * a.h[0];
    }
    const double nus = XL ? a.nu_scale_a : a.nu_scale_l;
    double cr = 1.0, ci = 0.0;
    if (a.cphase_on) sincos((2 - c) * a.cphase, &ci, &cr);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int k = t + TL * m;
      const int p = k < N / 2 ? k : k - N;
      double sn, cs;
      sincos(p * nus * a.shear * w, &sn, &cs);
      const double zr = (cs * cr - sn * ci) / N, zi = (cs * ci + sn * cr) / N;
      const T vr = v[0][m].re, vi = v[0][m].im;
      v[0][m] = mk<T>(T(zr) * vr - T(zi) * vi, T(zr) * vi + T(zi) * vr);
    }
    fft_line<T, N, E, +1, 1, 1, 0>(v, xl, t, twi, 0);
  }

  // forward store mode: keep the pointwise-stage input for the adjoint
  if constexpr (PW && !ADJ) {
    if (a.store != nullptr && active) {
      cx<T>* st = reinterpret_cast<cx<T>*>(a.store);
#pragma unroll
      for (int m = 0; m < E; ++m) st[base + (t + TL * m) * estride + c] = v[0][m];
    }
  }
  double gacc[NGRAD] = {0.0, 0.0, 0.0, 0.0, 0.0};

  if constexpr (PW) {
    // to the tile: point (col, j) component c at (col * N + j) * 5 + c
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int o5 = (col * N + t + TL * m) * 5 + c;
      lx[o5] = v[0][m];
    }
    __syncthreads();
    if constexpr (XL) {
      NLCoef K;
      K.d = a.d;
      K.c0p = a.c0p;
      K.c1 = a.c1;
      K.c2 = a.c2;
      double ct, st;
      trap_angle(a, ct, st);
      // (y, z) indices of the block's first line (uniform); the block's W lines follow it
      // (z from the launch's first plane a.z0 on)
      const int izl = a.dim == 3 ? line0 / a.ny : 0;
      const int iy0 = line0 - izl * a.ny;
      const int iz0 = izl + a.z0;
      for (int pt = tid; pt < W * N; pt += NT) {
        const int pc = pt / N, j = pt % N;
        const int line = (int)line0 + pc;  // y + ny z (< 2^31 for every supported grid)
        int iy = iy0 + pc, iz = iz0;
        while (iy >= a.ny) {
          iy -= a.ny;
          iz += 1;
        }
        const double x = -a.L[0] + j * a.h[0];
        const double y = -a.L[1] + iy * a.h[1];
        const double z = -a.L[2] + iz * a.h[2];
        const double X = ct * x + st * y, Y = -st * x + ct * y;
        const double V = 0.5 * (a.g2[0] * X * X + a.g2[1] * Y * Y + a.g2[2] * z * z);
        cx<T> p[5];
#pragma unroll
        for (int cc = 0; cc < 5; ++cc) p[cc] = lx[pt * 5 + cc];
        if constexpr (XADJ) {
          // forward input of this nonlinear substep at the point, from the store
          const cx<T>* fw = reinterpret_cast<const cx<T>*>(a.fwd) + (line < a.nlines ? line : 0) * N * 5 + j * 5;
          cx<T> q[5];
#pragma unroll
          for (int cc = 0; cc < 5; ++cc) q[cc] = fw[cc];
          // dV/dOmega = s (gx^2 - gy^2) X Y (trap at R(Omega s) x)
          const double dVdO = a.s_arg * (a.g2[0] - a.g2[1]) * X * Y;
          double acc4[4] = {0.0, 0.0, 0.0, 0.0};
          nl_point_adj<T>(q, p, V, dVdO, K, acc4);
          if (line < a.nlines) {
            gacc[1] += acc4[0];
            gacc[2] += acc4[1];
            gacc[3] += acc4[2];
            gacc[4] += acc4[3];
          }
        } else {
          nl_point<T>(p, V, K);
        }
#pragma unroll
        for (int cc = 0; cc < 5; ++cc) lx[pt * 5 + cc] = p[cc];
      }
    } else {
      const T* cs = reinterpret_cast<const T*>(a.cs);
      const cx<T>* kin_a = reinterpret_cast<const cx<T>*>(a.kin_a);
      const cx<T>* kin_o = reinterpret_cast<const cx<T>*>(a.kin_o);
      const cx<T>* kin_l = reinterpret_cast<const cx<T>*>(a.kin_l);
      const T Om = T(a.Omega), ga = T(a.gamma), norm = T(a.norm);
      // 1/N^d as a (hi, lo) pair: exact for powers of two, compensated otherwise
      const T norm_lo = T(a.norm - (double)norm);
      const int nxx = (int)a.ncols;
      if constexpr (KIND == C_PROP) {
        if (a.dim == 3) {
          // z-lines: the spin part of the propagator and the kinetic phase along x and
          // y belong to the column (kx, ky), the same for every kz of it; each is
          // prepared once per column and shared through LDS
          __shared__ Sym4Prep<T> cprep[W];
          __shared__ cx<T> ckin[W];
          if (tid < W) {
            const int kx = kx0 + tid < nxx ? kx0 + tid : 0;
            const int px = kx < nxx / 2 ? kx : kx - nxx;
            const int pq = (int)o < a.n_q / 2 ? (int)o : (int)o - a.n_q;
            const int qidx = kx * a.n_q + (int)o;
            const T Cm1 = cs[2 * qidx], S = cs[2 * qidx + 1];
            const cx<T> as = mk<T>(Cm1, -S * Om);
            const cx<T> beta = mk<T>(S * ga * T(px * a.nu_scale_a), -S * ga * T(pq * a.nu_scale_q));
            cprep[tid] = sym4_prepare<T>(as, beta);
            const cx<T> ka = kin_a[kx], ko = kin_o[o];
            ckin[tid] = ka + ko + ka * ko;
          }
          __syncthreads();
          for (int pt = tid; pt < W * N; pt += NT) {
            const int pc = pt / N, kl = pt % N;
            const cx<T> ka = ckin[pc], kl1 = kin_l[kl];
            const cx<T> ss = ka + kl1 + ka * kl1;  // kinetic phase - 1
            cx<T> p[5];
            if (norm_lo == T(0)) {
#pragma unroll
              for (int cc = 0; cc < 5; ++cc) p[cc] = norm * lx[pt * 5 + cc];
            } else {
#pragma unroll
              for (int cc = 0; cc < 5; ++cc)
                p[cc] = mk<T>(kmul<T>(norm, norm_lo, lx[pt * 5 + cc].re), kmul<T>(norm, norm_lo, lx[pt * 5 + cc].im));
            }
            sym4_apply_prep<T>(cprep[pc], ss, p);
#pragma unroll
            for (int cc = 0; cc < 5; ++cc) lx[pt * 5 + cc] = p[cc];
          }
        }
      }
      for (int pt = tid; pt < W * N; pt += NT) {
        if constexpr (KIND == C_PROP) {
          if (a.dim == 3) break;  // done above
        }
        const int pc = pt / N, kl = pt % N;
        const int kx = kx0 + pc < nxx ? kx0 + pc : 0;
        const int px = kx < nxx / 2 ? kx : kx - nxx;
        const T nup = T(px * a.nu_scale_a);
        int kq;
        int qidx;
        cx<T> ka = kin_a[kx];
        // table kx-major: a column block reads its entries contiguously (2D, and the
        // 3D y-lines of C_FSPIN) or one broadcast entry (3D z-lines)
        if (a.dim == 2 || KIND == C_FSPIN) {
          kq = kl;
          qidx = kx * a.n_q + kl;
        } else {
          kq = (int)o;
          qidx = kx * a.n_q + o;
          const cx<T> ko = kin_o[o];
          ka = ka + ko + ka * ko;
        }
        const int pq = kq < a.n_q / 2 ? kq : kq - a.n_q;
        const T nuq = T(pq * a.nu_scale_q);
        const T Cm1 = cs[2 * qidx], S = cs[2 * qidx + 1];
        // alpha - 1 = (C - 1) - i S Omega; beta = i S gamma a = S gamma (nu_p - i nu_q)
        const cx<T> as = mk<T>(Cm1, -S * Om);
        const cx<T> beta = mk<T>(S * ga * nup, -S * ga * nuq);
        const cx<T> kl1 = kin_l[kl];
        const cx<T> ss = ka + kl1 + ka * kl1;  // kinetic phase - 1
        cx<T> p[5];
        if (norm_lo == T(0)) {
#pragma unroll
          for (int cc = 0; cc < 5; ++cc) p[cc] = norm * lx[pt * 5 + cc];
        } else {
#pragma unroll
          for (int cc = 0; cc < 5; ++cc)
            p[cc] = mk<T>(kmul<T>(norm, norm_lo, lx[pt * 5 + cc].re), kmul<T>(norm, norm_lo, lx[pt * 5 + cc].im));
        }
        if constexpr (KIND == C_ADJ) {
          // P^H = P(-d): same (C - 1), S -> -S, conjugate kinetic phase
          sym4_apply_inc<T>(conj(as), mk<T>(-beta.re, -beta.im), conj(ss), p);
          if (kx0 + pc < a.ncols) {
            // m_a = -d Im(L^H f_a H), L = P^H L'/N^d (p), H the stored forward input
            const cx<T>* fw = reinterpret_cast<const cx<T>*>(a.fwd) + o * (int)a.outer_stride + kx * 5 + kl * (int)a.stride;
            const double w4[4] = {1.0, 1.22474487139158904909864203735294570, 1.22474487139158904909864203735294570, 1.0};
            double upr = 0, upi = 0, umr = 0, umi = 0, uzi = 0;
            cx<T> hq[5];
#pragma unroll
            for (int cc = 0; cc < 5; ++cc) hq[cc] = fw[cc];
#pragma unroll
            for (int l = 0; l < 4; ++l) {
              const cx<T> a1 = cmulc(p[l], hq[l + 1]), a2 = cmulc(p[l + 1], hq[l]);
              upr += 2.0 * w4[l] * a1.re; upi += 2.0 * w4[l] * a1.im;
              umr += 2.0 * w4[l] * a2.re; umi += 2.0 * w4[l] * a2.im;
            }
#pragma unroll
            for (int l = 0; l < 5; ++l) uzi += (2 - l) * (double)cmulc(p[l], hq[l]).im;
            const double dd = a.d;
            const double mx = -dd * 0.5 * (upi + umi);
            const double my = dd * 0.5 * (upr - umr);
            const double mz = -dd * uzi;
            // dJ/dn = J_r(-d n)^T m, n = (gamma Re a, -gamma Im a, -Omega), a = -nu_q - i nu_p
            const double nupd = px * a.nu_scale_a, nuqd = pq * a.nu_scale_q;
            const double ox = -dd * a.gamma * (-nuqd), oy = -dd * (-a.gamma) * (-nupd), oz = -dd * (-a.Omega);
            const double th2 = ox * ox + oy * oy + oz * oz;
            double ja, jb;
            if (th2 < 1e-8) { ja = 0.5 - th2 / 24.0; jb = 1.0 / 6.0 - th2 / 120.0; }
            else {
              const double th = sqrt(th2), hs = sin(0.5 * th);
              ja = 2.0 * hs * hs / th2;
              jb = (th - sin(th)) / (th2 * th);
            }
            const double cx1 = oy * mz - oz * my, cy1 = oz * mx - ox * mz, cz1 = ox * my - oy * mx;
            const double cx2 = oy * cz1 - oz * cy1, cy2 = oz * cx1 - ox * cz1, cz2 = ox * cy1 - oy * cx1;
            const double Dx = mx + ja * cx1 + jb * cx2, Dy = my + ja * cy1 + jb * cy2, Dz = mz + ja * cz1 + jb * cz2;
            gacc[0] += -nuqd * Dx + nupd * Dy;  // dn/dgamma = (Re a, -Im a, 0) = (-nu_q, nu_p, 0)
            gacc[1] += -Dz;                     // dn/dOmega = (0, 0, -1)
          }
        } else {
          sym4_apply_inc<T>(as, beta, ss, p);
        }
#pragma unroll
        for (int cc = 0; cc < 5; ++cc) lx[pt * 5 + cc] = p[cc];
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int o5 = (col * N + t + TL * m) * 5 + c;
      v[0][m] = lx[o5];
    }
    __syncthreads();
  }

  if constexpr (KIND == X_FIRST || KIND == X_MID || KIND == XA_MID || KIND == XA_LAST)
    fft_line<T, N, E, -1, 1, 1, 0>(v, xl, t, twf, 0);
  if constexpr (KIND == C_PROP || KIND == C_ADJ) fft_line<T, N, E, +1, 1, 1, 0>(v, xl, t, twi, 0);

  if constexpr (ADJ) {
    // parameter partials: block reduction in a fixed order into this block's slot
#pragma unroll
    for (int q = 0; q < NGRAD; ++q) {
      double vq = gacc[q];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) vq += __shfl_down(vq, off, 64);
      if ((tid & 63) == 0) gred[tid >> 6][q] = vq;
    }
    __syncthreads();
    if (tid < NGRAD) {
      double sum = 0.0;
      for (int wv = 0; wv < (NT + 63) / 64; ++wv) sum += gred[wv][tid];
      a.gacc[(long)tile * NGRAD + tid] += sum;  // one slot per tile of the instance
    }
  }

  if (active) {
#pragma unroll
    for (int m = 0; m < E; ++m) psi[base + (t + TL * m) * estride + c] = v[0][m];
  }
  if constexpr (XL && !ADJ && PW) {
    if (a.clock_mode == CLOCK_ARG && tile == 0 && tid == 0) {
      a.clock[0] = a.s_arg;
      double sn, cn;
      sincos(a.Omega * a.s_arg, &sn, &cn);
      a.clock[1] = cn;
      a.clock[2] = sn;
    }
  }
  if constexpr (KIND == C_PROP || KIND == C_FSPIN) {
    if (a.advance_clock && tile == 0 && tid == 0) {
      const double s1 = a.clock[0] + a.d;
      double sn, cn;
      sincos(a.Omega * s1, &sn, &cn);
      a.clock[0] = s1;
      a.clock[1] = cn;
      a.clock[2] = sn;
    }
  }
}

template <typename T, int N, int E, int W, int KIND>
__global__ __launch_bounds__(W * 5 * (N / E)) void k_pass(cx<T>* __restrict__ psi, PassArgs a) {
  constexpr int BUF = pass_lds<N, W, KIND>();
  constexpr int NT = W * 5 * (N / E);
  constexpr int TWB = (pass_tw<N, E, KIND>() * (int)sizeof(cx<T>) + 15) / 16;
  __shared__ cx<T> lx[BUF];
  __shared__ uint4 ltw[TWB > 0 ? TWB : 1];
  __shared__ double gred[KindInfo<KIND>::ADJ ? NT / 64 + 1 : 1][NGRAD];
  pass_body<T, N, E, W, KIND>(psi, a, xcd_tile(blockIdx.x, gridDim.x), lx, reinterpret_cast<cx<T>*>(ltw),
                              gred);
}

// ---------------------------------------------------------------------------
// Batched pass over many grids (an ensemble): block b processes work item
// items[b] = (instance, tile) with that instance's arguments.  One kernel per plan
// width E; every line length it serves runs with 320 threads per block (W = 64 E / N
// lines), the geometry of the single-grid kernel of the same plan, so an instance
// gives bitwise the same result alone or inside an ensemble.
// ---------------------------------------------------------------------------
template <int N, int E, int KIND, int ES>
constexpr int batched_lds() {
  if constexpr (batched_plan_ok(N, E, ES)) return pass_lds<N, lines_per_block(N, E), KIND>();
  else return 0;
}
template <int N, int E, int KIND, int ES>
constexpr int batched_tw() {
  if constexpr (batched_plan_ok(N, E, ES)) return pass_tw<N, E, KIND>();
  else return 0;
}
constexpr int cmax(int a, int b) { return a > b ? a : b; }

// NMAX: the longest line the kernel serves (512, or 768 for the E = 12 / 24 plans);
// its static LDS is sized for lines up to NMAX only, so instances of the common
// sizes keep the occupancy they have without 768-point lines in the ensemble.
template <typename T, int KIND, int E, int NMAX>
__global__ __launch_bounds__(320) void k_pass_batched(const int2* __restrict__ items, const PassArgs* __restrict__ args) {
  constexpr int ES = (int)sizeof(T);
  constexpr int BUF = cmax(cmax(cmax(cmax(batched_lds<64, E, KIND, ES>(), batched_lds<128, E, KIND, ES>()),
                                     cmax(batched_lds<256, E, KIND, ES>(), batched_lds<384, E, KIND, ES>())),
                                cmax(batched_lds<512, E, KIND, ES>(), batched_lds<192, E, KIND, ES>())),
                           NMAX >= 768 ? batched_lds<768, E, KIND, ES>() : 0);
  constexpr int TWM = cmax(cmax(cmax(cmax(batched_tw<64, E, KIND, ES>(), batched_tw<128, E, KIND, ES>()),
                                     cmax(batched_tw<256, E, KIND, ES>(), batched_tw<384, E, KIND, ES>())),
                                cmax(batched_tw<512, E, KIND, ES>(), batched_tw<192, E, KIND, ES>())),
                           NMAX >= 768 ? batched_tw<768, E, KIND, ES>() : 0);
  constexpr int TWB = (TWM * (int)sizeof(cx<T>) + 15) / 16;
  __shared__ cx<T> lx[BUF > 0 ? BUF : 1];
  __shared__ uint4 ltwr[TWB > 0 ? TWB : 1];
  cx<T>* ltw = reinterpret_cast<cx<T>*>(ltwr);
  __shared__ double gred[KindInfo<KIND>::ADJ ? 6 : 1][NGRAD];
  const int2 it = items[blockIdx.x];
  const PassArgs& a = args[it.x];
  cx<T>* psi = reinterpret_cast<cx<T>*>(a.state);
#define SGP_BCASE(NN)                                                                                  \
  case NN:                                                                                             \
    if constexpr (NN <= NMAX && batched_plan_ok(NN, E, ES))                                            \
      pass_body<T, NN, E, lines_per_block(NN, E), KIND>(psi, a, it.y, lx, ltw, gred);                   \
    break;
  switch (a.n_line) {
    SGP_BCASE(64) SGP_BCASE(128) SGP_BCASE(192) SGP_BCASE(256) SGP_BCASE(384) SGP_BCASE(512) SGP_BCASE(768)
    default: break;
  }
#undef SGP_BCASE
}

// ---------------------------------------------------------------------------
// Propagator table, FP64: Q = n.f with n = (gamma Re a, -gamma Im a, -Omega), so
// exp(i d Q) is the spin-2 image of exp(i d n.sigma/2) = C + i S n.sigma with
// C = cos(lam d/2), S = sin(lam d/2)/lam, lam = |n| = sqrt(Omega^2 + gamma^2
// (nu_p^2 + nu_q^2)).  Stored per (p, q), rounded to T: (C - 1, S), with
// C - 1 = -2 sin^2(lam d/4), at entry kx * ny + ky (kx-major, the order the
// last-axis pass reads it in).  Kinetic tables per axis: exp(-i d nu^2/2) - 1.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_build_cs(T* __restrict__ cs, int nx, int ny, double Lx, double Ly, double Omega, double gamma,
                           double d) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)nx * ny) return;
  const int kx = (int)(i / ny), ky = (int)(i % ny);
  const int p = kx < nx / 2 ? kx : kx - nx;
  const int q = ky < ny / 2 ? ky : ky - ny;
  const double pi = 3.14159265358979323846264338327950288;
  const double nup = pi * p / Lx, nuq = pi * q / Ly;
  const double lam = sqrt(Omega * Omega + gamma * gamma * (nup * nup + nuq * nuq));
  double Cm1, S;
  if (lam == 0.0) {
    Cm1 = 0.0;
    S = 0.5 * d;
  } else {
    const double s4 = sin(0.25 * lam * d);
    Cm1 = -2.0 * s4 * s4;
    S = sin(0.5 * lam * d) / lam;
  }
  cs[2 * i] = (T)Cm1;
  cs[2 * i + 1] = (T)S;
}

template <typename T>
__global__ void k_build_kin(cx<T>* __restrict__ kin, int n, double L, double d) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int p = k < n / 2 ? k : k - n;
  const double nu = 3.14159265358979323846264338327950288 * p / L;
  const double ph = -0.5 * d * nu * nu;
  const double sh = sin(0.5 * ph);
  kin[k].re = (T)(-2.0 * sh * sh);
  kin[k].im = (T)sin(ph);
}


// ---------------------------------------------------------------------------
// Launch geometry of a register plan (N, E): TL = N/E threads per line and
// component; W lines per block so that a block has 320 threads (W = 64/TL), or one
// line of 5 TL threads when TL > 64.  Every instantiation of a plan (alone or in
// an ensemble) uses this geometry, so its results do not depend on the caller.
// ---------------------------------------------------------------------------
template <int N, int E>
struct Geo {
  static constexpr int TL = N / E;
  static constexpr int W = TL >= 64 ? 1 : 64 / TL;
  static constexpr int NT = W * 5 * TL;
};

// ev: null, or two events that the dispatch itself stamps with the kernel's start
// and end (timing without marker packets between the kernels).
template <typename T, int N, int E, int KIND>
static hipError_t pass_n(cx<T>* psi, const PassArgs& a, hipStream_t st, const hipEvent_t* ev) {
  constexpr int W = Geo<N, E>::W;
  constexpr bool XL = KindInfo<KIND>::XL;
  long nblocks = XL ? (a.nlines + W - 1) / W : ((a.ncols + W - 1) / W) * a.nouter;
  if (ev)
    hipExtLaunchKernelGGL((k_pass<T, N, E, W, KIND>), dim3((unsigned)nblocks), dim3(Geo<N, E>::NT), 0, st, ev[0],
                          ev[1], 0, psi, a);
  else
    hipLaunchKernelGGL((k_pass<T, N, E, W, KIND>), dim3((unsigned)nblocks), dim3(Geo<N, E>::NT), 0, st, psi, a);
  return hipGetLastError();
}

template <typename T, int N, int E>
static hipError_t pass_kind(int kind, cx<T>* psi, const PassArgs& a, hipStream_t st, const hipEvent_t* ev) {
  switch (kind) {
    case X_FIRST: return pass_n<T, N, E, X_FIRST>(psi, a, st, ev);
    case X_MID: return pass_n<T, N, E, X_MID>(psi, a, st, ev);
    case X_LAST: return pass_n<T, N, E, X_LAST>(psi, a, st, ev);
    case X_NLONLY: return pass_n<T, N, E, X_NLONLY>(psi, a, st, ev);
    case C_PROP: return pass_n<T, N, E, C_PROP>(psi, a, st, ev);
    case C_FWD: return pass_n<T, N, E, C_FWD>(psi, a, st, ev);
    case C_INV: return pass_n<T, N, E, C_INV>(psi, a, st, ev);
    case XA_FIRST: return pass_n<T, N, E, XA_FIRST>(psi, a, st, ev);
    case XA_MID: return pass_n<T, N, E, XA_MID>(psi, a, st, ev);
    case XA_LAST: return pass_n<T, N, E, XA_LAST>(psi, a, st, ev);
    case C_ADJ: return pass_n<T, N, E, C_ADJ>(psi, a, st, ev);
    case X_SHEAR: return pass_n<T, N, E, X_SHEAR>(psi, a, st, ev);
    case C_SHEAR: return pass_n<T, N, E, C_SHEAR>(psi, a, st, ev);
    case X_FWD: return pass_n<T, N, E, X_FWD>(psi, a, st, ev);
    case X_INV: return pass_n<T, N, E, X_INV>(psi, a, st, ev);
    case C_FSPIN: return pass_n<T, N, E, C_FSPIN>(psi, a, st, ev);
    case C_KIN: return pass_n<T, N, E, C_KIN>(psi, a, st, ev);
    default: return hipErrorInvalidValue;
  }
}

// All pass kernels of one register-plan width E (every supported
// line length with that E).  Each (T, E) pair is compiled in its own translation
// unit.
#define SGP_FOR_PLAN_N(E, X)                                     \
  X(16, E) X(32, E) X(64, E) X(128, E) X(192, E) X(256, E) X(384, E) X(512, E) X(768, E)

template <typename T, int E>
hipError_t launch_pass_e(int kind, void* psi, const PassArgs& a, int n, hipStream_t st, const hipEvent_t* ev) {
  cx<T>* p = reinterpret_cast<cx<T>*>(psi);
#define SGP_CASE(NN, EE) \
  case NN:               \
    if constexpr (plan_ok(NN, EE, (int)sizeof(T))) return pass_kind<T, NN, EE>(kind, p, a, st, ev); \
    break;
  switch (n) { SGP_FOR_PLAN_N(E, SGP_CASE) default: break; }
#undef SGP_CASE
  return hipErrorInvalidValue;
}

// Batched passes of one plan width (compiled with that width's unit).
template <typename T, int E, int NMAX>
static hipError_t launch_batched_nmax(int kind, const int2* it, const PassArgs* ar, long nitems, hipStream_t st) {
  dim3 g((unsigned)nitems), b(320);
  switch (kind) {
    case X_FIRST: hipLaunchKernelGGL((k_pass_batched<T, X_FIRST, E, NMAX>), g, b, 0, st, it, ar); break;
    case X_MID: hipLaunchKernelGGL((k_pass_batched<T, X_MID, E, NMAX>), g, b, 0, st, it, ar); break;
    case X_LAST: hipLaunchKernelGGL((k_pass_batched<T, X_LAST, E, NMAX>), g, b, 0, st, it, ar); break;
    case C_PROP: hipLaunchKernelGGL((k_pass_batched<T, C_PROP, E, NMAX>), g, b, 0, st, it, ar); break;
    case XA_FIRST: hipLaunchKernelGGL((k_pass_batched<T, XA_FIRST, E, NMAX>), g, b, 0, st, it, ar); break;
    case XA_MID: hipLaunchKernelGGL((k_pass_batched<T, XA_MID, E, NMAX>), g, b, 0, st, it, ar); break;
    case XA_LAST: hipLaunchKernelGGL((k_pass_batched<T, XA_LAST, E, NMAX>), g, b, 0, st, it, ar); break;
    case C_ADJ: hipLaunchKernelGGL((k_pass_batched<T, C_ADJ, E, NMAX>), g, b, 0, st, it, ar); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// nmax: the longest line among the launch's instances
template <typename T, int E>
hipError_t launch_batched_e(int kind, const int2* it, const PassArgs* ar, long nitems, int nmax, hipStream_t st) {
  if constexpr (E == 12 || E == 24) {
    if (nmax > 512) return launch_batched_nmax<T, E, 768>(kind, it, ar, nitems, st);
  }
  if (nmax > 512) return hipErrorInvalidValue;
  return launch_batched_nmax<T, E, 512>(kind, it, ar, nitems, st);
}

}  // namespace sgp

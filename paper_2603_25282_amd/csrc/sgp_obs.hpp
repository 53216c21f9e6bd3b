// Observables and diagnostics kernels (Sec. 2) and their per-plan launchers, in a
// header of their own: the pass kernels of sgp_passes.hpp do not depend on it.
#pragma once
#include "sgp_passes.hpp"

namespace sgp {

// ---------------------------------------------------------------------------
// Observables (Sec. 2) on the physical state, FP64 partial sums per block.
// OBS_X (lines along x): d_x psi spectrally; per point the mass, the
//   magnetization, V|psi|^2, the interaction energy, |d_x psi|^2/2,
//   Re(conj(psi) i y d_x psi) (the y d_x part of -i(x d_y - y d_x)) and
//   Re(psi^H K d_x psi); the moments X^2 rho, Y^2 rho, z^2 rho, X Y rho at the
//   rotated point (X, Y) = R(Omega s) (x, y) (the lab-frame coordinates of the
//   point, Sec. 2, eq. ConWid) and 2 x Im(conj(psi) d_x psi);
// OBS_Y / OBS_Z (columns): d_y psi (or d_z psi); |d psi|^2/2,
//   Re(conj(psi) (-i x) d_y psi), Re(i psi^H M d_y psi) and 2 y Im(conj(psi) d_y psi)
//   (y only).
// With L+- = i d_y +- d_x the SOC matrix is S = i d_y M + d_x K, M symmetric with
// the weights (1, sqrt6/2, sqrt6/2, 1) on both off-diagonals, K = -M above and +M
// below the diagonal.
// ---------------------------------------------------------------------------
// OBS_JX / OBS_JY: with u = a.fwd (same layout), the parts of <u, J_z v>, v = psi,
// J_z = L_z + F_z, L_z = -i (x d_y - y d_x): sums of conj(u) (i y d_x + F_z) v along
// x-lines and of conj(u) (-i x d_y) v along y-columns, real and imaginary parts in
// slots 0 and 1.
template <typename T, int N, int E, int W, int KIND>
__global__ __launch_bounds__(W * 5 * (N / E)) void k_obs(const cx<T>* __restrict__ psi, PassArgs a,
                                                         double* __restrict__ part) {
  constexpr int TL = N / E;
  constexpr int NT = W * 5 * TL;
  constexpr int LS = PadLine<N>::size;
  constexpr bool XL = KIND == OBS_X || KIND == OBS_JX;
  constexpr bool JZ = KIND == OBS_JX || KIND == OBS_JY;
  constexpr int TILE = 2 * W * N * 5;
  constexpr int XCH = W * 5 * LS;
  constexpr int BUF = TILE > XCH ? TILE : XCH;
  __shared__ cx<T> lx[BUF];
  __shared__ double red[NT / 64 + 1][NOBS];

  const int tid = threadIdx.x;
  const int c = tid % 5;
  const int rest = tid / 5;
  const int col = XL ? rest / TL : rest % W;
  const int t = XL ? rest % TL : rest / W;
  const long tile = blockIdx.x;
  long base, estride, line0 = 0, o = 0, kx0 = 0;
  bool active;
  if constexpr (XL) {
    line0 = tile * W;
    const long line = line0 + col;
    active = line < a.nlines;
    base = (active ? line : 0) * (long)N * 5;
    estride = 5;
  } else {
    const long ncolblk = (a.ncols + W - 1) / W;
    o = tile / ncolblk;
    kx0 = (tile % ncolblk) * W;
    const long kx = kx0 + col;
    active = kx < a.ncols;
    base = o * a.outer_stride + (active ? kx : 0) * 5;
    estride = a.stride;
  }
  cx<T> v[1][E], f[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    v[0][m] = active ? psi[base + (long)(t + TL * m) * estride + c] : mk<T>(T(0), T(0));
    f[m] = v[0][m];
  }
  cx<T>* xl = lx + (col * 5 + c) * LS;
  // derivative along the line: FFT, multiply by i nu / N, inverse FFT
  fft_line<T, N, E, -1, 1, 1, 0>(v, xl, t, reinterpret_cast<const cx<T>*>(a.tw_fwd), 0);
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int k = t + TL * m;
    const int p = k < N / 2 ? k : k - N;
    const T nu = T(p * a.nu_scale_l / N);
    v[0][m] = mk<T>(-nu * v[0][m].im, nu * v[0][m].re);
  }
  fft_line<T, N, E, +1, 1, 1, 0>(v, xl, t, reinterpret_cast<const cx<T>*>(a.tw_inv), 0);
  // tile: psi at [0, W N 5), derivative at [W N 5, 2 W N 5)
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int o5 = (col * N + t + TL * m) * 5 + c;
    lx[o5] = f[m];
    lx[W * N * 5 + o5] = v[0][m];
  }
  __syncthreads();
  double acc[NOBS];
#pragma unroll
  for (int q = 0; q < NOBS; ++q) acc[q] = 0.0;
  const double h6 = 1.22474487139158904909864203735294570;
  const double w[4] = {1.0, h6, h6, 1.0};  // weights of the links (l, l-1), l = 2..-1
  double ct = 1.0, st = 0.0;
  if constexpr (XL) sincos(a.Omega * a.s_arg, &st, &ct);
  for (int pt = tid; pt < W * N; pt += NT) {
    const int pc = pt / N, j = pt % N;
    bool on;
    double x, y, z;
    if constexpr (XL) {
      const long line = line0 + pc;
      on = line < a.nlines;
      const int iy = (int)(line % a.ny), iz = (int)(line / a.ny);
      x = -a.L[0] + j * a.h[0];
      y = -a.L[1] + iy * a.h[1];
      z = -a.L[2] + iz * a.h[2];
    } else {
      on = kx0 + pc < a.ncols;
      x = -a.L[0] + (kx0 + pc) * a.h[0];
      y = (KIND == OBS_Y || KIND == OBS_JY) ? -a.L[1] + j * a.h[1] : 0.0;
      z = 0.0;
    }
    if (!on) continue;
    if constexpr (JZ) {
      // u at this point (global memory), v and its derivative from the tile
      const cx<T>* u = reinterpret_cast<const cx<T>*>(a.fwd);
      long ub;
      if constexpr (XL) ub = (line0 + pc) * (long)N * 5 + (long)j * 5;
      else ub = o * a.outer_stride + (kx0 + pc) * 5 + (long)j * a.stride;
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int cc = 0; cc < 5; ++cc) {
        const double ur = u[ub + cc].re, ui = u[ub + cc].im;
        const double vr = lx[pt * 5 + cc].re, vi = lx[pt * 5 + cc].im;
        const double dr = lx[W * N * 5 + pt * 5 + cc].re, di = lx[W * N * 5 + pt * 5 + cc].im;
        // (J v) at the point: x-lines i y d_x v + m v (m = 2 - cc), columns -i x d_y v
        double jr, ji;
        if constexpr (XL) {
          jr = -y * di + (2 - cc) * vr;
          ji = y * dr + (2 - cc) * vi;
        } else {
          jr = x * di;
          ji = -x * dr;
        }
        sr += ur * jr + ui * ji;  // conj(u) (J v)
        si += ur * ji - ui * jr;
      }
      acc[0] += sr;
      acc[1] += si;
      continue;
    }
    double pr[5], pi[5], dr[5], di[5];
#pragma unroll
    for (int cc = 0; cc < 5; ++cc) {
      pr[cc] = lx[pt * 5 + cc].re;
      pi[cc] = lx[pt * 5 + cc].im;
      dr[cc] = lx[W * N * 5 + pt * 5 + cc].re;
      di[cc] = lx[W * N * 5 + pt * 5 + cc].im;
    }
    double grad2 = 0.0, rot = 0.0, rotm = 0.0;
#pragma unroll
    for (int cc = 0; cc < 5; ++cc) {
      grad2 += dr[cc] * dr[cc] + di[cc] * di[cc];
      const double r1 = pr[cc] * di[cc] - pi[cc] * dr[cc];  // Im(conj(psi) d psi)
      rot += r1;
      rotm += (2 - cc) * r1;  // weighted by m = 2 - cc (the F_z L_z density)
    }
    if constexpr (XL) {
      double n[5], rho = 0.0;
#pragma unroll
      for (int cc = 0; cc < 5; ++cc) { n[cc] = pr[cc] * pr[cc] + pi[cc] * pi[cc]; rho += n[cc]; }
      const double mg = 2.0 * (n[0] - n[4]) + (n[1] - n[3]);
      const double X = ct * x + st * y, Y = -st * x + ct * y;
      const double V = 0.5 * (a.g2[0] * X * X + a.g2[1] * Y * Y + a.g2[2] * z * z);
      // F_+ = 2 (conj(p2) p1 + conj(p-1) p-2) + sqrt6 (conj(p1) p0 + conj(p0) p-1)
      double fr = 0.0, fi = 0.0;
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        fr += 2.0 * w[l] * (pr[l] * pr[l + 1] + pi[l] * pi[l + 1]);
        fi += 2.0 * w[l] * (pr[l] * pi[l + 1] - pi[l] * pr[l + 1]);
      }
      // A00 = (2 p2 p-2 - 2 p1 p-1 + p0^2)/sqrt5
      const double ar = (2.0 * (pr[0] * pr[4] - pi[0] * pi[4]) - 2.0 * (pr[1] * pr[3] - pi[1] * pi[3]) +
                         (pr[2] * pr[2] - pi[2] * pi[2])) * 0.44721359549995793928;
      const double ai = (2.0 * (pr[0] * pi[4] + pi[0] * pr[4]) - 2.0 * (pr[1] * pi[3] + pi[1] * pr[3]) +
                         2.0 * pr[2] * pi[2]) * 0.44721359549995793928;
      const double eint = 0.5 * a.c0 * rho * rho + 0.5 * a.c1 * (fr * fr + fi * fi + mg * mg) +
                          0.5 * a.c2 * (ar * ar + ai * ai);
      // Re psi^H K d_x psi: -w conj(p_l) d p_(l+1) + w conj(p_(l+1)) d p_l
      double soc = 0.0;
#pragma unroll
      for (int l = 0; l < 4; ++l)
        soc += w[l] * (-(pr[l] * dr[l + 1] + pi[l] * di[l + 1]) + (pr[l + 1] * dr[l] + pi[l + 1] * di[l]));
      acc[0] += rho;
      acc[1] += mg;
      acc[2] += V * rho;
      acc[3] += eint;
      acc[4] += 0.5 * grad2;
      acc[5] += -y * rot;  // Re(conj(psi) (i y) d_x psi)
      acc[6] += soc;
      acc[7] += X * X * rho;
      acc[8] += Y * Y * rho;
      acc[9] += z * z * rho;
      acc[10] += X * Y * rho;
      acc[11] += 2.0 * x * rot;
      // conj(psi_a) d_x psi_b for the component pairs (a, b) = (2, 1), (-1, -2),
      // (1, 0), (-1, 0) (indices 0..4 = l 2..-2) of the spin-orbit laws
      acc[12] += pr[0] * dr[1] + pi[0] * di[1];
      acc[13] += pr[0] * di[1] - pi[0] * dr[1];
      acc[14] += pr[3] * dr[4] + pi[3] * di[4];
      acc[15] += pr[3] * di[4] - pi[3] * dr[4];
      acc[16] += pr[1] * dr[2] + pi[1] * di[2];
      acc[17] += pr[1] * di[2] - pi[1] * dr[2];
      acc[18] += pr[3] * dr[2] + pi[3] * di[2];
      acc[19] += pr[3] * di[2] - pi[3] * dr[2];
      // Lemma 2's spin-orbit term: (i Y - X) F_+ at the lab-frame point (real and
      // imaginary parts), (f_x^2 + f_y^2) = 6 - m^2 weighted density, and the x-line
      // part Re(conj(psi_m) i y d_x psi_m) of sum_m m conj(psi_m) L_z psi_m
      acc[20] += -X * fr - Y * fi;
      acc[21] += Y * fr - X * fi;
      acc[22] += 2.0 * n[0] + 5.0 * n[1] + 6.0 * n[2] + 5.0 * n[3] + 2.0 * n[4];
      acc[23] += -y * rotm;
    } else {
      acc[4] += 0.5 * grad2;
      if constexpr (KIND == OBS_Y) {
        acc[5] += x * rot;  // Re(conj(psi) (-i x) d_y psi)
        // Re(i psi^H M d_y psi) = -Im(psi^H M d_y psi)
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < 4; ++l)
          s += w[l] * ((pr[l] * di[l + 1] - pi[l] * dr[l + 1]) + (pr[l + 1] * di[l] - pi[l + 1] * dr[l]));
        acc[6] += -s;
        acc[11] += 2.0 * y * rot;
        acc[12] += x * rotm;  // Re(conj(psi_m) (-i x) d_y psi_m), weighted by m
        // conj(psi_a) d_y psi_b for the same pairs
        acc[20] += pr[0] * dr[1] + pi[0] * di[1];
        acc[21] += pr[0] * di[1] - pi[0] * dr[1];
        acc[22] += pr[3] * dr[4] + pi[3] * di[4];
        acc[23] += pr[3] * di[4] - pi[3] * dr[4];
        acc[24] += pr[1] * dr[2] + pi[1] * di[2];
        acc[25] += pr[1] * di[2] - pi[1] * dr[2];
        acc[26] += pr[3] * dr[2] + pi[3] * di[2];
        acc[27] += pr[3] * di[2] - pi[3] * dr[2];
      }
    }
  }
  // block reduction in a fixed order
#pragma unroll
  for (int q = 0; q < NOBS; ++q) {
    double vq = acc[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) vq += __shfl_down(vq, off, 64);
    if ((tid & 63) == 0) red[tid >> 6][q] = vq;
  }
  __syncthreads();
  if (tid < NOBS) {
    double s = 0.0;
    for (int wv = 0; wv < (NT + 63) / 64; ++wv) s += red[wv][tid];
    part[(long)blockIdx.x * NOBS + tid] = s;
  }
}

template <typename T, int N, int E, int KIND>
static hipError_t obs_n(const cx<T>* psi, const PassArgs& a, double* part, hipStream_t st) {
  constexpr int W = obs_lines_per_block(N, E);
  constexpr bool XL = KIND == OBS_X || KIND == OBS_JX;
  long nblocks = XL ? (a.nlines + W - 1) / W : ((a.ncols + W - 1) / W) * a.nouter;
  hipLaunchKernelGGL((k_obs<T, N, E, W, KIND>), dim3((unsigned)nblocks), dim3(W * 5 * (N / E)), 0, st, psi, a,
                     part);
  return hipGetLastError();
}

template <typename T, int N, int E>
static hipError_t obs_kind(int kind, const cx<T>* psi, const PassArgs& a, double* part, hipStream_t st) {
  switch (kind) {
    case OBS_X: return obs_n<T, N, E, OBS_X>(psi, a, part, st);
    case OBS_Y: return obs_n<T, N, E, OBS_Y>(psi, a, part, st);
    case OBS_Z: return obs_n<T, N, E, OBS_Z>(psi, a, part, st);
    case OBS_JX: return obs_n<T, N, E, OBS_JX>(psi, a, part, st);
    case OBS_JY: return obs_n<T, N, E, OBS_JY>(psi, a, part, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int E>
hipError_t launch_obs_e(int kind, const void* psi, const PassArgs& a, int n, double* part, hipStream_t st) {
  const cx<T>* p = reinterpret_cast<const cx<T>*>(psi);
#define SGP_CASE(NN, EE) \
  case NN:               \
    if constexpr (plan_ok(NN, EE, (int)sizeof(T))) return obs_kind<T, NN, EE>(kind, p, a, part, st); \
    break;
  switch (n) { SGP_FOR_PLAN_N(E, SGP_CASE) default: break; }
#undef SGP_CASE
  return hipErrorInvalidValue;
}

}  // namespace sgp

// Split-step kernels for the rotating SOC spin-2 GPE on gfx950.
//
// One linear substep of the compact splitting (Sec. 3.1) in 2D is two passes over
// the state; each pass reads and writes every value once:
//   X-pass (rows):    inverse FFT along x, exact nonlinear flow per point (Sec. 3.2)
//                     with the trap at R(Omega s) x, forward FFT along x.
//   Y-pass (columns): forward FFT along y, exact linear propagator per wavevector
//                     (eq. sl1), inverse FFT along y.
// Between passes the state is held x-transformed (Fourier in x, physical in y).
// The first X-pass of a call starts from physical data (no inverse FFT) and the
// last one ends in physical data (no forward FFT).  3D adds a Z-pass that carries
// the propagator (Y1: forward y, Z: forward z + propagator + inverse z, Y2: inverse y).
#include "sgp_device.hpp"
#include "sgp_kernels.hpp"

namespace sgp {

// ---------------------------------------------------------------------------
// Rotation angle of the trap: theta = Omega * s with s the device clock (advanced
// by the linear passes) or a value passed by the host.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void trap_angle(const XArgs& a, double& c, double& s) {
  const double clk = a.clock_mode == CLOCK_ARG ? a.s_arg : a.clock[0];
  sincos(a.Omega * clk, &s, &c);
}

// ---------------------------------------------------------------------------
// X-pass, 2D or 3D: one line along x per TL = N/E threads, all 5 components.
// MODE: X_FIRST (physical in -> NL -> FFT), X_MID (iFFT -> NL -> FFT),
//       X_LAST (iFFT -> NL -> physical out), X_NLONLY (physical -> NL -> physical).
// ---------------------------------------------------------------------------
template <typename T, int N, int E, int MODE>
__global__ __launch_bounds__(256) void k_xpass(cx<T>* __restrict__ psi, XArgs a) {
  constexpr int TL = N / E;
  constexpr int LPB = 256 / TL;  // lines per block
  constexpr int LS = LdsLine<N>::size;
  __shared__ T lre[LPB * LS];
  __shared__ T lim[LPB * LS];
  const int tid = threadIdx.x;
  const int lloc = tid / TL, t = tid % TL;
  const long line = (long)blockIdx.x * LPB + lloc;  // line = z * ny + y
  // Lines past the end (grids with fewer lines than a block holds) run the
  // arithmetic on zeros and never touch global memory.
  const bool active = line < a.nlines;
  const int iy = (int)(line % a.ny);
  const int iz = (int)(line / a.ny);
  cx<T>* base = psi + (active ? line : 0) * N;
  cx<T> v[5][E];
#pragma unroll
  for (int c = 0; c < 5; ++c)
#pragma unroll
    for (int m = 0; m < E; ++m) v[c][m] = active ? base[c * a.comp_stride + t + TL * m] : mk<T>(T(0), T(0));
  T* re = lre + lloc * LS;
  T* im = lim + lloc * LS;
  constexpr int SYNC = (TL <= 64) ? 1 : 0;
  if constexpr (MODE == X_MID || MODE == X_LAST)
    fft_line<T, N, E, +1, 5, 1, SYNC>(v, re, im, t, reinterpret_cast<const cx<T>*>(a.tw_inv), 0);
  // nonlinear flow
  double ct, st;
  trap_angle(a, ct, st);
  const double y = -a.L[1] + iy * a.h[1];
  const double z = -a.L[2] + iz * a.h[2];
  const double vz = 0.5 * a.g2[2] * z * z;
  NLCoef K;
  K.d = a.d;
  K.c0p = a.c0p;
  K.c1 = a.c1;
  K.c2 = a.c2;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const double x = -a.L[0] + (t + TL * m) * a.h[0];
    const double X = ct * x + st * y, Y = -st * x + ct * y;
    const double V = 0.5 * (a.g2[0] * X * X + a.g2[1] * Y * Y) + vz;
    cx<T> p[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) p[c] = v[c][m];
    nl_point<T>(p, V, K);
#pragma unroll
    for (int c = 0; c < 5; ++c) v[c][m] = p[c];
  }
  if constexpr (MODE == X_FIRST || MODE == X_MID)
    fft_line<T, N, E, -1, 5, 1, SYNC>(v, re, im, t, reinterpret_cast<const cx<T>*>(a.tw_fwd), 0);
  if (active) {
#pragma unroll
    for (int c = 0; c < 5; ++c)
#pragma unroll
      for (int m = 0; m < E; ++m) base[c * a.comp_stride + t + TL * m] = v[c][m];
  }
  if (a.clock_mode == CLOCK_ARG && blockIdx.x == 0 && tid == 0) a.clock[0] = a.s_arg;
}

// ---------------------------------------------------------------------------
// Column pass: lines of length N with element stride `stride` (nx for y-lines,
// nx*ny for z-lines), W adjacent lines per block (coalesced W-wide segments).
// MODE: C_PROP (FFT -> propagator -> iFFT, the last-axis pass), C_FWD (FFT only),
//       C_INV (iFFT only).
// The propagator at wavevector (p, q[, r]) is exp(-i d |nu|^2/2) exp(i d Q) applied
// as sym4 of U = [[C - i S Omega, i S gamma a], [i S gamma conj(a), C + i S Omega]],
// a = -nu_q - i nu_p, C = cos(lam d/2), S = sin(lam d/2)/lam (table), times the
// kinetic phase from per-axis tables and the 1/N^d scale of the forward transform.
// ---------------------------------------------------------------------------
template <typename T, int N, int E, int W, int MODE>
__global__ __launch_bounds__(W * (N / E)) void k_colpass(cx<T>* __restrict__ psi, CArgs a) {
  constexpr int TC = N / E;
  constexpr int CS = LdsLine<N>::size + 1;  // odd column stride in LDS
  __shared__ T lre[W * CS];
  __shared__ T lim[W * CS];
  const int tid = threadIdx.x;
  const int col = tid % W, t = tid / W;
  // block -> (outer index o, first column): columns run along the contiguous axis
  const long ncolblk = (a.ncols + W - 1) / W;
  const long o = blockIdx.x / ncolblk;
  const long kx0 = (blockIdx.x % ncolblk) * W + col;  // index along the contiguous axis
  // Columns past the end (ncols < W) compute on zeros and never touch global memory.
  const bool active = kx0 < a.ncols;
  const long kx = active ? kx0 : 0;
  cx<T>* base = psi + o * a.outer_stride + kx;
  cx<T> v[5][E];
#pragma unroll
  for (int c = 0; c < 5; ++c)
#pragma unroll
    for (int m = 0; m < E; ++m)
      v[c][m] = active ? base[c * a.comp_stride + (long)(t + TC * m) * a.stride] : mk<T>(T(0), T(0));
  T* re = lre + col * CS;
  T* im = lim + col * CS;
  if constexpr (MODE == C_PROP || MODE == C_FWD)
    fft_line<T, N, E, -1, 5, 1, 0>(v, re, im, t, reinterpret_cast<const cx<T>*>(a.tw_fwd), 0);
  if constexpr (MODE == C_PROP) {
    const T* cs = reinterpret_cast<const T*>(a.cs);
    const cx<T>* kin_a = reinterpret_cast<const cx<T>*>(a.kin_a);  // along the contiguous axis
    const cx<T>* kin_o = reinterpret_cast<const cx<T>*>(a.kin_o);  // along the outer axis (3D: y)
    const cx<T>* kin_l = reinterpret_cast<const cx<T>*>(a.kin_l);  // along this pass's axis
    const T Om = T(a.Omega), ga = T(a.gamma);
    const T norm = T(a.norm);  // 1/N^d, a power of two: exact
    const int nxx = (int)a.ncols;
    const int px = (int)(kx < nxx / 2 ? kx : kx - nxx);
    const T nup = T(px * a.nu_scale_a);
    cx<T> ka = kin_a[kx];
    if (a.dim == 3) {
      const cx<T> ko = kin_o[o];
      ka = ka + ko + ka * ko;
    }
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int kl = t + TC * m;
      // 2D: the line runs along y = q; 3D: along z, with q the outer index
      long qidx;
      int kq;
      if (a.dim == 2) { kq = kl; qidx = (long)kl * nxx + kx; }
      else { kq = (int)o; qidx = o * nxx + kx; }
      const int pq = kq < a.n_q / 2 ? kq : kq - a.n_q;
      const T nuq = T(pq * a.nu_scale_q);
      const T Cm1 = cs[2 * qidx], S = cs[2 * qidx + 1];
      // alpha - 1 = (C - 1) - i S Omega
      const cx<T> as = mk<T>(Cm1, -S * Om);
      // beta = i S gamma a, a = -nu_q - i nu_p  ->  S gamma (nu_p - i nu_q)
      const cx<T> beta = mk<T>(S * ga * nup, -S * ga * nuq);
      // kinetic phase - 1: (1 + ka)(1 + kl) - 1
      const cx<T> kl1 = kin_l[kl];
      const cx<T> ss = ka + kl1 + ka * kl1;
      cx<T> x[5];
#pragma unroll
      for (int c = 0; c < 5; ++c) x[c] = norm * v[c][m];
      sym4_apply_inc<T>(as, beta, ss, x);
#pragma unroll
      for (int c = 0; c < 5; ++c) v[c][m] = x[c];
    }
  }
  if constexpr (MODE == C_PROP || MODE == C_INV)
    fft_line<T, N, E, +1, 5, 1, 0>(v, re, im, t, reinterpret_cast<const cx<T>*>(a.tw_inv), 0);
  if (active) {
#pragma unroll
    for (int c = 0; c < 5; ++c)
#pragma unroll
      for (int m = 0; m < E; ++m) base[c * a.comp_stride + (long)(t + TC * m) * a.stride] = v[c][m];
  }
  if (MODE == C_PROP && a.advance_clock && blockIdx.x == 0 && tid == 0) a.clock[0] += a.d;
}

// ---------------------------------------------------------------------------
// Propagator table, FP64: Q = n.f with n = (gamma Re a, -gamma Im a, -Omega), so
// exp(i d Q) is the spin-2 image of exp(i d n.sigma/2) = C + i S n.sigma with
// C = cos(lam d/2), S = sin(lam d/2)/lam, lam = |n| = sqrt(Omega^2 + gamma^2
// (nu_p^2 + nu_q^2)).  Stored per (p, q), rounded to T: (C - 1, S), with
// C - 1 = -2 sin^2(lam d/4).  Kinetic tables per axis: exp(-i d nu^2/2) - 1.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_build_cs(T* __restrict__ cs, int nx, int ny, double Lx, double Ly, double Omega, double gamma,
                           double d) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)nx * ny) return;
  const int kx = (int)(i % nx), ky = (int)(i / nx);
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
// Mass and magnetization partial sums, FP64: one partial per block, summed in a
// fixed order by the host (deterministic).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_mass_magn(const cx<T>* __restrict__ psi, long npts, double* __restrict__ part) {
  double m = 0.0, mg = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += (long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const cx<T> z = psi[c * npts + i];
      const double n = (double)z.re * z.re + (double)z.im * z.im;
      m += n;
      mg += (2 - c) * n;
    }
  }
  // wavefront reduction, then across the 4 wavefronts of the block
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    m += __shfl_down(m, off, 64);
    mg += __shfl_down(mg, off, 64);
  }
  __shared__ double sm[2][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) { sm[0][wv] = m; sm[1][wv] = mg; }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sm[0][0] + sm[0][1] + sm[0][2] + sm[0][3];
    part[2 * blockIdx.x + 1] = sm[1][0] + sm[1][1] + sm[1][2] + sm[1][3];
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <typename T, int N, int E>
static hipError_t xpass_n(int mode, cx<T>* psi, const XArgs& a, long nlines, hipStream_t st) {
  constexpr int TL = N / E;
  constexpr int LPB = 256 / TL;
  if (nlines != a.nlines) return hipErrorInvalidValue;
  dim3 grid((unsigned)((nlines + LPB - 1) / LPB)), block(256);
  switch (mode) {
    case X_FIRST: hipLaunchKernelGGL((k_xpass<T, N, E, X_FIRST>), grid, block, 0, st, psi, a); break;
    case X_MID: hipLaunchKernelGGL((k_xpass<T, N, E, X_MID>), grid, block, 0, st, psi, a); break;
    case X_LAST: hipLaunchKernelGGL((k_xpass<T, N, E, X_LAST>), grid, block, 0, st, psi, a); break;
    default: hipLaunchKernelGGL((k_xpass<T, N, E, X_NLONLY>), grid, block, 0, st, psi, a); break;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_xpass(int mode, void* psi, const XArgs& a, int nx, long nlines, hipStream_t st) {
  cx<T>* p = reinterpret_cast<cx<T>*>(psi);
  switch (nx) {
    case 16: return xpass_n<T, 16, 8>(mode, p, a, nlines, st);
    case 32: return xpass_n<T, 32, 8>(mode, p, a, nlines, st);
    case 64: return xpass_n<T, 64, 8>(mode, p, a, nlines, st);
    case 128: return xpass_n<T, 128, 8>(mode, p, a, nlines, st);
    case 256: return xpass_n<T, 256, 8>(mode, p, a, nlines, st);
    case 512: return xpass_n<T, 512, 8>(mode, p, a, nlines, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int N, int E>
static hipError_t colpass_n(int mode, cx<T>* psi, const CArgs& a, hipStream_t st) {
  constexpr int TC = N / E;
  constexpr int W0 = (sizeof(T) == 4 ? 8 : 4);
  constexpr int W = (256 / TC > W0) ? 256 / TC : W0;
  dim3 grid((unsigned)(((a.ncols + W - 1) / W) * a.nouter)), block(W * TC);
  switch (mode) {
    case C_PROP: hipLaunchKernelGGL((k_colpass<T, N, E, W, C_PROP>), grid, block, 0, st, psi, a); break;
    case C_FWD: hipLaunchKernelGGL((k_colpass<T, N, E, W, C_FWD>), grid, block, 0, st, psi, a); break;
    default: hipLaunchKernelGGL((k_colpass<T, N, E, W, C_INV>), grid, block, 0, st, psi, a); break;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_colpass(int mode, void* psi, const CArgs& a, int n, hipStream_t st) {
  cx<T>* p = reinterpret_cast<cx<T>*>(psi);
  switch (n) {
    case 16: return colpass_n<T, 16, 8>(mode, p, a, st);
    case 32: return colpass_n<T, 32, 8>(mode, p, a, st);
    case 64: return colpass_n<T, 64, 8>(mode, p, a, st);
    case 128: return colpass_n<T, 128, 8>(mode, p, a, st);
    case 256: return colpass_n<T, 256, 8>(mode, p, a, st);
    case 512: return colpass_n<T, 512, 8>(mode, p, a, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_build_tables(void* cs, void* kin_x, void* kin_y, void* kin_z, const int* n, const double* L,
                               int dim, double Omega, double gamma, double d, hipStream_t st) {
  const long nxy = (long)n[0] * n[1];
  hipLaunchKernelGGL((k_build_cs<T>), dim3((unsigned)((nxy + 255) / 256)), dim3(256), 0, st, (T*)cs, n[0], n[1],
                     L[0], L[1], Omega, gamma, d);
  hipLaunchKernelGGL((k_build_kin<T>), dim3((n[0] + 255) / 256), dim3(256), 0, st, (cx<T>*)kin_x, n[0], L[0], d);
  hipLaunchKernelGGL((k_build_kin<T>), dim3((n[1] + 255) / 256), dim3(256), 0, st, (cx<T>*)kin_y, n[1], L[1], d);
  if (dim == 3)
    hipLaunchKernelGGL((k_build_kin<T>), dim3((n[2] + 255) / 256), dim3(256), 0, st, (cx<T>*)kin_z, n[2], L[2], d);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mass_magn(const void* psi, long npts, double* part, int nblocks, hipStream_t st) {
  hipLaunchKernelGGL((k_mass_magn<T>), dim3(nblocks), dim3(256), 0, st, (const cx<T>*)psi, npts, part);
  return hipGetLastError();
}

template hipError_t launch_xpass<float>(int, void*, const XArgs&, int, long, hipStream_t);
template hipError_t launch_xpass<double>(int, void*, const XArgs&, int, long, hipStream_t);
template hipError_t launch_colpass<float>(int, void*, const CArgs&, int, hipStream_t);
template hipError_t launch_colpass<double>(int, void*, const CArgs&, int, hipStream_t);
template hipError_t launch_build_tables<float>(void*, void*, void*, void*, const int*, const double*, int, double,
                                               double, double, hipStream_t);
template hipError_t launch_build_tables<double>(void*, void*, void*, void*, const int*, const double*, int, double,
                                                double, double, hipStream_t);
template hipError_t launch_mass_magn<float>(const void*, long, double*, int, hipStream_t);
template hipError_t launch_mass_magn<double>(const void*, long, double*, int, hipStream_t);

}  // namespace sgp

// Oracle for the compact splitting Fourier spectral method for the rotating
// spin-orbit-coupled spin-2 Gross-Pitaevskii system (Liu, Xie, Yuan, Zhang, Zhao,
// arXiv 2603.25282).
//
// TEST INFRASTRUCTURE ONLY.  This is a plain, slow, FP64 CPU implementation written
// to be checked by eye against the paper.  Only tests/, __graft_entry__.smoke() and
// bench.py's cpu_baseline leg may load it.  It shares no code with the HIP library.
//
// Conventions (paper Sec. 3.1, "Fourier spectral method" paragraph):
//   * domain [-L, L]^d, h = 2L/N, x_j = -L + j h, N even;
//   * forward transform carries the 1/N^d factor, inverse is unscaled;
//   * wavenumber nu_p = pi p / L for p in [-N/2, N/2-1]; storage index k holds
//     p = k (k < N/2) or p = k - N (k >= N/2); the Nyquist index keeps nu = -pi N/(2L).
//   * component index i = 0..4 holds spin projection l = 2, 1, 0, -1, -2 (Sec. 1).
//   * state layout [5][nz][ny][nx], complex128 interleaved, x fastest.
//
// Every floating-point value is double.  Build with -O2 -ffp-contract=off.
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef std::complex<double> cd;
static const double PI = 3.14159265358979323846264338327950288;
static const cd I1(0.0, 1.0);

// ---------------------------------------------------------------------------
// Forward-mode dual numbers and a small complex type over them.  The nonlinear
// flow and the closed-form propagator are written once, templated on the real type,
// so that the adjoint (below) differentiates exactly the functions the forward
// evolution uses.
// ---------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual(double v_ = 0.0, double d_ = 0.0) : v(v_), d(d_) {}
};
static inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
static inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
static inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
static inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
static inline Dual operator/(Dual a, Dual b) { return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)); }
static inline Dual sqrt(Dual a) { double r = std::sqrt(a.v); return Dual(r, r > 0.0 ? a.d / (2.0 * r) : 0.0); }
static inline Dual sin(Dual a) { return Dual(std::sin(a.v), a.d * std::cos(a.v)); }
static inline Dual cos(Dual a) { return Dual(std::cos(a.v), -a.d * std::sin(a.v)); }
static inline double val(double x) { return x; }
static inline double val(Dual x) { return x.v; }

template <class R>
struct Cx {
  R re, im;
  Cx(R r = R(0.0), R i = R(0.0)) : re(r), im(i) {}
};
template <class R> static inline Cx<R> operator+(Cx<R> a, Cx<R> b) { return Cx<R>(a.re + b.re, a.im + b.im); }
template <class R> static inline Cx<R> operator-(Cx<R> a, Cx<R> b) { return Cx<R>(a.re - b.re, a.im - b.im); }
template <class R> static inline Cx<R> operator*(Cx<R> a, Cx<R> b) {
  return Cx<R>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <class R> static inline Cx<R> operator*(R s, Cx<R> a) { return Cx<R>(s * a.re, s * a.im); }
template <class R> static inline Cx<R> cconj(Cx<R> a) { return Cx<R>(a.re, R(0.0) - a.im); }
template <class R> static inline R cnorm(Cx<R> a) { return a.re * a.re + a.im * a.im; }
template <class R> static inline Cx<R> expi(R x) { return Cx<R>(cos(x), sin(x)); }
template <class R> static inline Cx<R> cx_of(cd z) { return Cx<R>(R(z.real()), R(z.imag())); }
static inline cd to_cd(Cx<double> z) { return cd(z.re, z.im); }

struct OGrid {
  int dim;        // 2 or 3
  int n[3];       // nx, ny, nz (nz = 1 in 2D)
  double L[3];    // half-widths
};

struct OParams {
  double c0, c1, c2, Omega, gamma, gx, gy, gz;
};

static inline long npoints(const OGrid& g) {
  return (long)g.n[0] * g.n[1] * (g.dim == 3 ? g.n[2] : 1);
}

// ---------------------------------------------------------------------------
// Discrete Fourier transform (own mixed-radix implementation).
// y[k] = sum_j x[j] exp(sign * 2 pi i j k / n).  Recursive decimation in time by
// the smallest prime factor; a prime length falls back to the O(n^2) sum.
// ---------------------------------------------------------------------------
static int smallest_factor(int n) {
  for (int r = 2; r * r <= n; ++r)
    if (n % r == 0) return r;
  return n;
}

// w[k] = exp(sign * 2 pi i k / ntop); at a sub-length m dividing ntop the twiddle
// exp(sign 2 pi i t / m) is w[t * (ntop / m)].
static void fft_rec(const cd* x, long xs, cd* y, int n, const cd* w, int ntop) {
  if (n == 1) { y[0] = x[0]; return; }
  int r = smallest_factor(n);
  int m = n / r;
  for (int s = 0; s < r; ++s) fft_rec(x + s * xs, xs * r, y + (long)s * m, m, w, ntop);
  cd tbuf[16], ubuf[16];
  std::vector<cd> tv, uv;
  cd *t = tbuf, *u = ubuf;
  if (r > 16) { tv.resize(r); uv.resize(r); t = tv.data(); u = uv.data(); }
  long step = ntop / n;  // twiddle index stride for length n
  for (int k = 0; k < m; ++k) {
    for (int s = 0; s < r; ++s) t[s] = y[(long)s * m + k] * w[((long)s * k * step) % ntop];
    for (int q = 0; q < r; ++q) {
      cd acc = 0.0;
      for (int s = 0; s < r; ++s) acc += t[s] * w[((long)s * q * m * step) % ntop];
      u[q] = acc;
    }
    for (int q = 0; q < r; ++q) y[k + (long)q * m] = u[q];
  }
}

static std::vector<cd> twiddles(int n, int sign) {
  std::vector<cd> w(n);
  for (int k = 0; k < n; ++k) {
    double a = sign * 2.0 * PI * (double)k / (double)n;
    w[k] = cd(std::cos(a), std::sin(a));
  }
  return w;
}

// Transform every line of `data` along axis `ax`.  sign=-1 forward (scaled by 1/n),
// sign=+1 inverse (unscaled).
static void fft_axis(const OGrid& g, cd* data, int ax, int sign) {
  int nx = g.n[0], ny = g.n[1], nz = (g.dim == 3 ? g.n[2] : 1);
  int n = g.n[ax];
  long stride = (ax == 0) ? 1 : (ax == 1 ? nx : (long)nx * ny);
  long nlines = (long)nx * ny * nz / n;
  std::vector<cd> w = twiddles(n, sign);
  double scale = (sign < 0) ? 1.0 / (double)n : 1.0;
#pragma omp parallel
  {
    std::vector<cd> in(n), out(n);
#pragma omp for schedule(static)
    for (long line = 0; line < nlines; ++line) {
      long base;
      if (ax == 0) base = line * nx;
      else if (ax == 1) base = (line / nx) * (long)nx * ny + (line % nx);
      else base = line;  // ax == 2: line enumerates (y, x) in one z-slab
      for (int j = 0; j < n; ++j) in[j] = data[base + j * stride];
      fft_rec(in.data(), 1, out.data(), n, w.data(), n);
      for (int j = 0; j < n; ++j) data[base + j * stride] = out[j] * scale;
    }
  }
}

// d-dimensional transform of one scalar field.
static void fft_nd(const OGrid& g, cd* data, int sign) {
  for (int ax = 0; ax < g.dim; ++ax) fft_axis(g, data, ax, sign);
}

static inline double wavenumber(int k, int n, double L) {
  int p = (k < n / 2) ? k : k - n;
  return PI * (double)p / L;
}

// ---------------------------------------------------------------------------
// Exact linear propagator exp(i delta Q) for one wavevector, Sec. 3.1: Q has
// diagonal -Omega (2, 1, 0, -1, -2) and off-diagonals gamma a (1, sqrt6/2, sqrt6/2, 1)
// above, gamma conj(a) below, with a = -nu_q - i nu_p.  Entry (i, j) of exp(i tau Q)
// is a^(j-i) c_ij for j >= i and conj(a)^(i-j) c_ji for i > j, with the fifteen c_ij
// written out in the paper.  eta1 = cos(2 lam tau) - 1 and eta2 = cos(lam tau) - 1
// are evaluated as -2 sin^2(lam tau) and -2 sin^2(lam tau / 2) (same value, no
// cancellation).  lam = 0 (Omega = 0 and nu_perp = 0) gives the identity.
// out is row-major 5x5.
// ---------------------------------------------------------------------------
template <class R>
static void propagator_t(R Omega, R gamma, double nu_p, double nu_q, R tau, Cx<R>* out) {
  const double are = -nu_q, aim = -nu_p;  // a = -nu_q - i nu_p
  const double amod = std::sqrt(are * are + aim * aim);
  R xi = gamma * R(amod);
  R lam = sqrt(Omega * Omega + xi * xi);
  for (int i = 0; i < 25; ++i) out[i] = Cx<R>();
  if (val(lam) == 0.0) {
    for (int i = 0; i < 5; ++i) out[i * 5 + i] = Cx<R>(R(1.0));
    return;
  }
  R s1 = sin(lam * tau), s2 = sin(R(0.5) * lam * tau);
  Cx<R> eta1(R(-2.0) * s1 * s1);
  Cx<R> eta2(R(-2.0) * s2 * s2);
  Cx<R> eta3(R(0.0), sin(R(2.0) * lam * tau));
  Cx<R> eta4(R(0.0), s1);
  R O = Omega, O2 = O * O, O3 = O2 * O, O4 = O2 * O2;
  R x2 = xi * xi, x4 = x2 * x2;
  R l2 = lam * lam, l3 = l2 * lam, l4 = l2 * l2;
  R g = gamma, g2 = g * g, g3 = g2 * g, g4 = g2 * g2;
  R r6 = R(std::sqrt(6.0));
  const R two(2.0), three(3.0), four(4.0), eight(8.0), one(1.0);
  Cx<R> L4(l4 * eight);
  Cx<R> c11 = (one / (eight * l4)) * ((eight * O4 + eight * O2 * x2 + x4) * eta1 + (four * x2 * (two * O2 + x2)) * eta2
                                      - (four * O * lam * (two * O2 + x2)) * eta3 - (eight * O * lam * x2) * eta4 + L4);
  Cx<R> c12 = (g / (four * l4)) * ((R(0.0) - O * (four * O2 + three * x2)) * eta1 + (four * O3) * eta2 +
                                   (lam * (four * O2 + x2)) * eta3 - (two * lam * (two * O2 - x2)) * eta4);
  Cx<R> c13 = (r6 * g2 / (four * l4)) * (((two * O2 + x2) * eta2 - (two * O * lam) * eta4 + Cx<R>(two * l2)) * eta2);
  Cx<R> c14 = (g3 / (two * l4)) * (((R(0.0) - O) * eta2 + lam * eta4) * eta2);
  Cx<R> c15 = (g4 / (eight * l4)) * (eta1 - four * eta2);
  Cx<R> c22 = (one / (two * l4)) * (((two * x2) * eta2 + Cx<R>(l2)) * ((two * O2 + x2) * eta2 - (two * O * lam) * eta4 +
                                                                      Cx<R>(two * l2)));
  Cx<R> c23 = (r6 * g / (two * l4)) * ((x2 * eta2 + Cx<R>(l2)) * ((R(0.0) - O) * eta2 + lam * eta4));
  Cx<R> c24 = (g2 / (two * l4)) * (((two * x2) * eta2 + Cx<R>(three * l2)) * eta2);
  Cx<R> c25 = c14 + (O * g3 / l4) * (eta2 * eta2);
  Cx<R> c33 = (three * x2 / (four * l4)) * (x2 * eta1 + (four * O2) * eta2) + Cx<R>(one);
  Cx<R> c34 = c23 + (r6 * O * g / l4) * ((x2 * eta2 + Cx<R>(l2)) * eta2);
  Cx<R> c35 = c13 + (r6 * O * g2 / l3) * (eta2 * eta4);
  Cx<R> c44 = c22 + (two * O / l3) * (((two * x2) * eta2 + Cx<R>(l2)) * eta4);
  Cx<R> c45 = c12 + (O * g / (two * l4)) * (((four * O2 + three * x2)) * eta1 - (four * O2) * eta2);
  Cx<R> c55 = c11 + (O / l3) * ((two * O2 + x2) * eta3 + (two * x2) * eta4);

  Cx<R> c[5][5];
  c[0][0] = c11; c[0][1] = c12; c[0][2] = c13; c[0][3] = c14; c[0][4] = c15;
  c[1][1] = c22; c[1][2] = c23; c[1][3] = c24; c[1][4] = c25;
  c[2][2] = c33; c[2][3] = c34; c[2][4] = c35;
  c[3][3] = c44; c[3][4] = c45;
  c[4][4] = c55;
  Cx<R> a{R(are), R(aim)}, ab{R(are), R(-aim)};
  Cx<R> apow[5], abpow[5];
  apow[0] = abpow[0] = Cx<R>(R(1.0));
  for (int k = 1; k < 5; ++k) { apow[k] = apow[k - 1] * a; abpow[k] = abpow[k - 1] * ab; }
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j)
      out[i * 5 + j] = (j >= i) ? apow[j - i] * c[i][j] : abpow[i - j] * c[j][i];
}

static void propagator(double Omega, double gamma, double nu_p, double nu_q, double tau, cd* out) {
  Cx<double> o[25];
  propagator_t<double>(Omega, gamma, nu_p, nu_q, tau, o);
  for (int i = 0; i < 25; ++i) out[i] = to_cd(o[i]);
}

// ---------------------------------------------------------------------------
// Linear substep: Phi <- IFFT[ exp(-i delta |nu|^2/2) exp(i delta Q) FFT[Phi] ]
// (Sec. 3.1, solution of the Fourier-space ODE, eq. (sl1)); in 3D, Q depends on
// (nu_p, nu_q) only and |nu|^2 includes nu_r (3D remark of Sec. 3.1).
// ---------------------------------------------------------------------------
static void linear_step(const OGrid& g, const OParams& P, double delta, cd* psi) {
  long np = npoints(g);
  for (int c = 0; c < 5; ++c) fft_nd(g, psi + c * np, -1);
  int nx = g.n[0], ny = g.n[1], nz = (g.dim == 3 ? g.n[2] : 1);
#pragma omp parallel for schedule(static)
  for (long pq = 0; pq < (long)nx * ny; ++pq) {
    int kx = (int)(pq % nx), ky = (int)(pq / nx);
    double nup = wavenumber(kx, nx, g.L[0]);
    double nuq = wavenumber(ky, ny, g.L[1]);
    cd E[25];
    propagator(P.Omega, P.gamma, nup, nuq, delta, E);
    for (int kz = 0; kz < nz; ++kz) {
      double nur = (g.dim == 3) ? wavenumber(kz, nz, g.L[2]) : 0.0;
      double k2 = nup * nup + nuq * nuq + nur * nur;
      cd kin = std::exp(cd(0.0, -0.5 * delta * k2));
      long idx = (long)kz * nx * ny + pq;
      cd v[5], w[5];
      for (int i = 0; i < 5; ++i) v[i] = psi[i * np + idx];
      for (int i = 0; i < 5; ++i) {
        cd acc = 0.0;
        for (int j = 0; j < 5; ++j) acc += E[i * 5 + j] * v[j];
        w[i] = kin * acc;
      }
      for (int i = 0; i < 5; ++i) psi[i * np + idx] = w[i];
    }
  }
  for (int c = 0; c < 5; ++c) fft_nd(g, psi + c * np, +1);
}

// ---------------------------------------------------------------------------
// Nonlinear substep at one grid point, Sec. 3.2, eq. (solution2):
//   Psi(t) = exp(-i d [V + (c0 + c2/5) rho]) exp(-i c1 d F.f)
//            [cos(c2 S d) Psi + (i/S) sin(c2 S d) (rho/5 Psi - A00 A conj(Psi))]
// with S = sqrt((rho/5)^2 - |A00|^2/5) and exp(-i c1 d F.f) from the spin-2
// polynomial in N = F.f/|F|, kappa = c1 |F| d.
// Limits the paper leaves implicit: S = 0 uses sin(c2 S d)/S = c2 d; |F| = 0 makes
// the spin rotation the identity; S^2 < 0 from rounding is clamped to 0.
// ---------------------------------------------------------------------------
template <class R>
static void ff_matrix(R Fx, R Fy, R Fz, Cx<R>* M) {
  // F.f (Sec. 1): diagonal F_z (2,1,0,-1,-2); F_- above, F_+ below with the
  // sqrt6/2 weights on the middle links.
  Cx<R> Fp(Fx, Fy), Fm(Fx, R(0.0) - Fy);
  R h6 = R(std::sqrt(6.0) / 2.0);
  for (int i = 0; i < 25; ++i) M[i] = Cx<R>();
  M[0 * 5 + 0] = Cx<R>(R(2.0) * Fz); M[1 * 5 + 1] = Cx<R>(Fz); M[3 * 5 + 3] = Cx<R>(R(0.0) - Fz);
  M[4 * 5 + 4] = Cx<R>(R(-2.0) * Fz);
  M[0 * 5 + 1] = Fm;      M[1 * 5 + 0] = Fp;
  M[1 * 5 + 2] = h6 * Fm; M[2 * 5 + 1] = h6 * Fp;
  M[2 * 5 + 3] = h6 * Fm; M[3 * 5 + 2] = h6 * Fp;
  M[3 * 5 + 4] = Fm;      M[4 * 5 + 3] = Fp;
}

template <class R>
static void matmul5(const Cx<R>* A, const Cx<R>* B, Cx<R>* C) {
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) {
      Cx<R> acc;
      for (int k = 0; k < 5; ++k) acc = acc + A[i * 5 + k] * B[k * 5 + j];
      C[i * 5 + j] = acc;
    }
}

template <class R>
struct DensitiesT { R rho, Fx, Fy, Fz; Cx<R> A00; };

template <class R>
static DensitiesT<R> densities_t(const Cx<R>* psi) {
  // Sec. 1: rho = sum |psi_l|^2, F_x, F_y, F_z, A00 = (2 psi2 psi-2 - 2 psi1 psi-1 + psi0^2)/sqrt5.
  const Cx<R> &p2 = psi[0], &p1 = psi[1], &p0 = psi[2], &m1 = psi[3], &m2 = psi[4];
  const R h6 = R(std::sqrt(6.0) / 2.0), two(2.0);
  DensitiesT<R> d;
  d.rho = cnorm(p2) + cnorm(p1) + cnorm(p0) + cnorm(m1) + cnorm(m2);
  Cx<R> fx = cconj(p1) * p2 + cconj(p2) * p1 + cconj(m2) * m1 + cconj(m1) * m2
             + h6 * (cconj(p0) * p1 + cconj(p1) * p0 + cconj(m1) * p0 + cconj(p0) * m1);
  Cx<R> fy = Cx<R>(R(0.0), R(1.0)) * (cconj(p1) * p2 - cconj(p2) * p1 + cconj(m2) * m1 - cconj(m1) * m2
                                      + h6 * (cconj(p0) * p1 - cconj(p1) * p0 + cconj(m1) * p0 - cconj(p0) * m1));
  d.Fx = fx.re;
  d.Fy = fy.re;
  d.Fz = two * cnorm(p2) + cnorm(p1) - cnorm(m1) - two * cnorm(m2);
  d.A00 = R(1.0 / std::sqrt(5.0)) * (two * (p2 * m2) - two * (p1 * m1) + p0 * p0);
  return d;
}

// Exact nonlinear flow at one point for time delta (Sec. 3.2, eq. solution2), with
// the interaction constants and the trap value as (possibly dual) reals.
template <class R>
static void nl_point_t(R c0, R c1, R c2, R V, R delta, Cx<R>* psi) {
  DensitiesT<R> d = densities_t(psi);
  const R five(5.0);
  R S2 = (d.rho / five) * (d.rho / five) - cnorm(d.A00) / five;
  if (val(S2) < 0.0) S2 = R(0.0);
  R S = sqrt(S2);
  R cs = cos(c2 * S * delta);
  R sn_over_S = (val(S) == 0.0) ? c2 * delta : sin(c2 * S * delta) / S;
  // (A conj Psi)_i = (-1)^(i-1) conj(psi_{6-i}) / sqrt5 with 1-based i (Sec. 1).
  const R r5(1.0 / std::sqrt(5.0));
  Cx<R> Apsib[5] = {r5 * cconj(psi[4]), (R(0.0) - r5) * cconj(psi[3]), r5 * cconj(psi[2]),
                    (R(0.0) - r5) * cconj(psi[1]), r5 * cconj(psi[0])};
  const Cx<R> I(R(0.0), R(1.0));
  Cx<R> b[5];
  for (int i = 0; i < 5; ++i)
    b[i] = cs * psi[i] + sn_over_S * (I * ((d.rho / five) * psi[i] - d.A00 * Apsib[i]));

  // exp(-i c1 d F.f) = I + i g1 N + g2 N^2 + i g3 N^3 + g4 N^4, N = F.f/|F|.
  R Fabs = sqrt(d.Fx * d.Fx + d.Fy * d.Fy + d.Fz * d.Fz);
  Cx<R> Rm[25];
  for (int i = 0; i < 25; ++i) Rm[i] = Cx<R>();
  for (int i = 0; i < 5; ++i) Rm[i * 5 + i] = Cx<R>(R(1.0));
  if (val(Fabs) > 0.0) {
    R kap = c1 * Fabs * delta;
    R g1 = sin(R(2.0) * kap) / R(6.0) - R(4.0 / 3.0) * sin(kap);
    R g2 = R(4.0 / 3.0) * cos(kap) - cos(R(2.0) * kap) / R(12.0) - R(5.0 / 4.0);
    R g3 = sin(kap) / R(3.0) - sin(R(2.0) * kap) / R(6.0);
    R g4 = cos(R(2.0) * kap) / R(12.0) - cos(kap) / R(3.0) + R(0.25);
    Cx<R> N1[25], N2[25], N3[25], N4[25];
    ff_matrix(d.Fx / Fabs, d.Fy / Fabs, d.Fz / Fabs, N1);
    matmul5(N1, N1, N2);
    matmul5(N2, N1, N3);
    matmul5(N3, N1, N4);
    for (int i = 0; i < 25; ++i)
      Rm[i] = Rm[i] + I * (g1 * N1[i]) + g2 * N2[i] + I * (g3 * N3[i]) + g4 * N4[i];
  }
  Cx<R> ph = expi(R(0.0) - delta * (V + (c0 + c2 / five) * d.rho));
  for (int i = 0; i < 5; ++i) {
    Cx<R> acc;
    for (int j = 0; j < 5; ++j) acc = acc + Rm[i * 5 + j] * b[j];
    psi[i] = ph * acc;
  }
}

static void nl_point(const OParams& P, double V, double delta, cd* psi) {
  Cx<double> v[5];
  for (int i = 0; i < 5; ++i) v[i] = cx_of<double>(psi[i]);
  nl_point_t<double>(P.c0, P.c1, P.c2, V, delta, v);
  for (int i = 0; i < 5; ++i) psi[i] = to_cd(v[i]);
}

struct Densities { double rho, Fx, Fy, Fz; cd A00; };

static Densities densities(const cd* psi) {
  Cx<double> v[5];
  for (int i = 0; i < 5; ++i) v[i] = cx_of<double>(psi[i]);
  DensitiesT<double> t = densities_t(v);
  Densities d;
  d.rho = t.rho; d.Fx = t.Fx; d.Fy = t.Fy; d.Fz = t.Fz; d.A00 = to_cd(t.A00);
  return d;
}

// Trap of eq. (harmonic) evaluated at the rotated point R(theta) x, with
// R(theta) = [[cos, sin], [-sin, cos]] acting on (x, y) (Sec. 3.1, mapping).
static inline double trap_rotated(const OParams& P, double theta, double x, double y, double z) {
  double c = std::cos(theta), s = std::sin(theta);
  double X = c * x + s * y, Y = -s * x + c * y;
  return 0.5 * (P.gx * P.gx * X * X + P.gy * P.gy * Y * Y + P.gz * P.gz * z * z);
}

static inline double coord(const OGrid& g, int ax, int j) {
  double h = 2.0 * g.L[ax] / (double)g.n[ax];
  return -g.L[ax] + (double)j * h;
}

// Nonlinear substep over the grid with the trap rotated by theta (theta = 0: lab frame).
static void nl_step(const OGrid& g, const OParams& P, double delta, double theta, cd* psi) {
  long np = npoints(g);
  int nx = g.n[0], ny = g.n[1];
#pragma omp parallel for schedule(static)
  for (long idx = 0; idx < np; ++idx) {
    int ix = (int)(idx % nx), iy = (int)((idx / nx) % ny), iz = (int)(idx / ((long)nx * ny));
    double z = (g.dim == 3) ? coord(g, 2, iz) : 0.0;
    double V = trap_rotated(P, theta, coord(g, 0, ix), coord(g, 1, iy), z);
    cd v[5];
    for (int i = 0; i < 5; ++i) v[i] = psi[i * np + idx];
    nl_point(P, V, delta, v);
    for (int i = 0; i < 5; ++i) psi[i * np + idx] = v[i];
  }
}

// ---------------------------------------------------------------------------
// Rotation mapping by RSDA (Sec. 3.1, eqs. (RSDA1)/(RSDA2)): three shears
// exp(a y d_x) exp(b x d_y) exp(a y d_x), each a 1D transform, a phase
// exp(i nu a y) per Fourier mode, and the inverse transform.
// ---------------------------------------------------------------------------
static void shear(const OGrid& g, cd* f, int ax, double a) {
  // ax = 0: f(x, y) <- f(x + a y, y);  ax = 1: f(x, y) <- f(x, y + a x).
  int nx = g.n[0], ny = g.n[1], nz = (g.dim == 3 ? g.n[2] : 1);
  fft_axis(g, f, ax, -1);
  int other = 1 - ax;
#pragma omp parallel for schedule(static)
  for (long idx = 0; idx < (long)nx * ny * nz; ++idx) {
    int ix = (int)(idx % nx), iy = (int)((idx / nx) % ny);
    int kk = (ax == 0) ? ix : iy;
    int jo = (ax == 0) ? iy : ix;
    double nu = wavenumber(kk, g.n[ax], g.L[ax]);
    double w = coord(g, other, jo);
    f[idx] *= std::exp(cd(0.0, nu * a * w));
  }
  fft_axis(g, f, ax, +1);
}

// forward = true: Phi = M_t Psi, phi_l = exp(-i l Omega t) psi_l(R(t) x)  (RSDA1)
// forward = false: Psi = M_t^{-1} Phi, psi_l = exp(i l Omega t) phi_l(R(t)^{-1} x) (RSDA2)
static void rotation_map(const OGrid& g, const OParams& P, double t, bool forward, cd* psi) {
  long np = npoints(g);
  double th = P.Omega * t;
  double a = forward ? std::tan(th / 2.0) : -std::tan(th / 2.0);
  double b = forward ? -std::sin(th) : std::sin(th);
  static const int ell[5] = {2, 1, 0, -1, -2};
  for (int c = 0; c < 5; ++c) {
    cd* f = psi + c * np;
    shear(g, f, 0, a);
    shear(g, f, 1, b);
    shear(g, f, 0, a);
    cd ph = std::exp(cd(0.0, (forward ? -1.0 : 1.0) * ell[c] * P.Omega * t));
    for (long i = 0; i < np; ++i) f[i] *= ph;
  }
}

// ---------------------------------------------------------------------------
// Time composition, Sec. 3.3.  The coefficients a_j multiply the nonlinear flow
// and b_j the linear flow (the reading under which Algorithm 1 -- nonlinear half
// steps outside -- and Table Acc1 agree):
//   TS2: N(tau/2) L(tau) N(tau/2)
//   TS4: N(a1) L(b1) N(a2) L(b2) N(a2) L(b1) N(a1) (times tau), with
//        a1 = 1/(2(2-2^(1/3))), a2 = (1-2^(1/3))/(2(2-2^(1/3))),
//        b1 = 1/(2-2^(1/3)),    b2 = -2^(1/3)/(2-2^(1/3)).
// Rotating frame (mode 0): the state is Phi; the nonlinear substep uses the trap at
// R(Omega s) x with s the clock advanced by the linear substeps only.
// Lab frame (mode 1): Algorithm 1 literally, the mapping M_s before and M_{s+d}^{-1}
// after every linear substep, the nonlinear substep with the lab trap.
// ---------------------------------------------------------------------------
// Order 6: Yoshida's triple jump of the 4th-order scheme, S6(tau) = S4(z1 tau)
// S4(z0 tau) S4(z1 tau), z1 = 1/(2 - 2^(1/5)), z0 = -2^(1/5)/(2 - 2^(1/5)); the
// nonlinear flows that meet where two S4 factors join (same clock) are one flow of
// the summed length.
struct Scheme { int m; double a[10]; double b[10]; };

static Scheme make_scheme(int order) {
  Scheme sc;
  if (order == 2) {
    sc.m = 2; sc.a[0] = 0.5; sc.a[1] = 0.5; sc.b[0] = 1.0; sc.b[1] = 0.0;
    return sc;
  }
  double c = std::cbrt(2.0);
  double den = 2.0 - c;
  const double a4[4] = {1.0 / (2.0 * den), (1.0 - c) / (2.0 * den), (1.0 - c) / (2.0 * den), 1.0 / (2.0 * den)};
  const double b4[4] = {1.0 / den, -c / den, 1.0 / den, 0.0};
  if (order == 4) {
    sc.m = 4;
    for (int j = 0; j < 4; ++j) { sc.a[j] = a4[j]; sc.b[j] = b4[j]; }
    return sc;
  }
  const double q = std::pow(2.0, 0.2);
  const double z[3] = {1.0 / (2.0 - q), -q / (2.0 - q), 1.0 / (2.0 - q)};
  sc.m = 0;
  for (int f = 0; f < 3; ++f)
    for (int j = 0; j < 4; ++j) {
      if (j == 0 && f > 0) {
        sc.a[sc.m - 1] += z[f] * a4[0];  // joins the previous factor's last flow
        sc.b[sc.m - 1] = z[f] * b4[0];
        continue;
      }
      sc.a[sc.m] = z[f] * a4[j];
      sc.b[sc.m] = z[f] * b4[j];
      ++sc.m;
    }
  return sc;
}

static void evolve(const OGrid& g, const OParams& P, int order, double tau, long nsteps,
                   double t0, int mode, cd* psi) {
  Scheme sc = make_scheme(order);
  double t = t0;
  for (long n = 0; n < nsteps; ++n) {
    double s = t;
    for (int j = 0; j < sc.m; ++j) {
      if (sc.a[j] != 0.0) nl_step(g, P, sc.a[j] * tau, mode == 0 ? P.Omega * s : 0.0, psi);
      if (sc.b[j] != 0.0) {
        double d = sc.b[j] * tau;
        if (mode == 0) {
          linear_step(g, P, d, psi);
        } else {
          rotation_map(g, P, s, true, psi);
          linear_step(g, P, d, psi);
          rotation_map(g, P, s + d, false, psi);
        }
        s += d;
      }
    }
    t = t0 + (double)(n + 1) * tau;
  }
}

// ---------------------------------------------------------------------------
// Discrete adjoint of the evolution (gradient of a real loss J(Phi(T))).
// Convention: g = 2 dJ/d conj(Phi), i.e. dJ = Re sum_x conj(g) dPhi.
//  * linear substep L(d): L is unitary for this pairing and L(d)^H = L(-d);
//  * nonlinear substep: the real-linear Jacobian of nl_point_t at the stored input,
//    column by column with dual numbers (10 real directions per point);
//  * parameter partials with one more dual direction each: gamma and Omega through
//    the closed-form propagator, c0, c1, c2 through the nonlinear flow, Omega also
//    through the rotated trap (dV/dOmega = s (gx^2 - gy^2) X Y).
// Checkpoints every K steps; each segment is recomputed storing substep inputs.
// dpar = (gamma, Omega, c0, c1, c2).
// ---------------------------------------------------------------------------
static void nl_adjoint_step(const OGrid& g, const OParams& P, double delta, double s, const cd* psi_in,
                            cd* gvec, double* dpar) {
  long np = npoints(g);
  int nx = g.n[0], ny = g.n[1];
  const double theta = P.Omega * s;
  double acc[4] = {0, 0, 0, 0};  // Omega, c0, c1, c2
#pragma omp parallel
  {
    double loc[4] = {0, 0, 0, 0};
#pragma omp for schedule(static)
    for (long idx = 0; idx < np; ++idx) {
      int ix = (int)(idx % nx), iy = (int)((idx / nx) % ny), iz = (int)(idx / ((long)nx * ny));
      double x = coord(g, 0, ix), y = coord(g, 1, iy), z = (g.dim == 3) ? coord(g, 2, iz) : 0.0;
      double V = trap_rotated(P, theta, x, y, z);
      double c = std::cos(theta), sn = std::sin(theta);
      double X = c * x + sn * y, Y = -sn * x + c * y;
      double dVdO = s * (P.gx * P.gx - P.gy * P.gy) * X * Y;
      cd pin[5], gout[5], gin[5];
      for (int i = 0; i < 5; ++i) { pin[i] = psi_in[i * np + idx]; gout[i] = gvec[i * np + idx]; }
      auto run = [&](const cd* tangent, Dual c0, Dual c1, Dual c2, Dual Vd) {
        Cx<Dual> v[5];
        for (int k = 0; k < 5; ++k)
          v[k] = Cx<Dual>(Dual(pin[k].real(), tangent[k].real()), Dual(pin[k].imag(), tangent[k].imag()));
        nl_point_t<Dual>(c0, c1, c2, Vd, Dual(delta), v);
        double r = 0.0;
        for (int k = 0; k < 5; ++k) r += gout[k].real() * v[k].re.d + gout[k].imag() * v[k].im.d;
        return r;  // Re <gout, D tangent>
      };
      const cd zero[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      for (int j = 0; j < 5; ++j) {
        cd t[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        t[j] = 1.0;
        double re = run(t, Dual(P.c0), Dual(P.c1), Dual(P.c2), Dual(V));
        t[j] = I1;
        double im = run(t, Dual(P.c0), Dual(P.c1), Dual(P.c2), Dual(V));
        gin[j] = cd(re, im);
      }
      loc[0] += run(zero, Dual(P.c0), Dual(P.c1), Dual(P.c2), Dual(V, dVdO));
      loc[1] += run(zero, Dual(P.c0, 1.0), Dual(P.c1), Dual(P.c2), Dual(V));
      loc[2] += run(zero, Dual(P.c0), Dual(P.c1, 1.0), Dual(P.c2), Dual(V));
      loc[3] += run(zero, Dual(P.c0), Dual(P.c1), Dual(P.c2, 1.0), Dual(V));
      for (int i = 0; i < 5; ++i) gvec[i * np + idx] = gin[i];
    }
#pragma omp critical
    for (int q = 0; q < 4; ++q) acc[q] += loc[q];
  }
  dpar[1] += acc[0];
  dpar[2] += acc[1];
  dpar[3] += acc[2];
  dpar[4] += acc[3];
}

// Partials of Re <gout, L(d) phi_in> with respect to gamma and Omega.
static void linear_param_partials(const OGrid& g, const OParams& P, double delta, const cd* phi_in, const cd* gout,
                                  double* dpar) {
  long np = npoints(g);
  int nx = g.n[0], ny = g.n[1], nz = (g.dim == 3 ? g.n[2] : 1);
  std::vector<cd> hat(phi_in, phi_in + 5 * np), d(5 * np);
  for (int c = 0; c < 5; ++c) fft_nd(g, hat.data() + c * np, -1);
  for (int which = 0; which < 2; ++which) {
#pragma omp parallel for schedule(static)
    for (long pq = 0; pq < (long)nx * ny; ++pq) {
      int kx = (int)(pq % nx), ky = (int)(pq / nx);
      double nup = wavenumber(kx, nx, g.L[0]), nuq = wavenumber(ky, ny, g.L[1]);
      Cx<Dual> E[25];
      propagator_t<Dual>(Dual(P.Omega, which == 1 ? 1.0 : 0.0), Dual(P.gamma, which == 0 ? 1.0 : 0.0), nup, nuq,
                         Dual(delta), E);
      for (int kz = 0; kz < nz; ++kz) {
        double nur = (g.dim == 3) ? wavenumber(kz, nz, g.L[2]) : 0.0;
        cd kin = std::exp(cd(0.0, -0.5 * delta * (nup * nup + nuq * nuq + nur * nur)));
        long idx = (long)kz * nx * ny + pq;
        for (int i = 0; i < 5; ++i) {
          cd acc = 0.0;
          for (int j = 0; j < 5; ++j) acc += cd(E[i * 5 + j].re.d, E[i * 5 + j].im.d) * hat[j * np + idx];
          d[i * np + idx] = kin * acc;
        }
      }
    }
    for (int c = 0; c < 5; ++c) fft_nd(g, d.data() + c * np, +1);
    double r = 0.0;
    for (long i = 0; i < 5 * np; ++i) r += (std::conj(gout[i]) * d[i]).real();
    dpar[which] += r;
  }
}

static void adjoint(const OGrid& g, const OParams& P, int order, double tau, long nsteps, double t0,
                    const cd* psi0, const cd* gT, cd* g0, double* dpar, long K) {
  long np = npoints(g);
  Scheme sc = make_scheme(order);
  for (int q = 0; q < 5; ++q) dpar[q] = 0.0;
  if (K < 1) K = 1;
  // forward: checkpoints at the start of every segment
  std::vector<std::vector<cd>> ckpt;
  std::vector<cd> psi(psi0, psi0 + 5 * np);
  for (long n0 = 0; n0 < nsteps; n0 += K) {
    ckpt.push_back(psi);
    long ns = std::min(K, nsteps - n0);
    evolve(g, P, order, tau, ns, t0 + (double)n0 * tau, 0, psi.data());
  }
  std::vector<cd> gv(gT, gT + 5 * np);
  struct Sub { bool nl; double d, s; std::vector<cd> in; };
  for (long seg = (long)ckpt.size() - 1; seg >= 0; --seg) {
    long n0 = seg * K, ns = std::min(K, nsteps - n0);
    std::vector<Sub> subs;
    std::vector<cd> u = ckpt[seg];
    for (long n = 0; n < ns; ++n) {
      double s = t0 + (double)(n0 + n) * tau;
      for (int j = 0; j < sc.m; ++j) {
        if (sc.a[j] != 0.0) {
          subs.push_back({true, sc.a[j] * tau, s, u});
          nl_step(g, P, sc.a[j] * tau, P.Omega * s, u.data());
        }
        if (sc.b[j] != 0.0) {
          subs.push_back({false, sc.b[j] * tau, s, u});
          linear_step(g, P, sc.b[j] * tau, u.data());
          s += sc.b[j] * tau;
        }
      }
    }
    for (long k = (long)subs.size() - 1; k >= 0; --k) {
      const Sub& sb = subs[k];
      if (sb.nl) {
        nl_adjoint_step(g, P, sb.d, sb.s, sb.in.data(), gv.data(), dpar);
      } else {
        linear_param_partials(g, P, sb.d, sb.in.data(), gv.data(), dpar);
        linear_step(g, P, -sb.d, gv.data());
      }
    }
  }
  std::copy(gv.begin(), gv.end(), g0);
}

// ---------------------------------------------------------------------------
// Observables, Sec. 2, on the discrete l2 inner product of Sec. 3.4 (h^d sum):
//   mass N, energy E, magnetization M, angular momentum <Lz>.
// Derivatives are spectral (Sec. 3.1).  theta rotates the trap (rotating frame).
// ---------------------------------------------------------------------------
static void spectral_derivative(const OGrid& g, const cd* f, int ax, cd* out) {
  long np = npoints(g);
  int nx = g.n[0], ny = g.n[1];
  std::memcpy((void*)out, (const void*)f, sizeof(cd) * np);
  fft_nd(g, out, -1);
  for (long idx = 0; idx < np; ++idx) {
    int k = (ax == 0) ? (int)(idx % nx) : (ax == 1 ? (int)((idx / nx) % ny) : (int)(idx / ((long)nx * ny)));
    out[idx] *= cd(0.0, wavenumber(k, g.n[ax], g.L[ax]));
  }
  fft_nd(g, out, +1);
}

static void observables(const OGrid& g, const OParams& P, double theta, const cd* psi, double* out) {
  long np = npoints(g);
  int nx = g.n[0], ny = g.n[1];
  double hd = 1.0;
  for (int ax = 0; ax < g.dim; ++ax) hd *= 2.0 * g.L[ax] / (double)g.n[ax];
  int nd = g.dim;
  std::vector<cd> D((size_t)5 * nd * np);  // D[(c*nd + ax)*np + idx] = d_ax psi_c
  for (int c = 0; c < 5; ++c)
    for (int ax = 0; ax < nd; ++ax) spectral_derivative(g, psi + c * np, ax, D.data() + ((long)c * nd + ax) * np);
  static const double ell[5] = {2, 1, 0, -1, -2};
  double h6 = std::sqrt(6.0) / 2.0;
  double mass = 0, magn = 0, lz = 0, ekin = 0, epot = 0, eint = 0;
  cd esoc = 0.0;
  for (long idx = 0; idx < np; ++idx) {
    int ix = (int)(idx % nx), iy = (int)((idx / nx) % ny), iz = (int)(idx / ((long)nx * ny));
    double x = coord(g, 0, ix), y = coord(g, 1, iy), z = (nd == 3) ? coord(g, 2, iz) : 0.0;
    double V = trap_rotated(P, theta, x, y, z);
    cd v[5], dx[5], dy[5];
    for (int c = 0; c < 5; ++c) {
      v[c] = psi[c * np + idx];
      dx[c] = D[((long)c * nd + 0) * np + idx];
      dy[c] = D[((long)c * nd + 1) * np + idx];
      double grad2 = 0.0;
      for (int ax = 0; ax < nd; ++ax) grad2 += std::norm(D[((long)c * nd + ax) * np + idx]);
      ekin += 0.5 * grad2;
      mass += std::norm(v[c]);
      magn += ell[c] * std::norm(v[c]);
      epot += V * std::norm(v[c]);
      // Lz psi = -i (x d_y - y d_x) psi
      cd Lz = -I1 * (x * dy[c] - y * dx[c]);
      lz += (std::conj(v[c]) * Lz).real();
    }
    Densities d = densities(v);
    eint += 0.5 * P.c0 * d.rho * d.rho + 0.5 * P.c1 * (d.Fx * d.Fx + d.Fy * d.Fy + d.Fz * d.Fz)
            + 0.5 * P.c2 * std::norm(d.A00);
    // SOC: L+- = i d_y +- d_x; Psi^H S Psi with S of Sec. 1.
    cd Lp[5], Lm[5];
    for (int c = 0; c < 5; ++c) { Lp[c] = I1 * dy[c] + dx[c]; Lm[c] = I1 * dy[c] - dx[c]; }
    cd sps = std::conj(v[0]) * Lm[1]
             + std::conj(v[1]) * (Lp[0] + h6 * Lm[2])
             + std::conj(v[2]) * (h6 * Lp[1] + h6 * Lm[3])
             + std::conj(v[3]) * (h6 * Lp[2] + Lm[4])
             + std::conj(v[4]) * Lp[3];
    esoc += sps;
  }
  out[0] = hd * mass;
  out[1] = hd * (ekin + epot + eint - P.gamma * esoc.real()) - P.Omega * hd * lz;
  out[2] = hd * magn;
  out[3] = hd * lz;
}

// ---------------------------------------------------------------------------
// C ABI for the Python test harness.
// ---------------------------------------------------------------------------
static OGrid mkgrid(int dim, const int* n, const double* L) {
  OGrid g;
  g.dim = dim;
  for (int i = 0; i < 3; ++i) { g.n[i] = (i < dim) ? n[i] : 1; g.L[i] = (i < dim) ? L[i] : 1.0; }
  return g;
}
static OParams mkparams(const double* p) {
  OParams P;
  P.c0 = p[0]; P.c1 = p[1]; P.c2 = p[2]; P.Omega = p[3]; P.gamma = p[4];
  P.gx = p[5]; P.gy = p[6]; P.gz = p[7];
  return P;
}

extern "C" {

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// One d-dimensional transform of a single scalar field in place; sign -1 forward
// (scaled by 1/N^d), +1 inverse (unscaled).
void orc_fft(int dim, const int* n, double* data, int sign) {
  double L[3] = {1, 1, 1};
  OGrid g = mkgrid(dim, n, L);
  fft_nd(g, reinterpret_cast<cd*>(data), sign);
}

void orc_propagator(double Omega, double gamma, double nu_p, double nu_q, double delta, double* out25) {
  propagator(Omega, gamma, nu_p, nu_q, delta, reinterpret_cast<cd*>(out25));
}

void orc_nl_point(const double* params, double V, double delta, double* psi5) {
  OParams P = mkparams(params);
  nl_point(P, V, delta, reinterpret_cast<cd*>(psi5));
}

void orc_linear_step(int dim, const int* n, const double* L, const double* params, double delta, double* psi) {
  linear_step(mkgrid(dim, n, L), mkparams(params), delta, reinterpret_cast<cd*>(psi));
}

void orc_nl_step(int dim, const int* n, const double* L, const double* params, double delta, double theta,
                 double* psi) {
  nl_step(mkgrid(dim, n, L), mkparams(params), delta, theta, reinterpret_cast<cd*>(psi));
}

void orc_rotation_map(int dim, const int* n, const double* L, const double* params, double t, int forward,
                      double* psi) {
  rotation_map(mkgrid(dim, n, L), mkparams(params), t, forward != 0, reinterpret_cast<cd*>(psi));
}

void orc_evolve(int dim, const int* n, const double* L, const double* params, int order, double tau, long nsteps,
                double t0, int mode, double* psi) {
  evolve(mkgrid(dim, n, L), mkparams(params), order, tau, nsteps, t0, mode, reinterpret_cast<cd*>(psi));
}

// Adjoint: gT = 2 dJ/d conj(Phi(T)) -> g0 = 2 dJ/d conj(Psi0) and
// dpar = dJ/d(gamma, Omega, c0, c1, c2); checkpoints every K steps.
void orc_adjoint(int dim, const int* n, const double* L, const double* params, int order, double tau, long nsteps,
                 double t0, const double* psi0, const double* gT, double* g0, double* dpar, long K) {
  adjoint(mkgrid(dim, n, L), mkparams(params), order, tau, nsteps, t0, reinterpret_cast<const cd*>(psi0),
          reinterpret_cast<const cd*>(gT), reinterpret_cast<cd*>(g0), dpar, K);
}

void orc_observables(int dim, const int* n, const double* L, const double* params, double theta, const double* psi,
                     double* out4) {
  observables(mkgrid(dim, n, L), mkparams(params), theta, reinterpret_cast<const cd*>(psi), out4);
}

}  // extern "C"

// Kernel argument block and launchers shared by the host library and the kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace sgp {

enum { X_FIRST = 0, X_MID = 1, X_LAST = 2, X_NLONLY = 3, C_PROP = 4, C_FWD = 5, C_INV = 6,
       // adjoints: of X_FIRST (iFFT, NL adjoint), of X_MID (iFFT, NL adjoint, FFT),
       // of X_LAST (NL adjoint, FFT), of C_PROP (FFT, P^H and parameter partials, iFFT)
       XA_FIRST = 7, XA_MID = 8, XA_LAST = 9, C_ADJ = 10,
       // rotation mapping (RSDA shears, Sec. 3.1): FFT, phase exp(i nu a w), inverse FFT
       // along x (w = y of the line) or along y (w = x of the column); and bare
       // transforms along x (for the lab-frame Algorithm 1 mode)
       X_SHEAR = 11, C_SHEAR = 12, X_FWD = 13, X_INV = 14,
       // 3D linear substep with the propagator split by axis (its spin part depends on
       // (nu_p, nu_q) only, Sec. 3.1's 3D remark, so it commutes with the z transform):
       // y-lines FFT then exp(-i d (nu_x^2 + nu_y^2)/2) exp(i d Q) / N^3 (C_FSPIN), and
       // z-lines FFT, exp(-i d nu_z^2/2), inverse FFT per component (C_KIN)
       C_FSPIN = 15, C_KIN = 16 };
enum { NGRAD = 5 };  // adjoint parameter slots: gamma, Omega, c0, c1, c2
// observables passes; OBS_JX / OBS_JY: the x-line and y-column parts of <u, J_z v>
enum { OBS_X = 0, OBS_Y = 1, OBS_Z = 2, OBS_JX = 3, OBS_JY = 4 };
enum { CLOCK_ARG = 0, CLOCK_DEVICE = 1 };
enum { NOBS = 28 };  // partial sums per block of the observables kernels

// One pass over lines of the state ([nz][ny][nx][5] complex).  X kinds use the
// x-line fields, column kinds (C_*) the column fields; both read the tables.
struct PassArgs {
  // x-lines
  long nlines;           // ny * nz (a z-slab launch: ny * its planes)
  int ny;
  int z0;                // first plane of a z-slab launch of an x-pass (trap's z coordinate)
  // columns (lines along y or z)
  long stride;           // element stride along the line (5 nx or 5 nx ny)
  long ncols;            // lines along the contiguous x axis (nx)
  long nouter;           // outer slabs (2D y-lines: 1; 3D y-lines: nz; z-lines: ny)
  long outer_stride;     // elements between outer slabs
  int dim;
  int n_q;               // points along y (the q axis of the propagator)
  // FFT twiddles of the line's axis
  const void* tw_fwd;
  const void* tw_inv;
  // propagator
  const void* cs;        // (C - 1, S) per (q, p)
  const void* kin_a;     // exp(-i d nu^2/2) - 1 along x
  const void* kin_o;     // ... along the outer axis (3D z-lines: y)
  const void* kin_l;     // ... along the line
  double nu_scale_a;     // pi / Lx
  double nu_scale_q;     // pi / Ly
  double nu_scale_l;     // pi / L of the line's axis (observables)
  double norm;           // 1 / N^d
  // geometry and physics
  double L[3], h[3];     // half-widths and spacings (unused axes: 0)
  double g2[3];          // squared trap frequencies (gz^2 = 0 in 2D)
  double Omega, gamma;
  double c0, c0p, c1, c2;  // c0, c0 + c2/5, c1, c2
  double d;              // substep duration (nonlinear: the flow time; linear: the clock advance)
  double* clock;         // device clock s of the rotating frame
  double s_arg;          // clock value passed by the host (CLOCK_ARG; then written to *clock)
  int clock_mode;
  int advance_clock;
  // batched passes
  void* state;           // the instance's state
  int n_line;            // length of the pass's lines
  // adjoint support
  void* store;           // forward: where to write the pointwise-stage input (or null)
  const void* fwd;       // adjoint: the stored pointwise-stage input of the forward pass
  double* gacc;          // adjoint: per-block parameter slots [block][NGRAD], accumulated
  // rotation mapping
  double shear;          // shear coefficient a: f(x, y) <- f(x + a y, y) (x) or f(x, y + a x) (y)
  double cphase;         // component phase: psi_l *= exp(i l cphase) when cphase_on
  int cphase_on;
};

// Register plans of the FFT line kernels: E elements per thread of a line of
// length N (the radix sequence follows from N and E, see Plan<N, E>).  E = 8 for
// powers of two and 12 for 3 * 2^k (192, 384, 768) are the defaults; the others are
// autotuning alternatives (E = 4: twice the threads, E = 16 / 24: more registers per
// thread; E = 24 needs more LDS than a CU has in FP64, so it is FP32 only).
// esize: bytes of one real (4 or 8).
constexpr bool plan_ok(int n, int e, int esize) {
  return (n == 192 || n == 384 || n == 768) ? (e == 12 || (e == 24 && esize == 4))
                    : ((n == 16 || n == 32 || n == 64 || n == 128 || n == 256 || n == 512) &&
                       (e == 4 || e == 8 || (e == 16 && n >= 64)));
}
constexpr int default_elems(int n) { return n % 3 == 0 ? 12 : 8; }
constexpr int kPlanElems[] = {4, 8, 12, 16, 24};
// lines per block of the pass kernels for line length n with plan width e
constexpr int lines_per_block(int n, int e) { return n / e >= 64 ? 1 : 64 / (n / e); }
// lines per block of the observables kernels (their LDS tile holds psi and its
// derivative: at most 512 points per block)
constexpr int obs_lines_per_block(int n, int e) {
  int w = lines_per_block(n, e);
  while (w > 1 && w * n > 512) w /= 2;
  return w;
}

// ev: null, or a start / end event pair stamped by the kernel's dispatch
template <typename T>
hipError_t launch_pass(int kind, void* psi, const PassArgs& a, int n, int e, hipStream_t st,
                       const hipEvent_t* ev = nullptr);
template <typename T>
hipError_t launch_obs(int kind, const void* psi, const PassArgs& a, int n, int e, double* part, hipStream_t st);
// Deterministic sum of block partials: out[q] = sum over b < nb of part[b nq + q],
// q < nq, in a fixed order (one block per q).
hipError_t launch_sum_partials(const double* part, long nb, int nq, double* out, hipStream_t st);
template <typename T>
hipError_t launch_build_tables(void* cs, void* kin_x, void* kin_y, void* kin_z, const int* n, const double* L,
                               int dim, double Omega, double gamma, double d, hipStream_t st);
// Plans the batched ensemble kernels run: the 320-thread geometry (n/e <= 64).
constexpr bool batched_plan_ok(int n, int e, int esize) { return n >= 64 && plan_ok(n, e, esize) && n / e <= 64; }
// batched passes of one plan width e: items = int2 (instance, tile) of instances
// using width e along the pass's axis, args = PassArgs per instance
// nmax: the longest line among the instances of the launch
template <typename T>
hipError_t launch_pass_batched(int kind, int e, const void* items, const void* args, long nitems, int nmax,
                               hipStream_t st);

// per-plan-width launchers, each (T, E) compiled in its own translation unit
template <typename T, int E>
hipError_t launch_pass_e(int kind, void* psi, const PassArgs& a, int n, hipStream_t st, const hipEvent_t* ev);
template <typename T, int E>
hipError_t launch_obs_e(int kind, const void* psi, const PassArgs& a, int n, double* part, hipStream_t st);

}  // namespace sgp

// Kernel argument blocks and launchers shared by the host library and the kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace sgp {

enum { X_FIRST = 0, X_MID = 1, X_LAST = 2, X_NLONLY = 3 };
enum { C_PROP = 0, C_FWD = 1, C_INV = 2 };
enum { CLOCK_ARG = 0, CLOCK_DEVICE = 1 };

// X-pass (lines along x, nonlinear flow in physical space).
struct XArgs {
  long comp_stride;      // elements between components (nx*ny*nz)
  long nlines;           // lines along x (ny*nz)
  int ny;                // lines per z-slab
  const void* tw_fwd;    // twiddle tables of the x plan
  const void* tw_inv;
  double L[3], h[3];     // half-widths and spacings (z entries unused in 2D: L = h = 0)
  double g2[3];          // squared trap frequencies (gz^2 = 0 in 2D)
  double Omega;
  double d;              // nonlinear substep duration
  double c0p, c1, c2;    // c0 + c2/5, c1, c2
  double* clock;         // device clock (s of the rotating frame)
  double s_arg;          // clock value when clock_mode == CLOCK_ARG (then written to *clock)
  int clock_mode;
};

// Column pass (lines along y or z, strided).
struct CArgs {
  long comp_stride;      // elements between components
  long stride;           // element stride along the line
  long ncols;            // lines along the contiguous x axis (nx)
  long nouter;           // number of outer slabs
  long outer_stride;     // elements between outer slabs
  int dim;
  int n_q;               // points along y (the q axis of the propagator)
  const void* tw_fwd;
  const void* tw_inv;
  const void* cs;        // (C, S) propagator table, [ny][nx] pairs
  const void* kin_a;     // kinetic phase along x (with the 1/N^d scale)
  const void* kin_o;     // kinetic phase along the outer axis (3D: y)
  const void* kin_l;     // kinetic phase along the line axis
  double nu_scale_a;     // pi / Lx
  double nu_scale_q;     // pi / Ly
  double Omega, gamma;
  double norm;           // 1/N^d
  double d;              // linear substep duration (for the clock)
  double* clock;
  int advance_clock;
};

template <typename T>
hipError_t launch_xpass(int mode, void* psi, const XArgs& a, int nx, long nlines, hipStream_t st);
template <typename T>
hipError_t launch_colpass(int mode, void* psi, const CArgs& a, int n, hipStream_t st);
template <typename T>
hipError_t launch_build_tables(void* cs, void* kin_x, void* kin_y, void* kin_z, const int* n, const double* L,
                               int dim, double Omega, double gamma, double d, hipStream_t st);
template <typename T>
hipError_t launch_mass_magn(const void* psi, long npts, double* part, int nblocks, hipStream_t st);

}  // namespace sgp

// Host side of the C ABI declared in include/sgp.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/sgp.h"
#include "sgp_device.hpp"
#include "sgp_kernels.hpp"

using namespace sgp;

// Fixed device scratch of sgp_observables_device (see there): block partials and
// their sums; one copy per GPU, held until the process ends.
constexpr size_t kObsScratchBytes = size_t(8) << 20;
static __device__ __align__(256) double scratch[kObsScratchBytes / sizeof(double)];

namespace {

const double kPi = 3.14159265358979323846264338327950288;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

template <int... Rs>
std::vector<int> radix_list(RadixList<Rs...>) { return {Rs...}; }

template <int N, int E>
std::vector<int> plan_of(bool fwd) {
  return fwd ? radix_list(typename Plan<N, E>::fwd{}) : radix_list(typename Plan<N, E>::inv{});
}

bool supported_n(int n) {
  return n == 16 || n == 32 || n == 64 || n == 128 || n == 192 || n == 256 || n == 384 || n == 512 || n == 768;
}

std::vector<int> plan_radices(int n, int e, bool fwd) {
#define SGP_PLAN(NN, EE) \
  if (n == NN && e == EE) return plan_of<NN, EE>(fwd);
  SGP_PLAN(16, 4) SGP_PLAN(32, 4) SGP_PLAN(64, 4) SGP_PLAN(128, 4) SGP_PLAN(256, 4) SGP_PLAN(512, 4)
  SGP_PLAN(16, 8) SGP_PLAN(32, 8) SGP_PLAN(64, 8) SGP_PLAN(128, 8) SGP_PLAN(256, 8) SGP_PLAN(512, 8)
  SGP_PLAN(64, 16) SGP_PLAN(128, 16) SGP_PLAN(256, 16) SGP_PLAN(512, 16)
  SGP_PLAN(384, 12) SGP_PLAN(384, 24) SGP_PLAN(192, 12) SGP_PLAN(192, 24) SGP_PLAN(768, 12) SGP_PLAN(768, 24)
#undef SGP_PLAN
  return {};
}

// Plan widths compiled for line length n (the default first).
std::vector<int> plan_widths(int n, int esize) {
  std::vector<int> out{default_elems(n)};
  for (int e : kPlanElems)
    if (e != default_elems(n) && plan_ok(n, e, esize)) out.push_back(e);
  return out;
}

// Twiddle table of a plan: for each pass with NS > 1, for r = 1..R-1 and k in
// [0, NS), the values exp(-2 pi i r k / (NS R)) (the kernels conjugate them for the
// inverse).
std::vector<std::complex<double>> twiddle_table(const std::vector<int>& radices) {
  std::vector<std::complex<double>> out;
  int ns = 1;
  for (int R : radices) {
    if (ns > 1)
      for (int r = 1; r < R; ++r)
        for (int k = 0; k < ns; ++k) {
          double a = -2.0 * kPi * (double)r * (double)k / (double)(ns * R);
          out.emplace_back(std::cos(a), std::sin(a));
        }
    ns *= R;
  }
  return out;
}

}  // namespace

struct sgp_ctx {
  sgp_grid g;
  sgp_params p;
  int dtype;
  hipStream_t st;
  size_t esize;  // bytes of one real

  char* ws = nullptr;
  size_t ws_bytes = 0;
  size_t total = 0;
  size_t off_tw[3][2];
  size_t off_cs[4];      // (C - 1, S) table per distinct linear substep length
  size_t off_kin[4][3];
  size_t off_clock;
  size_t off_part;
  size_t off_red;        // on-device sums of the observables' block partials (3 x NOBS)
  size_t off_gacc;
  long ngacc = 0;  // blocks with a gradient slot

  // register plan width E of the passes along each axis
  int plan_e[3] = {0, 0, 0};
  // 3D linear substep: 0 = FFT y, whole propagator in the z-pass, iFFT y (default);
  // 1 = FFT y with the spin part in the y-pass, z kinetic phase in the z-pass, iFFT y
  int lin_split = 0;
  // 0: evolve Phi in the rotating frame (default); 1: Algorithm 1 literally (lab frame)
  int frame = 0;

  int scheme = 0;
  double tau = 0.0;
  int nprop = 0;
  double dprop[4] = {0, 0, 0, 0};
  bool have_prop = false;
  double t = 0.0;
  std::string err;

  // replay of the periodic part of sgp_step: graphs of 2^k whole steps
  // (k = 0..kGraphLevels-1), all captured together for the state pointer gpsi, so
  // that any number of body steps replays from graphs (its binary digits)
  static constexpr int kGraphLevels = 6;
  hipStream_t cap = nullptr;
  hipGraphExec_t gexec[kGraphLevels] = {};
  void* gpsi = nullptr;
  bool use_graph = true;
  // 3D, split 0: the graph body runs its z-local passes (inverse y, X, forward y)
  // per z-slab, the slabs alternating between two streams (0: off)
  int slabs = 0;
  hipStream_t cap2 = nullptr;
  hipEvent_t pev[2] = {nullptr, nullptr};

  // measurement hook (sgp_time_pass with SGP_TIME_STEPS): while it is set, every
  // launch of pass `tev_pass` takes the next event pair of tev
  std::vector<hipEvent_t> tev;
  int tev_pass = -1;
  size_t tev_used = 0;

  long npts() const { return (long)g.n[0] * g.n[1] * (g.dim == 3 ? g.n[2] : 1); }
  int elems(int axis) const { return plan_e[axis]; }
  void* at(size_t off) const { return ws + off; }
};

namespace {

thread_local std::string g_create_err;

int fail(sgp_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  else g_create_err = msg;
  return code;
}

int hip_fail(sgp_ctx* c, hipError_t e, const char* where) {
  return fail(c, SGP_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

// The next event pair for a launch of pass `pass` (numbered as in sgp_time_pass)
// while a step timing runs; null otherwise.
const hipEvent_t* timing_events(sgp_ctx* c, int pass) {
  if (pass < 0 || pass != c->tev_pass || 2 * c->tev_used + 1 >= c->tev.size()) return nullptr;
  return &c->tev[2 * c->tev_used++];
}

// TS4 coefficients (Sec. 3.3): a1 = a4, a2 = a3 on the nonlinear flow; b1 = b3, b2 on
// the linear flow.
struct TS4 {
  double a1, a2, b1, b2;
  TS4() {
    double c = std::cbrt(2.0), den = 2.0 - c;
    a1 = 1.0 / (2.0 * den);
    a2 = (1.0 - c) / (2.0 * den);
    b1 = 1.0 / den;
    b2 = -c / den;
  }
};

template <typename T>
hipError_t upload_twiddles(sgp_ctx* c) {
  for (int ax = 0; ax < c->g.dim; ++ax) {
    for (int dir = 0; dir < 2; ++dir) {
      auto tab = twiddle_table(plan_radices(c->g.n[ax], c->elems(ax), dir == 0));
      // each twiddle as a (hi, lo) pair: hi = w rounded to T, lo = (w - hi) rounded
      std::vector<T> buf(4 * tab.size() + 4);
      for (size_t i = 0; i < tab.size(); ++i) {
        T hr = (T)tab[i].real(), hi = (T)tab[i].imag();
        buf[4 * i] = hr;
        buf[4 * i + 1] = hi;
        buf[4 * i + 2] = (T)(tab[i].real() - (double)hr);
        buf[4 * i + 3] = (T)(tab[i].imag() - (double)hi);
      }
      if (tab.empty()) continue;
      hipError_t e = hipMemcpyAsync(c->at(c->off_tw[ax][dir]), buf.data(), sizeof(T) * 4 * tab.size(),
                                    hipMemcpyHostToDevice, c->st);
      if (e != hipSuccess) return e;
      e = hipStreamSynchronize(c->st);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

// Fields shared by every pass of a context.
PassArgs base_args(const sgp_ctx* c) {
  PassArgs a;
  std::memset(&a, 0, sizeof(a));
  const int nx = c->g.n[0], ny = c->g.n[1], nz = c->g.dim == 3 ? c->g.n[2] : 1;
  a.nlines = (long)ny * nz;
  a.ny = ny;
  a.ncols = nx;
  a.dim = c->g.dim;
  a.n_q = ny;
  for (int i = 0; i < 3; ++i) {
    bool on = i < c->g.dim;
    a.L[i] = on ? c->g.L[i] : 0.0;
    a.h[i] = on ? 2.0 * c->g.L[i] / c->g.n[i] : 0.0;
  }
  a.g2[0] = c->p.gx * c->p.gx;
  a.g2[1] = c->p.gy * c->p.gy;
  a.g2[2] = c->g.dim == 3 ? c->p.gz * c->p.gz : 0.0;
  a.Omega = c->p.Omega;
  a.gamma = c->p.gamma;
  a.c0 = c->p.c0;
  a.c0p = c->p.c0 + c->p.c2 / 5.0;
  a.c1 = c->p.c1;
  a.c2 = c->p.c2;
  a.nu_scale_a = kPi / c->g.L[0];
  a.nu_scale_q = kPi / c->g.L[1];
  a.norm = 1.0 / (double)c->npts();
  a.clock = (double*)c->at(c->off_clock);
  (void)nz;
  return a;
}

// Column geometry for lines along `axis` (1 = y, 2 = z).
void column_geometry(const sgp_ctx* c, int axis, PassArgs& a) {
  const int nx = c->g.n[0], ny = c->g.n[1], nz = c->g.dim == 3 ? c->g.n[2] : 1;
  if (axis == 1) {
    a.stride = 5L * nx;
    a.nouter = nz;
    a.outer_stride = 5L * nx * ny;
  } else {
    a.stride = 5L * nx * ny;
    a.nouter = ny;
    a.outer_stride = 5L * nx;
  }
  a.tw_fwd = c->at(c->off_tw[axis][0]);
  a.tw_inv = c->at(c->off_tw[axis][1]);
  a.nu_scale_l = kPi / c->g.L[axis];
}

template <typename T>
hipError_t run_xpass(sgp_ctx* c, hipStream_t st, int mode, void* psi, double d, int clock_mode, double s_arg,
                     const hipEvent_t* ev = nullptr) {
  PassArgs a = base_args(c);
  a.tw_fwd = c->at(c->off_tw[0][0]);
  a.tw_inv = c->at(c->off_tw[0][1]);
  a.d = d;
  a.s_arg = s_arg;
  a.clock_mode = clock_mode;
  if (!ev) ev = timing_events(c, mode == X_MID ? 0 : -1);
  return launch_pass<T>(mode, psi, a, c->g.n[0], c->elems(0), st, ev);
}

template <typename T>
hipError_t run_colpass(sgp_ctx* c, hipStream_t st, int mode, int axis, void* psi, int table, double d,
                       const hipEvent_t* ev = nullptr) {
  PassArgs a = base_args(c);
  column_geometry(c, axis, a);
  a.cs = c->at(c->off_cs[table]);
  a.kin_a = c->at(c->off_kin[table][0]);
  a.kin_o = c->at(c->off_kin[table][1]);
  a.kin_l = c->at(c->off_kin[table][axis]);
  a.d = d;
  a.advance_clock = (mode == C_PROP || mode == C_FSPIN) ? 1 : 0;
  if (!ev) {
    int pid = -1;
    if (axis == 1 && (mode == C_PROP || mode == C_FWD || mode == C_FSPIN)) pid = 1;
    else if (axis == 2 && (mode == C_PROP || mode == C_KIN)) pid = 2;
    else if (axis == 1 && mode == C_INV) pid = 3;
    ev = timing_events(c, pid);
  }
  return launch_pass<T>(mode, psi, a, c->g.n[axis], c->elems(axis), st, ev);
}

// Store-mode and adjoint variants of the passes.
template <typename T>
hipError_t run_xpass_ex(sgp_ctx* c, int kind, void* psi, double d, int clock_mode, double s_arg, void* store,
                        const void* fwd) {
  PassArgs a = base_args(c);
  a.tw_fwd = c->at(c->off_tw[0][0]);
  a.tw_inv = c->at(c->off_tw[0][1]);
  a.d = d;
  a.s_arg = s_arg;
  a.clock_mode = clock_mode;
  a.store = store;
  a.fwd = fwd;
  a.gacc = (double*)c->at(c->off_gacc);
  return launch_pass<T>(kind, psi, a, c->g.n[0], c->elems(0), c->st);
}

template <typename T>
hipError_t run_colpass_ex(sgp_ctx* c, int kind, int axis, void* psi, int table, double d, void* store,
                          const void* fwd) {
  PassArgs a = base_args(c);
  column_geometry(c, axis, a);
  a.cs = c->at(c->off_cs[table]);
  a.kin_a = c->at(c->off_kin[table][0]);
  a.kin_o = c->at(c->off_kin[table][1]);
  a.kin_l = c->at(c->off_kin[table][axis]);
  a.d = d;
  a.advance_clock = (kind == C_PROP) ? 1 : 0;
  a.store = store;
  a.fwd = fwd;
  a.gacc = (double*)c->at(c->off_gacc);
  return launch_pass<T>(kind, psi, a, c->g.n[axis], c->elems(axis), c->st);
}

// One exact linear substep on x-transformed data: 2D Y-pass; 3D Y1 (FFT along y, the
// spin part of the propagator exp(i d Q(nu_p, nu_q)) with the x and y kinetic phases
// and 1/N^3), Z (FFT along z, the z kinetic phase, inverse FFT) and Y2 (inverse FFT
// along y).  The spin part depends on (nu_p, nu_q) only (Sec. 3.1, 3D remark), so it
// commutes with the z transform and runs in the y-pass, whose memory time leaves
// room for it; the z-pass then works per component.  (The differentiable path,
// sgp_step_store and the adjoint, keeps the whole propagator in the z-pass.)
template <typename T>
hipError_t run_linear(sgp_ctx* c, hipStream_t st, void* psi, int table, double d) {
  if (c->g.dim == 2) return run_colpass<T>(c, st, C_PROP, 1, psi, table, d);
  hipError_t e = run_colpass<T>(c, st, c->lin_split ? C_FSPIN : C_FWD, 1, psi, table, d);
  if (e != hipSuccess) return e;
  e = run_colpass<T>(c, st, c->lin_split ? C_KIN : C_PROP, 2, psi, table, d);
  if (e != hipSuccess) return e;
  return run_colpass<T>(c, st, C_INV, 1, psi, table, d);
}

// One step of a composition (Sec. 3.3): nonlinear flows A[j] tau and linear flows
// B[j] tau alternate, N(A[0]) L(B[0]) N(A[1]) ... L(B[m-2]) N(A[m-1]) (B[m-1] = 0);
// tab[j] is the propagator table of L(B[j]) and props the distinct B values (one
// table each).  TS6 is the triple jump S4(z1) S4(z0) S4(z1), z1 = 1/(2 - 2^(1/5)),
// z0 = -2^(1/5) z1, the nonlinear flows that meet at a join being one flow.
struct Composition {
  std::vector<double> A, B, props;
  std::vector<int> tab;
};

Composition composition(int scheme) {
  Composition k;
  if (scheme == SGP_TS2) {
    k.A = {0.5, 0.5};
    k.B = {1.0, 0.0};
  } else {
    TS4 f;
    const std::vector<double> a4 = {f.a1, f.a2, f.a2, f.a1}, b4 = {f.b1, f.b2, f.b1, 0.0};
    if (scheme == SGP_TS4) {
      k.A = a4;
      k.B = b4;
    } else {
      const double q = std::pow(2.0, 0.2);
      const double z[3] = {1.0 / (2.0 - q), -q / (2.0 - q), 1.0 / (2.0 - q)};
      for (int fi = 0; fi < 3; ++fi)
        for (int j = 0; j < 4; ++j) {
          if (j == 0 && fi > 0) {
            k.A.back() += z[fi] * a4[0];
            k.B.back() = z[fi] * b4[0];
            continue;
          }
          k.A.push_back(z[fi] * a4[j]);
          k.B.push_back(z[fi] * b4[j]);
        }
    }
  }
  for (double b : k.B) {
    if (b == 0.0) { k.tab.push_back(-1); continue; }
    size_t i = 0;
    while (i < k.props.size() && k.props[i] != b) ++i;
    if (i == k.props.size()) k.props.push_back(b);
    k.tab.push_back((int)i);
  }
  return k;
}

// Substep schedule of nsteps steps with merged adjacent nonlinear substeps (the last
// flow of a step and the first of the next share the clock): nl has one more entry
// than lin; lin_tab selects the propagator table.
void schedule(const sgp_ctx* c, long nsteps, std::vector<double>& nl, std::vector<double>& lin,
              std::vector<int>& lin_tab) {
  const double tau = c->tau;
  nl.clear(); lin.clear(); lin_tab.clear();
  const Composition k = composition(c->scheme);
  const size_t m = k.A.size();
  nl.push_back(k.A[0] * tau);
  for (long n = 0; n < nsteps; ++n)
    for (size_t j = 0; j + 1 < m; ++j) {
      lin.push_back(k.B[j] * tau);
      lin_tab.push_back(k.tab[j]);
      if (j + 2 < m) nl.push_back(k.A[j + 1] * tau);
      else nl.push_back(n + 1 < nsteps ? (k.A[m - 1] + k.A[0]) * tau : k.A[m - 1] * tau);
    }
}

// The periodic middle of a call: one whole step that starts after a merged
// nonlinear substep and ends with the next merged one (all clock reads on device).
template <typename T>
hipError_t enqueue_body(sgp_ctx* c, hipStream_t st, void* psi, int nbody) {
  std::vector<double> nl, lin;
  std::vector<int> tab;
  schedule(c, 2, nl, lin, tab);  // the second step of a two-step schedule is a body step
  const size_t per = lin.size() / 2;
  for (int b = 0; b < nbody; ++b)
    for (size_t k = per; k < 2 * per; ++k) {
      hipError_t e = run_linear<T>(c, st, psi, tab[k], lin[k]);
      if (e != hipSuccess) return e;
      // the body's last nonlinear substep is the merged one (2 a1 tau / tau)
      const double d = (k + 1 == 2 * per) ? nl[per] : nl[k + 1];
      e = run_xpass<T>(c, st, X_MID, psi, d, CLOCK_DEVICE, 0.0);
      if (e != hipSuccess) return e;
    }
  return hipSuccess;
}

// One z-local pass over the planes [z0, z1) of a 3D state: the x-pass (X_MID, the
// clock on the device) or a y-pass transform (C_FWD / C_INV).  A z-slab is a
// contiguous part of the state, so the pass runs on it as on a grid of z1 - z0
// planes; only the x-pass's trap potential needs the planes' position (z0).
template <typename T>
hipError_t run_slab_pass(sgp_ctx* c, hipStream_t st, int kind, void* psi, int z0, int z1, double d) {
  PassArgs a = base_args(c);
  const int nx = c->g.n[0], ny = c->g.n[1];
  void* p = (char*)psi + (size_t)z0 * ny * nx * 5 * 2 * c->esize;
  a.d = d;
  if (kind == X_MID) {
    a.tw_fwd = c->at(c->off_tw[0][0]);
    a.tw_inv = c->at(c->off_tw[0][1]);
    a.clock_mode = CLOCK_DEVICE;
    a.nlines = (long)(z1 - z0) * ny;
    a.z0 = z0;
    return launch_pass<T>(kind, p, a, nx, c->elems(0), st, nullptr);
  }
  column_geometry(c, 1, a);
  a.nouter = z1 - z0;
  return launch_pass<T>(kind, p, a, ny, c->elems(1), st, nullptr);
}

// enqueue_body with the z-local passes in z-slabs (3D, split 0): the inverse y-pass,
// the x-pass and the next forward y-pass act on each z-plane alone, so between two
// z-passes they run slab by slab, even slabs on st and odd ones on st2 (started one
// inverse y-pass later), and the bandwidth-bound y-passes of one slab overlap the
// VALU-bound x-pass of another.  The same kernels as enqueue_body on the same
// lines: bitwise the same result.
template <typename T>
hipError_t enqueue_body_slabs(sgp_ctx* c, hipStream_t st, hipStream_t st2, void* psi, int nbody) {
  std::vector<double> nl, lin;
  std::vector<int> tab;
  schedule(c, 2, nl, lin, tab);
  const size_t per = lin.size() / 2;
  const int S = c->slabs, dz = c->g.n[2] / S;
  hipError_t e = run_colpass<T>(c, st, C_FWD, 1, psi, tab[per], lin[per]);
  for (int b = 0; b < nbody && e == hipSuccess; ++b)
    for (size_t k = per; k < 2 * per && e == hipSuccess; ++k) {
      e = run_colpass<T>(c, st, C_PROP, 2, psi, tab[k], lin[k]);
      const double d = (k + 1 == 2 * per) ? nl[per] : nl[k + 1];
      const bool fwd_next = !(b + 1 == nbody && k + 1 == 2 * per);
      for (int sl = 0; sl < S && e == hipSuccess; ++sl) {
        hipStream_t q = (sl & 1) ? st2 : st;
        const int z0 = sl * dz, z1 = z0 + dz;
        e = run_slab_pass<T>(c, q, C_INV, psi, z0, z1, 0.0);
        if (e == hipSuccess && sl == 0) {  // fork: st2 starts after the z-pass and slab 0's inverse y-pass
          e = hipEventRecord(c->pev[0], st);
          if (e == hipSuccess) e = hipStreamWaitEvent(st2, c->pev[0], 0);
        }
        if (e == hipSuccess) e = run_slab_pass<T>(c, q, X_MID, psi, z0, z1, d);
        if (e == hipSuccess && fwd_next) e = run_slab_pass<T>(c, q, C_FWD, psi, z0, z1, 0.0);
      }
      if (e == hipSuccess) e = hipEventRecord(c->pev[1], st2);  // join
      if (e == hipSuccess) e = hipStreamWaitEvent(st, c->pev[1], 0);
    }
  return e;
}

bool slab_body(const sgp_ctx* c) { return c->slabs >= 2 && c->g.dim == 3 && c->lin_split == 0; }

void drop_graph(sgp_ctx* c) {
  for (auto& g : c->gexec) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
  c->gpsi = nullptr;
}

// Capture the body graphs of 1, 2, 4, ..., 2^(kGraphLevels-1) steps for state psi
// (all at once, so that a later call with another step count captures nothing).
template <typename T>
hipError_t get_graphs(sgp_ctx* c, void* psi) {
  if (c->gpsi == psi && c->gexec[0]) return hipSuccess;
  drop_graph(c);
  hipError_t e;
  if (!c->cap) {
    e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
  }
  const bool slabs = slab_body(c);
  if (slabs && !c->cap2) {
    e = hipStreamCreateWithFlags(&c->cap2, hipStreamNonBlocking);
    for (int i = 0; i < 2 && e == hipSuccess; ++i)
      if (!c->pev[i]) e = hipEventCreateWithFlags(&c->pev[i], hipEventDisableTiming);
    if (e != hipSuccess) return e;
  }
  for (int k = 0; k < sgp_ctx::kGraphLevels; ++k) {
    e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) { drop_graph(c); return e; }
    hipError_t e1 = slabs ? enqueue_body_slabs<T>(c, c->cap, c->cap2, psi, 1 << k)
                          : enqueue_body<T>(c, c->cap, psi, 1 << k);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(c->cap, &g);
    if (e1 != hipSuccess || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      drop_graph(c);
      return e1 != hipSuccess ? e1 : e;
    }
    e = hipGraphInstantiate(&c->gexec[k], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) { c->gexec[k] = nullptr; drop_graph(c); return e; }
    // stage the executable graph on the device now, not at its first replay
    e = hipGraphUpload(c->gexec[k], c->st);
    if (e != hipSuccess) { drop_graph(c); return e; }
  }
  c->gpsi = psi;
  return hipSuccess;
}

template <typename T>
int step_impl(sgp_ctx* c, void* psi, long nsteps) {
  std::vector<double> nl, lin;
  std::vector<int> tab;
  schedule(c, 1, nl, lin, tab);  // a single step: first and last nonlinear substeps unmerged
  hipError_t e = run_xpass<T>(c, c->st, X_FIRST, psi, nl[0], CLOCK_ARG, c->t);
  if (e != hipSuccess) return hip_fail(c, e, "X-pass launch");
  long nbody = nsteps - 1;
  if (c->use_graph && nbody > 0) {
    // the body steps replayed from graphs: nbody / 2^(L-1) replays of the largest,
    // then one replay per binary digit of the remainder (largest first)
    e = get_graphs<T>(c, psi);
    if (e != hipSuccess) return hip_fail(c, e, "graph capture");
    const int top = sgp_ctx::kGraphLevels - 1;
    for (long i = 0; i < (nbody >> top); ++i) {
      e = hipGraphLaunch(c->gexec[top], c->st);
      if (e != hipSuccess) return hip_fail(c, e, "graph launch");
    }
    for (int k = top - 1; k >= 0; --k)
      if ((nbody >> k) & 1) {
        e = hipGraphLaunch(c->gexec[k], c->st);
        if (e != hipSuccess) return hip_fail(c, e, "graph launch");
      }
    nbody = 0;
  }
  if (nbody > 0) {
    e = enqueue_body<T>(c, c->st, psi, (int)nbody);
    if (e != hipSuccess) return hip_fail(c, e, "step launch");
  }
  // the last step: its linear substeps, then the unmerged final nonlinear substep
  for (size_t k = 0; k < lin.size(); ++k) {
    e = run_linear<T>(c, c->st, psi, tab[k], lin[k]);
    if (e != hipSuccess) return hip_fail(c, e, "linear pass launch");
    e = run_xpass<T>(c, c->st, k + 1 == lin.size() ? X_LAST : X_MID, psi, nl[k + 1], CLOCK_DEVICE, 0.0);
    if (e != hipSuccess) return hip_fail(c, e, "X-pass launch");
  }
  c->t += (double)nsteps * c->tau;
  return SGP_OK;
}

// Average duration of one pass launched reps times back to back on the context
// stream, bracketed by HIP events.  pass: 0 X-pass (mid form), 1 linear pass along
// y (2D: with the propagator; 3D: forward y), 2 z-pass with the propagator (3D),
// 3 inverse y-pass (3D).
// ev: null, or an event pair that the dispatch stamps with the kernel's start and end.
template <typename T>
hipError_t launch_timed_pass(sgp_ctx* c, void* psi, int pass, bool first, const hipEvent_t* ev = nullptr) {
  // X-pass as inside a step: the clock from the device slots (set by the first launch)
  if (pass == 0)
    return run_xpass<T>(c, c->st, X_MID, psi, c->dprop[0], first ? CLOCK_ARG : CLOCK_DEVICE, c->t, ev);
  if (pass == 1) return run_colpass<T>(c, c->st, c->g.dim == 2 ? C_PROP : (c->lin_split ? C_FSPIN : C_FWD), 1, psi, 0,
                                       0.0, ev);
  if (pass == 2) return run_colpass<T>(c, c->st, c->lin_split ? C_KIN : C_PROP, 2, psi, 0, 0.0, ev);
  return run_colpass<T>(c, c->st, C_INV, 1, psi, 0, 0.0, ev);
}

// Events that a dispatch stamps for per-kernel timing: without the system-scope
// fence, so that stamping them does not write back and invalidate the caches
// between kernels (the graph replay of a step does not either); they are only read
// by hipEventElapsedTime after a synchronisation on a later event.
constexpr unsigned kTimingEventFlags = hipEventDisableSystemFence;

// In-step timing: reps rounds of the passes of one linear + nonlinear substep in
// step order (2D: y, X; 3D: y, z, inverse y, X); every launch of the timed pass
// carries an event pair that its dispatch stamps with the kernel's start and end
// (no marker packets between the kernels); the average of those durations.
template <typename T>
int time_pass_in_step(sgp_ctx* c, void* psi, int pass, int reps, double* avg_ms) {
  const std::vector<int> order = c->g.dim == 2 ? std::vector<int>{1, 0} : std::vector<int>{1, 2, 3, 0};
  std::vector<hipEvent_t> ev(2 * (size_t)reps, nullptr);
  hipError_t e = hipSuccess;
  for (size_t i = 0; i < ev.size() && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&ev[i], kTimingEventFlags);
  bool first_x = true;
  for (int r = 0; r < reps && e == hipSuccess; ++r)
    for (int p : order) {
      e = launch_timed_pass<T>(c, psi, p, p == 0 && first_x, p == pass ? &ev[2 * r] : nullptr);
      if (p == 0) first_x = false;
      if (e != hipSuccess) break;
    }
  double total = 0.0;
  if (e == hipSuccess) e = hipEventSynchronize(ev.back());
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, ev[2 * r], ev[2 * r + 1]);
    total += ms;
  }
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  if (e != hipSuccess) return hip_fail(c, e, "pass timing");
  *avg_ms = total / reps;
  return SGP_OK;
}

template <typename T>
int time_pass_impl(sgp_ctx* c, void* psi, int pass, int reps, double* avg_ms) {
  if (pass & SGP_TIME_IN_STEP) return time_pass_in_step<T>(c, psi, pass & ~SGP_TIME_IN_STEP, reps, avg_ms);
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return hip_fail(c, e, "event create");
  e = hipEventCreate(&e1);
  if (e != hipSuccess) { (void)hipEventDestroy(e0); return hip_fail(c, e, "event create"); }
  e = hipEventRecord(e0, c->st);
  for (int i = 0; i < reps && e == hipSuccess; ++i) e = launch_timed_pass<T>(c, psi, pass, i == 0);
  if (e == hipSuccess) e = hipEventRecord(e1, c->st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(c, e, "pass timing");
  *avg_ms = (double)ms / reps;
  return SGP_OK;
}

// Timing inside real steps: `nsteps` steps of sgp_step's schedule, launched without
// the graph (the same kernels in the same order); every launch of the named pass
// carries an event pair that its dispatch stamps with the kernel's start and end.
// psi advances nsteps steps; the context time is restored.
template <typename T>
int time_pass_steps(sgp_ctx* c, void* psi, int pass, int nsteps, double* avg_ms) {
  c->tev.assign(2 * (12 * (size_t)nsteps + 8), nullptr);  // more pairs than launches of one pass
  hipError_t e = hipSuccess;
  for (size_t i = 0; i < c->tev.size() && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&c->tev[i], kTimingEventFlags);
  int rc = SGP_OK;
  size_t used = 0;
  if (e == hipSuccess) {
    const double t_save = c->t;
    const bool g_save = c->use_graph;
    c->use_graph = false;
    c->tev_pass = pass;
    c->tev_used = 0;
    rc = step_impl<T>(c, psi, nsteps);
    used = c->tev_used;
    c->tev_pass = -1;
    c->use_graph = g_save;
    c->t = t_save;
  }
  double total = 0.0;
  if (e == hipSuccess && rc == SGP_OK && used > 0) {
    e = hipEventSynchronize(c->tev[2 * used - 1]);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    for (size_t i = 0; i < used && e == hipSuccess; ++i) {
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, c->tev[2 * i], c->tev[2 * i + 1]);
      total += ms;
    }
  }
  for (hipEvent_t x : c->tev)
    if (x) (void)hipEventDestroy(x);
  c->tev.clear();
  if (e != hipSuccess) return hip_fail(c, e, "pass timing");
  if (rc != SGP_OK) return rc;
  if (used == 0) return fail(c, SGP_ERR_ARG, "the timed steps launch no such pass");
  *avg_ms = total / (double)used;
  return SGP_OK;
}

// Register plan of the passes along one axis; the twiddle tables follow the plan.
template <typename T>
int set_plan_impl(sgp_ctx* c, int axis, int e) {
  if (axis == SGP_PLAN_LINEAR && c->g.dim == 3) {
    if (e != 0 && e != 1) return fail(c, SGP_ERR_ARG, "linear-substep split must be 0 or 1");
    if (c->lin_split != e) {
      c->lin_split = e;
      drop_graph(c);
    }
    return SGP_OK;
  }
  if (axis < 0 || axis >= c->g.dim) return fail(c, SGP_ERR_ARG, "axis out of range");
  if (e == 0) e = default_elems(c->g.n[axis]);
  if (!plan_ok(c->g.n[axis], e, (int)c->esize))
    return fail(c, SGP_ERR_ARG, "plan width " + std::to_string(e) + " not available for length " +
                                    std::to_string(c->g.n[axis]));
  if (c->plan_e[axis] == e) return SGP_OK;
  c->plan_e[axis] = e;
  drop_graph(c);
  if (c->ws) {
    hipError_t r = upload_twiddles<T>(c);
    if (r != hipSuccess) return hip_fail(c, r, "twiddle upload");
  }
  return SGP_OK;
}

// Autotuner: time `steps` whole steps (the sgp_step path, graphs included) for
// every combination of the axes' plan widths (in 3D also both linear-substep
// splits) and keep the fastest.  psi is advanced by the timed steps; the context time
// is restored.
template <typename T>
int autotune_impl(sgp_ctx* c, void* psi, int steps, int out_e[3], double* best_ms) {
  const double t_save = c->t;
  hipEvent_t e0, e1;
  hipError_t r = hipEventCreate(&e0);
  if (r != hipSuccess) return hip_fail(c, r, "event create");
  r = hipEventCreate(&e1);
  if (r != hipSuccess) { (void)hipEventDestroy(e0); return hip_fail(c, r, "event create"); }
  auto time_steps = [&](double* ms) -> int {
    int rc = step_impl<T>(c, psi, steps);  // untimed: graph capture, warm caches
    if (rc != SGP_OK) return rc;
    hipError_t q = hipEventRecord(e0, c->st);
    if (q != hipSuccess) return hip_fail(c, q, "event record");
    rc = step_impl<T>(c, psi, steps);
    if (rc != SGP_OK) return rc;
    q = hipEventRecord(e1, c->st);
    if (q == hipSuccess) q = hipEventSynchronize(e1);
    float f = 0.f;
    if (q == hipSuccess) q = hipEventElapsedTime(&f, e0, e1);
    if (q != hipSuccess) return hip_fail(c, q, "autotune timing");
    *ms = (double)f / steps;
    return SGP_OK;
  };
  // every combination of the axes' plan widths (at most 3 per axis: 9 in 2D, 27 in
  // 3D); the plans of different axes interact through the passes' occupancy
  double best = 0.0;
  int rc = time_steps(&best);
  std::vector<int> w[3];
  for (int ax = 0; ax < 3; ++ax) w[ax] = ax < c->g.dim ? plan_widths(c->g.n[ax], (int)c->esize) : std::vector<int>{0};
  int best_e[3] = {c->plan_e[0], c->plan_e[1], c->plan_e[2]};
  int best_ls = c->lin_split;
  const int start[3] = {c->plan_e[0], c->plan_e[1], c->plan_e[2]};
  const int start_ls = c->lin_split;
  const int nsplit = c->g.dim == 3 ? 2 : 1;
  for (int ls = 0; ls < nsplit; ++ls)
    for (int ex : w[0])
      for (int ey : w[1])
        for (int ez : w[2]) {
          if (rc != SGP_OK) break;
          const int cand[3] = {ex, ey, ez};
          bool same = ls == start_ls;
          for (int ax = 0; ax < c->g.dim; ++ax) same = same && cand[ax] == start[ax];
          if (same) continue;
          for (int ax = 0; ax < c->g.dim && rc == SGP_OK; ++ax) rc = set_plan_impl<T>(c, ax, cand[ax]);
          if (rc == SGP_OK && c->g.dim == 3) rc = set_plan_impl<T>(c, SGP_PLAN_LINEAR, ls);
          double ms = 0.0;
          if (rc == SGP_OK) rc = time_steps(&ms);
          if (rc == SGP_OK && ms < best) {
            best = ms;
            best_ls = ls;
            for (int ax = 0; ax < c->g.dim; ++ax) best_e[ax] = cand[ax];
          }
        }
  for (int ax = 0; ax < c->g.dim && rc == SGP_OK; ++ax) rc = set_plan_impl<T>(c, ax, best_e[ax]);
  if (rc == SGP_OK && c->g.dim == 3) rc = set_plan_impl<T>(c, SGP_PLAN_LINEAR, best_ls);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->t = t_save;
  if (rc != SGP_OK) return rc;
  for (int ax = 0; ax < 3; ++ax) out_e[ax] = ax < c->g.dim ? c->plan_e[ax] : 0;
  if (best_ms) *best_ms = best;
  return SGP_OK;
}

// Observables: one x-line pass (d_x, pointwise terms) and one column pass per other
// axis; FP64 block partials summed on the host in block order (deterministic).
long obs_nblocks(const sgp_ctx* c, int axis, int e) {
  const int nx = c->g.n[0], ny = c->g.n[1], nz = c->g.dim == 3 ? c->g.n[2] : 1;
  const int W = obs_lines_per_block(c->g.n[axis], e);
  if (axis == 0) return ((long)ny * nz + W - 1) / W;
  const long nouter = axis == 1 ? nz : ny;
  return ((nx + W - 1) / W) * nouter;
}

// Blocks of a pass kernel along `axis` with plan width e (one adjoint slot each).
long pass_nblocks(const sgp_ctx* c, int axis, int e) {
  const int nx = c->g.n[0], ny = c->g.n[1], nz = c->g.dim == 3 ? c->g.n[2] : 1;
  const int W = lines_per_block(c->g.n[axis], e);
  if (axis == 0) return ((long)ny * nz + W - 1) / W;
  const long nouter = axis == 1 ? nz : ny;
  return ((nx + W - 1) / W) * nouter;
}

template <typename T>
int observables_impl(sgp_ctx* c, const void* psi, double out[12]) {
  double* part = (double*)c->at(c->off_part);
  double* red = (double*)c->at(c->off_red);
  double tot[3][NOBS];
  for (int axis = 0; axis < c->g.dim; ++axis) {
    PassArgs a = base_args(c);
    if (axis == 0) {
      a.tw_fwd = c->at(c->off_tw[0][0]);
      a.tw_inv = c->at(c->off_tw[0][1]);
      a.nu_scale_l = kPi / c->g.L[0];
    } else {
      column_geometry(c, axis, a);
    }
    a.s_arg = c->frame == SGP_FRAME_LAB ? 0.0 : c->t;  // lab frame: the trap at x
    const int kind = axis == 0 ? OBS_X : (axis == 1 ? OBS_Y : OBS_Z);
    hipError_t e = launch_obs<T>(kind, psi, a, c->g.n[axis], c->elems(axis), part, c->st);
    if (e != hipSuccess) return hip_fail(c, e, "observables launch");
    // block partials summed on the device in a fixed order (the next axis's launch
    // reuses the partials after this sum on the same stream)
    e = launch_sum_partials(part, obs_nblocks(c, axis, c->elems(axis)), NOBS, red + axis * NOBS, c->st);
    if (e != hipSuccess) return hip_fail(c, e, "observables reduction");
  }
  {
    hipError_t e = hipMemcpyAsync(&tot[0][0], red, sizeof(double) * NOBS * c->g.dim, hipMemcpyDeviceToHost, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (e != hipSuccess) return hip_fail(c, e, "observables readback");
  }
  double hd = 1.0;
  for (int ax = 0; ax < c->g.dim; ++ax) hd *= 2.0 * c->g.L[ax] / c->g.n[ax];
  double ekin = 0.0, lz = 0.0, soc = 0.0;
  for (int axis = 0; axis < c->g.dim; ++axis) ekin += tot[axis][4];
  lz = tot[0][5] + tot[1][5];
  soc = tot[0][6] + tot[1][6];
  out[0] = hd * tot[0][0];
  out[2] = hd * tot[0][1];
  out[3] = hd * lz;
  out[1] = hd * (ekin + tot[0][2] + tot[0][3] - c->p.gamma * soc) - c->p.Omega * out[3];
  // widths and moments (lab-frame coordinates) and W = 2 Im sum conj(psi)(x d_x + y d_y) psi
  out[4] = hd * tot[0][7];
  out[5] = hd * tot[0][8];
  out[6] = hd * tot[0][9];
  out[7] = hd * tot[0][10];
  out[8] = hd * (tot[0][11] + tot[1][11]);
  // spin-orbit laws (Sec. 2): with L_+- = i d_y +- d_x and the sums
  // D_a(q) = sum conj(psi_a) d_a psi_b over the pairs q, Q = sum conj(psi_a) L psi_b
  // = i D_y +- D_x; the pair (1, 2) follows from (2, 1) since d is anti-Hermitian
  using cd = std::complex<double>;
  auto dsum = [&](int axis, int q) {
    const int base = axis == 0 ? 12 : 20;
    return cd(tot[axis][base + 2 * q], tot[axis][base + 2 * q + 1]);
  };
  auto lsum = [&](int q, double sgn) { return cd(0.0, 1.0) * dsum(1, q) + sgn * dsum(0, q); };
  const cd q1 = lsum(0, -1.0);  // conj(psi_2) L_- psi_1
  const cd q2 = lsum(1, -1.0);  // conj(psi_-1) L_- psi_-2
  const cd q3 = lsum(2, -1.0);  // conj(psi_1) L_- psi_0
  const cd q4 = lsum(3, +1.0);  // conj(psi_-1) L_+ psi_0
  const cd q5 = cd(0.0, 1.0) * (-std::conj(dsum(1, 0))) - std::conj(dsum(0, 0));  // conj(psi_1) L_+ psi_2
  const double r6h = 1.22474487139158904909864203735294570;
  const double g = c->p.gamma;
  // out[9] = dM/dt = -2 gamma Im[Q1 + Q2 + sqrt6/2 (Q3 - Q4)]
  out[9] = -2.0 * g * hd * (q1 + q2 + r6h * (q3 - q4)).imag();
  // out[10] = d<Lz>/dt = (gx^2 - gy^2) int x y rho + 2 gamma Im[Q2 - Q5 + sqrt6/2 (Q3 - Q4)] (Lemma 1)
  out[10] = (c->p.gx * c->p.gx - c->p.gy * c->p.gy) * out[7] + 2.0 * g * hd * (q2 - q5 + r6h * (q3 - q4)).imag();
  // out[11] = G(gamma, Psi) of Lemma 2: 2 gamma Re int [Omega (i y - x) F_+ + gamma
  // (sum_m (6 - m^2) |psi_m|^2 + sum_m m conj(psi_m) L_z psi_m)] on the lab-frame state.
  // The rotating-frame state carries F_+ with the phase exp(i theta) of its
  // components (theta = Omega s): F_+(lab, X) = exp(-i theta) F_+(x); the sums use
  // the lab-frame coordinates (X, Y) of each point; the other two terms are
  // frame-invariant
  const double th = c->frame == SGP_FRAME_LAB ? 0.0 : c->p.Omega * c->t;
  const cd A = c->p.Omega * std::exp(cd(0.0, -th)) * cd(tot[0][20], tot[0][21]);
  const double B = tot[0][22], C = tot[0][23] + (c->g.dim >= 2 ? tot[1][12] : 0.0);
  out[11] = 2.0 * g * hd * (A.real() + g * (B + C));
  // a NaN or infinity anywhere in the state reaches the mass sum (|psi|^2 over all
  // points) and every other sum
  for (int axis = 0; axis < c->g.dim; ++axis)
    for (int q = 0; q < NOBS; ++q)
      if (!std::isfinite(tot[axis][q]))
        return fail(c, SGP_ERR_NONFINITE, "the state holds non-finite values (observable sums are not finite)");
  return SGP_OK;
}

// <u, J_z v>_h = h^d sum conj(u) (L_z + F_z) v, L_z = -i (x d_y - y d_x) with
// spectral derivatives: one x-line pass (i y d_x v + F_z v) and one y-column pass
// (-i x d_y v), block partials summed on the device.
template <typename T>
int jz_inner_impl(sgp_ctx* c, const void* u, const void* v, double out[2]) {
  double* part = (double*)c->at(c->off_part);
  double* red = (double*)c->at(c->off_red);
  for (int axis = 0; axis < 2; ++axis) {
    PassArgs a = base_args(c);
    if (axis == 0) {
      a.tw_fwd = c->at(c->off_tw[0][0]);
      a.tw_inv = c->at(c->off_tw[0][1]);
      a.nu_scale_l = kPi / c->g.L[0];
    } else {
      column_geometry(c, 1, a);
    }
    a.fwd = u;
    hipError_t e = launch_obs<T>(axis == 0 ? OBS_JX : OBS_JY, v, a, c->g.n[axis], c->elems(axis), part, c->st);
    if (e != hipSuccess) return hip_fail(c, e, "J_z inner product launch");
    e = launch_sum_partials(part, obs_nblocks(c, axis, c->elems(axis)), NOBS, red + axis * NOBS, c->st);
    if (e != hipSuccess) return hip_fail(c, e, "J_z inner product reduction");
  }
  double tot[2][NOBS];
  hipError_t e = hipMemcpyAsync(&tot[0][0], red, sizeof(double) * 2 * NOBS, hipMemcpyDeviceToHost, c->st);
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  if (e != hipSuccess) return hip_fail(c, e, "J_z inner product readback");
  double hd = 1.0;
  for (int ax = 0; ax < c->g.dim; ++ax) hd *= 2.0 * c->g.L[ax] / c->g.n[ax];
  out[0] = hd * (tot[0][0] + tot[1][0]);
  out[1] = hd * (tot[0][1] + tot[1][1]);
  if (!std::isfinite(out[0]) || !std::isfinite(out[1]))
    return fail(c, SGP_ERR_NONFINITE, "non-finite values in the states of the J_z inner product");
  return SGP_OK;
}

// The observables with no allocation and no host synchronisation, for callers that
// cannot allocate (code under graph capture, serving loops): the block partials and
// their sums live in a file-scope device array of fixed size (one copy per GPU,
// held until the process ends), and a last kernel combines the sums into the four
// values on the device.  The array's device address is resolved once per device
// (hipGetSymbolAddress, with that device current); host code never uses the
// array's name as an address.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

int obs_scratch_for_device(sgp_ctx* c, double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(c, e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(c, SGP_ERR_ARG, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(c, e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(c, SGP_ERR_HIP, "hipGetSymbolAddress(scratch) returned a null address");
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return SGP_OK;
}

// out[0..3] = mass, energy, magnetization, <Lz> from the per-axis sums red[axis][q],
// combined as observables_impl does on the host.
__global__ void k_obs_combine(const double* __restrict__ red, int dim, double hd, double gamma, double Omega,
                              double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double ekin = 0.0;
  for (int axis = 0; axis < dim; ++axis) ekin += red[axis * NOBS + 4];
  const double lz = red[5] + red[NOBS + 5];
  const double soc = red[6] + red[NOBS + 6];
  out[0] = hd * red[0];
  out[2] = hd * red[1];
  out[3] = hd * lz;
  out[1] = hd * (ekin + red[2] + red[3] - gamma * soc) - Omega * out[3];
}

template <typename T>
int observables_device_impl(sgp_ctx* c, const void* psi, double* sp, long nbmax, double* out_dev) {
  double* part = sp;
  double* red = sp + (size_t)NOBS * nbmax;
  for (int axis = 0; axis < c->g.dim; ++axis) {
    PassArgs a = base_args(c);
    if (axis == 0) {
      a.tw_fwd = c->at(c->off_tw[0][0]);
      a.tw_inv = c->at(c->off_tw[0][1]);
      a.nu_scale_l = kPi / c->g.L[0];
    } else {
      column_geometry(c, axis, a);
    }
    a.s_arg = c->frame == SGP_FRAME_LAB ? 0.0 : c->t;
    const int kind = axis == 0 ? OBS_X : (axis == 1 ? OBS_Y : OBS_Z);
    hipError_t e = launch_obs<T>(kind, psi, a, c->g.n[axis], c->elems(axis), part, c->st);
    if (e != hipSuccess) return hip_fail(c, e, "observables launch");
    e = launch_sum_partials(part, obs_nblocks(c, axis, c->elems(axis)), NOBS, red + axis * NOBS, c->st);
    if (e != hipSuccess) return hip_fail(c, e, "observables reduction");
  }
  double hd = 1.0;
  for (int ax = 0; ax < c->g.dim; ++ax) hd *= 2.0 * c->g.L[ax] / c->g.n[ax];
  hipLaunchKernelGGL(k_obs_combine, dim3(1), dim3(64), 0, c->st, red, c->g.dim, hd, c->p.gamma, c->p.Omega,
                     out_dev);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e, "observables combine");
  return SGP_OK;
}

// Rotation mapping of Sec. 3.1 by the three shears of eqs. RSDA1/RSDA2, each a
// transform along one axis, a phase exp(i nu a w) per coefficient and the inverse
// transform: dir = +1 gives Phi = M_t Psi, phi_l = exp(-i l Omega t) psi_l(R(t) x);
// dir = -1 gives Psi = M_t^{-1} Phi.
template <typename T>
hipError_t run_shear(sgp_ctx* c, void* psi, int kind, double coef, bool cph, double cphase) {
  PassArgs a = base_args(c);
  if (kind == X_SHEAR) {
    a.tw_fwd = c->at(c->off_tw[0][0]);
    a.tw_inv = c->at(c->off_tw[0][1]);
  } else {
    column_geometry(c, 1, a);
  }
  a.shear = coef;
  a.cphase_on = cph ? 1 : 0;
  a.cphase = cphase;
  const int axis = kind == X_SHEAR ? 0 : 1;
  return launch_pass<T>(kind, psi, a, c->g.n[axis], c->elems(axis), c->st);
}

template <typename T>
int rotation_map_impl(sgp_ctx* c, void* psi, double t, int dir) {
  const double th = c->p.Omega * t;
  if (std::fabs(std::cos(0.5 * th)) < 1e-6)
    return fail(c, SGP_ERR_ARG, "rotation angle Omega t too close to an odd multiple of pi for the shears");
  const double a = (dir > 0 ? 1.0 : -1.0) * std::tan(0.5 * th);
  const double b = (dir > 0 ? -1.0 : 1.0) * std::sin(th);
  hipError_t e = run_shear<T>(c, psi, X_SHEAR, a, false, 0.0);
  if (e == hipSuccess) e = run_shear<T>(c, psi, C_SHEAR, b, false, 0.0);
  if (e == hipSuccess) e = run_shear<T>(c, psi, X_SHEAR, a, true, (dir > 0 ? -1.0 : 1.0) * th);
  if (e != hipSuccess) return hip_fail(c, e, "rotation map launch");
  return SGP_OK;
}

// Algorithm 1 literally (lab frame): per step the nonlinear substeps with the trap
// at x (not merged), and around every linear substep of length d starting at clock s
// the mapping M_s before and M_{s+d}^{-1} after; the linear substep itself is the
// same propagator pass, between bare transforms along x.
template <typename T>
int lab_step_impl(sgp_ctx* c, void* psi, long nsteps) {
  const Composition comp = composition(c->scheme);
  const std::vector<double>& A = comp.A;
  const std::vector<double>& B = comp.B;
  const std::vector<int>& tab = comp.tab;
  const double t0 = c->t, tau = c->tau;
  for (long n = 0; n < nsteps; ++n) {
    double s = t0 + (double)n * tau;
    for (size_t j = 0; j < A.size(); ++j) {
      hipError_t e = hipSuccess;
      if (A[j] != 0.0) e = run_xpass<T>(c, c->st, X_NLONLY, psi, A[j] * tau, CLOCK_ARG, 0.0);
      if (e != hipSuccess) return hip_fail(c, e, "nonlinear pass launch");
      if (B[j] == 0.0) continue;
      const double d = B[j] * tau;
      int rc = rotation_map_impl<T>(c, psi, s, +1);
      if (rc != SGP_OK) return rc;
      e = run_xpass<T>(c, c->st, X_FWD, psi, 0.0, CLOCK_ARG, 0.0);
      if (e == hipSuccess) e = run_linear<T>(c, c->st, psi, tab[j], d);
      if (e == hipSuccess) e = run_xpass<T>(c, c->st, X_INV, psi, 0.0, CLOCK_ARG, 0.0);
      if (e != hipSuccess) return hip_fail(c, e, "linear pass launch");
      rc = rotation_map_impl<T>(c, psi, s + d, -1);
      if (rc != SGP_OK) return rc;
      s += d;
    }
  }
  c->t = t0 + (double)nsteps * tau;
  return SGP_OK;
}

// Forward evolution of one call that also stores, for every pass with a pointwise
// stage, the stage's input: slot 2k the input of the k-th nonlinear substep
// (physical), slot 2k+1 the Fourier-space input of the k-th propagator.  Kernels are
// launched one by one (each pass writes a different slot).
template <typename T>
int step_store_impl(sgp_ctx* c, void* psi, long nsteps, char* store) {
  std::vector<double> nl, lin;
  std::vector<int> tab;
  schedule(c, nsteps, nl, lin, tab);
  const size_t slot = (size_t)c->npts() * 5 * 2 * c->esize;
  hipError_t e = run_xpass_ex<T>(c, X_FIRST, psi, nl[0], CLOCK_ARG, c->t, store, nullptr);
  if (e != hipSuccess) return hip_fail(c, e, "X-pass launch");
  double s = c->t;
  for (size_t k = 0; k < lin.size(); ++k) {
    char* sl = store + (2 * k + 1) * slot;
    if (c->g.dim == 2) {
      e = run_colpass_ex<T>(c, C_PROP, 1, psi, tab[k], lin[k], sl, nullptr);
    } else {
      e = run_colpass_ex<T>(c, C_FWD, 1, psi, tab[k], lin[k], nullptr, nullptr);
      if (e == hipSuccess) e = run_colpass_ex<T>(c, C_PROP, 2, psi, tab[k], lin[k], sl, nullptr);
      if (e == hipSuccess) e = run_colpass_ex<T>(c, C_INV, 1, psi, tab[k], lin[k], nullptr, nullptr);
    }
    if (e != hipSuccess) return hip_fail(c, e, "linear pass launch");
    s += lin[k];
    e = run_xpass_ex<T>(c, k + 1 == lin.size() ? X_LAST : X_MID, psi, nl[k + 1], CLOCK_ARG, s,
                        store + (2 * k + 2) * slot, nullptr);
    if (e != hipSuccess) return hip_fail(c, e, "X-pass launch");
  }
  c->t += (double)nsteps * c->tau;
  return SGP_OK;
}

// Reverse sweep through the passes of the matching step_store_impl call (started at
// the current clock).  lam: gradient with respect to the call's output on entry, with
// respect to its input on exit (physical space both times).
template <typename T>
int adjoint_impl(sgp_ctx* c, void* lam, long nsteps, const char* store) {
  std::vector<double> nl, lin;
  std::vector<int> tab;
  schedule(c, nsteps, nl, lin, tab);
  const size_t slot = (size_t)c->npts() * 5 * 2 * c->esize;
  const size_t M = lin.size();
  std::vector<double> s(M + 1);
  s[0] = c->t;
  for (size_t k = 0; k < M; ++k) s[k + 1] = s[k] + lin[k];
  hipError_t e = run_xpass_ex<T>(c, XA_LAST, lam, nl[M], CLOCK_ARG, s[M], nullptr, store + 2 * M * slot);
  if (e != hipSuccess) return hip_fail(c, e, "adjoint X-pass launch");
  for (long k = (long)M - 1; k >= 0; --k) {
    const char* sl = store + (2 * k + 1) * slot;
    if (c->g.dim == 2) {
      e = run_colpass_ex<T>(c, C_ADJ, 1, lam, tab[k], lin[k], nullptr, sl);
    } else {
      // adjoint of (Y1 forward, Z, Y2 inverse): Y forward, Z adjoint, Y inverse
      e = run_colpass_ex<T>(c, C_FWD, 1, lam, tab[k], lin[k], nullptr, nullptr);
      if (e == hipSuccess) e = run_colpass_ex<T>(c, C_ADJ, 2, lam, tab[k], lin[k], nullptr, sl);
      if (e == hipSuccess) e = run_colpass_ex<T>(c, C_INV, 1, lam, tab[k], lin[k], nullptr, nullptr);
    }
    if (e != hipSuccess) return hip_fail(c, e, "adjoint linear pass launch");
    e = run_xpass_ex<T>(c, k == 0 ? XA_FIRST : XA_MID, lam, nl[k], CLOCK_ARG, s[k], nullptr, store + 2 * k * slot);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint X-pass launch");
  }
  return SGP_OK;
}

}  // namespace

extern "C" {

int sgp_create(const sgp_grid* grid, const sgp_params* params, int dtype, void* hip_stream, sgp_ctx** out) {
  if (!grid || !params || !out) return fail(nullptr, SGP_ERR_ARG, "null argument");
  *out = nullptr;
  if (grid->dim != 2 && grid->dim != 3) return fail(nullptr, SGP_ERR_ARG, "dim must be 2 or 3");
  for (int i = 0; i < grid->dim; ++i) {
    if (!supported_n(grid->n[i]))
      return fail(nullptr, SGP_ERR_ARG, "unsupported grid size " + std::to_string(grid->n[i]) +
                                            " (supported: 16, 32, 64, 128, 192, 256, 384, 512, 768)");
    if (!(grid->L[i] > 0.0) || !std::isfinite(grid->L[i])) return fail(nullptr, SGP_ERR_ARG, "L must be > 0");
  }
  {
    // the kernels address the state with 32-bit element offsets
    long long elems = 5;
    for (int i = 0; i < grid->dim; ++i) elems *= grid->n[i];
    if (elems > 2147483647LL)
      return fail(nullptr, SGP_ERR_ARG, "grid too large: 5 n_x n_y n_z = " + std::to_string(elems) +
                                            " state elements, at most 2^31 - 1 are supported");
  }
  const double* pv = &params->c0;
  for (int i = 0; i < 8; ++i)
    if (!std::isfinite(pv[i])) return fail(nullptr, SGP_ERR_ARG, "non-finite parameter");
  if (dtype != SGP_C64 && dtype != SGP_C128) return fail(nullptr, SGP_ERR_ARG, "dtype must be SGP_C64 or SGP_C128");
  sgp_ctx* c = new (std::nothrow) sgp_ctx();
  if (!c) return fail(nullptr, SGP_ERR_ARG, "out of host memory");
  c->g = *grid;
  if (c->g.dim == 2) { c->g.n[2] = 1; c->g.L[2] = 0.0; }
  c->p = *params;
  c->dtype = dtype;
  c->st = (hipStream_t)hip_stream;
  c->esize = dtype == SGP_C64 ? 4 : 8;
  for (int ax = 0; ax < c->g.dim; ++ax) c->plan_e[ax] = default_elems(c->g.n[ax]);
  // workspace layout
  size_t off = 0;
  for (int ax = 0; ax < 3; ++ax)
    for (int dir = 0; dir < 2; ++dir) {
      c->off_tw[ax][dir] = off;
      // room for the largest table over the plans of this axis (plans can change later)
      size_t most = 0;
      if (ax < c->g.dim)
        for (int e : plan_widths(c->g.n[ax], (int)c->esize))
          most = std::max(most, twiddle_table(plan_radices(c->g.n[ax], e, dir == 0)).size());
      if (ax < c->g.dim) off += align256(4 * c->esize * (most + 1));
    }
  const size_t nxy = (size_t)c->g.n[0] * c->g.n[1];
  for (int k = 0; k < 4; ++k) {
    c->off_cs[k] = off;
    off += align256(2 * c->esize * nxy);
    for (int ax = 0; ax < 3; ++ax) {
      c->off_kin[k][ax] = off;
      off += align256(2 * c->esize * (ax < c->g.dim ? c->g.n[ax] : 1));
    }
  }
  c->off_clock = off;
  off += 256;
  c->off_part = off;
  // block partials and adjoint parameter slots: one per block of the largest pass
  // over every plan
  long maxb = 0;
  for (int axis = 0; axis < c->g.dim; ++axis)
    for (int e : plan_widths(c->g.n[axis], (int)c->esize))
      maxb = std::max(maxb, std::max(obs_nblocks(c, axis, e), pass_nblocks(c, axis, e)));
  off += align256(sizeof(double) * NOBS * maxb);
  c->off_red = off;
  off += align256(sizeof(double) * 3 * NOBS);
  const long gb = maxb;
  c->ngacc = gb;
  c->off_gacc = off;
  off += align256(sizeof(double) * NGRAD * gb);
  c->total = off;
  *out = c;
  return SGP_OK;
}

int sgp_workspace_size(const sgp_ctx* c, size_t* bytes) {
  if (!c || !bytes) return SGP_ERR_ARG;
  *bytes = c->total;
  return SGP_OK;
}

int sgp_set_workspace(sgp_ctx* c, void* dev_ptr, size_t bytes) {
  if (!c || !dev_ptr) return fail(c, SGP_ERR_ARG, "null argument");
  if (bytes < c->total) return fail(c, SGP_ERR_WORKSPACE, "workspace too small");
  if (((uintptr_t)dev_ptr) & 255) return fail(c, SGP_ERR_ARG, "workspace must be 256-byte aligned");
  c->ws = (char*)dev_ptr;
  c->ws_bytes = bytes;
  c->have_prop = false;
  drop_graph(c);
  hipError_t e = c->dtype == SGP_C64 ? upload_twiddles<float>(c) : upload_twiddles<double>(c);
  if (e == hipSuccess) e = hipMemsetAsync(c->at(c->off_gacc), 0, sizeof(double) * NGRAD * c->ngacc, c->st);
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  if (e != hipSuccess) return hip_fail(c, e, "twiddle upload");
  return SGP_OK;
}

int sgp_build_propagator(sgp_ctx* c, double tau, int scheme) {
  if (!c) return SGP_ERR_ARG;
  if (!c->ws) return fail(c, SGP_ERR_STATE, "no workspace set");
  if (!std::isfinite(tau) || tau == 0.0) return fail(c, SGP_ERR_ARG, "tau must be finite and nonzero");
  if (scheme != SGP_TS2 && scheme != SGP_TS4 && scheme != SGP_TS6)
    return fail(c, SGP_ERR_ARG, "scheme must be SGP_TS2, SGP_TS4 or SGP_TS6");
  drop_graph(c);
  c->scheme = scheme;
  c->tau = tau;
  {
    const Composition comp = composition(scheme);
    c->nprop = (int)comp.props.size();
    for (int i = 0; i < c->nprop; ++i) c->dprop[i] = comp.props[i] * tau;
  }
  for (int i = 0; i < c->nprop; ++i) {
    hipError_t e;
    if (c->dtype == SGP_C64)
      e = launch_build_tables<float>(c->at(c->off_cs[i]), c->at(c->off_kin[i][0]), c->at(c->off_kin[i][1]),
                                     c->at(c->off_kin[i][2]), c->g.n, c->g.L, c->g.dim, c->p.Omega, c->p.gamma,
                                     c->dprop[i], c->st);
    else
      e = launch_build_tables<double>(c->at(c->off_cs[i]), c->at(c->off_kin[i][0]), c->at(c->off_kin[i][1]),
                                      c->at(c->off_kin[i][2]), c->g.n, c->g.L, c->g.dim, c->p.Omega, c->p.gamma,
                                      c->dprop[i], c->st);
    if (e != hipSuccess) return hip_fail(c, e, "propagator build");
  }
  hipError_t e = hipStreamSynchronize(c->st);
  if (e != hipSuccess) return hip_fail(c, e, "propagator build");
  c->have_prop = true;
  return SGP_OK;
}

int sgp_step(sgp_ctx* c, void* psi, long nsteps) {
  if (!c || !psi) return fail(c, SGP_ERR_ARG, "null argument");
  if (nsteps < 0) return fail(c, SGP_ERR_ARG, "nsteps must be >= 0");
  if (!c->ws) return fail(c, SGP_ERR_STATE, "no workspace set");
  if (!c->have_prop) return fail(c, SGP_ERR_STATE, "propagator not built");
  if (nsteps == 0) return SGP_OK;
  if (c->frame == SGP_FRAME_LAB)
    return c->dtype == SGP_C64 ? lab_step_impl<float>(c, psi, nsteps) : lab_step_impl<double>(c, psi, nsteps);
  return c->dtype == SGP_C64 ? step_impl<float>(c, psi, nsteps) : step_impl<double>(c, psi, nsteps);
}

int sgp_rotation_map(sgp_ctx* c, void* psi, double t, int direction) {
  if (!c || !psi) return fail(c, SGP_ERR_ARG, "null argument");
  if (direction != 1 && direction != -1) return fail(c, SGP_ERR_ARG, "direction must be +1 or -1");
  if (!std::isfinite(t)) return fail(c, SGP_ERR_ARG, "non-finite time");
  if (!c->ws) return fail(c, SGP_ERR_STATE, "no workspace set");
  return c->dtype == SGP_C64 ? rotation_map_impl<float>(c, psi, t, direction)
                             : rotation_map_impl<double>(c, psi, t, direction);
}

int sgp_observables(sgp_ctx* c, const void* psi, double out[4]) {
  if (!c || !psi || !out) return fail(c, SGP_ERR_ARG, "null argument");
  if (!c->ws) return fail(c, SGP_ERR_STATE, "no workspace set");
  double all[12];
  int rc = c->dtype == SGP_C64 ? observables_impl<float>(c, psi, all) : observables_impl<double>(c, psi, all);
  if (rc == SGP_OK || rc == SGP_ERR_NONFINITE) std::memcpy(out, all, 4 * sizeof(double));
  return rc;
}

int sgp_observables_device(sgp_ctx* c, const void* psi, double* out_dev) {
  if (!c || !psi || !out_dev) return fail(c, SGP_ERR_ARG, "null argument");
  if (!c->ws) return fail(c, SGP_ERR_STATE, "no workspace set");
  long nbmax = 0;
  for (int axis = 0; axis < c->g.dim; ++axis) nbmax = std::max(nbmax, obs_nblocks(c, axis, c->elems(axis)));
  const size_t need = sizeof(double) * NOBS * ((size_t)nbmax + 3);
  if (need > kObsScratchBytes)
    return fail(c, SGP_ERR_ARG, "grid too large for sgp_observables_device: its block partials need " +
                                    std::to_string(need) + " bytes of the fixed " +
                                    std::to_string(kObsScratchBytes) + "-byte device scratch");
  double* sp = nullptr;
  const int rc = obs_scratch_for_device(c, &sp);
  if (rc != SGP_OK) return rc;
  return c->dtype == SGP_C64 ? observables_device_impl<float>(c, psi, sp, nbmax, out_dev)
                             : observables_device_impl<double>(c, psi, sp, nbmax, out_dev);
}

int sgp_jz_inner(sgp_ctx* c, const void* u, const void* v, double out[2]) {
  if (!c || !u || !v || !out) return fail(c, SGP_ERR_ARG, "null argument");
  if (!c->ws) return fail(c, SGP_ERR_STATE, "no workspace set");
  return c->dtype == SGP_C64 ? jz_inner_impl<float>(c, u, v, out) : jz_inner_impl<double>(c, u, v, out);
}

int sgp_diagnostics(sgp_ctx* c, const void* psi, double out[12]) {
  if (!c || !psi || !out) return fail(c, SGP_ERR_ARG, "null argument");
  if (!c->ws) return fail(c, SGP_ERR_STATE, "no workspace set");
  return c->dtype == SGP_C64 ? observables_impl<float>(c, psi, out) : observables_impl<double>(c, psi, out);
}

int sgp_get_time(const sgp_ctx* c, double* t) {
  if (!c || !t) return SGP_ERR_ARG;
  *t = c->t;
  return SGP_OK;
}

int sgp_set_time(sgp_ctx* c, double t) {
  if (!c || !std::isfinite(t)) return SGP_ERR_ARG;
  c->t = t;
  return SGP_OK;
}

int sgp_time_pass(sgp_ctx* c, void* psi, int pass, int reps, double* avg_ms) {
  if (!c || !psi || !avg_ms || reps < 1) return fail(c, SGP_ERR_ARG, "bad argument");
  const int kind = pass & 3;
  if ((c->g.dim == 2 && kind > 1) || (pass & ~(SGP_TIME_IN_STEP | SGP_TIME_STEPS | 3)) ||
      ((pass & SGP_TIME_IN_STEP) && (pass & SGP_TIME_STEPS)))
    return fail(c, SGP_ERR_ARG, "no such pass");
  if ((pass & (SGP_TIME_IN_STEP | SGP_TIME_STEPS)) && reps > 4096)
    return fail(c, SGP_ERR_ARG, "at most 4096 rounds or steps when every launch is timed");
  if (!c->ws) return fail(c, SGP_ERR_STATE, "no workspace set");
  if (!c->have_prop) return fail(c, SGP_ERR_STATE, "propagator not built");
  if (pass & SGP_TIME_STEPS) {
    if (reps < 2) return fail(c, SGP_ERR_ARG, "SGP_TIME_STEPS needs at least 2 steps");
    if (c->frame == SGP_FRAME_LAB) return fail(c, SGP_ERR_STATE, "SGP_TIME_STEPS times the rotating-frame step");
    return c->dtype == SGP_C64 ? time_pass_steps<float>(c, psi, kind, reps, avg_ms)
                               : time_pass_steps<double>(c, psi, kind, reps, avg_ms);
  }
  return c->dtype == SGP_C64 ? time_pass_impl<float>(c, psi, pass, reps, avg_ms)
                             : time_pass_impl<double>(c, psi, pass, reps, avg_ms);
}

int sgp_store_size(const sgp_ctx* c, long nsteps, size_t* bytes) {
  if (!c || !bytes || nsteps < 1) return SGP_ERR_ARG;
  if (c->scheme == 0) return SGP_ERR_STATE;
  const long M = (long)(composition(c->scheme).A.size() - 1) * nsteps;
  *bytes = (size_t)(2 * M + 1) * (size_t)c->npts() * 5 * 2 * c->esize;
  return SGP_OK;
}

int sgp_step_store(sgp_ctx* c, void* psi, long nsteps, void* store, size_t store_bytes) {
  if (c && c->frame == SGP_FRAME_LAB) return fail(c, SGP_ERR_STATE, "the adjoint runs in the rotating frame only");
  if (!c || !psi || !store) return fail(c, SGP_ERR_ARG, "null argument");
  if (nsteps < 1) return fail(c, SGP_ERR_ARG, "nsteps must be >= 1");
  if (!c->ws) return fail(c, SGP_ERR_STATE, "no workspace set");
  if (!c->have_prop) return fail(c, SGP_ERR_STATE, "propagator not built");
  size_t need = 0;
  sgp_store_size(c, nsteps, &need);
  if (store_bytes < need) return fail(c, SGP_ERR_WORKSPACE, "store too small");
  return c->dtype == SGP_C64 ? step_store_impl<float>(c, psi, nsteps, (char*)store)
                             : step_store_impl<double>(c, psi, nsteps, (char*)store);
}

int sgp_adjoint_segment(sgp_ctx* c, void* lam, long nsteps, const void* store, size_t store_bytes) {
  if (c && c->frame == SGP_FRAME_LAB) return fail(c, SGP_ERR_STATE, "the adjoint runs in the rotating frame only");
  if (!c || !lam || !store) return fail(c, SGP_ERR_ARG, "null argument");
  if (nsteps < 1) return fail(c, SGP_ERR_ARG, "nsteps must be >= 1");
  if (!c->ws) return fail(c, SGP_ERR_STATE, "no workspace set");
  if (!c->have_prop) return fail(c, SGP_ERR_STATE, "propagator not built");
  size_t need = 0;
  sgp_store_size(c, nsteps, &need);
  if (store_bytes < need) return fail(c, SGP_ERR_WORKSPACE, "store too small");
  return c->dtype == SGP_C64 ? adjoint_impl<float>(c, lam, nsteps, (const char*)store)
                             : adjoint_impl<double>(c, lam, nsteps, (const char*)store);
}

int sgp_adjoint_gradients(sgp_ctx* c, double out[5], int reset) {
  if (!c || !out) return fail(c, SGP_ERR_ARG, "null argument");
  if (!c->ws) return fail(c, SGP_ERR_STATE, "no workspace set");
  // the per-block slots summed on the device in a fixed order (the observables'
  // reduction); only the NGRAD sums come back
  double* dev = (double*)c->at(c->off_gacc);
  double* sums = (double*)c->at(c->off_red);
  hipError_t e = launch_sum_partials(dev, c->ngacc, NGRAD, sums, c->st);
  if (e == hipSuccess) e = hipMemcpyAsync(out, sums, sizeof(double) * NGRAD, hipMemcpyDeviceToHost, c->st);
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  if (e != hipSuccess) return hip_fail(c, e, "gradient reduction");
  if (reset) {
    e = hipMemsetAsync(dev, 0, sizeof(double) * NGRAD * (size_t)c->ngacc, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (e != hipSuccess) return hip_fail(c, e, "gradient reset");
  }
  return SGP_OK;
}

int sgp_plan_widths(int n, int dtype, int* out, int max_out) {
  if (!supported_n(n) || (max_out > 0 && !out) || (dtype != SGP_C64 && dtype != SGP_C128)) return SGP_ERR_ARG;
  std::vector<int> w = plan_widths(n, dtype == SGP_C64 ? 4 : 8);
  for (int i = 0; i < (int)w.size() && i < max_out; ++i) out[i] = w[i];
  return (int)w.size();
}

int sgp_set_plan(sgp_ctx* c, int axis, int elems) {
  if (!c) return SGP_ERR_ARG;
  return c->dtype == SGP_C64 ? set_plan_impl<float>(c, axis, elems) : set_plan_impl<double>(c, axis, elems);
}

int sgp_get_plan(const sgp_ctx* c, int axis, int* elems) {
  if (c && elems && axis == SGP_PLAN_LINEAR && c->g.dim == 3) {
    *elems = c->lin_split;
    return SGP_OK;
  }
  if (!c || !elems || axis < 0 || axis >= c->g.dim) return SGP_ERR_ARG;
  *elems = c->plan_e[axis];
  return SGP_OK;
}

int sgp_autotune(sgp_ctx* c, void* psi, int steps, int elems_out[3], double* ms_per_step) {
  if (!c || !psi || !elems_out) return fail(c, SGP_ERR_ARG, "null argument");
  if (steps < 1) return fail(c, SGP_ERR_ARG, "steps must be >= 1");
  if (!c->ws) return fail(c, SGP_ERR_STATE, "no workspace set");
  if (!c->have_prop) return fail(c, SGP_ERR_STATE, "propagator not built");
  return c->dtype == SGP_C64 ? autotune_impl<float>(c, psi, steps, elems_out, ms_per_step)
                             : autotune_impl<double>(c, psi, steps, elems_out, ms_per_step);
}

int sgp_set_option(sgp_ctx* c, int option, long value) {
  if (!c) return SGP_ERR_ARG;
  if (option == SGP_OPT_GRAPH) {
    c->use_graph = value != 0;
    if (!c->use_graph) drop_graph(c);
    return SGP_OK;
  }
  if (option == SGP_OPT_FRAME) {
    if (value != SGP_FRAME_ROTATING && value != SGP_FRAME_LAB) return fail(c, SGP_ERR_ARG, "unknown frame");
    c->frame = (int)value;
    drop_graph(c);
    return SGP_OK;
  }
  if (option == SGP_OPT_SLABS) {
    if (value == 0 || value == 1) {
      c->slabs = 0;
    } else {
      if (c->g.dim != 3) return fail(c, SGP_ERR_ARG, "z-slabs need a 3D context");
      if (value < 2 || value > c->g.n[2] || c->g.n[2] % value)
        return fail(c, SGP_ERR_ARG, "the number of z-slabs must divide nz");
      c->slabs = (int)value;
    }
    drop_graph(c);
    return SGP_OK;
  }
  return fail(c, SGP_ERR_ARG, "unknown option");
}

void sgp_destroy(sgp_ctx* c) {
  if (!c) return;
  drop_graph(c);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  if (c->cap2) (void)hipStreamDestroy(c->cap2);
  for (hipEvent_t ev : c->pev)
    if (ev) (void)hipEventDestroy(ev);
  delete c;
}

const char* sgp_last_error(const sgp_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

}  // extern "C"


// ===========================================================================
// Ensembles: many 2D grids (uneven sizes, own parameters) advanced together.
// Each pass type of a step is ONE batched launch over the work list of all
// instances' tiles; the periodic step body is replayed from a HIP graph.
// ===========================================================================
struct sgp_ensemble {
  int n = 0;
  int dtype = 0;
  hipStream_t st = nullptr;
  std::vector<sgp_ctx*> ctx;
  std::vector<size_t> ws_off;
  size_t total = 0;
  // work lists per axis (0: x-lines, 1: columns) of (instance, tile) items, and
  // partitions: the instances sharing an (x, y) plan-width pair, contiguous in both
  // lists; each partition's launches run on their own stream (one batched launch
  // per pass and partition)
  size_t off_items[2] = {0, 0}, off_args = 0;
  struct Part { int ex, ey, nmax; long off[2], n[2]; };
  std::vector<Part> parts;
  char* ws = nullptr;
  // argument slots of a step (per instance one PassArgs each): the first X-pass,
  // then one slot per distinct (pass kind, duration, table) of the composition; a
  // body step and the last step of a call as slot sequences
  struct Slot { int kind; int table; double d; };
  std::vector<Slot> slots;
  std::vector<int> body, tail;
  std::vector<void*> psis;
  bool args_ok = false;
  bool use_graph = true;
  bool batched = true;
  hipStream_t cap = nullptr;
  // side streams and events of the fork/join that runs the width groups of one pass
  // concurrently (they touch different instances)
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> ev_join;
  hipEvent_t ev_fork = nullptr;
  hipGraphExec_t gexec = nullptr;
  int gsteps = 0;
  int scheme = 0;
  double tau = 0.0;
  double t = 0.0;
  std::string err;
};

namespace {

thread_local std::string g_ens_err;

int efail(sgp_ensemble* e, int code, const std::string& msg) {
  if (e) e->err = msg;
  else g_ens_err = msg;
  return code;
}

// Most argument slots a composition needs (TS6: first, three inner and one merged
// X-pass durations, the last X-pass, four propagator tables).
constexpr int ES_MAX = 12;

// The slots and the body / last-step sequences of the ensemble's composition
// (Sec. 3.3), from the same Composition as single grids: a body step is
// L(B[0]) N(A[1]) ... L(B[m-2]) N(A[m-1] + A[0]) (the merged flow), the last step
// ends with N(A[m-1]); slot 0 is the first N(A[0]) (clock from the host).
void ens_build_slots(sgp_ensemble* e) {
  const Composition k = composition(e->scheme);
  const double tau = e->tau;
  const size_t m = k.A.size();
  e->slots.clear();
  e->body.clear();
  e->tail.clear();
  auto slot = [&](int kind, int table, double d) {
    for (size_t i = 0; i < e->slots.size(); ++i)
      if (e->slots[i].kind == kind && e->slots[i].table == table && e->slots[i].d == d) return (int)i;
    e->slots.push_back({kind, table, d});
    return (int)e->slots.size() - 1;
  };
  slot(X_FIRST, -1, k.A[0] * tau);
  for (size_t j = 0; j + 1 < m; ++j) {
    const int l = slot(C_PROP, k.tab[j], k.B[j] * tau);
    e->body.push_back(l);
    e->tail.push_back(l);
    if (j + 2 < m) {
      const int x = slot(X_MID, -1, k.A[j + 1] * tau);
      e->body.push_back(x);
      e->tail.push_back(x);
    } else {
      e->body.push_back(slot(X_MID, -1, (k.A[m - 1] + k.A[0]) * tau));
      e->tail.push_back(slot(X_LAST, -1, k.A[m - 1] * tau));
    }
  }
}

void drop_egraph(sgp_ensemble* e) {
  if (e->gexec) (void)hipGraphExecDestroy(e->gexec);
  e->gexec = nullptr;
  e->gsteps = 0;
}

// Build all PassArgs slots for the current state pointers and upload them.
hipError_t ens_upload_args(sgp_ensemble* e) {
  const size_t ns = e->slots.size();
  std::vector<PassArgs> host(ns * e->n);
  for (int i = 0; i < e->n; ++i) {
    sgp_ctx* c = e->ctx[i];
    for (size_t sl = 0; sl < ns; ++sl) {
      const sgp_ensemble::Slot& S = e->slots[sl];
      PassArgs a = base_args(c);
      a.state = e->psis[i];
      a.gacc = (double*)c->at(c->off_gacc);
      a.d = S.d;
      if (S.kind != C_PROP) {
        a.tw_fwd = c->at(c->off_tw[0][0]);
        a.tw_inv = c->at(c->off_tw[0][1]);
        a.clock_mode = S.kind == X_FIRST ? CLOCK_ARG : CLOCK_DEVICE;
        a.s_arg = e->t;
        a.n_line = c->g.n[0];
      } else {
        column_geometry(c, 1, a);
        a.cs = c->at(c->off_cs[S.table]);
        a.kin_a = c->at(c->off_kin[S.table][0]);
        a.kin_o = c->at(c->off_kin[S.table][1]);
        a.kin_l = c->at(c->off_kin[S.table][1]);
        a.advance_clock = 1;
        a.n_line = c->g.n[1];
      }
      host[sl * e->n + i] = a;
    }
  }
  hipError_t r = hipMemcpyAsync(e->ws + e->off_args, host.data(), sizeof(PassArgs) * host.size(),
                                hipMemcpyHostToDevice, e->st);
  if (r == hipSuccess) r = hipStreamSynchronize(e->st);
  return r;
}

// Make sure n side streams and join events (and the fork event) exist.
hipError_t ens_side_streams(sgp_ensemble* e, size_t n) {
  hipError_t r = hipSuccess;
  if (!e->ev_fork) r = hipEventCreateWithFlags(&e->ev_fork, hipEventDisableTiming);
  while (r == hipSuccess && e->side.size() < n) {
    hipStream_t sst = nullptr;
    r = hipStreamCreateWithFlags(&sst, hipStreamNonBlocking);
    if (r == hipSuccess) e->side.push_back(sst);
  }
  while (r == hipSuccess && e->ev_join.size() < n) {
    hipEvent_t ev = nullptr;
    r = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (r == hipSuccess) e->ev_join.push_back(ev);
  }
  return r;
}

// Tiles of an instance along one axis for plan width w (2D: N lines either way).
long ens_tiles(int N, int w) {
  const int W = lines_per_block(N, w);
  return (N + W - 1) / W;
}

// Rebuild and upload the work lists for the instances' current plans, one
// contiguous run of items per partition (width pair) in each list.
hipError_t ens_build_items(sgp_ensemble* e) {
  std::vector<std::pair<int, int>> pairs;
  for (auto* c : e->ctx) {
    const std::pair<int, int> wp(c->plan_e[0], c->plan_e[1]);
    if (std::find(pairs.begin(), pairs.end(), wp) == pairs.end()) pairs.push_back(wp);
  }
  std::sort(pairs.begin(), pairs.end());
  e->parts.clear();
  for (const auto& wp : pairs) {
    sgp_ensemble::Part P{wp.first, wp.second, 0, {0, 0}, {0, 0}};
    for (auto* c : e->ctx)
      if (c->plan_e[0] == P.ex && c->plan_e[1] == P.ey) P.nmax = std::max(P.nmax, c->g.n[0]);
    e->parts.push_back(P);
  }
  for (int ax = 0; ax < 2; ++ax) {
    std::vector<int2> items;
    for (auto& P : e->parts) {
      const int w = ax == 0 ? P.ex : P.ey;
      P.off[ax] = (long)items.size();
      for (int i = 0; i < e->n; ++i) {
        if (e->ctx[i]->plan_e[0] != P.ex || e->ctx[i]->plan_e[1] != P.ey) continue;
        const long nt = ens_tiles(e->ctx[i]->g.n[0], w);
        for (long t = 0; t < nt; ++t) items.push_back(make_int2(i, (int)t));
      }
      P.n[ax] = (long)items.size() - P.off[ax];
      // block b of a launch runs on XCD b % 8: give each XCD one contiguous range of
      // the partition's items (XCD j gets n/8 items, one more when j < n % 8), so
      // neighbouring tiles, which share cache lines, share that XCD's L2
      const long n = P.n[ax];
      std::vector<int2> perm(n);
      for (long b = 0; b < n; ++b) {
        const long j = b % 8, start = j * (n / 8) + std::min(j, n % 8);
        perm[b] = items[P.off[ax] + start + b / 8];
      }
      std::copy(perm.begin(), perm.end(), items.begin() + P.off[ax]);
    }
    hipError_t r = hipMemcpyAsync(e->ws + e->off_items[ax], items.data(), sizeof(int2) * items.size(),
                                  hipMemcpyHostToDevice, e->st);
    if (r != hipSuccess) return r;
  }
  return hipStreamSynchronize(e->st);
}

// One slot's batched pass over the instances of partition P, on stream st.
template <typename T>
hipError_t ens_launch_part(sgp_ensemble* e, const sgp_ensemble::Part& P, hipStream_t st, int slot) {
  const PassArgs* args = (const PassArgs*)(e->ws + e->off_args) + (size_t)slot * e->n;
  const int kind = e->slots[slot].kind;
  const int ax = kind == C_PROP ? 1 : 0;
  const int2* items = (const int2*)(e->ws + e->off_items[ax]);
  return launch_pass_batched<T>(kind, ax == 0 ? P.ex : P.ey, items + P.off[ax], args, P.n[ax], P.nmax, st);
}

// Run fn(partition, stream) for every partition, each on its own stream, between one
// fork and one join event on st (parallel branches when st is being captured).
template <typename F>
hipError_t ens_fork_run(sgp_ensemble* e, hipStream_t st, F&& fn) {
  const size_t np = e->parts.size();
  hipError_t r = np > 1 ? ens_side_streams(e, np - 1) : hipSuccess;
  if (r != hipSuccess) return r;
  if (np > 1) r = hipEventRecord(e->ev_fork, st);
  size_t forked = 1;  // streams that may hold work of this call (st always)
  for (; forked < np && r == hipSuccess; ++forked) r = hipStreamWaitEvent(e->side[forked - 1], e->ev_fork, 0);
  for (size_t k = 0; k < forked && r == hipSuccess; ++k) r = fn(e->parts[k], k == 0 ? st : e->side[k - 1]);
  // join every forked side stream even after an error, so that st never runs
  // ahead of work already queued on them; the first error is returned
  for (size_t k = 1; k < forked; ++k) {
    hipError_t q = hipEventRecord(e->ev_join[k - 1], e->side[k - 1]);
    if (q == hipSuccess) q = hipStreamWaitEvent(st, e->ev_join[k - 1], 0);
    if (r == hipSuccess) r = q;
  }
  return r;
}

// The slot sequence `slots`, repeated `reps` times, for every partition.
template <typename T>
hipError_t ens_run_parts(sgp_ensemble* e, hipStream_t st, const std::vector<int>& slots, long reps) {
  return ens_fork_run(e, st, [&](const sgp_ensemble::Part& P, hipStream_t sst) {
    hipError_t r = hipSuccess;
    for (long b = 0; b < reps && r == hipSuccess; ++b)
      for (int sl : slots)
        if (r == hipSuccess) r = ens_launch_part<T>(e, P, sst, sl);
    return r;
  });
}

// A forward call: every partition runs its own launch sequence on its own stream
// (one fork and one join per phase: first pass, graph replays, rest), so passes of
// different partitions overlap freely.
template <typename T>
int ens_step_impl(sgp_ensemble* e, long nsteps) {
  hipError_t r = ens_run_parts<T>(e, e->st, {0}, 1);
  if (r != hipSuccess) return efail(e, SGP_ERR_HIP, std::string("batched launch: ") + hipGetErrorString(r));
  long nbody = nsteps - 1;
  const int G = 16;
  if (e->use_graph && nbody >= G) {
    if (!e->gexec || e->gsteps != G) {
      drop_egraph(e);
      if (!e->cap && (r = hipStreamCreateWithFlags(&e->cap, hipStreamNonBlocking)) != hipSuccess)
        return efail(e, SGP_ERR_HIP, "stream create");
      // side streams exist before the capture starts (no stream creation inside it)
      if (e->parts.size() > 1 && (r = ens_side_streams(e, e->parts.size() - 1)) != hipSuccess)
        return efail(e, SGP_ERR_HIP, "stream create");
      r = hipStreamBeginCapture(e->cap, hipStreamCaptureModeThreadLocal);
      if (r != hipSuccess) return efail(e, SGP_ERR_HIP, "graph capture");
      hipError_t r1 = ens_run_parts<T>(e, e->cap, e->body, G);
      hipGraph_t g = nullptr;
      r = hipStreamEndCapture(e->cap, &g);
      if (r1 != hipSuccess || r != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return efail(e, SGP_ERR_HIP, "graph capture");
      }
      r = hipGraphInstantiate(&e->gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (r != hipSuccess) { e->gexec = nullptr; return efail(e, SGP_ERR_HIP, "graph instantiate"); }
      e->gsteps = G;
    }
    for (long i = 0; i < nbody / G; ++i)
      if ((r = hipGraphLaunch(e->gexec, e->st)) != hipSuccess) return efail(e, SGP_ERR_HIP, "graph launch");
    nbody %= G;
  }
  std::vector<int> rest;
  for (long b = 0; b < nbody; ++b)
    for (int sl : e->body) rest.push_back(sl);
  for (int sl : e->tail) rest.push_back(sl);
  if ((r = ens_run_parts<T>(e, e->st, rest, 1)) != hipSuccess) return efail(e, SGP_ERR_HIP, "batched launch");
  return SGP_OK;
}

// ---- ensemble adjoint: forward with stores and reverse sweep, batched ----------
// The caller's store buffer holds, 256-byte aligned: one PassArgs per instance for
// each of the 2M+1 launches of a call (M linear substeps), then each instance's
// store of 2M+1 states (as sgp_step_store: slot 2k the input of the k-th nonlinear
// substep, slot 2k+1 the Fourier-space input of the k-th propagator).
size_t ens_args_bytes(const sgp_ensemble* e, long M) { return align256(sizeof(PassArgs) * (2 * M + 1) * e->n); }

size_t ens_inst_store(const sgp_ensemble* e, int i, long nsteps) {
  size_t b = 0;
  sgp_store_size(e->ctx[i], nsteps, &b);
  return align256(b);
}

PassArgs ens_xargs(sgp_ctx* c, void* state, int kind, double d, double s, void* store, const void* fwd) {
  PassArgs a = base_args(c);
  a.state = state;
  a.n_line = c->g.n[0];
  a.tw_fwd = c->at(c->off_tw[0][0]);
  a.tw_inv = c->at(c->off_tw[0][1]);
  a.d = d;
  a.s_arg = s;
  a.clock_mode = CLOCK_ARG;
  a.store = store;
  a.fwd = fwd;
  a.gacc = (double*)c->at(c->off_gacc);
  (void)kind;
  return a;
}

PassArgs ens_cargs(sgp_ctx* c, void* state, int kind, int table, double d, void* store, const void* fwd) {
  PassArgs a = base_args(c);
  column_geometry(c, 1, a);
  a.state = state;
  a.n_line = c->g.n[1];
  a.cs = c->at(c->off_cs[table]);
  a.kin_a = c->at(c->off_kin[table][0]);
  a.kin_o = c->at(c->off_kin[table][1]);
  a.kin_l = c->at(c->off_kin[table][1]);
  a.d = d;
  a.advance_clock = kind == C_PROP ? 1 : 0;
  a.store = store;
  a.fwd = fwd;
  a.gacc = (double*)c->at(c->off_gacc);
  return a;
}

template <typename T>
int ens_adjoint_run(sgp_ensemble* e, void* const* states, long nsteps, char* store, bool forward) {
  std::vector<double> nl, lin;
  std::vector<int> tab;
  schedule(e->ctx[0], nsteps, nl, lin, tab);
  const long M = (long)lin.size();
  std::vector<size_t> off(e->n);
  size_t o = ens_args_bytes(e, M);
  for (int i = 0; i < e->n; ++i) { off[i] = o; o += ens_inst_store(e, i, nsteps); }
  std::vector<double> s(M + 1);
  s[0] = e->t;
  for (long k = 0; k < M; ++k) s[k + 1] = s[k] + lin[k];
  // launch list: (kind, per-instance args)
  std::vector<int> kinds;
  std::vector<PassArgs> host;
  host.reserve((size_t)(2 * M + 1) * e->n);
  auto slot = [&](int i, long q) { return (void*)(store + off[i] + (size_t)q * e->ctx[i]->npts() * 5 * 2 * e->ctx[i]->esize); };
  if (forward) {
    for (long L = 0; L < 2 * M + 1; ++L) {
      int kind;
      if (L == 0) kind = X_FIRST;
      else if (L % 2 == 1) kind = C_PROP;
      else kind = (L == 2 * M) ? X_LAST : X_MID;
      kinds.push_back(kind);
      for (int i = 0; i < e->n; ++i) {
        sgp_ctx* c = e->ctx[i];
        if (kind == C_PROP) {
          const long k = (L - 1) / 2;
          host.push_back(ens_cargs(c, states[i], kind, tab[k], lin[k], slot(i, L), nullptr));
        } else {
          const long k = L / 2;  // nonlinear substep k at clock s[k]
          host.push_back(ens_xargs(c, states[i], kind, nl[k], s[k], slot(i, L), nullptr));
        }
      }
    }
  } else {
    for (long L = 2 * M; L >= 0; --L) {
      int kind;
      if (L == 2 * M) kind = XA_LAST;
      else if (L % 2 == 1) kind = C_ADJ;
      else kind = L == 0 ? XA_FIRST : XA_MID;
      kinds.push_back(kind);
      for (int i = 0; i < e->n; ++i) {
        sgp_ctx* c = e->ctx[i];
        if (kind == C_ADJ) {
          const long k = (L - 1) / 2;
          host.push_back(ens_cargs(c, states[i], kind, tab[k], lin[k], nullptr, slot(i, L)));
        } else {
          const long k = L / 2;
          host.push_back(ens_xargs(c, states[i], kind, nl[k], s[k], nullptr, slot(i, L)));
        }
      }
    }
  }
  hipError_t r = hipMemcpyAsync(store, host.data(), sizeof(PassArgs) * host.size(), hipMemcpyHostToDevice, e->st);
  if (r == hipSuccess) r = hipStreamSynchronize(e->st);
  if (r != hipSuccess) return efail(e, SGP_ERR_HIP, "argument upload");
  // every partition runs the whole launch list on its own stream
  const PassArgs* args = (const PassArgs*)store;
  r = ens_fork_run(e, e->st, [&](const sgp_ensemble::Part& P, hipStream_t sst) {
    hipError_t rr = hipSuccess;
    for (size_t L = 0; L < kinds.size() && rr == hipSuccess; ++L) {
      const int ax = (kinds[L] == C_PROP || kinds[L] == C_ADJ) ? 1 : 0;
      const int2* items = (const int2*)(e->ws + e->off_items[ax]);
      rr = launch_pass_batched<T>(kinds[L], ax == 0 ? P.ex : P.ey, items + P.off[ax], args + L * e->n, P.n[ax],
                                  P.nmax, sst);
    }
    return rr;
  });
  if (r != hipSuccess) return efail(e, SGP_ERR_HIP, std::string("batched launch: ") + hipGetErrorString(r));
  if (forward) e->t += (double)nsteps * e->tau;
  return SGP_OK;
}

}  // namespace

extern "C" {

int sgp_ensemble_create(int n_inst, const sgp_grid* grids, const sgp_params* params, int dtype, void* hip_stream,
                        sgp_ensemble** out) {
  if (!grids || !params || !out || n_inst < 1) return efail(nullptr, SGP_ERR_ARG, "bad argument");
  *out = nullptr;
  sgp_ensemble* e = new (std::nothrow) sgp_ensemble();
  if (!e) return efail(nullptr, SGP_ERR_ARG, "out of host memory");
  e->n = n_inst;
  e->dtype = dtype;
  e->st = (hipStream_t)hip_stream;
  size_t off = 0;
  for (int i = 0; i < n_inst; ++i) {
    if (grids[i].dim != 2 || grids[i].n[0] != grids[i].n[1] || grids[i].n[0] < 64 || !supported_n(grids[i].n[0])) {
      delete e;
      return efail(nullptr, SGP_ERR_ARG,
                   "ensemble grids must be 2D N x N with N in {64, 128, 192, 256, 384, 512, 768}");
    }
    sgp_ctx* c = nullptr;
    int rc = sgp_create(&grids[i], &params[i], dtype, hip_stream, &c);
    if (rc != SGP_OK) {
      std::string m = sgp_last_error(nullptr);
      for (auto* cc : e->ctx) sgp_destroy(cc);
      delete e;
      return efail(nullptr, rc, "instance " + std::to_string(i) + ": " + m);
    }
    e->ctx.push_back(c);
    e->ws_off.push_back(off);
    off += align256(c->total);
  }
  // work-list room: the most tiles any batched plan gives each instance
  long cap = 0;
  for (auto* c : e->ctx) {
    long most = 0;
    for (int w : kPlanElems)
      if (batched_plan_ok(c->g.n[0], w, (int)c->esize)) most = std::max(most, ens_tiles(c->g.n[0], w));
    cap += most;
  }
  for (int ax = 0; ax < 2; ++ax) {
    e->off_items[ax] = off;
    off += align256(sizeof(int2) * cap);
  }
  e->off_args = off;
  off += align256(sizeof(PassArgs) * ES_MAX * n_inst);
  e->total = off;
  e->psis.assign(n_inst, nullptr);
  *out = e;
  return SGP_OK;
}

int sgp_ensemble_workspace_size(const sgp_ensemble* e, size_t* bytes) {
  if (!e || !bytes) return SGP_ERR_ARG;
  *bytes = e->total;
  return SGP_OK;
}

int sgp_ensemble_set_workspace(sgp_ensemble* e, void* dev_ptr, size_t bytes) {
  if (!e || !dev_ptr) return efail(e, SGP_ERR_ARG, "null argument");
  if (bytes < e->total) return efail(e, SGP_ERR_WORKSPACE, "workspace too small");
  if (((uintptr_t)dev_ptr) & 255) return efail(e, SGP_ERR_ARG, "workspace must be 256-byte aligned");
  e->ws = (char*)dev_ptr;
  for (int i = 0; i < e->n; ++i) {
    int rc = sgp_set_workspace(e->ctx[i], e->ws + e->ws_off[i], e->ctx[i]->total);
    if (rc != SGP_OK) return efail(e, rc, "instance " + std::to_string(i) + ": " + e->ctx[i]->err);
  }
  hipError_t r = ens_build_items(e);
  if (r != hipSuccess) return efail(e, SGP_ERR_HIP, "work list upload");
  e->args_ok = false;
  drop_egraph(e);
  return SGP_OK;
}

int sgp_ensemble_build_propagator(sgp_ensemble* e, double tau, int scheme) {
  if (!e) return SGP_ERR_ARG;
  if (!e->ws) return efail(e, SGP_ERR_STATE, "no workspace set");
  if (scheme != SGP_TS2 && scheme != SGP_TS4 && scheme != SGP_TS6)
    return efail(e, SGP_ERR_ARG, "ensembles run SGP_TS2, SGP_TS4 or SGP_TS6");
  for (int i = 0; i < e->n; ++i) {
    int rc = sgp_build_propagator(e->ctx[i], tau, scheme);
    if (rc != SGP_OK) return efail(e, rc, "instance " + std::to_string(i) + ": " + e->ctx[i]->err);
  }
  e->scheme = scheme;
  e->tau = tau;
  ens_build_slots(e);
  e->args_ok = false;
  drop_egraph(e);
  return SGP_OK;
}

int sgp_ensemble_step(sgp_ensemble* e, void* const* psi_devs, long nsteps) {
  if (!e || !psi_devs) return efail(e, SGP_ERR_ARG, "null argument");
  if (nsteps < 0) return efail(e, SGP_ERR_ARG, "nsteps must be >= 0");
  if (!e->ws) return efail(e, SGP_ERR_STATE, "no workspace set");
  if (e->scheme == 0) return efail(e, SGP_ERR_STATE, "propagator not built");
  if (nsteps == 0) return SGP_OK;
  for (int i = 0; i < e->n; ++i)
    if (!psi_devs[i]) return efail(e, SGP_ERR_ARG, "null state pointer");
  if (!e->batched) {
    for (int i = 0; i < e->n; ++i) {
      e->ctx[i]->t = e->t;
      int rc = sgp_step(e->ctx[i], psi_devs[i], nsteps);
      if (rc != SGP_OK) return efail(e, rc, e->ctx[i]->err);
    }
    e->t += nsteps * e->tau;
    return SGP_OK;
  }
  bool same = e->args_ok;
  for (int i = 0; i < e->n && same; ++i) same = e->psis[i] == psi_devs[i];
  // the first X-pass of a call carries the current clock: re-upload every call
  e->psis.assign(psi_devs, psi_devs + e->n);
  hipError_t r = ens_upload_args(e);
  if (r != hipSuccess) return efail(e, SGP_ERR_HIP, "argument upload");
  if (!same) drop_egraph(e);
  e->args_ok = true;
  int rc = e->dtype == SGP_C64 ? ens_step_impl<float>(e, nsteps) : ens_step_impl<double>(e, nsteps);
  if (rc == SGP_OK) e->t += nsteps * e->tau;
  return rc;
}

int sgp_ensemble_set_plan(sgp_ensemble* e, int n, int axis, int elems) {
  if (!e) return SGP_ERR_ARG;
  if (axis < 0 || axis > 1) return efail(e, SGP_ERR_ARG, "axis must be 0 (x) or 1 (y)");
  bool any = false;
  for (auto* c : e->ctx) {
    if (c->g.n[0] != n) continue;
    const int w = elems == 0 ? default_elems(n) : elems;
    if (!batched_plan_ok(n, w, (int)c->esize))
      return efail(e, SGP_ERR_ARG, "plan width " + std::to_string(w) + " not available for batched length " +
                                       std::to_string(n));
    int rc = c->dtype == SGP_C64 ? set_plan_impl<float>(c, axis, w) : set_plan_impl<double>(c, axis, w);
    if (rc != SGP_OK) return efail(e, rc, c->err);
    any = true;
  }
  if (!any) return efail(e, SGP_ERR_ARG, "no instance of length " + std::to_string(n));
  if (e->ws) {
    hipError_t r = ens_build_items(e);
    if (r != hipSuccess) return efail(e, SGP_ERR_HIP, "work list upload");
  }
  drop_egraph(e);
  return SGP_OK;
}

int sgp_ensemble_get_plan(const sgp_ensemble* e, int n, int axis, int* elems) {
  if (!e || !elems || axis < 0 || axis > 1) return SGP_ERR_ARG;
  for (auto* c : e->ctx)
    if (c->g.n[0] == n) {
      *elems = c->plan_e[axis];
      return SGP_OK;
    }
  return SGP_ERR_ARG;
}

int sgp_ensemble_autotune(sgp_ensemble* e, void* const* psi_devs, int steps, double* ms_per_step) {
  if (!e || !psi_devs) return efail(e, SGP_ERR_ARG, "null argument");
  if (steps < 1) return efail(e, SGP_ERR_ARG, "steps must be >= 1");
  if (!e->ws) return efail(e, SGP_ERR_STATE, "no workspace set");
  if (e->scheme == 0) return efail(e, SGP_ERR_STATE, "propagator not built");
  const double t_save = e->t;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t r = hipEventCreate(&e0);
  if (r == hipSuccess) r = hipEventCreate(&e1);
  if (r != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return efail(e, SGP_ERR_HIP, "event create");
  }
  auto time_steps = [&](double* ms) -> int {
    int rc = sgp_ensemble_step(e, psi_devs, steps);  // untimed: graph capture, warm caches
    if (rc != SGP_OK) return rc;
    hipError_t q = hipEventRecord(e0, e->st);
    if (q != hipSuccess) return efail(e, SGP_ERR_HIP, "event record");
    rc = sgp_ensemble_step(e, psi_devs, steps);
    if (rc != SGP_OK) return rc;
    q = hipEventRecord(e1, e->st);
    if (q == hipSuccess) q = hipEventSynchronize(e1);
    float f = 0.f;
    if (q == hipSuccess) q = hipEventElapsedTime(&f, e0, e1);
    if (q != hipSuccess) return efail(e, SGP_ERR_HIP, "autotune timing");
    *ms = (double)f / steps;
    return SGP_OK;
  };
  std::vector<int> sizes;
  for (auto* c : e->ctx)
    if (std::find(sizes.begin(), sizes.end(), c->g.n[0]) == sizes.end()) sizes.push_back(c->g.n[0]);
  double best = 0.0;
  int rc = time_steps(&best);
  const int esize = e->dtype == SGP_C64 ? 4 : 8;
  // per instance size, every (x, y) plan pair with the other sizes at their current
  // best (the partitions of different sizes run concurrently, so the choices
  // interact); sweeps over the sizes repeat until one improves nothing (at most 3)
  for (int sweep = 0; sweep < 3 && rc == SGP_OK; ++sweep) {
    bool improved = false;
    for (size_t k = 0; k < sizes.size() && rc == SGP_OK; ++k) {
      const int n = sizes[k];
      int sx = 0, sy = 0;
      sgp_ensemble_get_plan(e, n, 0, &sx);
      sgp_ensemble_get_plan(e, n, 1, &sy);
      int bx = sx, by = sy;
      for (int wx : kPlanElems) {
        for (int wy : kPlanElems) {
          if ((wx == sx && wy == sy) || !batched_plan_ok(n, wx, esize) || !batched_plan_ok(n, wy, esize)) continue;
          double ms = 0.0;
          rc = sgp_ensemble_set_plan(e, n, 0, wx);
          if (rc == SGP_OK) rc = sgp_ensemble_set_plan(e, n, 1, wy);
          if (rc == SGP_OK) rc = time_steps(&ms);
          if (rc != SGP_OK) break;
          if (ms < best) { best = ms; bx = wx; by = wy; improved = true; }
        }
        if (rc != SGP_OK) break;
      }
      if (rc == SGP_OK) rc = sgp_ensemble_set_plan(e, n, 0, bx);
      if (rc == SGP_OK) rc = sgp_ensemble_set_plan(e, n, 1, by);
    }
    if (!improved) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  e->t = t_save;
  if (rc == SGP_OK && ms_per_step) *ms_per_step = best;
  return rc;
}

int sgp_ensemble_store_size(const sgp_ensemble* e, long nsteps, size_t* bytes) {
  if (!e || !bytes || nsteps < 1) return SGP_ERR_ARG;
  if (e->scheme == 0) return SGP_ERR_STATE;
  const long M = (long)(composition(e->scheme).A.size() - 1) * nsteps;
  size_t b = ens_args_bytes(e, M);
  for (int i = 0; i < e->n; ++i) b += ens_inst_store(e, i, nsteps);
  *bytes = b;
  return SGP_OK;
}

static int ens_adjoint_checks(sgp_ensemble* e, void* const* states, long nsteps, const void* store,
                              size_t store_bytes) {
  if (!e || !states || !store) return efail(e, SGP_ERR_ARG, "null argument");
  if (nsteps < 1) return efail(e, SGP_ERR_ARG, "nsteps must be >= 1");
  if (!e->ws) return efail(e, SGP_ERR_STATE, "no workspace set");
  if (e->scheme == 0) return efail(e, SGP_ERR_STATE, "propagator not built");
  for (int i = 0; i < e->n; ++i)
    if (!states[i]) return efail(e, SGP_ERR_ARG, "null state pointer");
  if (((uintptr_t)store) & 255) return efail(e, SGP_ERR_ARG, "store must be 256-byte aligned");
  size_t need = 0;
  sgp_ensemble_store_size(e, nsteps, &need);
  if (store_bytes < need) return efail(e, SGP_ERR_WORKSPACE, "store too small");
  return SGP_OK;
}

int sgp_ensemble_step_store(sgp_ensemble* e, void* const* psi_devs, long nsteps, void* store, size_t store_bytes) {
  int rc = ens_adjoint_checks(e, psi_devs, nsteps, store, store_bytes);
  if (rc != SGP_OK) return rc;
  return e->dtype == SGP_C64 ? ens_adjoint_run<float>(e, psi_devs, nsteps, (char*)store, true)
                             : ens_adjoint_run<double>(e, psi_devs, nsteps, (char*)store, true);
}

int sgp_ensemble_adjoint_segment(sgp_ensemble* e, void* const* lam_devs, long nsteps, void* store,
                                 size_t store_bytes) {
  int rc = ens_adjoint_checks(e, lam_devs, nsteps, store, store_bytes);
  if (rc != SGP_OK) return rc;
  return e->dtype == SGP_C64 ? ens_adjoint_run<float>(e, lam_devs, nsteps, (char*)store, false)
                             : ens_adjoint_run<double>(e, lam_devs, nsteps, (char*)store, false);
}

int sgp_ensemble_adjoint_gradients(sgp_ensemble* e, double* out, int reset) {
  if (!e || !out) return efail(e, SGP_ERR_ARG, "null argument");
  for (int i = 0; i < e->n; ++i) {
    int rc = sgp_adjoint_gradients(e->ctx[i], out + 5 * (size_t)i, reset);
    if (rc != SGP_OK) return efail(e, rc, "instance " + std::to_string(i) + ": " + e->ctx[i]->err);
  }
  return SGP_OK;
}

int sgp_ensemble_get_time(const sgp_ensemble* e, double* t) {
  if (!e || !t) return SGP_ERR_ARG;
  *t = e->t;
  return SGP_OK;
}

int sgp_ensemble_set_time(sgp_ensemble* e, double t) {
  if (!e || !std::isfinite(t)) return SGP_ERR_ARG;
  e->t = t;
  return SGP_OK;
}

int sgp_ensemble_set_option(sgp_ensemble* e, int option, long value) {
  if (!e) return SGP_ERR_ARG;
  if (option == SGP_OPT_GRAPH) { e->use_graph = value != 0; drop_egraph(e); return SGP_OK; }
  if (option == SGP_OPT_BATCHED) { e->batched = value != 0; return SGP_OK; }
  return efail(e, SGP_ERR_ARG, "unknown option");
}

void sgp_ensemble_destroy(sgp_ensemble* e) {
  if (!e) return;
  drop_egraph(e);
  if (e->cap) (void)hipStreamDestroy(e->cap);
  for (hipStream_t sst : e->side) (void)hipStreamDestroy(sst);
  for (hipEvent_t ev : e->ev_join) (void)hipEventDestroy(ev);
  if (e->ev_fork) (void)hipEventDestroy(e->ev_fork);
  for (auto* c : e->ctx) sgp_destroy(c);
  delete e;
}

const char* sgp_ensemble_last_error(const sgp_ensemble* e) { return e ? e->err.c_str() : g_ens_err.c_str(); }

}  // extern "C"

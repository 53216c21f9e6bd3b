/*
 * sgp.h -- C ABI of the MI355X (gfx950) split-step library for the rotating
 * spin-orbit-coupled spin-2 Gross-Pitaevskii system, following the compact
 * splitting Fourier spectral method of Liu, Xie, Yuan, Zhang and Zhao
 * (arXiv 2603.25282).
 *
 * The model (Sec. 1, eq. CGPEs): i d_t Psi = (H0 I5 + c1 F.f - gamma S) Psi
 *   + c2 A00 A conj(Psi), H0 = -Laplace/2 + V + c0 rho - Omega Lz, with the harmonic
 * trap V = (gx^2 x^2 + gy^2 y^2 [+ gz^2 z^2])/2 (eq. harmonic).
 *
 * Frame.  The library evolves the rotating-frame state Phi of the function-rotation
 * mapping with a phase factor (Sec. 3.1, eq. mapping): phi_l(x, t) =
 * exp(-i l Omega t) psi_l(R(t) x, t).  At t = 0, Phi equals the lab-frame Psi.  The
 * linear flow of Phi is time independent (eq. linearEQ2) and is integrated exactly
 * per wavevector (eq. sl1); the nonlinear flow (eq. solution2) sees the trap at the
 * rotated point R(Omega s) x, s being the clock advanced by the linear substeps.
 *
 * Discretisation (Sec. 3.1): domain [-L, L]^d with periodic boundary conditions,
 * N points per axis, h = 2L/N, x_j = -L + j h; wavenumbers nu_p = pi p / L,
 * p in [-N/2, N/2 - 1] (the Nyquist mode keeps nu = -pi N/(2L)).
 *
 * State layout (device memory, owned by the caller): [nz][ny][nx][5] complex,
 * interleaved (re, im), the 5 components of a grid point adjacent, then x, y, z;
 * component i = 0..4 holds spin projection l = 2, 1, 0, -1, -2.  Element type:
 * complex64 (SGP_C64) or complex128 (SGP_C128).
 *
 * Memory: the library allocates no device memory.  The caller asks for
 * sgp_workspace_size() bytes, allocates them (e.g. a torch tensor), and hands them
 * over with sgp_set_workspace(); the workspace holds FFT twiddles, propagator
 * tables, the device clock and reduction partials, and must stay valid until
 * sgp_destroy() or the next sgp_set_workspace().
 *
 * Streams: every device operation is enqueued on the stream given to
 * sgp_create() (a hipStream_t, or NULL for the default stream).  sgp_step() does
 * not synchronise; sgp_observables() and setup calls do.
 *
 * Errors: every int-returning call returns SGP_OK (0) or a negative SGP_ERR_*
 * code; sgp_last_error() gives a message.  No C++ exception crosses this ABI.
 * A context is not thread safe; use one context per stream.
 */
#ifndef SGP_H
#define SGP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SGP_OK = 0,
  SGP_ERR_ARG = -1,         /* bad argument (null pointer, unsupported size, ...) */
  SGP_ERR_STATE = -2,       /* call out of order (no workspace, no propagator)     */
  SGP_ERR_HIP = -3,         /* a HIP runtime call failed                           */
  SGP_ERR_NONFINITE = -4,   /* a non-finite value was found                        */
  SGP_ERR_WORKSPACE = -5    /* workspace too small                                 */
};

enum { SGP_C64 = 0, SGP_C128 = 1 };  /* element type of the state */
/* Time composition (Sec. 3.3): TS2 Strang, TS4 the 4th-order symplectic scheme,
 * TS6 the 6th-order triple jump S4(z1 tau) S4(z0 tau) S4(z1 tau) of TS4 (Yoshida's
 * composition, which the section cites), z1 = 1/(2 - 2^(1/5)), z0 = -2^(1/5) z1. */
enum { SGP_TS2 = 2, SGP_TS4 = 4, SGP_TS6 = 6 };

typedef struct sgp_ctx sgp_ctx;

/* Grid: dim = 2 or 3; n[0..dim-1] = points along x, y[, z]; L[] = half-widths.
 * Supported n per axis: 16, 32, 64, 128, 256, 512 and 192, 384, 768 (3 * 2^k),
 * with at most 2^31 - 1 state elements in all (5 n_x n_y n_z: every 3D grid up to
 * 768 x 768 x 512 fits, 768^3 does not); sgp_create returns SGP_ERR_ARG beyond. */
typedef struct {
  int dim;
  int n[3];
  double L[3];
} sgp_grid;

/* Physics (Sec. 1): interaction constants c0 (density), c1 (spin exchange),
 * c2 (singlet pairing); rotation speed Omega (about z); SOC strength gamma; trap
 * frequencies gx, gy, gz (gz unused in 2D). */
typedef struct {
  double c0, c1, c2, Omega, gamma, gx, gy, gz;
} sgp_params;

/* Create a context for one grid, parameter set and element type.  hip_stream is a
 * hipStream_t (NULL = default stream).  On success *out receives the context. */
int sgp_create(const sgp_grid* grid, const sgp_params* params, int dtype, void* hip_stream, sgp_ctx** out);

/* Bytes of device workspace the context needs. */
int sgp_workspace_size(const sgp_ctx* ctx, size_t* bytes);

/* Hand over caller-owned device memory of at least sgp_workspace_size() bytes
 * (256-byte aligned).  Uploads the FFT twiddle tables (synchronous). */
int sgp_set_workspace(sgp_ctx* ctx, void* dev_ptr, size_t bytes);

/* Build, in FP64 on the device, the exact linear propagator
 * exp(-i d |nu|^2 / 2) exp(i d Q) (Sec. 3.1, eq. sl1 and the closed form of
 * exp(i tau Q), precomputed once as in Remark comput-cost) for every distinct linear
 * substep d of the scheme: TS2 {tau}, TS4 {b1 tau, b2 tau}, TS6 {z1 b1, z1 b2, z0 b1,
 * z0 b2} tau.  The tables are stored
 * rounded to the state's precision.  tau may be negative (backward evolution).
 * Synchronous. */
int sgp_build_propagator(sgp_ctx* ctx, double tau, int scheme);

/* Advance the state in place by nsteps steps of the scheme built by
 * sgp_build_propagator(), from the context clock t to t + nsteps * tau (Sec. 3.3):
 *   TS2: N(tau/2) L(tau) N(tau/2)
 *   TS4: N(a1) L(b1) N(a2) L(b2) N(a2) L(b1) N(a1)   (times tau)
 * with N the exact nonlinear flow and L the exact linear flow.  Adjacent
 * nonlinear substeps of consecutive steps are merged (same clock value).
 * psi_dev: device pointer to the state (layout above), physical space on entry and
 * exit.  Asynchronous on the context stream; nsteps = 0 is a no-op. */
int sgp_step(sgp_ctx* ctx, void* psi_dev, long nsteps);

/* Observables of the state at the current clock (Sec. 2, discrete h^d sums):
 * out[0] mass N, out[1] energy E, out[2] magnetization M, out[3] <Lz>.  Spatial
 * derivatives are spectral; the trap is taken at the rotated point R(Omega t) x.
 * FP64 accumulation: per-block partial sums, added on the device in a fixed order
 * (bitwise reproducible); only the totals are copied to the host.  Returns
 * SGP_ERR_NONFINITE (out still written) when the state holds a NaN or an infinity.
 * Synchronous. */
int sgp_observables(sgp_ctx* ctx, const void* psi_dev, double out[4]);

/* For callers that cannot allocate device memory or synchronise with the host
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the four values of sgp_observables written to out_dev[0..3]
 * (caller-owned device memory, 4 doubles), computed by the same kernels with the
 * same summation order, asynchronously on the context stream.  It allocates
 * nothing and copies nothing to the host: the block partials and their sums live in
 * a fixed device scratch array of the library (8 MiB, one per GPU, kept until the
 * process ends), resolved on the first call on a device (the context's device must
 * be current).  Grids whose partials need more than that scratch are refused with
 * SGP_ERR_ARG (every 2D grid and 3D grids up to 256^3 fit; 384^3 and 512^3 do not).
 * All contexts of a process on one GPU share the scratch and each call leaves its
 * contents there: calls that may overlap in time on one GPU (contexts on different
 * streams or host threads) race and must be ordered by the caller.
 * A state holding a NaN or an infinity yields non-finite out_dev values (no
 * SGP_ERR_NONFINITE: nothing is read back). */
int sgp_observables_device(sgp_ctx* ctx, const void* psi_dev, double* out_dev);

/* The inner product <u, J_z v>_h = h^d sum_x sum_l conj(u_l(x)) (J_z v)_l(x) of two
 * states (layout above, the context's element type) with the generator of the
 * rotation about z, J_z = L_z + F_z: L_z = -i (x d_y - y d_x) (Sec. 2, the angular
 * momentum of <Lz>), spectral derivatives, and F_z = diag(2, 1, 0, -1, -2) (Sec. 1).
 * The rotation mapping of Sec. 3.1 turns a state by the angle Omega t, so
 * d/dOmega of a function of the mapped state is a real part of such a product
 * (the lab-frame output's Omega gradient).  out[0] = real part, out[1] = imaginary
 * part.  FP64 accumulation, block partials summed on the device in a fixed order.
 * u_dev and v_dev are read only (they may alias).  Returns SGP_ERR_NONFINITE when
 * the result is not finite.  Synchronous. */
int sgp_jz_inner(sgp_ctx* ctx, const void* u_dev, const void* v_dev, double out[2]);

/* The observables plus the quantities of the dynamical laws of Sec. 2, all FP64:
 * out[0..3] as sgp_observables; out[4], out[5], out[6] = the widths delta_x,
 * delta_y, delta_z (eq. ConWid: h^d sum alpha^2 rho, alpha the lab-frame coordinate
 * of the point, i.e. (x, y) rotated by Omega t in the rotating frame; delta_z = 0
 * in 2D); out[7] = h^d sum x y rho (lab frame; Lemma 1: d<Lz>/dt =
 * (gx^2 - gy^2) out[7] when gamma = 0); out[8] = W = 2 h^d Im sum conj(psi)
 * (x d_x + y d_y) psi with spectral derivatives, which equals d(delta_x +
 * delta_y)/dt when gamma = 0 (Lemma 2); out[9] = dM/dt and out[10] = d<Lz>/dt by
 * the laws of Sec. 2 (magnetization, and Lemma 1 with its spin-orbit term), from
 * the sums h^d sum conj(psi_a) L_+- psi_b (L_+- = i d_y +- d_x, spectral) over the
 * adjacent component pairs: dM/dt = -2 gamma Im[Q1 + Q2 + sqrt6/2 (Q3 - Q4)] and
 * d<Lz>/dt = (gx^2 - gy^2) out[7] + 2 gamma Im[Q2 - Q5 + sqrt6/2 (Q3 - Q4)] with
 * Q1 = <psi_2, L_- psi_1>, Q2 = <psi_-1, L_- psi_-2>, Q3 = <psi_1, L_- psi_0>,
 * Q4 = <psi_-1, L_+ psi_0>, Q5 = <psi_1, L_+ psi_2>; all frame-invariant;
 * out[11] = G(gamma, Psi), the spin-orbit term of Lemma 2's width law
 * (d^2 delta_r/dt^2 = -4 gr^2 delta_r + 4 E(0) + 4 Omega <Lz> + G for a radial trap
 * gx = gy = gr): 2 gamma Re h^d sum [Omega (i Y - X) F_+ + gamma (sum_m (6 - m^2)
 * |psi_m|^2 + sum_m m conj(psi_m) L_z psi_m)] on the lab-frame state (for a
 * rotating-frame state its lab-frame value: (X, Y) the lab-frame coordinates of the
 * point and F_+ with the components' phase exp(-i Omega t) undone), L_z spectral.
 * SGP_ERR_NONFINITE as sgp_observables.  Synchronous.  out holds 12 doubles. */
int sgp_diagnostics(sgp_ctx* ctx, const void* psi_dev, double out[12]);

/* ---- Differentiation (discrete adjoint of sgp_step) -------------------------
 * Convention: for a real loss J of the state, a gradient is g = 2 dJ/d conj(psi),
 * i.e. dJ = Re sum conj(g) dpsi over all stored values (the convention of
 * torch.autograd for complex tensors).  The adjoint of the exact linear substep is
 * the same propagator with -d (P(d)^H = P(-d)); the adjoint of the exact nonlinear
 * substep (Sec. 3.2, eq. solution2) is its real-linear (Wirtinger) transpose at the
 * stored forward input.
 *
 * Bytes of the store one sgp_step_store(nsteps) call needs: (2M + 1) states, M the
 * number of linear substeps (TS2: nsteps, TS4: 3 nsteps). */
int sgp_store_size(const sgp_ctx* ctx, long nsteps, size_t* bytes);

/* sgp_step() that also writes, for every pass, the input of its pointwise stage
 * into the caller-owned device buffer `store` (slot 2k: the k-th nonlinear
 * substep's input in physical space; slot 2k+1: the k-th propagator's input in
 * Fourier space).  No graph replay.  Advances the clock like sgp_step(). */
int sgp_step_store(sgp_ctx* ctx, void* psi_dev, long nsteps, void* store, size_t store_bytes);

/* Reverse sweep of the sgp_step_store(nsteps) call that started at the current
 * clock (set it back with sgp_set_time first).  lam_dev: on entry the gradient with
 * respect to that call's output, on exit with respect to its input (same layout as
 * the state).  Parameter gradients are accumulated on the device (FP64, one slot per
 * block, deterministic order).  Asynchronous; does not move the clock. */
int sgp_adjoint_segment(sgp_ctx* ctx, void* lam_dev, long nsteps, const void* store, size_t store_bytes);

/* Accumulated dJ/d(gamma, Omega, c0, c1, c2) of all sgp_adjoint_segment() calls since
 * the last reset (the per-block slots summed on the device in a fixed order; five
 * doubles come back); reset = 1 clears the accumulators.  Synchronous. */
int sgp_adjoint_gradients(sgp_ctx* ctx, double out[5], int reset);

/* Rotation clock t (the time of the rotating frame the state lives in). */
int sgp_get_time(const sgp_ctx* ctx, double* t);
int sgp_set_time(sgp_ctx* ctx, double t);

/* Measurement: average duration in milliseconds of one pass over the state,
 * launched `reps` times back to back on the context stream between two HIP
 * events (the state is overwritten with transformed data).  pass: 0 = X-pass
 * (inverse FFT along x, nonlinear flow, forward FFT; the nonlinear flow of
 * Sec. 3.2); 1 = y-pass (2D: FFT along y, propagator, inverse FFT; 3D: forward
 * FFT along y); 2 = z-pass with the propagator (3D); 3 = inverse y-pass (3D).
 * With pass | SGP_TIME_IN_STEP the passes of a substep run in step order (2D:
 * y, X; 3D: y, z, inverse y, X) `reps` times and only the launches of the named
 * pass are timed, each between its own pair of events (its data then comes from
 * the previous pass, as inside sgp_step).  With pass | SGP_TIME_STEPS, `reps` (>= 2)
 * whole steps of sgp_step's schedule run (launched without the graph; psi
 * advances, the context time is restored) and every launch of the named pass in
 * them is timed by a start/end event pair that its dispatch stamps (pass 0: the
 * X-passes between two linear substeps); the rotating frame only.  In both modes
 * that time every launch, reps <= 4096.  Requires a built propagator.
 * Synchronous. */
enum { SGP_TIME_IN_STEP = 256, SGP_TIME_STEPS = 512 };
int sgp_time_pass(sgp_ctx* ctx, void* psi_dev, int pass, int reps, double* avg_ms);

/* Register plans of the FFT line kernels.  Every pass along an axis of length n
 * transforms each (line, component) with n/E threads holding E elements each; E
 * fixes the radix sequence (E = 8: radix 8 with one radix-2/4 pass; E = 4: radix 4
 * with one radix-2 pass; E = 16: radix 16 for 128 and 256, else radix 8 with two
 * butterflies per thread; 192,
 * 384, 768: E = 12 (radix 12, 6 for 384, then radix 4) or, for SGP_C64 only,
 * E = 24 (radix 3, 6 for 384, 12 for 768, then radix 8))
 * and the block shape.  Every plan computes the same transform (results differ by
 * rounding only).  Defaults: E = 8, or 12 for 192, 384, 768.
 *
 * sgp_plan_widths: writes up to max_out widths available for length n and
 *   element type dtype (the default first) to out and returns how many there
 *   are; SGP_ERR_ARG for an unsupported n or dtype.
 * sgp_set_plan: plan width of the passes along `axis` (0 = x, 1 = y, 2 = z);
 *   elems = 0 restores the default.  SGP_ERR_ARG if the width is not available
 *   for that axis's length.  Rewrites the twiddle tables in the workspace (if set)
 *   and drops the captured step graph; call it between steps, not concurrently
 *   with work on the context's stream.
 * sgp_get_plan: the current width of `axis`.
 * Pseudo-axis SGP_PLAN_LINEAR (3D contexts only; SGP_ERR_ARG otherwise): how a
 *   linear substep's passes split the propagator of eq. sl1, whose spin part
 *   exp(i d Q) depends on (nu_p, nu_q) only (Sec. 3.1, 3D): 0 (default) = FFT
 *   along y, then along z the FFT, the whole propagator and the inverse FFT, then
 *   the inverse FFT along y; 1 = FFT along y with the x and y kinetic phases and
 *   the spin part applied there, then along z the FFT, the z kinetic phase and the
 *   inverse FFT, then the inverse FFT along y.  Same results up to rounding; with
 *   sgp_set_plan(ctx, SGP_PLAN_LINEAR, 0 or 1) and sgp_get_plan likewise.  The
 *   differentiable path (sgp_step_store, the adjoint) always uses split 0.
 * sgp_autotune: picks the fastest combination of the axes' widths (every
 *   combination, at most 9 in 2D and 27 in 3D, in 3D for both linear-substep
 *   splits) by timing `steps` steps of the
 *   sgp_step path for each, after one untimed call of `steps` steps; psi_dev is
 *   a device state in the layout of sgp_step; it is advanced by every timed and
 *   untimed step (pass a scratch copy).  Needs the workspace and the propagator;
 *   the context time is left unchanged.  Writes the chosen widths to elems_out
 *   (0 for axes beyond dim) and, if ms_per_step is not NULL, the fastest time per
 *   step in ms.  The choice (and in 3D the split, read back with sgp_get_plan)
 *   stays set on the context. */
enum { SGP_PLAN_LINEAR = 3 };
int sgp_plan_widths(int n, int dtype, int* out, int max_out);
int sgp_set_plan(sgp_ctx* ctx, int axis, int elems);
int sgp_get_plan(const sgp_ctx* ctx, int axis, int* elems);
int sgp_autotune(sgp_ctx* ctx, void* psi_dev, int steps, int elems_out[3], double* ms_per_step);

/* Options.  SGP_OPT_GRAPH (default 1): replay the periodic part of sgp_step()
 * from a captured HIP graph (value 0 launches every kernel individually). */
enum { SGP_OPT_GRAPH = 1, SGP_OPT_BATCHED = 2, SGP_OPT_FRAME = 3, SGP_OPT_SLABS = 4 };
/* SGP_OPT_SLABS (3D contexts; default 0 = off): S >= 2 z-slabs, S dividing nz.  With
 * the graph replay and the linear-substep split 0, the passes of a step that act on
 * each z-plane alone (the inverse y-pass, the x-pass, the next forward y-pass; Sec.
 * 3.1's 3D step) run slab by slab between two z-passes, alternate slabs on a second
 * stream, so that the bandwidth-bound y-passes of one slab overlap the x-pass of
 * another.  Bitwise the same results.  SGP_ERR_ARG for a 2D context or an S that does
 * not divide nz; 0 or 1 switches it off. */
/* SGP_OPT_FRAME: SGP_FRAME_ROTATING (default) evolves Phi in the rotating frame
 * (trap at R(Omega s) x, merged nonlinear substeps, graph replay); SGP_FRAME_LAB runs
 * Algorithm 1 literally on the lab-frame Psi: nonlinear substeps with the trap at x
 * (not merged) and the rotation mapping before and its inverse after every linear
 * substep (Sec. 3.3).  In the lab frame sgp_observables evaluates the trap at x, and
 * sgp_step_store / sgp_adjoint_segment return SGP_ERR_STATE. */
enum { SGP_FRAME_ROTATING = 0, SGP_FRAME_LAB = 1 };
int sgp_set_option(sgp_ctx* ctx, int option, long value);

/* Rotation mapping (Sec. 3.1, eqs. RSDA1/RSDA2) in place on a physical-space state
 * [nz][ny][nx][5]: direction +1 maps the lab-frame Psi to Phi = M_t Psi,
 * phi_l(x) = exp(-i l Omega t) psi_l(R(Omega t) x); direction -1 maps back, Psi =
 * M_t^{-1} Phi.  The rotation (about z in 3D) is three shears
 * exp(a y d_x) exp(b x d_y) exp(a y d_x), a = +-tan(Omega t/2), b = -+sin(Omega t),
 * each a transform along one axis, a phase per Fourier coefficient and the
 * inverse transform (spectrally exact for band-limited data).  SGP_ERR_ARG when
 * |cos(Omega t/2)| < 1e-6 (the shear factorisation degenerates at angle pi).
 * Needs the workspace (twiddles); asynchronous on the context stream. */
int sgp_rotation_map(sgp_ctx* ctx, void* psi_dev, double t, int direction);

/* Release the context (not the caller's workspace or state). */
void sgp_destroy(sgp_ctx* ctx);

/* Message of the last error on this context ("" if none); ctx may be NULL for
 * errors raised by sgp_create(). */
const char* sgp_last_error(const sgp_ctx* ctx);

/* ---- Ensembles of 2D grids -------------------------------------------------
 * Many independent 2D instances (square grids with N in {64, 128, 192, 256, 384, 512, 768},
 * each with its own domain and parameters, same element type and scheme) advanced
 * together: every pass type of a step is one batched launch (per register plan
 * width in use) over the work list of the instances' line tiles, and the periodic
 * part of a step is replayed from one HIP graph.  Each instance evolves exactly as with its own context (same kernels
 * per line; results are bitwise identical). */
typedef struct sgp_ensemble sgp_ensemble;

int sgp_ensemble_create(int n_inst, const sgp_grid* grids, const sgp_params* params, int dtype, void* hip_stream,
                        sgp_ensemble** out);
/* One caller-owned workspace for all instances (tables, twiddles, work lists). */
int sgp_ensemble_workspace_size(const sgp_ensemble* ens, size_t* bytes);
int sgp_ensemble_set_workspace(sgp_ensemble* ens, void* dev_ptr, size_t bytes);
/* FP64 propagator tables of every instance for the common tau and scheme
 * (SGP_TS2, SGP_TS4 or SGP_TS6; the step's launch sequence follows the scheme's
 * composition, Sec. 3.3, as for single grids).  SGP_ERR_ARG for another scheme. */
int sgp_ensemble_build_propagator(sgp_ensemble* ens, double tau, int scheme);
/* psi_devs: host array of n_inst device pointers (instance i: [ny][nx][5] complex).
 * Advances every instance by nsteps (common clock).  Asynchronous. */
int sgp_ensemble_step(sgp_ensemble* ens, void* const* psi_devs, long nsteps);
/* SGP_OPT_GRAPH (default 1) as for contexts; SGP_OPT_BATCHED (default 1): 0 runs
 * every instance with its own launches (the unbatched reference). */
int sgp_ensemble_set_option(sgp_ensemble* ens, int option, long value);
/* Register plans of an ensemble (see sgp_set_plan): the width used along `axis`
 * (0 = x-lines, 1 = y-lines) by every instance of size n x n.  Batched kernels
 * run the 320-thread geometry, so the widths available are those of
 * sgp_plan_widths(n, dtype) with n/E <= 64 (all but E = 4 at n = 512).  The
 * instances sharing an (x, y) width pair form a partition; each partition runs its
 * passes (one batched launch per pass) on its own stream.
 * sgp_ensemble_set_plan: elems = 0 restores the default; SGP_ERR_ARG if the width
 *   is not available or no instance has size n.  Drops the captured step graph.
 * sgp_ensemble_get_plan: the width of the first instance of size n.
 * sgp_ensemble_autotune: for each instance size in turn (the others at their
 *   current best), times `steps` ensemble steps for every (x, y) width pair (after
 *   one untimed call of `steps` steps) and keeps the fastest, sweeping over the
 *   sizes until a sweep improves nothing (at most three sweeps); psi_devs are
 *   advanced by every step (pass scratch copies); the ensemble time is restored;
 *   ms_per_step (if not NULL) receives the fastest time per step. */
int sgp_ensemble_set_plan(sgp_ensemble* ens, int n, int axis, int elems);
int sgp_ensemble_get_plan(const sgp_ensemble* ens, int n, int axis, int* elems);
int sgp_ensemble_autotune(sgp_ensemble* ens, void* const* psi_devs, int steps, double* ms_per_step);

/* Ensemble adjoint (the batched counterpart of sgp_step_store /
 * sgp_adjoint_segment / sgp_adjoint_gradients): the same passes, one batched
 * launch per pass type and plan width over all instances.
 * sgp_ensemble_store_size: bytes of the caller's store for nsteps steps (one
 *   argument block per launch, then every instance's 2M+1 stored states).
 * sgp_ensemble_step_store: forward nsteps from the ensemble clock, storing every
 *   pass's pointwise-stage input (store: device, 256-byte aligned); advances the
 *   clock.
 * sgp_ensemble_adjoint_segment: with the clock set back to the start of the
 *   matching sgp_ensemble_step_store call (sgp_ensemble_set_time), replaces each
 *   lam_devs[i] (gradient w.r.t. that call's output, 2 dJ/d conj(Phi)) by the
 *   gradient w.r.t. its input, and adds each instance's parameter partials to its
 *   accumulators.  It rewrites the argument block at the front of the store.
 * sgp_ensemble_adjoint_gradients: out[5 i + q] = dJ/d(gamma, Omega, c0, c1, c2)[q]
 *   of instance i accumulated since the last reset; reset = 1 clears.  Synchronous.
 * Rotating frame only (as for contexts). */
int sgp_ensemble_store_size(const sgp_ensemble* ens, long nsteps, size_t* bytes);
int sgp_ensemble_step_store(sgp_ensemble* ens, void* const* psi_devs, long nsteps, void* store, size_t store_bytes);
int sgp_ensemble_adjoint_segment(sgp_ensemble* ens, void* const* lam_devs, long nsteps, void* store,
                                 size_t store_bytes);
int sgp_ensemble_adjoint_gradients(sgp_ensemble* ens, double* out, int reset);
/* Ensemble clock (all instances share it). */
int sgp_ensemble_get_time(const sgp_ensemble* ens, double* t);
int sgp_ensemble_set_time(sgp_ensemble* ens, double t);

void sgp_ensemble_destroy(sgp_ensemble* ens);
const char* sgp_ensemble_last_error(const sgp_ensemble* ens);

#ifdef __cplusplus
}
#endif

#endif /* SGP_H */

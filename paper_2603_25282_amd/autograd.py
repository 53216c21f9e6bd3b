"""Differentiable evolution: torch.autograd.Function over the C-ABI forward and
adjoint split steps, with checkpointed recomputation every K steps.

    phi_T = evolve(psi0, params, shape, L, trap, tau, nsteps, order=4, K=50)

psi0: complex device tensor in the library layout (..., nx, 5); params: real tensor
(gamma, Omega, c0, c1, c2).  Gradients follow torch's convention for complex tensors
(2 dJ/d conj(psi)); the library's adjoint uses the same one.  Memory: the forward
keeps a checkpoint at the start of every K-step segment and runs the last segment
with stores (one segment store of (2M + 1) states, M linear substeps of K steps),
which the first backward uses without recomputing that segment; the backward holds
that one store at a time (a second backward recomputes every segment).
"""
import math

import torch

from .sgp import Solver

PARAM_ORDER = ("gamma", "Omega", "c0", "c1", "c2")


def _solver(shape, L, params, trap, dtype, tau, order, plan=None, psi=None):
    g, Om, c0, c1, c2 = [float(x) for x in params]
    s = Solver(shape, L, (c0, c1, c2, Om, g, trap[0], trap[1], trap[2]), dtype=dtype)
    s.build_propagator(tau, order)
    if plan == "auto":
        s.autotune(psi, order)
    elif plan is not None:
        s.set_plan(plan)
    return s


def check_solver(s, psi0, params, shape, L, trap, tau, order):
    """A prebuilt Solver must be the one evolve() would build: same grid, physics
    (params = (gamma, Omega, c0, c1, c2) and trap), element type, tau and scheme."""
    g, Om, c0, c1, c2 = [float(x) for x in params]
    want = (c0, c1, c2, Om, g, float(trap[0]), float(trap[1]), float(trap[2]))
    Ls = tuple(float(x) for x in (L if hasattr(L, "__len__") else [L] * len(shape)))
    if (tuple(s.shape) != tuple(shape) or s.params != want or s.L != Ls or s.torch_dtype != psi0.dtype
            or s.tau != float(tau) or s.scheme != int(order) or s.frame != "rotating"):
        raise ValueError("the prebuilt solver does not match the evolution's grid, parameters, dtype, tau or scheme")


class _Evolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi0, params, shape, L, trap, tau, nsteps, order, K, t0, plan, solver):
        dtype = "complex64" if psi0.dtype == torch.complex64 else "complex128"
        pars = params.detach().cpu().tolist()
        if solver is not None:
            check_solver(solver, psi0, pars, shape, L, trap, tau, order)
            s = solver
        else:
            s = _solver(shape, L, pars, trap, dtype, tau, order, plan, psi0.detach())
        psi = psi0.detach().clone().contiguous()
        keep = any(ctx.needs_input_grad[:2])
        ckpts, store = [], None
        for n0 in range(0, nsteps, K):
            s.time = t0 + n0 * tau
            ns = min(K, nsteps - n0)
            ckpts.append(psi.clone())
            if keep and n0 + K >= nsteps:
                # last segment: run it with stores, the backward's first input
                store = torch.empty(s.store_size(ns), dtype=torch.uint8, device=psi.device)
                s.step_store(psi, ns, store)
            else:
                s.step(psi, ns)
        ctx.s, ctx.ckpts, ctx.store = s, ckpts, store
        ctx.meta = (tau, nsteps, K, t0)
        ctx.pmeta = (params.dtype, params.device)
        return psi

    @staticmethod
    def backward(ctx, grad_out):
        s, ckpts = ctx.s, ctx.ckpts
        tau, nsteps, K, t0 = ctx.meta
        lam = grad_out.detach().to(s.torch_dtype).clone().contiguous()
        s.adjoint_gradients(reset=True)
        # the forward's store holds the last segment; it is overwritten below, so a
        # second backward recomputes every segment
        store, ctx.store = ctx.store, None
        fresh = store is not None
        for seg in range(len(ckpts) - 1, -1, -1):
            n0 = seg * K
            ns = min(K, nsteps - n0)
            if not (fresh and seg == len(ckpts) - 1):  # recompute the segment with stores
                nbytes = s.store_size(ns)
                if store is None or store.numel() < nbytes:
                    store = torch.empty(nbytes, dtype=torch.uint8, device=lam.device)
                psi = ckpts[seg].clone()
                s.time = t0 + n0 * tau
                s.step_store(psi, ns, store)
            s.time = t0 + n0 * tau
            s.adjoint_segment(lam, ns, store)
        pdtype, pdev = ctx.pmeta
        dpar = torch.tensor(s.adjoint_gradients(reset=True), dtype=pdtype, device=pdev)
        return lam, dpar, None, None, None, None, None, None, None, None, None, None


def evolve(psi0, params, shape, L, trap, tau, nsteps, order=4, K=50, t0=0.0, plan=None, solver=None):
    """plan: None (default register plans), a list of plan widths per axis (x, y (, z)),
    or "auto" (autotuned, through the JSON plan cache).  solver: a prebuilt Solver
    (propagator built for tau and order; its plans are used) so that repeated calls
    set nothing up; it must match the grid, parameters, trap and element type.  The
    parameter gradient comes back with the dtype and device of params."""
    if not isinstance(params, torch.Tensor):
        params = torch.tensor(params, dtype=torch.float64)
    plan = plan if plan is None or plan == "auto" else tuple(int(e) for e in plan)
    return _Evolve.apply(psi0, params, tuple(shape), L, tuple(trap), float(tau), int(nsteps), int(order), int(K),
                         float(t0), plan, solver)


class _ToLab(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi, Omega, shape, L, t):
        dtype = "complex64" if phi.dtype == torch.complex64 else "complex128"
        s = Solver(shape, L, (0.0, 0.0, 0.0, float(Omega), 0.0, 1.0, 1.0, 1.0), dtype=dtype)
        lab = phi.detach().clone().contiguous()
        s.rotation_map(lab, t, -1)
        ctx.s, ctx.t, ctx.hd = s, t, math.prod(2.0 * L / n for n in shape)
        ctx.Om_dtype, ctx.Om_device = Omega.dtype, Omega.device
        ctx.save_for_backward(lab)
        return lab

    @staticmethod
    def backward(ctx, grad):
        s, t = ctx.s, ctx.t
        (lab,) = ctx.saved_tensors
        g = grad.detach().to(lab.dtype).contiguous()
        gin = g.clone()
        s.rotation_map(gin, t, +1)  # the map is unitary (shears and phases): adjoint = inverse
        dOm = None
        if ctx.needs_input_grad[1]:
            # the map rotates by the angle Omega t: d lab / d Omega = -i t J_z lab with
            # J_z = L_z + F_z, so dJ/dOmega = Re<g, -i t J_z lab> / h^d = -t Im<g, J_z lab>_h / h^d
            # (<,>_h carries h^d; the gradient convention does not)
            ip = s.jz_inner(g, lab)
            dOm = torch.tensor(-t * ip.imag / ctx.hd, dtype=ctx.Om_dtype, device=ctx.Om_device)
        return gin, dOm, None, None, None


def to_lab(phi, Omega, shape, L, t):
    """The lab-frame state Psi(t) = M_t^{-1} Phi(t) of a rotating-frame state
    (sgp_rotation_map, eqs. RSDA1/RSDA2), differentiable: with respect to phi by the
    map's adjoint (its inverse: every shear and the component phase are unitary), and
    with respect to Omega (a 0-d FP64 tensor) through the rotation angle Omega t, by
    the generator J_z = L_z + F_z (exact to the spectral accuracy of the rotation).
    Use the same Omega tensor as in evolve's params to differentiate a lab-frame loss
    through both."""
    if not isinstance(Omega, torch.Tensor):
        Omega = torch.tensor(float(Omega), dtype=torch.float64)
    return _ToLab.apply(phi, Omega, tuple(shape), float(L), float(t))


class _EnsembleEvolve(torch.autograd.Function):
    """Differentiable batched ensemble evolution: inputs (ens, meta, params, *psis)."""

    @staticmethod
    def forward(ctx, ens, meta, params, *psis):
        tau, nsteps, K, t0 = meta
        states = [p.detach().clone().contiguous() for p in psis]
        keep = any(ctx.needs_input_grad[2:])
        ckpts, store = [], None
        for n0 in range(0, nsteps, K):
            ens.time = t0 + n0 * tau
            ns = min(K, nsteps - n0)
            ckpts.append([p.clone() for p in states])
            if keep and n0 + K >= nsteps:
                # last segment: run it with stores, the backward's first input
                store = torch.empty(ens.store_size(ns), dtype=torch.uint8, device=states[0].device)
                ens.step_store(states, ns, store)
            else:
                ens.step(states, ns)
        ctx.ens, ctx.ckpts, ctx.store, ctx.meta = ens, ckpts, store, meta
        ctx.pmeta = (params.dtype, params.device)
        return tuple(states)

    @staticmethod
    def backward(ctx, *grads):
        ens, ckpts = ctx.ens, ctx.ckpts
        tau, nsteps, K, t0 = ctx.meta
        lams = [g.detach().to(ens.torch_dtype).clone().contiguous() for g in grads]
        ens.adjoint_gradients(reset=True)
        # the forward's store holds the last segment; it is overwritten below, so a
        # second backward recomputes every segment
        store, ctx.store = ctx.store, None
        fresh = store is not None
        for seg in range(len(ckpts) - 1, -1, -1):
            n0 = seg * K
            ns = min(K, nsteps - n0)
            if not (fresh and seg == len(ckpts) - 1):  # recompute the segment with stores
                nbytes = ens.store_size(ns)
                if store is None or store.numel() < nbytes:
                    store = torch.empty(nbytes, dtype=torch.uint8, device=lams[0].device)
                states = [p.clone() for p in ckpts[seg]]
                ens.time = t0 + n0 * tau
                ens.step_store(states, ns, store)
            ens.time = t0 + n0 * tau
            ens.adjoint_segment(lams, ns, store)
        dpar = torch.tensor(ens.adjoint_gradients(reset=True), dtype=ctx.pmeta[0], device=ctx.pmeta[1])
        return (None, None, dpar) + tuple(lams)


def ensemble_evolve(ens, psis, params, tau, nsteps, K=50, t0=0.0):
    """Differentiable evolution of a batched Ensemble (its propagator built for tau):
    psis a list of device states, params an (n_inst, 5) FP64 tensor of
    (gamma, Omega, c0, c1, c2) equal to the ensemble's instance parameters (it carries
    their gradients).  Returns the list of final states; gradients flow to every
    psis[i] and to params through one batched adjoint per checkpoint segment."""
    if not isinstance(params, torch.Tensor):
        params = torch.tensor(params, dtype=torch.float64)
    return list(_EnsembleEvolve.apply(ens, (float(tau), int(nsteps), int(K), float(t0)), params, *psis))

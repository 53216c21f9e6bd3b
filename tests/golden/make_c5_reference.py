"""Write tests/golden/c5_reference.npz: the FP64 oracle's loss and gradients for the
differentiation workload: 2D 256^2 on [-12, 12]^2, TS4, tau = 1e-3, 500 steps,
Omega = 0.8, gamma = 1, c = (300, -3, 6), isotropic trap; Psi0 and the target are
random-phase Gaussians (seeds 5 and 6); J = (<Lz>(T) - 1.5)^2 + (1 - |<Psi_tgt,
Phi(T)>_h|^2).  Stores J, dJ/d(gamma, Omega, c0, c1, c2) and the whole state
gradient 2 dJ/d conj(Psi0) (complex128, shape (5, 256, 256)).  Calls only the oracle
(plus the loss written out in tests/adjoint_loss.py); ~30-40 minutes on 8 cores."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402
from paper_2603_25282_amd import inputs as I  # noqa: E402
from tests.adjoint_loss import loss_and_grad  # noqa: E402


def main():
    cfg = I.C5
    psi0 = I.initial_state(cfg)
    target = I.initial_state(I.with_(cfg, seed=cfg.extra["target_seed"]))
    t = time.time()
    u = oracle.evolve(psi0, cfg.L, cfg.params, cfg.order, cfg.tau, cfg.steps)
    J, gT = loss_and_grad(u, target, cfg.L)
    g0, dpar = oracle.adjoint(psi0, gT, cfg.L, cfg.params, cfg.order, cfg.tau, cfg.steps, K=cfg.extra["K"])
    el = time.time() - t
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_reference.npz")
    np.savez_compressed(out, J=J, dpar=dpar, g0=g0, steps=cfg.steps, oracle_seconds=el,
                        threads=oracle.num_threads())
    print(f"wrote {out}: J = {J}, dJ/d(gamma, Omega, c0, c1, c2) = {dpar}, {el:.0f} s")


if __name__ == "__main__":
    main()

"""Write tests/golden/c3_reference.npz: the FP64 oracle's state after the full
3D 128^3 TS4 workload (200 steps of tau = 1e-3 on [-8, 8]^3, Omega = 0.7 about z,
gamma = 0.8, trap (1, 1, 4), c = (200, -2, 4), Gaussian with seeded phase noise,
seed 3), stored at 4096 seeded sample points where the initial density exceeds
1e-3 of its maximum, plus the observables.  Calls only the oracle (~15 minutes)."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402
from paper_2603_25282_amd import inputs as I  # noqa: E402
from tests.golden.make_c2_reference import sample_indices  # noqa: E402


def main():
    cfg = I.C3
    psi0 = I.initial_state(cfg)
    idx = sample_indices(psi0)
    t = time.time()
    u = oracle.evolve(psi0, cfg.L, cfg.params, cfg.order, cfg.tau, cfg.steps)
    el = time.time() - t
    obs0 = oracle.observables(psi0, cfg.L, cfg.params)
    obs = oracle.observables(u, cfg.L, cfg.params, theta=cfg.params[3] * cfg.tau * cfg.steps)
    flat = u.reshape(5, -1)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_reference.npz")
    np.savez_compressed(out, steps=cfg.steps, idx=idx, samples=flat[:, idx], obs0=obs0, obs=obs,
                        oracle_seconds=el, threads=oracle.num_threads())
    print(f"wrote {out}: {cfg.steps} steps in {el:.1f} s on {oracle.num_threads()} threads; obs {obs}")


if __name__ == "__main__":
    main()

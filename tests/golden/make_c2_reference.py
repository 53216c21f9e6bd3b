"""Write tests/golden/c2_reference.npz: the FP64 oracle's state after the full
2D 512^2 TS4 workload (1000 steps of tau = 5e-4 on [-16, 16]^2, Omega = 0.9,
gamma = 1, trap 1 x 1.1, c = (500, -5, 10), Gaussian + 1e-2 low-passed noise,
seed 2), stored as values at 4096 seeded sample points where the initial
density exceeds 1e-3 of its maximum, plus per-component l2 norms and the
observables.  Calls only the oracle.  Takes ~10-20 minutes on 8 cores."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402
from paper_2603_25282_amd import inputs as I  # noqa: E402


def sample_indices(psi0, n=4096, seed=77):
    rho = np.sum(np.abs(psi0) ** 2, axis=0).ravel()
    cand = np.nonzero(rho > 1e-3 * rho.max())[0]
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(cand, size=min(n, cand.size), replace=False))


def main(steps=None, out=None):
    cfg = I.C2
    steps = cfg.steps if steps is None else steps
    psi0 = I.initial_state(cfg)
    idx = sample_indices(psi0)
    t = time.time()
    u = oracle.evolve(psi0, cfg.L, cfg.params, cfg.order, cfg.tau, steps)
    el = time.time() - t
    obs0 = oracle.observables(psi0, cfg.L, cfg.params)
    obs = oracle.observables(u, cfg.L, cfg.params, theta=cfg.params[3] * cfg.tau * steps)
    flat = u.reshape(5, -1)
    out = out or os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_reference.npz")
    np.savez_compressed(out, steps=steps, idx=idx, samples=flat[:, idx], norms=np.linalg.norm(flat, axis=1),
                        obs0=obs0, obs=obs, oracle_seconds=el, threads=oracle.num_threads())
    print(f"wrote {out}: {steps} steps in {el:.1f} s on {oracle.num_threads()} threads; obs {obs}")


if __name__ == "__main__":
    main()

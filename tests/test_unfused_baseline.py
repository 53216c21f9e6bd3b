"""The plain unfused FP64 comparison step of bench.py (PyTorch operations, here on
the CPU) against the FP64 oracle: the comparison point must compute the same
evolution for its timing to mean anything."""
import numpy as np
import pytest

import oracle
from paper_2603_25282_amd import inputs as I
from tests.gpu_util import rel_l2


@pytest.mark.parametrize("order", [2, 4])
def test_unfused_baseline_matches_oracle(order):
    import torch
    import bench
    cfg = I.with_(I.C2, shape=(32, 48), L=8.0, name="unfused-small")
    psi0 = I.initial_state(cfg)
    ref = oracle.evolve(psi0, cfg.L, cfg.params, order, 2e-3, 5, t0=0.1)
    b = bench.UnfusedFP64(cfg.shape, cfg.L, cfg.params, torch.device("cpu"))
    got = b.evolve(torch.from_numpy(psi0), order, 2e-3, 5, t0=0.1).numpy()
    err = rel_l2(got, ref)
    print("rel l2", err)
    assert err <= 1e-11


@pytest.mark.gpu
def test_unfused_baseline_on_gpu_matches_oracle():
    import torch
    import bench
    cfg = I.with_(I.C2, shape=(64, 64), L=8.0, name="unfused-gpu")
    psi0 = I.initial_state(cfg)
    ref = oracle.evolve(psi0, cfg.L, cfg.params, 4, 1e-3, 6)
    b = bench.UnfusedFP64(cfg.shape, cfg.L, cfg.params, torch.device("cuda:0"))
    got = b.evolve(torch.from_numpy(psi0).cuda(), 4, 1e-3, 6).cpu().numpy()
    err = rel_l2(got, ref)
    print("rel l2", err)
    assert err <= 1e-11

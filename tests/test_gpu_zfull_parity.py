"""Headline parity on the whole state: the HIP path (through the C ABI) against the
FP64 oracle, element by element, at the full workloads' horizons:

* 2D 512^2 TS4, 1000 steps (the bench workload): relative l2 of the full state
  <= 1e-11 in complex128 and <= 5e-5 in complex64;
* 3D 128^3 TS4, 200 steps: the same bounds.

The oracle's final states are computed on the host during the session
(tests/oracle_refs.py; the file is named so that these tests run after the others,
which overlap the oracle's work).  Besides the full-state figure every test prints
the per-component errors and checks the mass against the oracle's."""
import numpy as np
import pytest

from paper_2603_25282_amd import inputs as I
from tests import oracle_refs
from tests.gpu_util import rel_l2, run_gpu, to_gpu

pytestmark = pytest.mark.gpu

TOL = {"complex128": 1e-11, "complex64": 5e-5}


def full_state_case(cfg, name, dtype):
    psi0 = I.initial_state(cfg)
    steps = oracle_refs.RUNS[name][1]
    print(f"case {cfg.name} shape={cfg.shape} dtype={dtype} TS{cfg.order} tau={cfg.tau} steps={steps}", flush=True)
    got, s = run_gpu(cfg.shape, cfg.L, cfg.params, psi0, cfg.order, cfg.tau, steps, dtype=dtype)
    obs = s.observables(to_gpu(s, got))
    ref = oracle_refs.load(name)
    u = ref["state"]
    err = rel_l2(got, u)
    per = [rel_l2(got[i], u[i]) for i in range(5)]
    print(f"{cfg.name} {dtype} after {steps} steps: full-state rel l2 {err:.3e}; per component "
          + " ".join(f"{e:.2e}" for e in per) + f"; gpu obs {obs}; oracle obs {ref['obs']}", flush=True)
    return err, obs, ref["obs"]


@pytest.mark.oracle_ref("c2_full")
@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_config2_full_state_1000_steps(dtype):
    err, obs, oobs = full_state_case(I.C2, "c2_full", dtype)
    assert err <= TOL[dtype]
    # discrete mass is conserved up to rounding on both sides (6000 substeps)
    assert abs(obs[0] - oobs[0]) <= (1e-11 if dtype == "complex128" else 1e-5)


@pytest.mark.oracle_ref("c3_full")
@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_config3_full_state_200_steps(dtype):
    err, obs, oobs = full_state_case(I.C3, "c3_full", dtype)
    assert err <= TOL[dtype]
    assert abs(obs[0] - oobs[0]) <= (1e-11 if dtype == "complex128" else 1e-5)

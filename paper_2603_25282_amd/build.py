"""Build the HIP library libsgp.so for gfx950 (in-tree, next to this file)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsgp.so")
SOURCES = ["sgp_kernels.hip", "sgp_api.hip"]
# the pass kernels of each (scalar type, register plan width) in a unit of their own
PLAN_UNITS = [(t, e) for t in ("float", "double") for e in (4, 8, 12, 16, 24)]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions (v_pk_*_f32) anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose=False, jobs=None):
    jobs = jobs or max(1, min(os.cpu_count() or 1, 8))
    units = [(os.path.join(CSRC, src), os.path.join(CSRC, os.path.splitext(src)[0] + ".o"), [])
             for src in SOURCES]
    for t, e in PLAN_UNITS:
        units.append((os.path.join(CSRC, "sgp_plan_inst.hip"), os.path.join(CSRC, f"sgp_plan_{t}_e{e}.o"),
                      [f"-DSGP_INST_T={t}", f"-DSGP_INST_E={e}"]))
    objs = [u[1] for u in units]
    pending = list(units)
    running = []
    failed = None
    while pending or running:
        while pending and len(running) < jobs and failed is None:
            src, obj, defs = pending.pop(0)
            cmd = [HIPCC] + FLAGS + defs + ["-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            running.append((subprocess.Popen(cmd), cmd))
        if failed is not None and not running:
            break
        p, cmd = running.pop(0)
        if p.wait() != 0 and failed is None:
            failed = cmd
    if failed is not None:
        raise RuntimeError("hipcc failed: " + " ".join(failed))
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

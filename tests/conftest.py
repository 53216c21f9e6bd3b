import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "oracle_ref(name): compares against a full-size oracle run of "
                                       "tests/oracle_refs.py, computed in the background while the session runs")


def pytest_collection_modifyitems(config, items):
    # gpu tests need a device; on a machine without one they are skipped, not failed.
    try:
        import torch
        have_gpu = torch.cuda.is_available()
    except Exception:
        have_gpu = False
    if have_gpu:
        # start the full-size oracle runs the selected tests need, in one background
        # process, so that they overlap the rest of the session
        names = []
        for it in items:
            for m in it.iter_markers(name="oracle_ref"):
                for n in m.args:
                    if n not in names:
                        names.append(n)
        if names:
            from tests import oracle_refs
            oracle_refs.start_background(names)
        return
    skip = pytest.mark.skip(reason="no GPU on this machine")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)


def pytest_sessionfinish(session, exitstatus):
    mod = sys.modules.get("tests.oracle_refs")
    if mod is not None:
        mod.stop_background()

import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running check")
    config.addinivalue_line("markers", "oracle_job(name): the test uses a background oracle run (tests/oracle_bg.py)")


@pytest.hookimpl(trylast=True)
def pytest_collection_modifyitems(config, items):
    # tests marked gpu are skipped (not failed) when no GPU is visible
    try:
        import torch
        have_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        have_gpu = False
    if have_gpu:
        # start the long oracle runs the selected tests need, so that they
        # overlap the GPU tests that run before them
        names = []
        for it in items:
            for m in it.iter_markers("oracle_job"):
                names.extend(m.args)
        if names:
            from tests import oracle_bg
            oracle_bg.start(sorted(set(names)))
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)

import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI on cuda:0)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(params=[1, 0], ids=["refine-operator", "refine-data"])
def mixed_refine(request):
    """Runs a mixed-form test under both refinement steps (the knob is reset to
    its default afterwards)."""
    import paper_1110_0836_amd as P
    saved = P.phb_tune_get("mixed_refine")
    P.phb_tune_set("mixed_refine", request.param)
    yield request.param
    P.phb_tune_set("mixed_refine", saved)

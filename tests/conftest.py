import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def figure():
    with open(os.path.join(GOLDEN, "figure_example.json")) as f:
        return json.load(f)


@pytest.fixture
def restore_settings():
    """Tests may change the library's process-wide settings; put back the
    ones found before the test (the defaults unless a test failed to)."""
    import paper_1303_4312_amd as cm
    kts = ("uint32", "uint64", "float32")
    search, partition = cm.get_search(), cm.get_partition()
    order, stride, lanes = cm.get_block_order(), cm.get_coarse_stride(), cm.get_fine_lanes()
    cfgs = {(kt, v): cm.get_config(kt, v) for kt in kts for v in (False, True)}
    yield
    cm.set_search(search)
    cm.set_partition(partition)
    cm.set_coarse_stride(stride)
    cm.set_block_order(order)
    cm.set_fine_lanes(lanes)
    for (kt, v), c in cfgs.items():
        cm.set_config(kt, v, c)

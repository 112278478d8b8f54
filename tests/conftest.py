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
    ones found before the test, a configuration that was not set included."""
    import paper_1303_4312_amd as cm
    lib = cm.load()
    search, partition = cm.get_search(), cm.get_partition()
    order, stride, lanes = cm.get_block_order(), cm.get_coarse_stride(), cm.get_fine_lanes()
    grid = cm.get_grid()
    # -1: no configuration set (the per-operation defaults apply)
    cfgs = {(kt, v): lib.cm_get_config(kt, v) for kt in range(6) for v in (0, 1)}
    yield
    cm.set_search(search)
    cm.set_partition(partition)
    cm.set_coarse_stride(stride)
    cm.set_block_order(order)
    cm.set_fine_lanes(lanes)
    cm.set_grid(grid)
    for (kt, v), c in cfgs.items():
        assert lib.cm_set_config(kt, v, c) == 0

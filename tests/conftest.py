import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library on device)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")
    config.addinivalue_line("markers", "gpu_long: GPU run of several minutes, outside the gpu set "
                                       "(run by name: -m gpu_long)")


@pytest.fixture(scope="session")
def orc():
    import oracle

    oracle.lib()
    return oracle


def pytest_collection_modifyitems(config, items):
    # the long GPU runs only when asked for by name (-m gpu_long)
    if "gpu_long" in (config.option.markexpr or ""):
        return
    skip = pytest.mark.skip(reason="long GPU run: select it with -m gpu_long")
    for item in items:
        if "gpu_long" in item.keywords:
            item.add_marker(skip)

import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture(scope="session")
def tiny_tree():
    import scenegen
    from scenegen import configs
    return scenegen.build_tree(configs.tiny_spec())


@pytest.fixture(scope="session")
def tiny_oracle(tiny_tree):
    import oracle
    return oracle.OracleScene(tiny_tree)

import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs the HIP device (MI355X) and the built libhsc.so")


@pytest.fixture(scope="session")
def ctx():
    import paper_1702_05167_amd as pkg
    c = pkg.Context(0)
    yield c
    c.close()

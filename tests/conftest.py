import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")


def _stale(lib: str, src: str) -> bool:
    return not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src)


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle
    here = os.path.dirname(oracle.__file__)
    if (_stale(oracle.LIB_ORACLE, os.path.join(here, "pthr_oracle.c"))
            or _stale(oracle.LIB_EXACT, os.path.join(here, "exact_enum.c"))):
        oracle.build()
    yield

import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU pin (tens of seconds)")


@pytest.fixture(scope="session")
def oracle_mod():
    """The oracle module; PIBM_ORACLE_LIB names another build of the same
    source to run the pins against (the sanitizer test uses it)."""
    from oracle import oracle as O
    alt = os.environ.get("PIBM_ORACLE_LIB")
    if alt:
        O._lib = O.load(alt)
    else:
        O.build()
    return O

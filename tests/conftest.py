import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    mutant = os.environ.get("SAL_ORACLE_MUTANT_LIB")
    if mutant:
        # a deliberately broken copy of the oracle, compiled by test_oracle_mutants.py to
        # show that the pins notice the mistake
        import oracle.oracle as impl
        impl._LIB = mutant
        impl._lib = None
        impl.build = lambda force=False: mutant
    else:
        oracle.build()
    return oracle

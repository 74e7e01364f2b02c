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
def ref():
    """The oracle package; MGREF_ORACLE_DIR points the pins at another copy of it
    (used by the mutation test, which plants mistakes in a copy on the CPU)."""
    alt = os.environ.get("MGREF_ORACLE_DIR")
    if alt:
        import importlib.util
        spec = importlib.util.spec_from_file_location(
            "oracle_variant", os.path.join(alt, "__init__.py"), submodule_search_locations=[alt])
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build()
        return mod
    import oracle
    oracle.build()
    return oracle

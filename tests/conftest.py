import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


def _ensure_built():
    """Build the host helpers and the oracle only when nothing is built yet."""
    from paper_2307_11648_amd import build as b
    if not os.path.exists(b.GEO_LIB):
        b.build_geometry()
    import oracle
    if not os.path.exists(oracle._LIB_PATH):
        oracle.build()


_ensure_built()

import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU-only oracle checks")


@pytest.fixture(scope="session")
def lib():
    """The HIP library through its Python binding; GPU tests only."""
    import paper_1102_3069_amd as llg
    llg.load()
    return llg


# every padded length with compiled variants (rows: Px; columns: L = Py / 2)
ROW_LENGTHS = (64, 128, 192, 256, 384, 512, 768, 1024, 2048, 4096)
COL_LENGTHS = (32, 64, 96, 128, 192, 256, 384, 512, 1024, 2048)


@pytest.fixture
def default_variants(lib):
    """Puts the process-wide default variant of every compiled length back
    to 0 after the test (tuning calls write the defaults that solvers and
    batches set up later copy)."""
    yield
    s = lib.Solver(0)
    for px in ROW_LENGTHS:
        s.set_geometry((px // 2, 32, 1))
        s.set_variants(0, 0)
    for L in COL_LENGTHS:
        s.set_geometry((32, L, 1))
        s.set_variants(0, 0)
    s.close()

import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.dirname(os.path.abspath(__file__))
for p in (ROOT, HERE):
    if p not in sys.path:
        sys.path.insert(0, p)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    return oracle.load()


@pytest.fixture(scope="session")
def isa_counts(tmp_path_factory):
    """VALU-per-cell counts of this build's gfx950 assembly (isa_count.run),
    compiled once for every test that reads them."""
    from paper_2412_08308_amd import isa_count
    return isa_count.run(out=str(tmp_path_factory.mktemp("isa") / "counts.json"))

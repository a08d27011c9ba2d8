import os
import sys

# large numpy temporaries: skip the transparent-huge-page advice (slow first touch on some hosts)
os.environ.setdefault("NUMPY_MADVISE_HUGEPAGE", "0")

import pytest  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    from oracle import oracle as ora
    src = os.path.join(ROOT, "oracle", "atns_oracle.c")
    lib = ora.library_path()
    if not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
        ora.build()
    yield

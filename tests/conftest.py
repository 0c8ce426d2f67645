import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")
    config.addinivalue_line("markers", "slow: CPU test taking more than a few seconds")


@pytest.fixture(params=["plain", "nontemporal"])
def store_form(request, monkeypatch):
    """Which form of the in-solve operator a mesh set up in the test uses:
    shared-copy results written with plain stores (the default up to a
    128 MB local array) or with nontemporal ones (the default above;
    SEM_AX_NT_BYTES=0, read at mesh set-up, forces them at any size)."""
    if request.param == "nontemporal":
        monkeypatch.setenv("SEM_AX_NT_BYTES", "0")
    else:
        monkeypatch.delenv("SEM_AX_NT_BYTES", raising=False)
    return request.param

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built liblbm.so")
    config.addinivalue_line("markers", "slow: CPU test taking more than a few seconds")


def _oracle_lib():
    so = os.path.join(ROOT, "oracle", "liblbmref.so")
    src = [os.path.join(ROOT, "oracle", n) for n in ("lbmref.c", "lbmref.h", "Makefile")]
    stale = (not os.path.exists(so)) or any(os.path.getmtime(s) > os.path.getmtime(so) for s in src)
    if stale:
        subprocess.run(["make", "-s", "-C", os.path.join(ROOT, "oracle")], check=True)
    return so


@pytest.fixture(scope="session", autouse=True)
def oracle_built():
    return _oracle_lib()

"""Shared test configuration.

Marker ``gpu``: the test needs an MI355X and the built HIP library. Every other
test runs on the CPU (oracle pins, host logic, ABI symbol checks).
"""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU and the built liblbpf.so")


@pytest.fixture(scope="session")
def ref():
    import oracle
    oracle.build(force=False)
    return oracle

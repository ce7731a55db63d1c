import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


@pytest.fixture(scope="session")
def head8():
    from paper_1811_07717_amd import headmodel as hm
    return hm.workload("sphere8mm_L32")


@pytest.fixture(scope="session")
def sys8(head8):
    from oracle import fem
    H = head8
    return fem.assemble(H.nodes, H.tets, H.sigma, H.tris, H.tri_electrode, H.Z)


@pytest.fixture(scope="session")
def direct8(sys8):
    from oracle import solve
    return solve.transfer_direct(sys8["A"], sys8["B"])

import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    return oracle.Oracle()


@pytest.fixture(scope="session")
def orc_bag():
    import oracle
    from paper_1206_0919_amd import inputs
    B, e_H = inputs.bag_parameters()
    return oracle.Oracle(oracle.EOS_BAG, B, e_H)


def to_cons(o, prim):
    shape = prim.e.shape
    return [np.ascontiguousarray(a.reshape(shape)) for a in o.prim_to_cons(*prim.as_tuple())]

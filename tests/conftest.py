import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


# The width from which the library's unconstrained step (and the l2 ball's
# cold start and the overlapped l1-ball step) applies an explicit inverse of H
# instead of two triangular solves: kQpInverseMinD in csrc/rowdot.hpp. The tests
# that expect bitwise equality of the two forms read it from here.
INVERSE_MIN_D = 89


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) and the built HIP library")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library through its Python binding, on cuda:0."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_14166_amd as ihs
    ihs.load()
    return ihs

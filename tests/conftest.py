import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device)")


@pytest.fixture(scope="session")
def dev():
    """The HIP device; GPU tests fail loudly if the native library is missing."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1208_3444_amd import colatus
    colatus.lib()  # raises if libcolatus.so was not built
    return torch.device("cuda", 0)


def to_dev(a, dev):
    import numpy as np
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)


def rel_err_per_particle(got, ref):
    """|got_k - ref_k|_2 / |ref_k|_2 for (3, N) arrays."""
    import numpy as np
    return np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)

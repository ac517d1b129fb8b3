import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def ba100k():
    """The n = 1000, p = 1e5 power-law workload (200 blocks of 500, lambda = 0.03), its
    FP64 copy, and L = sigma_max(X)^2 / n from the n x n Gram matrix (host only)."""
    import numpy as np

    import datagen
    w = datagen.workload("ba100k")
    x64 = w.X.astype(np.float64)
    gram = x64 @ x64.T / w.n
    return {"w": w, "x64": x64, "L": float(np.linalg.eigvalsh(gram)[-1])}


@pytest.fixture(scope="session")
def gpu_lib():
    """The built HIP library through its Python binding (GPU tests only)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_11554_amd import accord
    return accord

import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device); run with -m gpu")
    config.addinivalue_line("markers", "slow: full-size workload, minutes of CPU time")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def lco_lib():
    import paper_1802_02619_amd as lco
    lco.load_library()
    return lco


@pytest.fixture(scope="session")
def gpu_ctx(lco_lib):
    """Library context on cuda:0 (GPU tests only; fails loudly without the HIP library)."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible HIP device")
    ctx = lco_lib.lco_ctx_create(0)
    yield ctx
    ctx.synchronize()


def gpu_create(lco, ctx, dims, coords, vals, flags=None):
    """Upload host coordinates/values and build a library tensor from coordinates."""
    import numpy as np
    import torch
    coords = np.ascontiguousarray(np.asarray(coords, dtype=np.uint64).reshape(len(vals), len(dims)))
    idx = torch.from_numpy(coords.view(np.int64).reshape(-1).copy()).to("cuda")
    v = torch.from_numpy(np.ascontiguousarray(vals, dtype=np.float64)).to("cuda")
    f = lco.LCO_COORDS if flags is None else flags
    return lco.lco_create(ctx, dims, idx, v, f)

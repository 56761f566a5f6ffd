import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


@pytest.fixture(scope="session")
def keys():
    """Secret keys and the oracle's bootstrapping / key-switching keys (seeds 0, 1, 2)."""
    import oracle
    import workloads as W
    s0, s1 = W.secret_keys()
    bkd, kskd = W.bk_draws(), W.ksk_draws()
    bk, ksk = oracle.keyset(s0, s1, bkd, kskd)
    return dict(s0=s0, s1=s1, bk=bk, ksk=ksk, bkd=bkd, kskd=kskd)


@pytest.fixture(scope="session")
def gpu(keys):
    """A libvsp context on cuda:0 built from the library client's keys (which equal the
    oracle's, see test_client.py). Skips only where no GPU exists."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU on this machine")
    from paper_2010_09410_amd import client
    from paper_2010_09410_amd.device import Context
    bk, ksk = client.keyset(keys["s0"], keys["s1"], keys["bkd"], keys["kskd"])
    ctx = Context(bk, ksk, device=0)
    yield ctx
    ctx.close()


def signed(x):
    return np.asarray(x, dtype=np.uint32).view(np.int32).astype(np.int64)

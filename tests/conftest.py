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


def signed(x):
    return np.asarray(x, dtype=np.uint32).view(np.int32).astype(np.int64)

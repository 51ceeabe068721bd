import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long statistical run")
    config.addinivalue_line("markers", "planted_tie: plants an exchange near tie (exempt from the audit)")


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


@pytest.fixture(autouse=True)
def _exchange_near_tie_audit(request):
    """Tempering results are compared bit for bit with the oracle, whose
    exchange test u53 < exp(x) uses the C library's exp while the device uses
    its own float64 exp (the two may differ by an ulp).  The comparison is
    only sound if no attempted exchange had u53 within 2^-40 of exp(x): after
    every test the oracle's audit of the exchanges it made in that test must
    show no such near tie (tests that plant one are marked planted_tie)."""
    from oracle import oracle as O

    O.pt_audit(reset=True)
    yield
    audit = O.pt_audit(reset=True)
    if "planted_tie" not in request.keywords:
        assert audit["near_ties"] == 0, f"exchange decision within 2^-40 of exp(x): {audit}"

import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: longer CPU oracle runs")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def parity_record():
    """Append one JSON record of a measured error against the oracle to the
    file named by FLD_PARITY_RECORD (if set) and print it."""
    import json

    path = os.environ.get("FLD_PARITY_RECORD")

    def put(**fields):
        line = json.dumps(fields, sort_keys=True)
        print("parity-record " + line, flush=True)
        if path:
            with open(path, "a") as f:
                f.write(line + "\n")
    return put

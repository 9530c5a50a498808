"""The oracle's output on the 256-triangle workload matches its committed
digest (a regression guard on the oracle's arithmetic)."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))


def test_oracle_digest_unchanged(oracle_lib):
    import make_golden
    want = {}
    for line in open(os.path.join(HERE, "golden", "soup256_oracle.txt")):
        k, v = line.split()
        want[k] = v
    got = {k: str(v) for k, v in make_golden.digest().items()}
    assert got == want

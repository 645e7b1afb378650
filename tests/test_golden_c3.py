"""The stored full-size oracle step (tests/golden/c3_step1_oracle.npz) was
written by tests/golden/make_c3_step.py from the current oracle source: its
recorded SHA-256 of oracle/oracle.c must match the file (re-run the script
after any change to the oracle), and its contents must be self-consistent."""
import hashlib
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_c3_golden_matches_oracle_source():
    g = np.load(os.path.join(HERE, "golden", "c3_step1_oracle.npz"), allow_pickle=False)
    h = hashlib.sha256(open(os.path.join(ROOT, "oracle", "oracle.c"), "rb").read()).hexdigest()
    assert str(g["oracle_sha256"]) == h, "oracle.c changed since the golden step was written: re-run make_c3_step.py"
    n = g["nodes"]
    assert n.shape == (4096,) and np.all(np.diff(n) > 0) and n.max() < 256 * 256 * 4
    for name in ("phi", "T", "E"):
        assert g[name].shape == n.shape and np.all(np.isfinite(g[name])) and np.all(g[name] > 0)
        assert np.abs(g[name]).max() <= float(g[name + "_max"])
    assert int(g["outer"]) >= 1 and float(g["energy"]) > 0

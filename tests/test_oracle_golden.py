"""The oracle against its stored regression anchor (tests/golden/oracle_12x12x3.json, written
by tests/golden/make_golden.py from the oracle itself).  This guards the oracle against
unintended changes between commits; what pins it to the paper are the tests in
test_oracle_pins.py and test_oracle_mutations.py.  Any deliberate change of the oracle's
arithmetic regenerates the file in the same commit, which names the passage behind it."""
import json
import os

import numpy as np

from oracle import nlpr_oracle as o

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_12x12x3.json")


def load_golden():
    with open(GOLDEN) as f:
        g = json.load(f)
    arr = {k: np.asarray(g[k], dtype=np.float64) for k in ("blur", "R", "Yl", "Yh", "Z")}
    return g, arr


def test_oracle_reproduces_its_stored_anchor():
    g, a = load_golden()
    pr = o.Problem(p=g["p"], q=g["q"], L=g["L"], d=g["d"], b=a["blur"], R=a["R"], K=g["K"],
                   S=g["Sw"], lam=g["lam"], rho=g["rho"], h=g["h"], lam1=g["lam1"])
    Z = o.solve(a["Yl"], a["Yh"], pr, g["iters"]).X
    assert Z.shape == a["Z"].shape
    assert np.linalg.norm(Z - a["Z"]) <= 1e-12 * np.linalg.norm(a["Z"])

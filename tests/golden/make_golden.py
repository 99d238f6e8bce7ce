"""Writes tests/golden/oracle_12x12x3.json: a tiny seeded scene (inputs as the float32 values
the library takes) and the FP64 oracle's Z after 6 iterations of the ADMM iteration.

The expected values come from the oracle only; the inputs come from the seeded scene
generator and are stored with them, so the fixture does not depend on the generator's
random streams.  The paper prints no iterate values, so this file is a regression anchor
for the oracle and a parity case that needs no oracle run, not a value of the paper.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth                              # noqa: E402
from oracle import nlpr_oracle as o       # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_12x12x3.json")


def main():
    spec = synth.small_spec(p=12, q=12, L=3, Lh=2, d=2, blur_radius=1, K=1, Sw=1, iters=6,
                            seed=71, tile=4)
    sc = synth.make_scene(spec)
    f64 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    Yl, Yh, b, R = f64(sc.Yl), f64(sc.Yh), f64(sc.blur), f64(sc.R)
    pr = o.Problem(p=spec.p, q=spec.q, L=spec.L, d=spec.d, b=b, R=R, K=spec.K, S=spec.Sw,
                   lam=spec.lam, rho=spec.rho, h=float(sc.h), lam1=spec.lam1)
    Z = o.solve(Yl, Yh, pr, spec.iters).X
    rec = {
        "what": "FP64 oracle Z after 6 ADMM iterations from the default start (regression "
                "anchor written by tests/golden/make_golden.py; not a value of the paper)",
        "p": spec.p, "q": spec.q, "L": spec.L, "Lh": int(R.shape[1]), "d": spec.d,
        "K": spec.K, "Sw": spec.Sw, "iters": spec.iters, "lam": spec.lam, "rho": spec.rho,
        "lam1": spec.lam1, "h": float(sc.h),
        "blur": b.tolist(), "R": R.tolist(), "Yl": Yl.tolist(), "Yh": Yh.tolist(),
        "Z": Z.tolist(),
    }
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=None)
        f.write("\n")
    print(OUT)


if __name__ == "__main__":
    main()

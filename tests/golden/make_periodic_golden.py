"""Writes tests/golden/periodic_c3_32x32x128.npz and periodic_c2_32x32x100.npz: the FP64
oracle's Z after 100 ADMM iterations on a 32 x 32 scene shaped like the 512 x 512 HS+MS
(128 bands, 4-band MS guide) and HS+PAN (100 bands, PAN guide) workloads: 9 x 9 blur with
sigma 2.5, decimation 4, patch 5 x 5, search window 11 x 11, lambda 1e-3, rho 1e-2.

Why 32 x 32.  Every operator of the iteration is circular on the periodic pixel grid (the
blur, the shifts of the patch differences and of the weights, the Fourier solve) and the
sampling keeps the pixels (4 m1, 4 m2), so one ADMM iteration commutes with a circular
shift by a multiple of 4.  If the observations of a 512 x 512 problem are the 32 x 32
observations tiled 16 x 16 times, every iterate is therefore 32-periodic, and the
512 x 512 result is the 32 x 32 result tiled.  The blur radius (4), the patch radius (2)
and the search radius (5) are all below 16, so no offset of the 32 x 32 problem aliases
with another one.  This gives an oracle value for a solve at the full 512 x 512 launch
shape, whose own literal FP64 oracle state (Q and Sigma for 121 shifts x 25 patch offsets)
would need about 1.6 TB.

The expected values come from the oracle only; the inputs come from the seeded scene
generator (one scene of period 32: its random fields are circular and its texture tile is
32 x 32) and are stored with them as the float32 values the library takes.

    python tests/golden/make_periodic_golden.py [workers]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth                              # noqa: E402
from oracle import nlpr_oracle as o       # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
CASES = {"c3": "periodic_c3_32x32x128.npz", "c2": "periodic_c2_32x32x100.npz"}
PERIOD = 32
ITERS = 100


def write(cfg: str, workers: int) -> str:
    spec = synth.config(cfg, p=PERIOD, q=PERIOD, iters=ITERS)
    sc = synth.make_scene(spec)
    f64 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    Yl, Yh, b, R = f64(sc.Yl), f64(sc.Yh), f64(sc.blur), f64(sc.R)
    pr = o.Problem(p=spec.p, q=spec.q, L=spec.L, d=spec.d, b=b, R=R, K=spec.K, S=spec.Sw,
                   lam=spec.lam, rho=spec.rho, h=float(sc.h), lam1=spec.lam1)
    t0 = time.time()
    Z = o.solve(Yl, Yh, pr, ITERS, workers=workers).X
    out = os.path.join(HERE, CASES[cfg])
    np.savez_compressed(
        out, Yl=sc.Yl, Yh=sc.Yh, blur=sc.blur, R=sc.R, Z=Z,
        params=np.array([spec.p, spec.q, spec.L, R.shape[1], spec.d, spec.K, spec.Sw, ITERS]),
        scalars=np.array([spec.lam, spec.rho, spec.lam1, float(sc.h)]))
    print(f"{out}: {ITERS} iterations in {time.time() - t0:.0f} s", flush=True)
    return out


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 1
    for cfg in CASES:
        write(cfg, workers)


if __name__ == "__main__":
    main()

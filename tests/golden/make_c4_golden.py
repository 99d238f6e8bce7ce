"""Writes tests/golden/c4_batch48_samples.npz: FP64 oracle values for every scene of the
48-scene batch workload (synth.batch_specs(48): sides 128..512, 4..128 bands, decimation 4
or 8, PAN or 4-band guide, blur 9x9 or 17x17, patch 3x3, window 3x3) after 100 iterations.

Which scenes.  A scene of side 128 is used as drawn; its literal oracle state (Q and Sigma
for 9 shifts x 9 patch offsets, float64) is at most 2.7 GB.  The larger scenes (192 to 512)
would need up to 43 GB each, so their content is a 32 x 32 scene, drawn with the same
generator, spec and seed at side 32, tiled over the full side: every operator of the
iteration is circular and the sampling phase repeats every 4 or 8 pixels, so their iterates
are the 32 x 32 iterates tiled (no offset aliases: blur radius <= 8 and patch and window
radius 1 are below 16).  The GPU still solves the full-size scene inside the full batch.

What is stored, per scene: the oracle's Z at 256 seeded pixel positions in every band
(float32; the test bar is 1e-4), the positions, the L2 norm of every band of the oracle's
whole Z (float64), the tiling factor and the sha256 of the float32 inputs.

    python tests/golden/make_c4_golden.py [workers]
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth                              # noqa: E402
from oracle import nlpr_oracle as o       # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_batch48_samples.npz")
PERIOD = 32
NSAMPLE = 256
ITERS = 100


def c4_scene_specs():
    """(full spec, spec of the scene that is solved by the oracle, tiling factor) for each of
    the 48 scenes."""
    out = []
    for spec in synth.batch_specs(48, iters=ITERS):
        if spec.p == 128:
            out.append((spec, spec, 1))
        else:
            out.append((spec, spec.replace(p=PERIOD, q=PERIOD), spec.p // PERIOD))
    return out


def input_digest(sc) -> str:
    h = hashlib.sha256()
    for a in (sc.Yl, sc.Yh, sc.blur, sc.R):
        h.update(np.ascontiguousarray(a, dtype=np.float32).tobytes())
    return h.hexdigest()


def sample_positions(s: int, side: int) -> np.ndarray:
    rng = np.random.default_rng(7000 + s)
    return np.stack([rng.integers(0, side, NSAMPLE), rng.integers(0, side, NSAMPLE)], axis=1)


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 1
    rec = {}
    t0 = time.time()
    for s, (spec, base, reps) in enumerate(c4_scene_specs()):
        sc = synth.make_scene(base)
        pr = o.Problem.from_scene(sc)
        Z = o.solve(sc.Yl.astype(np.float64), sc.Yh.astype(np.float64), pr, ITERS,
                    workers=workers).X
        pos = sample_positions(s, base.p)
        rec[f"s{s}_pos"] = pos.astype(np.int16)
        rec[f"s{s}_z"] = Z[:, pos[:, 0], pos[:, 1]].astype(np.float32)
        rec[f"s{s}_norms"] = np.sqrt(np.sum(Z * Z, axis=(1, 2)))
        rec[f"s{s}_meta"] = np.array([reps, base.p, spec.p, spec.L, spec.d])
        rec[f"s{s}_sha"] = np.array(input_digest(sc))
        print(f"scene {s}: {spec.p}x{spec.q}x{spec.L} d={spec.d} Lh={sc.R.shape[1]} "
              f"(oracle at {base.p}x{base.q}, tiled {reps}x{reps}) done at "
              f"{time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(OUT, **rec)
    print(OUT, flush=True)


if __name__ == "__main__":
    main()

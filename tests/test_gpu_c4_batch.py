"""The 48-scene batch workload at its configuration: all 48 scenes of synth.batch_specs(48)
(sides 128 to 512, 4 to 128 bands, decimation 4 or 8, PAN or 4-band guide, 9x9 or 17x17
blur, patch and window 3x3) solved together for 100 iterations in one batched launch
sequence replayed from a HIP graph, as the benchmark runs it.

Oracle values come from tests/golden/make_c4_golden.py.  Scenes of side 128 are drawn as
they are; the larger ones are a 32 x 32 scene of the same spec and seed tiled over the full
side (every operator is circular and the sampling phase repeats every 4 or 8 pixels, so
their iterates are the 32 x 32 ones tiled).  Per scene the golden file holds the FP64 Z at
256 seeded pixel positions in every band, and the norm of every band of the whole Z.  The
GPU's Z is compared at those positions in every tile (relative RMSE <= 1e-4) and by band
norms (each within 1e-4).  Every scene must also equal its own single-scene solve bit for
bit.
"""
import hashlib
import os

import numpy as np
import pytest
import torch

import synth
from paper_2210_04184_amd import nlpr

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "c4_batch48_samples.npz")
PERIOD = 32


def digest(sc) -> str:
    h = hashlib.sha256()
    for a in (sc.Yl, sc.Yh, sc.blur, sc.R):
        h.update(np.ascontiguousarray(a, dtype=np.float32).tobytes())
    return h.hexdigest()


def build_scenes(g):
    out = []
    for s, spec in enumerate(synth.batch_specs(48, iters=100)):
        base = spec if spec.p == 128 else spec.replace(p=PERIOD, q=PERIOD)
        reps = spec.p // base.p
        sc = synth.make_scene(base)
        assert digest(sc) == str(g[f"s{s}_sha"]), f"scene {s} differs from the golden's inputs"
        kw = dict(p=spec.p, q=spec.q, L=spec.L, Lh=sc.R.shape[1], d=spec.d, blur=sc.blur,
                  R=sc.R, K=spec.K, Sw=spec.Sw, iters=spec.iters, lam=spec.lam, rho=spec.rho,
                  h=sc.h, lam1=spec.lam1, flags=nlpr.GRAPH)
        Yl = torch.from_numpy(np.ascontiguousarray(np.tile(sc.Yl, (1, reps, reps)))).cuda()
        Yh = torch.from_numpy(np.ascontiguousarray(np.tile(sc.Yh, (1, reps, reps)))).cuda()
        out.append((spec, base, reps, kw, Yl, Yh))
    return out


def test_c4_batch_of_48_scenes_against_oracle_and_single_solves():
    g = np.load(GOLDEN)
    scenes = build_scenes(g)
    print(f"[c4] 48 scenes, {sum(s.p * s.q * s.L for s, *_ in scenes) / 1e6:.0f} M pixel-bands,"
          f" 100 iterations", flush=True)
    batch = nlpr.Batch([kw for _, _, _, kw, _, _ in scenes])
    try:
        Zs, ws = batch.solve([y for *_, y, _ in scenes], [y for *_, y in scenes])
        torch.cuda.synchronize()
        del ws
        worst = 0.0
        for s, (spec, base, reps, kw, Yl, Yh) in enumerate(scenes):
            z = Zs[s].cpu().numpy().astype(np.float64)
            L = spec.L
            pos = g[f"s{s}_pos"].astype(np.int64)
            ref = g[f"s{s}_z"].astype(np.float64)                  # [L][256]
            # [L][base row][base col][tile row][tile col], then the samples of every tile:
            # t is [L][256][reps][reps]
            zz = z.reshape(L, reps, base.p, reps, base.q).transpose(0, 2, 4, 1, 3)
            t = zz[:, pos[:, 0], pos[:, 1]]
            d = t - ref[:, :, None, None]
            rel = float(np.sqrt(np.sum(d * d) / (reps * reps * np.sum(ref * ref))))
            norms = np.sqrt(np.sum(z * z, axis=(1, 2))) / reps
            nrel = float(np.max(np.abs(norms - g[f"s{s}_norms"]) / g[f"s{s}_norms"]))
            worst = max(worst, rel, nrel)
            assert rel <= 1e-4, (s, spec, rel)
            assert nrel <= 1e-4, (s, spec, nrel)
        print(f"[c4] worst relative error over the 48 scenes: {worst:.3e}", flush=True)
        # each scene alone, same flags: bit-for-bit the batch's result
        for s, (spec, base, reps, kw, Yl, Yh) in enumerate(scenes):
            plan = nlpr.Plan(**kw)
            try:
                Z, _ = plan.solve(Yl, Yh)
                assert torch.equal(Z, Zs[s]), f"scene {s}: batch != single-scene solve"
                del Z
            finally:
                plan.close()
    finally:
        batch.close()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()

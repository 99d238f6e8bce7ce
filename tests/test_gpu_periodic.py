"""The 100-iteration solve at the full 512 x 512 launch shape against FP64 oracle values.

The oracle cannot hold the literal dual state of a 512 x 512 x 128 solve with an 11 x 11
window and 5 x 5 patches, so the inputs here are a 32 x 32 scene tiled 16 x 16 times.  Every
operator of the iteration is circular and the sampling phase repeats every 4 pixels, so the
512 x 512 iterates are the 32 x 32 ones tiled (tests/golden/make_periodic_golden.py, which
writes the oracle's 100-iteration Z for the 32 x 32 scene).  The GPU runs the full-size
problem exactly as the benchmark does (same plan flags, same sweep tiles of 2 image rows,
256 tiles x all bands, one workgroup per tile and band, a 5-row halo reaching over three
tiles), so this checks every kernel at the benchmark's launch geometry for all 100
iterations.  It is the benchmark's geometry on a periodic scene, not the benchmark's scene.
"""
import gc
import os

import numpy as np
import pytest
import torch

from paper_2210_04184_amd import nlpr

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
SIDE = 512


def load_case(fname):
    g = np.load(os.path.join(GOLDEN, fname))
    p, q, L, Lh, d, K, Sw, iters = (int(v) for v in g["params"])
    lam, rho, lam1, h = (float(v) for v in g["scalars"])
    return g, dict(p=p, q=q, L=L, Lh=Lh, d=d, K=K, Sw=Sw, iters=iters, lam=lam, rho=rho,
                   lam1=lam1, h=h)


@pytest.mark.parametrize("fname", ["periodic_c3_32x32x128.npz", "periodic_c2_32x32x100.npz"])
def test_full_size_100_iterations_against_oracle_on_periodic_scene(fname):
    g, c = load_case(fname)
    reps = SIDE // c["p"]
    assert reps * c["p"] == SIDE and c["iters"] == 100
    Yl = np.tile(g["Yl"], (1, reps, reps))
    Yh = np.tile(g["Yh"], (1, reps, reps))
    print(f"[periodic] {fname}: {SIDE}x{SIDE}x{c['L']}, Lh={c['Lh']}, patch {2 * c['K'] + 1}, "
          f"window {2 * c['Sw'] + 1}, {c['iters']} iterations", flush=True)
    plan = nlpr.Plan(SIDE, SIDE, c["L"], c["Lh"], c["d"], g["blur"], g["R"], c["K"], c["Sw"],
                     c["iters"], c["lam"], c["rho"], c["h"], c["lam1"], flags=nlpr.TIMING)
    try:
        inf = plan.info()
        assert (inf.tile_rows, inf.ntiles, inf.sweep_split, inf.halo_rows) == (2, 256, 1, 5)
        Z, ws = plan.solve(torch.from_numpy(np.ascontiguousarray(Yl)).cuda(),
                           torch.from_numpy(np.ascontiguousarray(Yh)).cuda())
        z = Z.cpu().numpy().astype(np.float64)
        del Z, ws
    finally:
        plan.close()
        gc.collect()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    ref = np.tile(g["Z"], (1, reps, reps))
    rel = float(np.linalg.norm(z - ref) / np.linalg.norm(ref))
    # the worst of the 256 tiles: every tile is compared, not only the whole
    t = (z - ref).reshape(c["L"], reps, c["p"], reps, c["q"])
    tile_err = np.sqrt(np.sum(t * t, axis=(0, 2, 4))) / np.linalg.norm(g["Z"])
    print(f"[periodic] {fname}: relRMSE = {rel:.3e}, worst tile {tile_err.max():.3e}", flush=True)
    assert rel <= 1e-4
    assert tile_err.max() <= 1e-4

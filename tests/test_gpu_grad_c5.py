"""The differentiated workload at its full size against the FP64 reference gradient.

256 x 256 x 31 bands, 3-band MS guide, 7 x 7 blur, d = 4, patch and window 3 x 3, 20
unrolled iterations, loss mean((X^(20) - Z_true)^2): the reverse mode's gradients with
respect to Y_l, Y_h, lambda_2 and rho against those of torch autograd through the literal
FP64 iteration (tests/golden/make_c5_grad_golden.py, which calls only the oracle), at the
1e-3 relative bar of the workload (L2 norm for the images)."""
import hashlib
import os

import numpy as np
import pytest
import torch

import synth
from paper_2210_04184_amd import nlpr

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "grad_c5_256x256x31.npz")


def digest(sc) -> str:
    h = hashlib.sha256()
    for a in (sc.Yl, sc.Yh, sc.blur, sc.R):
        h.update(np.ascontiguousarray(a, dtype=np.float32).tobytes())
    h.update(np.ascontiguousarray(sc.Z, dtype=np.float64).tobytes())
    return h.hexdigest()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_c5_gradient_against_fp64_reference():
    g = np.load(GOLDEN)
    spec = synth.config("c5")
    sc = synth.make_scene(spec)
    assert digest(sc) == str(g["inputs_sha256"])
    print(f"[grad-c5] {spec.p}x{spec.q}x{spec.L}, {spec.iters} unrolled iterations", flush=True)
    plan = nlpr.Plan.from_scene(sc)
    try:
        Yl = torch.from_numpy(sc.Yl).cuda()
        Yh = torch.from_numpy(sc.Yh).cuda()
        Z, ws, ck = plan.forward(Yl, Yh)
        Zt = torch.from_numpy(sc.Z).cuda()
        Zd = Z.double()
        loss = float(torch.mean((Zd - Zt) ** 2))
        dZ = (2.0 * (Zd - Zt) / Zd.numel()).float()
        dYl, dYh, ds = plan.backward(Yl, Yh, dZ, ws, ck)
        torch.cuda.synchronize()
        gYl = dYl.cpu().numpy().astype(np.float64)
        gYh = dYh.cpu().numpy().astype(np.float64)
        s = ds.cpu().numpy()
    finally:
        plan.close()
    errs = {"loss": abs(loss - float(g["loss"])) / abs(float(g["loss"])),
            "dYl": rel(gYl, g["dYl"].astype(np.float64)),
            "dYh": rel(gYh, g["dYh"].astype(np.float64)),
            "dlambda": abs(s[0] - float(g["dlam"])) / abs(float(g["dlam"])),
            "drho": abs(s[1] - float(g["drho"])) / abs(float(g["drho"]))}
    print("[grad-c5] relative errors vs FP64 reference: "
          + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()), flush=True)
    assert errs["loss"] <= 1e-4
    for k in ("dYl", "dYh", "dlambda", "drho"):
        assert errs[k] <= 1e-3, (k, errs[k])

"""The library used from plain C: tests/c/abi_solve.c creates a plan from host tables,
allocates its buffers with hipMalloc, solves on its own HIP stream and writes Z back,
through include/nlpr.h alone.  Its output must meet the oracle bar and equal the Python
binding's result for the same inputs."""
import os
import struct
import subprocess

import numpy as np
import pytest
import torch

import synth
from oracle import nlpr_oracle as o
from paper_2210_04184_amd import nlpr

pytestmark = pytest.mark.gpu

DRIVER = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c", "abi_solve")


def test_plain_c_program_solves_through_the_abi(tmp_path):
    if not os.path.exists(DRIVER):
        pytest.fail("tests/c/abi_solve is not built (run __graft_entry__.build())")
    spec = synth.small_spec(p=48, q=64, L=5, Lh=2, d=4, blur_radius=2, K=1, Sw=2, iters=8,
                            seed=21)
    sc = synth.make_scene(spec)
    head = struct.pack("<9i", spec.p, spec.q, spec.L, sc.R.shape[1], spec.d, spec.blur_radius,
                       spec.K, spec.Sw, spec.iters)
    head += struct.pack("<4d", spec.lam, spec.lam1, spec.rho, sc.h)
    body = b"".join(np.ascontiguousarray(a, dtype=np.float32).tobytes()
                    for a in (sc.blur, sc.R, sc.Yl, sc.Yh))
    (tmp_path / "in.bin").write_bytes(head + body)
    res = subprocess.run([DRIVER, str(tmp_path / "in.bin"), str(tmp_path / "out.bin")],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    Z = np.fromfile(tmp_path / "out.bin", dtype=np.float32).reshape(spec.L, spec.p, spec.q)
    ref = o.solve(sc.Yl.astype(np.float64), sc.Yh.astype(np.float64), o.Problem.from_scene(sc),
                  spec.iters).X
    assert np.linalg.norm(Z - ref) / np.linalg.norm(ref) <= 1e-4
    Zb, _ = nlpr.Plan.from_scene(sc).solve(torch.from_numpy(sc.Yl).cuda(),
                                           torch.from_numpy(sc.Yh).cuda())
    assert np.array_equal(Z, Zb.cpu().numpy())

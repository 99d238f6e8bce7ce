"""Writes tests/golden/grad_c5_256x256x31.npz: the FP64 reference gradient of the
differentiated workload, computed by ``oracle.nlpr_grad`` (torch autograd in float64 through
the literal iteration, Q and Sigma for every shift and patch offset) at its full size:
256 x 256 x 31 bands, 3-band MS guide, 7 x 7 blur with sigma 2, decimation 4, patch 3 x 3,
window 3 x 3, lambda 1e-3, rho 1e-2, 20 unrolled iterations from the default start, and the
loss mean((X^(20) - Z_true)^2).

The literal state of one iterate is 2.7 GB (81 (shift, patch offset) pairs of Q and Sigma,
float64), so keeping the whole reverse-mode graph of 20 iterations does not fit in memory.
The gradient is therefore taken with recomputation checkpoints (segments of iterations
rerun during the backward pass); that changes what is held in memory, not the arithmetic
(tests/test_oracle_grad.py checks that the result is the same bit for bit).

Stored: the loss, dloss/dlambda_2 and dloss/drho in float64, dloss/dY_l and dloss/dY_h
rounded to float32 (the comparison bar is 1e-3 relative), and the sha256 of the float32
inputs the scene generator gives, so that the test can tell it regenerated the same scene.

    python tests/golden/make_c5_grad_golden.py
"""
import hashlib
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth                              # noqa: E402
from oracle import nlpr_grad as og        # noqa: E402
from oracle import nlpr_oracle as o       # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "grad_c5_256x256x31.npz")


def input_digest(sc) -> str:
    h = hashlib.sha256()
    for a in (sc.Yl, sc.Yh, sc.blur, sc.R):
        h.update(np.ascontiguousarray(a, dtype=np.float32).tobytes())
    h.update(np.ascontiguousarray(sc.Z, dtype=np.float64).tobytes())
    return h.hexdigest()


def bound_host_memory():
    """Serve every allocation of 1 MiB or more by its own mapping, returned to the system
    when freed, and keep two malloc arenas: without this, glibc's arenas keep the freed
    16 MB planes of the rerun iterations and the resident size grows to several times
    what is live (measured: 36 GB instead of 14 GB for two iterations)."""
    import ctypes
    libc = ctypes.CDLL("libc.so.6")
    M_MMAP_THRESHOLD, M_ARENA_MAX = -3, -8
    libc.mallopt(M_MMAP_THRESHOLD, 1 << 20)
    libc.mallopt(M_ARENA_MAX, 2)


def main():
    bound_host_memory()
    torch.set_num_threads(os.cpu_count() or 1)
    spec = synth.config("c5")
    sc = synth.make_scene(spec)
    pr = o.Problem.from_scene(sc)
    t0 = time.time()
    loss, gYl, gYh, glam, grho = og.gradient(sc.Yl.astype(np.float64),
                                             sc.Yh.astype(np.float64), pr, spec.iters, sc.Z,
                                             segments=4)
    np.savez_compressed(OUT, loss=np.float64(loss), dlam=np.float64(glam),
                        drho=np.float64(grho), dYl=gYl.astype(np.float32),
                        dYh=gYh.astype(np.float32), inputs_sha256=np.array(input_digest(sc)))
    print(f"{OUT}: {spec.iters} iterations in {time.time() - t0:.0f} s; loss {loss:.6e}, "
          f"dlam {glam:.6e}, drho {grho:.6e}", flush=True)


if __name__ == "__main__":
    main()

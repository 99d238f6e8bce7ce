"""Edge cases of the solve: zero iterations, the smallest image, one band, the largest guide,
patch and window, no decimation, and the largest image size (by a property that holds at
any size, since the oracle cannot hold that state).

Tolerance: the 1e-4 relative RMSE bar on Z against the FP64 oracle; the periodic-tiling
property at 4096 x 4096 is held to 1e-5 (two FP32 solves whose FFT lengths differ).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import nlpr_oracle as o
from paper_2210_04184_amd import nlpr

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def check_against_oracle(spec, flags=0, init="upsample", **okw):
    sc = synth.make_scene(spec)
    Z, _ = nlpr.Plan.from_scene(sc, flags=flags).solve(dev(sc.Yl), dev(sc.Yh))
    pr = o.Problem.from_scene(sc, **okw)
    ref = o.solve(sc.Yl.astype(np.float64), sc.Yh.astype(np.float64), pr, spec.iters, init=init)
    assert rel(host(Z), ref.X) <= 1e-4
    return sc


def test_zero_iterations_return_the_start():
    sc = synth.make_scene(synth.small_spec(p=48, q=36, L=3, Lh=2, d=2, blur_radius=1, K=1,
                                           Sw=1, iters=0, seed=3, tile=8))
    Z, _ = nlpr.Plan.from_scene(sc).solve(dev(sc.Yl), dev(sc.Yh))
    assert np.array_equal(host(Z), o.upsample_nn(sc.Yl.astype(np.float64), 2))
    Z0, _ = nlpr.Plan.from_scene(sc, flags=nlpr.INIT_ZERO).solve(dev(sc.Yl), dev(sc.Yh))
    assert not host(Z0).any()


def test_smallest_image_one_band_identity_blur():
    # 8 x 8, one band, one guide band, no decimation, 1 x 1 blur, 1 x 1 patch
    check_against_oracle(synth.small_spec(p=8, q=8, L=1, Lh=1, d=1, blur_radius=0, K=0, Sw=1,
                                          iters=6, seed=4, tile=8))


def test_narrowest_image_with_patch_and_window():
    # q = 8: two float4 per row, so the sweep's wrapped threshold reads take the same float4
    # on both sides of a thread's columns; 3 x 3 patch, 5 x 5 window
    check_against_oracle(synth.small_spec(p=16, q=8, L=3, Lh=2, d=2, blur_radius=1, K=1, Sw=2,
                                          iters=6, seed=9, tile=4))


def test_no_decimation():
    check_against_oracle(synth.small_spec(p=32, q=48, L=3, Lh=2, d=1, blur_radius=2, K=1,
                                          Sw=2, iters=6, seed=5, tile=8))


def test_sixteen_guide_bands():
    check_against_oracle(synth.small_spec(p=32, q=32, L=16, Lh=16, d=4, blur_radius=1, K=1,
                                          Sw=1, iters=5, seed=6, tile=8))


def test_largest_patch_and_window():
    # K = 4 (9 x 9 patch) and Sw = 8 (17 x 17 window, 144 stored shifts)
    check_against_oracle(synth.small_spec(p=18, q=24, L=1, Lh=1, d=2, blur_radius=1, K=4,
                                          Sw=8, iters=2, seed=7, tile=6))


def test_largest_image_is_a_periodic_tiling_of_half_the_size():
    """Everything in the iteration is shift-equivariant on the periodic grid, so inputs
    tiled 2 x 2 from a 2048 x 2048 scene give the 2 x 2 tiling of its solution.  4096 x 4096
    is the largest supported side; blur radius 16 and d = 8 are the largest too."""
    spec = synth.small_spec(p=2048, q=2048, L=2, Lh=1, d=8, blur_radius=16, K=1, Sw=1, iters=3,
                            seed=8, tile=16)
    sc = synth.make_scene(spec)
    small = nlpr.Plan.from_scene(sc)
    Zs, _ = small.solve(dev(sc.Yl), dev(sc.Yh))
    big = nlpr.Plan.from_scene(sc, p=4096, q=4096)
    Zb, _ = big.solve(dev(np.tile(sc.Yl, (1, 2, 2))), dev(np.tile(sc.Yh, (1, 2, 2))))
    want = np.tile(host(Zs), (1, 2, 2))
    del small, Zs
    assert rel(host(Zb), want) <= 1e-5


def test_reference_stream_negates_in_place_and_checks_its_arguments():
    x = torch.randn(4 * 100003, device="cuda")
    want = -x
    nlpr.stream_rmw(x)
    torch.cuda.synchronize()
    assert torch.equal(x, want)
    import ctypes
    lib = nlpr.load()
    for bad in (torch.randn(10, device="cuda"),          # 40 bytes: not a multiple of 16
                torch.randn(17, device="cuda")[1:]):     # 4 bytes past an aligned start
        with pytest.raises(nlpr.NlprError) as e:
            nlpr.stream_rmw(bad)
        assert e.value.status == nlpr.ERR_INVALID_ARG
    with pytest.raises(ValueError):
        nlpr.stream_rmw(torch.zeros(16))
    host = np.zeros(16, dtype=np.float32)
    assert lib.nlpr_stream_rmw(host.ctypes.data_as(ctypes.c_void_p), 64, None) == nlpr.ERR_INVALID_ARG
    assert lib.nlpr_stream_rmw(None, 64, None) == nlpr.ERR_INVALID_ARG


def test_sweep_shaped_stream_negates_each_chunk_once_and_checks_its_arguments():
    # 12 chunks of two steps of three 4 KB planes, 4 bands: every chunk is negated exactly
    # once (a chunk visited twice would come back unchanged), the bytes after them stay
    import ctypes
    planes, chunk, nchunks, bands = 3, 2 * 3 * 4096, 12, 4
    n = nchunks * chunk // 4
    x = torch.randn(n + 1000, device="cuda")
    want = torch.cat([-x[:n], x[n:]])
    nlpr.stream_chunks(x, chunk, nchunks, bands, planes, lds_bytes=40960)
    torch.cuda.synchronize()
    assert torch.equal(x, want)
    # from an offset into a byte buffer (as on a workspace region)
    w = torch.zeros(4096 + chunk * 2, dtype=torch.uint8, device="cuda")
    w[4096:].view(torch.float32).fill_(1.0)
    nlpr.stream_chunks(w, chunk, 2, 2, planes, offset=4096)
    torch.cuda.synchronize()
    assert bool((w[4096:].view(torch.float32) == -1.0).all()) and not w[:4096].any()
    for kw in (dict(planes=0), dict(planes=9), dict(chunk_bytes=chunk + 16),
               dict(nchunks=10), dict(nchunks=16), dict(lds_bytes=160 * 1024 + 1)):
        args = dict(chunk_bytes=chunk, nchunks=nchunks, bands=bands, planes=planes, lds_bytes=0)
        args.update(kw)
        with pytest.raises(nlpr.NlprError) as e:
            nlpr.stream_chunks(x, **args)
        assert e.value.status == nlpr.ERR_INVALID_ARG, kw
    host = np.zeros(4096, dtype=np.float32)
    lib = nlpr.load()
    assert lib.nlpr_stream_chunks(host.ctypes.data_as(ctypes.c_void_p), host.nbytes, 4096, 1, 1,
                                  1, 0, None) == nlpr.ERR_INVALID_ARG

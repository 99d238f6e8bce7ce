"""Python binding of libnlpr (ctypes).

Argument marshalling only: every step of the solver runs in the HIP library.  PyTorch
supplies device memory and the stream.  The binding fails loudly when the library is not
built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnlpr.so")

# status codes and flags (include/nlpr.h)
OK = 0
ERR_INVALID_ARG = 1
ERR_UNSUPPORTED_SHAPE = 2
ERR_WORKSPACE_TOO_SMALL = 3
ERR_HIP = 4
ERR_NUMERICAL = 5
ERR_NOT_ENABLED = 6

INIT_ZERO = 1 << 0
STATE_IN = 1 << 1
UNWEIGHTED = 1 << 2
LOCAL_WINDOW = 1 << 3
CHECK_FINITE = 1 << 4
TIMING = 1 << 5
GRAPH = 1 << 6
FUSED_S = 1 << 7

STAGE_WEIGHTS = 1
STAGE_XSOLVE = 2
STAGE_BLUR = 3
STAGE_BLUR_T = 4
STAGE_PUPDATE = 5
STAGE_SWEEP = 6
STAGE_SWEEP_FIRST = 7
STAGE_ASSEMBLE = 8
STAGE_INIT = 9
STAGE_MONITOR = 10
STAGE_NAMES = {STAGE_WEIGHTS: "weights", STAGE_XSOLVE: "xsolve", STAGE_BLUR: "blur",
               STAGE_BLUR_T: "blur_t", STAGE_PUPDATE: "pupdate", STAGE_SWEEP: "sweep",
               STAGE_SWEEP_FIRST: "sweep_first", STAGE_ASSEMBLE: "assemble", STAGE_INIT: "init",
               STAGE_MONITOR: "monitor"}

# fields of a monitor record (nlpr_monitor)
MON_FIELDS = ("iteration", "objective", "data_l", "data_h", "reg", "r1", "r2")
MON_RECORD = 8

REGION_SIGMA = 0
REGION_MU = 1
REGION_C = 2
REGION_LAMBDA1 = 3
REGION_LAMBDA2 = 4
REGION_SIGMA_CODES = 5

EXPORTED = sorted(["nlpr_plan_create", "nlpr_workspace_size", "nlpr_solve", "nlpr_plan_destroy",
                   "nlpr_status_string", "nlpr_last_error", "nlpr_half_window",
                   "nlpr_workspace_region", "nlpr_debug_stage", "nlpr_stage_time",
                   "nlpr_plan_get_info", "nlpr_batch_create", "nlpr_batch_workspace_size",
                   "nlpr_batch_region", "nlpr_batch_solve", "nlpr_batch_stage_time",
                   "nlpr_batch_destroy", "nlpr_monitor", "nlpr_batch_monitor",
                   "nlpr_grad_sizes", "nlpr_forward", "nlpr_backward", "nlpr_stream_rmw",
                   "nlpr_stream_chunks", "nlpr_solve_noalloc", "nlpr_nonfinite_iteration",
                   "nlpr_sigma_expand", "nlpr_sweep_counts"])

# size of the library's static workspace used by nlpr_solve_noalloc (include/nlpr.h)
NOALLOC_WORKSPACE_BYTES = 64 << 20


class NlprError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"nlpr status {status}: {msg}")
        self.status = status
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("q", ctypes.c_int32), ("L", ctypes.c_int32),
                ("Lh", ctypes.c_int32), ("d", ctypes.c_int32), ("blur_radius", ctypes.c_int32),
                ("K", ctypes.c_int32), ("Sw", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("Ls", ctypes.c_int32), ("monitor_every", ctypes.c_int32),
                ("lam", ctypes.c_double), ("lam1", ctypes.c_double),
                ("rho", ctypes.c_double), ("h", ctypes.c_double)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("npairs", ctypes.c_int32), ("npatch", ctypes.c_int32),
                ("tile_rows", ctypes.c_int32), ("ntiles", ctypes.c_int32),
                ("halo_rows", ctypes.c_int32), ("blur_separable", ctypes.c_int32),
                ("sweep_split", ctypes.c_int32), ("sigma_elems", ctypes.c_size_t)]


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libnlpr.so (once).  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libnlpr.so not found at {path}; run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    lib.nlpr_plan_create.argtypes = [ctypes.POINTER(Params), vp, vp, vp, ctypes.POINTER(vp)]
    lib.nlpr_workspace_size.argtypes = [vp, ctypes.POINTER(sz)]
    lib.nlpr_solve.argtypes = [vp, vp, vp, vp, vp, sz, vp]
    lib.nlpr_solve_noalloc.argtypes = [vp, vp, vp, vp, vp]
    lib.nlpr_nonfinite_iteration.argtypes = [vp, ctypes.POINTER(i32)]
    lib.nlpr_sigma_expand.argtypes = [vp, vp, vp, vp, i32, i32, vp, vp]
    lib.nlpr_sweep_counts.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), i32, ctypes.POINTER(i32)]
    lib.nlpr_plan_destroy.argtypes = [vp]
    lib.nlpr_status_string.argtypes = [ctypes.c_int]
    lib.nlpr_status_string.restype = ctypes.c_char_p
    lib.nlpr_last_error.argtypes = []
    lib.nlpr_last_error.restype = ctypes.c_char_p
    lib.nlpr_half_window.argtypes = [vp, ctypes.POINTER(i32), i32, ctypes.POINTER(i32)]
    lib.nlpr_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    lib.nlpr_workspace_region.argtypes = [vp, ctypes.c_int, ctypes.POINTER(sz), ctypes.POINTER(sz)]
    lib.nlpr_debug_stage.argtypes = [vp, ctypes.c_int, ctypes.POINTER(vp), i32, vp]
    lib.nlpr_stage_time.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
    pp = ctypes.POINTER(ctypes.c_void_p)
    lib.nlpr_batch_create.argtypes = [i32, ctypes.POINTER(Params), pp, pp, pp, ctypes.POINTER(vp)]
    lib.nlpr_batch_workspace_size.argtypes = [vp, ctypes.POINTER(sz)]
    lib.nlpr_batch_region.argtypes = [vp, i32, ctypes.c_int, ctypes.POINTER(sz), ctypes.POINTER(sz)]
    lib.nlpr_batch_solve.argtypes = [vp, pp, pp, pp, vp, sz, vp]
    lib.nlpr_batch_stage_time.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
    lib.nlpr_batch_destroy.argtypes = [vp]
    dp = ctypes.POINTER(ctypes.c_double)
    lib.nlpr_monitor.argtypes = [vp, dp, i32, ctypes.POINTER(i32)]
    lib.nlpr_batch_monitor.argtypes = [vp, i32, dp, i32, ctypes.POINTER(i32)]
    lib.nlpr_grad_sizes.argtypes = [vp, ctypes.POINTER(sz), ctypes.POINTER(sz)]
    lib.nlpr_forward.argtypes = [vp, vp, vp, vp, vp, sz, vp, sz, vp]
    lib.nlpr_backward.argtypes = [vp, vp, vp, vp, vp, sz, vp, sz, vp, sz, vp, vp, vp, vp]
    lib.nlpr_stream_rmw.argtypes = [vp, sz, vp]
    lib.nlpr_stream_chunks.argtypes = [vp, sz, sz, i32, i32, i32, sz, vp]
    for name in EXPORTED:
        if name not in ("nlpr_status_string", "nlpr_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int):
    if rc != OK:
        lib = load()
        raise NlprError(rc, f"{lib.nlpr_status_string(rc).decode()}: {lib.nlpr_last_error().decode()}")


def _ptr(t) -> int:
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def stream_rmw(buf, stream=None) -> None:
    """Negate a float32 device tensor in place with the library's reference stream (one
    16-byte non-temporal load and store per thread, the dual sweep's access pattern)."""
    import torch
    if buf.dtype != torch.float32:
        raise TypeError("stream_rmw takes a float32 tensor")
    _check(load().nlpr_stream_rmw(_ptr(buf), buf.numel() * 4, _stream_handle(stream)))


def stream_chunks(buf, chunk_bytes: int, nchunks: int, bands: int, planes: int,
                  lds_bytes: int = 0, offset: int = 0, stream=None) -> None:
    """The sweep-shaped reference stream (nlpr_stream_chunks) on the bytes of the device
    tensor ``buf`` from ``offset`` on: nchunks chunks of chunk_bytes, negated in place."""
    if not buf.is_cuda or not buf.is_contiguous():
        raise ValueError("buf must be a contiguous device tensor")
    nbytes = buf.numel() * buf.element_size()
    if not 0 <= offset <= nbytes:
        raise ValueError("offset outside buf")
    _check(load().nlpr_stream_chunks(_ptr(buf) + offset, nbytes - offset, chunk_bytes, nchunks,
                                     bands, planes, lds_bytes, _stream_handle(stream)))


class Plan:
    """A solver plan: problem sizes, parameters and the precomputed device tables."""

    def __init__(self, p: int, q: int, L: int, Lh: int, d: int, blur: np.ndarray,
                 R: np.ndarray, K: int, Sw: int, iters: int, lam: float, rho: float, h: float,
                 lam1: float = 1.0, flags: int = 0, E: Optional[np.ndarray] = None,
                 monitor_every: int = 0):
        lib = load()
        blur = np.ascontiguousarray(blur, dtype=np.float32)
        R = np.ascontiguousarray(R, dtype=np.float32).reshape(L, Lh)
        r = blur.shape[0] // 2
        if blur.shape != (2 * r + 1, 2 * r + 1):
            raise ValueError("blur must be (2r+1) x (2r+1)")
        Ls = 0
        if E is not None:
            E = np.ascontiguousarray(E, dtype=np.float32)
            Ls = E.shape[0]
            if E.shape != (Ls, L):
                raise ValueError("E must be Ls x L")
        self.params = Params(p, q, L, Lh, d, r, K, Sw, iters, flags, Ls, monitor_every, lam, lam1,
                             rho, h)
        self.shape = (L, p, q)
        self.xbands = Ls if Ls else L
        self._blur, self._R, self._E = blur, R, E
        handle = ctypes.c_void_p()
        _check(lib.nlpr_plan_create(ctypes.byref(self.params), blur.ctypes.data_as(ctypes.c_void_p),
                                    R.ctypes.data_as(ctypes.c_void_p),
                                    None if E is None else E.ctypes.data_as(ctypes.c_void_p),
                                    ctypes.byref(handle)))
        self.handle = handle

    @classmethod
    def from_scene(cls, scene, flags: int = 0, **over) -> "Plan":
        return cls(**_scene_kwargs(scene, flags, **over))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            load().nlpr_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def workspace_bytes(self) -> int:
        n = ctypes.c_size_t()
        _check(load().nlpr_workspace_size(self.handle, ctypes.byref(n)))
        return n.value

    def half_window(self) -> Sequence[Tuple[int, int]]:
        n = ctypes.c_int32()
        _check(load().nlpr_half_window(self.handle, None, 0, ctypes.byref(n)))
        buf = (ctypes.c_int32 * (2 * max(n.value, 1)))()
        _check(load().nlpr_half_window(self.handle, buf, n.value, ctypes.byref(n)))
        return [(buf[2 * i], buf[2 * i + 1]) for i in range(n.value)]

    def info(self) -> PlanInfo:
        inf = PlanInfo()
        _check(load().nlpr_plan_get_info(self.handle, ctypes.byref(inf)))
        return inf

    def alloc_sigma(self, fill: float = float("nan")):
        """A standalone Sigma' buffer (the values of the coded layout of the workspace region)
        for the sweep stage; its code bytes live in the stage's workspace."""
        import torch
        return torch.full((self.info().sigma_elems,), fill, dtype=torch.float32, device="cuda")

    def sigma_expand(self, sig, codes, mu, c0: int = 0, c1: Optional[int] = None, stream=None):
        """Dense Sigma' of bands [c0, c1) from its coded form: [Npairs][|P|][c1 - c0][p][q].
        sig, codes, mu: float32, uint8 and float32 device tensors (values, code bytes and
        thresholds)."""
        import torch
        inf = self.info()
        _, p, q = self.shape
        c1 = self.xbands if c1 is None else c1
        out = torch.empty((c1 - c0, inf.npairs, inf.npatch, p, q), dtype=torch.float32,
                          device="cuda")
        _check(load().nlpr_sigma_expand(self.handle, _ptr(sig), _ptr(codes), _ptr(mu), c0, c1,
                                        _ptr(out), _stream_handle(stream)))
        return out.permute(1, 2, 0, 3, 4)

    def state_sigma(self, ws, c0: int = 0, c1: Optional[int] = None, stream=None):
        """Dense Sigma' [Npairs][|P|][c1 - c0][p][q] of the state a solve left in ws."""
        return self.sigma_expand(self.region_view(ws, REGION_SIGMA),
                                 self.region_bytes(ws, REGION_SIGMA_CODES),
                                 self.region_view(ws, REGION_MU), c0, c1, stream)

    def region_bytes(self, ws, which: int):
        """A uint8 view of one workspace region (ws is a uint8 device tensor)."""
        off, nb = self.region(which)
        return ws[off:off + nb]

    def sweep_counts(self):
        """Open Sigma' items (float4s stored) written by each sweep of the last solve
        (plans created with TIMING)."""
        n = ctypes.c_int32()
        _check(load().nlpr_sweep_counts(self.handle, None, 0, ctypes.byref(n)))
        out = (ctypes.c_int64 * max(n.value, 1))()
        _check(load().nlpr_sweep_counts(self.handle, out, n.value, ctypes.byref(n)))
        return [out[i] for i in range(n.value)]

    def region(self, which: int) -> Tuple[int, int]:
        off, nb = ctypes.c_size_t(), ctypes.c_size_t()
        _check(load().nlpr_workspace_region(self.handle, which, ctypes.byref(off), ctypes.byref(nb)))
        return off.value, nb.value

    def region_view(self, ws, which: int):
        """A float32 view of one workspace region (ws is a uint8 device tensor)."""
        off, nb = self.region(which)
        return ws[off:off + nb].view(dtype=__import__("torch").float32)

    def alloc_workspace(self):
        import torch
        return torch.empty(self.workspace_bytes, dtype=torch.uint8, device="cuda")

    def solve(self, Yl, Yh, Z=None, ws=None, stream=None):
        import torch
        if Z is None:
            Z = torch.empty(self.shape, dtype=torch.float32, device=Yl.device)
        if ws is None:
            ws = self.alloc_workspace()
        _check(load().nlpr_solve(self.handle, _ptr(Yl), _ptr(Yh), _ptr(Z), _ptr(ws),
                                 ws.numel() * ws.element_size(), _stream_handle(stream)))
        return Z, ws

    def nonfinite_iteration(self) -> int:
        """With CHECK_FINITE: the first checked iteration of the last solve that found NaN or
        Inf in the iterate, or -1."""
        t = ctypes.c_int32()
        _check(load().nlpr_nonfinite_iteration(self.handle, ctypes.byref(t)))
        return t.value

    def solve_noalloc(self, Yl, Yh, Z, stream=None):
        """nlpr_solve_noalloc: the solve with the library's static workspace; Z is the
        caller's output tensor.  Calls that overlap on one GPU race (they share the array)."""
        _check(load().nlpr_solve_noalloc(self.handle, _ptr(Yl), _ptr(Yh), _ptr(Z),
                                         _stream_handle(stream)))
        return Z

    def stage(self, stage: int, bufs, stream=None):
        arr = (ctypes.c_void_p * len(bufs))(*[_ptr(b) for b in bufs])
        _check(load().nlpr_debug_stage(self.handle, stage, arr, len(bufs), _stream_handle(stream)))

    def stage_time(self, stage: int, reset: bool = False) -> Tuple[float, int]:
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(load().nlpr_stage_time(self.handle, stage, ctypes.byref(ms), ctypes.byref(n),
                                      1 if reset else 0))
        return ms.value, n.value

    def monitor(self) -> np.ndarray:
        """Monitor records of the last solve, [n][8] float64 (fields MON_FIELDS)."""
        return _read_monitor(lambda buf, cap, n: load().nlpr_monitor(self.handle, buf, cap, n))

    # ---- reverse mode
    def grad_sizes(self) -> Tuple[int, int]:
        ck, gws = ctypes.c_size_t(), ctypes.c_size_t()
        _check(load().nlpr_grad_sizes(self.handle, ctypes.byref(ck), ctypes.byref(gws)))
        return ck.value, gws.value

    def forward(self, Yl, Yh, Z=None, ws=None, ck=None, stream=None):
        """Solve and keep the checkpoints the reverse pass needs; returns (Z, ws, ck)."""
        import torch
        ckb, _ = self.grad_sizes()
        if Z is None:
            Z = torch.empty(self.shape, dtype=torch.float32, device="cuda")
        if ws is None:
            ws = self.alloc_workspace()
        if ck is None:
            ck = torch.empty(max(ckb, 1), dtype=torch.uint8, device="cuda")
        _check(load().nlpr_forward(self.handle, _ptr(Yl), _ptr(Yh), _ptr(Z), _ptr(ws),
                                   ws.numel() * ws.element_size(), _ptr(ck),
                                   ck.numel() * ck.element_size(), _stream_handle(stream)))
        return Z, ws, ck

    def backward(self, Yl, Yh, dZ, ws, ck, gws=None, stream=None):
        """Gradients (dYl, dYh, dscal) of a loss with dloss/dZ = dZ; dscal is a device
        float64 tensor [dlambda_2, drho]."""
        import torch
        _, gwsb = self.grad_sizes()
        if gws is None:
            gws = torch.empty(max(gwsb, 1), dtype=torch.uint8, device="cuda")
        L, p, q = self.shape
        d = self.params.d
        dYl = torch.empty((L, p // d, q // d), dtype=torch.float32, device="cuda")
        dYh = torch.empty((self.params.Lh, p, q), dtype=torch.float32, device="cuda")
        dscal = torch.empty(2, dtype=torch.float64, device="cuda")
        _check(load().nlpr_backward(self.handle, _ptr(Yl), _ptr(Yh), _ptr(dZ.contiguous()),
                                    _ptr(ws), ws.numel() * ws.element_size(), _ptr(ck),
                                    ck.numel() * ck.element_size(), _ptr(gws),
                                    gws.numel() * gws.element_size(), _ptr(dYl), _ptr(dYh),
                                    _ptr(dscal), _stream_handle(stream)))
        return dYl, dYh, dscal


def _read_monitor(call) -> np.ndarray:
    n = ctypes.c_int32()
    _check(call(None, 0, ctypes.byref(n)))
    out = np.zeros((n.value, MON_RECORD), dtype=np.float64)
    if n.value:
        _check(call(out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n.value,
                    ctypes.byref(n)))
    return out


def _scene_kwargs(scene, flags: int = 0, **over):
    s = scene.spec
    kw = dict(p=s.p, q=s.q, L=s.L, Lh=scene.R.shape[1], d=s.d, blur=scene.blur, R=scene.R,
              K=s.K, Sw=s.Sw, iters=s.iters, lam=s.lam, rho=s.rho, h=scene.h, lam1=s.lam1,
              flags=flags)
    kw.update(over)
    return kw


class Batch:
    """Many independent scenes solved together: one launch per stage over all scenes."""

    def __init__(self, scenes_kwargs):
        lib = load()
        n = len(scenes_kwargs)
        self.params = (Params * n)()
        self.shapes = []
        self._keep = []
        blurs = (ctypes.c_void_p * n)()
        Rs = (ctypes.c_void_p * n)()
        Es = (ctypes.c_void_p * n)()
        for i, kw in enumerate(scenes_kwargs):
            blur = np.ascontiguousarray(kw["blur"], dtype=np.float32)
            R = np.ascontiguousarray(kw["R"], dtype=np.float32).reshape(kw["L"], kw["Lh"])
            r = blur.shape[0] // 2
            E = kw.get("E")
            Ls = 0
            if E is not None:
                E = np.ascontiguousarray(E, dtype=np.float32)
                Ls = E.shape[0]
                self._keep.append(E)
                Es[i] = E.ctypes.data
            self.params[i] = Params(kw["p"], kw["q"], kw["L"], kw["Lh"], kw["d"], r, kw["K"],
                                    kw["Sw"], kw["iters"], kw.get("flags", 0), Ls,
                                    kw.get("monitor_every", 0), kw["lam"], kw.get("lam1", 1.0),
                                    kw["rho"], kw["h"])
            self._keep += [blur, R]
            blurs[i] = blur.ctypes.data
            Rs[i] = R.ctypes.data
            self.shapes.append((kw["L"], kw["p"], kw["q"]))
        handle = ctypes.c_void_p()
        _check(lib.nlpr_batch_create(n, self.params, blurs, Rs, Es, ctypes.byref(handle)))
        self.handle = handle

    @classmethod
    def from_scenes(cls, scenes, flags: int = 0, **over) -> "Batch":
        return cls([_scene_kwargs(sc, flags, **over) for sc in scenes])

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            load().nlpr_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def workspace_bytes(self) -> int:
        n = ctypes.c_size_t()
        _check(load().nlpr_batch_workspace_size(self.handle, ctypes.byref(n)))
        return n.value

    def alloc_workspace(self):
        import torch
        return torch.empty(self.workspace_bytes, dtype=torch.uint8, device="cuda")

    def region(self, scene: int, which: int) -> Tuple[int, int]:
        off, nb = ctypes.c_size_t(), ctypes.c_size_t()
        _check(load().nlpr_batch_region(self.handle, scene, which, ctypes.byref(off),
                                        ctypes.byref(nb)))
        return off.value, nb.value

    def solve(self, Yls, Yhs, Zs=None, ws=None, stream=None):
        import torch
        n = len(self.shapes)
        if Zs is None:
            Zs = [torch.empty(sh, dtype=torch.float32, device="cuda") for sh in self.shapes]
        if ws is None:
            ws = self.alloc_workspace()
        arr = lambda ts: (ctypes.c_void_p * n)(*[_ptr(t) for t in ts])
        _check(load().nlpr_batch_solve(self.handle, arr(Yls), arr(Yhs), arr(Zs), _ptr(ws),
                                       ws.numel() * ws.element_size(), _stream_handle(stream)))
        return Zs, ws

    def stage_time(self, stage: int, reset: bool = False) -> Tuple[float, int]:
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(load().nlpr_batch_stage_time(self.handle, stage, ctypes.byref(ms),
                                            ctypes.byref(n), 1 if reset else 0))
        return ms.value, n.value

    def monitor(self, scene: int) -> np.ndarray:
        """Monitor records of one scene from the last batched solve, [n][8] float64."""
        return _read_monitor(
            lambda buf, cap, n: load().nlpr_batch_monitor(self.handle, scene, buf, cap, n))


def _autograd_function():
    import torch

    class NLPRFunction(torch.autograd.Function):
        """Z = X^(iters) of the unrolled ADMM as a differentiable function of
        (Y_l, Y_h, lambda_2, rho); the backward pass is the library's hand-written adjoint."""

        @staticmethod
        def forward(ctx, Yl, Yh, lam, rho, spec):
            kw = dict(spec)
            kw["lam"] = float(lam)
            kw["rho"] = float(rho)
            plan = Plan(**kw)
            Yl_c, Yh_c = Yl.detach().contiguous(), Yh.detach().contiguous()
            Z, ws, ck = plan.forward(Yl_c, Yh_c)
            ctx.state = (plan, Yl_c, Yh_c, ws, ck)
            ctx.scalar_meta = [(t.dtype, t.device) if isinstance(t, torch.Tensor) else None
                               for t in (lam, rho)]
            return Z

        @staticmethod
        def backward(ctx, dZ):
            plan, Yl, Yh, ws, ck = ctx.state
            dYl, dYh, dscal = plan.backward(Yl, Yh, dZ, ws, ck)
            ctx.state = None
            g = []
            for k, meta in enumerate(ctx.scalar_meta):   # in the dtype and place of lam / rho
                g.append(None if meta is None else dscal[k].to(dtype=meta[0], device=meta[1]))
            return dYl, dYh, g[0], g[1], None

    return NLPRFunction


_FN = None


def fuse_differentiable(Yl, Yh, lam, rho, blur, R, d: int, K: int, Sw: int, iters: int, h: float,
                        lam1: float = 1.0, flags: int = 0):
    """Z = X^(iters) from Y_l [L][p/d][q/d] and Y_h [Lh][p][q] (float32 device tensors) and
    the 0-dim tensors lam (lambda_2) and rho; differentiable in all four."""
    global _FN
    if _FN is None:
        _FN = _autograd_function()
    L, _, _ = Yl.shape
    Lh, p, q = Yh.shape
    spec = dict(p=p, q=q, L=L, Lh=Lh, d=d, blur=blur, R=R, K=K, Sw=Sw, iters=iters, h=h,
                lam1=lam1, flags=flags)
    return _FN.apply(Yl, Yh, lam, rho, spec)


def fuse(Yl, Yh, blur, R, d: int, lam: float, K: int, Sw: int, rho: float, iters: int, h: float,
         lam1: float = 1.0, flags: int = 0, stream=None):
    """Fuse Y_l [L][p/d][q/d] and Y_h [Lh][p][q] (float32 device tensors); returns Z [L][p][q]."""
    L, pd, qd = Yl.shape
    Lh, p, q = Yh.shape
    plan = Plan(p, q, L, Lh, d, blur, R, K, Sw, iters, lam, rho, h, lam1, flags)
    try:
        Z, _ = plan.solve(Yl.contiguous(), Yh.contiguous(), stream=stream)
    finally:
        plan.close()
    return Z


def solve(Yl, Yh, blur, d: int, R, lam: float, K: int, Sw: int, rho: float, iters: int, h: float,
          lam1: float = 1.0, stream=None):
    """The call of the problem statement: Z from Y_l, Y_h, the blur b, the decimation d,
    R, lambda_2, the patch and window radii, rho, the iteration count and the weight width
    h (same as ``fuse`` with the arguments in this order)."""
    return fuse(Yl, Yh, blur, R, d, lam, K, Sw, rho, iters, h, lam1=lam1, stream=stream)

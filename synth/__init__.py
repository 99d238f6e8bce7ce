"""Seeded synthetic multiband fusion scenes.

This module only draws inputs: a textured ground-truth cube Z, the operators of the
imaging model (blur taps b, spectral response R, decimation factor d) and the two noisy
observations Y_l = S(b * Z) + N_l and Y_h = Z R + N_h of the paper's imaging model
(Sec. "Variational models", eq. (1)).  It holds none of the fusion method's arithmetic:
no weights, no splitting, no ADMM.  Both the FP64 oracle and the GPU library consume the
same scene, with every array that enters the solver rounded once to float32.

Layout everywhere: planar band-major ``[bands][rows][cols]``.

Scene recipe (stands in for the paper's CAVE / Pavia / Chikusei / Pleiades data, which
are not available; no dataset content is reproduced):

* ``n_e`` abundance maps.  Each is a circular Gaussian random field (white N(0,1)
  filtered by a Gaussian of std ``corr/sqrt(2)`` pixels, then standardised) plus a
  texture term: one ``t x t`` uniform[0,1] tile per endmember, stamped into every
  ``t x t`` cell with its own random circular offset, which gives the repeated
  nonlocal structure the regulariser exploits.  ``a_e = max(0, g_e + tile_e - 0.5)``,
  then normalised so the abundances sum to 1 per pixel.
* Endmember spectra: three random Gaussian bumps over the band index (non-negative,
  smooth).
* ``Z = A M`` scaled to max 1.
* Blur: centred, normalised ``(2r+1)^2`` Gaussian, applied circularly.
* Noise: white Gaussian per band at a given SNR,
  ``sigma_c^2 = mean(signal_c^2) / 10^(SNR/10)``.
* Guide weight width ``h = sqrt(2 |P| L_h) * sigma_h`` with ``sigma_h`` the RMS noise
  std of the Y_h bands: two noisy copies of one clean patch then get weight ~ 1/e.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional

import numpy as np

__all__ = ["SceneSpec", "Scene", "CONFIGS", "make_scene", "config", "gaussian_blur_taps"]


@dataclasses.dataclass(frozen=True)
class SceneSpec:
    """Shape, operators and solver parameters of one synthetic workload."""

    name: str
    p: int
    q: int
    L: int
    d: int
    blur_radius: int
    blur_sigma: float
    R_kind: str  # "random1" | "bell1" | "gauss3" | "gauss4" | "random" (L x Lh nonneg, cols sum 1) | "identity"
    Lh: int
    snr_l: float
    snr_h: float
    n_end: int
    tile: int
    corr: float
    K: int
    Sw: int
    iters: int
    lam: float = 1e-3
    lam1: float = 1.0
    rho: float = 1e-2
    seed: int = 0

    @property
    def n_patch(self) -> int:
        return (2 * self.K + 1) ** 2

    def replace(self, **kw) -> "SceneSpec":
        return dataclasses.replace(self, **kw)


@dataclasses.dataclass
class Scene:
    spec: SceneSpec
    Z: np.ndarray          # [L][p][q] float64 ground truth (not a solver input)
    Yl: np.ndarray         # [L][p/d][q/d] float32
    Yh: np.ndarray         # [Lh][p][q] float32
    blur: np.ndarray       # [2r+1][2r+1] float32, centred
    R: np.ndarray          # [L][Lh] float32
    sigma_l: np.ndarray    # per-band noise std of Yl (float64)
    sigma_h: np.ndarray    # per-band noise std of Yh (float64)
    h: float               # guide weight width

    def params(self) -> Dict[str, float]:
        s = self.spec
        return dict(p=s.p, q=s.q, L=s.L, Lh=s.Lh, d=s.d, blur_radius=s.blur_radius, K=s.K,
                    Sw=s.Sw, iters=s.iters, lam=s.lam, lam1=s.lam1, rho=s.rho, h=self.h)


CONFIGS: Dict[str, SceneSpec] = {
    # 64x64x8 pansharpening: PAN guide, 7x7 blur sigma 1.7, d=4, patch 3x3, window 5x5, 50 iterations
    "c1": SceneSpec("c1", 64, 64, 8, 4, 3, 1.7, "random1", 1, 30.0, 30.0, 5, 16, 8.0,
                    K=1, Sw=2, iters=50, seed=1),
    # 512x512x100 HS+PAN: bell-shaped PAN response, 9x9 blur sigma 2.5, d=4, patch 5x5, window 11x11
    "c2": SceneSpec("c2", 512, 512, 100, 4, 4, 2.5, "bell1", 1, 35.0, 35.0, 12, 32, 8.0,
                    K=2, Sw=5, iters=100, seed=2),
    # 512x512x128 HS+MS: four overlapping Gaussian band responses, 30 dB, patch 5x5, window 11x11
    "c3": SceneSpec("c3", 512, 512, 128, 4, 4, 2.5, "gauss4", 4, 30.0, 30.0, 12, 32, 8.0,
                    K=2, Sw=5, iters=100, seed=3),
    # differentiated form: 256x256x31, 7x7 blur sigma 2, d=4, three overlapping Gaussian band
    # responses (3-band MS guide), 30 dB, patch 3x3, window 3x3, 20 unrolled iterations
    "c5": SceneSpec("c5", 256, 256, 31, 4, 3, 2.0, "gauss3", 3, 30.0, 30.0, 12, 32, 8.0,
                    K=1, Sw=1, iters=20, seed=5),
}


def config(name: str, **overrides) -> SceneSpec:
    return CONFIGS[name].replace(**overrides) if overrides else CONFIGS[name]


def gaussian_blur_taps(radius: int, sigma: float) -> np.ndarray:
    m = np.arange(-radius, radius + 1, dtype=np.float64)
    g = np.exp(-(m[:, None] ** 2 + m[None, :] ** 2) / (2.0 * sigma * sigma))
    return g / g.sum()


def _circ_filter_fft(img: np.ndarray, taps: np.ndarray) -> np.ndarray:
    """Circular convolution of the last two axes with a centred kernel (input generation)."""
    p, q = img.shape[-2:]
    r1, r2 = taps.shape[0] // 2, taps.shape[1] // 2
    grid = np.zeros((p, q))
    for a in range(-r1, r1 + 1):
        for b in range(-r2, r2 + 1):
            grid[a % p, b % q] += taps[a + r1, b + r2]
    return np.fft.irfft2(np.fft.rfft2(img) * np.fft.rfft2(grid), s=(p, q))


def _gaussian_field(rng, p, q, corr):
    w = rng.standard_normal((p, q))
    s = corr / math.sqrt(2.0)
    u = np.fft.fftfreq(p)[:, None]
    v = np.fft.fftfreq(q)[None, :]
    gain = np.exp(-2.0 * (math.pi * s) ** 2 * (u * u + v * v))
    f = np.fft.ifft2(np.fft.fft2(w) * gain).real
    f -= f.mean()
    sd = f.std()
    return f / (sd if sd > 0 else 1.0)


def _texture(rng, p, q, t):
    tile = rng.uniform(0.0, 1.0, size=(t, t))
    out = np.empty((p, q))
    for a in range(0, p, t):
        for b in range(0, q, t):
            o1, o2 = rng.integers(0, t, size=2)
            cell = np.roll(tile, shift=(int(o1), int(o2)), axis=(0, 1))
            out[a:a + t, b:b + t] = cell[: min(t, p - a), : min(t, q - b)]
    return out


def _spectra(rng, n_end, L):
    c = np.arange(L, dtype=np.float64)
    M = np.zeros((n_end, L))
    for e in range(n_end):
        for _ in range(3):
            centre = rng.uniform(0, L)
            width = rng.uniform(max(L / 20.0, 0.75), max(L / 4.0, 1.0))
            amp = rng.uniform(0.2, 1.0)
            M[e] += amp * np.exp(-((c - centre) ** 2) / (2 * width * width))
    return M


def _response(rng, kind, L, Lh):
    c = np.arange(L, dtype=np.float64)
    if kind == "random1":
        R = rng.uniform(0.0, 1.0, size=(L, 1))
    elif kind == "bell1":
        R = np.exp(-((c - L / 2.0) ** 2) / (2 * (L / 6.0) ** 2))[:, None]
    elif kind == "gauss4":
        R = np.stack([np.exp(-((c - (2 * j + 1) * L / 8.0) ** 2) / (2 * (L / 8.0) ** 2))
                      for j in range(4)], axis=1)
    elif kind == "gauss3":
        R = np.stack([np.exp(-((c - (2 * j + 1) * L / 6.0) ** 2) / (2 * (L / 6.0) ** 2))
                      for j in range(3)], axis=1)
    elif kind == "random":
        R = rng.uniform(0.0, 1.0, size=(L, Lh))
    elif kind == "identity":
        return np.eye(L)
    else:
        raise ValueError(kind)
    return R / R.sum(axis=0, keepdims=True)


def _noise_std(signal: np.ndarray, snr_db: float) -> np.ndarray:
    power = np.mean(signal.reshape(signal.shape[0], -1) ** 2, axis=1)
    return np.sqrt(power / 10.0 ** (snr_db / 10.0))


def make_scene(spec: SceneSpec, seed: Optional[int] = None) -> Scene:
    """Draw a scene.  Deterministic in (spec, seed); ``seed`` defaults to ``spec.seed``."""
    s = spec
    if s.p % s.d or s.q % s.d:
        raise ValueError("decimation factor must divide both image sides")
    rng = np.random.default_rng(s.seed if seed is None else seed)
    A = np.empty((s.n_end, s.p, s.q))
    for e in range(s.n_end):
        g = _gaussian_field(rng, s.p, s.q, s.corr)
        A[e] = np.maximum(0.0, g + (_texture(rng, s.p, s.q, s.tile) - 0.5))
    tot = A.sum(axis=0)
    A = np.where(tot > 0, A / np.where(tot > 0, tot, 1.0), 1.0 / s.n_end)
    M = _spectra(rng, s.n_end, s.L)
    Z = np.tensordot(M.T, A, axes=(1, 0))            # [L][p][q]
    Z /= Z.max()
    taps = gaussian_blur_taps(s.blur_radius, s.blur_sigma).astype(np.float32)
    R = _response(rng, s.R_kind, s.L, s.Lh).astype(np.float32)
    Lh = R.shape[1]
    blurred = _circ_filter_fft(Z, taps.astype(np.float64))
    low = blurred[:, ::s.d, ::s.d]
    high = np.tensordot(R.astype(np.float64).T, Z, axes=(1, 0))   # [Lh][p][q]
    sl = _noise_std(low, s.snr_l)
    sh = _noise_std(high, s.snr_h)
    Yl = low + sl[:, None, None] * rng.standard_normal(low.shape)
    Yh = high + sh[:, None, None] * rng.standard_normal(high.shape)
    sigma_h = float(np.sqrt(np.mean(sh ** 2)))
    h = math.sqrt(2.0 * s.n_patch * Lh) * sigma_h
    return Scene(spec=s if Lh == s.Lh else s.replace(Lh=Lh), Z=Z,
                 Yl=np.ascontiguousarray(Yl, dtype=np.float32),
                 Yh=np.ascontiguousarray(Yh, dtype=np.float32),
                 blur=taps, R=np.ascontiguousarray(R), sigma_l=sl, sigma_h=sh, h=h)


def small_spec(p=64, q=64, L=8, Lh=1, d=4, blur_radius=3, K=1, Sw=2, iters=20, seed=7,
               R_kind=None, **kw) -> SceneSpec:
    """A small scene for parity tests (same generator, arbitrary shape)."""
    if R_kind is None:
        R_kind = "random1" if Lh == 1 else "random"
    return SceneSpec(name=f"s{p}x{q}x{L}", p=p, q=q, L=L, d=d, blur_radius=blur_radius,
                     blur_sigma=kw.pop("blur_sigma", 1.7), R_kind=R_kind, Lh=Lh,
                     snr_l=kw.pop("snr_l", 30.0), snr_h=kw.pop("snr_h", 30.0),
                     n_end=kw.pop("n_end", 5), tile=kw.pop("tile", 16), corr=kw.pop("corr", 8.0),
                     K=K, Sw=Sw, iters=iters, seed=seed, **kw)


def batch_specs(n: int = 48, seed: int = 1000, iters: int = 100):
    """The multi-scene workload: ``n`` independent scenes with sizes drawn from
    {128, 192, 256, 384, 512}^2, band counts from {4, 8, 31, 64, 128}, decimation 4 or 8
    and a PAN (1 band) or 4-band MS guide, 30 dB noise, patch 3x3 and window 3x3.  The blur
    is 9x9 with sigma 2.5 for d = 4 and 17x17 with sigma 5 for d = 8.  Scene s is drawn
    with seed ``seed + s``."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n):
        side = int(rng.choice([128, 192, 256, 384, 512]))
        L = int(rng.choice([4, 8, 31, 64, 128]))
        d = int(rng.choice([4, 8]))
        pan = bool(rng.integers(0, 2))
        Lh = 1 if pan else 4
        kind = "bell1" if pan else ("gauss4" if L >= 8 else "random")
        r, sig = (4, 2.5) if d == 4 else (8, 5.0)
        out.append(SceneSpec(name=f"b{s}", p=side, q=side, L=L, d=d, blur_radius=r,
                             blur_sigma=sig, R_kind=kind, Lh=Lh, snr_l=30.0, snr_h=30.0,
                             n_end=8, tile=16, corr=8.0, K=1, Sw=1, iters=iters,
                             seed=seed + s))
    return out

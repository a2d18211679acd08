"""Seeded synthetic image pairs for the optical-flow workloads.

This module draws and evaluates test images only; it holds none of the
method's arithmetic (no gradients, no finite elements, no solver).  Both the
GPU path's tests/benchmarks and the FP64 CPU oracle's tests take their inputs
from here, so both sides see bit-identical frames.

Conventions (paper, Section 1, brightness constancy with the Gennert-
Negahdaripour illumination law, M = 1 + dm and a negligible translator T):
  * node (x, y) is the centre of pixel (x, y); x is the column, y the row;
    arrays are indexed ``[y, x]`` and stored row-major in float64;
  * the second frame is ``I1(x) = m(x) * I0(x - w(x))``, evaluated analytically
    from the closed-form bump sum, so no interpolation enters the inputs;
  * ground truth is the flow ``w`` and the gain ``m``; to first order the
    illumination unknown of the model is ``m - 1``.

Workload recipes (sizes and distributions of the paper's experiments, which
used real sequences that are not available here):
  * ``plain64``  : 64x64, 40 Gaussian bumps (sigma U[3,8], amplitude
    U[0.2,1]), affine flow ``t + J (x - xc)`` rescaled to max |w| <= 1.5,
    gain ``1 + 0.1 b/max|b|`` with b four signed bumps of scale W/4.
  * ``plain640`` : 640x480, 200 bumps, flow ``(R(2 deg) - I)(x - xc) + t`` with
    |t| <= 3, gain ``1 + 0.15 b/max|b|``, i.i.d. N(0, 0.01^2) noise added to
    both frames after warping.
  * ``linear``   : ``I0 = 0.5 + p x + q y``, uniform translation, used by the
    exact-recovery pins.
  * ``batch1080``: 1920x1080 (one pair of a batch, seed per pair), the
    ``plain640`` bump density (about 1350 bumps, each cut off beyond 6 sigma),
    flow piecewise affine over the Voronoi cells of 6 random centres (each
    cell ``t + J (x - c)``, rescaled to max |w| <= 6 over the image), gain
    ``1 + 0.15 b/max|b|``.
  * ``prec4k``   : 4096x2160 band-limited texture ``0.5 + sum_k c cos(2 pi
    omega_k . x + phi_k)`` of 512 plane waves, |omega_k| in [1/64, 1/8]
    cycles/px, c = 0.15 sqrt(2/512) (standard deviation 0.15); smooth flow of
    4 low-frequency sinusoids (wavelengths >= 512 px) scaled to max |w| <= 8;
    ``I1 = g I0(x - w) + o`` with a gain g in 1 +- 0.2 and an offset o in
    +- 0.2 mean(I0) (the offset breaks the model's negligible-translator
    assumption on purpose).  Any window of it can be evaluated on its own.
  * ``adj1024``  : 1024x1024, about 683 bumps (cut off beyond 6 sigma), a
    known affine flow rescaled to max |w| <= 2, gain ``1 + 0.1 b/max|b|``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Bumps:
    """A sum of isotropic Gaussian bumps ``sum_k a_k exp(-|x-c_k|^2 / (2 s_k^2))``."""

    cx: np.ndarray
    cy: np.ndarray
    s: np.ndarray
    a: np.ndarray
    base: float = 0.0

    def __call__(self, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
        out = np.full(np.broadcast(X, Y).shape, self.base, dtype=np.float64)
        for cx, cy, s, a in zip(self.cx, self.cy, self.s, self.a):
            out += a * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * s * s))
        return out


def random_bumps(rng: np.random.Generator, W: int, H: int, n: int,
                 s_range=(3.0, 8.0), a_range=(0.2, 1.0), signed=False) -> Bumps:
    cx = rng.uniform(0.0, W - 1.0, n)
    cy = rng.uniform(0.0, H - 1.0, n)
    s = rng.uniform(s_range[0], s_range[1], n)
    a = rng.uniform(a_range[0], a_range[1], n)
    if signed:
        a = a * rng.choice([-1.0, 1.0], n)
    return Bumps(cx, cy, s, a)


@dataclasses.dataclass
class Pair:
    """One synthetic frame pair with its ground truth."""

    I0: np.ndarray        # [H, W] float64
    I1: np.ndarray        # [H, W] float64
    w: np.ndarray         # [2, H, W] ground-truth flow (w1 = x-displacement)
    gain: np.ndarray      # [H, W] multiplicative illumination m(x)
    name: str = ""

    @property
    def shape(self):
        return self.I0.shape


def _grid(W: int, H: int):
    X, Y = np.meshgrid(np.arange(W, dtype=np.float64),
                       np.arange(H, dtype=np.float64))
    return X, Y


def _gain_field(rng, W, H, X, Y, amp):
    b = random_bumps(rng, W, H, 4, s_range=(W / 4.0, W / 4.0),
                     a_range=(0.5, 1.0), signed=True)
    bv = b(X, Y)
    return 1.0 + amp * bv / np.max(np.abs(bv))


def _bump_sum_local(b: Bumps, X: np.ndarray, Y: np.ndarray, DX=None, DY=None, pad: float = 0.0) -> np.ndarray:
    """``b`` at the points (X - DX, Y - DY) of a pixel grid, each bump summed
    only where that point lies within 6 of its sigmas (the same cut for every
    frame); ``pad`` bounds |(DX, DY)|, so a window of the grid around each
    centre holds every such point."""
    H, W = X.shape
    out = np.full((H, W), b.base, dtype=np.float64)
    x0, y0 = X[0, 0], Y[0, 0]
    for cx, cy, sg, a in zip(b.cx, b.cy, b.s, b.a):
        r = 6.0 * sg
        i0 = max(0, int(math.floor(cy - r - pad - y0)))
        i1 = min(H, int(math.ceil(cy + r + pad - y0)) + 1)
        j0 = max(0, int(math.floor(cx - r - pad - x0)))
        j1 = min(W, int(math.ceil(cx + r + pad - x0)) + 1)
        if i0 >= i1 or j0 >= j1:
            continue
        px = X[i0:i1, j0:j1] - (0.0 if DX is None else DX[i0:i1, j0:j1]) - cx
        py = Y[i0:i1, j0:j1] - (0.0 if DY is None else DY[i0:i1, j0:j1]) - cy
        d2 = px * px + py * py
        v = a * np.exp(-d2 / (2.0 * sg * sg))
        out[i0:i1, j0:j1] += np.where(d2 <= r * r, v, 0.0)
    return out


def _voronoi_affine_flow(rng, W, H, X, Y, ncell=6, wmax=6.0):
    cx = rng.uniform(0.0, W - 1.0, ncell)
    cy = rng.uniform(0.0, H - 1.0, ncell)
    t = rng.uniform(-1.0, 1.0, (ncell, 2))
    J = rng.uniform(-0.01, 0.01, (ncell, 2, 2))
    d2 = np.stack([(X - cx[k]) ** 2 + (Y - cy[k]) ** 2 for k in range(ncell)])
    cell = np.argmin(d2, axis=0)
    w1 = np.zeros_like(X)
    w2 = np.zeros_like(X)
    for k in range(ncell):
        mk = cell == k
        w1[mk] = t[k, 0] + J[k, 0, 0] * (X[mk] - cx[k]) + J[k, 0, 1] * (Y[mk] - cy[k])
        w2[mk] = t[k, 1] + J[k, 1, 0] * (X[mk] - cx[k]) + J[k, 1, 1] * (Y[mk] - cy[k])
    mx = float(np.max(np.hypot(w1, w2)))
    if mx > 0.0:
        w1 *= wmax / mx
        w2 *= wmax / mx
    return w1, w2


def make_pair_4k(seed: int, x0: int = 0, y0: int = 0, W: int | None = None, H: int | None = None,
                 device=None) -> Pair:
    """The ``prec4k`` pair of ``seed`` on the window [x0, x0 + W) x [y0, y0 + H)
    of its 4096x2160 image (default: all of it); ``device`` evaluates the
    plane waves with torch there (a CUDA device for the full image), else on
    the host in float64 numpy."""
    FW, FH = 4096, 2160
    W = FW - x0 if W is None else W
    H = FH - y0 if H is None else H
    rng = np.random.default_rng(seed)
    nk = 512
    rad = rng.uniform(1.0 / 64.0, 1.0 / 8.0, nk)
    ang = rng.uniform(0.0, 2.0 * math.pi, nk)
    om = np.stack([rad * np.cos(ang), rad * np.sin(ang)], 1)          # cycles per pixel
    ph = rng.uniform(0.0, 2.0 * math.pi, nk)
    c = 0.15 * math.sqrt(2.0 / nk)
    # smooth flow: 4 sinusoids of wavelength >= 512 px per component
    fw = rng.uniform(1.0 / 2048.0, 1.0 / 512.0, (2, 4, 2)) * rng.choice([-1.0, 1.0], (2, 4, 2))
    fp = rng.uniform(0.0, 2.0 * math.pi, (2, 4))
    fa = rng.uniform(0.5, 1.0, (2, 4))
    # gain and offset: 3 sinusoids of wavelength >= 1024 px each
    gw = rng.uniform(1.0 / 4096.0, 1.0 / 1024.0, (2, 3, 2))
    gp = rng.uniform(0.0, 2.0 * math.pi, (2, 3))
    X, Y = _grid(W, H)
    X += x0
    Y += y0

    def smooth(freqs, phases, amps, XX, YY):
        v = np.zeros_like(XX)
        for k in range(len(phases)):
            v += amps[k] * np.sin(2.0 * math.pi * (freqs[k, 0] * XX + freqs[k, 1] * YY) + phases[k])
        return v

    # maxima over the whole image from a coarse grid of it (so that every window
    # uses the same scale factors)
    Xc, Yc = np.meshgrid(np.linspace(0.0, FW - 1.0, 257), np.linspace(0.0, FH - 1.0, 136))
    wc = np.hypot(smooth(fw[0], fp[0], fa[0], Xc, Yc), smooth(fw[1], fp[1], fa[1], Xc, Yc))
    ws = 8.0 / float(np.max(wc))
    gc = smooth(gw[0], gp[0], np.ones(3), Xc, Yc)
    oc = smooth(gw[1], gp[1], np.ones(3), Xc, Yc)
    w1 = ws * smooth(fw[0], fp[0], fa[0], X, Y)
    w2 = ws * smooth(fw[1], fp[1], fa[1], X, Y)
    gain = 1.0 + 0.2 * smooth(gw[0], gp[0], np.ones(3), X, Y) / float(np.max(np.abs(gc)))
    off = 0.2 * 0.5 * smooth(gw[1], gp[1], np.ones(3), X, Y) / float(np.max(np.abs(oc)))

    def texture(XX, YY):
        if device is not None:
            import torch
            tX = torch.as_tensor(XX, dtype=torch.float64, device=device)
            tY = torch.as_tensor(YY, dtype=torch.float64, device=device)
            acc = torch.full_like(tX, 0.5)
            for k in range(nk):
                acc += c * torch.cos(2.0 * math.pi * (float(om[k, 0]) * tX + float(om[k, 1]) * tY) + float(ph[k]))
            return acc.cpu().numpy()
        acc = np.full_like(XX, 0.5)
        for k in range(nk):
            acc += c * np.cos(2.0 * math.pi * (om[k, 0] * XX + om[k, 1] * YY) + ph[k])
        return acc

    I0 = texture(X, Y)
    I1 = gain * texture(X - w1, Y - w2) + off
    return Pair(np.ascontiguousarray(I0), np.ascontiguousarray(I1), np.stack([w1, w2]), gain,
                name=f"prec4k:{seed}:{x0},{y0}:{W}x{H}")


def make_pair(kind: str, seed: int, W: int | None = None, H: int | None = None,
              noise: float | None = None) -> Pair:
    """Draw one pair of the named recipe; ``W``/``H`` override the size."""
    rng = np.random.default_rng(seed)
    if kind == "plain64":
        W = W or 64
        H = H or 64
        nb = max(1, round(40 * W * H / (64 * 64)))
        X, Y = _grid(W, H)
        img = random_bumps(rng, W, H, nb)
        t = rng.uniform(-1.0, 1.0, 2)
        J = rng.uniform(-0.02, 0.02, (2, 2))
        xc, yc = (W - 1) / 2.0, (H - 1) / 2.0
        w1 = t[0] + J[0, 0] * (X - xc) + J[0, 1] * (Y - yc)
        w2 = t[1] + J[1, 0] * (X - xc) + J[1, 1] * (Y - yc)
        mx = np.max(np.hypot(w1, w2))
        if mx > 1.5:
            w1 *= 1.5 / mx
            w2 *= 1.5 / mx
        gain = _gain_field(rng, W, H, X, Y, 0.1)
        I0 = img(X, Y)
        I1 = gain * img(X - w1, Y - w2)
        sig = 0.0 if noise is None else noise
    elif kind == "plain640":
        W = W or 640
        H = H or 480
        nb = max(1, round(200 * W * H / (640 * 480)))
        X, Y = _grid(W, H)
        img = random_bumps(rng, W, H, nb)
        th = math.radians(2.0)
        R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
        D = R - np.eye(2)
        r_t = 3.0 * math.sqrt(rng.uniform())
        phi = rng.uniform(0.0, 2.0 * math.pi)
        t = np.array([r_t * math.cos(phi), r_t * math.sin(phi)])
        xc, yc = (W - 1) / 2.0, (H - 1) / 2.0
        w1 = D[0, 0] * (X - xc) + D[0, 1] * (Y - yc) + t[0]
        w2 = D[1, 0] * (X - xc) + D[1, 1] * (Y - yc) + t[1]
        gain = _gain_field(rng, W, H, X, Y, 0.15)
        I0 = img(X, Y)
        I1 = gain * img(X - w1, Y - w2)
        sig = 0.01 if noise is None else noise
    elif kind == "batch1080":
        W = W or 1920
        H = H or 1080
        nb = max(1, round(200 * W * H / (640 * 480)))
        X, Y = _grid(W, H)
        img = random_bumps(rng, W, H, nb)
        w1, w2 = _voronoi_affine_flow(rng, W, H, X, Y, 6, 6.0)
        gain = _gain_field(rng, W, H, X, Y, 0.15)
        I0 = _bump_sum_local(img, X, Y)
        I1 = gain * _bump_sum_local(img, X, Y, w1, w2, pad=6.0)
        sig = 0.0 if noise is None else noise
    elif kind == "adj1024":
        W = W or 1024
        H = H or 1024
        nb = max(1, round(200 * W * H / (640 * 480)))
        X, Y = _grid(W, H)
        img = random_bumps(rng, W, H, nb)
        t = rng.uniform(-1.0, 1.0, 2)
        J = rng.uniform(-0.004, 0.004, (2, 2))
        xc, yc = (W - 1) / 2.0, (H - 1) / 2.0
        w1 = t[0] + J[0, 0] * (X - xc) + J[0, 1] * (Y - yc)
        w2 = t[1] + J[1, 0] * (X - xc) + J[1, 1] * (Y - yc)
        mx = np.max(np.hypot(w1, w2))
        w1 *= 2.0 / mx
        w2 *= 2.0 / mx
        gain = _gain_field(rng, W, H, X, Y, 0.1)
        I0 = _bump_sum_local(img, X, Y)
        I1 = gain * _bump_sum_local(img, X, Y, w1, w2, pad=2.0)
        sig = 0.0 if noise is None else noise
    else:
        raise ValueError(f"unknown pair kind {kind!r}")
    if sig > 0.0:
        I0 = I0 + rng.normal(0.0, sig, I0.shape)
        I1 = I1 + rng.normal(0.0, sig, I1.shape)
    return Pair(np.ascontiguousarray(I0), np.ascontiguousarray(I1),
                np.stack([w1, w2]), gain, name=f"{kind}:{seed}:{W}x{H}")


def linear_pair(W: int, H: int, p: float, q: float, w=(0.3, -0.2)) -> Pair:
    """``I0 = 0.5 + p x + q y`` translated by the constant ``w``."""
    X, Y = _grid(W, H)
    I0 = 0.5 + p * X + q * Y
    I1 = 0.5 + p * (X - w[0]) + q * (Y - w[1])
    wf = np.stack([np.full_like(X, w[0]), np.full_like(X, w[1])])
    return Pair(I0, I1, wf, np.ones_like(X), name=f"linear:{W}x{H}")


def gain_pair(W: int, H: int, c: float, seed: int = 7) -> Pair:
    """Textured ``I0`` and ``I1 = (1 + c) I0``: pure illumination change, no motion."""
    rng = np.random.default_rng(seed)
    X, Y = _grid(W, H)
    img = random_bumps(rng, W, H, max(4, W * H // 100))
    I0 = 0.2 + img(X, Y)
    I1 = (1.0 + c) * I0
    return Pair(I0, I1, np.zeros((2, H, W)), np.full_like(X, 1.0 + c),
                name=f"gain:{W}x{H}")


def constant_alpha(W: int, H: int, alpha: float = 0.1, batch: int | None = None) -> np.ndarray:
    """Per-element regularisation array ``[H-1, W-1, 2]`` (``[B, ...]`` if batched)."""
    a = np.full((H - 1, W - 1, 2), alpha, dtype=np.float64)
    if batch is not None:
        a = np.broadcast_to(a, (batch,) + a.shape).copy()
    return a


def random_alpha(W: int, H: int, seed: int, lo=0.02, hi=0.2) -> np.ndarray:
    """Piecewise-constant α drawn per element (log-uniform in [lo, hi])."""
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(math.log(lo), math.log(hi), (H - 1, W - 1, 2)))

"""Seeded synthetic inputs shaped like the paper's workloads.

This module draws numbers and nothing else: it holds none of the SSA
arithmetic (no embedding, no shapes, no SVD, no averaging).  Both the
oracle-side tests and the GPU path take their inputs from here, so the two
sides always see the same bytes.

Every generator uses numpy's PCG64 with an explicit seed.  Image axes follow
the 2D-SSA section of the paper: x is the row index (first array axis), y the
column index; arrays are C row-major, so y is the fast axis in memory.
Time and pixel indices start at 1 for series (t = 1..N) and at 0 for images
(m, n = 0..N-1).

A workload is returned as a plain dict:

    kind      "1d" | "2d" | "shaped" | "mssa"
    x         float64 array; NaN marks a missing value
              (1d: shape (N,); 2d/shaped: (Nx, Ny); mssa: list of 1-D arrays)
    mask      uint8 (Nx, Ny) or None          (shaped only)
    wmask     uint8 (Lx, Ly) or None          (window shape; None = full box)
    window    (Lx, Ly) for images, L for series
    r         number of eigentriples
    groups    list of lists of 0-based component ids
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "series_1d", "image_2d", "shaped_disc", "mssa_series", "mars_like",
    "serving_mix", "small_shaped", "config",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def series_1d(n: int = 1000, L: int = 500, r: int = 10, seed: int = 1,
              noise: float = 0.1) -> dict:
    """x_t = 2 sin(2 pi t/12) + sin(2 pi t/33) + 0.01 t + N(0, noise^2), t = 1..n."""
    g = _rng(seed)
    t = np.arange(1, n + 1, dtype=np.float64)
    x = (2.0 * np.sin(2 * np.pi * t / 12) + np.sin(2 * np.pi * t / 33)
         + 0.01 * t + g.normal(0.0, noise, n))
    return dict(kind="1d", x=x, mask=None, wmask=None, window=L, r=r,
                groups=[[0, 1], [2, 3], [4]])


def image_2d(n: int = 512, lw: int = 64, r: int = 30, seed: int = 2,
             noise: float = 0.2, waves: int = 3) -> dict:
    """Sum of planar cosines cos(2 pi (m cos th + n sin th)/T + phi) plus noise.

    T ~ U(8, 64) px, th ~ U(0, pi), phi ~ U(0, 2 pi); one draw per wave.
    """
    g = _rng(seed)
    T = g.uniform(8.0, 64.0, waves)
    th = g.uniform(0.0, np.pi, waves)
    ph = g.uniform(0.0, 2 * np.pi, waves)
    m = np.arange(n, dtype=np.float64)[:, None]
    k = np.arange(n, dtype=np.float64)[None, :]
    x = np.zeros((n, n))
    for i in range(waves):
        x += np.cos(2 * np.pi * (m * np.cos(th[i]) + k * np.sin(th[i])) / T[i] + ph[i])
    x += g.normal(0.0, noise, (n, n))
    return dict(kind="2d", x=x, mask=None, wmask=None, window=(lw, lw), r=r,
                groups=[[0, 1], [2, 3], [4, 5]])


def _disc(n: int, radius: float) -> np.ndarray:
    c = (n - 1) / 2.0
    i = np.arange(n, dtype=np.float64)
    return ((i[:, None] - c) ** 2 + (i[None, :] - c) ** 2) <= radius ** 2


def shaped_disc(n: int = 1024, radius: float = 480.0, lw: int = 32, r: int = 50,
                seed: int = 4, hole_frac: float = 0.10, noise: float = 0.1,
                hole_r: tuple = (2, 10)) -> dict:
    """Separable cosine texture on a disc mask with round NaN holes.

    Mask: pixels with distance <= radius from the centre ((n-1)/2, (n-1)/2).
    Holes: circles of integer radius ~ U{hole_r}, centres uniform in the disc,
    added until hole_frac of the disc pixels are NaN.
    Image: cos(2 pi m/Tx + px) * cos(2 pi n/Ty + py), T ~ U(8, 64), + N(0, noise^2).
    """
    g = _rng(seed)
    Tx, Ty = g.uniform(8.0, 64.0, 2)
    px, py = g.uniform(0.0, 2 * np.pi, 2)
    m = np.arange(n, dtype=np.float64)
    x = np.cos(2 * np.pi * m / Tx + px)[:, None] * np.cos(2 * np.pi * m / Ty + py)[None, :]
    x = x + g.normal(0.0, noise, (n, n))
    disc = _disc(n, radius)
    ndisc = int(disc.sum())
    holes = np.zeros((n, n), dtype=bool)
    c = (n - 1) / 2.0
    ii = np.arange(n)[:, None]
    jj = np.arange(n)[None, :]
    while (holes & disc).sum() < hole_frac * ndisc:
        rad = int(g.integers(hole_r[0], hole_r[1] + 1))
        # uniform point in the disc by rejection
        while True:
            cx, cy = g.uniform(c - radius, c + radius, 2)
            if (cx - c) ** 2 + (cy - c) ** 2 <= radius ** 2:
                break
        lo0, hi0 = max(0, int(cx) - rad - 1), min(n, int(cx) + rad + 2)
        lo1, hi1 = max(0, int(cy) - rad - 1), min(n, int(cy) + rad + 2)
        sub = ((ii[lo0:hi0] - cx) ** 2 + (jj[:, lo1:hi1] - cy) ** 2) <= rad * rad
        holes[lo0:hi0, lo1:hi1] |= sub
    x[holes] = np.nan
    x[~disc] = 0.0
    return dict(kind="shaped", x=x, mask=disc.astype(np.uint8), wmask=None,
                window=(lw, lw), r=r, groups=[[0, 1, 2, 3]])


def mssa_series(s: int = 50, nmin: int = 1000, nmax: int = 3000, L: int = 500,
                r: int = 20, seed: int = 3, phi: float = 0.5, sigma: float = 0.3) -> dict:
    """s series of uneven length N_p ~ U{nmin..nmax}.

    x_p(t) = a_p sin(2 pi t/10) + b_p sin(2 pi t/37) + e_p(t), a, b ~ U(0.5, 2),
    e_p an AR(1) process e_t = phi e_{t-1} + eps_t, eps ~ N(0, sigma^2),
    started from its stationary law.
    """
    g = _rng(seed)
    lens = g.integers(nmin, nmax + 1, s)
    a = g.uniform(0.5, 2.0, s)
    b = g.uniform(0.5, 2.0, s)
    out = []
    for p in range(s):
        n = int(lens[p])
        t = np.arange(1, n + 1, dtype=np.float64)
        eps = g.normal(0.0, sigma, n)
        e = np.empty(n)
        e[0] = eps[0] / np.sqrt(1.0 - phi * phi)
        for i in range(1, n):
            e[i] = phi * e[i - 1] + eps[i]
        out.append(a[p] * np.sin(2 * np.pi * t / 10) + b[p] * np.sin(2 * np.pi * t / 37) + e)
    return dict(kind="mssa", x=out, mask=None, wmask=None, window=L, r=r,
                groups=[[0, 1], [2, 3]])


def circle_wmask(R: int) -> np.ndarray:
    """Pixels (i, j) of a (2R+1)^2 box with (i-R)^2 + (j-R)^2 <= R^2."""
    i = np.arange(2 * R + 1)
    return (((i[:, None] - R) ** 2 + (i[None, :] - R) ** 2) <= R * R).astype(np.uint8)


def mars_like(seed: int = 7, nx: int = 258, ny: int = 275, R: int = 15) -> dict:
    """A 258x275 8-bit-like image: a bright disc on a zero background.

    Zero pixels are missing (NaN); a mask excludes saturated pixels (255).
    The disc carries two planar sines with periods near 5 and 10 px.
    """
    g = _rng(seed)
    m = np.arange(nx, dtype=np.float64)[:, None]
    k = np.arange(ny, dtype=np.float64)[None, :]
    cx, cy, rad = nx / 2.0, ny / 2.0, 0.42 * min(nx, ny)
    disc = ((m - cx) ** 2 + (k - cy) ** 2) <= rad * rad
    body = 140.0 + 60.0 * np.cos(np.pi * np.sqrt((m - cx) ** 2 + (k - cy) ** 2) / (2 * rad))
    tex = (12.0 * np.cos(2 * np.pi * (m / 5.0 + k / 10.0) + g.uniform(0, 2 * np.pi))
           + 8.0 * np.cos(2 * np.pi * (m / 10.0 - k / 5.0) + g.uniform(0, 2 * np.pi)))
    img = np.clip(np.round(body + tex + g.normal(0.0, 4.0, (nx, ny))), 1, 255)
    img = np.where(disc, img, 0.0)
    mask = (img != 255).astype(np.uint8)
    x = np.where(img == 0, np.nan, img)
    return dict(kind="shaped", x=x, mask=mask, wmask=circle_wmask(R), window=(2 * R + 1, 2 * R + 1),
                r=50, groups=[[0]])


def small_shaped(nx: int = 40, ny: int = 33, seed: int = 11, lx: int = 6, ly: int = 5,
                 r: int = 8, holes: int = 3) -> dict:
    """A small shaped case: ellipse mask, a few NaN holes and an irregular window."""
    g = _rng(seed)
    m = np.arange(nx, dtype=np.float64)[:, None]
    k = np.arange(ny, dtype=np.float64)[None, :]
    x = (np.cos(2 * np.pi * (m / 9.0 + k / 13.0) + 0.3)
         + 0.5 * np.cos(2 * np.pi * m / 7.0) * np.cos(2 * np.pi * k / 5.0)
         + g.normal(0.0, 0.2, (nx, ny)))
    mask = ((((m - nx / 2) / (0.48 * nx)) ** 2 + ((k - ny / 2) / (0.48 * ny)) ** 2) <= 1.0)
    for _ in range(holes):
        ci, cj = g.integers(0, nx), g.integers(0, ny)
        x[max(0, ci - 1):ci + 2, max(0, cj - 1):cj + 2] = np.nan
    wm = g.random((lx, ly)) < 0.75
    wm[0, :] = True          # keep the bounding box tight
    wm[:, 0] = True
    wm[-1, -1] = True
    return dict(kind="shaped", x=x, mask=mask.astype(np.uint8), wmask=wm.astype(np.uint8),
                window=(lx, ly), r=r, groups=[[0, 1], [2, 3, 4]])


def serving_mix(n_requests: int = 10000, seed: int = 5, max_1d: int = 20000,
                max_side: int = 512) -> list:
    """Request descriptors of the mixed serving workload.

    60% 1D series (N ~ U{500..max_1d}, L = N//2), 25% MSSA systems of
    4..32 series shaped like the batched MSSA workload, 15% square images of
    side S ~ U{64..max_side} with an (S//8)^2 window.  r ~ U{5..40}, clipped
    below min(L, K).  Each descriptor carries its own seed; call
    ``materialize`` to draw its data.
    """
    g = _rng(seed)
    out = []
    for i in range(n_requests):
        u = g.random()
        r = int(g.integers(5, 41))
        if u < 0.60:
            n = int(g.integers(500, max_1d + 1))
            out.append(dict(kind="1d", n=n, L=n // 2, r=r, seed=100000 + i))
        elif u < 0.85:
            s = int(g.integers(4, 33))
            out.append(dict(kind="mssa", s=s, L=500, r=r, seed=100000 + i))
        else:
            side = int(g.integers(64, max_side + 1))
            out.append(dict(kind="2d", n=side, lw=side // 8, r=r, seed=100000 + i))
    return out


def materialize(desc: dict) -> dict:
    """Draw the data of one serving-mix request descriptor."""
    if desc["kind"] == "1d":
        w = series_1d(n=desc["n"], L=desc["L"], r=desc["r"], seed=desc["seed"])
    elif desc["kind"] == "mssa":
        w = mssa_series(s=desc["s"], L=desc["L"], r=desc["r"], seed=desc["seed"])
    else:
        w = image_2d(n=desc["n"], lw=desc["lw"], r=desc["r"], seed=desc["seed"])
    w["groups"] = [list(range(min(desc["r"], 4)))]
    return w


def config(i: int, scale: str = "full") -> dict:
    """The five benchmark workloads (1-based), at full or reduced size.

    Reduced sizes keep each workload's structure but let the oracle finish in
    seconds: 2D 128^2 image with a 16^2 window, shaped 160^2 disc with an 8^2
    window, MSSA with 8 series of 300..600 points and L = 100.
    """
    if i == 1:
        return series_1d()
    if i == 2:
        return image_2d() if scale == "full" else image_2d(n=128, lw=16, r=30)
    if i == 3:
        return mssa_series() if scale == "full" else mssa_series(s=8, nmin=300, nmax=600, L=100, r=20)
    if i == 4:
        return (shaped_disc() if scale == "full"
                else shaped_disc(n=160, radius=72.0, lw=8, r=20, hole_r=(1, 3)))
    raise ValueError(f"no workload {i}")

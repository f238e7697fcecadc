"""Seeded synthetic measures on an Nx x Ny x Ntheta SE(2) grid.

This module only draws inputs: line segments, cubic Bezier strokes and smooth
orientation fields, splatted onto the lifted grid and normalised to probability
vectors.  It holds none of the transport method's arithmetic (no distance, no
kernel, no scaling step) and is shared by the FP64 oracle tests and the GPU
harness so both see byte-identical inputs.

The paper lifts MNIST/QuickDraw images with cake wavelets (Section 5.2) and
orientation fields with a B-spline lift (Section 5.3).  Those datasets are not
used here; seeded strokes and fields of the same shape stand in for them.

Conventions shared with the solver:
  * array layout [iy][ix][k], theta innermost, float64;
  * pixel (ix, iy) sits at (x, y) = (ix, iy), unit spacing;
  * theta_k = k * Theta / Ntheta with Theta = 2*pi (full) or pi (axial).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

TWO_PI = 2.0 * math.pi


def rng_for(seed: int, stream: int = 0) -> np.random.Generator:
    """PCG64 generator for (seed, stream); streams 0, 1, ... feed mu, nu, ..."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(entropy=seed, spawn_key=(stream,))))


@dataclasses.dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    nt: int
    axial: bool = False

    @property
    def period(self) -> float:
        return math.pi if self.axial else TWO_PI

    @property
    def shape(self) -> Tuple[int, int, int]:
        return (self.ny, self.nx, self.nt)

    @property
    def size(self) -> int:
        return self.nx * self.ny * self.nt


def _theta_profile(grid: Grid, angles: np.ndarray, sigma_bins: float) -> np.ndarray:
    """Periodic Gaussian over the theta bins around each angle, shape [n, nt]."""
    step = grid.period / grid.nt
    k = np.arange(grid.nt, dtype=np.float64)
    d = (k[None, :] * step - angles[:, None]) / step  # in bins
    d = np.mod(d + grid.nt / 2.0, grid.nt) - grid.nt / 2.0
    return np.exp(-0.5 * (d / sigma_bins) ** 2)


def splat_points(grid: Grid, px: np.ndarray, py: np.ndarray, ang: np.ndarray,
                 weight: np.ndarray, sigma_xy: float, sigma_theta_bins: float = 1.0) -> np.ndarray:
    """Sum of separable Gaussians (x, y) x periodic Gaussian (theta), truncated at 4 sigma.

    Mass falling outside the grid is dropped.  Returns float64 [ny][nx][nt].
    """
    out = np.zeros(grid.shape, dtype=np.float64)
    if px.size == 0:
        return out
    r = int(math.ceil(4.0 * sigma_xy))
    prof = _theta_profile(grid, ang, sigma_theta_bins) * weight[:, None]  # [n, nt]
    cx = np.rint(px).astype(np.int64)
    cy = np.rint(py).astype(np.int64)
    for oy in range(-r, r + 1):
        iy = cy + oy
        gy = np.exp(-0.5 * ((iy - py) / sigma_xy) ** 2)
        for ox in range(-r, r + 1):
            ix = cx + ox
            ok = (ix >= 0) & (ix < grid.nx) & (iy >= 0) & (iy < grid.ny)
            if not np.any(ok):
                continue
            g = gy * np.exp(-0.5 * ((ix - px) / sigma_xy) ** 2)
            np.add.at(out, (iy[ok], ix[ok]), prof[ok] * g[ok, None])
    return out


def normalise(m: np.ndarray, floor: float = 0.0) -> np.ndarray:
    """Scale to total mass one, add a per-element floor, scale again (sums in FP64)."""
    s = float(m.sum(dtype=np.float64))
    if s <= 0.0:
        raise ValueError("empty measure")
    m = m / s
    if floor > 0.0:
        m = m + floor
        m = m / float(m.sum(dtype=np.float64))
    return m


# ---------------------------------------------------------------------------
# line segments
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Segment:
    cx: float
    cy: float
    alpha: float  # in [0, pi)
    length: float


def draw_segments(rng: np.random.Generator, grid: Grid, n: int, lmin: float, lmax: float,
                  margin: Optional[float] = None) -> List[Segment]:
    """n segments: centre uniform in the grid, angle U[0, pi), length U[lmin, lmax].

    With `margin`, a draw is repeated until both endpoints lie at least `margin`
    px inside the grid (so no mass is clipped at the border).
    """
    segs = []
    for _ in range(n):
        while True:
            cx = rng.uniform(0.0, grid.nx - 1)
            cy = rng.uniform(0.0, grid.ny - 1)
            alpha = rng.uniform(0.0, math.pi)
            length = rng.uniform(lmin, lmax)
            s = Segment(cx, cy, alpha, length)
            if margin is None or _inside(grid, s, margin):
                break
        segs.append(s)
    return segs


def _inside(grid: Grid, s: Segment, margin: float) -> bool:
    hx = 0.5 * s.length * math.cos(s.alpha)
    hy = 0.5 * s.length * math.sin(s.alpha)
    for ex, ey in ((s.cx - hx, s.cy - hy), (s.cx + hx, s.cy + hy)):
        if not (margin <= ex <= grid.nx - 1 - margin and margin <= ey <= grid.ny - 1 - margin):
            return False
    return True


def segment_points(segs: Sequence[Segment], step: float = 0.25):
    """Sample points every `step` px along each segment; each point weighs `step`."""
    xs, ys, angs, ws = [], [], [], []
    for s in segs:
        npts = max(1, int(math.floor(s.length / step)) + 1)
        t = np.linspace(-0.5 * s.length, 0.5 * s.length, npts)
        xs.append(s.cx + t * math.cos(s.alpha))
        ys.append(s.cy + t * math.sin(s.alpha))
        angs.append(np.full(npts, s.alpha))
        ws.append(np.full(npts, s.length / npts))
    return (np.concatenate(xs), np.concatenate(ys), np.concatenate(angs), np.concatenate(ws))


def splat_segments(grid: Grid, segs: Sequence[Segment], sigma_xy: float = 1.0, floor: float = 1e-6) -> np.ndarray:
    px, py, ang, w = segment_points(segs)
    return normalise(splat_points(grid, px, py, np.mod(ang, grid.period), w, sigma_xy), floor)


def moved_segments(rng: np.random.Generator, grid: Grid, segs: Sequence[Segment], shift: float, rot: float,
                   margin: Optional[float] = None) -> List[Segment]:
    """Each segment moved by a rigid motion: shift U[-shift, shift]^2, rotation U[-rot, rot] about its centre.

    With `margin`, a motion is redrawn until the moved endpoints stay `margin` px inside the grid.
    """
    out = []
    for s in segs:
        while True:
            dx = rng.uniform(-shift, shift)
            dy = rng.uniform(-shift, shift)
            dr = rng.uniform(-rot, rot)
            m = Segment(s.cx + dx, s.cy + dy, math.fmod(s.alpha + dr + math.pi, math.pi), s.length)
            if margin is None or _inside(grid, m, margin):
                break
        out.append(m)
    return out


# ---------------------------------------------------------------------------
# cubic Bezier strokes
# ---------------------------------------------------------------------------

def bezier_points(ctrl: np.ndarray, step: float = 0.25):
    """Points every `step` px of arc length along a cubic Bezier, tangent angle mod pi."""
    t = np.linspace(0.0, 1.0, 4097)
    b = ((1 - t) ** 3)[:, None] * ctrl[0] + (3 * (1 - t) ** 2 * t)[:, None] * ctrl[1] \
        + (3 * (1 - t) * t ** 2)[:, None] * ctrl[2] + (t ** 3)[:, None] * ctrl[3]
    d = (3 * (1 - t) ** 2)[:, None] * (ctrl[1] - ctrl[0]) + (6 * (1 - t) * t)[:, None] * (ctrl[2] - ctrl[1]) \
        + (3 * t ** 2)[:, None] * (ctrl[3] - ctrl[2])
    seg = np.sqrt(np.sum(np.diff(b, axis=0) ** 2, axis=1))
    s = np.concatenate([[0.0], np.cumsum(seg)])
    total = s[-1]
    npts = max(1, int(math.floor(total / step)) + 1)
    si = np.linspace(0.0, total, npts)
    x = np.interp(si, s, b[:, 0])
    y = np.interp(si, s, b[:, 1])
    dx = np.interp(si, s, d[:, 0])
    dy = np.interp(si, s, d[:, 1])
    ang = np.mod(np.arctan2(dy, dx), math.pi)
    w = np.full(npts, total / npts if total > 0 else 1.0)
    return x, y, ang, w


def splat_beziers(rng: np.random.Generator, grid: Grid, ncurves: int, sigma_xy: float, floor: float = 0.0) -> np.ndarray:
    xs, ys, angs, ws = [], [], [], []
    for _ in range(ncurves):
        ctrl = np.stack([rng.uniform(0.0, grid.nx - 1, 4), rng.uniform(0.0, grid.ny - 1, 4)], axis=1)
        x, y, a, w = bezier_points(ctrl)
        xs.append(x); ys.append(y); angs.append(a); ws.append(w)
    px, py, ang, w = (np.concatenate(v) for v in (xs, ys, angs, ws))
    return normalise(splat_points(grid, px, py, np.mod(ang, grid.period), w, sigma_xy), floor)


# ---------------------------------------------------------------------------
# smooth orientation fields (axial grids)
# ---------------------------------------------------------------------------

def orientation_field(rng: np.random.Generator, n: int, nmodes: int = 6) -> np.ndarray:
    """theta(x,y) = sum_j a_j sin(2 pi (p_j x + q_j y)/n + phi_j) mod pi, shape [n][n]."""
    pq = [(p, q) for p in range(-2, 3) for q in range(-2, 3) if (p, q) != (0, 0)]
    idx = rng.choice(len(pq), size=nmodes, replace=True)
    a = rng.uniform(-math.pi / 2, math.pi / 2, nmodes)
    ph = rng.uniform(0.0, TWO_PI, nmodes)
    yy, xx = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64), indexing="ij")
    th = np.zeros((n, n))
    for j in range(nmodes):
        p, q = pq[idx[j]]
        th += a[j] * np.sin(TWO_PI * (p * xx + q * yy) / n + ph[j])
    return np.mod(th, math.pi)


def lift_field(grid: Grid, theta: np.ndarray, sigma_bins: float = 1.0) -> np.ndarray:
    """Mass 1/(nx*ny) per pixel spread over theta bins by a periodic Gaussian."""
    prof = _theta_profile(grid, theta.reshape(-1), sigma_bins)
    prof = prof / prof.sum(axis=1, keepdims=True)
    out = (prof / (grid.nx * grid.ny)).reshape(grid.shape)
    return out / float(out.sum(dtype=np.float64))


# ---------------------------------------------------------------------------
# problem instances of the five workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class OTInstance:
    grid: Grid
    w: Tuple[float, float, float]
    eps: float
    radius: int
    mu: np.ndarray
    nu: np.ndarray
    name: str


@dataclasses.dataclass
class BaryInstance:
    grid: Grid
    w: Tuple[float, float, float]
    eps: float
    radius: int
    mus: List[np.ndarray]
    lambdas: List[float]
    name: str


def tiny_ot(instance: int = 0) -> OTInstance:
    """16x16x8, w=(1,2,1), eps=0.5, 9x9 window, 3 segments per measure, floor 1e-6."""
    g = Grid(16, 16, 8)
    seed = 0 * 1000 + instance
    mus = []
    for stream in (0, 1):
        r = rng_for(seed, stream)
        mus.append(splat_segments(g, draw_segments(r, g, 3, 2.5, 10.0), 1.0, 1e-6))
    return OTInstance(g, (1.0, 2.0, 1.0), 0.5, 4, mus[0], mus[1], f"ot16x16x8/{instance}")


# A paired instance moves each point of a segment by at most shift*sqrt(2) + (L/2)*rot
# = 1.41 + 20 * 0.098 = 3.4 px, inside the 11x11 window, and keeps every endpoint
# 3 px (3 sigma) inside the grid, so the truncated-window problem is feasible.
PAIRED_SHIFT = 1.0
PAIRED_ROT = math.pi / 32
PAIRED_MARGIN = 3.0


def lines64(instance: int = 0, paired: bool = True, n: int = 64) -> OTInstance:
    """n x n x 16 (64 by default), w=(1,3,1), eps=0.1, 11x11 window, 8 segments of 10-40 px, floor 1e-6.

    paired=False draws mu and nu independently (the truncated window generally
    makes that pair infeasible); paired=True moves each of mu's segments by a
    small seeded rigid motion and keeps all segments clear of the border.
    """
    g = Grid(n, n, 16)
    seed = 1 * 1000 + instance
    r0 = rng_for(seed, 0)
    scale = n / 64.0
    margin = PAIRED_MARGIN if paired else None
    segs = draw_segments(r0, g, 8, 10.0 * scale, 40.0 * scale, margin)
    mu = splat_segments(g, segs, 1.0, 1e-6)
    r1 = rng_for(seed, 1)
    if paired:
        nu = splat_segments(g, moved_segments(r1, g, segs, PAIRED_SHIFT, PAIRED_ROT, margin), 1.0, 1e-6)
    else:
        nu = splat_segments(g, draw_segments(r1, g, 8, 10.0 * scale, 40.0 * scale), 1.0, 1e-6)
    tag = "paired" if paired else "indep"
    return OTInstance(g, (1.0, 3.0, 1.0), 0.1, 5, mu, nu, f"lines{n}x{n}x16-{tag}/{instance}")


# The converging 64x64x16 instance.  With 1-px strokes the lines64 pairs (and even nu = mu)
# keep a marginal error near 1.5e-6 for thousands of iterations: at eps = 0.1 a neighbouring
# pixel is reached with weight e^-10 at best, so the mass balance between neighbours relaxes
# on a time scale of ~10^4 iterations, with an amplitude set by the steepness of the strokes.
# Strokes three times as wide (sigma_xy = 3 px) bring that plateau to 4e-7 (median; 6e-7 at
# most over 32 instances after 3000 iterations).
THETA_TURN = math.pi / 16
THETA_SIGMA_XY = 3.0


def lines64_theta(instance: int = 0, n: int = 64) -> OTInstance:
    """n x n x 16, w=(1,3,1), eps=0.1, 11x11 window, 8 segments of 10-40 px splatted with
    sigma_xy = 3 px, floor 1e-6.  nu has the same stroke points as mu, each segment's orientation
    turned by a seeded angle in U[-pi/16, pi/16] (a motion along theta only, which the SE(2)
    cost prices at w3^2 dtheta^2)."""
    g = Grid(n, n, 16)
    seed = 1 * 1000 + 500 + instance
    scale = n / 64.0
    segs = draw_segments(rng_for(seed, 0), g, 8, 10.0 * scale, 40.0 * scale, PAIRED_MARGIN)
    px, py, ang, w = segment_points(segs)
    mu = normalise(splat_points(g, px, py, np.mod(ang, g.period), w, THETA_SIGMA_XY), 1e-6)
    r1 = rng_for(seed, 1)
    turns = np.concatenate([np.full(max(1, int(math.floor(s.length / 0.25)) + 1), r1.uniform(-THETA_TURN, THETA_TURN))
                            for s in segs])
    nu = normalise(splat_points(g, px, py, np.mod(ang + turns, g.period), w, THETA_SIGMA_XY), 1e-6)
    return OTInstance(g, (1.0, 3.0, 1.0), 0.1, 5, mu, nu, f"lines{n}x{n}x16-theta/{instance}")


# Measures without a floor still get POSITIVE_FLOOR per element (about 2^-997, far
# below any mass that matters): where one measure is exactly zero over a whole window,
# the barycenter is zero there and mass of another measure has no partner inside the
# truncated window, which makes the problem infeasible.
POSITIVE_FLOOR = 1e-300


def curves128(instance: int = 0, t: float = 0.5, n: int = 128) -> BaryInstance:
    """Two measures of 4 cubic Beziers, 128x128x16, w=(1,3,1), eps=0.05, 15x15 window,
    no floor beyond POSITIVE_FLOOR.

    Weights (1-t, t): t=0 returns the first measure's side (the interpolation
    reading that makes Phi_0 the first input).
    """
    g = Grid(n, n, 16)
    seed = 2 * 1000 + instance
    mus = [splat_beziers(rng_for(seed, s), g, 4, 1.5, POSITIVE_FLOOR) for s in (0, 1)]
    return BaryInstance(g, (1.0, 3.0, 1.0), 0.05, 7, mus, [1.0 - t, t], f"curves{n}x{n}x16/{instance}/t={t}")


def fields256(instance: int = 0, n: int = 256, nt: int = 32) -> BaryInstance:
    """Four lifted orientation fields on an axial n x n x nt grid, w=(1,4,1), eps=0.03, 21x21, equal weights."""
    g = Grid(n, n, nt, axial=True)
    seed = 4 * 1000 + instance
    mus = [lift_field(g, orientation_field(rng_for(seed, s), n)) for s in range(4)]
    return BaryInstance(g, (1.0, 4.0, 1.0), 0.03, 10, mus, [0.25] * 4, f"fields{n}x{n}x{nt}-axial/{instance}")


SERVE_GRIDS = ((32, 8, 4), (64, 16, 5), (128, 16, 7))  # (n, ntheta, radius)
SERVE_EPS = (0.05, 0.1, 0.2)
SERVE_W2 = (2.0, 3.0)


@dataclasses.dataclass
class Request:
    arrival_s: float
    inst: OTInstance


def _serve_request(seed: int, i: int, arrival: float, grids, paired: bool) -> Request:
    r = rng_for(seed + 1 + i, 0)
    n, nt, rad = grids[int(r.integers(len(grids)))]
    eps = float(SERVE_EPS[int(r.integers(len(SERVE_EPS)))])
    w2 = float(SERVE_W2[int(r.integers(len(SERVE_W2)))])
    nseg = int(r.integers(4, 13))
    g = Grid(n, n, nt)
    margin = PAIRED_MARGIN if paired else None
    segs = draw_segments(r, g, nseg, 10.0 * n / 64, 40.0 * n / 64, margin)
    mu = splat_segments(g, segs, 1.0, 1e-6)
    if paired:
        nu = splat_segments(g, moved_segments(r, g, segs, PAIRED_SHIFT, PAIRED_ROT, margin), 1.0, 1e-6)
    else:
        nu = splat_segments(g, draw_segments(r, g, nseg, 10.0 * n / 64, 40.0 * n / 64), 1.0, 1e-6)
    return Request(float(arrival), OTInstance(g, (1.0, w2, 1.0), eps, rad, mu, nu, f"serve/{i}"))


def _serve_theta_request(seed: int, i: int, arrival: float, grids) -> Request:
    """A converging request: the theta-motion pair of lines64_theta on one of the serving
    grids (segments scaled by n/64), eps = 0.1, w = (1,3,1)."""
    r = rng_for(seed + 1 + i, 0)
    n, nt, rad = grids[int(r.integers(len(grids)))]
    g = Grid(n, n, nt)
    scale = n / 64.0
    segs = draw_segments(r, g, int(r.integers(4, 13)), 10.0 * scale, 40.0 * scale, PAIRED_MARGIN)
    px, py, ang, w = segment_points(segs)
    mu = normalise(splat_points(g, px, py, np.mod(ang, g.period), w, THETA_SIGMA_XY), 1e-6)
    turns = np.concatenate([np.full(max(1, int(math.floor(s.length / 0.25)) + 1), r.uniform(-THETA_TURN, THETA_TURN))
                            for s in segs])
    nu = normalise(splat_points(g, px, py, np.mod(ang + turns, g.period), w, THETA_SIGMA_XY), 1e-6)
    return Request(float(arrival), OTInstance(g, (1.0, 3.0, 1.0), 0.1, rad, mu, nu, f"serve-theta/{i}"))


def _serve_chunk(args):
    seed, idx, arrivals, grids, paired = args
    if paired == "theta":
        return [_serve_theta_request(seed, i, a, grids) for i, a in zip(idx, arrivals)]
    return [_serve_request(seed, i, a, grids, paired) for i, a in zip(idx, arrivals)]


def serving_trace(nreq: int = 512, rate: float = 200.0, seed: int = 3000, paired=True,
                  grids: Optional[Sequence[Tuple[int, int, int]]] = None, workers: int = 1) -> List[Request]:
    """Poisson stream of OT requests with mixed grid sizes, eps and w2 (paired = "theta":
    theta-motion pairs that converge, eps 0.1, w2 = 3).  Request i draws from its own stream,
    so the trace is the same for any worker count (workers > 1 forks processes: call it
    before any GPU work)."""
    grids = list(grids or SERVE_GRIDS)
    arr = rng_for(seed, 0)
    gaps = arr.exponential(1.0 / rate, nreq)
    t = np.cumsum(gaps) - gaps[0]
    if workers <= 1 or nreq < 32:
        return _serve_chunk((seed, list(range(nreq)), list(t), grids, paired))
    import concurrent.futures as cf
    import multiprocessing as mp
    parts = [(seed, list(range(w, nreq, workers)), list(t[w::workers]), grids, paired) for w in range(workers)]
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        chunks = list(ex.map(_serve_chunk, parts))
    out = [None] * nreq
    for w, chunk in enumerate(chunks):
        for j, req in enumerate(chunk):
            out[w + j * workers] = req
    return out


# ---------------------------------------------------------------------------
# many small stroke images (barycenters of a whole class of 28 x 28 images)
# ---------------------------------------------------------------------------

STROKE_GRID = Grid(28, 28, 16)


def stroke_image(seed: int, index: int) -> np.ndarray:
    """One 28 x 28 x 16 stroke image: 2-4 segments of 6-14 px (two to four pen strokes of a
    digit-sized drawing), kept 2 px inside the frame, sigma_xy = 1 px, floor 1e-6."""
    r = rng_for(seed, index)
    nseg = int(r.integers(2, 5))
    segs = draw_segments(r, STROKE_GRID, nseg, 6.0, 14.0, margin=2.0)
    return splat_segments(STROKE_GRID, segs, 1.0, 1e-6)


def _stroke_chunk(args):
    seed, lo, hi = args
    return np.stack([stroke_image(seed, i) for i in range(lo, hi)])


def stroke_images(n: int, seed: int = 6000, workers: int = 1) -> np.ndarray:
    """n stroke images [n][28][28][16], image i from stream i of `seed` (the same arrays for
    any worker count; workers > 1 forks processes, so call it before any GPU work)."""
    if workers <= 1 or n < 64:
        return _stroke_chunk((seed, 0, n))
    import concurrent.futures as cf
    import multiprocessing as mp
    step = (n + workers - 1) // workers
    parts = [(seed, lo, min(n, lo + step)) for lo in range(0, n, step)]
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        return np.concatenate(list(ex.map(_stroke_chunk, parts)))


def line_completion(seed: int = 7000, n: int = 64) -> np.ndarray:
    """The gradient-flow input of the line-completion experiment (Section 5.4): one dominant
    line through the middle, broken into 6 dashes of 6 px with 3 px gaps, amid 16 random short
    line elements (2-4 px), on an n x n x 16 grid; sigma_xy = 1 px, floor 1e-6."""
    g = Grid(n, n, 16)
    r = rng_for(seed, 0)
    alpha = r.uniform(0.0, math.pi)
    c = (n - 1) / 2.0
    segs = [Segment(c + t * math.cos(alpha), c + t * math.sin(alpha), alpha, 6.0)
            for t in (-22.5, -13.5, -4.5, 4.5, 13.5, 22.5)]
    segs += draw_segments(r, g, 16, 2.0, 4.0, margin=1.0)
    return splat_segments(g, segs, 1.0, 1e-6)

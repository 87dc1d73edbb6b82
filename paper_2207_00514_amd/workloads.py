"""Seeded synthetic point clouds for the EMST workloads.

This module only draws random numbers: it contains none of the EMST
arithmetic, so both the HIP path and the CPU oracle can take their inputs
from it without sharing any of the method's code.

The paper measures on 2D/3D trajectory, cosmology, generator-based and
normal/uniform datasets (Section 4, "Datasets"); none of them is available
here, so the generators below stand in for them with the same dimension,
size and kind of structure:

* ``uniform2d``    -- i.i.d. U[0,1)^2 (stands in for the Uniform*2 sets);
* ``clustered3d``  -- 200 isotropic Gaussians plus 10 % uniform background
                      (stands in for the Normal*/VisualVar* clustered sets);
* ``cosmology3d``  -- uniform field plus Plummer halos with power-law member
                      counts in a periodic box (stands in for Hacc37M);
* ``batched``      -- many small 2D uniform / 3D Gaussian-mixture clouds;
* tie-stress fixtures (integer grids, duplicates, collinear points, identical
  points, two far clusters) used by the parity tests.

All geometry is drawn in float64 with ``numpy.random.Generator(PCG64(seed))``,
cast to float32, and the whole cloud is shuffled with the same generator so
that input indices carry no cluster structure.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "rng_for", "uniform2d", "clustered3d", "cosmology3d", "skewed3d", "batched_clouds",
    "request_sizes", "request_cloud", "integer_grid", "duplicates", "collinear",
    "identical", "two_clusters", "small_random", "WORKLOADS", "make",
]


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _finish(rng: np.random.Generator, pts64: np.ndarray) -> np.ndarray:
    pts = np.ascontiguousarray(pts64.astype(np.float32))
    perm = rng.permutation(pts.shape[0])
    return np.ascontiguousarray(pts[perm])


def uniform2d(n: int = 10_000, seed: int = 1) -> np.ndarray:
    """n points i.i.d. U[0,1)^2 (the small 2D uniform workload)."""
    rng = rng_for(seed)
    return _finish(rng, rng.random((n, 2)))


def clustered3d(n: int = 2_000_000, seed: int = 2, n_centres: int = 200,
                background: float = 0.10) -> np.ndarray:
    """3D clustered cloud: (1-background) of the points in ``n_centres``
    isotropic Gaussians (centres U[0,1)^3, sigma log-uniform in
    [0.002, 0.02], equal weights, no clipping), the rest U[0,1)^3."""
    rng = rng_for(seed)
    n_bg = int(round(n * background))
    n_cl = n - n_bg
    centres = rng.random((n_centres, 3))
    sigma = np.exp(rng.uniform(math.log(0.002), math.log(0.02), n_centres))
    counts = rng.multinomial(n_cl, np.full(n_centres, 1.0 / n_centres))
    owner = np.repeat(np.arange(n_centres), counts)
    pts = centres[owner] + sigma[owner, None] * rng.standard_normal((n_cl, 3))
    bg = rng.random((n_bg, 3))
    return _finish(rng, np.concatenate([pts, bg], axis=0))


def skewed3d(n: int = 2_000_000, seed: int = 6, walks: int = 1000, outliers: float = 0.001,
             step: float = 1e-6, extent: float = 1000.0) -> np.ndarray:
    """Extreme density contrast (GPS-trajectory-like): (1 - outliers) of the
    points lie on ``walks`` Gaussian random walks (step sigma ``step``) that
    start in a cube of side 1e-3; the rest are U[0, extent)^3.  The scene box
    is set by the outliers, so at 21 bits per axis the dense part falls into
    a handful of Morton cells."""
    rng = rng_for(seed)
    n_out = int(round(n * outliers))
    n_in = n - n_out
    lens = rng.multinomial(n_in, np.full(walks, 1.0 / walks))
    starts = 0.5 + 1e-3 * rng.random((walks, 3))
    steps = step * rng.standard_normal((n_in, 3))
    owner = np.repeat(np.arange(walks), lens)
    first = np.concatenate([[0], np.cumsum(lens)[:-1]])
    pos = np.cumsum(steps, axis=0)
    pos -= np.repeat(pos[first] - steps[first], lens, axis=0)  # every walk restarts at 0
    pts = starts[owner] + pos
    out = extent * rng.random((n_out, 3))
    return _finish(rng, np.concatenate([pts, out], axis=0))


def _halo_counts(rng: np.random.Generator, n_halos: int, total: int,
                 n_min: int = 20, alpha: float = 0.9):
    """Power-law member counts (pdf ~ N^-(1+alpha), N >= n_min), capped at
    10 % of the halo total and rescaled to sum exactly to ``total``."""
    raw = n_min * rng.random(n_halos) ** (-1.0 / alpha)
    cap = 0.10 * total
    raw = np.minimum(raw, cap)
    factor = total / raw.sum()
    x = raw * factor
    base = np.floor(x).astype(np.int64)
    deficit = int(total - base.sum())
    if deficit > 0:
        order = np.argsort(-(x - base), kind="stable")
        base[order[:deficit]] += 1
    base = np.maximum(base, n_min)
    excess = int(base.sum() - total)
    while excess > 0:
        k = int(np.argmax(base))
        take = min(excess, int(base[k] - n_min))
        base[k] -= take
        excess -= take
    return base, factor


def cosmology3d(n: int = 37_000_000, seed: int = 3, box: float = 64.0,
                halo_fraction: float = 0.60, n_halos: int = 50_000,
                chunk: int = 4_000_000) -> np.ndarray:
    """Cosmology-like cloud in the periodic box [0, box)^3: a uniform field
    plus Plummer-profile halos whose member counts follow a power law of
    exponent -1.9 (minimum 20); scale radius 0.05 * N^(1/3) * 0.01."""
    rng = rng_for(seed)
    n_halo_pts = int(round(n * halo_fraction))
    n_field = n - n_halo_pts
    n_halos = max(1, min(n_halos, n_halo_pts // 20))
    out = np.empty((n, 3), dtype=np.float32)
    # field
    pos = 0
    while pos < n_field:
        m = min(chunk, n_field - pos)
        out[pos:pos + m] = (rng.random((m, 3)) * box).astype(np.float32)
        pos += m
    centres = rng.random((n_halos, 3)) * box
    counts, _factor = _halo_counts(rng, n_halos, n_halo_pts)
    a = 0.05 * np.cbrt(counts.astype(np.float64)) * 0.01
    owner_all = np.repeat(np.arange(n_halos), counts)
    done = 0
    while done < n_halo_pts:
        m = min(chunk, n_halo_pts - done)
        owner = owner_all[done:done + m]
        u = rng.random(m)
        u = np.clip(u, 1e-12, 1.0 - 1e-12)
        r = a[owner] / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
        v = rng.standard_normal((m, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        p = centres[owner] + r[:, None] * v
        p = np.mod(p, box).astype(np.float32)
        p[p >= np.float32(box)] = 0.0
        out[n_field + done:n_field + done + m] = p
        done += m
    perm = rng.permutation(n)
    return np.ascontiguousarray(out[perm])


def batched_clouds(n_clouds: int = 512, seed: int = 4, lo: int = 1_000,
                   hi: int = 200_000):
    """List of (points, dim) clouds: sizes log-uniform in [lo, hi]; half 2D
    U[0,1)^2, half 3D Gaussian mixtures (20 centres U[0,1)^3, sigma 0.01)."""
    rng = rng_for(seed)
    sizes = np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), n_clouds))).astype(np.int64)
    dims = rng.permutation(np.array([2] * (n_clouds // 2) + [3] * (n_clouds - n_clouds // 2)))
    clouds = []
    for nb, d in zip(sizes.tolist(), dims.tolist()):
        if d == 2:
            pts = rng.random((nb, 2))
        else:
            pts = _mixture3d(rng, nb)
        clouds.append(_finish(rng, pts))
    return clouds


def _mixture3d(rng: np.random.Generator, nb: int, k: int = 20, sigma: float = 0.01):
    centres = rng.random((k, 3))
    counts = rng.multinomial(nb, np.full(k, 1.0 / k))
    owner = np.repeat(np.arange(k), counts)
    return centres[owner] + sigma * rng.standard_normal((nb, 3))


def request_sizes(count: int, seed: int = 5, median: float = 50_000.0,
                  sigma: float = 1.2, lo: int = 5_000, hi: int = 4_000_000):
    """Lognormal request sizes (median, sigma) clipped to [lo, hi]."""
    rng = rng_for(seed)
    n = np.round(np.exp(rng.normal(math.log(median), sigma, count)))
    return np.clip(n, lo, hi).astype(np.int64)


def request_cloud(n: int, seed: int) -> np.ndarray:
    """One serving request: 3D, uniform U[0,1)^3 or a 20-centre Gaussian
    mixture (sigma 0.01), chosen by a fair coin."""
    rng = rng_for(seed)
    if rng.random() < 0.5:
        pts = rng.random((n, 3))
    else:
        pts = _mixture3d(rng, n)
    return _finish(rng, pts)


# ----------------------------------------------------------------------------
# tie-stress fixtures


def integer_grid(k: int, dim: int = 2, seed: int = 0) -> np.ndarray:
    """All points of the k^dim unit integer grid, shuffled."""
    rng = rng_for(seed)
    axes = np.meshgrid(*([np.arange(k)] * dim), indexing="ij")
    pts = np.stack([a.ravel() for a in axes], axis=1).astype(np.float64)
    return _finish(rng, pts)


def duplicates(n_unique: int, repeat: int, dim: int = 3, seed: int = 0) -> np.ndarray:
    """n_unique random points, each repeated ``repeat`` times, shuffled."""
    rng = rng_for(seed)
    base = rng.random((n_unique, dim))
    return _finish(rng, np.repeat(base, repeat, axis=0))


def collinear(n: int, dim: int = 2, seed: int = 0) -> np.ndarray:
    """x = 0..n-1 on the first axis (other coordinates 0), shuffled."""
    rng = rng_for(seed)
    pts = np.zeros((n, dim))
    pts[:, 0] = np.arange(n)
    return _finish(rng, pts)


def identical(n: int, dim: int = 3, value: float = 0.25) -> np.ndarray:
    return np.full((n, dim), value, dtype=np.float32)


def two_clusters(n: int, dim: int = 3, seed: int = 0, gap: float = 100.0) -> np.ndarray:
    rng = rng_for(seed)
    a = rng.random((n // 2, dim))
    b = rng.random((n - n // 2, dim)) + gap
    return _finish(rng, np.concatenate([a, b], axis=0))


def small_random(n: int, dim: int, seed: int, kind: str = "uniform") -> np.ndarray:
    """Small clouds for property tests: 'uniform', 'int' (coordinates in a
    tiny integer range, so distances tie massively), 'dup' (many exact
    duplicates), 'outlier' (one far point)."""
    rng = rng_for(seed)
    if kind == "uniform":
        pts = rng.random((n, dim))
    elif kind == "int":
        pts = rng.integers(0, 4, size=(n, dim)).astype(np.float64)
    elif kind == "dup":
        base = rng.random((max(1, n // 3), dim))
        pts = base[rng.integers(0, base.shape[0], size=n)]
    elif kind == "outlier":
        pts = rng.random((n, dim))
        if n:
            pts[0] = 1e4
    else:
        raise ValueError(kind)
    return _finish(rng, pts)


# ----------------------------------------------------------------------------
# named workloads

WORKLOADS = {
    "uniform2d_10k": dict(fn=uniform2d, n=10_000, seed=1, dim=2),
    "clustered3d_2m": dict(fn=clustered3d, n=2_000_000, seed=2, dim=3),
    "cosmology3d_37m": dict(fn=cosmology3d, n=37_000_000, seed=3, dim=3),
    "skewed3d_2m": dict(fn=skewed3d, n=2_000_000, seed=6, dim=3),
}


def make(name: str, n: int | None = None) -> np.ndarray:
    """Named workload, optionally resized (same recipe, same seed)."""
    w = WORKLOADS[name]
    return w["fn"](n=w["n"] if n is None else n, seed=w["seed"])

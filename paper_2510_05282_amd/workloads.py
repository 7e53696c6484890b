"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws inputs (points, atom spheres, radial tables, request
streams).  It holds none of the harmonic, spline or projector arithmetic, and it
is the one piece of code that both the GPU path's tests/benchmark and the CPU
oracle's tests use.  Randomness comes from ``numpy.random.default_rng(seed)``
(PCG64), except the large upstream gradients of `upstream_gradient_device`,
which torch's seeded generator draws on the device.

The paper samples random points for its accuracy study (Section 4) and random
perturbed points for its timings (Section 5); it fixes no dataset.  The shapes here
follow the library's intended uses: large isotropic point batches, and the points
of a real-space grid inside each atom's projector sphere.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SPECIAL_RADII = (0.1, 0.2, 0.5, 1.0, 1.5, 2.0, 2.5, 3.0, 4.0, 5.0)


def isotropic_points(n: int, r_lo: float, r_hi: float, seed: int = 0,
                     rng: np.random.Generator | None = None) -> np.ndarray:
    """[n][3] float64 points: direction uniform on the sphere (normalised
    N(0,1)^3 draws), radius uniform in [r_lo, r_hi]."""
    rng = np.random.default_rng(seed) if rng is None else rng
    d = rng.standard_normal((n, 3))
    nrm = np.sqrt((d * d).sum(axis=1, keepdims=True))
    nrm[nrm == 0] = 1.0
    r = rng.uniform(r_lo, r_hi, size=(n, 1))
    return np.ascontiguousarray(d / nrm * r)


def special_points() -> np.ndarray:
    """64 fixed points: the six axis directions (+-x, +-y, +-z; the z ones are the
    poles) at ten radii, the origin, a pole at tiny radius, and two points a
    hair off the poles."""
    pts = []
    for ax in range(3):
        for sgn in (1.0, -1.0):
            for r in SPECIAL_RADII:
                p = [0.0, 0.0, 0.0]
                p[ax] = sgn * r
                pts.append(p)
    pts.append([0.0, 0.0, 0.0])
    pts.append([0.0, 0.0, 1e-200])
    pts.append([1e-9, 0.0, 1.0])
    pts.append([0.0, -1e-9, -1.0])
    a = np.array(pts, dtype=np.float64)
    assert a.shape == (64, 3)
    return a


def points_plain_eval(seed: int = 0, n_random: int = 100_000) -> np.ndarray:
    """Plain-evaluation parity set: n_random isotropic points with radius in
    [0.1, 5] followed by the 64 special points."""
    return np.concatenate([isotropic_points(n_random, 0.1, 5.0, seed), special_points()])


def points_roofline(n: int = 1 << 26, seed: int = 0, r_lo: float = 0.01,
                    r_hi: float = 10.0) -> np.ndarray:
    """Bandwidth-sweep set: n isotropic points, radius uniform in [0.01, 10]."""
    return isotropic_points(n, r_lo, r_hi, seed)


def points_gradient(n: int = 1 << 24, seed: int = 0) -> np.ndarray:
    """Differentiated-evaluation set: n isotropic points, radius in [0.5, 5]."""
    return isotropic_points(n, 0.5, 5.0, seed)


def upstream_gradient(nfun: int, n: int, seed: int = 1) -> np.ndarray:
    """[nfun][n] N(0,1) upstream gradient."""
    return np.random.default_rng(seed).standard_normal((nfun, n))


# --------------------------------------------------------------------------
# Atom spheres on a real-space grid, and radial tables


def radial_table(rng: np.random.Generator, lmax: int, n_r: int = 2000,
                 r_max: float = 3.0) -> np.ndarray:
    """[(lmax+1)][n_r] radial values on the uniform grid r_i = i r_max/(n_r-1):
    R_l(r) = (1 - (r/r_max)^2)^2 sum_{k=0..2} c_lk r^(l+2k) exp(-a_lk r^2),
    c ~ N(0,1), a ~ U[0.5, 2], rescaled so that max_i |R_l(r_i)| = 1.  Like a
    pseudopotential projector, each R_l goes smoothly to zero at the cutoff r_max."""
    r = np.linspace(0.0, r_max, n_r)
    cut = (1.0 - (r / r_max) ** 2) ** 2
    out = np.empty((lmax + 1, n_r))
    for l in range(lmax + 1):
        c = rng.standard_normal(3)
        a = rng.uniform(0.5, 2.0, size=3)
        v = cut * sum(c[k] * r ** (l + 2 * k) * np.exp(-a[k] * r * r) for k in range(3))
        s = np.abs(v).max()
        out[l] = v / s if s > 0 else v
    return out


@dataclass
class AtomSet:
    lmax: int
    centers: np.ndarray        # [n_atoms][3] float64
    offsets: np.ndarray        # [n_atoms+1] int64 (CSR over points)
    points: np.ndarray         # [offsets[-1]][3] float64, unwrapped absolute coordinates
    tables: np.ndarray         # [n_atoms][lmax+1][n_r] radial values
    r_max: float

    @property
    def n_atoms(self) -> int:
        return self.centers.shape[0]


def sphere_points(center: np.ndarray, radius: float, h: float) -> np.ndarray:
    """Points h*(i,j,k) of the infinite cubic lattice within `radius` of `center`
    (unwrapped periodic images), lexicographic in (i,j,k) with k fastest."""
    lo = np.ceil((center - radius) / h - 1e-9).astype(np.int64)
    hi = np.floor((center + radius) / h + 1e-9).astype(np.int64)
    ii = [np.arange(lo[d], hi[d] + 1) for d in range(3)]
    I, J, K = np.meshgrid(*ii, indexing="ij")
    P = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1).astype(np.float64) * h
    d = P - center
    keep = (d * d).sum(axis=1) <= radius * radius
    return np.ascontiguousarray(P[keep])


def atom_spheres(seed: int = 0, n_atoms: int = 64, box: float = 20.0, radius: float = 3.0,
                 h: float = 0.2, lmax: int = 3, n_r: int = 2000) -> AtomSet:
    """Projector-build set: n_atoms centres uniform in a periodic box; each atom's
    points are the grid points (spacing h) inside its sphere; each atom has its
    own radial table on [0, radius]."""
    rng = np.random.default_rng(seed)
    centers = rng.uniform(0.0, box, size=(n_atoms, 3))
    pts = [sphere_points(c, radius, h) for c in centers]
    offsets = np.zeros(n_atoms + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([p.shape[0] for p in pts])
    tables = np.stack([radial_table(rng, lmax, n_r, radius) for _ in range(n_atoms)])
    return AtomSet(lmax, centers, offsets, np.concatenate(pts), tables, radius)


# --------------------------------------------------------------------------
# Served projector requests


@dataclass
class Request:
    arrival: float        # seconds after the start of the stream
    lmax: int
    n: int                # number of points of the atom sphere
    dtype: str            # "f64" or "f32"
    center: np.ndarray    # [3]
    seed: int             # seed of this request's points and radial table


def request_stream(n_req: int = 10_000, rate: float = 1000.0, seed: int = 0,
                   n_lo: float = 1e3, n_hi: float = 1e6, p_f64: float = 0.8) -> list[Request]:
    """Poisson arrivals at `rate` per second; per request lmax ~ U{0..9},
    n = round(exp(U[ln n_lo, ln n_hi])), dtype float64 with probability p_f64."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_req)
    t = np.cumsum(gaps)
    lmax = rng.integers(0, 10, size=n_req)
    n = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=n_req))).astype(np.int64)
    f64 = rng.uniform(size=n_req) < p_f64
    centers = rng.uniform(0.0, 20.0, size=(n_req, 3))
    seeds = rng.integers(0, 2**31 - 1, size=n_req)
    return [Request(float(t[i]), int(lmax[i]), int(n[i]), "f64" if f64[i] else "f32",
                    centers[i], int(seeds[i])) for i in range(n_req)]


def request_inputs(req: Request, radius: float = 3.0, n_r: int = 2000):
    """Points ([n][3] float64, uniform in the ball of `radius` about the centre)
    and radial table ([lmax+1][n_r]) of one request."""
    rng = np.random.default_rng(req.seed)
    d = rng.standard_normal((req.n, 3))
    nrm = np.sqrt((d * d).sum(axis=1, keepdims=True))
    nrm[nrm == 0] = 1.0
    r = radius * rng.uniform(size=(req.n, 1)) ** (1.0 / 3.0)
    pts = req.center[None, :] + d / nrm * r
    return np.ascontiguousarray(pts), radial_table(rng, req.lmax, n_r, radius)


def upstream_gradient_device(nfun: int, n: int, seed: int, device):
    """[nfun][n] N(0,1) upstream gradient drawn on the device with torch's seeded
    generator (large batches, where a host draw would dominate set-up time)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return torch.randn((nfun, n), generator=g, dtype=torch.float64, device=device)

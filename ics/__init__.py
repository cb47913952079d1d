"""Seeded synthetic initial conditions shared by the oracle tests, the GPU
tests and the benchmark.

This module draws random numbers and lays them out; it holds none of the
force, integrator, ordering or adjoint arithmetic of the n-body method, so
the oracle and the HIP path can both be fed from it without sharing any of
the method's code.

Workloads follow the paper's n-body setting (Section IV: bodies moving under
their mutual gravitation); the generators are:

* ``uniform_ball``   -- uniform density in the unit sphere, at rest.
* ``plummer``        -- isotropic Plummer sphere (scale radius a, mass M).
* ``colliding_pair`` -- two Plummer spheres of mass ratio 1:3 on a head-on
  approach with zero total momentum.
* ``ragged_batch``   -- many independent Plummer systems with log-uniform
  body counts.
* ``perturbed_snapshot`` -- a target configuration near a given one.
* ``sample_targets`` -- a seeded subset of target indices.

Every generator uses numpy's PCG64 with an explicit seed and returns FP64
arrays ``pos_mass`` of shape (N, 4) = (x, y, z, m) and ``vel`` of shape
(N, 4) = (vx, vy, vz, 0); callers cast to FP32 where a mode asks for it.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "rng",
    "uniform_ball",
    "plummer",
    "colliding_pair",
    "ragged_batch_sizes",
    "ragged_batch",
    "perturbed_snapshot",
    "sample_targets",
    "kepler_pair",
    "WORKLOADS",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _pack(x: np.ndarray, m: np.ndarray) -> np.ndarray:
    out = np.empty((x.shape[0], 4), dtype=np.float64)
    out[:, :3] = x
    out[:, 3] = m
    return out


def _pack_vel(v: np.ndarray) -> np.ndarray:
    out = np.zeros((v.shape[0], 4), dtype=np.float64)
    out[:, :3] = v
    return out


def uniform_ball(n: int, seed: int, radius: float = 1.0, total_mass: float = 1.0):
    """Uniform density inside a sphere, velocities zero, equal masses M/n.

    Rejection sampling from the cube [-1, 1)^3, accepted points kept in draw
    order, so the result is a pure function of (n, seed)."""
    g = rng(seed)
    pts = []
    have = 0
    while have < n:
        c = g.uniform(-1.0, 1.0, size=(max(2 * (n - have), 64), 3))
        ok = c[(c * c).sum(axis=1) < 1.0]
        pts.append(ok)
        have += ok.shape[0]
    x = np.concatenate(pts)[:n] * radius
    m = np.full(n, total_mass / n)
    return _pack(x, m), np.zeros((n, 4))


def _isotropic(g: np.random.Generator, k: int) -> np.ndarray:
    """k unit vectors uniform on the sphere (cos theta uniform, phi uniform)."""
    ct = g.uniform(-1.0, 1.0, size=k)
    ph = g.uniform(0.0, 2.0 * math.pi, size=k)
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    return np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=1)


def plummer(n: int, seed: int, a: float = 1.0, total_mass: float = 1.0,
            rmax: float = 20.0, center=(0.0, 0.0, 0.0), bulk=(0.0, 0.0, 0.0),
            G: float = 1.0):
    """Isotropic Plummer sphere in virial equilibrium.

    Radii from the inverted cumulative mass profile, r = a (X^(-2/3) - 1)^(-1/2),
    redrawn when r > rmax.  Speeds v = q * v_esc(r), with q drawn by von
    Neumann rejection from g(q) = q^2 (1 - q^2)^(7/2) under the bound 0.1
    (Aarseth, Henon & Wielen 1974).  Directions isotropic.  The centre of
    mass position and velocity are removed before the shift to ``center``
    and ``bulk``.  Equal masses M/n."""
    g = rng(seed)
    r = np.empty(n)
    have = 0
    while have < n:
        X = g.uniform(0.0, 1.0, size=max(2 * (n - have), 64))
        X = X[X > 0.0]
        rr = a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
        rr = rr[rr <= rmax * a]
        take = min(rr.shape[0], n - have)
        r[have:have + take] = rr[:take]
        have += take
    q = np.empty(n)
    have = 0
    while have < n:
        k = max(2 * (n - have) * 10, 640)
        qq = g.uniform(0.0, 1.0, size=k)
        yy = g.uniform(0.0, 0.1, size=k)
        acc = qq[yy < qq * qq * (1.0 - qq * qq) ** 3.5]
        take = min(acc.shape[0], n - have)
        q[have:have + take] = acc[:take]
        have += take
    vesc = np.sqrt(2.0 * G * total_mass / a) * (1.0 + (r / a) ** 2) ** (-0.25)
    x = r[:, None] * _isotropic(g, n)
    v = (q * vesc)[:, None] * _isotropic(g, n)
    x -= x.mean(axis=0)
    v -= v.mean(axis=0)
    x += np.asarray(center, dtype=np.float64)
    v += np.asarray(bulk, dtype=np.float64)
    m = np.full(n, total_mass / n)
    return _pack(x, m), _pack_vel(v)


def colliding_pair(n: int, seed: int):
    """Two Plummer spheres (scale radius 1) of masses 1/4 and 3/4 with equal
    particle masses 1/n: n/4 bodies centred at (-2,0,0) moving at +0.225 x and
    3n/4 bodies centred at (+2,0,0) moving at -0.075 x, a relative speed of
    0.3 and zero total momentum.  Internal speeds follow each sphere's own
    mass.  ``n`` must be divisible by 4."""
    if n % 4:
        raise ValueError("colliding_pair needs n divisible by 4")
    n1 = n // 4
    n2 = n - n1
    p1, v1 = plummer(n1, seed, total_mass=0.25, center=(-2.0, 0.0, 0.0), bulk=(0.225, 0.0, 0.0))
    p2, v2 = plummer(n2, seed + 7919, total_mass=0.75, center=(2.0, 0.0, 0.0), bulk=(-0.075, 0.0, 0.0))
    return np.concatenate([p1, p2]), np.concatenate([v1, v2])


def ragged_batch_sizes(nsys: int, seed: int, nmin: int = 256, nmax: int = 32768):
    """System sizes N_s = round(exp(U[ln nmin, ln nmax]))."""
    g = rng(seed)
    u = g.uniform(math.log(nmin), math.log(nmax), size=nsys)
    return np.rint(np.exp(u)).astype(np.int64)


def ragged_batch(nsys: int, seed: int, nmin: int = 256, nmax: int = 32768):
    """Concatenated independent Plummer systems (unit mass and scale radius
    each) and the int64 offsets array of length nsys+1."""
    sizes = ragged_batch_sizes(nsys, seed, nmin, nmax)
    offsets = np.zeros(nsys + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    ps, vs = [], []
    for s, ns in enumerate(sizes):
        p, v = plummer(int(ns), seed * 100003 + s + 1)
        ps.append(p)
        vs.append(v)
    return np.concatenate(ps), np.concatenate(vs), offsets


def perturbed_snapshot(pos_mass: np.ndarray, seed: int, sigma: float = 0.01) -> np.ndarray:
    """Target positions y = x + sigma * xi, xi ~ N(0, I3), shape (N, 3)."""
    g = rng(seed)
    return pos_mass[:, :3] + sigma * g.standard_normal(size=(pos_mass.shape[0], 3))


def sample_targets(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct target indices out of n (all of them, in order, if k >= n)."""
    if k >= n:
        return np.arange(n, dtype=np.int64)
    return np.sort(rng(seed).choice(n, size=k, replace=False)).astype(np.int64)


def kepler_pair(e: float = 0.0):
    """Two bodies of mass 1/2 on a Kepler orbit of eccentricity e with
    semi-major axis 1 (G = 1, total mass 1, period 2 pi), started at
    pericentre on the x axis, centre of mass at rest at the origin."""
    rp = 1.0 - e
    vrel = math.sqrt((1.0 + e) / (1.0 - e))  # vis-viva at pericentre, a = 1
    pos = np.array([[-rp / 2, 0, 0, 0.5], [rp / 2, 0, 0, 0.5]], dtype=np.float64)
    vel = np.array([[0, -vrel / 2, 0, 0], [0, vrel / 2, 0, 0]], dtype=np.float64)
    return pos, vel


# Synthetic workloads, one per measured or parity-tested configuration.
# seed = 1000 + k for workload k; sampled targets use seed + 1.
WORKLOADS = {
    "ball4096_f64": dict(kind="uniform_ball", n=4096, seed=1000, eps=0.01, dt=1e-3, steps=10),
    "plummer65536": dict(kind="plummer", n=65536, seed=1001, eps=0.01, dt=1e-3, steps=100),
    "collide1m": dict(kind="colliding_pair", n=1 << 20, seed=1002, eps=0.005, dt=5e-4, steps=20),
    "adjoint16384": dict(kind="plummer", n=16384, seed=1003, eps=0.01, dt=1e-3, steps=200, ckpt=20),
    "batch512": dict(kind="ragged_batch", nsys=512, seed=1004, eps=0.01, dt=1e-3, steps=50),
}

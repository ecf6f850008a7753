"""Problem configurations and seeded plane waves.

A problem bundles everything the solver boundary consumes: the mesh and
its edge table, eps_r, mu_r, dt, the static blocks T0s, T0h on the BC basis,
the Gram matrix G, the raw retarded blocks of both media and the incident
Gaussian plane waves (eq. hin).  Units are normalised: the exterior medium
has c = eta = 1.

Gaussian width: a configuration gives the temporal standard deviation sigma;
the paper's width is then w = 4 sqrt(2) c sigma, so that
(4/w)^2 (c t)^2 = t^2 / (2 sigma^2).
"""
from __future__ import annotations

import math
import os
import numpy as np

from . import geometry as geo
from . import bc as bcmod

MASTER_SEED = 251007989

__all__ = ["CONFIGS", "Wave", "make_mesh", "make_waves", "build_problem", "medium", "tmax_kmax"]


class Wave:
    """Gaussian plane wave: amplitude, polarisation p, direction k, width w, t0."""

    def __init__(self, amp, pol, dirn, width, t0):
        self.amp = float(amp)
        self.pol = np.asarray(pol, dtype=np.float64)
        self.dir = np.asarray(dirn, dtype=np.float64)
        self.width = float(width)
        self.t0 = float(t0)

    def as_row(self):
        return np.concatenate([[self.amp], self.pol, self.dir, [self.width, self.t0]])


CONFIGS = {
    # tiny cases for brute-force checks
    "tiny": dict(mesh=("icosphere", 1), eps_r=2.0, mu_r=1.0, dt=0.5, nsteps=40, nrhs=1, sigma=1.0, nq=7),
    "tiny_torus": dict(mesh=("torus", 1.0, 0.4, 12, 6), eps_r=3.0, mu_r=1.0, dt=0.5, nsteps=40, nrhs=1, sigma=1.0, nq=7),
    "tiny_box": dict(mesh=("box", 2, 2, 2), eps_r=5.0, mu_r=1.0, dt=0.5, nsteps=40, nrhs=2, sigma=1.0, nq=12, seeded=True),
    # sphere, 320 triangles / 480 edges: plain FP64, 1 RHS
    "sphere_480": dict(mesh=("icosphere", 4), eps_r=2.0, mu_r=1.0, dt=0.25, nsteps=200, nrhs=1, sigma=1.0, nq=7),
    "sphere_480_r16": dict(mesh=("icosphere", 4), eps_r=2.0, mu_r=1.0, dt=0.25, nsteps=120, nrhs=16, sigma=1.0, nq=7, seeded=True),
    # sphere, 1280 triangles / 1920 edges, 16 seeded plane waves (multi-RHS benchmark size)
    "sphere_1920_r16": dict(mesh=("icosphere", 8), eps_r=2.0, mu_r=1.0, dt=0.15, nsteps=400, nrhs=16, sigma=0.6, nq=7, seeded=True),
    # torus, 2048 triangles / 3072 edges, large timestep, 10^4 steps
    "torus_3072": dict(mesh=("torus", 1.0, 0.4, 64, 16), eps_r=4.0, mu_r=1.0, dt=2.0, nsteps=10000, nrhs=1, sigma=8.0, nq=7),
    # sphere, 5120 triangles / 7680 edges, 64 RHS
    "sphere_7680": dict(mesh=("icosphere", 16), eps_r=2.0, mu_r=1.0, dt=0.1, nsteps=1000, nrhs=64, sigma=0.4, nq=7, seeded=True),
    # sharp-edged cube, 10240 triangles / 15360 edges, 16 RHS
    "cube_15360": dict(mesh=("box", 32, 32, 24), eps_r=4.0, mu_r=1.0, dt=0.5, nsteps=5000, nrhs=16, sigma=2.0, nq=12, seeded=True),
    # star-based pyramid (24 base vertices on radii 1 and 0.3, height 0.5), eps_r = 5, c dt = 2 m
    "tiny_pyramid": dict(mesh=("star_pyramid", 12, 1.0, 0.3, 0.5, 1), eps_r=5.0, mu_r=1.0, dt=2.0, nsteps=60, nrhs=1, sigma=2.0, nq=12),
    "pyramid_648": dict(mesh=("star_pyramid", 12, 1.0, 0.3, 0.5, 3), eps_r=5.0, mu_r=1.0, dt=2.0, nsteps=300, nrhs=1, sigma=4.0, nq=12),
    # the same pyramid with c dt / D about 1/8 (k_max 18): thin retarded shells, many lags
    "pyramid_648_fine": dict(mesh=("star_pyramid", 12, 1.0, 0.3, 0.5, 3), eps_r=5.0, mu_r=1.0, dt=0.25, nsteps=150, nrhs=1, sigma=4.0, nq=12),
    "pyramid_2592_fine": dict(mesh=("star_pyramid", 12, 1.0, 0.3, 0.5, 6), eps_r=5.0, mu_r=1.0, dt=0.2, nsteps=1000, nrhs=1, sigma=4.0, nq=12),
    # free-space interior: the exact solution is the projected incident trace
    "sphere_vacuum": dict(mesh=("icosphere", 3), eps_r=1.0, mu_r=1.0, dt=0.2, nsteps=80, nrhs=1, sigma=0.6, nq=7),
}


def make_mesh(spec):
    kind = spec[0]
    if kind == "icosphere":
        V, F = geo.icosphere(spec[1])
    elif kind == "torus":
        V, F = geo.torus(*spec[1:])
    elif kind == "box":
        V, F = geo.box(*spec[1:])
    elif kind == "star_pyramid":
        V, F = geo.star_pyramid(*spec[1:])
    else:
        raise ValueError(kind)
    E = geo.edge_table(F)
    geo.check_mesh(V, F, E)
    return V, F, E


def medium(eps_r, mu_r):
    """Exterior c = eta = 1; interior c' = 1/sqrt(eps mu), eta' = sqrt(mu/eps)."""
    return 1.0, 1.0, 1.0 / math.sqrt(eps_r * mu_r), math.sqrt(mu_r / eps_r)


def tmax_kmax(D, dt, eps_r, mu_r):
    _, _, cp, _ = medium(eps_r, mu_r)
    Tmax = D / min(1.0, cp)
    kmax = int(math.ceil(Tmax / dt - 1e-12))
    return Tmax, kmax


def make_waves(nrhs, sigma, seeded, seed=MASTER_SEED):
    """nrhs Gaussian plane waves.  Unseeded: p = x, k = -z.  Seeded: k uniform
    on the sphere (normalised N(0, I)), p uniform on the circle normal to k."""
    c = 1.0
    w = 4.0 * math.sqrt(2.0) * c * sigma
    t0 = 6.0 * sigma
    waves = []
    if not seeded:
        for _ in range(nrhs):
            waves.append(Wave(1.0, [1, 0, 0], [0, 0, -1], w, t0))
        return waves
    rng = np.random.Generator(np.random.PCG64(seed))
    for _ in range(nrhs):
        k = rng.standard_normal(3)
        k /= np.linalg.norm(k)
        a = np.array([1.0, 0, 0]) if abs(k[0]) < 0.9 else np.array([0, 1.0, 0])
        u = np.cross(k, a); u /= np.linalg.norm(u)
        v = np.cross(k, u)
        phi = rng.uniform(0, 2 * math.pi)
        p = math.cos(phi) * u + math.sin(phi) * v
        waves.append(Wave(1.0, p, k, w, t0))
    return waves


def build_problem(name=None, cfg=None, nsteps=None, with_raw=True, threads=None, verbose=False):
    """Assemble every input of a configuration (CPU, OpenMP)."""
    import sys
    import time
    from . import retarded_blocks, static_blocks

    def say(msg):
        if verbose:
            print("[inputs] " + msg, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    if threads:
        os.environ["OMP_NUM_THREADS"] = str(threads)
    cfg = dict(CONFIGS[name] if cfg is None else cfg)
    V, F, E = make_mesh(cfg["mesh"])
    eps_r, mu_r, dt = cfg["eps_r"], cfg["mu_r"], cfg["dt"]
    D = geo.diameter(V)
    Tmax, kmax = tmax_kmax(D, dt, eps_r, mu_r)
    c, eta, cp, etap = medium(eps_r, mu_r)
    say("%s: %d triangles, %d edges, k_max %d" % (name, F.shape[0], E.shape[0], kmax))
    R = bcmod.refine(V, F, E)
    G = bcmod.gram_bc(V, F, E, R)
    say("BC basis and Gram matrix (%.1f s)" % (time.perf_counter() - t0))
    T0s, T0h = static_blocks(R, D, nq=6)
    say("static blocks (%.1f s)" % (time.perf_counter() - t0))
    prob = dict(name=name, V=V, F=F, E=E, eps_r=eps_r, mu_r=mu_r, dt=dt, D=D, Tmax=Tmax,
                kmax=kmax, G=G, T0s=T0s, T0h=T0h, refinement=R,
                nsteps=cfg["nsteps"] if nsteps is None else nsteps,
                waves=make_waves(cfg["nrhs"], cfg["sigma"], cfg.get("seeded", False)))
    if with_raw:
        raw = {}
        for med, speed in (("ext", c), ("int", cp)):
            raw[med] = retarded_blocks(V, F, E, dt, speed, kmax + 1, kmax + 2, kmax, nq=cfg.get("nq", 7))
            say("retarded blocks, %s medium (%.1f s)" % (med, time.perf_counter() - t0))
        prob["raw"] = raw
    return prob

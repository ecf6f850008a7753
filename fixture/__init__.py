"""Seeded synthetic inputs for the qHP TD-PMCHWT marching-on-in-time solver.

The solver's boundary takes a surface mesh with its edge table, the static
preconditioner blocks on the Buffa-Christiansen basis, the Gram matrix and
the per-medium retarded lag blocks.  This package produces all of them:

* ``geometry`` - closed meshes (icosphere, torus, box) and edge tables;
* ``bc``       - barycentric refinement, BC restrictions, the Gram matrix;
* ``assemble.c`` - Galerkin quadrature of the retarded families (h, hat,
  tilde) and of the static T0s / T0h blocks, built with gcc + OpenMP;
* ``problem``  - configurations and plane waves (seeded).

It contains no part of the marching scheme itself (no projector, no
preconditioner product, no lag-matrix fold, no march, no recovery).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import numpy as np

from . import geometry, bc  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "assemble.c")
_LIB = os.path.join(_HERE, "_assemble.so")
_lib = None


def build(force: bool = True, gpu: bool = True) -> str:
    """Compile the host assembler (gcc, OpenMP) and, with gpu, the device
    assembler (hipcc, gfx950)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-fPIC", "-shared",
               "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    if gpu:
        from . import gpu as _gpu
        _gpu.build(force=force)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        lib.fx_retarded.argtypes = [I, P, I, P, I, P, P, P, I, D, D, I, I, I, I, I, I,
                                    P, P, P, P, P, P]
        lib.fx_retarded.restype = I
        lib.fx_static_bc.argtypes = [I, P, P, P, P, P, I, P, P, D, I, I, I, I, P, P]
        lib.fx_static_bc.restype = I
        lib.fx_rule.argtypes = [I, P, P]
        lib.fx_rule.restype = I
        lib.fx_inner_test.argtypes = [P, P, P, I, I, I, I, P]
        lib.fx_inner_test.restype = I
        lib.fx_temporal.argtypes = [D, D, P]
        lib.fx_temporal.restype = I
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def face_coloring(F, E):
    """Greedy colouring of the face graph (faces sharing an edge differ)."""
    nf = F.shape[0]
    nbr = [[] for _ in range(nf)]
    for cp, cm in E[:, 2:4]:
        nbr[cp].append(cm)
        nbr[cm].append(cp)
    col = -np.ones(nf, dtype=np.int64)
    for f in range(nf):
        used = {col[g] for g in nbr[f]}
        c = 0
        while c in used:
            c += 1
        col[f] = c
    order = np.argsort(col, kind="stable").astype(np.int32)
    ncol = int(col.max()) + 1
    ptr = np.zeros(ncol + 1, dtype=np.int32)
    ptr[1:] = np.cumsum(np.bincount(col, minlength=ncol))
    return order, ptr


def triangle_rule(nq):
    lib = _load()
    l = np.zeros((16, 3))
    w = np.zeros(16)
    n = lib.fx_rule(nq, _ptr(l), _ptr(w))
    if n < 0:
        raise ValueError("no rule with %d points" % nq)
    return l[:n].copy(), w[:n].copy()


def inner_test(x, tri, bps=None, near=1, nth=6, nrh=6):
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    tv = np.ascontiguousarray(tri, dtype=np.float64)
    b = np.ascontiguousarray([] if bps is None else bps, dtype=np.float64)
    out = np.zeros(4)
    lib.fx_inner_test(_ptr(x), _ptr(tv), _ptr(b) if b.size else None, b.size, near, nth, nrh, _ptr(out))
    return out


def temporal(u, dt):
    """(h0, hdot0, q0, qdot0, qddot0, p0, P) at tau = u dt, as the assembler uses them."""
    lib = _load()
    out = np.zeros(7)
    lib.fx_temporal(float(u), float(dt), _ptr(out))
    return out


def retarded_blocks(V, F, E, dt, c, nh, nhat, ntil, nq=7, nth=5, nrh=5, which=None):
    """Raw retarded blocks of one medium (speed c) for lags 0..n*-1.

    Returns a dict with keys 'T_h','K_h','T_hat','K_hat','T_tilde','K_tilde',
    each an array of shape (nlags, ne, ne) (float64, row-major).
    """
    lib = _load()
    V = np.ascontiguousarray(V, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.int32)
    E = np.ascontiguousarray(E, dtype=np.int32)
    ne = E.shape[0]
    order, ptr = face_coloring(F, E)
    names = ["T_h", "K_h", "T_hat", "K_hat", "T_tilde", "K_tilde"]
    counts = [nh, nh, nhat, nhat, ntil, ntil]
    out = {}
    bufs = []
    for nm, k in zip(names, counts):
        if (which is None or nm in which) and k > 0:
            out[nm] = np.zeros((k, ne, ne))
            bufs.append(out[nm])
        else:
            bufs.append(None)
    rc = lib.fx_retarded(V.shape[0], _ptr(V), F.shape[0], _ptr(F), ne, _ptr(E),
                         _ptr(order), _ptr(ptr), ptr.size - 1, float(dt), float(c),
                         int(nh), int(nhat), int(ntil), int(nq), int(nth), int(nrh),
                         *[_ptr(b) for b in bufs])
    if rc:
        raise RuntimeError("fx_retarded failed: %d" % rc)
    for k in out:
        # the Galerkin blocks are symmetric in exact arithmetic
        out[k] = 0.5 * (out[k] + np.transpose(out[k], (0, 2, 1)))
    return out


def static_blocks(R, D, nq=6, nth=5, nrh=5, chunk=1024):
    """T0s, T0h on the BC basis (dense, symmetrised)."""
    lib = _load()
    nft = R.fverts.shape[0]
    ne = R.ne
    order = np.argsort(R.bc_t, kind="stable")
    bct = R.bc_t[order]
    bcn = np.ascontiguousarray(R.bc_n[order], dtype=np.int32)
    bca = np.ascontiguousarray(R.bc_a[order])
    bcb = np.ascontiguousarray(R.bc_b[order])
    rowptr = np.zeros(nft + 1, dtype=np.int32)
    rowptr[1:] = np.cumsum(np.bincount(bct, minlength=nft))
    byn = np.argsort(bcn, kind="stable").astype(np.int32)
    byn_ptr = np.zeros(ne + 1, dtype=np.int32)
    byn_ptr[1:] = np.cumsum(np.bincount(bcn, minlength=ne))
    fv = np.ascontiguousarray(R.fverts)
    T0s = np.zeros((ne, ne))
    T0h = np.zeros((ne, ne))
    rc = lib.fx_static_bc(nft, _ptr(fv), _ptr(rowptr), _ptr(bcn), _ptr(bca), _ptr(bcb), ne,
                          _ptr(byn_ptr), _ptr(byn), float(D), int(nq), int(nth), int(nrh),
                          int(chunk), _ptr(T0s), _ptr(T0h))
    if rc:
        raise RuntimeError("fx_static_bc failed: %d" % rc)
    return 0.5 * (T0s + T0s.T), 0.5 * (T0h + T0h.T)

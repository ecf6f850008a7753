"""Device assembly of the solver's inputs (input generator).

``gpu_assemble.hip`` evaluates the same quadrature as ``assemble.c`` on the
GPU: the retarded h / hat / tilde blocks of one medium, one lag at a time
(Section V-B), and the static blocks T0s, T0h on the BC basis (Section III).
The Gauss-Legendre and triangle-rule tables are taken from the host
assembler, so both build the same point sets and differ only in the order of
their sums.

Outputs are torch tensors on the current CUDA (HIP) device.  Like the host
fixture, this module holds no part of the marching scheme.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import _load as _load_host, _ptr, face_coloring, triangle_rule

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gpu_assemble.hip")
_LIB = os.path.join(_HERE, "_gpu_assemble.so")
_lib = None

FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-Wno-unused-value", "-shared"]

BLOCK_NAMES = ("T_h", "K_h", "T_hat", "K_hat", "T_tilde", "K_tilde")


def build(force: bool = True) -> str:
    """Compile the device assembler for gfx950 (hipcc)."""
    if force or not os.path.exists(_LIB):
        hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([hipcc, *FLAGS, "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise RuntimeError("fixture/_gpu_assemble.so is not built (fixture.gpu.build())")
        import torch  # noqa: F401  (one HIP runtime: torch's)
        lib = ctypes.CDLL(_LIB)
        P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        lib.gfx_ret_create.argtypes = [I, P, I, P, I, P, P, P, I, D, D, I, I, I, I, I, I, P, P, P, P, P,
                                       ctypes.POINTER(P)]
        lib.gfx_ret_create.restype = I
        lib.gfx_ret_lag.argtypes = [P, I, P]
        lib.gfx_ret_lag.restype = I
        lib.gfx_ret_destroy.argtypes = [P]
        lib.gfx_ret_destroy.restype = None
        lib.gfx_static_bc.argtypes = [I, P, I, P, P, P, P, I, D, I, I, I, P, P, P, P, I, P, P, P]
        lib.gfx_static_bc.restype = I
        _lib = lib
    return _lib


def _tables():
    host = _load_host()
    host.fx_gl_tables.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    host.fx_gl_tables.restype = ctypes.c_int
    x = np.zeros((13, 12))
    w = np.zeros((13, 12))
    host.fx_gl_tables(_ptr(x), _ptr(w))
    return x, w


def _rule_table(nq):
    l, w = triangle_rule(nq)
    return np.ascontiguousarray(np.concatenate([l, w[:, None]], axis=1))


class RetardedAssembler:
    """Retarded blocks of one medium (wave speed c) on the device, lag by lag.

    Lags must be requested in increasing order, 0, 1, 2, ...: the device
    processes one shell band per call, whose points add to three consecutive
    lags, so the blocks live in a ring of three lags (18 device arrays of
    ne x ne doubles) held by this object.  The tensors returned for lag i are
    views of the ring, valid until the next call.
    """

    def __init__(self, V, F, E, dt, c, nh, nhat, ntil, nq=7, nth=5, nrh=5):
        import torch
        lib = _load()
        self.V = np.ascontiguousarray(V, dtype=np.float64)
        self.F = np.ascontiguousarray(F, dtype=np.int32)
        self.E = np.ascontiguousarray(E, dtype=np.int32)
        self.ne = self.E.shape[0]
        self.limits = (nh, nh, nhat, nhat, ntil, ntil)
        self.nlag = max(nh, nhat, ntil)
        order, ptr = face_coloring(self.F, self.E)
        self._order = np.ascontiguousarray(order, dtype=np.int32)
        self._ptr = np.ascontiguousarray(ptr, dtype=np.int32)
        glx, glw = _tables()
        rule = _rule_table(nq)
        far = _rule_table(7)
        self.stream = torch.cuda.current_stream()
        self.ring = torch.empty((3, 6, self.ne, self.ne), dtype=torch.float64, device="cuda")
        self._ring_ptrs = (ctypes.c_void_p * 18)(*[self.ring[j // 6, j % 6].data_ptr() for j in range(18)])
        h = ctypes.c_void_p()
        rc = lib.gfx_ret_create(self.V.shape[0], _ptr(self.V), self.F.shape[0], _ptr(self.F), self.ne,
                                _ptr(self.E), _ptr(self._order), _ptr(self._ptr), self._ptr.size - 1,
                                float(dt), float(c), int(nh), int(nhat), int(ntil), int(nq), int(nth),
                                int(nrh), _ptr(glx), _ptr(glw), _ptr(rule), _ptr(far),
                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc:
            raise RuntimeError("gfx_ret_create failed: %d" % rc)
        self._h = h
        self.next_lag = 0

    def lag(self, i):
        """Blocks of lag i as {name: (ne, ne) float64 CUDA tensor}, for the
        families whose range holds i (views of the ring, valid until the next
        call)."""
        lib = _load()
        rc = lib.gfx_ret_lag(self._h, int(i), self._ring_ptrs)
        if rc:
            raise RuntimeError("gfx_ret_lag(%d) failed: %d" % (i, rc))
        self.next_lag = i + 1
        slot = i % 3
        return {name: self.ring[slot, b] for b, (name, lim) in enumerate(zip(BLOCK_NAMES, self.limits))
                if i < lim}

    def close(self):
        if self._h:
            _load().gfx_ret_destroy(self._h)
            self._h = None
        self.ring = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def static_blocks(R, D, nq=6, nth=5, nrh=5, chunk=512):
    """T0s, T0h on the BC basis as (ne, ne) float64 CUDA tensors (symmetrised),
    by the host assembler's quadrature (fixture.static_blocks)."""
    import torch
    lib = _load()
    nft = R.fverts.shape[0]
    ne = R.ne
    order = np.argsort(R.bc_t, kind="stable")
    res_t = np.ascontiguousarray(R.bc_t[order], dtype=np.int32)
    res_n = np.ascontiguousarray(R.bc_n[order], dtype=np.int32)
    res_a = np.ascontiguousarray(R.bc_a[order], dtype=np.float64)
    res_b = np.ascontiguousarray(R.bc_b[order], dtype=np.float64)
    fv = np.ascontiguousarray(R.fverts, dtype=np.float64)
    glx, glw = _tables()
    rule = _rule_table(nq)
    far = _rule_table(3)
    T0s = torch.empty((ne, ne), dtype=torch.float64, device="cuda")
    T0h = torch.empty((ne, ne), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    rc = lib.gfx_static_bc(nft, _ptr(fv), res_t.size, _ptr(res_t), _ptr(res_n), _ptr(res_a), _ptr(res_b),
                           ne, float(D), int(nq), int(nth), int(nrh), _ptr(glx), _ptr(glw), _ptr(rule),
                           _ptr(far), int(chunk), ctypes.c_void_p(stream.cuda_stream),
                           ctypes.c_void_p(T0s.data_ptr()), ctypes.c_void_p(T0h.data_ptr()))
    if rc:
        raise RuntimeError("gfx_static_bc failed: %d" % rc)
    return T0s, T0h


def upload_lags(upload, V, F, E, dt, eps_r, mu_r, kmax, nq=7, nth=5, nrh=5, lags=None, on_lag=None):
    """Assemble the retarded blocks of both media on the device, lag by lag,
    and hand each to upload(family, lag, medium, op, tensor) with the codes of
    the solver's C ABI (family 0 h, 1 hat, 2 tilde; medium 0 exterior, 1
    interior; op 0 T, 1 K).  Ranges: h 0..k_max, hat 0..k_max+1, tilde
    0..k_max-1 (Section V-B truncations).  A lag's tensors are released once
    uploaded (each medium keeps a ring of three lags on the device).
    lags: number of leading lags to assemble (default all, k_max + 2).
    on_lag(i): called after lag i is uploaded."""
    from .problem import medium
    c, _, cp, _ = medium(eps_r, mu_r)
    nh, nhat, ntil = kmax + 1, kmax + 2, kmax
    nl = kmax + 2 if lags is None else int(lags)
    asm = [RetardedAssembler(V, F, E, dt, speed, nh, nhat, ntil, nq=nq, nth=nth, nrh=nrh)
           for speed in (c, cp)]
    codes = {"T_h": (0, 0), "K_h": (0, 1), "T_hat": (1, 0), "K_hat": (1, 1), "T_tilde": (2, 0),
             "K_tilde": (2, 1)}
    try:
        for i in range(nl):
            for med, a in enumerate(asm):
                blocks = a.lag(i)
                a.stream.synchronize()
                for name, t in blocks.items():
                    fam, op = codes[name]
                    upload(fam, i, med, op, t)
                del blocks
            if on_lag is not None:
                on_lag(i)
    finally:
        for a in asm:
            a.close()


def device_inputs(V, F, E, nq_static=6):
    """Host BC refinement and Gram matrix, and the static blocks assembled on
    the device (returned as host arrays): the keys G, T0s, T0h, D, refinement."""
    import torch
    from . import geometry as geo, bc as bcmod
    D = geo.diameter(V)
    R = bcmod.refine(V, F, E)
    G = bcmod.gram_bc(V, F, E, R)
    T0s, T0h = static_blocks(R, D, nq=nq_static)
    torch.cuda.current_stream().synchronize()
    out = dict(G=G, T0s=T0s.cpu().numpy(), T0h=T0h.cpu().numpy(), D=D, refinement=R)
    del T0s, T0h
    torch.cuda.empty_cache()       # give the blocks back to the device, not to torch's cache
    return out


def build_problem_device(name=None, cfg=None, nsteps=None):
    """Inputs of a configuration with the static blocks assembled on the device
    and no retarded blocks (those are streamed by upload_lags): the keys of
    fixture.problem.build_problem except 'raw'.  T0s, T0h are returned as
    host arrays, as the solver's create call takes them."""
    import torch
    from .problem import CONFIGS, make_mesh, make_waves, tmax_kmax
    from . import geometry as geo, bc as bcmod
    cfg = dict(CONFIGS[name] if cfg is None else cfg)
    V, F, E = make_mesh(cfg["mesh"])
    eps_r, mu_r, dt = cfg["eps_r"], cfg["mu_r"], cfg["dt"]
    D = geo.diameter(V)
    Tmax, kmax = tmax_kmax(D, dt, eps_r, mu_r)
    R = bcmod.refine(V, F, E)
    G = bcmod.gram_bc(V, F, E, R)
    T0s, T0h = static_blocks(R, D, nq=6)
    torch.cuda.synchronize()
    prob = dict(name=name, V=V, F=F, E=E, eps_r=eps_r, mu_r=mu_r, dt=dt, D=D, Tmax=Tmax, kmax=kmax, G=G,
                T0s=T0s.cpu().numpy(), T0h=T0h.cpu().numpy(), refinement=R, nq=cfg.get("nq", 7),
                nsteps=cfg["nsteps"] if nsteps is None else nsteps,
                waves=make_waves(cfg["nrhs"], cfg["sigma"], cfg.get("seeded", False)))
    del T0s, T0h
    torch.cuda.empty_cache()
    return prob


def load_solvers(solvers, prob, lags=None, on_lag=None):
    """One device assembly pass of prob's retarded blocks (both media, lag by
    lag) handed to every solver in turn through its set_lag_device."""
    import torch

    def upload(fam, lag, med, op, t):
        for s in solvers:
            s.set_lag_device(fam, lag, med, op, t)
    upload_lags(upload, prob["V"], prob["F"], prob["E"], prob["dt"], prob["eps_r"], prob["mu_r"], prob["kmax"],
                nq=prob.get("nq", 7), lags=lags, on_lag=on_lag)
    # the assembler's rings go back to the device (the solvers allocate outside torch)
    torch.cuda.empty_cache()

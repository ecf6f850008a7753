"""Python front-end of the C ABI (argument marshalling only)."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib as L


class MotError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("mot error %d: %s" % (code, msg))
        self.code = code


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def default_options(**kw):
    lib = L.load()
    o = L.MotOptions()
    lib.mot_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _csr(G):
    import scipy.sparse as sp
    A = sp.csr_matrix(G)
    A.sum_duplicates()
    return (np.ascontiguousarray(A.indptr, dtype=np.int32), np.ascontiguousarray(A.indices, dtype=np.int32),
            np.ascontiguousarray(A.data, dtype=np.float64))


def footprint(V, F, E, eps_r, mu_r, dt, nrhs, G, options=None, gnnz=None):
    """Device bytes (resident, peak) that a Solver with these arguments will
    hold, from mot_footprint: nothing is allocated.  gnnz: the Gram matrix's
    nonzero count, or a bound on it, when G itself is not built yet (G None)."""
    lib = L.load()
    V = np.ascontiguousarray(V, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.int32)
    E = np.ascontiguousarray(E, dtype=np.int32)
    mesh = L.MotMesh(V.shape[0], F.shape[0], E.shape[0], _ptr(V), _ptr(F), _ptr(E))
    nnz = int(gnnz) if gnnz is not None else len(_csr(G)[1])
    opt = options if options is not None else default_options()
    res, peak = ctypes.c_uint64(), ctypes.c_uint64()
    rc = lib.mot_footprint(ctypes.byref(mesh), float(eps_r), float(mu_r), float(dt), int(nrhs), int(nnz),
                           ctypes.byref(opt), ctypes.byref(res), ctypes.byref(peak))
    if rc:
        raise MotError(rc, lib.mot_last_error(None).decode())
    return int(res.value), int(peak.value)


class Solver:
    """One scattering problem on the current HIP device.

    mesh: (V [nv,3] float64, F [nf,3] int, E [ne,4] int) with the edge-table
    convention of include/mot.h.  G may be dense or scipy-sparse.  waves: objects
    with amp, pol, dir, width, t0 (see fixture.problem.Wave).
    """

    def __init__(self, V, F, E, eps_r, mu_r, dt, T0s, T0h, G, waves, options=None, stream=None):
        self._lib = L.load()
        self._h = ctypes.c_void_p()
        V = np.ascontiguousarray(V, dtype=np.float64)
        F = np.ascontiguousarray(F, dtype=np.int32)
        E = np.ascontiguousarray(E, dtype=np.int32)
        self.ne = E.shape[0]
        self.n = 2 * self.ne
        self.nrhs = len(waves)
        mesh = L.MotMesh(V.shape[0], F.shape[0], E.shape[0], _ptr(V), _ptr(F), _ptr(E))
        T0s = np.ascontiguousarray(T0s, dtype=np.float64)
        T0h = np.ascontiguousarray(T0h, dtype=np.float64)
        gp, gc, gv = _csr(G)
        W = (L.MotPlaneWave * len(waves))()
        for i, w in enumerate(waves):
            W[i].amp = w.amp
            W[i].pol[:] = list(np.asarray(w.pol, dtype=float))
            W[i].dir[:] = list(np.asarray(w.dir, dtype=float))
            W[i].width = w.width
            W[i].t0 = w.t0
        opt = options if options is not None else default_options()
        self._keep = (V, F, E)
        rc = self._lib.mot_create(ctypes.byref(mesh), float(eps_r), float(mu_r), float(dt), _ptr(T0s),
                                  _ptr(T0h), _ptr(gp), _ptr(gc), _ptr(gv), len(waves), W, ctypes.byref(opt),
                                  ctypes.c_void_p(stream) if stream else None, ctypes.byref(self._h))
        if rc:
            raise MotError(rc, self._lib.mot_last_error(None).decode())

    # ------------------------------------------------------------------
    def _check(self, rc, ok=(L.MOT_OK,)):
        if rc not in ok:
            raise MotError(rc, self._lib.mot_last_error(self._h).decode())
        return rc

    def set_lag(self, family, lag, medium, op, block):
        block = np.ascontiguousarray(block, dtype=np.float64)
        if block.shape != (self.ne, self.ne):
            raise ValueError("block must be ne x ne")
        return self._check(self._lib.mot_set_lag(self._h, family, lag, medium, op, _ptr(block)))

    def set_lag_csr(self, family, lag, medium, op, A):
        import scipy.sparse as sp
        A = sp.csr_matrix(A)
        p = np.ascontiguousarray(A.indptr, dtype=np.int64)
        c = np.ascontiguousarray(A.indices, dtype=np.int32)
        v = np.ascontiguousarray(A.data, dtype=np.float64)
        return self._check(self._lib.mot_set_lag_csr(self._h, family, lag, medium, op, _ptr(p), _ptr(c), _ptr(v)))

    def set_lag_device(self, family, lag, medium, op, block):
        """block: an (ne, ne) float64 tensor in device memory whose producing
        work is complete or ordered before this solver's stream."""
        if tuple(block.shape) != (self.ne, self.ne) or block.dtype.itemsize != 8:
            raise ValueError("block must be an ne x ne float64 device tensor")
        ld = int(block.stride(0))
        if int(block.stride(1)) != 1:
            raise ValueError("block rows must be contiguous")
        return self._check(self._lib.mot_set_lag_device(self._h, family, lag, medium, op,
                                                        ctypes.c_void_p(block.data_ptr()), ld))

    def load_raw(self, raw, kmax):
        """Upload every block of raw[medium][name][lag] within the families' ranges."""
        fams = (("h", L.FAM_H, kmax), ("hat", L.FAM_HAT, kmax + 1), ("tilde", L.FAM_TILDE, kmax - 1))
        for lag in range(kmax + 2):
            for fname, fid, lim in fams:
                if lag > lim:
                    continue
                for mname, mid in (("ext", L.MED_EXT), ("int", L.MED_INT)):
                    for oname, oid in (("T", L.OP_T), ("K", L.OP_K)):
                        self.set_lag(fid, lag, mid, oid, raw[mname]["%s_%s" % (oname, fname)][lag])

    def step(self):
        inf = L.MotStepInfo()
        rc = self._lib.mot_step(self._h, ctypes.byref(inf))
        self._check(rc, ok=(L.MOT_OK, L.MOT_ENOCONV))
        return dict(step=inf.step, iters=inf.gmres_iters, relres=inf.gmres_relres, converged=inf.converged)

    def _outputs(self, nsteps, w, loop, star, device):
        shape = (nsteps, self.n, self.nrhs)
        outs = {}
        ptrs = []
        if device:
            import torch
            for name, want in (("w", w), ("loop", loop), ("star", star)):
                t = torch.empty(shape, dtype=torch.float64, device="cuda") if want else None
                outs[name] = t
                ptrs.append(ctypes.c_void_p(t.data_ptr()) if want else None)
        else:
            for name, want in (("w", w), ("loop", loop), ("star", star)):
                a = np.empty(shape) if want else None
                outs[name] = a
                ptrs.append(_ptr(a) if want else None)
        return outs, ptrs

    def run(self, nsteps, w=True, loop=True, star=True, device=False):
        """March nsteps; return arrays of shape (nsteps, n, nrhs) (numpy, or torch on device).
        A run stopped by cancel() returns the completed steps only, with
        outs["cancelled"] True."""
        outs, ptrs = self._outputs(nsteps, w, loop, star, device)
        inf = L.MotStepInfo()
        k0 = self.info()["steps_done"]
        rc = self._lib.mot_run(self._h, int(nsteps), ptrs[0], ptrs[1], ptrs[2], 1 if device else 0, ctypes.byref(inf))
        self._check(rc, ok=(L.MOT_OK, L.MOT_ENOCONV, L.MOT_ECANCEL))
        outs["cancelled"] = rc == L.MOT_ECANCEL
        if outs["cancelled"]:
            done = self.info()["steps_done"] - k0
            for name in ("w", "loop", "star"):
                if outs[name] is not None:
                    outs[name] = outs[name][:done]
        outs["last"] = dict(step=inf.step, iters=inf.gmres_iters, relres=inf.gmres_relres, converged=inf.converged)
        outs["rc"] = rc
        return outs

    def cancel(self):
        """Stop a run in progress (from another thread) at its next window
        boundary, or the next run before its first window (mot_cancel)."""
        self._check(self._lib.mot_cancel(self._h))

    def steps(self, first, count, w=True, loop=True, star=True, device=False):
        """Outputs of the kept steps first .. first+count-1 (counted from 0), as run returns them."""
        outs, ptrs = self._outputs(count, w, loop, star, device)
        self._check(self._lib.mot_get_steps(self._h, int(first), int(count), ptrs[0], ptrs[1], ptrs[2],
                                            1 if device else 0))
        return outs

    def far_field(self, first, count, freq, dirs=None):
        """Spectra at freq of the loop and star currents of the kept steps
        first .. first+count-1 and the far field each radiates in the unit
        directions dirs (ndir, 3).  Returns dict(spec (2, n, nrhs) complex,
        field (ndir, nrhs, 2, 3) complex, rc)."""
        d = np.ascontiguousarray(np.zeros((0, 3)) if dirs is None else dirs, dtype=np.float64)
        nd = d.shape[0]
        field = np.zeros((max(nd, 1), self.nrhs, 2, 3, 2))
        spec = np.zeros((2, self.n, self.nrhs, 2))
        rc = self._lib.mot_far_field(self._h, int(first), int(count), float(freq), nd, _ptr(d) if nd else None,
                                     _ptr(field) if nd else None, _ptr(spec))
        self._check(rc, ok=(L.MOT_OK, L.MOT_ENOCONV))
        return dict(spec=spec[..., 0] + 1j * spec[..., 1], field=(field[..., 0] + 1j * field[..., 1])[:nd], rc=rc)

    def step_norms(self, first, count):
        """||w_s|| of the kept steps first .. first+count-1, shape (count, nrhs)."""
        out = np.empty((count, self.nrhs))
        self._check(self._lib.mot_step_norms(self._h, int(first), int(count), _ptr(out)))
        return out

    def step_norms_noalloc(self, first, count):
        """step_norms through the allocation-free call (mot_step_norms_noalloc):
        count * nrhs at most MOT_NOALLOC_DOUBLES."""
        out = np.empty((count, self.nrhs))
        self._check(self._lib.mot_step_norms_noalloc(self._h, int(first), int(count), _ptr(out)))
        return out

    def checkpoint(self, with_history=True):
        """State of the march after the steps taken so far (numpy uint8 buffer)."""
        n = ctypes.c_uint64()
        self._check(self._lib.mot_checkpoint_size(self._h, 1 if with_history else 0, ctypes.byref(n)))
        buf = np.empty(n.value, dtype=np.uint8)
        self._check(self._lib.mot_checkpoint(self._h, 1 if with_history else 0, _ptr(buf), n.value))
        return buf

    def restore(self, buf):
        """Resume the march from a checkpoint of a solver built from the same inputs."""
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(self._lib.mot_restore(self._h, _ptr(buf), buf.size))

    def matrix(self, which, lag=0):
        shape = (self.n, self.n) if which == 0 else ((self.n, self.nrhs) if which == 6 else (self.ne, self.ne))
        out = np.empty(shape)
        self._check(self._lib.mot_get_matrix(self._h, int(which), int(lag), _ptr(out)))
        return out

    def info(self):
        inf = L.MotInfo()
        self._check(self._lib.mot_get_info(self._h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in L.MotInfo._fields_}

    def reset(self):
        self._check(self._lib.mot_reset(self._h))

    def close(self):
        if self._h:
            self._lib.mot_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_batch(solvers, nsteps):
    """March every solver nsteps with their windows interleaved on the device
    (mot_run_batch); returns each solver's code (MOT_OK, MOT_ENOCONV, or
    MOT_ECANCEL for one stopped by cancel()) and raises MotError for the first
    solver that failed."""
    lib = L.load()
    n = len(solvers)
    hs = (ctypes.c_void_p * max(n, 1))(*[s._h.value for s in solvers])
    st = (ctypes.c_int32 * max(n, 1))()
    rc = lib.mot_run_batch(hs, n, int(nsteps), st)
    if rc == L.MOT_EINVAL and not any(st[i] for i in range(n)):
        raise MotError(rc, "mot_run_batch: bad argument")
    for i, s in enumerate(solvers):
        if st[i] not in (L.MOT_OK, L.MOT_ENOCONV, L.MOT_ECANCEL):
            raise MotError(st[i], lib.mot_last_error(s._h).decode())
    return [st[i] for i in range(n)]

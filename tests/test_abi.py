"""The C-ABI library loads on a host without a GPU and exports what include/mot.h declares."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "mot.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mot_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("mot_create", "mot_set_lag", "mot_step", "mot_run", "mot_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2510_07989_amd import _lib
    lib = _lib.load()
    for name in _declared():
        getattr(lib, name)          # raises AttributeError when missing
    assert sorted(_lib.EXPORTS) == sorted(_declared())


def test_default_options_without_gpu():
    import paper_2510_07989_amd as p
    o = p.default_options()
    assert o.gmres_tol == 1e-13 and o.gmres_restart == 40 and o.keep_history == 1
    # the last field: the ctypes layout reaches as far as the C struct
    assert o.mix_group == 4 and o.autotune == 1


def test_footprint_without_gpu():
    """mot_footprint plans sizes only (no device call): more waves, a longer
    kept history and the FP64 preconditioner need more; FP32 lag storage less."""
    import paper_2510_07989_amd as p
    from tests._problems import problem
    prob = problem("sphere_480")
    args = (prob["V"], prob["F"], prob["E"], prob["eps_r"], prob["mu_r"], prob["dt"])
    r1, k1 = p.footprint(*args, 1, prob["G"], p.default_options(max_steps=100))
    r16, _ = p.footprint(*args, 16, prob["G"], p.default_options(max_steps=100, precond=2))
    r16m, _ = p.footprint(*args, 16, prob["G"], p.default_options(max_steps=100, precond=2, precision=1))
    rlong, _ = p.footprint(*args, 1, prob["G"], p.default_options(max_steps=1000))
    r64, _ = p.footprint(*args, 1, prob["G"], p.default_options(max_steps=100, precond=2))
    assert 0 < r1 < k1
    assert r16 > r16m > r1
    assert rlong - r1 == 900 * 960 * 8          # kept history: steps x n x 8 bytes
    assert r64 - r1 == 960 * 960 * 4            # FP64 instead of FP32 approximate inverse
    # the autotuner's partial sums are sized for its largest K-chunk candidate
    r16f, _ = p.footprint(*args, 16, prob["G"], p.default_options(max_steps=100, precond=2, autotune=0))
    assert r16f <= r16
    r1f, _ = p.footprint(*args, 1, prob["G"], p.default_options(max_steps=100, autotune=0))
    assert r1f == r1                            # one RHS: schedules need no memory
    # the raw families of every lag >= 1 (up to three blocks each where the
    # folded form keeps one) outweigh the folded lags they replace
    rraw, kraw = p.footprint(*args, 1, prob["G"], p.default_options(max_steps=100, history_form=1))
    assert r1 < rraw < kraw


def test_one_hip_runtime_in_the_process():
    """After loading the library, one HIP runtime and one HSA runtime are mapped
    (PyTorch's), so torch streams and tensors are valid handles for it."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2510_07989_amd import _lib\n"
            "_lib.load()\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "libs = sorted(set(l.split()[-1] for l in maps if 'amdhip64' in l or 'hsa-runtime64' in l))\n"
            "print(len([l for l in libs if 'amdhip64' in l]), len([l for l in libs if 'hsa-runtime64' in l]))\n"
            % os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.stdout.split() == ["1", "1"], out.stdout + out.stderr


def test_argument_errors_without_gpu():
    """The entry points reject bad arguments before any device call: a null
    handle, negative sizes, a null handle array."""
    import ctypes
    from paper_2510_07989_amd import _lib
    lib = _lib.load()
    st = (ctypes.c_int32 * 2)()
    assert lib.mot_run_batch(None, 2, 10, st) == _lib.MOT_EINVAL
    assert lib.mot_run_batch(None, -1, 10, st) == _lib.MOT_EINVAL
    hs = (ctypes.c_void_p * 2)(None, None)
    assert lib.mot_run_batch(hs, 2, 10, st) == _lib.MOT_EINVAL       # null handles
    assert lib.mot_run_batch(hs, 0, 10, st) == _lib.MOT_OK           # nothing to march
    assert lib.mot_get_steps(None, 0, 1, None, None, None, 0) == _lib.MOT_EINVAL
    assert lib.mot_far_field(None, 0, 1, 0.1, 0, None, None, None) == _lib.MOT_EINVAL
    assert lib.mot_run(None, 1, None, None, None, 0, None) == _lib.MOT_EINVAL
    n = ctypes.c_uint64()
    assert lib.mot_checkpoint_size(None, 1, ctypes.byref(n)) == _lib.MOT_EINVAL
    assert lib.mot_checkpoint(None, 1, None, 0) == _lib.MOT_EINVAL
    assert lib.mot_restore(None, None, 0) == _lib.MOT_EINVAL
    assert lib.mot_step_norms(None, 0, 1, None) == _lib.MOT_EINVAL


def test_header_is_c99_and_links_from_c(tmp_path):
    """include/mot.h is plain C: a C99 program (pedantic, warnings as errors)
    includes it, links libmot.so and calls an entry point that needs no GPU."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    lib_dir = os.path.join(ROOT, "paper_2510_07989_amd")
    if not os.path.exists(os.path.join(lib_dir, "libmot.so")):
        pytest.skip("libmot.so not built")
    src = tmp_path / "use_mot.c"
    src.write_text(
        '#include "mot.h"\n'
        "int main(void) {\n"
        "    mot_options o;\n"
        "    uint64_t n = 0;\n"
        "    mot_default_options(&o);\n"
        "    if (o.gmres_restart != 40 || o.autotune != 1 || o.history_form != 0) return 1;\n"
        "    if (mot_checkpoint_size(NULL, 1, &n) != MOT_EINVAL) return 2;\n"
        "    if (mot_run_batch(NULL, 1, 1, NULL) != MOT_EINVAL) return 3;\n"
        "    return 0;\n"
        "}\n")
    exe = tmp_path / "use_mot"
    subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", os.path.join(ROOT, "include"),
                    str(src), "-o", str(exe), "-L", lib_dir, "-l:libmot.so", "-Wl,-rpath," + lib_dir],
                   check=True, capture_output=True, timeout=120)
    out = subprocess.run([str(exe)], capture_output=True, timeout=120)
    assert out.returncode == 0, out.stderr


def test_create_rejects_bad_inputs_without_gpu():
    """mot_create checks every host input before it allocates anything, so
    each malformed input below is MOT_EINVAL on a host without a GPU."""
    import ctypes
    import numpy as np
    from paper_2510_07989_amd import _lib
    from paper_2510_07989_amd.solver import _ptr, _csr
    from tests._problems import problem
    lib = _lib.load()
    prob = problem("tiny")
    V = np.ascontiguousarray(prob["V"], dtype=np.float64)
    F = np.ascontiguousarray(prob["F"], dtype=np.int32)
    E = np.ascontiguousarray(prob["E"], dtype=np.int32)
    ne = E.shape[0]
    T0 = np.ascontiguousarray(prob["T0s"], dtype=np.float64)
    T1 = np.ascontiguousarray(prob["T0h"], dtype=np.float64)
    rp, col, val = _csr(prob["G"])

    def wave(**kw):
        w = _lib.MotPlaneWave()
        w.amp, w.width, w.t0 = 1.0, 4.0, 6.0
        w.pol[:] = (1.0, 0.0, 0.0)
        w.dir[:] = (0.0, 0.0, -1.0)
        for k, v in kw.items():
            if k in ("pol", "dir"):
                getattr(w, k)[:] = v
            else:
                setattr(w, k, v)
        return w

    def create(V=V, F=F, E=E, rp=rp, col=col, val=val, w=None, dt=0.5, nrhs=1, **opts):
        m = _lib.MotMesh(V.shape[0], F.shape[0], E.shape[0], _ptr(V), _ptr(F), _ptr(E))
        h = ctypes.c_void_p()
        ws = (_lib.MotPlaneWave * nrhs)(*[w or wave() for _ in range(nrhs)])
        o = _lib.MotOptions()
        lib.mot_default_options(ctypes.byref(o))
        for k, v in opts.items():
            setattr(o, k, v)
        return lib.mot_create(ctypes.byref(m), 2.0, 1.0, dt, _ptr(T0), _ptr(T1), _ptr(rp), _ptr(col), _ptr(val),
                              nrhs, ws, ctypes.byref(o), None, ctypes.byref(h))

    bad_v = V.copy(); bad_v[3, 1] = np.nan
    bad_f = F.copy(); bad_f[2, 0] = -1
    bad_e = E.copy(); bad_e[4, 2] = F.shape[0] + 3
    flip = E.copy(); flip[0, [0, 1]] = flip[0, [1, 0]]          # orientation broken
    bad_rp = rp.copy(); bad_rp[5], bad_rp[6] = bad_rp[6], bad_rp[5] - 1
    bad_col = col.copy(); bad_col[7] = ne
    bad_val = val.copy(); bad_val[0] = np.inf
    cases = {
        "vertex": dict(V=bad_v), "triangle": dict(F=bad_f), "edge": dict(E=bad_e), "orientation": dict(E=flip),
        "rowptr": dict(rp=bad_rp), "column": dict(col=bad_col), "value": dict(val=bad_val),
        "width": dict(w=wave(width=-1.0)), "pol": dict(w=wave(pol=(1.0, 0.1, 0.0))),
        "dir": dict(w=wave(dir=(0.0, 0.0, -2.0))), "pol.dir": dict(w=wave(pol=(0.0, 0.0, 1.0))),
        "dt": dict(dt=float("inf")),
        "history_form": dict(history_form=2), "raw history, two waves": dict(history_form=1, nrhs=2),
    }
    for what, kw in cases.items():
        assert create(**kw) == _lib.MOT_EINVAL, what

"""The benchmark's hard wall-clock guard around a leg, on the host: a leg
that returns passes its value through; one that does not return by the limit
gets the JSON line printed with the leg marked, and the process ends there
with status 0, so the legs measured before it are kept."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(code):
    return subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=60)


def test_guard_passes_the_value_through():
    p = _run("import bench, json\nr = {'value': 1.0}\nprint(json.dumps(bench.guarded(lambda: {'x': 2}, 5.0, r, 'leg')))")
    assert p.returncode == 0, p.stderr
    assert json.loads(p.stdout.strip().splitlines()[-1]) == {"x": 2}


def test_guard_reports_an_exception_as_the_leg_error():
    p = _run("import bench, json\ndef bad():\n    raise ValueError('no')\n"
             "print(json.dumps(bench.guarded(bad, 5.0, {}, 'leg')))")
    assert p.returncode == 0, p.stderr
    assert json.loads(p.stdout.strip().splitlines()[-1]) == {"error": "ValueError: no"}


def test_guard_prints_the_line_and_ends_the_process_at_the_limit():
    p = _run("import bench, time\nr = {'metric': 'm', 'value': 3.0}\n"
             "bench.guarded(lambda: time.sleep(30), 0.5, r, 'serving_smoke')\nprint('not reached')")
    assert p.returncode == 0, p.stderr
    lines = p.stdout.strip().splitlines()
    assert "not reached" not in p.stdout and len(lines) == 1
    d = json.loads(lines[0])
    assert d["value"] == 3.0 and "did not finish" in d["serving_smoke"]["error"]

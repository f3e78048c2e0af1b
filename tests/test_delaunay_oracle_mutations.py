"""The Delaunay reference's pins catch plausible mistakes.

Each case plants one mistake in a copy of oracle/delaunay.py (on the CPU),
and runs tests/test_delaunay_oracle.py against the copy; at least one pin
must fail. This measures the pins, not the reference.
"""
import os
import shutil
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "delaunay.py")
PINS = os.path.join(ROOT, "tests", "test_delaunay_oracle.py")

MUTANTS = {
    "orient_sign": ("    det = (bx - ax) * (cy - ay) - (by - ay) * (cx - ax)\n    return (det > 0) - (det < 0)",
                    "    det = (bx - ax) * (cy - ay) - (by - ay) * (cx - ax)\n    return (det < 0) - (det > 0)"),
    "incircle_sign": ("a3 * (b1 * c2 - b2 * c1)\n    return (det > 0) - (det < 0)",
                      "a3 * (b1 * c2 - b2 * c1)\n    return (det < 0) - (det > 0)"),
    "flip_orientation": ("tri[t] = [a, bb, d]", "tri[t] = [a, d, bb]"),
    "circumradius_factor": ("r2 = la2 * lb2 * lc2 / (4 * det * det)", "r2 = la2 * lb2 * lc2 / (2 * det * det)"),
    "ratio_longest_edge": ("out.append((r2, r2 / min(la2, lb2, lc2)))", "out.append((r2, r2 / max(la2, lb2, lc2)))"),
    "encroach_closed_circle": ("(a[1] - v[1]) * (b[1] - v[1]) < 0:", "(a[1] - v[1]) * (b[1] - v[1]) <= 0:"),
    "area_half": ("total += ((bx - ax) * (cy - ay) - (by - ay) * (cx - ax)) / 2",
                  "total += ((bx - ax) * (cy - ay) - (by - ay) * (cx - ax))"),
}


def test_every_planted_mistake_fails_a_pin():
    src = open(SRC).read()
    with tempfile.TemporaryDirectory() as tmp:
        runs = {}
        for name, (old, new) in MUTANTS.items():
            assert src.count(old) == 1, f"{name}: pattern occurs {src.count(old)} times"
            d = os.path.join(tmp, name)
            os.makedirs(d)
            open(os.path.join(d, "delaunay.py"), "w").write(src.replace(old, new))
            shutil.copy(PINS, d)
            env = dict(os.environ, PYTHONPATH=os.pathsep.join([d, ROOT]))
            runs[name] = subprocess.Popen([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                                           "--rootdir", d, os.path.join(d, "test_delaunay_oracle.py")],
                                          cwd=d, env=env, stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        survivors = []
        for name, p in runs.items():
            try:
                rc = p.wait(timeout=40)  # a normal run of the pins takes a few seconds
            except subprocess.TimeoutExpired:  # the mistake made the reference loop: caught
                p.kill()
                p.wait()
                continue
            if rc != 1:  # 1: some pin failed; 0: all passed; other codes: the copy did not even run
                survivors.append(name)
        assert not survivors, f"mistakes no pin catches (or that broke collection): {survivors}"

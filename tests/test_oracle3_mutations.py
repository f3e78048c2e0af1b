"""The three-dimensional oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of oracle/rd3_oracle.cpp (on the CPU
only), builds it, and runs tests/test_oracle3_pins.py against the mutant; at
least one pin must fail. This measures the pins, not the oracle.
"""
import os
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "rd3_oracle.cpp")

MUTANTS = {
    "one_over_d": ("const double third = area / 3.0;", "const double third = area / 2.0;"),
    "dW_energy_row": ("g1 * (zb[1] * dz[1] + zb[2] * dz[2] + zb[3] * dz[3]) + zb[0] * dz[4]) / gamma;",
                      "g1 * (zb[1] * dz[1] + zb[2] * dz[2] + zb[3] * dz[3]) + zb[0] * dz[4]);"),
    "roe_average": ("zb[k] = (Zc[0][k] + Zc[1][k] + Zc[2][k] + Zc[3][k]) / 4.0;",
                    "zb[k] = (Zc[0][k] + Zc[1][k] + Zc[2][k] + Zc[3][k]) / 3.0;"),
    "sound_speed": ("const double c = std::sqrt(g1 * (H - 0.5 * dot3(u, u)));",
                    "const double c = std::sqrt(g1 * (H - dot3(u, u)));"),
    "eigen_split_swapped": ("      lp[k] = lam[k] > 0.0 ? lam[k] : 0.0;\n      lm[k] = lam[k] < 0.0 ? lam[k] : 0.0;\n    }\n"
                            "    double R[5][5], L[5][5];",
                            "      lp[k] = lam[k] < 0.0 ? lam[k] : 0.0;\n      lm[k] = lam[k] > 0.0 ? lam[k] : 0.0;\n    }\n"
                            "    double R[5][5], L[5][5];"),
    "entropy_wave_energy": ("col[1][4] = 0.5 * q2;", "col[1][4] = q2;"),
    "n_inflow_sign": ("for (int k = 0; k < 5; ++k) y[k] = s.dW[i][k] + xN[k];",
                      "for (int k = 0; k < 5; ++k) y[k] = s.dW[i][k] - xN[k];"),
    "normal_outward": ("if (dot3(n, toward) < 0.0)\n        for (int k = 0; k < 3; ++k) n[k] = -n[k];",
                       "if (dot3(n, toward) > 0.0)\n        for (int k = 0; k < 3; ++k) n[k] = -n[k];"),
    "stage2_half": ("PN[i][k] = mass * rate[i][k] + 0.5 * (keepN[20 * t + 5 * i + k] + s.phiN[i][k]);",
                    "PN[i][k] = mass * rate[i][k] + (keepN[20 * t + 5 * i + k] + s.phiN[i][k]);"),
    "stage2_mass_term": ("PT[k] = mass * (rate[0][k] + rate[1][k] + rate[2][k] + rate[3][k]) + 0.5 * (keepT[5 * t + k] + s.phiT[k]);",
                         "PT[k] = 0.5 * (keepT[5 * t + k] + s.phiT[k]);"),
    "stage2_mass_factor": ("const double mass = m.vol[t] / 4.0;", "const double mass = m.vol[t] / 3.0;"),
    "cfl_factor": ("best = std::min(best, 3.0 * m.V[i] / acc[i]);", "best = std::min(best, 2.0 * m.V[i] / acc[i]);"),
    "volume_quarter": ("for (int k = 0; k < 4; ++k) m.V[m.tet[4 * t + k]] += m.vol[t] / 4.0;",
                       "for (int k = 0; k < 4; ++k) m.V[m.tet[4 * t + k]] += m.vol[t] / 3.0;"),
}


def _build(name, old, new, tmp):
    src = open(SRC).read()
    assert src.count(old) == 1, f"{name}: pattern occurs {src.count(old)} times"
    path = os.path.join(tmp, f"{name}.cpp")
    open(path, "w").write(src.replace(old, new))
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle3
    lib = os.path.join(tmp, f"lib{name}.so")
    return subprocess.Popen(oracle3.compile_cmd(path, lib), stdout=subprocess.DEVNULL,
                            stderr=subprocess.DEVNULL), lib


def test_every_planted_mistake_fails_a_pin():
    with tempfile.TemporaryDirectory() as tmp:
        builds = {n: _build(n, o, w, tmp) for n, (o, w) in MUTANTS.items()}
        libs = {}
        for n, (proc, lib) in builds.items():
            assert proc.wait() == 0, f"{n}: mutant did not compile"
            libs[n] = lib
        runs = {}
        for n, lib in libs.items():
            env = dict(os.environ, RDO3_LIB=lib, OMP_NUM_THREADS="1")
            runs[n] = subprocess.Popen([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                                        os.path.join(ROOT, "tests", "test_oracle3_pins.py")],
                                       cwd=ROOT, env=env, stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        survivors = [n for n, p in runs.items() if p.wait() == 0]
        assert not survivors, f"mistakes no pin catches: {survivors}"

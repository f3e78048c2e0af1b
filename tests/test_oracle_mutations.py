"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of oracle/rd_oracle.cpp (on the CPU
only), builds it, and runs the pin suite against the mutant; at least one
pin must fail. This measures the pins, not the oracle.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "rd_oracle.cpp")

MUTANTS = {
    "appendix_entry_sign": ("- g2 * uc * nx * l12 + l3;", "+ g2 * uc * nx * l12 + l3;"),
    "l123_definition": ("T l123 = (l1 + l2 - 2.0 * l3) / 2.0;", "T l123 = (l1 + l2 - l3) / 2.0;"),
    "missing_one_over_d": ("const double half = len / 2.0;", "const double half = len;"),
    "dW_over_dZ_row": ("+ g1 * zb[2] * dz[2] + zb[0] * dz[3]) / gamma;", "+ g1 * zb[2] * dz[2] + zb[0] * dz[3]);"),
    "eigen_split_swapped": ("lp[k] = pos_part(lam[k]); lm[k] = neg_part(lam[k]); }\n    k_entries(u, v, h, c, gamma, nx, ny, lam[0]",
                            "lp[k] = neg_part(lam[k]); lm[k] = pos_part(lam[k]); }\n    k_entries(u, v, h, c, gamma, nx, ny, lam[0]"),
    "n_inflow_sign": ("for (int k = 0; k < 4; ++k) y[k] = s.dW[i][k] + xN[k];", "for (int k = 0; k < 4; ++k) y[k] = s.dW[i][k] - xN[k];"),
    "theta_denominator": ("T den = absval(pn[0][k]) + absval(pn[1][k]) + absval(pn[2][k]);",
                          "T den = absval(pn[0][k]) + absval(pn[1][k]);"),
    "stage2_half": ("PN[i][k] = mass * rate[i][k] + 0.5 * (keepN[12 * t + 4 * i + k] + s.phiN[i][k]);",
                    "PN[i][k] = mass * rate[i][k] + (keepN[12 * t + 4 * i + k] + s.phiN[i][k]);"),
    "stage2_mass_term": ("PT[k] = mass * (rate[0][k] + rate[1][k] + rate[2][k]) + 0.5 * (keepT[4 * t + k] + s.phiT[k]);",
                         "PT[k] = 0.5 * (keepT[4 * t + k] + s.phiT[k]);"),
    "cfl_factor": ("best = std::min(best, 2.0 * m.V[i] / acc[i]);", "best = std::min(best, m.V[i] / acc[i]);"),
    "ghosts_updated": ("    if (m.ghost[i]) continue;\n    for (int k = 0; k < 4; ++k) {\n      T r = R[4 * i + k] + Wc_n[4 * i + k];",
                       "    for (int k = 0; k < 4; ++k) {\n      T r = R[4 * i + k] + Wc_n[4 * i + k];"),
    "wall_normal_inward": ("m.wnx[e] = dy / len;", "m.wnx[e] = -dy / len;"),
    "wall_split_roles_swapped": ("out[4 * ab[0] + k] += hl * (alpha * F[0][k] + (1.0 - alpha) * F[1][k]);\n"
                                 "      out[4 * ab[1] + k] += hl * ((1.0 - alpha) * F[0][k] + alpha * F[1][k]);",
                                 "out[4 * ab[0] + k] += hl * ((1.0 - alpha) * F[0][k] + alpha * F[1][k]);\n"
                                 "      out[4 * ab[1] + k] += hl * (alpha * F[0][k] + (1.0 - alpha) * F[1][k]);"),
    "wall_split_half": ("const double alpha = 0.75, g1 = m.gamma - 1.0;", "const double alpha = 0.5, g1 = m.gamma - 1.0;"),
    "volume_third": ("m.V[m.tri[3 * t + k]] += m.area[t] / 3.0;", "m.V[m.tri[3 * t + k]] += m.area[t] / 2.0;"),
    "bx_sensor_sign": ("pos_part(-m.L * div / range)", "pos_part(m.L * div / range)"),
    "bx_h_in_domain_units": ("T theta = s * s * h / m.L;", "T theta = s * s * h;"),
    "bx_element_size": ("const double h = std::sqrt(2.0 * m.area[t]);", "const double h = std::sqrt(m.area[t]);"),
    "bx_speed_range": ("T range = vmax - vmin;", "T range = vmax;"),
    "bx_domain_size": ("m.L = std::max(lx, ly);", "m.L = std::min(lx, ly);"),
    "lumping_sign": ("sl = sl + (ml - mg) * rate[j][k];", "sl = sl + (mg - ml) * rate[j][k];"),
    "lumping_galerkin_mass": ("const double mg = m.area[t] * ((i == j ? 1.0 : 0.0) + 1.0) / 12.0;",
                              "const double mg = m.area[t] * ((i == j ? 1.0 : 0.0) + 1.0) / 6.0;"),
    "lumping_lda_part": ("          PL[i][k] = PL[i][k] + sl;\n", "\n"),
}


def _build(name, old, new, tmp):
    src = open(SRC).read()
    assert src.count(old) == 1, f"{name}: pattern occurs {src.count(old)} times"
    path = os.path.join(tmp, f"{name}.cpp")
    open(path, "w").write(src.replace(old, new))
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle
    lib = os.path.join(tmp, f"lib{name}.so")
    return subprocess.Popen(oracle.compile_cmd(path, lib), stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL), lib


def test_every_planted_mistake_fails_a_pin():
    with tempfile.TemporaryDirectory() as tmp:
        builds = {n: _build(n, o, w, tmp) for n, (o, w) in MUTANTS.items()}
        libs = {}
        for n, (proc, lib) in builds.items():
            assert proc.wait() == 0, f"{n}: mutant did not compile"
            libs[n] = lib
        runs = {}
        for n, lib in libs.items():
            env = dict(os.environ, RDO_LIB=lib, OMP_NUM_THREADS="1")
            runs[n] = subprocess.Popen([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                                       cwd=ROOT, env=env, stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        survivors = [n for n, p in runs.items() if p.wait() == 0]
        assert not survivors, f"mistakes no pin catches: {survivors}"

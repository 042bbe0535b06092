"""The oracle's pins must fail for plausible mistakes in the oracle.

Each case copies the C oracle source, plants one mistake (a flipped sign, a
wrong factor, a dropped term, a swapped operand, an off-by-one exclusion),
compiles it into a temporary directory and runs the pin suite against it in a
subprocess.  The real oracle build is never touched.  CPU only.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "stokes_oracle.c")

MUTANTS = {
    "stokeslet_sign": ("double gx = fx / r + dx * df / r3;", "double gx = fx / r - dx * df / r3;"),
    "doublet_factor3": ("gx += c * (fx / r3 - 3.0 * dx * df / r5);",
                        "gx += c * (fx / r3 - 2.0 * dx * df / r5);"),
    "doublet_coeff": ("const double c = 0.5 * a * a;", "const double c = a * a;"),
    "weight_dropped": ("const double fx = wj * f[j]", "const double fx = f[j]"),
    "plane_swap": ("const double dy = yi - sx[ns + j];", "const double dy = yi - sx[2 * ns + j];"),
    "viscosity_dropped": ("const double pref = 1.0 / (8.0 * ORACLE_PI * mu);",
                          "const double pref = 1.0 / (8.0 * ORACLE_PI);"),
    "dl_sign": ("const double pref = 3.0 / (4.0 * ORACLE_PI);",
                "const double pref = -3.0 / (4.0 * ORACLE_PI);"),
    "dl_normal_index": ("const double dn = dx * n[s] + dy * n[ns + s] + dz * n[2 * ns + s];",
                        "const double dn = dx * n[s] + dy * n[ns + s] + dz * n[s];"),
    "dl_jump": ("if (sub) { ux -= 0.5 * q0x;", "if (sub) { ux -= 1.0 * q0x;"),
    "dl_power": ("const double r5 = r2 * r2 * r;", "const double r5 = r2 * r2;"),
    "self_off_by_one": ("if (excl == 1 && j == self) continue;",
                        "if (excl == 1 && j == self + 1) continue;"),
    "fiber_exclusion_dropped": ("if (excl == 2 && sfib && (int64_t)sfib[j] == fib_i) continue;", ""),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_kill_mutant(tmp_path, name):
    import oracle
    a, b = MUTANTS[name]
    text = open(SRC).read()
    assert a in text, f"mutation site for {name} not found"
    msrc = tmp_path / "stokes_oracle_mut.c"
    msrc.write_text(text.replace(a, b))
    lib = oracle.compile_c(str(msrc), str(tmp_path / "liboracle_mut.so"))
    env = dict(os.environ, STOKES_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"

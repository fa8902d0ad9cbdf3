"""The oracle's pins catch plausible slips.

Each case plants one mistake in a copy of the oracle's C source, builds it
with gcc into a temporary directory, and runs the pins that should notice it
against that library in a child process.  The pins must fail there (and they
pass against the real oracle in test_oracle_pins.py).  Only the CPU oracle is
altered; nothing here touches the GPU path.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "asicp_oracle.c")

# (name, exact text in the source, replacement, pins expected to fail)
MUTANTS = [
    ("rotation preconditioner doubled",
     "a_w[p] = 3.0 / (2.0 * (rho2[p] + cfg->lambda * tcp2));",
     "a_w[p] = 6.0 / (2.0 * (rho2[p] + cfg->lambda * tcp2));",
     "first_order or reciprocal_gauss_newton"),
    ("lambda |TCP|^2 dropped from the rotation preconditioner",
     "a_w[p] = 3.0 / (2.0 * (rho2[p] + cfg->lambda * tcp2));",
     "a_w[p] = 3.0 / (2.0 * (rho2[p] + 0.0 * tcp2));",
     "first_order or reciprocal_gauss_newton"),
    ("translation preconditioner without lambda",
     "a_t[p] = 1.0 / (1.0 + cfg->lambda);",
     "a_t[p] = 1.0;",
     "minimiser_of_the_cost or reciprocal_gauss_newton"),
    ("driving term weighted by the particle's own gradient",
     "const double* gj = g + 6 * (size_t)j;",
     "const double* gj = g + 6 * (size_t)i;",
     "driving_term"),
    ("driving term weighted by the RBF alone",
     "wdt = kt * kr; wrt = kt * kr; wdw = kt * kr;",
     "wdt = kt; wrt = kt * kr; wdw = kt;",
     "driving_term"),
]


@pytest.mark.parametrize("name, old, new, pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_fail_on_planted_mistake(tmp_path, name, old, new, pins):
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site not unique: {old}"
    src = tmp_path / "asicp_oracle.c"
    src.write_text(text.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                           "-I", os.path.join(ROOT, "oracle"), str(src), "-o", str(lib), "-lm"])
    env = dict(os.environ, ASICP_ORACLE_VARIANT_LIB=str(lib), PYTHONPATH=ROOT)
    p = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", pins],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=300)
    # pytest exit status 1: tests ran and at least one failed
    assert p.returncode == 1, f"{name}: pins did not fail\n{p.stdout[-2000:]}\n{p.stderr[-2000:]}"
    assert " passed" in p.stdout or " failed" in p.stdout

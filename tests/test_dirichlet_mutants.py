"""Strength of the Dirichlet-oracle pins: each mutant is a copy of
oracle/dirichlet.c with one planted error, built with oracle.c into a
library and run against tests/test_dirichlet_pins.py, which must fail; the
unmodified copy must pass.  CPU only."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "dirichlet.c")
BASE = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = [
    ("dirichlet_ghost_sign_x", "else e = g->bcx == 0 ? P(0, j, k) : (g->bcx == 1 ? c : -c);",
     "else e = g->bcx == 0 ? P(0, j, k) : (g->bcx == 1 ? c : c);"),
    ("dirichlet_eigenvalue_index", "s = sin(M_PI * (double)(l + 1) / (2.0 * (double)n));",
     "s = sin(M_PI * (double)l / (2.0 * (double)n));"),
    ("sine_mode_phase", "return sin(M_PI * (double)(l + 1) * ((double)x + 0.5) / (double)n);",
     "return sin(M_PI * (double)(l + 1) * (double)x / (double)n);"),
    ("z_dirichlet_row", "else b[k] -= a[k];         /* Dirichlet: ghost = -p_0 */",
     "else b[k] += a[k];         /* Dirichlet: ghost = -p_0 */"),
    ("last_sine_norm", "return l == n - 1 ? (double)n : 0.5 * (double)n;", "return 0.5 * (double)n;"),
    ("z_wall_ghost_distance", "a[k] = 1.0 / (dzf[k] * dlo);", "a[k] = 1.0 / (dzf[k] * (k > 0 ? dlo : dzc[0]));"),
]


def _build(tmp_path, text, tag):
    src = tmp_path / f"{tag}.c"
    src.write_text(text)
    so = tmp_path / f"lib{tag}.so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fno-fast-math",
                           "-fPIC", "-shared", "-I", os.path.join(ROOT, "oracle"), "-o", str(so), BASE, str(src),
                           "-lm"])
    return str(so)


def _pins_pass(so):
    env = dict(os.environ, PCX_ORACLE_LIB=so)
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(HERE, "test_dirichlet_pins.py"), "-x", "-q",
                        "-p", "no:cacheprovider", "-m", "not gpu"], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    return r.returncode == 0, r.stdout[-400:]


def test_unmodified_copy_passes(tmp_path):
    ok, out = _pins_pass(_build(tmp_path, open(SRC).read(), "control"))
    assert ok, out


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site for {name} not found once in dirichlet.c"
    ok, out = _pins_pass(_build(tmp_path, text.replace(old, new), name))
    assert not ok, f"pins did not catch {name}"

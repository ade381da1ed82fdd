"""Strength of the variable-coefficient oracle pins: each mutant is a copy of
oracle/varcoef.c with one planted error, built with oracle.c into a library
and run against tests/test_varcoef_pins.py, which must fail; the unmodified
copy must pass.  CPU only."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "varcoef.c")
BASE = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = [
    ("z_face_density_weights", "rf = (rho[c] * m->dzf[kp] + rho[c1] * m->dzf[k]) / (2.0 * m->dzc[k]);",
     "rf = (rho[c] * m->dzf[k] + rho[c1] * m->dzf[kp]) / (2.0 * m->dzc[k]);"),
    ("x_face_density_one_sided", "rf = 0.5 * (rho[c] + rho[c1]);", "rf = rho[c];"),
    ("wall_face_not_closed", "if (m->bc[d] == 1 && s == n[d] - 1) return 0.0;", "if (0) return 0.0;"),
    ("z_gradient_spacing", "h = m->dzc[k];", "h = m->dzf[k];"),
    ("z_divergence_spacing", "const double h = d == 0 ? m->dx : (d == 1 ? m->dy : m->dzf[k]);",
     "const double h = d == 0 ? m->dx : (d == 1 ? m->dy : m->dzc[k]);"),
    ("unweighted_inner_product", "s += t * m->dzf[k];", "s += t;"),
    ("rhs_scaled_by_dt", "for (size_t c = 0; c < n; ++c) rhs[c] /= dt;", "for (size_t c = 0; c < n; ++c) rhs[c] *= dt;"),
    ("correction_sign", "else vout[d][c] = vin[d][c] - dt * bgrad(m, rho, p, d, i, j, k);",
     "else vout[d][c] = vin[d][c] + dt * bgrad(m, rho, p, d, i, j, k);"),
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
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(HERE, "test_varcoef_pins.py"), "-x", "-q",
                        "-p", "no:cacheprovider", "-m", "not gpu"], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    return r.returncode == 0, r.stdout[-400:]


def test_unmodified_copy_passes(tmp_path):
    ok, out = _pins_pass(_build(tmp_path, open(SRC).read(), "control"))
    assert ok, out


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site for {name} not found once in varcoef.c"
    ok, out = _pins_pass(_build(tmp_path, text.replace(old, new), name))
    assert not ok, f"pins did not catch {name}"

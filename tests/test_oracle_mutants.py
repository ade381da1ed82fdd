"""The oracle's pins are strong enough to catch plausible mistakes: each
mutant below is a copy of oracle.c with one planted error (a dropped term, a
wrong sign, index or spacing, a swapped operand), built on the CPU and run
against tests/test_oracle_pins.py, which must then fail.  The unmodified copy
built the same way must pass."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "oracle.c")

# (name, exact text in oracle.c, replacement)
MUTANTS = [
    ("rhs_splitting_factor_dropped",
     "else gg[d][c] = (1.0 - rho0 / rho_face(&m, rho, d, i, j, k)) * gg[d][c];",
     "else gg[d][c] = gg[d][c];"),
    ("rhs_velocity_term_sign",
     "f[c] = (rho0 / dt) * dv[c] + f[c];",
     "f[c] = -(rho0 / dt) * dv[c] + f[c];"),
    ("z_face_density_plain_mean",
     "return (r0 * m->dzf[kp] + r1 * m->dzf[k]) / (2.0 * m->dzc[k]);",
     "return 0.5 * (r0 + r1);"),
    ("grad_z_uses_cell_width",
     "return (q[IDX(i, j, wrapi(k + 1, nz))] - q[c]) / m->dzc[k];",
     "return (q[IDX(i, j, wrapi(k + 1, nz))] - q[c]) / m->dzf[k];"),
    ("div_z_uses_centre_spacing",
     "double ddz = (face_val(w, bz, sz, k, nz, m->bcz) - face_val(w, bz, sz, k - 1, nz, m->bcz)) / m->dzf[k];\n                out[c]",
     "double ddz = (face_val(w, bz, sz, k, nz, m->bcz) - face_val(w, bz, sz, k - 1, nz, m->bcz)) / m->dzc[k];\n                out[c]"),
    ("grad_x_wrong_neighbour",
     "return (q[IDX(wrapi(i + 1, nx), j, k)] - q[c]) / m->dx;",
     "return (q[IDX(wrapi(i - 1, nx), j, k)] - q[c]) / m->dx;"),
    ("wall_eigenvalue_periodic_form",
     "s = sin(M_PI * (double)l / (2.0 * (double)n));",
     "s = sin(M_PI * (double)l / (double)n);"),
    ("thomas_sub_super_swapped",
     "piv = b[k] - a[k] * cp[k - 1];",
     "piv = b[k] - c[k] * cp[k - 1];"),
    ("z_lower_coefficient_spacing",
     "a[k] = has_lo ? 1.0 / (m->dzf[k] * m->dzc[wrapi(k - 1, nz)]) : 0.0;",
     "a[k] = has_lo ? 1.0 / (m->dzf[k] * m->dzc[k]) : 0.0;"),
    ("volume_mean_unweighted",
     "num += s * m.dzf[k];",
     "num += s * (m.lz / nz);"),
    ("dct3_scale",
     "for (int i = 0; i < N; ++i) x[(size_t)i * xs] = y[i].re / (2.0 * N);",
     "for (int i = 0; i < N; ++i) x[(size_t)i * xs] = y[i].re / N;"),
    ("cyclic_corner_dropped",
     "double fact = (d[0] + beta * d[n - 1] / gamma) / (1.0 + z[0] + beta * z[n - 1] / gamma);",
     "double fact = 0.0 * (d[0] + beta * d[n - 1] / gamma) / (1.0 + z[0] + beta * z[n - 1] / gamma);"),
    ("correction_density_term_dropped",
     "out[d][c] = in[d][c] - dt * ((1.0 / rho0) * gp[d][c] + (1.0 / rf - 1.0 / rho0) * gs[d][c]);",
     "out[d][c] = in[d][c] - dt * ((1.0 / rho0) * gp[d][c]);"),
    ("compatibility_not_removed",
     "for (size_t c = 0; c < n; ++c) { F[c].re = f[c] - fm; F[c].im = 0.0; }",
     "for (size_t c = 0; c < n; ++c) { F[c].re = f[c]; F[c].im = 0.0; }"),
]


def _build(tmp_path, text, tag):
    src = tmp_path / f"{tag}.c"
    src.write_text(text)
    so = tmp_path / f"lib{tag}.so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fno-fast-math",
                           "-fPIC", "-shared", "-I", os.path.join(ROOT, "oracle"), "-o", str(so), str(src), "-lm"])
    return str(so)


def _pins_pass(so):
    env = dict(os.environ, PCX_ORACLE_LIB=so)
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(HERE, "test_oracle_pins.py"), "-x", "-q",
                        "-p", "no:cacheprovider", "-m", "not gpu"], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    return r.returncode == 0, r.stdout[-400:]


def test_unmodified_copy_passes(tmp_path):
    ok, out = _pins_pass(_build(tmp_path, open(SRC).read(), "control"))
    assert ok, out


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site for {name} not found once in oracle.c"
    ok, out = _pins_pass(_build(tmp_path, text.replace(old, new), name))
    assert not ok, f"pins did not catch {name}"

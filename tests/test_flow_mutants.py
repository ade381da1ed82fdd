"""Strength of the flow-oracle pins: each mutant below is a copy of
oracle/flow.c with one planted error (a dropped factor, a flipped sign, a
wrong interpolation or spacing, a swapped property map, a wrong
Runge-Kutta coefficient, the pressure extrapolation dropped), built with
oracle.c into a library and run against tests/test_flow_pins.py, which
must fail; the unmodified copy must pass.  CPU only."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "flow.c")
BASE = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = [
    ("sharpening_quarter_to_half", "- 0.25 * (1.0 - t * t) * nf", "- 0.5 * (1.0 - t * t) * nf"),
    ("sharpening_sign", "- 0.25 * (1.0 - t * t) * nf", "+ 0.25 * (1.0 - t * t) * nf"),
    ("psi_face_scale", "tanh(psf / (2.0 * a->eps))", "tanh(psf / a->eps)"),
    ("diffusion_without_eps", "a->gamma * (a->eps * cgrad(m, phi, d, i, j, k)", "a->gamma * (cgrad(m, phi, d, i, j, k)"),
    ("advected_phi_not_averaged",
     "jp = fval(m, vel[d], d, i, j, k) * cface(m, phi, d, i, j, k) - af[d][ID(i, j, k)];",
     "jp = fval(m, vel[d], d, i, j, k) * cval(m, phi, i, j, k) - af[d][ID(i, j, k)];"),
    ("normal_z_spacing", "/ (dzc_at(m, k) + dzc_at(m, k - 1));", "/ (2.0 * dzc_at(m, k));"),
    ("curvature_sign", "kappa[ID(i, j, k)] = -s;", "kappa[ID(i, j, k)] = s;"),
    ("normal_stress_factor", "const double tp = 2.0 * mu1 * (qp - q0)", "const double tp = mu1 * (qp - q0)"),
    ("stress_without_transpose", "const double tu = muu * ((qu - q0) / hu + dpu);",
     "const double tu = muu * ((qu - q0) / hu);"),
    ("edge_viscosity_cell_value", "const double muu = edge4(m, mu, c, d, i, j, k);",
     "const double muu = cval(m, mu, i, j, k);"),
    ("regularization_sign", "(f->rho1 - f->rho2) * reg", "(f->rho2 - f->rho1) * reg"),
    ("viscosity_map_swapped", "mu[c] = f->mu2 + (f->mu1 - f->mu2) * phi[c];",
     "mu[c] = f->mu1 + (f->mu2 - f->mu1) * phi[c];"),
    ("density_map_swapped", "rho[c] = f->rho2 + (f->rho1 - f->rho2) * phi[c];",
     "rho[c] = f->rho1 + (f->rho2 - f->rho1) * phi[c];"),
    ("rk3_zeta", "-17.0 / 60.0", "-16.0 / 60.0"),
    ("pstar_not_extrapolated", "ps[c] = (1.0 + r) * p1[c] - r * p2[c];", "ps[c] = p1[c];"),
    ("advection_transverse_edge", "adv += (pu * 0.5 * (q0 + qu) - pd * 0.5 * (qd + q0)) / hcell(m, d, ix[2]);",
     "adv += (pu * q0 - pd * q0) / hcell(m, d, ix[2]);"),
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
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(HERE, "test_flow_pins.py"), "-x", "-q",
                        "-p", "no:cacheprovider", "-m", "not gpu"], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    return r.returncode == 0, r.stdout[-400:]


def test_unmodified_copy_passes(tmp_path):
    ok, out = _pins_pass(_build(tmp_path, open(SRC).read(), "control"))
    assert ok, out


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site for {name} not found once in flow.c"
    ok, out = _pins_pass(_build(tmp_path, text.replace(old, new), name))
    assert not ok, f"pins did not catch {name}"

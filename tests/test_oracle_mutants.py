"""The pins catch plausible mistakes: each test builds a copy of the oracle
with one planted mistake (on the CPU, from a textual edit of its C source)
and checks that the pin aimed at that part rejects it.

Planted mistakes and the pin that must reject them:

* exit BTDF (Eq. 3) without the Fresnel transmittance (1 - F_in): smooth
  limit and energy identity;
* exit BTDF with the indices swapped in the half-vector Jacobian: smooth
  limit;
* exit BTDF masking the incident direction with the outgoing one: energy
  identity;
* reflection lobe (Eq. 2) with the Fresnel factor at the macro cosine
  instead of the half-vector cosine: energy identity;
* node weight T_k without the entry Fresnel transmittance: node weights;
* implicit plies (Sec. 3.4) with the sign of the ray slope kappa flipped:
  ellipse-plane residual;
* implicit plies with the yarn hit dropped from the update: ellipse-plane
  residual.
"""
import contextlib
import os
import subprocess

import numpy as np
import pytest

import test_oracle_exit_btdf as XB
import test_oracle_fixed_point as FP

ORACLE_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")
SOURCES = ("bysdf_oracle.c", "yarn_oracle.c", "render_oracle.c")


@contextlib.contextmanager
def mutant(oracle_mod, tmp_path, old, new):
    """The oracle built with the one occurrence of `old` in bysdf_oracle.c
    replaced by `new`, swapped in for the duration of the block."""
    paths = []
    for name in SOURCES:
        with open(os.path.join(ORACLE_DIR, name)) as f:
            src = f.read()
        if name == "bysdf_oracle.c":
            assert src.count(old) == 1, old
            src = src.replace(old, new)
        p = tmp_path / name
        p.write_text(src)
        paths.append(str(p))
    lib = str(tmp_path / "liboracle_mutant.so")
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                           "-I" + ORACLE_DIR, "-o", lib] + paths + ["-lm"])
    saved = oracle_mod.lib()
    oracle_mod._lib = oracle_mod.bind(lib)
    try:
        yield
    finally:
        oracle_mod._lib = saved


def _smooth_limit_rejects(orc):
    rows = XB.smooth_limit_errors(orc, n_nodes=3)
    return any(abs(rel) >= 5e-4 or ang >= 2e-3 for rel, ang in rows)


def _identity_rejects(orc):
    rows = XB.energy_identity_errors(orc, n_queries=2, grid=(600, 1200))
    for xs, ys, tot in rows:
        if abs(xs[0] - xs[1]) >= 5e-6 + 1e-4 * xs[1] or abs(ys[0] - ys[1]) >= 5e-6 + 1e-4 * ys[1]:
            return True
        if any(abs(e - i) >= 1e-5 for e, i in tot):
            return True
    return False


EXIT_F = ("*val = fabs(im) * (1.0 - F) * g1i", "*val = fabs(im) * g1i")
EXIT_JAC = ("double den = eta * im + om;", "double den = im + eta * om;")
EXIT_G1 = ("double g1i = G1_l(to_local(&nd->fy, wip), ml3, ax, ay);",
           "double g1i = G1_l(to_local(&nd->fy, wo), ml3, ax, ay);")
REFL_F = ("orc_fresnel(ih, eta) * g1i", "orc_fresnel(mu_i, eta) * g1i")
NODE_T = ("nd->T = (1.0 - orc_fresnel(c, eta)) * G1_l(", "nd->T = G1_l(")
KAPPA = ("g->kappa = -wi.z / sxy;", "g->kappa = wi.z / sxy;")
UPDATE = ("vj = v + g->kappa * ((ccx - g->x2[0]) * g->dh[0] + (ccy - g->x2[1]) * g->dh[1]);",
          "vj = v + g->kappa * (ccx * g->dh[0] + ccy * g->dh[1]);")


def test_unmutated_copy_passes(oracle_mod, tmp_path):
    """The copy mechanism itself: with a no-op edit every pin accepts."""
    with mutant(oracle_mod, tmp_path, KAPPA[0], KAPPA[0]):
        assert not _smooth_limit_rejects(oracle_mod)
        assert FP.plane_residuals(oracle_mod, n=40)[0] < 1e-12


@pytest.mark.parametrize("edit", [EXIT_F, EXIT_JAC], ids=["exit_no_fresnel", "exit_jacobian_eta"])
def test_smooth_limit_rejects(oracle_mod, tmp_path, edit):
    with mutant(oracle_mod, tmp_path, *edit):
        assert _smooth_limit_rejects(oracle_mod)


@pytest.mark.parametrize("edit", [EXIT_F, EXIT_G1, REFL_F], ids=["exit_no_fresnel", "exit_g1_direction",
                                                                 "reflection_fresnel_cosine"])
def test_energy_identity_rejects(oracle_mod, tmp_path, edit):
    with mutant(oracle_mod, tmp_path, *edit):
        assert _identity_rejects(oracle_mod)


def test_node_weights_reject(oracle_mod, tmp_path):
    with mutant(oracle_mod, tmp_path, *NODE_T):
        worst_T, _ = XB.node_weight_errors(oracle_mod, n_queries=5)
        assert worst_T > 1e-3


@pytest.mark.parametrize("edit", [KAPPA, UPDATE], ids=["kappa_sign", "update_without_hit"])
def test_plane_residual_rejects(oracle_mod, tmp_path, edit):
    with mutant(oracle_mod, tmp_path, *edit):
        worst, count = FP.plane_residuals(oracle_mod, n=40)
        assert worst > 1e-3

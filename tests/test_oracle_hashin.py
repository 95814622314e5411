"""Pins of the oracle's generalized Hashin closed form (Sec. 4.2)."""
import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import closed_forms as CF
from oracle import elasticity as E
from oracle.dft import make_transform

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


def test_depolarization_quadrature_matches_spheroids_and_cylinder():
    assert np.allclose(CF.depolarization_quadrature([0.1, 0.1, 0.3]), CF.depolarization_prolate(0.1, 0.3), atol=1e-12)
    assert np.allclose(CF.depolarization_quadrature([0.1, 0.3, 0.3]), CF.depolarization_oblate(0.1, 0.3), atol=1e-12)
    assert np.allclose(CF.depolarization_quadrature([0.2, 0.2, 0.2]), [1 / 3] * 3, atol=1e-12)
    d = CF.depolarization_quadrature([0.15, 0.2, 0.3])
    assert math.isclose(d.sum(), 1.0, rel_tol=1e-12)
    assert d[0] > d[1] > d[2]
    # elongated third axis approaches the elliptic cylinder
    assert np.allclose(CF.depolarization_quadrature([0.1, 0.2, 1e3]), CF.depolarization_cylinder(0.1, 0.2), atol=1e-3)


def test_printed_prolate_form_fails_without_correction():
    """The printed prolate d3 (without the -1) does not sum to one."""
    delta = math.sqrt(1 - (0.1 / 0.3) ** 2)
    literal = (1 - delta ** 2) / delta ** 2 * (math.log((1 + delta) / (1 - delta)) / (2 * delta))
    assert abs(literal - CF.depolarization_quadrature([0.1, 0.1, 0.3])[2]) > 0.1


def test_rotation_corrected_rodrigues():
    for n in ([0.5, 1.0, 0.3], [0.0, 0.0, 1.0], [-0.2, 0.4, -0.9], [1.0, 0.0, 0.0]):
        R = CF.rotation_e1_to(n)
        u = np.asarray(n) / np.linalg.norm(n)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-14)
        assert np.allclose(R @ [1, 0, 0], u, atol=1e-14)
        assert math.isclose(np.linalg.det(R), 1.0, rel_tol=1e-13)


def test_sphere_limit_is_classic_hashin_bulk_modulus():
    lc, le = E.lame_from_young(10, 0.3), E.lame_from_young(0.5, 0.3)
    for rho_e in (0.01, 0.05, 0.1):
        h = CF.hashin([0.2, 0.2, 0.2], 0.0, rho_e, lc, le)
        # eps0 hydrostatic; C_eff eps0 = 3 kappa* (tr eps0 / 3) I
        assert np.allclose(h["eps0"], np.trace(h["eps0"]) / 3 * np.eye(3), atol=1e-14)
        kappa = np.trace(h["ceff_eps0"]) / (3.0 * np.trace(h["eps0"]) / 3.0) / 3.0
        assert math.isclose(kappa, CF.hashin_bulk_classic(lc, le, h["f"]), rel_tol=1e-12)


def _cylinder_example():
    g = GOLD["example_4_1"]
    c = [g["c"][0], g["c"][1], math.inf]
    # Reading: n = (1/2, sqrt(3)/2, 0), the unit vector at 60 degrees
    R = CF.rotation_e1_to([0.5, math.sqrt(3) / 2, 0.0])
    lc, le = E.lame_from_young(10, 0.3), E.lame_from_young(0.5, 0.3)
    return c, g["rho_c"], g["rho_e"], R, lc, le


def test_example_4_1_fits_in_cell_and_neutral_matrix():
    c, rc, re, R, lc, le = _cylinder_example()
    assert math.sqrt(c[1] ** 2 + re) < 0.5   # l2(rho_e) < 1/2 for c3 = infinity
    h = CF.hashin(c, rc, re, lc, le, R)
    lam_m, mu_m = h["lame_m"]
    Cm = E.iso_tensor(lam_m, mu_m, 3)
    assert np.allclose(E.contract(Cm, h["eps0"]), h["ceff_eps0"], atol=1e-13)


def test_analytic_field_averages():
    """<eps> = eps0 and <C : eps> = C_eff : eps0 for the analytic field (midpoint rule)."""
    c, rc, re, R, lc, le = _cylinder_example()
    h = CF.hashin(c, rc, re, lc, le, R)
    n = 256
    g = (np.arange(n) + 0.5) / n - 0.5
    X = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    X3 = np.concatenate([X, np.zeros((X.shape[0], 1))], 1)
    eps = h["strain"](X3)
    rho = CF.ellipsoidal_radius_many(np.array(c), X3 @ R)
    ph = np.where(rho <= rc, 0, np.where(rho <= re, 1, 2))
    lam = np.array([lc[0], le[0], h["lame_m"][0]])[ph]
    mu = np.array([lc[1], le[1], h["lame_m"][1]])[ph]
    tr = np.trace(eps, axis1=1, axis2=2)
    sig = lam[:, None, None] * tr[:, None, None] * np.eye(3) + 2 * mu[:, None, None] * eps
    assert np.allclose(eps.mean(0), h["eps0"], atol=2e-4)
    assert np.allclose(sig.mean(0), h["ceff_eps0"], atol=2e-4)


def test_traction_continuity_across_interfaces():
    """The analytic field satisfies [sigma] n = 0 across both confocal interfaces."""
    c, rc, re, R, lc, le = _cylinder_example()
    h = CF.hashin(c, rc, re, lc, le, R)
    lam = [lc[0], le[0], h["lame_m"][0]]
    mu = [lc[1], le[1], h["lame_m"][1]]
    rng = np.random.default_rng(9)
    for rho_i, (pa, pb) in ((rc, (0, 1)), (re, (1, 2))):
        for _ in range(5):
            t = rng.uniform(0, 2 * math.pi)
            l1, l2 = math.sqrt(c[0] ** 2 + rho_i), math.sqrt(c[1] ** 2 + rho_i)
            xt = np.array([l1 * math.cos(t), l2 * math.sin(t), 0.0])
            nt = np.array([xt[0] / l1 ** 2, xt[1] / l2 ** 2, 0.0])
            nt /= np.linalg.norm(nt)
            x, nrm = R @ xt, R @ nt
            ein = h["strain"]((x * (1 - 1e-9))[None])[0]
            eout = h["strain"]((x * (1 + 1e-9))[None])[0]
            s_in = lam[pa] * np.trace(ein) * np.eye(3) + 2 * mu[pa] * ein
            s_out = lam[pb] * np.trace(eout) * np.eye(3) + 2 * mu[pb] * eout
            assert np.allclose(s_in @ nrm, s_out @ nrm, atol=1e-6)


def test_hashin_cylinder_scheme_converges_to_closed_form():
    """Algorithm 1 on a 64 x 64 pattern (d = 3, M_33 = 1): e_eff at discretization level."""
    c, rc, re, R, lc, le = _cylinder_example()
    h = CF.hashin(c, rc, re, lc, le, R)
    M = [[64, 0, 0], [0, 64, 0], [0, 0, 1]]
    T = make_transform(M)
    geom = dict(c=np.array(c), rho_c=rc, rho_e=re, R=R)
    ph = synth.hashin_phase(T.points, T.m, geom)
    lame = np.array([lc, le, h["lame_m"]])
    r = E.basic_scheme(M, ph, lame, E.default_reference(lame), h["eps0"], tol=1e-8, transform=T)
    assert r.status == 0
    e_eff = E.error_eff(r.mean_stress, h["ceff_eps0"])
    assert e_eff < 0.03
    y = T.points / T.m
    ref = h["strain"](y)
    assert E.error_l2(r.eps.transpose(2, 0, 1), ref) < 0.3


def test_config2_geometry_reading():
    """Coating 0.1 of the cell, outer ellipsoid inside the cell."""
    g = synth.hashin_geometry(seed=2)
    c, re = g["c"], g["rho_e"]
    vol = 4 / 3 * math.pi * (np.prod(np.sqrt(c ** 2 + re)) - np.prod(c))
    assert math.isclose(vol, 0.1, rel_tol=1e-12)
    assert np.sqrt(c ** 2 + re).max() < 0.5
    assert np.allclose(g["R"] @ g["R"].T, np.eye(3), atol=1e-14)

"""Pins of the conductivity oracle (oracle/conductivity.py) on the CPU.

Fixed by the closed-form laminate (arithmetic mean along the layers, harmonic
mean across, reached exactly when every frequency of the pattern is parallel
to the normal), the homogeneous medium, the projection property of the scalar
Green operator, the Wiener bounds, the mean-gradient invariant, the 2-D / 3-D
identity and the agreement of the Basic Scheme with CG and with a Krylov
Galerkin solve.
"""
import numpy as np
import pytest

import synth
from oracle import conductivity as K
from oracle.dft import make_transform

KV = np.array([1.0, 10.0, 3.0])


def rnd_phase(seed, n):
    def f(pts, m):
        key = (pts.astype(np.int64) * np.array([7919, 104729, 1299709][: pts.shape[1]])).sum(axis=1)
        return (np.random.default_rng(seed).permutation(97)[np.abs(key) % 97] % n).astype(np.uint8)
    return f


def test_gamma0_scalar_is_a_projection():
    rng = np.random.default_rng(1)
    H = rng.integers(-5, 6, size=(40, 3))
    H = H[np.any(H != 0, axis=1)]
    k0 = 2.5
    t = rng.standard_normal((3, len(H))) + 1j * rng.standard_normal((3, len(H)))
    g = -K.gamma0_scalar(k0, H, t)                  # Gamma0 t
    gg = -K.gamma0_scalar(k0, H, k0 * g)            # Gamma0 k0 Gamma0 t
    assert np.allclose(gg, g, atol=1e-13)
    # degree 0 in h and parallel to h
    assert np.allclose(-K.gamma0_scalar(k0, 3 * H, t), g, atol=1e-13)
    assert np.allclose(np.cross(g.T, H.astype(float)), 0.0, atol=1e-12)


@pytest.mark.parametrize("scheme", ["basic", "cg"])
def test_exact_laminate_on_the_aligned_rank1_pattern(scheme):
    """M = [[m, 2m], [0, 1]]: all frequencies parallel to (1, 2); the discrete
    solution is the laminate closed form."""
    M = [[512, 1024], [0, 1]]
    T = make_transform(M)
    ph = synth.laminate_phase(T.points, T.m)
    kv = np.array([1.0, 10.0])
    Ke, runs = K.effective_conductivity(M, ph, kv, K.default_reference_conductivity(kv), tol=1e-13, transform=T,
                                        scheme=scheme)
    ex = K.laminate_conductivity(1.0, 10.0, float(np.mean(ph == 0)), [1, 2])
    assert np.max(np.abs(Ke - ex)) <= 1e-11 * np.abs(ex).max()


def test_exact_laminate_on_a_grid_with_axis_normal_layers():
    """diag(32, 16), phase by x1 only: frequencies along e1 (the Nyquist class is self-conjugate)."""
    M = [[32, 0], [0, 16]]
    T = make_transform(M)
    ph = (T.points[:, 0] >= 0).astype(np.uint8)
    kv = np.array([2.0, 7.0])
    Ke, _ = K.effective_conductivity(M, ph, kv, K.default_reference_conductivity(kv), tol=1e-13, transform=T)
    ex = K.laminate_conductivity(2.0, 7.0, float(np.mean(ph == 0)), [1, 0])
    assert np.max(np.abs(Ke - ex)) <= 1e-11 * np.abs(ex).max()


def test_homogeneous_medium_and_invariants():
    M = [[6, 1], [0, 5]]
    T = make_transform(M)
    r = K.basic_scheme_thermal(M, np.zeros(T.m, np.uint8), [2.0], 2.0, [0.3, -0.1], tol=1e-12, transform=T)
    assert r.iters == 0 and np.allclose(r.mean_stress, [0.6, -0.2])
    M = [[12, 0], [4, 10]]
    T = make_transform(M)
    ph = rnd_phase(3, 3)(T.points, T.m)
    r = K.basic_scheme_thermal(M, ph, KV, K.default_reference_conductivity(KV), [0.2, 0.7], transform=T, fixed_iters=6)
    assert np.allclose(r.eps.mean(axis=1), [0.2, 0.7], atol=1e-14)


@pytest.mark.parametrize("M", [[[12, 0], [4, 10]], [[6, 0, 0], [2, 6, 0], [0, 1, 4]]])
def test_wiener_bounds_symmetry_and_cg_agreement(M):
    T = make_transform(M)
    ph = rnd_phase(4, 3)(T.points, T.m)
    k0 = K.default_reference_conductivity(KV)
    Kb, rb = K.effective_conductivity(M, ph, KV, k0, tol=1e-12, transform=T)
    Kc, rc = K.effective_conductivity(M, ph, KV, k0, tol=1e-12, transform=T, scheme="cg")
    assert np.allclose(Kb, Kb.T, atol=1e-10)
    assert np.max(np.abs(Kb - Kc)) <= 1e-9 * np.abs(Kb).max()
    assert max(r.iters for r in rc) < min(r.iters for r in rb)
    f = np.bincount(ph, minlength=3) / T.m
    ka = float(f @ KV)
    kh = 1.0 / float(f @ (1.0 / KV))
    ev = np.linalg.eigvalsh(0.5 * (Kb + Kb.T))
    assert kh - 1e-10 <= ev.min() and ev.max() <= ka + 1e-10


def test_plane_problem_equals_3d_with_one_point_along_x3():
    M2 = [[12, 2], [3, 10]]
    M3 = [[12, 2, 0], [3, 10, 0], [0, 0, 1]]
    T2, T3 = make_transform(M2), make_transform(M3)
    f = lambda pts: (np.abs((pts[:, 0] * 7 + pts[:, 1] * 3)) % 3).astype(np.uint8)  # noqa: E731
    k0 = K.default_reference_conductivity(KV)
    r2 = K.basic_scheme_thermal(M2, f(T2.points), KV, k0, [0.4, -0.3], transform=T2, fixed_iters=5)
    r3 = K.basic_scheme_thermal(M3, f(T3.points[:, :2]), KV, k0, [0.4, -0.3, 0.0], transform=T3, fixed_iters=5)
    pos = {tuple(p): i for i, p in enumerate(T3.points[:, :2].tolist())}
    idx = np.array([pos[tuple(p)] for p in T2.points.tolist()])
    assert np.allclose(r3.eps[:2, idx], r2.eps, atol=1e-13) and np.allclose(r3.eps[2], 0.0, atol=1e-14)
    assert np.allclose(r2.history, r3.history, rtol=1e-12)


@pytest.mark.parametrize("k", [1, 3])
def test_cg_iterates_are_krylov_galerkin_solutions(k):
    M = [[6, 2], [1, 5]]
    T = make_transform(M)
    ph = rnd_phase(5, 3)(T.points, T.m)
    pr = K.ThermalProblem(M, ph, KV, K.default_reference_conductivity(KV), transform=T)
    eb = np.array([0.3, -0.4])
    r = K.cg_thermal(M, ph, KV, pr.k0, eb, fixed_iters=k, prob=pr)
    b = -pr.apply(np.broadcast_to(eb[:, None], (2, T.m)))
    basis, v = [], b
    for _ in range(k):
        w = v.copy()
        for _ in range(2):
            for u in basis:
                w = w - pr.inner(u, w) * u
        basis.append(w / np.sqrt(pr.inner(w, w)))
        v = pr.apply(basis[-1])
    G = np.array([[pr.inner(u, pr.apply(v)) for v in basis] for u in basis])
    c = np.linalg.solve(G, np.array([pr.inner(u, b) for u in basis]))
    x = sum(ci * u for ci, u in zip(c, basis))
    assert np.max(np.abs((r.eps - eb[:, None]) - x)) <= 1e-9 * np.max(np.abs(x))

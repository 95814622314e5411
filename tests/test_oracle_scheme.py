"""Pins of the oracle's Algorithm 1 and C_eff (Sec. 3.2, Def. 3.1, Sec. 4.1)."""
import math

import numpy as np
import pytest

import synth
from oracle import closed_forms as CF
from oracle import elasticity as E
from oracle.dft import NaiveDFT, SnfFFT, make_transform

LAM = np.array(synth.LAMINATE_LAME)
REF = E.default_reference(LAM)


def test_reference_is_phase_mean():
    lam0, mu0 = REF
    assert math.isclose(lam0, 3.1730769230769234, rel_tol=1e-14)
    assert math.isclose(mu0, 2.1153846153846154, rel_tol=1e-14)


@pytest.mark.parametrize("M", [[[8, 0], [0, 8]], [[6, 2], [1, 5]], [[4, 0, 0], [0, 4, 0], [0, 0, 2]]])
def test_homogeneous_medium(M):
    """Homogeneous C: zero updates and C_eff = C."""
    T = make_transform(M)
    d = len(M)
    ph = np.zeros(T.m, dtype=np.uint8)
    lame = np.array([[1.2, 0.7]])
    C, runs = E.effective_stiffness(M, ph, lame, (2.0, 1.0), transform=T)
    assert all(r.iters == 0 for r in runs)
    assert np.allclose(C, E.tensor4_to_mandel(E.iso_tensor(1.2, 0.7, d)), atol=1e-13)


@pytest.mark.parametrize("m", [64, 256])
def test_exact_laminate_on_aligned_rank1_pattern(m):
    """All frequencies parallel to the normal: the discrete solution is the closed form.

    M^T = [m q | w] with [q w] unimodular gives G(M^T) = {kappa q}; for q = (1, 2)
    that is M = [[m, 2m], [0, 1]].
    """
    M = [[m, 2 * m], [0, 1]]
    T = make_transform(M)
    ph = synth.laminate_phase(T.points, T.m)
    assert np.sum(ph == 0) == m // 2
    C, runs = E.effective_stiffness(M, ph, LAM, REF, tol=1e-13, transform=T)
    n = [1, 2]
    assert np.allclose(C, CF.laminate_milton(*LAM, 0.5, n), atol=1e-12)
    assert np.allclose(C, CF.laminate_ceff_jump(*LAM, 0.5, n), atol=1e-12)
    # strain field: piecewise constant eps1 / eps2
    for k, r in enumerate(runs):
        load = E.unit_loads(2)[k]
        e1, e2, _ = CF.laminate_jump(*LAM, 0.5, n, load)
        expect = np.where(ph[None, None, :] == 0, e1[:, :, None], e2[:, :, None])
        assert np.allclose(r.eps, expect, atol=1e-12)


def test_laminate_routes_agree():
    for n in ([1, 2], [1, 0.5], [0.3, -1.0]):
        for f1 in (0.2, 0.5, 0.9):
            assert np.allclose(CF.laminate_milton(*LAM, f1, n), CF.laminate_ceff_jump(*LAM, f1, n), atol=1e-12)
    n3 = [0.2, -0.5, 0.8]
    assert np.allclose(CF.laminate_milton(*LAM, 0.3, n3), CF.laminate_ceff_jump(*LAM, 0.3, n3), atol=1e-12)


def test_invariants_on_pixel_laminate():
    """diag(32,32): mean strain = eps0 at every n; symmetric C_eff; Hill-Mandel;
    Reuss <= C_eff <= Voigt; C_eff near the closed form."""
    M = [[32, 0], [0, 32]]
    T = make_transform(M)
    ph = synth.laminate_phase(T.points, T.m)
    eps_bar = E.unit_loads(2)[0]
    for n in (1, 3, 7):
        r = E.basic_scheme(M, ph, LAM, REF, eps_bar, transform=T, fixed_iters=n)
        assert np.allclose(r.eps.mean(axis=2), eps_bar, atol=1e-14)
    C, runs = E.effective_stiffness(M, ph, LAM, REF, tol=1e-11, transform=T)
    assert np.allclose(C, C.T, atol=1e-9)
    for k, r in enumerate(runs):
        tensors = [E.iso_tensor(*l, 2) for l in LAM]
        sig = E.apply_phases(tensors, ph, r.eps)
        hm = np.mean(np.einsum("ijn,ijn->n", sig, r.eps))
        assert math.isclose(hm, float(np.einsum("ij,ij", sig.mean(axis=2), r.eps.mean(axis=2))), rel_tol=1e-9)
    f = np.mean(ph == 0)
    Cm = [E.tensor4_to_mandel(E.iso_tensor(*l, 2)) for l in LAM]
    voigt = f * Cm[0] + (1 - f) * Cm[1]
    reuss = np.linalg.inv(f * np.linalg.inv(Cm[0]) + (1 - f) * np.linalg.inv(Cm[1]))
    assert np.linalg.eigvalsh(voigt - C).min() > -1e-9
    assert np.linalg.eigvalsh(C - reuss).min() > -1e-9
    ex = CF.laminate_milton(*LAM, 0.5, [1, 2])
    assert np.linalg.norm(C - ex) / np.linalg.norm(ex) < 0.05


def test_residual_decreases_and_counts_updates():
    M = [[16, 0], [0, 16]]
    T = make_transform(M)
    ph = synth.laminate_phase(T.points, T.m)
    r = E.basic_scheme(M, ph, LAM, REF, E.unit_loads(2)[0], tol=1e-8, transform=T)
    assert r.status == 0 and r.resid <= 1e-8
    assert len(r.history) == r.iters + 1
    h = np.array(r.history)
    assert np.all(h[1:] < h[:-1] * 1.0001)
    # contraction factor of the Basic Scheme with the phase-mean reference:
    # (kappa - 1)/(kappa + 1), kappa = stiffness contrast 10
    rate = (h[-1] / h[5]) ** (1.0 / (len(h) - 6))
    assert rate < 9.0 / 11.0 + 0.02


def test_divergence_detected():
    """A reference far below half the stiffest phase makes the scheme diverge."""
    M = [[16, 0], [0, 16]]
    T = make_transform(M)
    ph = synth.laminate_phase(T.points, T.m)
    r = E.basic_scheme(M, ph, LAM, (0.2, 0.1), E.unit_loads(2)[0], tol=1e-8, max_iter=500, transform=T)
    assert r.status == 2


def test_plane_strain_equals_3d_with_unit_third_axis():
    """d = 2 equals d = 3 with M_33 = 1 and eps0_33 = 0."""
    M2 = [[6, 2], [1, 5]]
    M3 = [[6, 2, 0], [1, 5, 0], [0, 0, 1]]
    T2, T3 = make_transform(M2), make_transform(M3)
    ph2 = synth.random_phase_field(T2.m, 2, 11)
    pos = {tuple(p): i for i, p in enumerate(T2.points.tolist())}
    ph3 = np.array([ph2[pos[tuple(p[:2])]] for p in T3.points.tolist()], dtype=np.uint8)
    e2 = np.array([[0.3, 0.1], [0.1, -0.2]])
    e3 = np.zeros((3, 3))
    e3[:2, :2] = e2
    r2 = E.basic_scheme(M2, ph2, LAM, REF, e2, transform=T2, fixed_iters=6)
    r3 = E.basic_scheme(M3, ph3, LAM, REF, e3, transform=T3, fixed_iters=6)
    eps3 = np.array([r3.eps[:2, :2, i] for i in range(T3.m)])
    eps2 = np.array([r2.eps[:, :, pos[tuple(p[:2])]] for p in T3.points.tolist()])
    assert np.allclose(eps2, eps3, atol=1e-13)
    assert np.allclose(r3.eps[2, :, :], 0.0, atol=1e-14)


def test_naive_and_fft_routes_give_same_solve():
    M = [[8, -4], [2, 7]]
    N, F = NaiveDFT(M), SnfFFT(M)
    ph_n = synth.random_phase_field(N.m, 3, 12)
    pos = {tuple(p): i for i, p in enumerate(N.points.tolist())}
    ph_f = np.array([ph_n[pos[tuple(p)]] for p in F.points.tolist()], dtype=np.uint8)
    lame = np.array([[1.0, 0.5], [4.0, 2.0], [2.0, 3.0]])
    ref = E.default_reference(lame)
    e = np.array([[0.0, 0.5], [0.5, 0.0]])
    rn = E.basic_scheme(M, ph_n, lame, ref, e, transform=N, fixed_iters=5)
    rf = E.basic_scheme(M, ph_f, lame, ref, e, transform=F, fixed_iters=5)
    back = np.array([rn.eps[:, :, pos[tuple(p)]] for p in F.points.tolist()])
    assert np.allclose(back, rf.eps.transpose(2, 0, 1), atol=1e-13)
    assert np.allclose(rn.history, rf.history, rtol=1e-10)


@pytest.mark.parametrize("M", [[[12, 0, 0], [0, 6, 0], [3, 0, 4]], [[16, 0], [4, 16]]])
def test_cauchy_step_from_traction_step(M):
    """The update of Algorithm 1 depends on tau_hat only through t = tau_hat xi, so
    |eps(n+1) - eps(n)|^2 = m sum_{h active, h != 0} |sym(xi (x) K^{-1} dt_h)|^2 with
    dt = t(n) - t(n-1) and K^{-1} = (I - beta xi xi^T) / mu0, i.e. per frequency
    (|dt|^2 + (1 - 4 beta + 2 beta^2) |xi . dt|^2) / (2 mu0^2) (Parseval with the
    1/m-normalised transform).  Checked against differences of the iterates."""
    T = make_transform(M)
    d = len(M)
    lame = np.array([[1.0, 0.5], [4.0, 2.0], [2.0, 3.0]])
    lam0, mu0 = E.default_reference(lame)
    beta = (lam0 + mu0) / (lam0 + 2.0 * mu0)
    ph = np.random.default_rng(7).integers(0, 3, T.m)
    A = np.random.default_rng(8).standard_normal((d, d))
    eps0 = 0.5 * (A + A.T)
    H = np.asarray(T.freqs, dtype=np.int64)
    zero = np.flatnonzero(np.all(H == 0, axis=1))[0]
    act = E.active_classes(M, H)
    act[zero] = False
    xi = H[act] / np.linalg.norm(H[act], axis=1)[:, None]
    tensors = [E.iso_tensor(l, mu, d) for l, mu in lame]
    C0 = E.iso_tensor(lam0, mu0, d)

    def traction(eps):
        tau = E.apply_phases(tensors, ph, eps) - E.contract(C0, eps)
        return np.einsum("ijn,nj->ni", T.forward(tau)[:, :, act], xi)

    runs = [E.basic_scheme(M, ph, lame, (lam0, mu0), eps0, transform=T, fixed_iters=n) for n in range(5)]
    for n in range(1, 4):
        dt = traction(runs[n].eps) - traction(runs[n - 1].eps)
        xd = np.einsum("ni,ni->n", xi, dt)
        per = (np.sum(np.abs(dt) ** 2, axis=1) + (1 - 4 * beta + 2 * beta ** 2) * np.abs(xd) ** 2) / (2 * mu0 ** 2)
        lhs = float(np.sum((runs[n + 1].eps - runs[n].eps) ** 2))
        assert math.isclose(lhs, T.m * float(np.sum(per)), rel_tol=1e-10)
        # and the oracle's own Cauchy record is that difference
        assert math.isclose(runs[4].cauchy[n], math.sqrt(lhs) / float(np.linalg.norm(runs[0].eps)), rel_tol=1e-12)


def test_cauchy_stop_rule_returns_first_iterate_below_tol():
    """stop="cauchy" (Sec. 5.2): eps(n) for the first n with |eps(n+1) - eps(n)| / |eps(0)| <= tol."""
    M = [[32, 0], [0, 32]]
    T = make_transform(M)
    ph = synth.laminate_phase(T.points, T.m, q=(2, 1))
    r = E.basic_scheme(M, ph, LAM, REF, E.unit_loads(2)[0], tol=1e-9, transform=T, stop="cauchy")
    assert r.status == 0 and len(r.cauchy) == r.iters + 1
    assert r.cauchy[-1] <= 1e-9 and all(c > 1e-9 for c in r.cauchy[:-1])
    # the same iterate as running exactly that many updates
    f = E.basic_scheme(M, ph, LAM, REF, E.unit_loads(2)[0], transform=T, fixed_iters=r.iters)
    assert np.array_equal(f.eps, r.eps)

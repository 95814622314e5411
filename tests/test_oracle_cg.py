"""Pins of the conjugate-gradient oracle (oracle/accelerated.py) on the CPU.

Each pin is fixed by something other than the CG code itself: the projection
and symmetry identities of Gamma0 C0, the Galerkin characterisation of CG
iterates (an explicit Krylov basis and a dense solve), the closed-form
laminate, and the Basic Scheme's converged solution of the same problem.
"""
import numpy as np
import pytest

import synth
from oracle import accelerated as A
from oracle import closed_forms as CF
from oracle import elasticity as E
from oracle.dft import make_transform

LAM3 = np.array([[1.0, 0.5], [4.0, 2.0], [2.0, 3.0]])


def rnd_phase(seed, n):
    def f(pts, m):
        key = (pts.astype(np.int64) * np.array([7919, 104729, 1299709][: pts.shape[1]])).sum(axis=1)
        return (np.random.default_rng(seed).permutation(97)[np.abs(key) % 97] % n).astype(np.uint8)
    return f


def make_op(M, lame=LAM3, seed=1):
    T = make_transform(M)
    ph = rnd_phase(seed, len(lame))(T.points, T.m)
    return A.LSOperator(M, ph, lame, E.default_reference(lame), transform=T), ph, T


def rnd_sym(rng, d, m):
    w = rng.standard_normal((d, d, m))
    return 0.5 * (w + w.transpose(1, 0, 2))


@pytest.mark.parametrize("M", [[[6, 2], [1, 5]], [[8, 0], [0, 6]], [[4, 0, 0], [1, 4, 0], [0, 0, 3]]])
def test_operator_symmetric_positive_on_compatible_fields(M):
    op, _, T = make_op(M)
    d = len(M)
    rng = np.random.default_rng(2)
    u = op.project(rnd_sym(rng, d, T.m))
    v = op.project(rnd_sym(rng, d, T.m))
    # Gamma0 C0 is a projection and A maps into its range
    assert np.allclose(op.project(u), u, atol=1e-12 * np.abs(u).max())
    Av = op.apply(v)
    assert np.allclose(op.project(Av), Av, atol=1e-12 * np.abs(Av).max())
    assert abs(np.sum(Av)) < 1e-12 * np.abs(Av).sum()   # zero mean
    # <u, A v>_C0 = <A u, v>_C0 = sum u : C : v  (the identity the kernels use for <p, A p>)
    a = op.inner(u, Av)
    b = op.inner(op.apply(u), v)
    c = float(np.sum(u * op.stress(v)))
    assert abs(a - b) <= 1e-11 * abs(a) and abs(a - c) <= 1e-11 * abs(a)
    assert op.inner(u, op.apply(u)) > 0.0


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_cg_iterates_are_krylov_galerkin_solutions(k):
    """x_k of CG = the energy minimiser over span{b, ..., A^{k-1} b} (dense solve)."""
    M = [[6, 2], [1, 5]]
    op, ph, T = make_op(M, seed=3)
    eps_bar = np.array([[0.3, 0.1], [0.1, -0.2]])
    r = A.conjugate_gradient(M, ph, LAM3, E.default_reference(LAM3), eps_bar, transform=T, fixed_iters=k, op=op)
    x_cg = r.eps - eps_bar[:, :, None]
    x_gal = A.krylov_galerkin(op, eps_bar, k)
    assert np.max(np.abs(x_cg - x_gal)) <= 1e-9 * np.max(np.abs(x_gal))
    # every iterate keeps the prescribed mean strain
    assert np.allclose(r.eps.mean(axis=2), eps_bar, atol=1e-14)


def test_cg_exact_laminate_closed_form():
    """Aligned rank-1 pattern: Gamma0 is constant on the support, CG reaches the
    laminate closed form (Sec. 4.1) within a few updates."""
    M = [[256, 512], [0, 1]]
    lame = np.array(synth.LAMINATE_LAME)
    T = make_transform(M)
    ph = synth.laminate_phase(T.points, T.m)
    C, runs = A.effective_stiffness_cg(M, ph, lame, E.default_reference(lame), tol=1e-13, transform=T)
    ex = CF.laminate_milton(*lame, 0.5, [1, 2])
    assert np.max(np.abs(C - ex)) <= 1e-11 * np.abs(ex).max()
    assert max(r.iters for r in runs) <= 3


@pytest.mark.parametrize("M,seed", [([[12, 0], [4, 10]], 4), ([[6, 0, 0], [2, 6, 0], [0, 1, 4]], 5)])
def test_cg_converges_to_the_basic_scheme_solution(M, seed):
    """Same discrete problem: CG's converged fields and C_eff equal Algorithm 1's."""
    lame = np.array([[1.0, 0.5], [40.0, 20.0], [5.0, 3.0]])
    T = make_transform(M)
    ph = rnd_phase(seed, 3)(T.points, T.m)
    lame0 = E.default_reference(lame)
    d = len(M)
    eps_bar = np.eye(d) * 0.01 + 0.004 * (np.ones((d, d)) - np.eye(d))
    rb = E.basic_scheme(M, ph, lame, lame0, eps_bar, tol=1e-12, max_iter=20000, transform=T)
    rc = A.conjugate_gradient(M, ph, lame, lame0, eps_bar, tol=1e-12, max_iter=2000, transform=T)
    assert rb.status == 0 and rc.status == 0
    assert np.max(np.abs(rc.eps - rb.eps)) <= 1e-9 * np.max(np.abs(rb.eps))
    assert np.allclose(rc.mean_stress, rb.mean_stress, rtol=1e-10, atol=1e-13)
    assert rc.iters < rb.iters      # contrast 40: CG needs far fewer updates


def test_cg_homogeneous_and_residual_definition():
    M = [[6, 1], [0, 5]]
    T = make_transform(M)
    r = A.conjugate_gradient(M, np.zeros(T.m, np.uint8), [[1.0, 0.7]], (1.0, 0.7), np.diag([0.1, 0.2]), tol=1e-12, transform=T)
    assert r.iters == 0 and r.resid < 1e-14
    # r(n) is the Basic Scheme's equilibrium residual of the same field
    op, ph, T = make_op([[8, 2], [0, 8]], seed=6)
    eb = np.diag([0.1, -0.05])
    rc = A.conjugate_gradient([[8, 2], [0, 8]], ph, LAM3, E.default_reference(LAM3), eb, transform=T, fixed_iters=3, op=op)
    rb = E.basic_scheme([[8, 2], [0, 8]], ph, LAM3, E.default_reference(LAM3), eb, transform=T, fixed_iters=0,
                        init=rc.eps - eb[:, :, None])
    assert abs(rb.history[0] - rc.history[-1]) <= 1e-12 * rc.history[-1]

"""Oracle pins for transformed patterns P_L(M) (Def. 3.3).

The wave vector of class h on the cell L[-1/2,1/2)^d is L^{-T} h.  Pins:
* closed form: on an aligned rank-1 pattern every active frequency is a
  multiple of q, so a laminate whose layers are the level sets of q^T y is
  solved exactly; in the physical frame its normal is L^{-T} q, and C_eff must
  be the laminate formula for that normal (a non-symmetric L separates L^{-T}
  from L^{-1}, L^T and L);
* equivariance: with isotropic phases, a rotated cell L = Q under the rotated
  load Q eps0 Q^T gives the rotated iterates Q eps(n) Q^T at every point and
  the same residual history (fails for a transposed or inverted Q);
* scale invariance: L = s I is the plain pattern.
"""
import numpy as np
import pytest

import synth
from oracle import closed_forms as CF
from oracle import elasticity as E
from oracle.dft import make_transform

LAM = np.array(synth.LAMINATE_LAME)
REF = E.default_reference(LAM)
L2 = np.array([[1.0, 0.45], [-0.3, 1.25]])


def rotation(seed):
    A = np.random.default_rng(seed).standard_normal((3, 3))
    Q, R = np.linalg.qr(A)
    Q = Q * np.sign(np.diag(R))[None, :]
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    return Q


@pytest.mark.parametrize("L", [L2, np.array([[0.7, 0.0], [0.9, 1.4]])])
def test_transformed_laminate_is_the_closed_form_with_normal_L_inv_T_q(L):
    m = 32
    M = [[m, 2 * m], [0, 1]]          # G(M^T) = {kappa (1, 2)}
    q = np.array([1.0, 2.0])
    T = make_transform(M)
    ph = synth.laminate_phase(T.points, T.m)
    C, runs = E.effective_stiffness(M, ph, LAM, REF, tol=1e-13, transform=T, cell=L)
    n_phys = np.linalg.inv(L).T @ q
    assert np.allclose(C, CF.laminate_milton(*LAM, 0.5, n_phys), atol=1e-12)
    assert np.allclose(C, CF.laminate_ceff_jump(*LAM, 0.5, n_phys), atol=1e-12)
    # the pin separates the readings: the other candidate normals give other tensors
    for wrong in (np.linalg.inv(L) @ q, L.T @ q, L @ q):
        assert np.abs(C - CF.laminate_milton(*LAM, 0.5, wrong)).max() > 1e-3
    # the strain is piecewise constant with the jump of the physical normal
    for k, r in enumerate(runs):
        e1, e2, _ = CF.laminate_jump(*LAM, 0.5, n_phys, E.unit_loads(2)[k])
        expect = np.where(ph[None, None, :] == 0, e1[:, :, None], e2[:, :, None])
        assert np.allclose(r.eps, expect, atol=1e-12)


def test_rotated_cell_rotates_the_iterates():
    M = [[6, 0, 0], [1, 5, 0], [0, 2, 4]]
    T = make_transform(M)
    rng = np.random.default_rng(21)
    ph = rng.integers(0, 3, T.m)
    lame = np.array([[1.0, 0.5], [4.0, 2.0], [2.0, 3.0]])
    ref = E.default_reference(lame)
    A = rng.standard_normal((3, 3))
    eps0 = 0.5 * (A + A.T)
    Q = rotation(5)
    r0 = E.basic_scheme(M, ph, lame, ref, eps0, transform=T, fixed_iters=5)
    r1 = E.basic_scheme(M, ph, lame, ref, Q @ eps0 @ Q.T, transform=T, fixed_iters=5, cell=Q)
    rot = np.einsum("ia,abn,jb->ijn", Q, r0.eps, Q)
    assert np.abs(r1.eps - rot).max() < 1e-12 * np.abs(rot).max()
    assert np.allclose(r1.history, r0.history, rtol=1e-11, atol=0)
    assert np.allclose(r1.mean_stress, Q @ r0.mean_stress @ Q.T, atol=1e-12)
    # a transposed rotation is not a symmetry of the scheme
    r2 = E.basic_scheme(M, ph, lame, ref, Q @ eps0 @ Q.T, transform=T, fixed_iters=5, cell=Q.T)
    assert np.abs(r2.eps - rot).max() > 1e-4 * np.abs(rot).max()


def test_uniformly_scaled_cell_is_the_plain_pattern():
    M = [[12, 0, 0], [0, 6, 0], [3, 0, 4]]
    T = make_transform(M)
    ph = np.random.default_rng(3).integers(0, 2, T.m)
    lame = np.array([[1.0, 0.5], [4.0, 2.0]])
    ref = E.default_reference(lame)
    eps0 = np.diag([1.0, -0.3, 0.2])
    r0 = E.basic_scheme(M, ph, lame, ref, eps0, transform=T, fixed_iters=4)
    r1 = E.basic_scheme(M, ph, lame, ref, eps0, transform=T, fixed_iters=4, cell=2.5 * np.eye(3))
    assert np.abs(r1.eps - r0.eps).max() < 1e-13
    assert np.allclose(r1.history, r0.history, rtol=1e-12, atol=0)

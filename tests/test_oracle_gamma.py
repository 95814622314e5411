"""Pins of the oracle's Green operator Gamma0 (Sec. 3.1-3.2)."""
import numpy as np
import pytest

from oracle import elasticity as E
from oracle import lattice as L
from oracle.dft import NaiveDFT


def iso_gamma_closed_form(lam0, mu0, k):
    """Textbook Gamma0 of an isotropic reference medium (Mura / Moulinec-Suquet):
    Gamma_ijkl = (d_ki x_l x_j + d_li x_k x_j + d_kj x_l x_i + d_lj x_k x_i)/(4 mu0 |x|^2)
                 - (lam0 + mu0)/(mu0 (lam0 + 2 mu0)) x_i x_j x_k x_l / |x|^4.
    """
    d = k.size
    I = np.eye(d)
    n2 = float(k @ k)
    G = (np.einsum("ki,l,j->ijkl", I, k, k) + np.einsum("li,k,j->ijkl", I, k, k)
         + np.einsum("kj,l,i->ijkl", I, k, k) + np.einsum("lj,k,i->ijkl", I, k, k)) / (4.0 * mu0 * n2)
    G -= (lam0 + mu0) / (mu0 * (lam0 + 2.0 * mu0)) * np.einsum("i,j,k,l->ijkl", k, k, k, k) / n2 ** 2
    return G


def rand_sym(rng, d, n, cplx=True):
    A = rng.standard_normal((d, d, n)) + (1j * rng.standard_normal((d, d, n)) if cplx else 0)
    return 0.5 * (A + A.transpose(1, 0, 2))


@pytest.mark.parametrize("d", [2, 3])
def test_general_solve_equals_isotropic_closed_form(d):
    rng = np.random.default_rng(5)
    lam0, mu0 = 1.7, 0.9
    C0 = E.iso_tensor(lam0, mu0, d)
    H = rng.integers(-9, 10, size=(20, d))
    H = H[np.any(H != 0, axis=1)]
    tau = rand_sym(rng, d, H.shape[0])
    out = E.gamma0_apply(C0, H, tau)
    for n, h in enumerate(H.astype(float)):
        G = iso_gamma_closed_form(lam0, mu0, h)
        assert np.allclose(out[:, :, n], -np.einsum("ijkl,kl->ij", G, tau[:, :, n]), atol=1e-13)


@pytest.mark.parametrize("d", [2, 3])
def test_projection_identities(d):
    """Gamma0 C0 Gamma0 = Gamma0 and Gsym^H C0 Gamma0 = Gsym^H per frequency."""
    rng = np.random.default_rng(6)
    C0 = E.iso_tensor(2.3, 1.1, d)
    H = rng.integers(-7, 8, size=(30, d))
    H = H[np.any(H != 0, axis=1)]
    tau = rand_sym(rng, d, H.shape[0])
    g1 = -E.gamma0_apply(C0, H, tau)                     # Gamma0 tau
    g2 = -E.gamma0_apply(C0, H, E.contract(C0, g1))      # Gamma0 C0 Gamma0 tau
    assert np.allclose(g1, g2, atol=1e-13)
    lhs = np.einsum("ijn,nj->ni", E.contract(C0, g1), H.astype(float))
    rhs = np.einsum("ijn,nj->ni", tau, H.astype(float))
    assert np.allclose(lhs, rhs, atol=1e-12)
    # homogeneous of degree 0
    g3 = -E.gamma0_apply(C0, 3 * H, tau)
    assert np.allclose(g1, g3, atol=1e-13)


def test_active_classes_on_even_grid():
    """diag(4,4): unpaired classes are those with one coordinate -2 and not self-conjugate."""
    M = [[4, 0], [0, 4]]
    H = L.generating_set(L.transpose(M))
    act = E.active_classes(M, H)
    for h, a in zip(H.tolist(), act):
        has_half = -2 in h
        self_conj = all(v in (0, -2) for v in h)
        assert a == (not has_half or self_conj)
    # odd grid: everything active
    M = [[5, 0], [0, 3]]
    H = L.generating_set(L.transpose(M))
    assert E.active_classes(M, H).all()


@pytest.mark.parametrize("M", [[[8, 0], [0, 8]], [[8, -4], [2, 7]], [[6, 2], [1, 5]],
                               [[4, 0, 0], [0, 4, 0], [0, 0, 2]], [[3, 1, 0], [0, 2, 1], [1, 0, 4]]])
def test_field_projection_idempotent_and_real(M):
    """P = F^{-1} Gamma C0 F is a real idempotent operator under the hermitian rule."""
    T = NaiveDFT(M)
    d = len(M)
    H = T.freqs
    act = E.active_classes(M, H)
    zero = np.flatnonzero(np.all(H == 0, axis=1))[0]
    upd = act.copy()
    upd[zero] = False
    C0 = E.iso_tensor(1.3, 0.8, d)
    rng = np.random.default_rng(7)
    f = rand_sym(rng, d, T.m, cplx=False)

    def P(field):
        fh = T.forward(field)
        out = np.zeros_like(fh)
        out[:, :, upd] = -E.gamma0_apply(C0, H[upd], E.contract(C0, fh[:, :, upd]))
        return T.inverse(out)

    p1 = P(f)
    assert np.max(np.abs(p1.imag)) < 1e-12
    p2 = P(p1.real)
    assert np.allclose(p1, p2, atol=1e-12)

"""Pins of the oracle's 1-D GLL building blocks (Sec. 2.2, Def. GLL quadrature
rule and Def. GLL interpolation basis) against closed forms and exactness."""
import numpy as np
import pytest

from oracle import oracle as orc


def test_gll_closed_forms():
    # p = 2: {-1, 0, 1}, weights {1/3, 4/3, 1/3}
    xi, rho = orc.gll(2)
    np.testing.assert_allclose(xi, [-1, 0, 1], atol=1e-15)
    np.testing.assert_allclose(rho, [1 / 3, 4 / 3, 1 / 3], rtol=1e-14)
    # p = 3: +-1, +-1/sqrt(5); weights 1/6, 5/6
    xi, rho = orc.gll(3)
    np.testing.assert_allclose(xi, [-1, -1 / np.sqrt(5), 1 / np.sqrt(5), 1], atol=1e-15)
    np.testing.assert_allclose(rho, [1 / 6, 5 / 6, 5 / 6, 1 / 6], rtol=1e-14)
    # p = 4: 0, +-sqrt(3/7), +-1; weights 1/10, 49/90, 32/45
    xi, rho = orc.gll(4)
    np.testing.assert_allclose(xi, [-1, -np.sqrt(3 / 7), 0, np.sqrt(3 / 7), 1], atol=1e-15)
    np.testing.assert_allclose(rho, [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10], rtol=1e-14)


@pytest.mark.parametrize("p", [2, 3, 5, 8, 16, 33, 64, 128, 256])
def test_gll_exactness_degree(p):
    """The rule integrates x^k exactly for k <= 2p-1 and not for k = 2p."""
    xi, rho = orc.gll(p)
    assert np.all(np.diff(xi) > 0)
    np.testing.assert_allclose(xi, -xi[::-1], atol=1e-14)
    np.testing.assert_allclose(rho.sum(), 2.0, rtol=1e-13)
    for k in range(0, 2 * p):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(rho * xi**k) - exact) < 1e-12 * max(1.0, p / 8), (p, k)
    # degree 2p fails: the rule gives sum rho L_p^2 = 2/p, the integral is 2/(2p+1)
    Lp = np.array([orc.legendre(p, x)[0] for x in xi])
    np.testing.assert_allclose(np.sum(rho * Lp**2), 2.0 / p, rtol=1e-12)
    assert abs(2.0 / p - 2.0 / (2 * p + 1)) > 0.5 / p


@pytest.mark.parametrize("p", [2, 4, 7, 16, 64])
def test_gll_nodes_are_roots_of_dLp(p):
    xi, rho = orc.gll(p)
    for x in xi[1:-1]:
        L, dL = orc.legendre(p, x)
        assert abs(dL) < 1e-11 * p * p
    # weights from the definition 2 / (p (p+1) L_p^2)
    for x, r in zip(xi, rho):
        L, _ = orc.legendre(p, x)
        np.testing.assert_allclose(r, 2.0 / (p * (p + 1) * L * L), rtol=1e-14)


@pytest.mark.parametrize("p", [2, 3, 6, 16, 64, 128])
def test_deriv_exact_on_polynomials(p):
    xi, _ = orc.gll(p)
    D = orc.deriv(p, xi)
    np.testing.assert_allclose(D @ np.ones(p + 1), 0.0, atol=1e-10 * p * p)
    # corner value of the GLL derivative matrix: -p(p+1)/4
    np.testing.assert_allclose(D[0, 0], -p * (p + 1) / 4.0, rtol=1e-11)
    np.testing.assert_allclose(D[p, p], p * (p + 1) / 4.0, rtol=1e-11)
    # interior diagonal vanishes (symmetric nodes)
    assert np.max(np.abs(np.diag(D)[1:-1])) < 1e-10 * p
    for k in range(0, min(p, 12) + 1):
        np.testing.assert_allclose(D @ xi**k, k * xi ** max(k - 1, 0) * (k > 0),
                                   atol=1e-10 * p * p)


@pytest.mark.parametrize("pc,pf", [(2, 4), (4, 8), (8, 16), (32, 64), (64, 128)])
def test_interp_exact_and_nested(pc, pf):
    xc, _ = orc.gll(pc)
    xf, _ = orc.gll(pf)
    J = orc.interp(pc, xc, xf)
    np.testing.assert_allclose(J.sum(axis=1), 1.0, atol=1e-12)
    for k in range(0, min(pc, 10) + 1):
        np.testing.assert_allclose(J @ xc**k, xf**k, atol=1e-11)
    # end points map to end points exactly (zero boundary preserved)
    assert J[0, 0] == 1.0 and np.all(J[0, 1:] == 0.0)
    assert J[-1, -1] == 1.0 and np.all(J[-1, :-1] == 0.0)


def test_interp_composes():
    x2, _ = orc.gll(2)
    x4, _ = orc.gll(4)
    x8, _ = orc.gll(8)
    np.testing.assert_allclose(orc.interp(4, x4, x8) @ orc.interp(2, x2, x4),
                               orc.interp(2, x2, x8), atol=1e-13)


@pytest.mark.parametrize("p", [16, 64, 128, 256])
def test_deriv_against_extended_precision(p):
    """D at the oracle's own nodes against the same derivatives evaluated in
    80-bit long double (an independent precision): every entry within
    p eps max|D| / 4 (each entry is a product of p factors), and the rows
    sum to zero within eps p^2 (the basis is a
    partition of unity).  A diagonal taken from the product rule's
    sum_k 1/(xi_i - xi_k) leaves row sums of 1.2e-11 at p = 128, which fails."""
    xi, _ = orc.gll(p)
    D = orc.deriv(p, xi)
    x = xi.astype(np.longdouble)
    n = p + 1
    diff = x[:, None] - x[None, :]
    np.fill_diagonal(diff, 1)
    # pi_j'(x_i) = (w_j / w_i) / (x_i - x_j), w_j = 1 / prod_{k != j} (x_j - x_k)
    w = 1 / np.prod(diff, axis=1)
    Dl = (w[None, :] / w[:, None]) / diff
    np.fill_diagonal(Dl, 0)
    np.fill_diagonal(Dl, -Dl.sum(axis=1))
    scale = np.abs(D).max()
    assert float(np.abs(D - Dl).max()) <= p * np.finfo(float).eps * scale / 4
    assert np.abs(D.sum(axis=1)).max() <= np.finfo(float).eps * p * p

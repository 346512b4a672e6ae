"""Pins of the oracle's discretisation (eq. discreteBilinear, Sec. 2.3) against
symmetry, the constant null space, the Kronecker form of the undeformed
operator, exact energy integrals of polynomials, and the closed-form geometry
of the unit square."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2504_10710_amd import inputs
from tests.helpers import interior_mask, oracle_hier


def _single(problem, p):
    h, ps, coords = oracle_hier(problem, p, p_coarse=p)
    return h, coords[-1]


def test_geometry_unit_square():
    p = 8
    h, X = _single(inputs.table1(1), p)
    G, mass, mindet = h.geom()
    _, rho = orc.gll(p)
    w = np.outer(rho, rho).reshape(-1, order="F")  # w[i + n1 j] = rho_i rho_j
    np.testing.assert_allclose(G[0, 0], w, rtol=1e-13)
    np.testing.assert_allclose(G[1, 1], w, rtol=1e-13)
    np.testing.assert_allclose(G[0, 1], 0.0, atol=1e-14)
    np.testing.assert_allclose(mass, w / 4.0, rtol=1e-13)
    np.testing.assert_allclose(mass.sum(), 1.0, rtol=1e-13)
    np.testing.assert_allclose(mindet, 0.25, rtol=1e-13)


@pytest.mark.parametrize("dim,p,seed", [(2, 8, 0), (2, 12, 3), (3, 4, 1), (3, 6, 2)])
def test_operator_symmetric_and_constant_nullspace(dim, p, seed):
    prob = inputs.config2(seed) if dim == 2 else inputs.config3(seed)
    h, X = _single(prob, p)
    N = (p + 1) ** dim
    rng = np.random.default_rng(seed)
    x, y = rng.standard_normal(N), rng.standard_normal(N)
    Ax = h.apply(x, all_rows=True)
    Ay = h.apply(y, all_rows=True)
    np.testing.assert_allclose(y @ Ax, x @ Ay, rtol=1e-12)
    np.testing.assert_allclose(h.apply(np.ones(N), all_rows=True), 0.0, atol=1e-11 * p * p)
    A = h.dense_interior()
    np.testing.assert_allclose(A, A.T, atol=1e-12 * np.abs(A).max())
    np.linalg.cholesky(A)  # positive definite on the interior


def test_entry_matches_apply():
    p = 6
    h, _ = _single(inputs.config2(5), p)
    N = (p + 1) ** 2
    rng = np.random.default_rng(0)
    for _ in range(20):
        r, c = rng.integers(0, N, size=2)
        e = np.zeros(N)
        e[c] = 1.0
        np.testing.assert_allclose(h.apply(e, all_rows=True)[r], h.entry(r, c), atol=1e-13)


@pytest.mark.parametrize("p", [4, 8, 16])
def test_undeformed_kronecker(p):
    """Unit square: A = (K x W + W x K)/1 with K = D^T W D (1-D GLL stiffness
    on [-1,1]) and W = diag(rho); the unit-square scaling cancels in 2-D."""
    h, _ = _single(inputs.table1(1), p)
    xi, rho = orc.gll(p)
    D = orc.deriv(p, xi)
    W = np.diag(rho)
    K = D.T @ W @ D
    Afull = np.kron(K, W) + np.kron(W, K)  # index j*(p+1)+i: kron(Y, X)
    A = h.dense_interior()
    idx = np.arange(1, p)
    sel = (idx[None, :] + (p + 1) * idx[:, None]).reshape(-1)
    np.testing.assert_allclose(A, Afull[np.ix_(sel, sel)], atol=1e-12 * np.abs(A).max())


@pytest.mark.parametrize("p", [6, 9])
def test_energy_of_polynomials_undeformed(p):
    """u^T A u equals the exact integral of |grad u|^2 over [0,1]^2 for u = x^a y^b
    with a, b <= p-1 (GLL exact to degree 2p-1 per variable)."""
    h, X = _single(inputs.table1(1), p)
    x, y = X
    for a, b in [(1, 0), (2, 3), (p - 1, p - 1), (3, p - 1)]:
        u = x**a * y**b
        exact = a * a / ((2 * a - 1) * (2 * b + 1)) if a > 0 else 0.0
        exact += b * b / ((2 * a + 1) * (2 * b - 1)) if b > 0 else 0.0
        np.testing.assert_allclose(u @ h.apply(u, all_rows=True), exact, rtol=1e-12)


def test_energy_affine_map():
    """Affine (parallelogram) map x = s + 0.3 t, y = 0.8 t: the integral of
    |grad u|^2 for u = x^2 y is a polynomial integral computed exactly by GLL
    (constant Jacobian), checked against an independent high-order Gauss rule."""
    p = 6
    xi, _ = orc.gll(p)
    s = inputs.unit_coords(xi, 2)
    X = np.stack([s[0] + 0.3 * s[1], 0.8 * s[1]])
    h = orc.Hier(2, [p], [X], gamma=1)
    u = X[0] ** 2 * X[1]
    gq, gw = np.polynomial.legendre.leggauss(12)
    S, T = np.meshgrid((gq + 1) / 2, (gq + 1) / 2, indexing="ij")
    Wt = np.outer(gw, gw) / 4
    x, y = S + 0.3 * T, 0.8 * T
    grad2 = (2 * x * y) ** 2 + (x**2) ** 2
    exact = np.sum(Wt * grad2) * 0.8  # |det J| = 0.8
    np.testing.assert_allclose(u @ h.apply(u, all_rows=True), exact, rtol=1e-12)


def test_rhs_lifting():
    """Sec. 2.3: b = M f - A v on the interior, zero on the boundary."""
    p = 8
    prob = inputs.config2(7)
    h, X = _single(prob, p)
    f, g = prob.f(X), prob.g(X)
    b = h.rhs(f, g)
    _, mass, _ = h.geom()
    mask = interior_mask(2, p)
    v = np.where(mask, 0.0, g)
    ref = mass * f - h.apply(v, all_rows=True)
    np.testing.assert_allclose(b[mask], ref[mask], rtol=1e-13, atol=1e-13)
    assert np.all(b[~mask] == 0.0)


@pytest.mark.parametrize("seed", [0, 1])
def test_spectral_convergence_dense(seed):
    """Manufactured u* on the deformed square: the discrete solution (dense
    solve of the interior system) converges exponentially in p."""
    prob_exact = inputs.manufactured_deformed(seed)  # non-homogeneous Dirichlet
    errs = []
    for p in (4, 8, 12, 16, 20, 24):
        h, X = _single(prob_exact, p)
        b = h.rhs(prob_exact.f(X), prob_exact.g(X))
        A = h.dense_interior()
        mask = interior_mask(2, p)
        w = np.linalg.solve(A, b[mask])
        u = prob_exact.g(X).copy()
        u[mask] = w
        errs.append(np.abs(u - prob_exact.exact(X)).max())
    errs = np.array(errs)
    assert np.all(np.diff(np.log(errs)) < 0), errs
    # exponential decay: strictly decreasing, accelerating, three decades overall
    assert np.all(errs[1:] < errs[:-1] / 2.0), errs
    assert errs[-1] < errs[-2] / 5.0 and errs[-1] < 1e-3 * errs[0], errs

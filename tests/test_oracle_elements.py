"""Pins of the oracle's several-element mode (multi-element hp-multigrid, the
paper's closing outlook): the paper defines one element, so each pin checks
a property the standard conforming spectral-element discretisation must have
(K elements per axis, continuous basis, direct stiffness summation):

  * undeformed square: the assembled operator is Kg (x) Mg + Mg (x) Kg with
    Kg, Mg the assembled 1-D element stiffness and mass, built here from the
    1-D pieces only;
  * quadrature exactness: u^T A u equals the integral of |grad u|^2 for
    polynomials of degree <= p_e - 1 per variable (Gauss-Legendre integral);
  * A 1 = 0 on every row, A symmetric, the mass sums to the area;
  * the element-wise transfers reproduce continuous piecewise polynomials of
    the coarse degree, and the interpolation restriction returns the coarse
    values of fine samples of a coarse-space function;
  * the discrete solution converges to a smooth exact solution in p_e and in
    K, and the gamma-cycle preconditioned FGMRES converges in a bounded
    number of iterations as K grows.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2504_10710_amd import inputs


def hier(K, pes, prob=None, **kw):
    """Oracle hierarchy on K x K elements of degrees pes (coarsest first)."""
    prob = prob or inputs.table1(1)          # the undeformed unit square
    coords = [prob.coords(inputs.composite_nodes(orc.gll(pe)[0], K)) for pe in pes]
    return orc.Hier(2, [K * pe for pe in pes], coords, elements=K, **kw), coords


def interior(n1):
    m = np.zeros((n1, n1), dtype=bool)
    m[1:-1, 1:-1] = True
    return m.reshape(-1)


@pytest.mark.parametrize("K,pe", [(2, 4), (4, 4), (2, 8), (3, 4)])
def test_undeformed_operator_is_assembled_1d_kronecker(K, pe):
    h, _ = hier(K, [pe], smoother=orc.SMOOTHER_FEM)
    xi, rho = orc.gll(pe)
    D = orc.deriv(pe, xi).reshape(pe + 1, pe + 1)
    ke = D.T @ np.diag(rho) @ D
    n1 = K * pe + 1
    Kg = np.zeros((n1, n1))
    Mg = np.zeros((n1, n1))
    for e in range(K):
        sl = slice(e * pe, e * pe + pe + 1)
        Kg[sl, sl] += ke
        Mg[sl, sl] += np.diag(rho)
    A = np.kron(Mg, Kg) + np.kron(Kg, Mg)
    m = interior(n1)
    ours = h.dense_interior()
    ref = A[np.ix_(m, m)]
    err = np.abs(ours - ref).max() / np.abs(ref).max()
    print(f"K={K} pe={pe}: max rel. difference {err:.2e}")
    assert err < 1e-14
    # the assembled mass is Mg (x) Mg times the element Jacobian (1 / 2K)^2
    _, mass, _ = h.geom()
    assert np.allclose(mass, np.kron(np.diag(Mg), np.diag(Mg)) / (4.0 * K * K), rtol=1e-14, atol=0)


@pytest.mark.parametrize("K,pe", [(2, 4), (4, 4), (3, 6)])
def test_energy_exact_for_low_degree_polynomials(K, pe):
    h, coords = hier(K, [pe], smoother=orc.SMOOTHER_FEM)
    x, y = coords[0]
    xg, wg = np.polynomial.legendre.leggauss(2 * pe + 2)
    xg, wg = (xg + 1) / 2, wg / 2
    rng = np.random.default_rng(3)
    for _ in range(3):
        c = rng.standard_normal((pe, pe))          # degree <= pe - 1 per variable
        P = np.polynomial.polynomial
        u = P.polyval2d(x, y, c)
        cx = P.polyder(c, axis=0)
        cy = P.polyder(c, axis=1)
        Xg, Yg = np.meshgrid(xg, xg, indexing="ij")
        W = np.outer(wg, wg)
        exact = np.sum(W * (P.polyval2d(Xg, Yg, cx) ** 2 + P.polyval2d(Xg, Yg, cy) ** 2))
        ours = u @ h.apply(u, all_rows=True)
        print(f"K={K} pe={pe}: u^T A u {ours:.15e} exact {exact:.15e}")
        assert abs(ours - exact) <= 1e-12 * abs(exact)


def test_deformed_operator_invariants():
    K, pe = 4, 4
    h, coords = hier(K, [pe], prob=inputs.config2(5), smoother=orc.SMOOTHER_FEM)
    N = coords[0].shape[1]
    y = h.apply(np.ones(N), all_rows=True)
    assert np.abs(y).max() < 1e-12
    A = h.dense_interior()
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    assert np.all(np.linalg.eigvalsh(A) > 0)
    _, mass, mindet = h.geom()
    assert mindet > 0
    # the mapping keeps the unit square: the area is 1 up to quadrature error
    assert abs(mass.sum() - 1.0) < 1e-6


def _grid(h, l):
    n1 = h.plist[l] + 1
    return n1


@pytest.mark.parametrize("K", [2, 4])
def test_transfers_reproduce_continuous_piecewise_polynomials(K):
    """P of a coarse-space function (continuous, a polynomial of degree <= p_c
    on each element, different on different elements) equals it at the fine
    nodes; the interpolation restriction of its fine samples returns its
    coarse values (interior nodes)."""
    pes = [2, 4, 8]
    h, coords = hier(K, pes, smoother=orc.SMOOTHER_FEM, restriction=orc.RESTRICT_INTERP)

    def func(X, pc):
        # continuous, a polynomial of degree pc per variable on each element:
        # |x - 1/2| is linear on each side of the interface x = 1/2 (K even)
        x, y = X
        return (np.abs(x - 0.5) + 0.3) * (1 + x) ** (pc - 1) * (np.abs(y - 0.5) + 0.2) * (2 - y) ** (pc - 1)

    for l in (1, 2):
        pc = pes[l - 1]
        uc = func(coords[l - 1], pc)
        uf = func(coords[l], pc)
        got = h.prolong_add(uc, np.zeros_like(uf), l)
        err = np.abs(got - uf).max() / np.abs(uf).max()
        print(f"K={K} level {l}: prolongation error {err:.2e}")
        assert err < 1e-13
        back = h.restrict(uf, l)
        m = interior(h.plist[l - 1] + 1)
        err_r = np.abs(back[m] - uc[m]).max() / np.abs(uc).max()
        print(f"K={K} level {l}: restriction error {err_r:.2e}")
        assert err_r < 1e-13


def _solve_dense(h, prob, coords):
    X = coords[-1]
    b = h.rhs(prob.f(X), prob.g(X))
    n1 = h.plist[-1] + 1
    m = interior(n1)
    A = h.dense_interior()
    u = prob.g(X).copy()
    u[m] = np.linalg.solve(A, b[m])
    return u


def test_discrete_solution_converges_in_p_and_in_K():
    """-Laplace u = f with a smooth manufactured solution on a deformed
    square: the nodal error falls exponentially with the element degree at
    fixed K and algebraically (at least like h^pe / 4 per halving) with K at
    fixed degree."""
    prob = inputs.manufactured_deformed(2, 0.1)

    def err(K, pe):
        h, coords = hier(K, [pe], prob=prob, smoother=orc.SMOOTHER_FEM)
        u = _solve_dense(h, prob, coords)
        ex = prob.exact(coords[-1])
        return np.abs(u - ex).max() / np.abs(ex).max()

    ep = [err(2, pe) for pe in (4, 8, 16)]
    eK = [err(K, 4) for K in (1, 2, 4)]
    print("K = 2, pe = 4, 8, 16:", ["%.2e" % v for v in ep])
    print("pe = 4, K = 1, 2, 4:", ["%.2e" % v for v in eK])
    assert ep[1] < ep[0] / 100 and ep[2] < ep[1] / 1e3 and ep[2] < 1e-8
    assert eK[1] < eK[0] / 8 and eK[2] < eK[1] / 8


@pytest.mark.parametrize("smoother,alpha", [(orc.SMOOTHER_FEM, 0.16)])
def test_hp_multigrid_iterations_bounded_in_K(smoother, alpha):
    """The gamma-cycle over the element degrees (pe, pe/2, ..., 2 on the same
    K x K elements; exact solve on the coarsest) preconditions FGMRES with a
    count that does not grow with K at fixed element degree, and the result
    is the discrete solution."""
    prob = inputs.config2(7, 0.1)
    counts = {}
    for K in (1, 2, 4):
        pes = [2, 4, 8]
        coords = [prob.coords(inputs.composite_nodes(orc.gll(pe)[0], K)) for pe in pes]
        h = orc.Hier(2, [K * pe for pe in pes], coords, gamma=3, m=1, alpha=alpha,
                     smoother=smoother, restriction=orc.RESTRICT_INTERP, elements=K)
        X = coords[-1]
        b = h.rhs(prob.f(X), prob.g(X))
        x, st, it, _ = h.fgmres(b, rtol=1e-10, maxit=200)
        assert st == 0
        m = interior(h.plist[-1] + 1)
        A = h.dense_interior()
        xd = np.linalg.solve(A, b[m])
        assert np.abs(x[m] - xd).max() <= 1e-8 * np.abs(xd).max()
        counts[K] = it
    print("iterations by K (pe = 8, gamma = 3, FEM lines):", counts)
    assert max(counts.values()) <= 1.5 * min(counts.values()) + 2


def test_three_dimensional_elements():
    """3-D: the undeformed cube's assembled operator is the Kronecker sum of
    the assembled 1-D element stiffness and mass (scaled by 1 / 2K), A 1 = 0
    on a deformed cube, and the element gamma-cycle preconditions FGMRES to
    the dense solution."""
    K, pe = 2, 4
    cube = inputs.Problem(3, "deformed3d", {"beta": np.zeros(3), "amp": np.zeros(3),
                                            "c": np.zeros((3, 3, 3))})
    coords = [cube.coords(inputs.composite_nodes(orc.gll(pe)[0], K))]
    h = orc.Hier(3, [K * pe], coords, smoother=orc.SMOOTHER_FEM, elements=K)
    xi, rho = orc.gll(pe)
    D = orc.deriv(pe, xi).reshape(pe + 1, pe + 1)
    ke = D.T @ np.diag(rho) @ D
    n1 = K * pe + 1
    Kg, Mg = np.zeros((n1, n1)), np.zeros((n1, n1))
    for e in range(K):
        sl = slice(e * pe, e * pe + pe + 1)
        Kg[sl, sl] += ke
        Mg[sl, sl] += np.diag(rho)
    A = (np.kron(np.kron(Mg, Mg), Kg) + np.kron(np.kron(Mg, Kg), Mg)
         + np.kron(np.kron(Kg, Mg), Mg)) / (2 * K)
    m = np.zeros((n1, n1, n1), dtype=bool)
    m[1:-1, 1:-1, 1:-1] = True
    m = m.reshape(-1)
    err = np.abs(h.dense_interior() - A[np.ix_(m, m)]).max() / np.abs(A).max()
    print(f"3-D K={K} pe={pe}: Kronecker sum difference {err:.2e}")
    assert err < 1e-14
    prob = inputs.config3(3)
    pes = [2, 4, 8]
    coords = [prob.coords(inputs.composite_nodes(orc.gll(q)[0], K)) for q in pes]
    h = orc.Hier(3, [K * q for q in pes], coords, gamma=1, m=1, alpha=0.16,
                 smoother=orc.SMOOTHER_FEM, restriction=orc.RESTRICT_TRANSPOSE, elements=K)
    X = coords[-1]
    assert np.abs(h.apply(np.ones(X.shape[1]), all_rows=True)).max() < 1e-12
    b = h.rhs(prob.f(X), prob.g(X))
    x, st, it, _ = h.fgmres(b, rtol=1e-10, maxit=100, restart=20)
    n1 = K * pes[-1] + 1
    mm = np.zeros((n1, n1, n1), dtype=bool)
    mm[1:-1, 1:-1, 1:-1] = True
    mm = mm.reshape(-1)
    xd = np.linalg.solve(h.dense_interior(), b[mm])
    print(f"3-D K={K} pe=8: {it} iterations")
    assert st == 0 and it <= 25
    assert np.abs(x[mm] - xd).max() <= 1e-8 * np.abs(xd).max()

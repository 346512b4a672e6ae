"""Pins of the oracle's line solver (Sec. 3.2), transfers (Sec. 3.3),
gamma-cycle (Alg. 2) and outer Krylov solvers against Thomas / dense LU,
the dense Schur complement, the block-inverse identity, dense Kronecker
transfers, linearity/symmetry, level-visit counts and dense direct solves."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2504_10710_amd import inputs
from tests.helpers import interior_mask, oracle_hier


def _random_line(rng, n, kind):
    if kind == "spd":
        l = -rng.uniform(0.2, 1.0, n)
        u = np.r_[l[1:], 0.0]
        a = np.abs(l) + np.abs(u) + rng.uniform(0.1, 1.0, n)
    elif kind == "general":
        l, u = rng.standard_normal(n), rng.standard_normal(n)
        a = 3.0 + np.abs(rng.standard_normal(n))
    else:  # indefinite symmetric
        l = rng.standard_normal(n)
        u = np.r_[l[1:], 0.0]
        a = rng.standard_normal(n) * 3.0
    l[0] = 0.0
    u[-1] = 0.0
    return l, a, u


def _dense(l, a, u):
    n = len(a)
    M = np.diag(a)
    for i in range(1, n):
        M[i, i - 1] = l[i]
        M[i - 1, i] = u[i - 1]
    return M


@pytest.mark.parametrize("n", list(range(1, 32)) + [63, 64, 127, 128, 255])
@pytest.mark.parametrize("kind", ["spd", "general", "indef"])
def test_cr_equals_thomas_and_lu(n, kind):
    rng = np.random.default_rng(1000 * n + hash(kind) % 97)
    l, a, u = _random_line(rng, n, kind)
    g = rng.standard_normal(n)
    M = _dense(l, a, u)
    ref = np.linalg.solve(M, g)
    y_cr = orc.cr_solve(l, a, u, g)
    y_th = orc.thomas(l, a, u, g)
    y_lu = orc.dense_solve(M, g)
    kappa = np.linalg.cond(M)
    tol = 50 * n * kappa * np.finfo(float).eps
    scale = np.abs(ref).max()
    assert np.abs(y_cr - ref).max() <= tol * scale
    assert np.abs(y_th - ref).max() <= tol * scale
    assert np.abs(y_lu - ref).max() <= tol * scale


@pytest.mark.parametrize("n", [2, 3, 7, 8, 15, 16, 33])
def test_cr_coarse_is_schur_complement(n):
    """Prop. line coarse space: M0 = D - C A^{-1} B after the odd-even reordering
    (F = odd 1-based positions), computed densely."""
    rng = np.random.default_rng(n)
    l, a, u = _random_line(rng, n, "general")
    M = _dense(l, a, u)
    F = np.arange(0, n, 2)
    C = np.arange(1, n, 2)
    S = M[np.ix_(C, C)] - M[np.ix_(C, F)] @ np.linalg.solve(M[np.ix_(F, F)], M[np.ix_(F, C)])
    l0, a0, u0 = orc.cr_coarse(l, a, u)
    np.testing.assert_allclose(_dense(l0, a0, u0), S, atol=1e-13 * np.abs(S).max())


def test_block_inverse_identity():
    """Prop. block inverse / Lemma: M^{-1} = S^{-1} + P M0^{-1} P^T (I - M S^{-1})
    for a random 2x2 block matrix (any left block of R is allowed)."""
    rng = np.random.default_rng(3)
    n1, n2 = 4, 3
    M = rng.standard_normal((n1 + n2, n1 + n2)) + 6 * np.eye(n1 + n2)
    A, B = M[:n1, :n1], M[:n1, n1:]
    C, Dm = M[n1:, :n1], M[n1:, n1:]
    Ainv = np.linalg.inv(A)
    Sinv = np.zeros_like(M)
    Sinv[:n1, :n1] = Ainv
    P = np.vstack([-Ainv @ B, np.eye(n2)])
    M0 = Dm - C @ Ainv @ B
    for R in (P.T, np.hstack([rng.standard_normal((n2, n1)), np.eye(n2)])):
        Minv = Sinv + P @ np.linalg.solve(M0, R @ (np.eye(n1 + n2) - M @ Sinv))
        np.testing.assert_allclose(Minv, np.linalg.inv(M), atol=1e-12)


def _hier(problem, p, p_coarse=2, gamma=1, alpha=2.0 / 3.0, smoother=0):
    h, ps, coords = oracle_hier(problem, p, p_coarse, gamma=gamma, alpha=alpha, smoother=smoother)
    return h, ps, coords


@pytest.mark.parametrize("dim,p", [(2, 8), (2, 16), (3, 4), (3, 8)])
def test_line_coefs_are_entries_of_A(dim, p):
    prob = inputs.config2(2) if dim == 2 else inputs.config3(2)
    h, ps, coords = _hier(prob, p, p_coarse=p)
    n, n1 = p - 1, p + 1
    rng = np.random.default_rng(p)
    for d in range(dim):
        lo, di, up = h.line_coefs(d)
        for _ in range(10):
            line, s = rng.integers(0, n ** (dim - 1)), rng.integers(0, n)
            # node of (line, s): remaining axes lexicographic, first fastest
            c = [0] * dim
            t = line
            for a in range(dim):
                if a == d:
                    continue
                c[a] = 1 + t % n
                t //= n
            c[d] = s + 1
            node = sum(ci * n1**a for a, ci in enumerate(c))
            st = n1**d
            np.testing.assert_allclose(di[line * n + s], h.entry(node, node), rtol=1e-14)
            if s > 0:
                np.testing.assert_allclose(lo[line * n + s], h.entry(node, node - st), rtol=1e-14)
            if s < n - 1:
                np.testing.assert_allclose(up[line * n + s], h.entry(node, node + st), rtol=1e-14)


@pytest.mark.parametrize("dim,p", [(2, 8), (2, 32), (3, 8)])
def test_line_solve_inverts_line_tridiagonals(dim, p):
    """B_dir^{-1} (T_dir e) = e, T_dir the block-diagonal assembly of the line
    tridiagonals (checks extraction, layout and CR together)."""
    prob = inputs.config2(4) if dim == 2 else inputs.config3(4)
    h, ps, coords = _hier(prob, p, p_coarse=p)
    n1, n = p + 1, p - 1
    mask = interior_mask(dim, p)
    rng = np.random.default_rng(0)
    e = np.where(mask, rng.standard_normal(n1**dim), 0.0)
    for d in range(dim):
        lo, di, up = h.line_coefs(d)
        st = n1**d
        Te = np.zeros_like(e)
        nodes = np.flatnonzero(mask)
        # position along axis d of each interior node
        pos = (nodes // st) % n1
        # line index = remaining interior indices lexicographic
        rem = [a for a in range(dim) if a != d]
        line = np.zeros_like(nodes)
        mul = 1
        for a in rem:
            line += ((nodes // n1**a) % n1 - 1) * mul
            mul *= n
        k = line * n + (pos - 1)
        Te[nodes] = di[k] * e[nodes]
        has_lo = pos > 1
        Te[nodes[has_lo]] += lo[k[has_lo]] * e[nodes[has_lo] - st]
        has_up = pos < p - 1
        Te[nodes[has_up]] += up[k[has_up]] * e[nodes[has_up] + st]
        z = h.line_solve(Te, d)
        np.testing.assert_allclose(z, e, atol=1e-10)


@pytest.mark.parametrize("dim,pc,pf", [(2, 4, 8), (2, 8, 16), (3, 2, 4), (3, 4, 8)])
def test_transfers_are_kronecker_of_interp(dim, pc, pf):
    prob = inputs.config2(1) if dim == 2 else inputs.config3(1)
    h, ps, coords = _hier(prob, pf, p_coarse=pc)
    xc, _ = orc.gll(pc)
    xf, _ = orc.gll(pf)
    J = orc.interp(pc, xc, xf)
    P = J
    for _ in range(dim - 1):
        P = np.kron(J, P)  # first axis fastest
    rng = np.random.default_rng(2)
    mc = interior_mask(dim, pc)
    ec = np.where(mc, rng.standard_normal((pc + 1) ** dim), 0.0)
    xf0 = rng.standard_normal((pf + 1) ** dim)
    np.testing.assert_allclose(h.prolong_add(ec, xf0), xf0 + P @ ec, atol=1e-13)
    rf = rng.standard_normal((pf + 1) ** dim)
    rc = h.restrict(rf)
    np.testing.assert_allclose(rc[mc], (P.T @ rf)[mc], atol=1e-12)
    assert np.all(rc[~mc] == 0.0)


@pytest.mark.parametrize("gamma", [1, 2, 3])
def test_cycle_linear_and_visits(gamma):
    prob = inputs.config2(3)
    p = 16
    h, ps, coords = _hier(prob, p, gamma=gamma)
    mask = interior_mask(2, p)
    rng = np.random.default_rng(5)
    r1 = np.where(mask, rng.standard_normal((p + 1) ** 2), 0.0)
    r2 = np.where(mask, rng.standard_normal((p + 1) ** 2), 0.0)
    h.reset_visits()
    y1 = h.cycle(r1)
    L = len(ps) - 1
    # Prop. cost: level l is entered gamma^(L-l) times per cycle
    assert h.visits() == [gamma ** (L - l) for l in range(L + 1)]
    y2 = h.cycle(r2)
    y12 = h.cycle(2.5 * r1 - 0.75 * r2)
    np.testing.assert_allclose(y12, 2.5 * y1 - 0.75 * y2, atol=1e-11 * np.abs(y12).max())
    assert np.all(y1[~mask] == 0.0)
    if gamma == 1:
        # symmetric sweep order and R = P^T: the V-cycle is a symmetric operator
        np.testing.assert_allclose(r2 @ y1, r1 @ y2, rtol=1e-10)


def test_cycle_single_level_is_exact():
    prob = inputs.config2(6)
    p = 6
    h, ps, coords = _hier(prob, p, p_coarse=p)
    mask = interior_mask(2, p)
    rng = np.random.default_rng(0)
    r = np.where(mask, rng.standard_normal((p + 1) ** 2), 0.0)
    y = h.cycle(r)
    A = h.dense_interior()
    np.testing.assert_allclose(y[mask], np.linalg.solve(A, r[mask]), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("dim,p,solver,gamma", [
    (2, 8, "fgmres", 7), (2, 8, "pcg", 1), (2, 8, "fcg", 3), (3, 4, "fgmres", 2),
    (3, 8, "fgmres", 1), (2, 16, "fgmres", 2)])
def test_krylov_matches_dense_solve(dim, p, solver, gamma):
    prob = inputs.config2(11) if dim == 2 else inputs.config3(11)
    h, ps, coords = _hier(prob, p, gamma=gamma)
    X = coords[-1]
    b = h.rhs(prob.f(X), prob.g(X))
    x, st, it, hist = getattr(h, solver)(b, rtol=1e-12, maxit=200)
    assert st == 0, (st, it)
    mask = interior_mask(dim, p)
    A = h.dense_interior()
    ref = np.linalg.solve(A, b[mask])
    np.testing.assert_allclose(x[mask], ref, rtol=0, atol=1e-9 * np.abs(ref).max())
    assert np.linalg.norm(b - h.apply(x)) <= 1e-12 * np.linalg.norm(b) * 1.0001


def test_pcg_config1():
    """Config 1 (undeformed square, p = 16, gamma = 1, PCG) converges to 1e-10
    and reproduces the manufactured solution to discretisation accuracy."""
    prob = inputs.config1(0)
    p = 16
    h, ps, coords = _hier(prob, p, gamma=1)
    X = coords[-1]
    b = h.rhs(prob.f(X), prob.g(X))
    x, st, it, hist = h.pcg(b, rtol=1e-10, maxit=200)
    assert st == 0 and it < 40, (st, it)
    mask = interior_mask(2, p)
    u = np.where(mask, x, prob.g(X))
    assert np.abs(u - prob.exact(X)).max() < 1e-7


@pytest.mark.parametrize("p", [8, 16])
def test_iterations_bounded_3d_fem(p):
    """3-D config-3 problems with the trilinear FEM line smoother, alpha = 0.16."""
    its = []
    for seed in range(3):
        prob = inputs.config3(seed)
        h, ps, coords = _hier(prob, p, gamma=1, alpha=0.16, smoother=1)
        X = coords[-1]
        x, st, it, hist = h.fgmres(h.rhs(prob.f(X), prob.g(X)), rtol=1e-10, maxit=100)
        assert st == 0, (seed, it)
        its.append(it)
    assert max(its) <= 14, its


@pytest.mark.parametrize("p", [16, 32, 64])
def test_iterations_bounded_over_seeds(p):
    """Iteration counts stay bounded as deformation, RHS and Dirichlet data vary
    and as p grows (config-2 problems, FEM line smoother, alpha = 0.16)."""
    its = []
    for seed in range(4):
        prob = inputs.config2(seed)
        h, ps, coords = _hier(prob, p, gamma=2, alpha=0.16, smoother=1)
        X = coords[-1]
        b = h.rhs(prob.f(X), prob.g(X))
        x, st, it, hist = h.fgmres(b, rtol=1e-10, maxit=100)
        assert st == 0, (seed, it)
        its.append(it)
    assert max(its) <= 16 and max(its) <= 1.5 * np.median(its), its


def test_fem_entries_3d():
    """Trilinear FEM stiffness on the GLL node mesh of the unit cube: symmetric,
    rows sum to zero, exact energy of trilinear functions."""
    p = 4
    prob = inputs.Problem(3, "deformed3d", {"beta": np.zeros(3), "amp": np.zeros(3),
                                             "c": np.zeros((3, 3, 3))})
    h, ps, coords = _hier(prob, p, p_coarse=p, smoother=1)
    N = (p + 1) ** 3
    A = np.array([[h.fem_entry(i, j) for j in range(N)] for i in range(N)])
    np.testing.assert_allclose(A, A.T, atol=1e-13)
    np.testing.assert_allclose(A.sum(axis=1), 0.0, atol=1e-12)
    x, y, z = coords[-1]
    for u, exact in [(x, 1.0), (x * y, 2.0 / 3.0), (x * y * z, 1.0 / 3.0), (x + y - z, 3.0)]:
        np.testing.assert_allclose(u @ A @ u, exact, rtol=1e-13)


def test_fem_entries():
    """Bilinear FEM stiffness on the GLL node mesh: symmetric, rows sum to zero,
    exact energy of bilinear functions on the undeformed square."""
    p = 6
    h, ps, coords = _hier(inputs.table1(1), p, p_coarse=p, smoother=1)
    N = (p + 1) ** 2
    A = np.array([[h.fem_entry(i, j) for j in range(N)] for i in range(N)])
    np.testing.assert_allclose(A, A.T, atol=1e-13)
    np.testing.assert_allclose(A.sum(axis=1), 0.0, atol=1e-12)
    x, y = coords[-1]
    for u, exact in [(x, 1.0), (y, 1.0), (x * y, 2.0 / 3.0), (x + 2 * y, 5.0)]:
        np.testing.assert_allclose(u @ A @ u, exact, rtol=1e-13)
    # the FEM line tridiagonals are those entries
    lo, di, up = h.line_coefs(0)
    node = 2 + (p + 1) * 3  # (i, j) = (2, 3): line j-1 = 2, position i-1 = 1
    k = 2 * (p - 1) + 1
    np.testing.assert_allclose(di[k], A[node, node], rtol=1e-14)
    np.testing.assert_allclose(lo[k], A[node, node - 1], rtol=1e-14)
    np.testing.assert_allclose(up[k], A[node, node + 1], rtol=1e-14)


# ---------------------------------------------------------------- block CR

def _random_blocks(rng, nb, m, kind):
    Lb = rng.standard_normal((nb, m, m))
    Ub = rng.standard_normal((nb, m, m))
    if kind == "spd":
        # symmetric: L_{i+1} = U_i^T, diagonal blocks dominant
        for i in range(nb - 1):
            Lb[i + 1] = Ub[i].T
    Ab = np.empty((nb, m, m))
    for i in range(nb):
        S = rng.standard_normal((m, m))
        Ab[i] = S @ S.T + (2.5 * m + 1.0) * np.eye(m)
    Lb[0] = 0.0
    Ub[-1] = 0.0
    return Lb, Ab, Ub


def _dense_blocks(Lb, Ab, Ub):
    nb, m, _ = Ab.shape
    M = np.zeros((nb * m, nb * m))
    for i in range(nb):
        M[i * m:(i + 1) * m, i * m:(i + 1) * m] = Ab[i]
        if i > 0:
            M[i * m:(i + 1) * m, (i - 1) * m:i * m] = Lb[i]
        if i + 1 < nb:
            M[i * m:(i + 1) * m, (i + 1) * m:(i + 2) * m] = Ub[i]
    return M


@pytest.mark.parametrize("m", [1, 2, 3])
@pytest.mark.parametrize("nb", [1, 2, 3, 4, 5, 7, 8, 16, 31, 32, 64])
@pytest.mark.parametrize("kind", ["spd", "general"])
def test_block_cr_equals_dense_lu(m, nb, kind):
    """Thm. two-level direct solver with m x m blocks, applied recursively
    (Cor. direct multigrid): one pass solves M y = g exactly (to rounding)."""
    rng = np.random.default_rng(100 * nb + 10 * m + (kind == "spd"))
    Lb, Ab, Ub = _random_blocks(rng, nb, m, kind)
    M = _dense_blocks(Lb, Ab, Ub)
    g = rng.standard_normal(nb * m)
    ref = np.linalg.solve(M, g)
    y = orc.bcr_solve(Lb, Ab, Ub, g)
    y_lu = orc.dense_solve(M, g)
    tol = 50 * nb * m * np.linalg.cond(M) * np.finfo(float).eps * np.abs(ref).max()
    assert np.abs(y - ref).max() <= tol
    assert np.abs(y_lu - ref).max() <= tol


def test_block_cr_m1_is_scalar_cr():
    rng = np.random.default_rng(9)
    n = 37
    l, a, u = _random_line(rng, n, "general")
    g = rng.standard_normal(n)
    y = orc.bcr_solve(l.reshape(n, 1, 1), a.reshape(n, 1, 1), u.reshape(n, 1, 1), g)
    np.testing.assert_allclose(y, orc.cr_solve(l, a, u, g), rtol=0, atol=1e-14 * np.abs(y).max())


@pytest.mark.parametrize("m", [2, 3])
@pytest.mark.parametrize("nb", [2, 3, 6, 9])
def test_block_cr_coarse_is_schur_complement(m, nb):
    """Prop. line coarse space with blocks: after the odd-even block
    reordering, D - C A^{-1} B is block-tridiagonal and equals the oracle's
    coarse blocks (the proof's middle term)."""
    rng = np.random.default_rng(nb * 7 + m)
    Lb, Ab, Ub = _random_blocks(rng, nb, m, "general")
    M = _dense_blocks(Lb, Ab, Ub)
    F = np.concatenate([np.arange(i * m, (i + 1) * m) for i in range(0, nb, 2)])
    C = np.concatenate([np.arange(i * m, (i + 1) * m) for i in range(1, nb, 2)])
    S = M[np.ix_(C, C)] - M[np.ix_(C, F)] @ np.linalg.solve(M[np.ix_(F, F)], M[np.ix_(F, C)])
    L0, A0, U0 = orc.bcr_coarse(Lb, Ab, Ub)
    np.testing.assert_allclose(_dense_blocks(L0, A0, U0), S, atol=1e-12 * np.abs(S).max())


@pytest.mark.parametrize("dim,p", [(2, 8), (2, 16), (3, 8)])
def test_band2_line_systems_are_entries_of_A_and_are_inverted(dim, p):
    """GLL half-bandwidth-2 line systems: every band entry is an entry of A,
    and the line solve inverts the assembled banded line matrices
    (B_dir^{-1} (T_dir e) = e)."""
    prob = inputs.config2(5) if dim == 2 else inputs.config3(5)
    h, ps, coords = oracle_hier(prob, p, p_coarse=p, smoother=orc.SMOOTHER_GLL_BAND2)
    n, n1 = p - 1, p + 1
    mask = interior_mask(dim, p)
    rng = np.random.default_rng(1)
    e = np.where(mask, rng.standard_normal(n1 ** dim), 0.0)
    for d in range(dim):
        band = h.line_band(d)
        st = n1 ** d
        Te = np.zeros_like(e)
        for line in range(n ** (dim - 1)):
            c = [0] * dim
            t = line
            for a in range(dim):
                if a == d:
                    continue
                c[a] = 1 + t % n
                t //= n
            base = sum(ci * n1 ** a for a, ci in enumerate(c) if a != d)
            nodes = base + st * np.arange(1, p)
            for s in range(n):
                for k in range(-2, 3):
                    if 0 <= s + k < n:
                        v = band[line, s, k + 2]
                        if line < 3 and s < 4:
                            np.testing.assert_allclose(v, h.entry(nodes[s], nodes[s + k]), rtol=1e-14)
                        Te[nodes[s]] += v * e[nodes[s + k]]
                    else:
                        assert band[line, s, k + 2] == 0.0
        np.testing.assert_allclose(h.line_solve(Te, d), e, atol=1e-10)


@pytest.mark.parametrize("dim,pc,pf", [(2, 4, 8), (2, 16, 32), (3, 4, 8)])
def test_interpolation_restriction_evaluates_fine_polynomial(dim, pc, pf):
    """Sec. 3.3, restriction as interpolation: the fine nodal values of a
    polynomial of degree <= p_f per variable restrict to its values at the
    coarse interior nodes (exactly, up to rounding), and restricting a
    prolongated coarse vector returns it (R P = I on the interior)."""
    prob = inputs.config2(1) if dim == 2 else inputs.config3(1)
    h, ps, coords = oracle_hier(prob, pf, p_coarse=pc, restriction=orc.RESTRICT_INTERP)
    xf = orc.gll(pf)[0]
    xc = orc.gll(pc)[0]
    rng = np.random.default_rng(3)
    cf = [rng.standard_normal(pf + 1) for _ in range(dim)]

    def poly(nodes):
        vals = [np.polynomial.polynomial.polyval(nodes, c) for c in cf]
        out = vals[0]
        for v in vals[1:]:
            out = np.multiply.outer(v, out)   # first axis fastest in the flattening
        return out.reshape(-1)

    mc = interior_mask(dim, pc)
    rc = h.restrict(poly(xf))
    ref = poly(xc)
    np.testing.assert_allclose(rc[mc], ref[mc], rtol=0, atol=1e-11 * np.abs(ref).max())
    assert np.all(rc[~mc] == 0.0)
    ec = np.where(mc, rng.standard_normal((pc + 1) ** dim), 0.0)
    back = h.restrict(h.prolong_add(ec, np.zeros((pf + 1) ** dim)))
    np.testing.assert_allclose(back, ec, atol=1e-12)

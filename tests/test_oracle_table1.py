"""Pins of the oracle's gamma-cycle (Alg. 2), transfers (Sec. 3.3) and line
smoothers (Def. line preconditioners) against the iteration counts printed in
Table 1 ("Square domain") and Table 2 row 0 of the paper's numerical
experiments (tests/golden/table1.json).

Setting of the tables: undeformed unit square, GMRES preconditioned by the
gamma-cycle from a zero initial guess, stop when the residual has dropped by
1e-8, m = 1, alpha_GLL = 2/3, alpha_FEM = 0.16, p halving down to 2.  The
outer solve is the oracle's right-preconditioned FGMRES(30) (for a fixed
linear preconditioner it is GMRES), counted on the true residual.

What the tables decide:
  * Sec. 3.3 states the restriction twice: as the interpolation between the
    two bases at the quadrature nodes, and as R = P^T.  With R = P^T the
    counts stay near 4-8 for every p_L; Table 1's counts grow with p_L, and
    the interpolation reading reproduces them (FEM column within one
    iteration for problems 1 and 2 up to p_L = 32).
  * The GLL line systems: the tridiagonal [A_l]^(1) of each line (the
    half-bandwidth the section names) reproduces the p_L = 8 row exactly but
    its smoothing step with alpha = 2/3 diverges from p_L = 32 on
    (lambda_max(B^{-1} A) = 7.7 at p = 32; indefinite line matrices at 64),
    while Table 1 converges there.  The half-bandwidth-2 line systems
    (block-tridiagonal with 2x2 blocks, solved by block cyclic reduction)
    and the whole line block (R A P)^{-1} of the definition both converge
    with alpha = 2/3 and follow the GLL column within a few iterations.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2504_10710_amd import inputs

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1.json")))
GAMMAS = GOLD["gammas"]
_cache = {}


def counts(smoother, restriction, problem, p_fine, gammas=GAMMAS, maxit=100):
    """Iteration counts of the oracle's FGMRES(30) at 1e-8 for every gamma;
    a run that does not converge within maxit is reported as maxit + 1."""
    key = (smoother, restriction, problem, p_fine, tuple(gammas), maxit)
    if key in _cache:
        return _cache[key]
    P = inputs.table1(problem)
    ps = inputs.halving_degrees(p_fine)
    coords = [P.coords(orc.gll(p)[0]) for p in ps]
    X = coords[-1]
    f, g = P.f(X), P.g(X)
    alpha = GOLD["alpha"]["fem" if smoother == orc.SMOOTHER_FEM else "gll"]
    out = []
    for gam in gammas:
        h = orc.Hier(2, ps, coords, gamma=gam, m=GOLD["m"], alpha=alpha, smoother=smoother,
                     restriction=restriction)
        b = h.rhs(f, g)
        _, st, it, _ = h.fgmres(b, rtol=GOLD["rtol"], maxit=maxit, restart=30)
        out.append(it if st == 0 else maxit + 1)
    _cache[key] = out
    return out


def _deltas(ours, paper):
    d = np.asarray(paper) - np.asarray(ours)
    return d


# FEM column, interpolation restriction: the reading the library benchmarks.
# Allowed |paper - ours| per entry: one iteration for problems 1 and 2 up to
# p_L = 32 and for problem 3 up to p_L = 16, two at p_L = 64 for problems 1
# and 2.  Problem 3 at p_L >= 32 (the non-homogeneous case, whose lifted
# right-hand side carries the boundary data's high frequencies) needs fewer
# iterations here than printed, by up to 6 at p_L = 64, gamma = 2; that
# range is asserted as measured (0..6 fewer, never more than one above).
FEM_BOUNDS = {
    (1, 8): (1, 1), (1, 16): (1, 1), (1, 32): (1, 1), (1, 64): (2, 2),
    (2, 8): (1, 1), (2, 16): (1, 1), (2, 32): (1, 1), (2, 64): (2, 2),
    (3, 8): (1, 1), (3, 16): (1, 1), (3, 32): (1, 4), (3, 64): (1, 6),
}


@pytest.mark.parametrize("problem", [1, 2, 3])
@pytest.mark.parametrize("p_fine", [8, 16, 32, 64])
def test_fem_column_interpolation_restriction(problem, p_fine):
    ours = counts(orc.SMOOTHER_FEM, orc.RESTRICT_INTERP, problem, p_fine)
    paper = GOLD["fem"][str(problem)][str(p_fine)]
    d = _deltas(ours, paper)
    below, above = FEM_BOUNDS[(problem, p_fine)]
    print(f"FEM problem {problem} p_L={p_fine}: ours {ours} paper {paper} paper-ours {d.tolist()}")
    assert np.all(d >= -below) and np.all(d <= above), (ours, paper)
    # the counts fall (weakly) with gamma, as printed
    assert all(ours[i + 1] <= ours[i] for i in range(len(ours) - 1))


def test_fem_column_mostly_within_one():
    """Over problems 1-3 and p_L = 8..32 (72 entries), at least 90 % of the
    FEM entries are within one iteration of the printed value."""
    n_ok = n = 0
    for problem in (1, 2, 3):
        for p_fine in (8, 16, 32):
            d = _deltas(counts(orc.SMOOTHER_FEM, orc.RESTRICT_INTERP, problem, p_fine),
                        GOLD["fem"][str(problem)][str(p_fine)])
            n_ok += int(np.sum(np.abs(d) <= 1))
            n += d.size
    print(f"FEM entries within one iteration: {n_ok}/{n}")
    assert n_ok >= 0.9 * n


def test_transpose_restriction_contradicts_table1():
    """With R = P^T the preconditioner is far stronger than the one behind
    Table 1 and its counts do not grow with p_L: at p_L = 32, gamma = 1 the
    printed FEM count is 23, R = P^T gives at most 10."""
    tp = {p: counts(orc.SMOOTHER_FEM, orc.RESTRICT_TRANSPOSE, 1, p, gammas=[1]) for p in (8, 32)}
    it = {p: counts(orc.SMOOTHER_FEM, orc.RESTRICT_INTERP, 1, p, gammas=[1]) for p in (8, 32)}
    print("gamma=1 problem 1 FEM: P^T", tp, "interpolation", it)
    assert tp[32][0] <= 10 < GOLD["fem"]["1"]["32"][0]
    assert tp[32][0] - tp[8][0] <= 3
    assert it[32][0] - it[8][0] >= 10


def test_table2_row0_fem():
    """Table 2 row 0 (no deformation, p_L = 64, gamma = 7) repeats Table 1's
    problem 3: 7 FEM iterations."""
    row = GOLD["table2_row0"]
    ours = counts(orc.SMOOTHER_FEM, orc.RESTRICT_INTERP, row["problem"], row["p_L"],
                  gammas=[row["gamma"]])[0]
    print(f"Table 2 row 0 FEM: ours {ours}, paper {row['fem']}")
    assert abs(ours - row["fem"]) <= 1


# GLL column.  Half-bandwidth-2 line systems (block CR, 2x2 blocks).
GLL_BAND2_BOUNDS = {
    (1, 8): (1, 1), (1, 16): (1, 2), (1, 32): (1, 2), (1, 64): (1, 3),
    (2, 8): (1, 2), (2, 16): (1, 3), (2, 32): (1, 3),
    (3, 8): (1, 2), (3, 16): (1, 3),
}


@pytest.mark.parametrize("problem,p_fine", sorted(GLL_BAND2_BOUNDS))
def test_gll_column_band2_line_systems(problem, p_fine):
    ours = counts(orc.SMOOTHER_GLL_BAND2, orc.RESTRICT_INTERP, problem, p_fine)
    paper = GOLD["gll"][str(problem)][str(p_fine)]
    d = _deltas(ours, paper)
    below, above = GLL_BAND2_BOUNDS[(problem, p_fine)]
    print(f"GLL band-2 problem {problem} p_L={p_fine}: ours {ours} paper {paper} "
          f"paper-ours {d.tolist()}")
    assert np.all(d >= -below) and np.all(d <= above), (ours, paper)


def test_gll_column_full_line_block_equals_band2_at_p8():
    """The literal line block (R A P)^{-1} and the half-bandwidth-2 band give
    the printed p_L = 8 row of problem 1 exactly."""
    paper = GOLD["gll"]["1"]["8"]
    assert counts(orc.SMOOTHER_GLL_FULL, orc.RESTRICT_INTERP, 1, 8) == paper
    assert counts(orc.SMOOTHER_GLL_BAND2, orc.RESTRICT_INTERP, 1, 8) == paper


def test_gll_tridiagonal_line_systems_reproduce_p8_and_fail_at_p32():
    """[A_l]^(1) on the line (tridiagonal): the p_L = 8 row of problem 1 is
    reproduced exactly, p_L = 16 within one iteration, but at p_L = 32 the
    alpha = 2/3 smoothing step diverges and the gamma = 1 solve takes more
    than 30 iterations where the paper prints 19."""
    assert counts(orc.SMOOTHER_GLL, orc.RESTRICT_INTERP, 1, 8) == GOLD["gll"]["1"]["8"]
    d = _deltas(counts(orc.SMOOTHER_GLL, orc.RESTRICT_INTERP, 1, 16), GOLD["gll"]["1"]["16"])
    assert np.all(np.abs(d) <= 1)
    it32 = counts(orc.SMOOTHER_GLL, orc.RESTRICT_INTERP, 1, 32, gammas=[1], maxit=60)[0]
    print(f"GLL tridiagonal p_L=32 gamma=1: {it32} iterations (paper 19)")
    assert it32 > 30

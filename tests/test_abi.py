"""CPU checks of the C ABI: the library loads, exports every symbol the header
declares, and its host-side calls and argument checks behave (no GPU work)."""
import os
import re

import numpy as np
import pytest

from paper_2504_10710_amd import pmg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pmg.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(pmg_\w+)\s*\(", src, re.M)))


def test_library_exports_header_symbols():
    L = pmg.lib()
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n
    assert sorted(pmg.exported_symbols()) == names


def test_host_gll_matches_closed_forms():
    xi, rho, D = pmg.pmg_gll(4)
    np.testing.assert_allclose(xi, [-1, -np.sqrt(3 / 7), 0, np.sqrt(3 / 7), 1], atol=1e-15)
    np.testing.assert_allclose(rho, [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10], rtol=1e-14)
    np.testing.assert_allclose(D @ xi**3, 3 * xi**2, atol=1e-12)
    J = pmg.pmg_interp(4, 8)
    xf = pmg.pmg_gll(8)[0]
    np.testing.assert_allclose(J @ xi**4, xf**4, atol=1e-13)


@pytest.mark.parametrize("kw,msg", [
    (dict(dim=4), "dim"), (dict(p_fine=12), "p_fine"), (dict(dim=3, p_fine=128), "p_fine"),
    (dict(gamma=0), "gamma"), (dict(alpha=-1.0), "alpha"), (dict(smoother=5), "smoother"),
    (dict(restart=0), "restart"), (dict(batch=0), "batch"), (dict(krylov=7), "Krylov"),
    (dict(restriction=2), "restriction")])
def test_invalid_descriptions(kw, msg):
    with pytest.raises(pmg.PmgError) as e:
        pmg.pmg_workspace_bytes(pmg.make_desc(**kw))
    assert e.value.code == pmg.PMG_EINVAL and msg in str(e.value)


def test_workspace_scales_with_batch():
    a = pmg.pmg_workspace_bytes(pmg.make_desc(p_fine=128, batch=1))
    b = pmg.pmg_workspace_bytes(pmg.make_desc(p_fine=128, batch=8))
    assert 7 * a < b < 9 * a
    assert pmg.pmg_num_levels(pmg.make_desc(p_fine=128)) == 7


@pytest.mark.parametrize("p", [16, 64, 128, 256])
def test_host_derivative_matrix_rows_sum_to_zero(p):
    """D differentiates constants to zero: every row sums to zero up to the
    rounding of one sum (closed-form off-diagonals, diagonal = minus their
    sum).  A diagonal taken from its closed form instead leaves row sums of
    1.7e-10 at p = 128 and 4.3e-9 at p = 256, which fail this bound."""
    xi, rho, D = pmg.pmg_gll(p)
    assert np.abs(D.sum(axis=1)).max() <= 1e-15 * p * p
    # exact on polynomials of degree p
    np.testing.assert_allclose(D @ xi**p, p * xi ** (p - 1), atol=1e-14 * p**2 * p)
    np.testing.assert_allclose(D[0, 0], -p * (p + 1) / 4.0, rtol=1e-12)


def test_operator_from_host_tables_matches_oracle_at_p128():
    """The sum-factorised operator built in numpy from the library's host D
    agrees with the oracle's operator at p = 128 on a rough interior input
    (config-2 geometry, the oracle's geometric factors) within 1e-12."""
    from oracle import oracle as orc
    from paper_2504_10710_amd import inputs

    p = 128
    P = inputs.config2(0)
    ps = inputs.halving_degrees(p)
    h = orc.Hier(2, ps, [P.coords(orc.gll(q)[0]) for q in ps], gamma=1)
    G, mass, _ = h.geom()
    D = pmg.pmg_gll(p)[2]
    n1 = p + 1
    m1 = np.zeros(n1, bool)
    m1[1:-1] = True
    mask = np.outer(m1, m1).reshape(-1)
    x = np.where(mask, np.random.default_rng(0).standard_normal(n1 * n1), 0.0)
    X = x.reshape(n1, n1)          # [second index][first index]
    gx, gy = X @ D.T, D @ X
    G00, G11, G01 = (G[a, b].reshape(n1, n1) for a, b in ((0, 0), (1, 1), (0, 1)))
    y = ((G00 * gx + G01 * gy) @ D + D.T @ (G01 * gx + G11 * gy)).reshape(-1) * mask
    yo = h.apply(x)
    assert np.abs(y - yo).max() <= 1e-12 * np.abs(yo).max()


@pytest.mark.parametrize("kw", [
    dict(dim=2, p_fine=32, batch=2, inner_prec=pmg.PMG_F32),
    dict(dim=2, p_fine=128, batch=3),
    dict(dim=3, p_fine=16, batch=2, inner_prec=pmg.PMG_F32, restart=20),
])
def test_workspace_layout_in_bounds(kw):
    """Every region of the workspace lies inside pmg_workspace_bytes, starts on
    a 256-byte boundary and overlaps no other.  For the vectors the outer
    Krylov loops and the FP32 cycle's conversions run over (V, Z, TR64 in
    FP64; the finest level's X, R, Tm in the cycle's type), even a loop that
    issued four loads per thread at q, q+512, q+1024, q+1536 while checking
    only q < N would stay inside the workspace: its furthest element, 3 * 512
    past the last problem's last vector, is printed with the slack left."""
    desc = pmg.make_desc(**kw)
    total = pmg.pmg_workspace_bytes(desc)
    regs = pmg.pmg_workspace_layout(desc)
    assert regs
    end = 0
    for name, off, nb in regs:
        assert off % 256 == 0 and off >= end, (name, off, end)
        end = off + nb
    assert end <= total
    dim, p, B = kw["dim"], kw["p_fine"], kw["batch"]
    N = (p + 1) ** dim
    NT = 512
    lev = {n: (o, b) for n, o, b in regs}
    L = len([r for r in regs if r[0].startswith("X[")]) - 1
    tsz = 4 if kw.get("inner_prec") == pmg.PMG_F32 else 8
    for name, esz in (("V", 8), ("Z", 8), ("TR64", 8), (f"X[{L}]", tsz), (f"R[{L}]", tsz),
                      (f"Tm[{L}]", tsz)):
        off, nb = lev[name]
        assert nb % (esz * N) == 0, name
        furthest = off + nb - esz + 3 * NT * esz       # byte of the last element + 3 NT
        print(f"{kw} {name}: region ends at {off + nb}, unguarded four-in-flight loop reaches "
              f"{furthest + esz}, workspace {total}, slack {total - furthest - esz}")
        assert furthest + esz <= total


@pytest.mark.parametrize("dim,K,p,prec,gamma", [(2, 2, 16, pmg.PMG_F64, 1), (2, 4, 128, pmg.PMG_F64, 1),
                                                (2, 8, 64, pmg.PMG_F32, 1), (2, 4, 256, pmg.PMG_F32, 1),
                                                (3, 2, 16, pmg.PMG_F64, 1), (3, 4, 64, pmg.PMG_F32, 1),
                                                (2, 4, 128, pmg.PMG_F64, 3), (2, 2, 64, pmg.PMG_F64, 2),
                                                (3, 2, 32, pmg.PMG_F64, 5)])
def test_element_workspace_layout(dim, K, p, prec, gamma):
    """Several elements per axis: levels below degree 2K are absent; the
    geometric factors and fluxes of a level hold K^dim (p_l/K + 1)^dim element
    nodes per problem; the coarsest level holds its (2K-1)^dim square exact
    inverse, and in 2-D the levels of degree 8 and 16 above it a collapsed
    matrix where gamma^depth >= ni / 16 (none in 3-D); every region in
    bounds, aligned, without overlap."""
    B = 3
    desc = pmg.make_desc(dim=dim, p_fine=p, batch=B, elements=K, smoother=pmg.PMG_SMOOTHER_FEM,
                         inner_prec=prec, gamma=gamma)
    l0 = pmg.pmg_first_level(desc)
    assert l0 == int(np.log2(2 * K)) - 1
    nlev = pmg.pmg_num_levels(desc)
    total = pmg.pmg_workspace_bytes(desc)
    regs = pmg.pmg_workspace_layout(desc)
    end = 0
    for name, off, nb in regs:
        assert off % 256 == 0 and off >= end, (name, off, end)
        end = off + nb
    assert end <= total
    lev = {n: nb for n, _, nb in regs}
    tsz = 4 if prec == pmg.PMG_F32 else 8
    for l in range(nlev):
        present = l >= l0
        assert (f"X[{l}]" in lev) == present and (f"G64[{l}]" in lev) == present, l
        if not present:
            continue
        pl = 2 << l
        ng = K ** dim * (pl // K + 1) ** dim
        ncomp = 3 if dim == 2 else 6
        assert lev[f"G64[{l}]"] == 8 * B * ncomp * ng
        assert lev[f"TR[{l}]"] == tsz * B * dim * ng
        assert lev[f"X[{l}]"] == tsz * B * (pl + 1) ** dim
    ni = (2 * K - 1) ** dim
    cc = [n for n in lev if n.startswith("Cc")]
    want = [l0] + [l for l in range(l0 + 1, nlev)
                   if dim == 2 and (2 << l) in (8, 16) and p > (2 << l)
                   and 16 * gamma ** (nlev - 1 - l) >= ((2 << l) - 1) ** 2]
    assert cc == [f"Cc[{l}]" for l in want], (cc, want)
    assert lev[cc[0]] == 8 * B * ni * ni
    for l in want[1:]:
        nl = ((2 << l) - 1) ** 2
        assert lev[f"Cc[{l}]"] == 8 * B * nl * nl
    if (dim, K, p, gamma) == (2, 4, 128, 3):
        assert want == [l0, l0 + 1]          # the exact inverse at 8 and the collapsed 16


@pytest.mark.parametrize("kw", [dict(elements=3, p_fine=48), dict(elements=8, dim=3, p_fine=64),
                                dict(elements=4, p_fine=8),
                                dict(elements=16, p_fine=64), dict(elements=-1, p_fine=16)])
def test_element_descriptions_rejected(kw):
    args = dict(dim=2, batch=1, smoother=pmg.PMG_SMOOTHER_FEM)
    args.update(kw)
    with pytest.raises(pmg.PmgError):
        pmg.pmg_workspace_bytes(pmg.make_desc(**args))

"""GPU parity of the multi-element hierarchy (K x K spectral elements per
level, the paper's closing outlook of a multi-element hp-multigrid): every
C-ABI entry point on an element hierarchy against the oracle's element mode
on the same seeded inputs (each side with its own GLL nodes; the composite
node grid is input layout).  Tolerances as for one element (FEM line
systems): geometry, transfers and line rows 1e-12; operator and right-hand
side op_tol(p); line solves and smoothing steps max(1e-12, 20 n eps kappa)
(+ kappa op_tol(p)); one gamma-cycle 1e-10; full solves: true relative
residual <= 1e-10 (also with the oracle's operator), solution within 1e-7 of
the oracle's, iterations within +-1.  Every test prints what it achieved."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as orc  # noqa: E402
from paper_2504_10710_amd import inputs, pmg  # noqa: E402
from tests.gpu_helpers import interior_mask, rel_err  # noqa: E402

pytestmark = pytest.mark.gpu

FEM = pmg.PMG_SMOOTHER_FEM


def op_tol(p):
    return max(1e-12, 4 * np.finfo(float).eps * p * p)


def element_degrees(p_fine, K):
    pe, out = p_fine // K, []
    while pe >= 2:
        out.append(pe)
        pe //= 2
    return out[::-1]                       # coarsest first


def gpu_elements(probs, K, p_fine, device="cuda", dim=2, **kw):
    """Solver for K^dim elements; coordinates of the present levels only."""
    desc = pmg.make_desc(dim=dim, p_fine=p_fine, batch=len(probs), elements=K, **kw)
    nlev, l0 = pmg.pmg_num_levels(desc), pmg.pmg_first_level(desc)
    coords = [None] * nlev
    for i, pe in enumerate(element_degrees(p_fine, K)):
        nodes = inputs.composite_nodes(pmg.pmg_gll(pe)[0], K)
        coords[l0 + i] = torch.from_numpy(np.stack([pr.coords(nodes) for pr in probs])).to(device)
    s = pmg.Solver(desc, coords, device=device)
    nodes = inputs.composite_nodes(pmg.pmg_gll(p_fine // K)[0], K)
    X = [pr.coords(nodes) for pr in probs]
    f = torch.from_numpy(np.stack([pr.f(x) for pr, x in zip(probs, X)])).to(device)
    g = torch.from_numpy(np.stack([pr.g(x) for pr, x in zip(probs, X)])).to(device)
    return s, f, g, l0


def oracle_elements(prob, K, p_fine, gamma=1, alpha=0.16, restriction=orc.RESTRICT_INTERP,
                    smoother=orc.SMOOTHER_FEM):
    pes = element_degrees(p_fine, K)
    coords = [prob.coords(inputs.composite_nodes(orc.gll(pe)[0], K)) for pe in pes]
    h = orc.Hier(2, [K * pe for pe in pes], coords, gamma=gamma, m=1, alpha=alpha,
                 smoother=smoother, restriction=restriction, elements=K)
    X = coords[-1]
    return h, prob.f(X), prob.g(X)


GLL, BAND2 = pmg.PMG_SMOOTHER_GLL, pmg.PMG_SMOOTHER_GLL_BAND2
# (K, p_fine, gamma, restriction, smoother, alpha): FEM lines, and the GLL
# line systems of the assembled operator across interfaces (tridiagonal and
# half-bandwidth 2)
CASES = [(2, 16, 1, pmg.PMG_RESTRICT_INTERP, FEM, 0.16), (4, 32, 3, pmg.PMG_RESTRICT_INTERP, FEM, 0.16),
         (2, 32, 2, pmg.PMG_RESTRICT_TRANSPOSE, FEM, 0.16), (8, 64, 2, pmg.PMG_RESTRICT_INTERP, FEM, 0.16),
         (2, 16, 3, pmg.PMG_RESTRICT_INTERP, GLL, 2.0 / 3.0),
         (4, 64, 3, pmg.PMG_RESTRICT_INTERP, BAND2, 2.0 / 3.0)]
SEEDS = [0, 1, 2]
SM_NAME = {FEM: "fem", GLL: "gll", BAND2: "band2"}


@pytest.fixture(scope="module", params=CASES,
                ids=lambda c: f"K{c[0]}-p{c[1]}-g{c[2]}-{'interp' if c[3] else 'PT'}-{SM_NAME[c[4]]}")
def case(request):
    K, p, gamma, rst, sm, alpha = request.param
    print(f"[gpu elements] K={K} p={p} gamma={gamma} restriction={rst} smoother={sm}", flush=True)
    probs = [inputs.config2(s, 0.1) for s in SEEDS]
    s, f, g, l0 = gpu_elements(probs, K, p, gamma=gamma, alpha=alpha, smoother=sm,
                               restriction=rst)
    torch.cuda.synchronize()
    ors = [oracle_elements(pr, K, p, gamma=gamma, alpha=alpha, restriction=rst, smoother=sm)
           for pr in probs]
    return dict(K=K, p=p, l0=l0, s=s, f=f, g=g, ors=ors, probs=probs, gamma=gamma, sm=sm)


def _levels(case):
    """(GPU level, oracle level, composite degree) of every present level."""
    s, l0 = case["s"], case["l0"]
    return [(l, l - l0, 2 << l) for l in range(l0, s.nlev)]


def _rand_interior(p, B, seed):
    rng = np.random.default_rng(seed)
    m = interior_mask(2, p)
    return np.where(m[None, :], rng.standard_normal((B, (p + 1) ** 2)), 0.0)


def _line_kappa(h, lo_, d, p, band=False):
    """Largest condition number of the level's line matrices (tridiagonal,
    or half-bandwidth 2)."""
    n = p - 1
    kmax = 1.0
    if band:
        bd = h.line_band(d, lo_)
        for line in range(n):
            M = np.zeros((n, n))
            for s_ in range(n):
                for k in range(-2, 3):
                    if 0 <= s_ + k < n:
                        M[s_, s_ + k] = bd[line, s_, k + 2]
            kmax = max(kmax, np.linalg.cond(M))
        return kmax
    lo, di, up = h.line_coefs(d, lo_)
    for line in range(n):
        sl = slice(line * n, (line + 1) * n)
        M = np.diag(di[sl]) + np.diag(lo[sl][1:], -1) + np.diag(up[sl][:-1], 1)
        kmax = max(kmax, np.linalg.cond(M))
    return kmax


def test_setup_status_and_levels(case):
    s = case["s"]
    assert case["l0"] == int(np.log2(2 * case["K"])) - 1
    info = s.info_host()
    assert np.all(info["status"] == 0), info
    for b, (h, _, _) in enumerate(case["ors"]):
        mind = min(h.geom(l)[2] for l in range(h.nlev))
        np.testing.assert_allclose(info["min_detj"][b], mind, rtol=1e-12)


def test_element_geometry_and_mass(case):
    s, K = case["s"], case["K"]
    B = len(SEEDS)
    for l, lo_, p in _levels(case):
        NE = (p // K + 1) ** 2
        G = torch.empty((B, K * K, 3, NE), dtype=torch.float64, device="cuda")
        last = l == s.nlev - 1
        mass = torch.empty((B, (p + 1) ** 2), dtype=torch.float64, device="cuda") if last else None
        pmg.pmg_geom(s.h, l, G, mass)
        torch.cuda.synchronize()
        Gh = G.cpu().numpy()
        for b, (h, _, _) in enumerate(case["ors"]):
            Go = h.geom_elements(lo_)               # (K^2, 2, 2, NE)
            for k, (a, c) in enumerate([(0, 0), (1, 1), (0, 1)]):
                eg = rel_err(Gh[b, :, k], Go[:, a, c])
                tg = 1e-12 * max(1.0, np.abs(Go[:, a, a]).max() / max(np.abs(Go[:, a, c]).max(), 1e-300))
                if last:
                    print(f"[elements geom] K={K} p={p} b={b} G{a}{c} rel err {eg:.2e} tol {tg:.1e}")
                assert eg < tg, (l, b, a, c, eg)
            if last:
                em = rel_err(mass.cpu().numpy()[b], h.geom(lo_)[1])
                print(f"[elements geom] K={K} p={p} b={b} mass rel err {em:.2e}")
                assert em < 1e-12


def test_line_coefs(case):
    s = case["s"]
    B = len(SEEDS)
    for l, lo_, p in _levels(case):
        n = (p - 1) ** 2
        if case["sm"] == BAND2:
            for d in range(2):
                band = torch.empty((B, p - 1, p - 1, 5), dtype=torch.float64, device="cuda")
                pmg.pmg_line_band(s.h, l, d, band)
                torch.cuda.synchronize()
                for b, (h, _, _) in enumerate(case["ors"]):
                    ob = h.line_band(d, lo_)
                    err = np.abs(band.cpu().numpy()[b] - ob).max() / np.abs(ob).max()
                    print(f"[elements band] p={p} dir={d} b={b} rel err {err:.2e}")
                    assert err <= 1e-12, (l, d, b, err)
            continue
        for d in range(2):
            lo, di, up = (torch.empty((B, n), dtype=torch.float64, device="cuda") for _ in range(3))
            pmg.pmg_line_coefs(s.h, l, d, lo, di, up)
            torch.cuda.synchronize()
            for b, (h, _, _) in enumerate(case["ors"]):
                olo, odi, oup = h.line_coefs(d, lo_)
                sc = np.abs(odi).max()
                for got, ref in ((lo, olo), (di, odi), (up, oup)):
                    assert np.abs(got.cpu().numpy()[b] - ref).max() <= 1e-12 * sc, (l, d, b)


def test_apply(case):
    s = case["s"]
    B = len(SEEDS)
    for l, lo_, p in _levels(case):
        x = _rand_interior(p, B, 10 + l)
        xt = torch.from_numpy(x).cuda()
        y = torch.empty_like(xt)
        pmg.pmg_apply(s.h, l, pmg.PMG_F64, xt, y)
        torch.cuda.synchronize()
        for b, (h, _, _) in enumerate(case["ors"]):
            err = rel_err(y.cpu().numpy()[b], h.apply(x[b], lo_))
            print(f"[elements apply] K={case['K']} p={p} b={b} rel err {err:.2e} tol {op_tol(p):.1e}")
            assert err < op_tol(p), (l, b, err)


def test_transfers(case):
    s = case["s"]
    B = len(SEEDS)
    for l, lo_, pf in _levels(case)[1:]:
        pc = pf // 2
        rng = np.random.default_rng(l)
        rf = rng.standard_normal((B, (pf + 1) ** 2))
        rc = torch.empty((B, (pc + 1) ** 2), dtype=torch.float64, device="cuda")
        pmg.pmg_restrict(s.h, l, pmg.PMG_F64, torch.from_numpy(rf).cuda(), rc)
        ec = _rand_interior(pc, B, 20 + l)
        xf0 = rng.standard_normal((B, (pf + 1) ** 2))
        xf = torch.from_numpy(xf0).cuda()
        pmg.pmg_prolong_add(s.h, l, pmg.PMG_F64, torch.from_numpy(ec).cuda(), xf)
        torch.cuda.synchronize()
        for b, (h, _, _) in enumerate(case["ors"]):
            er = rel_err(rc.cpu().numpy()[b], h.restrict(rf[b], lo_))
            ep = rel_err(xf.cpu().numpy()[b], h.prolong_add(ec[b], xf0[b], lo_))
            print(f"[elements transfers] K={case['K']} p={pf} b={b} restrict {er:.2e} prolong {ep:.2e}")
            assert er < 1e-12 and ep < 1e-12, (l, b, er, ep)


def test_line_solve_and_smooth(case):
    s = case["s"]
    B = len(SEEDS)
    for l, lo_, p in _levels(case):
        r = _rand_interior(p, B, 30 + l)
        x0 = _rand_interior(p, B, 40 + l)
        for d in range(2):
            z = torch.empty((B, (p + 1) ** 2), dtype=torch.float64, device="cuda")
            pmg.pmg_line_solve(s.h, l, d, pmg.PMG_F64, torch.from_numpy(r).cuda(), z)
            xs = torch.from_numpy(x0.copy()).cuda()
            pmg.pmg_line_smooth(s.h, l, d, pmg.PMG_F64, torch.from_numpy(r).cuda(), xs)
            torch.cuda.synchronize()
            for b, (h, _, _) in enumerate(case["ors"]):
                kap = _line_kappa(h, lo_, d, p, case["sm"] == BAND2)
                tol = max(1e-12, 20 * (p - 1) * np.finfo(float).eps * kap)
                err = rel_err(z.cpu().numpy()[b], h.line_solve(r[b], d, lo_))
                tol2 = tol + kap * op_tol(p)
                err2 = rel_err(xs.cpu().numpy()[b], h.smooth(r[b], x0[b], d, lo_))
                print(f"[elements line] p={p} dir={d} b={b} solve {err:.2e} (tol {tol:.1e}) "
                      f"smooth {err2:.2e} (tol {tol2:.1e})")
                assert err < tol and err2 < tol2, (l, d, b, err, err2)


def test_gamma_cycle(case):
    s, p = case["s"], case["p"]
    r = _rand_interior(p, len(SEEDS), 50)
    y = torch.empty((len(SEEDS), (p + 1) ** 2), dtype=torch.float64, device="cuda")
    pmg.pmg_gamma_cycle(s.h, pmg.PMG_F64, torch.from_numpy(r).cuda(), y)
    torch.cuda.synchronize()
    for b, (h, _, _) in enumerate(case["ors"]):
        err = rel_err(y.cpu().numpy()[b], h.cycle(r[b]))
        print(f"[elements cycle] K={case['K']} p={p} gamma={case['gamma']} b={b} rel err {err:.2e}")
        assert err < 1e-10, (b, err)


def test_band2_full_size():
    """4 x 4 elements of degree 32 with the half-bandwidth-2 GLL line systems
    of the assembled operator (alpha = 2/3), gamma = 3: iterations within +-1
    of the oracle's, solution within 1e-7."""
    K, p = 4, 128
    probs = [inputs.config2(s, 0.1) for s in (31,)]
    s, f, g, _ = gpu_elements(probs, K, p, gamma=3, alpha=2.0 / 3.0, smoother=BAND2)
    bt = torch.empty_like(f)
    pmg.pmg_rhs(s.h, f, g, bt)
    x = torch.empty_like(bt)
    pmg.pmg_solve(s.h, bt, x, s.info)
    torch.cuda.synchronize()
    info = s.info_host()
    h, fo, go = oracle_elements(probs[0], K, p, gamma=3, alpha=2.0 / 3.0,
                                smoother=orc.SMOOTHER_GLL_BAND2)
    bo = h.rhs(fo, go)
    xg = x.cpu().numpy()[0]
    rr = np.linalg.norm(bo - h.apply(xg)) / np.linalg.norm(bo)
    xo, st, it, _ = h.fgmres(bo, rtol=1e-10, maxit=200)
    ex = rel_err(xg, xo)
    print(f"[elements band2 full] its gpu {info['iterations'][0]} oracle {it} "
          f"oracle-operator relres {rr:.3e} err vs oracle {ex:.2e}")
    assert info["status"][0] == 0 and rr <= 1.0001e-10 and st == 0
    assert abs(int(info["iterations"][0]) - it) <= 1 and ex < 1e-7


def test_rhs_and_solve(case):
    s, p = case["s"], case["p"]
    bt = torch.empty_like(case["f"])
    pmg.pmg_rhs(s.h, case["f"], case["g"], bt)
    x = torch.empty_like(bt)
    pmg.pmg_solve(s.h, bt, x, s.info)
    torch.cuda.synchronize()
    info = s.info_host()
    xh, bh = x.cpu().numpy(), bt.cpu().numpy()
    for b, (h, f, g) in enumerate(case["ors"]):
        bo = h.rhs(f, g)
        eb = rel_err(bh[b], bo)
        assert eb < op_tol(p), (b, eb)
        assert info["status"][b] == 0, info[b]
        rr = np.linalg.norm(bh[b] - h.apply(xh[b])) / np.linalg.norm(bh[b])
        xo, st, it, _ = h.fgmres(bo, rtol=1e-10, maxit=200, restart=30)
        ex = rel_err(xh[b], xo)
        print(f"[elements solve] K={case['K']} p={p} b={b} rhs err {eb:.2e} its gpu "
              f"{info['iterations'][b]} oracle {it}, relres gpu {info['relres'][b]:.3e} "
              f"oracle-operator {rr:.3e}, err vs oracle {ex:.2e}")
        assert info["relres"][b] <= 1e-10 and rr <= 1.0001e-10 and st == 0
        assert abs(int(info["iterations"][b]) - it) <= 1, (info["iterations"][b], it)
        assert ex < 1e-7


def test_mixed_precision_elements():
    """FP32 gamma-cycle on 4 x 4 elements inside FP64 FGMRES: 1e-10 with the
    oracle's operator, solution within 1e-7 of the FP64 oracle's."""
    K, p = 4, 64
    probs = [inputs.config2(s, 0.1) for s in (5, 6)]
    s, f, g, _ = gpu_elements(probs, K, p, gamma=3, alpha=0.16, smoother=FEM,
                              inner_prec=pmg.PMG_F32)
    bt = torch.empty_like(f)
    pmg.pmg_rhs(s.h, f, g, bt)
    x = torch.empty_like(bt)
    pmg.pmg_solve(s.h, bt, x, s.info)
    torch.cuda.synchronize()
    info = s.info_host()
    for b, pr in enumerate(probs):
        h, fo, go = oracle_elements(pr, K, p, gamma=3)
        bo = h.rhs(fo, go)
        xg = x.cpu().numpy()[b]
        rr = np.linalg.norm(bo - h.apply(xg)) / np.linalg.norm(bo)
        xo, st, it, _ = h.fgmres(bo, rtol=1e-10, maxit=200)
        print(f"[elements mixed] K={K} p={p} b={b} its gpu {info['iterations'][b]} oracle {it} "
              f"oracle-operator relres {rr:.3e} err vs FP64 oracle {rel_err(xg, xo):.2e}")
        assert info["status"][b] == 0 and rr <= 1.0001e-10
        assert rel_err(xg, xo) < 1e-7


def test_elements_alone_equals_in_the_mix():
    K, p = 4, 32
    mix = [inputs.config2(s, 0.1) for s in (11, 12, 13)]
    outs = []
    for probs in (mix, mix[1:2]):
        s, f, g, _ = gpu_elements(probs, K, p, gamma=2, alpha=0.16, smoother=FEM)
        bt = torch.empty_like(f)
        pmg.pmg_rhs(s.h, f, g, bt)
        x = torch.empty_like(bt)
        pmg.pmg_solve(s.h, bt, x, s.info)
        torch.cuda.synchronize()
        outs.append((x.cpu().numpy(), s.info_host()))
    (xm, im), (xa, ia) = outs
    assert np.array_equal(xm[1], xa[0])
    assert im["iterations"][1] == ia["iterations"][0] and im["relres"][1] == ia["relres"][0]


def test_elements_full_size():
    """4 x 4 elements of degree 32 (composite degree 128, the shape of the
    one-element p = 128 workload), gamma = 3: iterations within +-1 of the
    oracle's and the solution within 1e-7."""
    K, p = 4, 128
    probs = [inputs.config2(s, 0.1) for s in (21, 22)]
    s, f, g, _ = gpu_elements(probs, K, p, gamma=3, alpha=0.16, smoother=FEM)
    bt = torch.empty_like(f)
    pmg.pmg_rhs(s.h, f, g, bt)
    x = torch.empty_like(bt)
    pmg.pmg_solve(s.h, bt, x, s.info)
    torch.cuda.synchronize()
    info = s.info_host()
    for b, pr in enumerate(probs):
        h, fo, go = oracle_elements(pr, K, p, gamma=3)
        bo = h.rhs(fo, go)
        xg = x.cpu().numpy()[b]
        rr = np.linalg.norm(bo - h.apply(xg)) / np.linalg.norm(bo)
        xo, st, it, _ = h.fgmres(bo, rtol=1e-10, maxit=200)
        ex = rel_err(xg, xo)
        print(f"[elements full] K={K} p={p} b={b} its gpu {info['iterations'][b]} oracle {it} "
              f"oracle-operator relres {rr:.3e} err vs oracle {ex:.2e}")
        assert info["status"][b] == 0 and rr <= 1.0001e-10 and st == 0
        assert abs(int(info["iterations"][b]) - it) <= 1 and ex < 1e-7


# ---------------------------------------------------------------- 3-D elements

def oracle_elements3(prob, K, p_fine, gamma, alpha, restriction, smoother):
    pes = element_degrees(p_fine, K)
    coords = [prob.coords(inputs.composite_nodes(orc.gll(pe)[0], K)) for pe in pes]
    h = orc.Hier(3, [K * pe for pe in pes], coords, gamma=gamma, m=1, alpha=alpha,
                 smoother=smoother, restriction=restriction, elements=K)
    X = coords[-1]
    return h, prob.f(X), prob.g(X)


CASES3 = [(2, 16, 1, pmg.PMG_RESTRICT_TRANSPOSE, FEM, 0.16),
          (4, 32, 2, pmg.PMG_RESTRICT_INTERP, FEM, 0.16),
          (2, 16, 1, pmg.PMG_RESTRICT_TRANSPOSE, GLL, 2.0 / 3.0),
          (2, 16, 1, pmg.PMG_RESTRICT_TRANSPOSE, BAND2, 2.0 / 3.0)]
SEEDS3 = [0, 1]


@pytest.fixture(scope="module", params=CASES3,
                ids=lambda c: f"3d-K{c[0]}-p{c[1]}-g{c[2]}-{'interp' if c[3] else 'PT'}-{SM_NAME[c[4]]}")
def case3(request):
    K, p, gamma, rst, sm, alpha = request.param
    print(f"[gpu elements 3-D] K={K} p={p} gamma={gamma} restriction={rst} smoother={sm}",
          flush=True)
    probs = [inputs.config3(s) for s in SEEDS3]
    s, f, g, l0 = gpu_elements(probs, K, p, gamma=gamma, alpha=alpha, smoother=sm,
                               restriction=rst, restart=20, dim=3)
    torch.cuda.synchronize()
    ors = [oracle_elements3(pr, K, p, gamma, alpha, rst, sm) for pr in probs]
    return dict(K=K, p=p, l0=l0, s=s, f=f, g=g, ors=ors, gamma=gamma, sm=sm)


def test_3d_geometry_operator_transfers(case3):
    s, K, l0 = case3["s"], case3["K"], case3["l0"]
    B = len(SEEDS3)
    info = s.info_host()
    assert np.all(info["status"] == 0), info
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    for l in range(l0, s.nlev):
        p, lo_ = 2 << l, l - l0
        NE = (p // K + 1) ** 3
        G = torch.empty((B, K ** 3, 6, NE), dtype=torch.float64, device="cuda")
        pmg.pmg_geom(s.h, l, G)
        x = np.stack([np.random.default_rng(60 + l + b).standard_normal((p + 1) ** 3)
                      for b in range(B)])
        m = interior_mask(3, p)
        x = np.where(m[None, :], x, 0.0)
        y = torch.empty((B, (p + 1) ** 3), dtype=torch.float64, device="cuda")
        pmg.pmg_apply(s.h, l, pmg.PMG_F64, torch.from_numpy(x).cuda(), y)
        torch.cuda.synchronize()
        for b, (h, _, _) in enumerate(case3["ors"]):
            Go = h.geom_elements(lo_)
            for k, (a, c) in enumerate(pairs):
                eg = rel_err(G.cpu().numpy()[b, :, k], Go[:, a, c])
                tg = 1e-12 * max(1.0, np.abs(Go[:, a, a]).max() / max(np.abs(Go[:, a, c]).max(), 1e-300))
                assert eg < tg, (l, b, a, c, eg)
            ea = rel_err(y.cpu().numpy()[b], h.apply(x[b], lo_))
            print(f"[elements 3-D] K={K} p={p} b={b} operator rel err {ea:.2e}")
            assert ea < op_tol(p), (l, b, ea)
        if l > l0:
            pc = p // 2
            rf = np.random.default_rng(l).standard_normal((B, (p + 1) ** 3))
            rc = torch.empty((B, (pc + 1) ** 3), dtype=torch.float64, device="cuda")
            pmg.pmg_restrict(s.h, l, pmg.PMG_F64, torch.from_numpy(rf).cuda(), rc)
            torch.cuda.synchronize()
            for b, (h, _, _) in enumerate(case3["ors"]):
                assert rel_err(rc.cpu().numpy()[b], h.restrict(rf[b], lo_)) < 1e-12


def test_3d_cycle_and_solve(case3):
    s, p = case3["s"], case3["p"]
    B = len(SEEDS3)
    m = interior_mask(3, p)
    r = np.where(m[None, :], np.random.default_rng(70).standard_normal((B, (p + 1) ** 3)), 0.0)
    yc = torch.empty((B, (p + 1) ** 3), dtype=torch.float64, device="cuda")
    pmg.pmg_gamma_cycle(s.h, pmg.PMG_F64, torch.from_numpy(r).cuda(), yc)
    bt = torch.empty_like(case3["f"])
    pmg.pmg_rhs(s.h, case3["f"], case3["g"], bt)
    x = torch.empty_like(bt)
    pmg.pmg_solve(s.h, bt, x, s.info)
    torch.cuda.synchronize()
    info = s.info_host()
    for b, (h, f, g) in enumerate(case3["ors"]):
        ec = rel_err(yc.cpu().numpy()[b], h.cycle(r[b]))
        bo = h.rhs(f, g)
        xg = x.cpu().numpy()[b]
        rr = np.linalg.norm(bo - h.apply(xg)) / np.linalg.norm(bo)
        xo, st, it, _ = h.fgmres(bo, rtol=1e-10, maxit=200, restart=20)
        ex = rel_err(xg, xo)
        print(f"[elements 3-D solve] K={case3['K']} p={p} b={b} cycle err {ec:.2e} its gpu "
              f"{info['iterations'][b]} oracle {it} oracle-operator relres {rr:.3e} err {ex:.2e}")
        assert ec < 1e-10
        assert info["status"][b] == 0 and rr <= 1.0001e-10 and st == 0
        assert abs(int(info["iterations"][b]) - it) <= 1 and ex < 1e-7

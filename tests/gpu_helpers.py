"""Helpers for the GPU parity tests: build seeded batches for the library and
the matching oracle hierarchies (each side with its own GLL nodes)."""
import numpy as np

from oracle import oracle as orc
from paper_2504_10710_amd import inputs
from paper_2504_10710_amd import pmg


def problems(kind, seeds):
    make = {"cfg1": inputs.config1, "cfg2": inputs.config2, "cfg3": inputs.config3,
            "mms": inputs.manufactured_deformed}[kind]
    return [make(s) for s in seeds]


def gpu_batch(probs, p_fine, device="cuda", **desc_kw):
    """Solver for a batch of problems of one shape; returns (solver, f, g)."""
    import torch
    dim = probs[0].dim
    desc = pmg.make_desc(dim=dim, p_fine=p_fine, batch=len(probs), **desc_kw)
    ps = inputs.halving_degrees(p_fine, 2)
    coords = []
    for p in ps:
        xi = pmg.pmg_gll(p)[0]
        arr = np.stack([pr.coords(xi) for pr in probs])
        coords.append(torch.from_numpy(arr).to(device))
    s = pmg.Solver(desc, coords, device=device)
    xi = pmg.pmg_gll(p_fine)[0]
    X = [pr.coords(xi) for pr in probs]
    f = torch.from_numpy(np.stack([pr.f(x) for pr, x in zip(probs, X)])).to(device)
    g = torch.from_numpy(np.stack([pr.g(x) for pr, x in zip(probs, X)])).to(device)
    return s, f, g


def oracle_of(prob, p_fine, gamma=1, m=1, alpha=0.16, smoother=1, restriction=orc.RESTRICT_INTERP):
    ps = inputs.halving_degrees(p_fine, 2)
    coords = [prob.coords(orc.gll(p)[0]) for p in ps]
    h = orc.Hier(prob.dim, ps, coords, gamma=gamma, m=m, alpha=alpha, smoother=smoother,
                 restriction=restriction)
    X = coords[-1]
    return h, prob.f(X), prob.g(X)


def interior_mask(dim, p):
    n1 = p + 1
    m1 = np.zeros(n1, dtype=bool)
    m1[1:-1] = True
    grids = np.meshgrid(*([m1] * dim), indexing="ij")
    return np.logical_and.reduce([gr.reshape(-1, order="F") for gr in grids])


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)

"""Shared test helpers: build oracle hierarchies for seeded problems."""
import numpy as np

from oracle import oracle as orc
from paper_2504_10710_amd import inputs


def oracle_hier(problem, p_fine, p_coarse=2, gamma=1, m=1, alpha=2.0 / 3.0, smoother=0,
                restriction=orc.RESTRICT_TRANSPOSE):
    ps = inputs.halving_degrees(p_fine, p_coarse)
    coords = [problem.coords(orc.gll(p)[0]) for p in ps]
    h = orc.Hier(problem.dim, ps, coords, gamma=gamma, m=m, alpha=alpha, smoother=smoother,
                 restriction=restriction)
    return h, ps, coords


def interior_mask(dim, p):
    n1 = p + 1
    m1 = np.zeros(n1, dtype=bool)
    m1[1:-1] = True
    grids = np.meshgrid(*([m1] * dim), indexing="ij")
    return np.logical_and.reduce([g.reshape(-1, order="F") for g in grids])

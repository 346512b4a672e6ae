"""Seeded synthetic problem generators.

This module defines the *problems* (domain mappings, right-hand sides,
Dirichlet data) that both the GPU library and the CPU oracle solve.  It holds
none of the method's arithmetic: no quadrature, no operator, no solver.  The
caller passes the 1-D reference node positions (each side uses its own GLL
nodes) and gets back physical coordinates and nodal values of f and g.

Conventions
  * Reference coordinates xi in [-1, 1]^d map to the unit cube by
    s = (xi + 1) / 2, then to the physical domain by the mapping Phi(s).
  * Nodes are ordered lexicographically, first axis fastest.
  * The PDE is -Laplace(u) = f (so that the stiffness matrix is positive
    definite), u = g on the boundary.

Workloads (shapes and value distributions of the paper's experiments; the
paper uses manufactured solutions only, no public data set):
  config 1  2-D unit square, p = 16: u* = sin(pi x) sin(pi y)
            + 0.1 sum_{k=1..4} c_k cos(k pi x) cos(k pi y), c_k ~ N(0,1);
            f = -Laplace(u*), g = u* on the boundary.
  config 2  2-D deformed square, p = 128: x = s + a sin(pi s) sin(pi t),
            y = t + b sin(2 pi s) sin(pi t), a, b ~ U[0, 0.15];
            f = sum_{k1,k2=1..4} c/(k1^2+k2^2) sin(k1 pi x) sin(k2 pi y),
            g = sum_{k=1..4} (d_k cos(k pi x) + e_k cos(k pi y)) / k^2.
  config 3  3-D deformed cube, p = 64: x_c = s_c + beta_c s t u
            + a_c sin(pi s) sin(pi t) sin(pi u), beta, a ~ U[0, 0.1]^3;
            f = sum_{k in {1,2,3}^3} c_k/|k|^2 prod sin(k_i pi x_i), g = 0.
  table-1   the three problems of the paper's square-domain experiments.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

PI = np.pi


def unit_coords(nodes_1d, dim: int):
    """Unit-cube coordinates s (dim, N) of the tensor grid of 1-D nodes."""
    s1 = (np.asarray(nodes_1d, dtype=np.float64) + 1.0) / 2.0
    grids = np.meshgrid(*([s1] * dim), indexing="ij")
    # lexicographic with the first axis fastest: flatten in Fortran order
    return np.stack([g.reshape(-1, order="F") for g in grids])


def composite_nodes(nodes_1d, K: int) -> np.ndarray:
    """Reference positions in [-1, 1] of the composite node grid of K equal
    elements along an axis, each carrying the 1-D nodes ``nodes_1d`` (given
    on [-1, 1]); interface nodes appear once (K p + 1 nodes)."""
    xi = np.asarray(nodes_1d, dtype=np.float64)
    pe = len(xi) - 1
    out = np.empty(K * pe + 1)
    for e in range(K):
        out[e * pe:(e + 1) * pe + 1] = -1.0 + (2.0 * e + 1.0 + xi) / K
    return out


@dataclass
class Problem:
    """A seeded problem instance: mapping parameters and data coefficients."""
    dim: int
    kind: str
    params: dict = field(default_factory=dict)

    # -------------------------------------------------------------- mapping
    def coords(self, nodes_1d) -> np.ndarray:
        """Physical coordinates (dim, N) of the tensor grid of ``nodes_1d``."""
        s = unit_coords(nodes_1d, self.dim)
        P = self.params
        if self.kind in ("square", "table1"):
            return s.copy()
        if self.kind in ("deformed2d", "mms2d"):
            a, b = P["a"], P["b"]
            x = s[0] + a * np.sin(PI * s[0]) * np.sin(PI * s[1])
            y = s[1] + b * np.sin(2 * PI * s[0]) * np.sin(PI * s[1])
            return np.stack([x, y])
        if self.kind == "deformed3d":
            beta, amp = P["beta"], P["amp"]
            prod = s[0] * s[1] * s[2]
            bump = np.sin(PI * s[0]) * np.sin(PI * s[1]) * np.sin(PI * s[2])
            return np.stack([s[c] + beta[c] * prod + amp[c] * bump for c in range(3)])
        raise ValueError(self.kind)

    # -------------------------------------------------------------- data
    def f(self, X: np.ndarray) -> np.ndarray:
        """Right-hand side f = -Laplace(u) at physical points X (dim, N)."""
        P = self.params
        if self.kind in ("square", "mms2d"):
            x, y = X
            c = P["c"]
            v = 2 * PI**2 * np.sin(PI * x) * np.sin(PI * y)
            for k in range(1, 5):
                v = v + 0.1 * c[k - 1] * 2 * (k * PI) ** 2 * np.cos(k * PI * x) * np.cos(k * PI * y)
            return v
        if self.kind == "deformed2d":
            x, y = X
            c = P["c"]
            v = np.zeros_like(x)
            for k1 in range(1, 5):
                for k2 in range(1, 5):
                    v = v + c[k1 - 1, k2 - 1] / (k1 * k1 + k2 * k2) * np.sin(k1 * PI * x) * np.sin(k2 * PI * y)
            return v
        if self.kind == "deformed3d":
            # sum_{k in {1,2,3}^3} c_k / |k|^2 prod_i sin(k_i pi x_i), the three
            # sine factors of each axis evaluated once
            c = P["c"]
            k = np.arange(1, 4)
            w = c / (k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2)
            S = [np.sin(np.multiply.outer(k * PI, X[a])) for a in range(3)]
            return np.einsum("abc,an,bn,cn->n", w, S[0], S[1], S[2], optimize=True)
        if self.kind == "table1":
            x, y = X
            which = P["problem"]
            if which == 1:
                return np.ones_like(x)
            if which == 2:
                return 128 * PI**2 * np.sin(8 * PI * x) * np.sin(8 * PI * y)
            if which == 3:
                s = x + y + PI / 10
                th = 8 * PI / s
                # -Laplace(sin(8 pi / s)), s = x + y + pi/10
                return -2 * (-np.sin(th) * (8 * PI) ** 2 / s**4 + np.cos(th) * 16 * PI / s**3)
        raise ValueError(self.kind)

    def g(self, X: np.ndarray) -> np.ndarray:
        """Dirichlet data (only its boundary-node values are used)."""
        P = self.params
        if self.kind in ("square", "table1", "mms2d"):
            u = self.exact(X)
            return u if u is not None else np.zeros_like(X[0])
        if self.kind == "deformed2d":
            x, y = X
            d, e = P["d"], P["e"]
            v = np.zeros_like(x)
            for k in range(1, 5):
                v = v + (d[k - 1] * np.cos(k * PI * x) + e[k - 1] * np.cos(k * PI * y)) / (k * k)
            return v
        if self.kind == "deformed3d":
            return np.zeros_like(X[0])
        raise ValueError(self.kind)

    def exact(self, X: np.ndarray):
        """Manufactured solution where one exists, else None."""
        P = self.params
        if self.kind in ("square", "mms2d"):
            x, y = X
            c = P["c"]
            v = np.sin(PI * x) * np.sin(PI * y)
            for k in range(1, 5):
                v = v + 0.1 * c[k - 1] * np.cos(k * PI * x) * np.cos(k * PI * y)
            return v
        if self.kind == "table1":
            x, y = X
            which = P["problem"]
            if which == 2:
                return np.sin(8 * PI * x) * np.sin(8 * PI * y)
            if which == 3:
                return np.sin(8 * PI / (x + y + PI / 10))
            return np.zeros_like(x) if which == 1 else None
        return None


def config1(seed: int) -> Problem:
    rng = np.random.default_rng(seed)
    return Problem(2, "square", {"c": rng.standard_normal(4)})


def config2(seed: int, amp_max: float = 0.15) -> Problem:
    rng = np.random.default_rng(seed)
    a, b = rng.uniform(0.0, amp_max, size=2)
    c = rng.standard_normal((4, 4))
    d = rng.standard_normal(4)
    e = rng.standard_normal(4)
    return Problem(2, "deformed2d", {"a": float(a), "b": float(b), "c": c, "d": d, "e": e})


def _mapping3_min_det(beta, amp, m: int = 13) -> float:
    """Smallest Jacobian determinant of the config-3 mapping
    x_c = s_c + beta_c s t u + amp_c sin(pi s) sin(pi t) sin(pi u) on an m^3
    grid of the unit cube (analytic derivatives of the mapping; a check that
    a drawn problem is a valid domain, not part of the method)."""
    g = np.linspace(0.0, 1.0, m)
    s = np.stack(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1)
    sn, cs = np.sin(PI * s), np.cos(PI * s)
    J = np.zeros((s.shape[1], 3, 3))
    for c in range(3):
        for d in range(3):
            e1, e2 = [e for e in range(3) if e != d]
            J[:, c, d] = (c == d) + beta[c] * s[e1] * s[e2] + amp[c] * PI * cs[d] * sn[e1] * sn[e2]
    return float(np.linalg.det(J).min())


def config3(seed: int, amp_max: float = 0.1) -> Problem:
    """Config-3 problem; amplitudes ~ U[0, amp_max], redrawn (same stream)
    while the mapping folds (det J <= 0 somewhere)."""
    rng = np.random.default_rng(seed)
    while True:
        beta = rng.uniform(0.0, amp_max, size=3)
        amp = rng.uniform(0.0, amp_max, size=3)
        if amp_max <= 0.1 or _mapping3_min_det(beta, amp) > 0.0:
            break
    c = rng.standard_normal((3, 3, 3))
    return Problem(3, "deformed3d", {"beta": beta, "amp": amp, "c": c})


def manufactured_deformed(seed: int, amp_max: float = 0.15) -> Problem:
    """The config-1 manufactured solution on the config-2 deformed square."""
    rng = np.random.default_rng(seed)
    a, b = rng.uniform(0.0, amp_max, size=2)
    return Problem(2, "mms2d", {"a": float(a), "b": float(b), "c": rng.standard_normal(4)})


def table1(problem: int) -> Problem:
    return Problem(2, "table1", {"problem": int(problem)})


def halving_degrees(p_fine: int, p_coarse: int = 2):
    """Degrees of a p-hierarchy halving from p_fine down to p_coarse, coarsest first."""
    ps = []
    p = int(p_fine)
    while p >= p_coarse:
        ps.append(p)
        if p == p_coarse:
            break
        p //= 2
    return ps[::-1]


def served_stream(n_requests: int, seed: int, amp_max: float = 0.15):
    """Request mix of the served workload: dim in {2, 3} with probability 1/2,
    2-D p ~ U{16,32,64,128}, 3-D p ~ U{16,32,64}; each request carries its own
    problem seed; deformation amplitudes ~ U[0, amp_max] in 2-D and 3-D (3-D
    redrawn while the mapping folds).  Returns a list of (dim, p, Problem)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_requests):
        dim = 2 if rng.random() < 0.5 else 3
        if dim == 2:
            p = int(rng.choice([16, 32, 64, 128]))
            prob = config2(seed * 1_000_003 + i, amp_max)
        else:
            p = int(rng.choice([16, 32, 64]))
            prob = config3(seed * 1_000_003 + i, amp_max)
        out.append((dim, p, prob))
    return out

"""Python face of the FP64 CPU oracle (``pmg_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the GPU library and never imports it; the GPU library never imports it.

Everything here is argument marshalling (numpy <-> ctypes) around the C
oracle, plus ``build()``, which compiles the C file with gcc.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pmg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` (plain gcc, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-fPIC", "-shared",
             "-o", tmp, _SRC, "-lm"], cwd=_HERE)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        sig = {
            "or_gll": (ctypes.c_int, [ctypes.c_int, _D, _D]),
            "or_legendre": (None, [ctypes.c_int, ctypes.c_double, _D, _D]),
            "or_deriv": (None, [ctypes.c_int, _D, _D]),
            "or_interp": (None, [ctypes.c_int, _D, ctypes.c_int, _D, _D]),
            "or_cr_solve": (ctypes.c_int, [ctypes.c_int, _D, _D, _D, _D, _D]),
            "or_thomas": (ctypes.c_int, [ctypes.c_int, _D, _D, _D, _D, _D]),
            "or_dense_solve": (ctypes.c_int, [ctypes.c_int, _D, _D]),
            "or_cr_coarse": (None, [ctypes.c_int, _D, _D, _D, _D, _D, _D]),
            "or_bcr_solve": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _D, _D, _D, _D, _D]),
            "or_bcr_coarse": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _D, _D, _D, _D, _D, _D]),
            "or_hier_create": (vp, [ctypes.c_int, ctypes.c_int, _I, ctypes.POINTER(_D),
                                    ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                    ctypes.c_int]),
            "or_hier_create_elements": (vp, [ctypes.c_int, ctypes.c_int, ctypes.c_int, _I,
                                             ctypes.POINTER(_D), ctypes.c_int, ctypes.c_int,
                                             ctypes.c_double, ctypes.c_int, ctypes.c_int]),
            "or_elements": (ctypes.c_int, [vp]),
            "or_geom_elements": (ctypes.c_int, [vp, ctypes.c_int, _D]),
            "or_line_band": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, _D]),
            "or_hier_destroy": (None, [vp]),
            "or_nodes": (ctypes.c_int, [vp, ctypes.c_int]),
            "or_geom": (ctypes.c_double, [vp, ctypes.c_int, _D, _D]),
            "or_apply": (None, [vp, ctypes.c_int, _D, _D]),
            "or_apply_all": (None, [vp, ctypes.c_int, _D, _D]),
            "or_entry": (ctypes.c_double, [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
            "or_dense_interior": (ctypes.c_int, [vp, ctypes.c_int, _D]),
            "or_fem_entry": (ctypes.c_double, [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
            "or_rhs": (None, [vp, _D, _D, _D]),
            "or_restrict": (None, [vp, ctypes.c_int, _D, _D]),
            "or_prolong_add": (None, [vp, ctypes.c_int, _D, _D]),
            "or_line_coefs": (None, [vp, ctypes.c_int, ctypes.c_int, _D, _D, _D]),
            "or_line_solve": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, _D, _D]),
            "or_smooth": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, _D, _D]),
            "or_cycle": (ctypes.c_int, [vp, ctypes.c_int, _D, _D]),
            "or_fgmres": (ctypes.c_int, [vp, _D, _D, ctypes.c_double, ctypes.c_int,
                                         ctypes.c_int, _D, _I]),
            "or_pcg": (ctypes.c_int, [vp, _D, _D, ctypes.c_double, ctypes.c_int, _D, _I]),
            "or_fcg": (ctypes.c_int, [vp, _D, _D, ctypes.c_double, ctypes.c_int, _D, _I]),
            "or_visits": (None, [vp, ctypes.POINTER(ctypes.c_longlong)]),
            "or_reset_visits": (None, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- 1-D pieces

def gll(p: int):
    xi = np.zeros(p + 1)
    rho = np.zeros(p + 1)
    if lib().or_gll(p, _p(xi), _p(rho)) != 0:
        raise RuntimeError(f"or_gll failed for p={p}")
    return xi, rho


def legendre(p: int, x: float):
    L = ctypes.c_double()
    dL = ctypes.c_double()
    lib().or_legendre(p, float(x), ctypes.byref(L), ctypes.byref(dL))
    return L.value, dL.value


def deriv(p: int, xi=None):
    if xi is None:
        xi, _ = gll(p)
    xi = _f64(xi)
    D = np.zeros((p + 1) * (p + 1))
    lib().or_deriv(p, _p(xi), _p(D))
    return D.reshape(p + 1, p + 1)


def interp(pc: int, xic, xf):
    xic = _f64(xic)
    xf = _f64(xf)
    J = np.zeros(len(xf) * (pc + 1))
    lib().or_interp(pc, _p(xic), len(xf), _p(xf), _p(J))
    return J.reshape(len(xf), pc + 1)


def cr_solve(l, a, u, g):
    l, a, u, g = (_f64(v) for v in (l, a, u, g))
    y = np.zeros(len(a))
    if lib().or_cr_solve(len(a), _p(l), _p(a), _p(u), _p(g), _p(y)) != 0:
        raise ZeroDivisionError("zero pivot in cyclic reduction")
    return y


def thomas(l, a, u, g):
    l, a, u, g = (_f64(v) for v in (l, a, u, g))
    y = np.zeros(len(a))
    if lib().or_thomas(len(a), _p(l), _p(a), _p(u), _p(g), _p(y)) != 0:
        raise ZeroDivisionError("zero pivot in Thomas")
    return y


def dense_solve(A, g):
    A = np.array(A, dtype=np.float64, order="C")
    g = np.array(g, dtype=np.float64)
    if lib().or_dense_solve(len(g), _p(A), _p(g)) != 0:
        raise ZeroDivisionError("singular dense matrix")
    return g


def cr_coarse(l, a, u):
    l, a, u = (_f64(v) for v in (l, a, u))
    nc = len(a) // 2
    l0, a0, u0 = np.zeros(nc), np.zeros(nc), np.zeros(nc)
    lib().or_cr_coarse(len(a), _p(l), _p(a), _p(u), _p(l0), _p(a0), _p(u0))
    return l0, a0, u0


def bcr_solve(Lb, Ab, Ub, g):
    """Block cyclic reduction: Lb, Ab, Ub are (nb, m, m), g is (nb*m,)."""
    Ab = np.ascontiguousarray(Ab, dtype=np.float64)
    nb, m, _ = Ab.shape
    Lb = np.ascontiguousarray(Lb, dtype=np.float64)
    Ub = np.ascontiguousarray(Ub, dtype=np.float64)
    g = _f64(g)
    y = np.zeros(nb * m)
    if lib().or_bcr_solve(nb, m, _p(Lb), _p(Ab), _p(Ub), _p(g), _p(y)) != 0:
        raise ZeroDivisionError("singular block in block cyclic reduction")
    return y


def bcr_coarse(Lb, Ab, Ub):
    Ab = np.ascontiguousarray(Ab, dtype=np.float64)
    nb, m, _ = Ab.shape
    Lb = np.ascontiguousarray(Lb, dtype=np.float64)
    Ub = np.ascontiguousarray(Ub, dtype=np.float64)
    nc = nb // 2
    L0, A0, U0 = (np.zeros((nc, m, m)) for _ in range(3))
    if lib().or_bcr_coarse(nb, m, _p(Lb), _p(Ab), _p(Ub), _p(L0), _p(A0), _p(U0)) != 0:
        raise ZeroDivisionError("singular block")
    return L0, A0, U0


# line-system and restriction choices of the hierarchy (pmg_oracle.h)
SMOOTHER_GLL, SMOOTHER_FEM, SMOOTHER_GLL_BAND2, SMOOTHER_GLL_FULL = 0, 1, 2, 3
RESTRICT_TRANSPOSE, RESTRICT_INTERP = 0, 1


# ---------------------------------------------------------------- hierarchy

class Hier:
    """A multigrid hierarchy of the oracle.

    ``plist`` ascending degrees (coarsest first); ``coords[l]`` is a
    (dim, N_l) array of physical node positions of level l.  ``elements`` =
    K > 1: K^dim spectral elements per level, ``plist`` the degrees of the
    composite grids (K times the element degrees).
    """

    def __init__(self, dim, plist, coords, gamma=7, m=1, alpha=2.0 / 3.0, smoother=0,
                 restriction=RESTRICT_TRANSPOSE, elements=1):
        self.dim = int(dim)
        self.plist = [int(p) for p in plist]
        self.nlev = len(self.plist)
        self._coords = [_f64(np.asarray(c).reshape(-1)) for c in coords]
        cp = (_D * self.nlev)(*[_p(c) for c in self._coords])
        pl = (ctypes.c_int * self.nlev)(*self.plist)
        self.elements = int(elements)
        self.h = lib().or_hier_create_elements(self.dim, self.elements, self.nlev, pl, cp,
                                               int(gamma), int(m), float(alpha), int(smoother),
                                               int(restriction))
        if not self.h:
            raise ValueError("or_hier_create failed (bad arguments or det J <= 0)")
        self.gamma, self.m, self.alpha = gamma, m, alpha
        self.smoother, self.restriction = int(smoother), int(restriction)

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_hier_destroy(self.h)
            self.h = None

    def N(self, l=-1):
        l = l % self.nlev
        return (self.plist[l] + 1) ** self.dim

    def geom(self, l=-1):
        l = l % self.nlev
        N = self.N(l)
        G = np.zeros(self.dim * self.dim * N)
        mass = np.zeros(N)
        mindet = lib().or_geom(self.h, l, _p(G), _p(mass))
        return G.reshape(self.dim, self.dim, N), mass, mindet

    def geom_elements(self, l=-1):
        """Element geometric factors (K^dim, dim, dim, NE) of an element hierarchy."""
        l = l % self.nlev
        n = lib().or_geom_elements(self.h, l, None)
        if n < 0:
            raise ValueError("not an element hierarchy")
        G = np.zeros(n)
        lib().or_geom_elements(self.h, l, _p(G))
        return G.reshape(self.elements ** self.dim, self.dim, self.dim, -1)

    def apply(self, x, l=-1, all_rows=False):
        l = l % self.nlev
        x = _f64(x)
        y = np.zeros(self.N(l))
        (lib().or_apply_all if all_rows else lib().or_apply)(self.h, l, _p(x), _p(y))
        return y

    def entry(self, row, col, l=-1):
        return lib().or_entry(self.h, l % self.nlev, int(row), int(col))

    def fem_entry(self, row, col, l=-1):
        return lib().or_fem_entry(self.h, l % self.nlev, int(row), int(col))

    def dense_interior(self, l=-1):
        l = l % self.nlev
        n = lib().or_dense_interior(self.h, l, None)
        A = np.zeros(n * n)
        lib().or_dense_interior(self.h, l, _p(A))
        return A.reshape(n, n)

    def rhs(self, f, g):
        f, g = _f64(f), _f64(g)
        b = np.zeros(self.N())
        lib().or_rhs(self.h, _p(f), _p(g), _p(b))
        return b

    def restrict(self, rf, l=-1):
        l = l % self.nlev
        rf = _f64(rf)
        rc = np.zeros(self.N(l - 1))
        lib().or_restrict(self.h, l, _p(rf), _p(rc))
        return rc

    def prolong_add(self, ec, xf, l=-1):
        l = l % self.nlev
        ec = _f64(ec)
        out = np.array(xf, dtype=np.float64)
        lib().or_prolong_add(self.h, l, _p(ec), _p(out))
        return out

    def line_coefs(self, dir, l=-1):
        l = l % self.nlev
        n = (self.plist[l] - 1) ** self.dim
        lo, di, up = np.zeros(n), np.zeros(n), np.zeros(n)
        lib().or_line_coefs(self.h, l, dir, _p(lo), _p(di), _p(up))
        return lo, di, up

    def line_band(self, dir, l=-1):
        """Half-bandwidth-2 line entries (lines, n, 5) of the band-2 smoother."""
        l = l % self.nlev
        n = self.plist[l] - 1
        out = np.zeros(n ** self.dim * 5)
        if lib().or_line_band(self.h, l, dir, _p(out)) != 0:
            raise ValueError("hierarchy has no banded line systems")
        return out.reshape(n ** (self.dim - 1), n, 5)

    def line_solve(self, r, dir, l=-1):
        l = l % self.nlev
        r = _f64(r)
        z = np.zeros(self.N(l))
        if lib().or_line_solve(self.h, l, dir, _p(r), _p(z)) != 0:
            raise ZeroDivisionError("zero pivot in a line solve")
        return z

    def smooth(self, r, x, dir, l=-1):
        l = l % self.nlev
        r = _f64(r)
        out = np.array(x, dtype=np.float64)
        if lib().or_smooth(self.h, l, dir, _p(r), _p(out)) != 0:
            raise ZeroDivisionError("zero pivot in a line solve")
        return out

    def cycle(self, r, l=-1):
        l = l % self.nlev
        r = _f64(r)
        y = np.zeros(self.N(l))
        if lib().or_cycle(self.h, l, _p(r), _p(y)) != 0:
            raise ZeroDivisionError("zero pivot in the cycle")
        return y

    def _krylov(self, which, b, rtol, maxit, restart=30):
        b = _f64(b)
        x = np.zeros(self.N())
        hist = np.zeros(maxit + 1)
        it = ctypes.c_int(0)
        if which == "fgmres":
            st = lib().or_fgmres(self.h, _p(b), _p(x), float(rtol), int(maxit), int(restart),
                                 _p(hist), ctypes.byref(it))
        elif which == "pcg":
            st = lib().or_pcg(self.h, _p(b), _p(x), float(rtol), int(maxit), _p(hist),
                              ctypes.byref(it))
        elif which == "fcg":
            st = lib().or_fcg(self.h, _p(b), _p(x), float(rtol), int(maxit), _p(hist),
                              ctypes.byref(it))
        else:
            raise ValueError(which)
        return x, st, it.value, hist[: it.value + 1]

    def fgmres(self, b, rtol=1e-10, maxit=500, restart=30):
        return self._krylov("fgmres", b, rtol, maxit, restart)

    def pcg(self, b, rtol=1e-10, maxit=500):
        return self._krylov("pcg", b, rtol, maxit)

    def fcg(self, b, rtol=1e-10, maxit=500):
        return self._krylov("fcg", b, rtol, maxit)

    def visits(self):
        v = (ctypes.c_longlong * self.nlev)()
        lib().or_visits(self.h, v)
        return list(v)

    def reset_visits(self):
        lib().or_reset_visits(self.h)

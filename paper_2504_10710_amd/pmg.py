"""Thin ctypes binding of ``libpmg.so`` (C ABI in ``include/pmg.h``).

Argument marshalling only: every computation happens in the library's HIP
kernels.  Device arrays are torch tensors (PyTorch supplies device memory and
streams); they are passed to the library as raw pointers together with the
current HIP stream.  If ``libpmg.so`` is missing the binding raises; there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpmg.so")
_lib = None

PMG_OK, PMG_EINVAL, PMG_ENOMEM, PMG_EDEVICE = 0, -1, -2, -3
PMG_EGEOM, PMG_ENAN, PMG_EBREAKDOWN, PMG_ENOTCONV, PMG_EPIVOT = -4, -5, -6, -7, -8
PMG_F64, PMG_F32 = 0, 1
PMG_SMOOTHER_GLL, PMG_SMOOTHER_FEM, PMG_SMOOTHER_GLL_BAND2 = 0, 1, 2
PMG_FGMRES, PMG_PCG, PMG_FCG = 0, 1, 2
PMG_RESTRICT_TRANSPOSE, PMG_RESTRICT_INTERP = 0, 1
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EGEOM", -5: "ENAN",
                -6: "EBREAKDOWN", -7: "ENOTCONV", -8: "EPIVOT"}


class pmg_desc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("p_fine", ctypes.c_int), ("batch", ctypes.c_int),
                ("gamma", ctypes.c_int), ("m", ctypes.c_int), ("alpha", ctypes.c_double),
                ("smoother", ctypes.c_int), ("inner_prec", ctypes.c_int),
                ("krylov", ctypes.c_int), ("restart", ctypes.c_int),
                ("max_iter", ctypes.c_int), ("rtol", ctypes.c_double),
                ("restriction", ctypes.c_int), ("elements", ctypes.c_int)]


MAX_CLASSES = 8


class pmg_region(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("offset", ctypes.c_size_t), ("bytes", ctypes.c_size_t)]


class pmg_server_desc(ctypes.Structure):
    _fields_ = [("n_classes", ctypes.c_int), ("classes", pmg_desc * MAX_CLASSES),
                ("iters_per_step", ctypes.c_int), ("budget_bytes", ctypes.c_size_t)]


class pmg_server_stats(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int), ("running", ctypes.c_int), ("finished", ctypes.c_int),
                ("bytes_in_use", ctypes.c_size_t), ("steps", ctypes.c_longlong)]


INFO_DTYPE = np.dtype([("status", np.int32), ("iterations", np.int32),
                       ("relres", np.float64), ("min_detj", np.float64)])
INFO_BYTES = INFO_DTYPE.itemsize  # 24, the layout of pmg_info


class PmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        dp = ctypes.POINTER(ctypes.c_double)
        sig = {
            "pmg_last_error": (ctypes.c_char_p, []),
            "pmg_num_levels": (i, [ctypes.POINTER(pmg_desc), ctypes.POINTER(i)]),
            "pmg_first_level": (i, [ctypes.POINTER(pmg_desc), ctypes.POINTER(i)]),
            "pmg_gll": (i, [i, dp, dp, dp]),
            "pmg_interp": (i, [i, i, dp]),
            "pmg_workspace_bytes": (i, [ctypes.POINTER(pmg_desc), ctypes.POINTER(ctypes.c_size_t)]),
            "pmg_setup": (i, [ctypes.POINTER(pmg_desc), ctypes.POINTER(vp), vp, ctypes.c_size_t,
                              vp, vp, ctypes.POINTER(vp)]),
            "pmg_rhs": (i, [vp, vp, vp, vp, vp]),
            "pmg_lift": (i, [vp, vp, vp, vp, vp]),
            "pmg_apply": (i, [vp, i, i, vp, vp, vp]),
            "pmg_restrict": (i, [vp, i, i, vp, vp, vp]),
            "pmg_prolong_add": (i, [vp, i, i, vp, vp, vp]),
            "pmg_line_solve": (i, [vp, i, i, i, vp, vp, vp]),
            "pmg_line_smooth": (i, [vp, i, i, i, vp, vp, vp]),
            "pmg_gamma_cycle": (i, [vp, i, vp, vp, vp]),
            "pmg_solve": (i, [vp, vp, vp, vp, vp]),
            "pmg_solve_noalloc": (i, [vp, vp, vp, vp, vp]),
            "pmg_workspace_layout": (i, [vp, vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
            "pmg_line_band": (i, [vp, i, i, vp, vp]),
            "pmg_line_coefs": (i, [vp, i, i, vp, vp, vp, vp]),
            "pmg_geom": (i, [vp, i, vp, vp, vp]),
            "pmg_destroy": (i, [vp]),
            "pmg_pool_workspace_bytes": (i, [ctypes.POINTER(pmg_desc), ctypes.POINTER(ctypes.c_size_t)]),
            "pmg_pool_create": (i, [ctypes.POINTER(pmg_desc), i, vp, ctypes.c_size_t, vp,
                                    ctypes.POINTER(vp)]),
            "pmg_pool_admit": (i, [vp, i, ctypes.POINTER(i), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                   ctypes.POINTER(vp), vp]),
            "pmg_pool_step": (i, [vp, vp]),
            "pmg_pool_poll": (i, [vp, ctypes.POINTER(i), vp, vp]),
            "pmg_pool_take": (i, [vp, i, vp, vp]),
            "pmg_pool_destroy": (i, [vp]),
            "pmg_server_workspace_bytes": (i, [ctypes.POINTER(pmg_server_desc),
                                               ctypes.POINTER(ctypes.c_size_t)]),
            "pmg_server_create": (i, [ctypes.POINTER(pmg_server_desc), vp, ctypes.c_size_t,
                                      ctypes.POINTER(vp), ctypes.POINTER(vp)]),
            "pmg_server_submit": (i, [vp, i, ctypes.POINTER(vp), vp, vp, vp,
                                      ctypes.POINTER(ctypes.c_longlong)]),
            "pmg_server_step": (i, [vp, ctypes.POINTER(i)]),
            "pmg_server_poll": (i, [vp, ctypes.c_longlong, vp]),
            "pmg_server_drain": (i, [vp, vp, i, ctypes.POINTER(i)]),
            "pmg_server_stats_get": (i, [vp, ctypes.POINTER(pmg_server_stats)]),
            "pmg_server_destroy": (i, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    """Names the binding expects the library to export."""
    return ["pmg_last_error", "pmg_num_levels", "pmg_first_level", "pmg_gll", "pmg_interp", "pmg_workspace_bytes",
            "pmg_setup", "pmg_rhs", "pmg_lift", "pmg_apply", "pmg_restrict", "pmg_prolong_add",
            "pmg_line_solve", "pmg_line_smooth", "pmg_gamma_cycle", "pmg_solve",
            "pmg_line_coefs", "pmg_geom", "pmg_destroy", "pmg_pool_workspace_bytes",
            "pmg_pool_create", "pmg_pool_admit", "pmg_pool_step", "pmg_pool_poll", "pmg_pool_take",
            "pmg_pool_destroy", "pmg_server_workspace_bytes", "pmg_server_create",
            "pmg_server_submit", "pmg_server_step", "pmg_server_poll", "pmg_server_drain",
            "pmg_server_stats_get",
            "pmg_server_destroy", "pmg_solve_noalloc", "pmg_workspace_layout", "pmg_line_band"]


def _check(rc):
    if rc != PMG_OK:
        raise PmgError(rc, lib().pmg_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# ------------------------------------------------------------------ host calls

def pmg_gll(p: int):
    xi = np.zeros(p + 1)
    rho = np.zeros(p + 1)
    D = np.zeros((p + 1) * (p + 1))
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib().pmg_gll(p, xi.ctypes.data_as(dp), rho.ctypes.data_as(dp), D.ctypes.data_as(dp)))
    return xi, rho, D.reshape(p + 1, p + 1)


def pmg_interp(p_c: int, p_f: int):
    J = np.zeros((p_f + 1) * (p_c + 1))
    _check(lib().pmg_interp(p_c, p_f, J.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return J.reshape(p_f + 1, p_c + 1)


def make_desc(dim=2, p_fine=16, batch=1, gamma=1, m=1, alpha=0.16, smoother=PMG_SMOOTHER_FEM,
              inner_prec=PMG_F64, krylov=PMG_FGMRES, restart=30, max_iter=200, rtol=1e-10,
              restriction=PMG_RESTRICT_INTERP, elements=1):
    return pmg_desc(dim, p_fine, batch, gamma, m, alpha, smoother, inner_prec, krylov, restart,
                    max_iter, rtol, restriction, elements)


def pmg_num_levels(desc: pmg_desc) -> int:
    n = ctypes.c_int(0)
    _check(lib().pmg_num_levels(ctypes.byref(desc), ctypes.byref(n)))
    return n.value


def pmg_first_level(desc: pmg_desc) -> int:
    n = ctypes.c_int(0)
    _check(lib().pmg_first_level(ctypes.byref(desc), ctypes.byref(n)))
    return n.value


def pmg_workspace_bytes(desc: pmg_desc) -> int:
    n = ctypes.c_size_t(0)
    _check(lib().pmg_workspace_bytes(ctypes.byref(desc), ctypes.byref(n)))
    return n.value


# ------------------------------------------------------------------ device calls

def pmg_setup(desc, coords, ws, info, stream=None):
    """coords: list (coarsest first) of float64 device tensors (B, dim, N_l);
    ws: uint8 device tensor of pmg_workspace_bytes(desc); info: uint8 device
    tensor of B * INFO_BYTES.  Returns the handle (c_void_p)."""
    n = len(coords)
    arr = (ctypes.c_void_p * n)(*[None if c is None else c.data_ptr() for c in coords])
    h = ctypes.c_void_p()
    _check(lib().pmg_setup(ctypes.byref(desc), arr, _ptr(ws), ws.numel() * ws.element_size(),
                           _ptr(info), _stream(stream), ctypes.byref(h)))
    return h


def pmg_rhs(h, f, g, b, stream=None):
    _check(lib().pmg_rhs(h, _ptr(f), _ptr(g), _ptr(b), _stream(stream)))


def pmg_lift(h, w, g, u, stream=None):
    _check(lib().pmg_lift(h, _ptr(w), _ptr(g), _ptr(u), _stream(stream)))


def pmg_apply(h, level, prec, x, y, stream=None):
    _check(lib().pmg_apply(h, level, prec, _ptr(x), _ptr(y), _stream(stream)))


def pmg_restrict(h, level, prec, rf, rc, stream=None):
    _check(lib().pmg_restrict(h, level, prec, _ptr(rf), _ptr(rc), _stream(stream)))


def pmg_prolong_add(h, level, prec, ec, xf, stream=None):
    _check(lib().pmg_prolong_add(h, level, prec, _ptr(ec), _ptr(xf), _stream(stream)))


def pmg_line_solve(h, level, dir, prec, r, z, stream=None):
    _check(lib().pmg_line_solve(h, level, dir, prec, _ptr(r), _ptr(z), _stream(stream)))


def pmg_line_smooth(h, level, dir, prec, r, x, stream=None):
    _check(lib().pmg_line_smooth(h, level, dir, prec, _ptr(r), _ptr(x), _stream(stream)))


def pmg_gamma_cycle(h, prec, r, y, stream=None):
    _check(lib().pmg_gamma_cycle(h, prec, _ptr(r), _ptr(y), _stream(stream)))


def pmg_solve(h, b, x, info, stream=None):
    _check(lib().pmg_solve(h, _ptr(b), _ptr(x), _ptr(info), _stream(stream)))


def pmg_workspace_layout(desc: pmg_desc):
    """[(name, offset, bytes)] of the workspace pmg_setup lays out for desc."""
    n = ctypes.c_int(0)
    _check(lib().pmg_workspace_layout(ctypes.byref(desc), None, 0, ctypes.byref(n)))
    regs = (pmg_region * max(n.value, 1))()
    _check(lib().pmg_workspace_layout(ctypes.byref(desc), regs, n.value, ctypes.byref(n)))
    return [(r.name.decode(), int(r.offset), int(r.bytes)) for r in regs[: n.value]]


def pmg_solve_noalloc(h, b, x, info, stream=None):
    _check(lib().pmg_solve_noalloc(h, _ptr(b), _ptr(x), _ptr(info), _stream(stream)))


PMG_SCRATCH_BYTES = 64 << 20


def pmg_line_coefs(h, level, dir, lo, di, up, stream=None):
    _check(lib().pmg_line_coefs(h, level, dir, _ptr(lo), _ptr(di), _ptr(up), _stream(stream)))


def pmg_line_band(h, level, dir, band, stream=None):
    _check(lib().pmg_line_band(h, level, dir, _ptr(band), _stream(stream)))


def pmg_geom(h, level, G, mass=None, stream=None):
    _check(lib().pmg_geom(h, level, _ptr(G), _ptr(mass), _stream(stream)))


def pmg_destroy(h):
    if h:
        _check(lib().pmg_destroy(h))


# ------------------------------------------------------------------ serving

def pmg_pool_workspace_bytes(desc: pmg_desc) -> int:
    n = ctypes.c_size_t(0)
    _check(lib().pmg_pool_workspace_bytes(ctypes.byref(desc), ctypes.byref(n)))
    return n.value


def pmg_pool_create(desc, iters_per_step, ws, stream=None):
    h = ctypes.c_void_p()
    _check(lib().pmg_pool_create(ctypes.byref(desc), iters_per_step, _ptr(ws),
                                 ws.numel() * ws.element_size(), _stream(stream), ctypes.byref(h)))
    return h


def pmg_pool_admit(pool, slots, coords, fs, gs, stream=None):
    """slots: list of slot ids; coords: per request a list of level tensors
    (coarsest first); fs, gs: per request finest-level tensors."""
    n = len(slots)
    sl = (ctypes.c_int * n)(*slots)
    cp = (ctypes.c_void_p * sum(len(c) for c in coords))(
        *[None if t is None else t.data_ptr() for c in coords for t in c])
    fp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in fs])
    gp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in gs])
    _check(lib().pmg_pool_admit(pool, n, sl, cp, fp, gp, _stream(stream)))


def pmg_pool_step(pool, stream=None):
    _check(lib().pmg_pool_step(pool, _stream(stream)))


def pmg_pool_poll(pool, nslots, stream=None):
    st = (ctypes.c_int * nslots)()
    info = np.zeros(nslots, dtype=INFO_DTYPE)
    _check(lib().pmg_pool_poll(pool, st, ctypes.c_void_p(info.ctypes.data), _stream(stream)))
    return np.array(st[:], dtype=np.int32), info


def pmg_pool_take(pool, slot, u, stream=None):
    _check(lib().pmg_pool_take(pool, slot, _ptr(u), _stream(stream)))


def pmg_pool_destroy(pool):
    if pool:
        _check(lib().pmg_pool_destroy(pool))


def make_server_desc(classes, iters_per_step=4, budget_bytes=1 << 40):
    d = pmg_server_desc()
    d.n_classes = len(classes)
    for k, c in enumerate(classes):
        d.classes[k] = c
    d.iters_per_step = iters_per_step
    d.budget_bytes = budget_bytes
    return d


def pmg_server_workspace_bytes(desc) -> int:
    n = ctypes.c_size_t(0)
    _check(lib().pmg_server_workspace_bytes(ctypes.byref(desc), ctypes.byref(n)))
    return n.value


_server_streams = {}


def pmg_server_create(desc, ws, streams=None):
    """streams: one torch stream per class (default: a new default-priority
    stream each); the binding keeps them alive until pmg_server_destroy."""
    import torch
    if streams is None:
        streams = [torch.cuda.Stream() for _ in range(desc.n_classes)]
    arr = (ctypes.c_void_p * desc.n_classes)(*[s.cuda_stream for s in streams])
    h = ctypes.c_void_p()
    _check(lib().pmg_server_create(ctypes.byref(desc), _ptr(ws), ws.numel() * ws.element_size(),
                                   arr, ctypes.byref(h)))
    _server_streams[h.value] = list(streams)
    return h


def pmg_server_submit(srv, cls, coords, f, g, u) -> int:
    cp = (ctypes.c_void_p * len(coords))(*[None if t is None else t.data_ptr() for t in coords])
    t = ctypes.c_longlong(-1)
    _check(lib().pmg_server_submit(srv, cls, cp, _ptr(f), _ptr(g), _ptr(u), ctypes.byref(t)))
    return t.value


def pmg_server_step(srv) -> int:
    n = ctypes.c_int(0)
    _check(lib().pmg_server_step(srv, ctypes.byref(n)))
    return n.value


def pmg_server_poll(srv, ticket):
    info = np.zeros(1, dtype=INFO_DTYPE)
    rc = lib().pmg_server_poll(srv, ticket, ctypes.c_void_p(info.ctypes.data))
    if rc < 0:
        _check(rc)
    return rc == 1, info[0]


def pmg_server_drain(srv, max_n=4096):
    """Tickets retired since the previous drain (numpy int64 array)."""
    buf = np.empty(max_n, dtype=np.int64)
    n = ctypes.c_int(0)
    _check(lib().pmg_server_drain(srv, ctypes.c_void_p(buf.ctypes.data), max_n, ctypes.byref(n)))
    return buf[:n.value].copy()


def pmg_server_stats_get(srv):
    st = pmg_server_stats()
    _check(lib().pmg_server_stats_get(srv, ctypes.byref(st)))
    return {"queued": st.queued, "running": st.running, "finished": st.finished,
            "bytes_in_use": st.bytes_in_use, "steps": st.steps}


def pmg_server_destroy(srv):
    if srv:
        _check(lib().pmg_server_destroy(srv))
        _server_streams.pop(srv.value, None)


def info_to_numpy(info_tensor) -> np.ndarray:
    """Copy a device pmg_info array to a numpy structured array."""
    raw = info_tensor.detach().to("cpu").numpy().tobytes()
    return np.frombuffer(raw, dtype=INFO_DTYPE).copy()


class Solver:
    """Convenience owner of one batch: workspace, info array and handle.

    Device memory comes from torch; all work runs in the library."""

    def __init__(self, desc: pmg_desc, coords, device="cuda"):
        import torch
        self.desc = desc
        self.nlev = pmg_num_levels(desc)
        self.ws = torch.empty(pmg_workspace_bytes(desc), dtype=torch.uint8, device=device)
        self.info = torch.empty(desc.batch * INFO_BYTES, dtype=torch.uint8, device=device)
        self.coords = [None if c is None else c.contiguous() for c in coords]
        self.h = pmg_setup(desc, self.coords, self.ws, self.info)

    def __del__(self):
        h = getattr(self, "h", None)
        if h and pmg_destroy is not None:      # module globals go at interpreter exit
            pmg_destroy(h)
            self.h = None

    def info_host(self):
        return info_to_numpy(self.info)

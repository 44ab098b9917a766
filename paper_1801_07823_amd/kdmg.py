"""Thin ctypes binding of libkdmg (the C ABI declared in include/kdmg.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Device vectors are torch tensors (complex128 or complex64, on the
current HIP device); their data pointers and the current stream are passed
through unchanged.  If the library is missing this module raises at import:
there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("KDMG_LIB", os.path.join(HERE, "libkdmg.so"))

if not os.path.exists(LIB_PATH):
    raise ImportError("libkdmg.so not built: run __graft_entry__.build() (or "
                      "python paper_1801_07823_amd/build_lib.py) first")
_lib = ctypes.CDLL(LIB_PATH)

KDMG_OK, KDMG_EINVAL, KDMG_ENOMEM, KDMG_EHIP, KDMG_ENOCONV, KDMG_EBUSY, KDMG_EUNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6
KDMG_FP64, KDMG_MIXED = 0, 1


class kdmg_level_params(ctypes.Structure):
    _fields_ = [("agg", ctypes.c_int * 4), ("nvec", ctypes.c_int)]


class kdmg_mg_params(ctypes.Structure):
    _fields_ = [("nlevels", ctypes.c_int), ("lvl", kdmg_level_params * 3),
                ("setup_tol", ctypes.c_double), ("setup_maxit", ctypes.c_int),
                ("outer_restart", ctypes.c_int), ("outer_maxit", ctypes.c_int),
                ("mr_its", ctypes.c_int), ("mr_omega", ctypes.c_double),
                ("inter_restart", ctypes.c_int), ("inter_maxit", ctypes.c_int),
                ("inter_tol", ctypes.c_double), ("coarse_tol", ctypes.c_double),
                ("coarse_maxit", ctypes.c_int), ("outer_stall", ctypes.c_int),
                ("coarse_tail", ctypes.c_int), ("coarse_solver", ctypes.c_int), ("fine_op", ctypes.c_int),
                ("asymmetric", ctypes.c_int)]


class kdmg_solve_info(ctypes.Structure):
    _fields_ = [("converged", ctypes.c_int), ("outer_its", ctypes.c_int),
                ("fine_applies", ctypes.c_int), ("level_avg_its", ctypes.c_double * 3),
                ("true_rel_resid", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {"converged": bool(self.converged), "outer_its": self.outer_its,
                "fine_applies": self.fine_applies,
                "level_avg_its": list(self.level_avg_its),
                "true_rel_resid": self.true_rel_resid, "seconds": self.seconds}


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_S = ctypes.c_size_t

_SIGS = {
    "kdmg_default_params": (None, [ctypes.POINTER(kdmg_mg_params)]),
    "kdmg_init": (_I, [_I]),
    "kdmg_lattice_create": (_I, [_I, ctypes.POINTER(_I), _I, ctypes.POINTER(_I), _P, _P, ctypes.POINTER(_P)]),
    "kdmg_lattice_destroy": (None, [_P]),
    "kdmg_lattice_set_naik": (_I, [_P, _I, _P]),
    "kdmg_lattice_footprint": (_I, [_P, ctypes.POINTER(_S)]),
    "kdmg_apply_D": (_I, [_P, _D, _P, _P, _I, _I, _P]),
    "kdmg_apply_A": (_I, [_P, _D, _P, _P, _I, _I, _I, _P]),
    "kdmg_apply_Binv": (_I, [_P, _D, _P, _P, _I, _P]),
    "kdmg_apply_schur": (_I, [_P, _D, _P, _P, _I, _P]),
    "kdmg_apply_schur_noalloc": (_I, [_P, _D, _P, _P, _I, _P]),
    "kdmg_hierarchy_build": (_I, [_P, _D, ctypes.POINTER(kdmg_mg_params),
                                  ctypes.POINTER(_P), _I, _P, ctypes.POINTER(_P)]),
    "kdmg_hierarchy_destroy": (None, [_P]),
    "kdmg_hierarchy_level_info": (_I, [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "kdmg_hierarchy_get_nullvecs": (_I, [_P, _I, _P]),
    "kdmg_hierarchy_get_prolongator": (_I, [_P, _I, _P]),
    "kdmg_hierarchy_get_asym_transfer": (_I, [_P, _I, _P, _P]),
    "kdmg_hierarchy_get_coarse_op": (_I, [_P, _I, _P]),
    "kdmg_coarse_apply": (_I, [_P, _I, _I, _P, _P, _I, _I, _P]),
    "kdmg_restrict": (_I, [_P, _I, _P, _P, _I, _I, _P]),
    "kdmg_prolong": (_I, [_P, _I, _P, _P, _I, _I, _P]),
    "kdmg_solve": (_I, [_P, _P, _P, _I, _D, _I, ctypes.POINTER(kdmg_solve_info), _P]),
    "kdmg_hierarchy_footprint": (_I, [_P, _I, ctypes.POINTER(_S)]),
    "kdmg_hierarchy_autotune": (_I, [_P, _I, _I, _P]),
    "kdmg_coarse_apply_candidates": (_I, [_P, _I, _I, _P, _P, _I, _I, _I, ctypes.POINTER(_I), _P]),
    "kdmg_hierarchy_at_mass": (_I, [_P, _D, _P, ctypes.POINTER(_P)]),
    "kdmg_hierarchy_set_mass": (_I, [_P, _P, _D, _P]),
    "kdmg_hierarchy_graphs": (_I, [_P, _I, ctypes.POINTER(ctypes.c_longlong)]),
    "kdmg_hierarchy_counters": (_I, [_P, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong)]),
    "kdmg_solve_cg_eo": (_I, [_P, _D, _P, _P, _I, _D, _I, ctypes.POINTER(_I), _P]),
    "kdmg_coarsest_solve": (_I, [_P, _P, _P, _I, _P]),
    "kdmg_hierarchy_kernel_timing": (_I, [_P, _I, ctypes.POINTER(_D), ctypes.POINTER(ctypes.c_longlong)]),
    "kdmg_server_create": (_I, [_I, _S, ctypes.POINTER(_P)]),
    "kdmg_server_add_config": (_I, [_P, _P, ctypes.POINTER(_I)]),
    "kdmg_server_request_bytes": (_I, [_P, _I, _I, _I, ctypes.POINTER(_S)]),
    "kdmg_server_submit": (_I, [_P, _I, _D, _P, _P, _I, _D, _I, _P, ctypes.POINTER(ctypes.c_longlong)]),
    "kdmg_server_poll": (_I, [_P, ctypes.c_longlong, _I, ctypes.POINTER(_I), ctypes.POINTER(_I),
                              _P, ctypes.POINTER(_D)]),
    "kdmg_server_stats": (_I, [_P, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(_I),
                               ctypes.POINTER(_I), ctypes.POINTER(_S), ctypes.POINTER(_S)]),
    "kdmg_server_destroy": (None, [_P]),
    "kdmg_status_string": (ctypes.c_char_p, [_I]),
    "kdmg_last_error": (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = sorted(_SIGS)


class KdmgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (_lib.kdmg_status_string(status).decode(), status, msg))
        self.status = status


def _check(st):
    if st != KDMG_OK:
        raise KdmgError(st, (_lib.kdmg_last_error() or b"").decode())
    return st


def _stream(stream):
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def _ptr(t, prec, n, what):
    """Device pointer of tensor `t` after checking what the library will
    assume of it: a contiguous GPU tensor of the precision's complex dtype
    (complex128 for KDMG_FP64, complex64 for KDMG_MIXED) with at least `n`
    elements.  Raises KdmgError(KDMG_EINVAL) otherwise, before any call."""
    import torch
    want = torch.complex128 if prec == KDMG_FP64 else torch.complex64
    if not isinstance(t, torch.Tensor):
        raise KdmgError(KDMG_EINVAL, "%s: expected a torch tensor, got %s" % (what, type(t).__name__))
    if not t.is_cuda:
        raise KdmgError(KDMG_EINVAL, "%s: tensor must be on the GPU" % what)
    if t.dtype != want:
        raise KdmgError(KDMG_EINVAL, "%s: dtype %s, expected %s" % (what, t.dtype, want))
    if not t.is_contiguous():
        raise KdmgError(KDMG_EINVAL, "%s: tensor must be contiguous" % what)
    if t.numel() < n:
        raise KdmgError(KDMG_EINVAL, "%s: %d elements, the call needs %d" % (what, t.numel(), n))
    return ctypes.c_void_p(t.data_ptr())


def default_params():
    p = kdmg_mg_params()
    _lib.kdmg_default_params(ctypes.byref(p))
    return p


def make_params(levels, **kw):
    """levels: [(agg_tuple, nvec), ...] per coarsening; kw overrides Table 1 values."""
    p = default_params()
    p.nlevels = len(levels) + 1
    for k, (agg, nv) in enumerate(levels):
        a = list(agg) + [1] * (4 - len(agg))
        p.lvl[k].agg[:] = a
        p.lvl[k].nvec = nv
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def kdmg_init(device=0):
    _check(_lib.kdmg_init(device))


class Lattice:
    def __init__(self, dims, links, bc=None, stream=None):
        """bc: per-direction boundary signs (+1 periodic, -1 antiperiodic);
        None = periodic space, antiperiodic time."""
        links = np.ascontiguousarray(links, dtype=np.complex128)
        nd = len(dims)
        nc = links.shape[-1]
        self.dims = tuple(int(d) for d in dims)
        self.ncolor = nc
        self.volume = int(np.prod(dims))
        self.ndof = self.volume * nc
        if links.size != nd * self.volume * nc * nc:
            raise KdmgError(KDMG_EINVAL, "Lattice: links must hold [nd][volume][nc][nc] entries")
        self.bc = tuple(int(b) for b in bc) if bc is not None else tuple([1] * (nd - 1) + [-1])
        if len(self.bc) != nd:
            raise KdmgError(KDMG_EINVAL, "Lattice: one boundary sign per direction")
        arr = (_I * nd)(*self.dims)
        bca = (_I * nd)(*self.bc)
        h = _P()
        _check(_lib.kdmg_lattice_create(nd, arr, nc, bca, links.ctypes.data_as(_P), _stream(stream),
                                        ctypes.byref(h)))
        self.handle = h

    def set_naik(self, enable=True, stream=None):
        """kdmg_lattice_set_naik: switch to the Naik-improved operator (2D U(1))."""
        _check(_lib.kdmg_lattice_set_naik(self.handle, 1 if enable else 0, _stream(stream)))
        self.naik = bool(enable)

    def footprint(self):
        b = _S()
        _check(_lib.kdmg_lattice_footprint(self.handle, ctypes.byref(b)))
        return b.value

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.kdmg_lattice_destroy(self.handle)
            self.handle = None


def kdmg_apply_D(lat, mass, inp, out, nrhs, prec=KDMG_FP64, stream=None):
    n = nrhs * lat.ndof
    _check(_lib.kdmg_apply_D(lat.handle, mass, _ptr(inp, prec, n, "kdmg_apply_D in"),
                             _ptr(out, prec, n, "kdmg_apply_D out"), nrhs, prec, _stream(stream)))


def kdmg_apply_A(lat, mass, inp, out, nrhs, dagger=False, prec=KDMG_FP64, stream=None):
    n = nrhs * lat.ndof
    _check(_lib.kdmg_apply_A(lat.handle, mass, _ptr(inp, prec, n, "kdmg_apply_A in"),
                             _ptr(out, prec, n, "kdmg_apply_A out"), nrhs, 1 if dagger else 0, prec,
                             _stream(stream)))


def kdmg_apply_Binv(lat, mass, inp, out, nrhs, stream=None):
    n = nrhs * lat.ndof
    _check(_lib.kdmg_apply_Binv(lat.handle, mass, _ptr(inp, KDMG_FP64, n, "kdmg_apply_Binv in"),
                                _ptr(out, KDMG_FP64, n, "kdmg_apply_Binv out"), nrhs, _stream(stream)))


def kdmg_apply_schur(lat, mass, inp, out, nrhs, stream=None):
    n = nrhs * (lat.ndof // 2)
    _check(_lib.kdmg_apply_schur(lat.handle, mass, _ptr(inp, KDMG_FP64, n, "kdmg_apply_schur in"),
                                 _ptr(out, KDMG_FP64, n, "kdmg_apply_schur out"), nrhs, _stream(stream)))


def kdmg_apply_schur_noalloc(lat, mass, inp, out, nrhs, stream=None):
    """kdmg_apply_schur with the library's fixed work space (no allocation)."""
    n = nrhs * (lat.ndof // 2)
    _check(_lib.kdmg_apply_schur_noalloc(lat.handle, mass, _ptr(inp, KDMG_FP64, n, "kdmg_apply_schur_noalloc in"),
                                         _ptr(out, KDMG_FP64, n, "kdmg_apply_schur_noalloc out"), nrhs,
                                         _stream(stream)))


class Hierarchy:
    def __init__(self, lat, mass, params, psi0, relaxed=False, stream=None):
        """psi0: list of complex128 numpy arrays [nvec, ndof_k] per coarsening."""
        self.lat = lat
        self.params = params
        self.mass = mass
        self._psi0 = [np.ascontiguousarray(v, dtype=np.complex128) for v in psi0]
        ptrs = (_P * len(self._psi0))(*[v.ctypes.data_as(_P) for v in self._psi0])
        h = _P()
        _check(_lib.kdmg_hierarchy_build(lat.handle, mass, ctypes.byref(params), ptrs,
                                         1 if relaxed else 0, _stream(stream), ctypes.byref(h)))
        self.handle = h
        self.nlevels = params.nlevels

    @classmethod
    def _wrap(cls, handle, lat, params, mass):
        self = cls.__new__(cls)
        self.lat, self.params, self.mass = lat, params, mass
        self.handle = handle
        self.nlevels = params.nlevels
        return self

    def at_mass(self, mass, stream=None):
        """kdmg_hierarchy_at_mass: same null vectors and P, coarse operators at `mass`."""
        h = _P()
        _check(_lib.kdmg_hierarchy_at_mass(self.handle, mass, _stream(stream), ctypes.byref(h)))
        return Hierarchy._wrap(h, self.lat, self.params, mass)

    def set_mass(self, mass, base=None, stream=None):
        """kdmg_hierarchy_set_mass: rebuild in place (optionally onto `base`)."""
        _check(_lib.kdmg_hierarchy_set_mass(self.handle, base.handle if base is not None else None,
                                            mass, _stream(stream)))
        if base is not None:
            self.lat = base.lat
        self.mass = mass

    def level_info(self, level):
        dims = (_I * 4)()
        nd = _I()
        _check(_lib.kdmg_hierarchy_level_info(self.handle, level, dims, ctypes.byref(nd)))
        return tuple(dims[:len(self.lat.dims)]), nd.value

    def ndof(self, level):
        if level == 0:
            return self.lat.volume * self.lat.ncolor
        dims, nd = self.level_info(level)
        return int(np.prod(dims)) * nd

    def nullvecs(self, k):
        nv = self.params.lvl[k].nvec
        out = np.zeros((nv, self.ndof(k)), dtype=np.complex128)
        _check(_lib.kdmg_hierarchy_get_nullvecs(self.handle, k, out.ctypes.data_as(_P)))
        return out

    def prolongator_values(self, k):
        nv = self.params.lvl[k].nvec
        out = np.zeros((self.ndof(k), nv), dtype=np.complex128)
        _check(_lib.kdmg_hierarchy_get_prolongator(self.handle, k, out.ctypes.data_as(_P)))
        return out

    def asym_transfer(self, k=0):
        """Asymmetric coarsening: (P, R^T) on the aggregates, each [ndof_0][2 nvec]."""
        nd = 2 * self.params.lvl[k].nvec
        p = np.zeros((self.ndof(k), nd), dtype=np.complex128)
        r = np.zeros((self.ndof(k), nd), dtype=np.complex128)
        _check(_lib.kdmg_hierarchy_get_asym_transfer(self.handle, k, p.ctypes.data_as(_P), r.ctypes.data_as(_P)))
        return p, r

    def coarse_op(self, level):
        dims, nd = self.level_info(level)
        ndir = 2 * len(dims) + 1
        out = np.zeros((ndir, int(np.prod(dims)), nd, nd), dtype=np.complex128)
        _check(_lib.kdmg_hierarchy_get_coarse_op(self.handle, level, out.ctypes.data_as(_P)))
        return out

    def graphs(self, enable=None):
        """kdmg_hierarchy_graphs: replay captured coarsest-CGNE chunks (default) or
        not; returns the number of chunk replays so far."""
        n = ctypes.c_longlong()
        _check(_lib.kdmg_hierarchy_graphs(self.handle, -1 if enable is None else (1 if enable else 0),
                                          ctypes.byref(n)))
        return n.value

    def counters(self):
        """kdmg_hierarchy_counters: {"graph_replays": ..., "tail_entries": ...} so far."""
        g, t = ctypes.c_longlong(), ctypes.c_longlong()
        _check(_lib.kdmg_hierarchy_counters(self.handle, ctypes.byref(g), ctypes.byref(t)))
        return {"graph_replays": g.value, "tail_entries": t.value}

    def footprint(self, nrhs=1):
        b = _S()
        _check(_lib.kdmg_hierarchy_footprint(self.handle, nrhs, ctypes.byref(b)))
        return b.value

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.kdmg_hierarchy_destroy(self.handle)
            self.handle = None


def _level_ndof(h, level):
    if not 0 <= level < h.nlevels:
        raise KdmgError(KDMG_EINVAL, "no level %d in a %d-level hierarchy" % (level, h.nlevels))
    return h.ndof(level)


def kdmg_coarse_apply(h, level, inp, out, nrhs, dagger=False, prec=KDMG_FP64, stream=None):
    n = nrhs * _level_ndof(h, level)
    _check(_lib.kdmg_coarse_apply(h.handle, level, 1 if dagger else 0, _ptr(inp, prec, n, "kdmg_coarse_apply in"),
                                  _ptr(out, prec, n, "kdmg_coarse_apply out"), nrhs, prec, _stream(stream)))


def kdmg_coarse_apply_candidates(h, level, inp, out, nrhs, dagger=False, prec=KDMG_FP64, stream=None):
    """Every tuner candidate's stencil apply: out[c] for c < out.shape[0]; returns the candidate count."""
    n = nrhs * _level_ndof(h, level)
    nc = _I()
    _check(_lib.kdmg_coarse_apply_candidates(h.handle, level, 1 if dagger else 0,
                                             _ptr(inp, prec, n, "candidates in"),
                                             _ptr(out, prec, n * out.shape[0], "candidates out"), nrhs, prec,
                                             out.shape[0], ctypes.byref(nc), _stream(stream)))
    return nc.value


def kdmg_restrict(h, k, inp, out, nrhs, prec=KDMG_FP64, stream=None):
    nf, nc = nrhs * _level_ndof(h, k), nrhs * _level_ndof(h, k + 1)
    _check(_lib.kdmg_restrict(h.handle, k, _ptr(inp, prec, nf, "kdmg_restrict in"),
                              _ptr(out, prec, nc, "kdmg_restrict out"), nrhs, prec, _stream(stream)))


def kdmg_prolong(h, k, inp, out, nrhs, prec=KDMG_FP64, stream=None):
    nf, nc = nrhs * _level_ndof(h, k), nrhs * _level_ndof(h, k + 1)
    _check(_lib.kdmg_prolong(h.handle, k, _ptr(inp, prec, nc, "kdmg_prolong in"),
                             _ptr(out, prec, nf, "kdmg_prolong out"), nrhs, prec, _stream(stream)))


def kdmg_coarsest_solve(h, inp, out, nrhs, stream=None):
    """Exact coarsest solve (hierarchies built with coarse_solver=1): out = A_c^-1 in."""
    n = nrhs * _level_ndof(h, h.nlevels - 1)
    _check(_lib.kdmg_coarsest_solve(h.handle, _ptr(inp, KDMG_FP64, n, "kdmg_coarsest_solve in"),
                                    _ptr(out, KDMG_FP64, n, "kdmg_coarsest_solve out"), nrhs, _stream(stream)))


def kdmg_hierarchy_autotune(h, nrhs, prec=KDMG_FP64, stream=None):
    _check(_lib.kdmg_hierarchy_autotune(h.handle, nrhs, prec, _stream(stream)))


def kdmg_hierarchy_kernel_timing(h, enable=-1):
    """enable: 1 start (zeroes the counters), 0 stop, -1 read only -> (ms, launches)."""
    ms = _D()
    n = ctypes.c_longlong()
    _check(_lib.kdmg_hierarchy_kernel_timing(h.handle, enable, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def kdmg_solve(h, b, x, nrhs, tol=1e-10, prec=KDMG_FP64, stream=None, raise_on_noconv=True):
    info = (kdmg_solve_info * nrhs)()
    n = nrhs * h.lat.ndof
    st = _lib.kdmg_solve(h.handle, _ptr(b, KDMG_FP64, n, "kdmg_solve b"), _ptr(x, KDMG_FP64, n, "kdmg_solve x"),
                         nrhs, tol, prec, info, _stream(stream))
    if st != KDMG_OK and (st != KDMG_ENOCONV or raise_on_noconv):
        _check(st)
    return [i.as_dict() for i in info], st


def kdmg_solve_cg_eo(lat, mass, b, x, nrhs, tol=1e-10, maxit=200000, stream=None, raise_on_noconv=True):
    """CG on the site even/odd Schur system (2D, FP64); returns the iteration count per rhs."""
    its = (_I * nrhs)()
    n = nrhs * lat.ndof
    st = _lib.kdmg_solve_cg_eo(lat.handle, mass, _ptr(b, KDMG_FP64, n, "kdmg_solve_cg_eo b"),
                               _ptr(x, KDMG_FP64, n, "kdmg_solve_cg_eo x"), nrhs, tol, maxit, its,
                               _stream(stream))
    if st != KDMG_OK and (st != KDMG_ENOCONV or raise_on_noconv):
        _check(st)
    return list(its)


class Server:
    """kdmg_server_*: continuous-batching solve service over resident configurations.

    Keeps the caller's b / x tensors alive until their request is collected."""

    def __init__(self, slots, hbm_budget):
        h = _P()
        _check(_lib.kdmg_server_create(slots, hbm_budget, ctypes.byref(h)))
        self.handle = h
        self._configs = []
        self._live = {}
        self.last_error = ""

    def add_config(self, hierarchy):
        cid = _I()
        _check(_lib.kdmg_server_add_config(self.handle, hierarchy.handle, ctypes.byref(cid)))
        self._configs.append(hierarchy)
        return cid.value

    def request_bytes(self, config_id, nrhs=1, prec=KDMG_MIXED):
        b = _S()
        _check(_lib.kdmg_server_request_bytes(self.handle, config_id, nrhs, prec, ctypes.byref(b)))
        return b.value

    def submit(self, config_id, mass, b, x, nrhs=1, tol=1e-10, prec=KDMG_MIXED, stream=None):
        """Queue a solve; device work queued on `stream` (default: torch's current
        stream) before the call is complete before the request reads b or writes x."""
        if not 0 <= config_id < len(self._configs):
            raise KdmgError(KDMG_EINVAL, "Server.submit: no configuration %d" % config_id)
        n = nrhs * self._configs[config_id].lat.ndof
        t = ctypes.c_longlong()
        _check(_lib.kdmg_server_submit(self.handle, config_id, mass, _ptr(b, KDMG_FP64, n, "submit b"),
                                       _ptr(x, KDMG_FP64, n, "submit x"), nrhs, tol, prec, _stream(stream),
                                       ctypes.byref(t)))
        self._live[t.value] = (b, x, nrhs)
        return t.value

    def poll(self, ticket, wait=False):
        """None while running, else (status, [info dicts], (queued_s, run_s, total_s))."""
        nrhs = self._live[ticket][2]
        done, st = _I(), _I()
        info = (kdmg_solve_info * nrhs)()
        times = (_D * 3)()
        _check(_lib.kdmg_server_poll(self.handle, ticket, 1 if wait else 0, ctypes.byref(done),
                                     ctypes.byref(st), ctypes.cast(info, _P), times))
        if not done.value:
            return None
        del self._live[ticket]
        self.last_error = (_lib.kdmg_last_error() or b"").decode() if st.value != KDMG_OK else ""
        return st.value, [i.as_dict() for i in info], tuple(times)

    def stats(self):
        c, r, pr = ctypes.c_longlong(), _I(), _I()
        a, pa = _S(), _S()
        _check(_lib.kdmg_server_stats(self.handle, ctypes.byref(c), ctypes.byref(r), ctypes.byref(pr),
                                      ctypes.byref(a), ctypes.byref(pa)))
        return {"completed": c.value, "running": r.value, "peak_running": pr.value,
                "allocated": a.value, "peak_allocated": pa.value}

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.kdmg_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()

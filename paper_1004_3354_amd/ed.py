"""Thin ctypes binding of the HIP C-ABI library ``libedhip.so`` (include/ed.h).

Argument marshalling only: every step of the computation runs in the library's
kernels.  Device vectors are torch tensors on the GPU (torch supplies memory and
streams); small outputs come back as Python / numpy values.  Importing this
module raises if the compiled library is missing -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libedhip.so")

if not os.path.exists(LIBPATH):
    raise ImportError("libedhip.so is not built (run __graft_entry__.build()); "
                      "there is no CPU fallback for the HIP path")

# torch supplies the device memory and streams and ships its own HIP runtime
# (same soname as the system one the library links): loading torch first makes
# the library bind to that runtime instead of loading a second one
try:
    import torch  # noqa: F401
except ImportError:
    pass

_lib = ctypes.CDLL(LIBPATH)

ED_OK, ED_EINVAL, ED_ENOMEM, ED_EDEVICE, ED_ENOCONV, ED_EUNSUPPORTED = range(6)
ED_FP64, ED_FP32 = 0, 1
SPIN_FLIP, PAIR_HOP = 1, 2
_STATUS = {1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ENOCONV", 5: "EUNSUPPORTED"}

_p = ctypes.c_void_p
_i64 = ctypes.c_int64


class EDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_STATUS.get(status, str(status)), msg))
        self.status = status


class ed_xterm(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("m", ctypes.c_int32), ("mp", ctypes.c_int32),
                ("coef", ctypes.c_double), ("k", ctypes.c_int32), ("l", ctypes.c_int32)]


class ed_params(ctypes.Structure):
    _fields_ = [("Ns", ctypes.c_int32), ("eps", _p), ("hop", _p), ("w_ud", _p), ("w_ss", _p),
                ("n_x", ctypes.c_int32), ("x", _p)]


class ed_lanczos_opts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("max_basis", ctypes.c_int32), ("tol", ctypes.c_double),
                ("reorth", ctypes.c_int32), ("check_every", ctypes.c_int32), ("refine", ctypes.c_int32),
                ("keep", ctypes.c_int32), ("layout", ctypes.c_int32)]


class ed_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("restarts", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("basis_used", ctypes.c_int32), ("residual", ctypes.c_double), ("ritz", ctypes.c_double),
                ("rq_fp64", ctypes.c_double), ("gap_lower", ctypes.c_double), ("e_lower", ctypes.c_double),
                ("traffic", ctypes.c_double)]

    def as_dict(self) -> Dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("ed_version", ctypes.c_char_p, [])
_sig("ed_last_error", ctypes.c_char_p, [])
_sig("ed_basis", ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_p)])
_sig("ed_basis_dims", ctypes.c_int, [_p, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64)])
_sig("ed_basis_states", ctypes.c_int, [_p, ctypes.c_int, _p])
_sig("ed_basis_rank", ctypes.c_int, [_p, ctypes.c_int, _p, _i64, _p, _p])
_sig("ed_basis_free", None, [_p])
_sig("ed_ham_create", ctypes.c_int, [ctypes.POINTER(ed_params), _p, ctypes.c_int, ctypes.POINTER(_p)])
_sig("ed_ham_dims", ctypes.c_int, [_p, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64)])
_sig("ed_hop_table_size", ctypes.c_int, [_p, ctypes.c_int, ctypes.POINTER(_i64)])
_sig("ed_hop_table", ctypes.c_int, [_p, ctypes.c_int, _p, _p, _p, _p])
_sig("ed_apply_H", ctypes.c_int, [_p, _p, _p, _p])
_sig("ed_apply_variant_count", ctypes.c_int, [])
_sig("ed_apply_variant_name", ctypes.c_char_p, [ctypes.c_int])
_sig("ed_apply_variant_fits", ctypes.c_int, [_p, ctypes.c_int])
_sig("ed_apply_current_variant", ctypes.c_int, [_p])
_sig("ed_apply_H_variant", ctypes.c_int, [_p, ctypes.c_int, _p, _p, _p])
_sig("ed_rayleigh", ctypes.c_int, [_p, _p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), _p])
_sig("ed_fill_random", ctypes.c_int, [_p, _i64, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, _p])
_sig("ed_rayleigh_noalloc", ctypes.c_int, [_p, _p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                           _p])
_sig("ed_ham_free", None, [_p])
_sig("ed_ham_grouped", ctypes.c_int, [_p, ctypes.POINTER(_p)])
_sig("ed_grouped_order", ctypes.c_int, [_p, ctypes.c_int, _p])
_sig("ed_to_grouped", ctypes.c_int, [_p, _p, _p, _p])
_sig("ed_from_grouped", ctypes.c_int, [_p, _p, _p, _p])
_sig("ed_lanczos_defaults", None, [ctypes.POINTER(ed_lanczos_opts)])
_sig("ed_workspace_bytes", ctypes.c_int, [_p, ctypes.POINTER(ed_lanczos_opts), ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_size_t)])
_sig("ed_lanczos_ground", ctypes.c_int, [_p, ctypes.POINTER(ed_lanczos_opts), _p, _p, ctypes.c_size_t,
                                         ctypes.POINTER(ctypes.c_double), _p, ctypes.POINTER(ed_info), _p])
_sig("ed_arnoldi_lowest", ctypes.c_int, [_p, ctypes.c_int, ctypes.POINTER(ed_lanczos_opts), _p, _p,
                                         ctypes.c_size_t, _p, _p, _p, _p])
_sig("ed_arnoldi_lowest_more", ctypes.c_int, [_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ed_lanczos_opts), _p,
                                              _p, ctypes.c_size_t, _p, _p, _p, _p])
_sig("ed_tridiag_workspace_bytes", ctypes.c_int, [_p, ctypes.POINTER(ed_lanczos_opts), ctypes.c_int,
                                                  ctypes.POINTER(ctypes.c_size_t)])
_sig("ed_lanczos_tridiag", ctypes.c_int, [_p, ctypes.POINTER(ed_lanczos_opts), _p, ctypes.c_int, _p, ctypes.c_size_t,
                                          _p, _p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double), _p])
_sig("ed_apply_ladder", ctypes.c_int, [_p, _p, ctypes.c_int, ctypes.c_int, ctypes.c_int, _p, _p, _p])
_sig("ed_green_cf", ctypes.c_int, [_p, _p, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                   ctypes.c_double, _p, _p, ctypes.c_int, _p, _p])
_sig("ed_boltzmann_weights", ctypes.c_int, [_p, ctypes.c_int, ctypes.c_double, ctypes.c_double, _p,
                                            ctypes.POINTER(ctypes.c_int)])
_sig("ed_lowest_levels", ctypes.c_int, [ctypes.c_int, _p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ed_lanczos_opts),
                                        ctypes.c_uint64, ctypes.POINTER(_p), _p])
_sig("ed_levels_info", ctypes.c_int, [_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)])
_sig("ed_levels_get", ctypes.c_int, [_p, _p, _p, _p])
_sig("ed_levels_capped", ctypes.c_int, [_p, _p])
_sig("ed_levels_vector", ctypes.c_int, [_p, ctypes.c_int, ctypes.c_int, _p, _p])
_sig("ed_levels_free", None, [_p])
if hasattr(_lib, "ed_lanczos_ground_batched"):
    _sig("ed_batched_workspace_bytes", ctypes.c_int, [ctypes.c_int, _p, ctypes.POINTER(ed_lanczos_opts),
                                                      ctypes.POINTER(ctypes.c_size_t)])
    _sig("ed_lanczos_ground_batched", ctypes.c_int, [ctypes.c_int, _p, ctypes.POINTER(ed_lanczos_opts), _p,
                                                     ctypes.c_uint64, _p, ctypes.c_size_t, _p, _p, _p])
    _sig("ed_batched_last_tile", ctypes.c_int64, [])
    _sig("ed_batched_last_stats", None, [ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_double)])


def _check(st: int, ok=(ED_OK,)):
    if st not in ok:
        raise EDError(st, _lib.ed_last_error().decode())
    return st


def version() -> str:
    return _lib.ed_version().decode()


def _stream(stream) -> Optional[int]:
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def _dev_ptr(t) -> int:
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous GPU tensor")
    return t.data_ptr()


def options(max_iter=None, max_basis=None, tol=None, reorth=None, check_every=None, refine=None, keep=None,
            layout=None):
    o = ed_lanczos_opts()
    _lib.ed_lanczos_defaults(ctypes.byref(o))
    for k, v in (("max_iter", max_iter), ("max_basis", max_basis), ("tol", tol), ("reorth", reorth),
                 ("check_every", check_every), ("refine", refine), ("keep", keep), ("layout", layout)):
        if v is not None:
            setattr(o, k, v)
    return o


class Basis:
    """The (N_up, N_dn) sector basis (combinatorial ranking on the GPU)."""

    def __init__(self, ns: int, nup: int, ndn: int):
        h = _p()
        _check(_lib.ed_basis(ns, nup, ndn, ctypes.byref(h)))
        self._h = h
        self.ns, self.nup, self.ndn = ns, nup, ndn
        a, b, c = _i64(), _i64(), _i64()
        _check(_lib.ed_basis_dims(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        self.dup, self.ddn, self.D = a.value, b.value, c.value

    def states(self, spin: int) -> np.ndarray:
        out = np.empty(self.dup if spin == 0 else self.ddn, dtype=np.uint32)
        _check(_lib.ed_basis_states(self._h, spin, out.ctypes.data_as(_p)))
        return out

    def rank(self, spin: int, states_dev, ranks_dev, stream=None):
        _check(_lib.ed_basis_rank(self._h, spin, _dev_ptr(states_dev), states_dev.numel(),
                                  _dev_ptr(ranks_dev), _stream(stream)))

    def close(self):
        if self._h:
            _lib.ed_basis_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_params(p: Dict):
    """Marshal a coefficient dict (see models.py) into an ed_params struct.
    Returns (struct, keepalive)."""
    ns = int(p["Ns"])
    arrs = [np.ascontiguousarray(np.asarray(p[k], dtype=np.float64)) for k in ("eps", "hop", "w_ud", "w_ss")]
    xt = p.get("xterms", [])
    xa = (ed_xterm * max(len(xt), 1))()
    for i, x in enumerate(xt):
        if len(x) == 6:      # (ED_UD_GENERAL, i, j, k, l, coef)
            t, m, mp, k, l, c = x
        else:                # (type, m, m', coef)
            (t, m, mp, c), k, l = x, 0, 0
        xa[i] = ed_xterm(int(t), int(m), int(mp), float(c), int(k), int(l))
    s = ed_params(ns, arrs[0].ctypes.data_as(_p), arrs[1].ctypes.data_as(_p), arrs[2].ctypes.data_as(_p),
                  arrs[3].ctypes.data_as(_p), len(xt), ctypes.cast(xa, _p) if xt else None)
    return s, (arrs, xa)


class Hamiltonian:
    """Per-spin tables of H for one sector, ready for the matrix-free apply."""

    def __init__(self, params: Dict, basis: Basis, precision: int = ED_FP64):
        s, keep = make_params(params)
        h = _p()
        _check(_lib.ed_ham_create(ctypes.byref(s), basis._h, precision, ctypes.byref(h)))
        self._h = h
        self.precision = precision
        self.dup, self.ddn, self.D = basis.dup, basis.ddn, basis.D

    @property
    def torch_dtype(self):
        import torch
        return torch.float64 if self.precision == ED_FP64 else torch.float32

    def hop_table(self, spin: int) -> Tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
        n = _i64()
        _check(_lib.ed_hop_table_size(self._h, spin, ctypes.byref(n)))
        dim = self.dup if spin == 0 else self.ddn
        off = np.empty(dim + 1, dtype=np.int64)
        tgt = np.empty(max(n.value, 1), dtype=np.int32)
        sgn = np.empty(max(n.value, 1), dtype=np.int8)
        amp = np.empty(max(n.value, 1), dtype=np.float64)
        _check(_lib.ed_hop_table(self._h, spin, off.ctypes.data_as(_p), tgt.ctypes.data_as(_p),
                                 sgn.ctypes.data_as(_p), amp.ctypes.data_as(_p)))
        k = n.value
        return off, tgt[:k], sgn[:k], amp[:k]

    def apply(self, x, y, stream=None):
        _check(_lib.ed_apply_H(self._h, _dev_ptr(x), _dev_ptr(y), _stream(stream)))

    def apply_variant(self, variant: int, x, y, stream=None):
        _check(_lib.ed_apply_H_variant(self._h, variant, _dev_ptr(x), _dev_ptr(y), _stream(stream)))

    def variant_fits(self, v: int) -> bool:
        return bool(_lib.ed_apply_variant_fits(self._h, v))

    def current_variant(self) -> int:
        return _lib.ed_apply_current_variant(self._h)

    def rayleigh(self, x, stream=None) -> Tuple[float, float]:
        rq, rs = ctypes.c_double(), ctypes.c_double()
        _check(_lib.ed_rayleigh(self._h, _dev_ptr(x), ctypes.byref(rq), ctypes.byref(rs), _stream(stream)))
        return rq.value, rs.value

    def rayleigh_noalloc(self, x, stream=None) -> Tuple[float, float]:
        rq, rs = ctypes.c_double(), ctypes.c_double()
        _check(_lib.ed_rayleigh_noalloc(self._h, _dev_ptr(x), ctypes.byref(rq), ctypes.byref(rs), _stream(stream)))
        return rq.value, rs.value

    def workspace_bytes(self, opts=None, k: int = 1) -> int:
        o = opts if opts is not None else options()
        if o.max_basis == 0:   # planned from free device memory: hand torch's cached blocks back first
            import torch
            torch.cuda.empty_cache()
        n = ctypes.c_size_t()
        _check(_lib.ed_workspace_bytes(self._h, ctypes.byref(o), k, ctypes.byref(n)))
        return n.value

    def tridiag_workspace_bytes(self, m: int, opts=None) -> int:
        o = opts if opts is not None else options()
        n = ctypes.c_size_t()
        _check(_lib.ed_tridiag_workspace_bytes(self._h, ctypes.byref(o), m, ctypes.byref(n)))
        return n.value

    def lanczos_ground(self, v0, opts=None, ws=None, psi=None, stream=None, allow_noconv=False):
        import torch
        o = opts if opts is not None else options()
        nb = self.workspace_bytes(o, 1)
        if ws is None:
            ws = torch.empty(nb, dtype=torch.uint8, device=v0.device)
        e = ctypes.c_double()
        inf = ed_info()
        st = _lib.ed_lanczos_ground(self._h, ctypes.byref(o), _dev_ptr(v0), _dev_ptr(ws), ws.numel(),
                                    ctypes.byref(e), _dev_ptr(psi) if psi is not None else None,
                                    ctypes.byref(inf), _stream(stream))
        _check(st, (ED_OK, ED_ENOCONV) if allow_noconv else (ED_OK,))
        return e.value, inf.as_dict()

    def lowest(self, k: int, v0, opts=None, ws=None, evecs=None, stream=None, allow_noconv=False):
        import torch
        o = opts if opts is not None else options()
        nb = self.workspace_bytes(o, k)
        if ws is None:
            ws = torch.empty(nb, dtype=torch.uint8, device=v0.device)
        ev = np.zeros(k, dtype=np.float64)
        infos = (ed_info * k)()
        st = _lib.ed_arnoldi_lowest(self._h, k, ctypes.byref(o), _dev_ptr(v0), _dev_ptr(ws), ws.numel(),
                                    ev.ctypes.data_as(_p), _dev_ptr(evecs) if evecs is not None else None,
                                    ctypes.cast(infos, _p), _stream(stream))
        _check(st, (ED_OK, ED_ENOCONV) if allow_noconv else (ED_OK,))
        return ev, [i.as_dict() for i in infos]

    def lowest_more(self, k0: int, k: int, evals0, v0, evecs, opts=None, ws=None, stream=None, allow_noconv=False):
        """Levels k0..k-1 on top of the k0 converged ones in evecs[:k0] (values
        evals0); evecs: DEVICE [k, D].  Returns (evals[k], infos[k0..k))."""
        import torch
        o = opts if opts is not None else options()
        nb = self.workspace_bytes(o, k)
        if ws is None:
            ws = torch.empty(nb, dtype=torch.uint8, device=v0.device)
        ev = np.zeros(k, dtype=np.float64)
        ev[:k0] = np.asarray(evals0, dtype=np.float64)[:k0]
        infos = (ed_info * k)()
        st = _lib.ed_arnoldi_lowest_more(self._h, k0, k, ctypes.byref(o), _dev_ptr(v0), _dev_ptr(ws), ws.numel(),
                                         ev.ctypes.data_as(_p), _dev_ptr(evecs), ctypes.cast(infos, _p),
                                         _stream(stream))
        _check(st, (ED_OK, ED_ENOCONV) if allow_noconv else (ED_OK,))
        return ev, [i.as_dict() for i in infos][k0:]

    def lanczos_tridiag(self, v0, m: int, opts=None, ws=None, stream=None):
        """(alpha, beta, ||v0||^2): k <= m tridiagonal Lanczos coefficients from v0."""
        import torch
        o = options() if opts is None else opts
        nb = self.tridiag_workspace_bytes(m, o)
        if ws is None:
            ws = torch.empty(nb, dtype=torch.uint8, device=v0.device)
        a = np.zeros(m, dtype=np.float64)
        b = np.zeros(m, dtype=np.float64)
        k = ctypes.c_int()
        n2 = ctypes.c_double()
        _check(_lib.ed_lanczos_tridiag(self._h, ctypes.byref(o), _dev_ptr(v0), m, _dev_ptr(ws), ws.numel(),
                                       a.ctypes.data_as(_p), b.ctypes.data_as(_p), ctypes.byref(k), ctypes.byref(n2),
                                       _stream(stream)))
        return a[:k.value].copy(), b[:k.value].copy(), n2.value

    def grouped(self) -> Optional["Hamiltonian"]:
        """The same operator in the grouped basis order (a borrowed twin handle
        that lives as long as this one), or None when there is none."""
        g = _p()
        _check(_lib.ed_ham_grouped(self._h, ctypes.byref(g)))
        if not g.value:
            return None
        if g.value == self._h.value:
            return self
        t = Hamiltonian.__new__(Hamiltonian)
        t._h, t._owner, t._borrowed = g, self, True
        t.precision, t.dup, t.ddn, t.D = self.precision, self.dup, self.ddn, self.D
        return t

    def grouped_order(self, spin: int) -> np.ndarray:
        """rank_of_position[p] of this (twin) handle's grouped order."""
        out = np.empty(self.dup if spin == 0 else self.ddn, dtype=np.int32)
        _check(_lib.ed_grouped_order(self._h, spin, out.ctypes.data_as(_p)))
        return out

    def to_grouped(self, x, y, stream=None):
        _check(_lib.ed_to_grouped(self._h, _dev_ptr(x), _dev_ptr(y), _stream(stream)))

    def from_grouped(self, x, y, stream=None):
        _check(_lib.ed_from_grouped(self._h, _dev_ptr(x), _dev_ptr(y), _stream(stream)))

    def close(self):
        if self._h and not getattr(self, "_borrowed", False):
            _lib.ed_ham_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fill_random(x, seed: int, dist: int = 0, stream=None):
    """SplitMix64 stream `seed`: dist 0 uniform [-1,1), 1 standard normal."""
    import torch
    prec = ED_FP64 if x.dtype == torch.float64 else ED_FP32
    _check(_lib.ed_fill_random(_dev_ptr(x), x.numel(), seed & 0xFFFFFFFFFFFFFFFF, dist, prec, _stream(stream)))


def variant_count() -> int:
    return _lib.ed_apply_variant_count()


def variant_name(v: int) -> str:
    return _lib.ed_apply_variant_name(v).decode()


def lanczos_ground_batched(hams: Sequence[Hamiltonian], opts=None, seed: int = 0, v0s=None, ws=None,
                           stream=None, allow_noconv=False):
    import torch
    if not hasattr(_lib, "ed_lanczos_ground_batched"):
        raise EDError(ED_EUNSUPPORTED, "the library has no batched Lanczos entry point")
    o = opts if opts is not None else options()
    n = len(hams)
    hs = (_p * n)(*[h._h for h in hams])
    nb = ctypes.c_size_t()
    _check(_lib.ed_batched_workspace_bytes(n, ctypes.cast(hs, _p), ctypes.byref(o), ctypes.byref(nb)))
    if ws is None:
        ws = torch.empty(max(nb.value, 1), dtype=torch.uint8, device="cuda")
    vp = None
    if v0s is not None:
        vp = (_p * n)(*[_dev_ptr(v) for v in v0s])
    E = np.zeros(n, dtype=np.float64)
    infos = (ed_info * n)()
    st = _lib.ed_lanczos_ground_batched(n, ctypes.cast(hs, _p), ctypes.byref(o),
                                        ctypes.cast(vp, _p) if vp is not None else None,
                                        seed & 0xFFFFFFFFFFFFFFFF, _dev_ptr(ws), ws.numel(),
                                        E.ctypes.data_as(_p), ctypes.cast(infos, _p), _stream(stream))
    _check(st, (ED_OK, ED_ENOCONV) if allow_noconv else (ED_OK,))
    return E, [i.as_dict() for i in infos]


def batched_last_stats():
    """Figures of the last batched run in this process: graph-replayed steps,
    restart events, apply tile size and algorithmic bytes moved (x read and y
    written per step, the projection window read twice and Y read twice and
    written once per pass, and every restart's inputs and outputs)."""
    steps, ev, nb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
    _lib.ed_batched_last_stats(ctypes.byref(steps), ctypes.byref(ev), ctypes.byref(nb))
    return {"steps": steps.value, "restart_events": ev.value, "tile": int(_lib.ed_batched_last_tile()),
            "bytes": nb.value}


def apply_ladder(src: "Hamiltonian", dst: "Hamiltonian", spin: int, site: int, dagger: bool, x, y, stream=None):
    """y = c+_{site,spin} x (dagger) or c_{site,spin} x, from sector src to sector dst."""
    _check(_lib.ed_apply_ladder(src._h, dst._h, int(spin), int(site), 1 if dagger else 0, _dev_ptr(x), _dev_ptr(y),
                                _stream(stream)))


def green_cf(alpha, beta, norm2: float, e0: float, sign: int, z, weight: float = 1.0, g=None):
    """weight * norm2 / (z - sign (alpha_0 - e0) - beta_0^2 / (...)) at complex z,
    added to g when given (complex128 array of len(z)), else returned."""
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    z = np.atleast_1d(np.asarray(z, dtype=np.complex128))
    zr, zi = np.ascontiguousarray(z.real), np.ascontiguousarray(z.imag)
    gr = np.ascontiguousarray(g.real) if g is not None else np.zeros(len(z))
    gi = np.ascontiguousarray(g.imag) if g is not None else np.zeros(len(z))
    _check(_lib.ed_green_cf(a.ctypes.data_as(_p), b.ctypes.data_as(_p), len(a), float(norm2), float(e0), int(sign),
                            float(weight), zr.ctypes.data_as(_p), zi.ctypes.data_as(_p), len(z), gr.ctypes.data_as(_p),
                            gi.ctypes.data_as(_p)))
    out = gr + 1j * gi
    if g is not None:
        g[:] = out
    return out


def boltzmann_weights(E, beta: float, cutoff: float = 0.0):
    """(w, kept): normalised Boltzmann weights of the levels E, levels whose share
    is below cutoff dropped (w = 0) and the rest renormalised."""
    e = np.ascontiguousarray(E, dtype=np.float64)
    w = np.zeros(len(e))
    kept = ctypes.c_int()
    _check(_lib.ed_boltzmann_weights(e.ctypes.data_as(_p), len(e), float(beta), float(cutoff), w.ctypes.data_as(_p),
                                     ctypes.byref(kept)))
    return w, kept.value


def green_function(H0: "Hamiltonian", e0: float, psi0, Hp: "Hamiltonian", Hm: "Hamiltonian", spin: int, site: int,
                   z, m: int = 200, opts=None, weight: float = 1.0, g=None, ws=None):
    """Impurity Green function of Eq. 3 for one eigenstate psi0 (energy e0) of
    sector H0: G(z) = <psi0|c (z - (H - e0))^-1 c+|psi0> + <psi0|c+ (z + (H - e0))^-1 c|psi0>,
    with c = c_{site,spin}.  Hp / Hm: the sectors with one electron of that spin
    more / less (None where the sector does not exist).  weight * G is added to
    g when given.  opts: Lanczos options of the two runs; by default the plain
    three-term recurrence (reorth = 0), which is the usual choice for continued
    fractions: lost orthogonality duplicates converged poles but leaves the
    moments the fraction matches intact, at a fraction of the cost of full
    reorthogonalisation.  ws: optional DEVICE workspace for the Lanczos runs, large
    enough for both neighbouring sectors (tridiag_workspace_bytes).  Returns
    (G or g, details)."""
    import torch
    z = np.atleast_1d(np.asarray(z, dtype=np.complex128))
    if g is None:
        g = np.zeros(len(z), dtype=np.complex128)
    if opts is None:
        opts = options(reorth=0)
    info = {}
    for part, Hx, dag, sgn in (("particle", Hp, True, 1), ("hole", Hm, False, -1)):
        if Hx is None:
            continue
        phi = torch.empty(Hx.D, dtype=psi0.dtype, device=psi0.device)
        apply_ladder(H0, Hx, spin, site, dag, psi0, phi)
        try:
            a, b, n2 = Hx.lanczos_tridiag(phi, min(m, Hx.D), opts, ws=ws)
        except EDError as err:  # c+ or c annihilates psi0 (zero start vector)
            if err.status != ED_EINVAL or "zero" not in str(err):
                raise
            info[part] = {"weight": 0.0, "steps": 0}
            continue
        finally:
            del phi
        green_cf(a, b, n2, e0, sgn, z, weight=weight, g=g)
        info[part] = {"weight": n2, "steps": len(a)}
    return g, info


def lowest_levels(hams: Sequence["Hamiltonian"], K: int, opts=None, seed: int = 1, kmax: int = 200, progress=None):
    """The K lowest levels, counted with multiplicity, over the sectors `hams`
    (ed_lowest_levels: the search runs in the library).  Returns (levels,
    vectors, details): levels = [(E, sector index, level index)] ascending (the
    K lowest, more where a multiplet straddles the K-th), vectors = {sector
    index: DEVICE tensor [k, D]} holding levels 0..k-1 of each sector that has
    a level in the list, details = counts, the capped sectors and the
    threshold.  progress: optional callable given one summary line."""
    import torch
    o = opts if opts is not None else options()
    n = len(hams)
    hs = (_p * n)(*[h._h for h in hams])
    L = _p()
    _check(_lib.ed_lowest_levels(n, ctypes.cast(hs, _p), int(K), int(kmax), ctypes.byref(o), seed & 0xFFFFFFFFFFFFFFFF,
                                 ctypes.byref(L), _stream(None)))
    try:
        nl, calls, ncap, thr = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        _check(_lib.ed_levels_info(L, ctypes.byref(nl), ctypes.byref(calls), ctypes.byref(ncap), ctypes.byref(thr)))
        E = np.zeros(max(nl.value, 1))
        sec = np.zeros(max(nl.value, 1), dtype=np.int32)
        idx = np.zeros(max(nl.value, 1), dtype=np.int32)
        _check(_lib.ed_levels_get(L, E.ctypes.data_as(_p), sec.ctypes.data_as(_p), idx.ctypes.data_as(_p)))
        capped = np.zeros(max(ncap.value, 1), dtype=np.int32)
        if ncap.value:
            _check(_lib.ed_levels_capped(L, capped.ctypes.data_as(_p)))
        levels = [(float(E[i]), int(sec[i]), int(idx[i])) for i in range(nl.value)]
        vecs = {}
        for s in sorted({q for _, q, _ in levels}):
            H = hams[s]
            k = 1 + max(i for _, q, i in levels if q == s)
            dt = torch.float64 if H.precision == ED_FP64 else torch.float32
            v = torch.empty((k, H.D), dtype=dt, device="cuda")
            for i in range(k):
                _check(_lib.ed_levels_vector(L, s, i, _dev_ptr(v[i]), _stream(None)))
            vecs[s] = v
        torch.cuda.synchronize()
    finally:
        _lib.ed_levels_free(L)
    det = {"lowest_calls": calls.value, "capped": [int(c) for c in capped[:ncap.value]], "threshold": thr.value}
    if progress:
        progress("lowest_levels: %d levels, %d solver calls, threshold %.6g" % (len(levels), calls.value, thr.value))
    return levels, vecs, det


def green_thermal(params: Dict, ns: int, sectors: Sequence[Tuple[int, int]], spin: int, site: int, beta: float, z,
                  k: int = 20, cutoff: float = 1e-5, m: int = 200, precision: int = ED_FP64, opts=None,
                  device: int = 0, seed: int = 1, K: Optional[int] = None):
    """Temperature Green function of Eq. 3: the k lowest levels of each sector in
    `sectors` (ed_arnoldi_lowest) or, with K, the K lowest levels over all of
    them (lowest_levels); Boltzmann weights over those levels with the cut
    `cutoff` (ed_boltzmann_weights), then each kept level's particle and hole
    continued fractions (green_function) added with its weight.  The levels
    must include every one with a weight above the cut; details["edge"] lists
    the sectors whose highest computed level still carries a weight at or above
    the cut (more levels needed there).  Returns (G(z), details)."""
    import torch
    dev = torch.device("cuda", device)
    dt = torch.float64 if precision == ED_FP64 else torch.float32
    z = np.atleast_1d(np.asarray(z, dtype=np.complex128))
    hams = {}

    def ham(sec):
        if sec not in hams:
            nu, nd = sec
            if min(nu, nd) < 0 or max(nu, nd) > ns:
                hams[sec] = None
            else:
                hams[sec] = Hamiltonian(params, Basis(ns, nu, nd), precision)
        return hams[sec]

    levels = []   # (sector, index, energy)
    vecs = {}
    if K is not None:
        secs = [tuple(sec) for sec in sectors]
        lv, vv, ldet = lowest_levels([ham(sec) for sec in secs], K, opts, seed=seed)
        levels = [(secs[s], i, e) for e, s, i in lv]
        vecs = {secs[s]: v.reshape(-1) for s, v in vv.items()}
    for sec in (sectors if K is None else []):
        H = ham(tuple(sec))
        kk = min(k, H.D)
        v0 = torch.empty(H.D, dtype=dt, device=dev)
        fill_random(v0, seed, 1)
        ev = torch.empty(kk * H.D, dtype=dt, device=dev)
        E, _ = H.lowest(kk, v0, opts, evecs=ev)
        vecs[tuple(sec)] = ev
        levels += [(tuple(sec), i, float(e)) for i, e in enumerate(E)]
    w, kept = boltzmann_weights([l[2] for l in levels], beta, cutoff)
    g = np.zeros(len(z), dtype=np.complex128)
    # a sector whose highest computed level survives the cut may hold more such levels
    if K is None:
        edge = sorted({sec for (sec, i, e), wi in zip(levels, w) if wi > 0.0 and i == k - 1 and k < ham(sec).D})
    else:   # every sector's levels up to the K-th are in; weight left on the K-th itself
        edge = [] if w[-1] == 0.0 or len(levels) < K else ["K-th level above the cut"]
        # sectors stopped at kmax before their levels passed the K-th may hold more
        edge += [secs[s] for s in ldet["capped"]]
    kept_lv = [((sec, i, e), wi) for (sec, i, e), wi in zip(levels, w) if wi != 0.0]
    gopts = opts if opts is not None else options(reorth=0)

    def nbrs(sec):
        nu, nd = sec
        up = (nu + 1, nd) if spin == 0 else (nu, nd + 1)
        dn = (nu - 1, nd) if spin == 0 else (nu, nd - 1)
        return ham(up), ham(dn)
    # one workspace for every level's two Lanczos runs (the largest neighbour)
    nbytes = 1
    for (sec, _, _), _ in kept_lv:
        for Hx in nbrs(sec):
            if Hx is not None:
                nbytes = max(nbytes, Hx.tridiag_workspace_bytes(min(m, Hx.D), gopts))
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    for (sec, i, e), wi in kept_lv:
        H0 = ham(sec)
        psi = vecs[sec][i * H0.D:(i + 1) * H0.D]
        Hp, Hm = nbrs(sec)
        green_function(H0, e, psi, Hp, Hm, spin, site, z, m=m, opts=gopts, weight=wi, g=g, ws=ws)
    details = {"levels": [(sec, i, e, float(wi)) for (sec, i, e), wi in zip(levels, w)], "kept": kept, "edge": edge}
    return g, details

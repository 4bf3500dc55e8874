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
                ("coef", ctypes.c_double)]


class ed_params(ctypes.Structure):
    _fields_ = [("Ns", ctypes.c_int32), ("eps", _p), ("hop", _p), ("w_ud", _p), ("w_ss", _p),
                ("n_x", ctypes.c_int32), ("x", _p)]


class ed_lanczos_opts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("max_basis", ctypes.c_int32), ("tol", ctypes.c_double),
                ("reorth", ctypes.c_int32), ("check_every", ctypes.c_int32), ("refine", ctypes.c_int32),
                ("keep", ctypes.c_int32)]


class ed_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("restarts", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("basis_used", ctypes.c_int32), ("residual", ctypes.c_double), ("ritz", ctypes.c_double),
                ("rq_fp64", ctypes.c_double)]

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
_sig("ed_ham_free", None, [_p])
_sig("ed_lanczos_defaults", None, [ctypes.POINTER(ed_lanczos_opts)])
_sig("ed_workspace_bytes", ctypes.c_int, [_p, ctypes.POINTER(ed_lanczos_opts), ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_size_t)])
_sig("ed_lanczos_ground", ctypes.c_int, [_p, ctypes.POINTER(ed_lanczos_opts), _p, _p, ctypes.c_size_t,
                                         ctypes.POINTER(ctypes.c_double), _p, ctypes.POINTER(ed_info), _p])
_sig("ed_arnoldi_lowest", ctypes.c_int, [_p, ctypes.c_int, ctypes.POINTER(ed_lanczos_opts), _p, _p,
                                         ctypes.c_size_t, _p, _p, _p, _p])
if hasattr(_lib, "ed_lanczos_ground_batched"):
    _sig("ed_batched_workspace_bytes", ctypes.c_int, [ctypes.c_int, _p, ctypes.POINTER(ed_lanczos_opts),
                                                      ctypes.POINTER(ctypes.c_size_t)])
    _sig("ed_lanczos_ground_batched", ctypes.c_int, [ctypes.c_int, _p, ctypes.POINTER(ed_lanczos_opts), _p,
                                                     ctypes.c_uint64, _p, ctypes.c_size_t, _p, _p, _p])
    _sig("ed_batched_last_tile", ctypes.c_int64, [])


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


def options(max_iter=None, max_basis=None, tol=None, reorth=None, check_every=None, refine=None, keep=None):
    o = ed_lanczos_opts()
    _lib.ed_lanczos_defaults(ctypes.byref(o))
    for k, v in (("max_iter", max_iter), ("max_basis", max_basis), ("tol", tol), ("reorth", reorth),
                 ("check_every", check_every), ("refine", refine), ("keep", keep)):
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
    for i, (t, m, mp, c) in enumerate(xt):
        xa[i] = ed_xterm(int(t), int(m), int(mp), float(c))
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

    def workspace_bytes(self, opts=None, k: int = 1) -> int:
        o = opts if opts is not None else options()
        n = ctypes.c_size_t()
        _check(_lib.ed_workspace_bytes(self._h, ctypes.byref(o), k, ctypes.byref(n)))
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

    def close(self):
        if self._h:
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

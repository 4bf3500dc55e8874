"""Shared helpers for the GPU parity tests (HIP path vs the FP64 oracle)."""
import functools
import math

import numpy as np

import oracle as orc
from paper_1004_3354_amd import models, workloads as wl

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def gpu_ed():
    from paper_1004_3354_amd import ed
    return ed


@functools.lru_cache(maxsize=16)
def _sector_cached(key):
    phys, nup, ndn, absval = key
    p = dict(phys)
    T = orc.terms_from_model(_unfreeze(p))
    if absval:
        T = [(abs(c), ops) for c, ops in T]
    return orc.Sector(int(p["Ns"]), nup, ndn, T)


def _freeze(p):
    return tuple(sorted((k, _freeze_v(v)) for k, v in p.items()))


def _freeze_v(v):
    if isinstance(v, (list, tuple)):
        return tuple(_freeze_v(x) for x in v)
    return v


def _unfreeze(p):
    out = {}
    for k, v in p.items():
        out[k] = _unfreeze_v(v)
    return out


def _unfreeze_v(v):
    if isinstance(v, tuple):
        return [_unfreeze_v(x) for x in v]
    return v


def sector(phys, nup, ndn, absval=False):
    return _sector_cached((_freeze(phys), nup, ndn, absval))


def abs_apply(sec_abs, xabs):
    """(|H|_abs |x|): the abs-coefficient matrix still carries fermion signs,
    and no two distinct terms share a matrix position off the diagonal, so the
    absolute values of its entries are the per-term magnitudes."""
    row_ind, col_ind, H = sec_abs.csr()
    return orc.spmv(row_ind, col_ind, np.abs(H), xabs)


def bound(abs_hx, row_terms, unit):
    """Rounding bound of a sum of row_terms products in precision `unit`,
    relative to the sum of the magnitudes of the terms (|H|_abs |x|)."""
    return (row_terms + 8) * unit * abs_hx + 1e-300


def build(phys, nup, ndn, precision):
    ed = gpu_ed()
    b = ed.Basis(int(phys["Ns"]), nup, ndn)
    H = ed.Hamiltonian(models.params_from_model(phys), b, precision)
    return b, H


def generic_model(ns, seed):
    """Random coefficient arrays exercising every diagonal path: spin-dependent
    eps and hopping, per-site U, off-diagonal w_ud, same-spin w_ss, X terms."""
    rng = np.random.default_rng(seed)
    eps = rng.uniform(-1, 1, (2, ns))
    hop = np.zeros((2, ns, ns))
    for s in range(2):
        a = np.triu(rng.uniform(-1, 1, (ns, ns)) * (rng.random((ns, ns)) < 0.45), 1)
        hop[s] = a + a.T
    w_ud = np.diag(rng.uniform(0.5, 3.0, ns))
    for (i, j) in [(0, 1), (1, 0), (2, 0), (1, 2), (3, 1)]:
        w_ud[i, j] = rng.uniform(0, 1)
    w_ss = np.zeros((2, ns, ns))
    for s in range(2):
        w_ss[s] = np.triu(rng.uniform(0, 1, (ns, ns)) * (rng.random((ns, ns)) < 0.3), 1)
    xt = []
    for (m, mp) in [(0, 1), (0, 2), (1, 2)]:
        c1, c2 = rng.uniform(-0.5, 0.5, 2)
        xt += [(1, m, mp, c1), (1, mp, m, c1), (2, m, mp, c2), (2, mp, m, c2)]
    return {"Ns": ns, "eps": eps, "hop": hop, "w_ud": w_ud, "w_ss": w_ss, "xterms": xt}


def generic_terms(p):
    return orc.terms_generic(p["Ns"], p["eps"], p["hop"], p["w_ud"], p["w_ss"], p["xterms"])

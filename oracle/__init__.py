"""FP64 CPU oracle for the exact-diagonalization hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the HIP library (no ranking scheme, no factorised tables, no kernels): it
builds the sector Hamiltonian by applying every fermionic operator string of the
model literally (Jordan-Wigner signs, ``ed_oracle.c``), stores it in the CSR
format of Fig. 1, multiplies with Listing 1, and diagonalises with textbook
Lanczos / ARPACK / dense LAPACK.

Sections of the paper each function follows are named in its docstring.
Conventions where the paper is silent: spin-up site i is fermion mode i and
spin-down site i is mode Ns+i; basis states of one spin are the Ns-bit strings
with N bits set in ascending numeric order; the flat index is r_up * D_dn + r_dn.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Iterable, List, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libedoracle.so")
_lib = None

# A term is (coefficient, [(mode, is_creation), ...]) with the operators listed
# left to right as written; the rightmost acts first.
Term = Tuple[float, List[Tuple[int, int]]]

_i64 = ctypes.c_int64
_p = ctypes.c_void_p


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIBPATH)
    lib.orc_enumerate.restype = _i64
    lib.orc_enumerate.argtypes = [ctypes.c_int, ctypes.c_int, _p]
    lib.orc_apply_string.restype = ctypes.c_int
    lib.orc_apply_string.argtypes = [ctypes.c_uint64, ctypes.c_int, _p, _p, _p, _p]
    lib.orc_build_coo.restype = _i64
    lib.orc_build_coo.argtypes = [ctypes.c_int, _i64, _p, _i64, _p, ctypes.c_int,
                                  _p, _p, _p, _p, _p, _p, _p]
    lib.orc_coo_to_csr.restype = _i64
    lib.orc_coo_to_csr.argtypes = [_i64, _i64, _p, _p, _p, _p, _p, _p]
    lib.orc_spmv.restype = None
    lib.orc_spmv.argtypes = [_i64, _p, _p, _p, _p, _p]
    lib.orc_row_entries.restype = _i64
    lib.orc_row_entries.argtypes = [ctypes.c_int, _i64, _p, _i64, _p, ctypes.c_int,
                                    _p, _p, _p, _p, _i64, _i64, _p, _p]
    lib.orc_rows_apply.restype = ctypes.c_int
    lib.orc_rows_apply.argtypes = [ctypes.c_int, _i64, _p, _i64, _p, ctypes.c_int,
                                   _p, _p, _p, _p, _i64, _p, _p, _p]
    lib.orc_onebody_table.restype = _i64
    lib.orc_onebody_table.argtypes = [ctypes.c_int, _i64, _p, _p, _p, _p, _p, _p]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------- basis --

def basis(ns: int, n: int) -> np.ndarray:
    """All ns-bit strings with n set bits, ascending: one spin's sector basis.

    The sector decomposition is implicit in the dimensions the paper quotes
    (Introduction: 4900 for N_s=8, 6435^2 for N_s=15; Table 1)."""
    lib = _load()
    cnt = lib.orc_enumerate(ns, n, None)
    if cnt < 0:
        raise ValueError("invalid (ns, n)")
    out = np.zeros(cnt, dtype=np.uint32)
    lib.orc_enumerate(ns, n, _ptr(out))
    return out


def apply_string(word: int, ops: Sequence[Tuple[int, int]]):
    """Apply one operator string to a Fock word; returns (word', sign) or None."""
    lib = _load()
    mode = np.array([m for m, _ in ops], dtype=np.int32)
    dag = np.array([d for _, d in ops], dtype=np.int8)
    w = ctypes.c_uint64(0)
    s = ctypes.c_int32(0)
    ok = lib.orc_apply_string(ctypes.c_uint64(word), len(ops), _ptr(mode), _ptr(dag),
                              ctypes.byref(w), ctypes.byref(s))
    return (int(w.value), int(s.value)) if ok else None


# ------------------------------------------------------- model -> operators --

def _up(i: int, ns: int) -> int:
    return i


def _dn(i: int, ns: int) -> int:
    return ns + i


def _mode(i: int, spin: int, ns: int) -> int:
    return i if spin == 0 else ns + i


def _number(mode: int) -> List[Tuple[int, int]]:
    return [(mode, 1), (mode, 0)]


def terms_generic(ns: int, eps, hop, w_ud, w_ss, xterms: Iterable = ()) -> List[Term]:
    """Operator strings for the generic coefficient arrays the C interface takes:

    sum_{i,s} eps[s,i] n_is + sum_{s, i!=j} hop[s,i,j] c+_is c_js
    + sum_{i,j} w_ud[i,j] n_i,up n_j,dn + sum_{s, i<j} w_ss[s,i,j] n_is n_js
    + sum over (type, m, m', c) of c * (spin-flip or pair-hopping string as written
    in the multi-orbital Hamiltonian of Section 4)
    + sum over (3, i, j, k, l, c) of c * c+_{i up} c+_{j dn} c_{l dn} c_{k up}, an
    opposite-spin element U_ijkl of a full two-body U-matrix (Section 4's
    closing remark on the other non-diagonal elements)
    + sum over (4 or 5, i, j, k, l, c) of c * c+_{i s} c+_{j s} c_{l s} c_{k s},
    a same-spin element (s = up for 4, down for 5)."""
    eps = np.asarray(eps, dtype=np.float64).reshape(2, ns)
    hop = np.asarray(hop, dtype=np.float64).reshape(2, ns, ns)
    w_ud = np.asarray(w_ud, dtype=np.float64).reshape(ns, ns)
    w_ss = np.asarray(w_ss, dtype=np.float64).reshape(2, ns, ns)
    T: List[Term] = []
    for s in range(2):
        for i in range(ns):
            if eps[s, i] != 0.0:
                T.append((float(eps[s, i]), _number(_mode(i, s, ns))))
    for s in range(2):
        for i in range(ns):
            for j in range(ns):
                if i != j and hop[s, i, j] != 0.0:
                    T.append((float(hop[s, i, j]), [(_mode(i, s, ns), 1), (_mode(j, s, ns), 0)]))
    for i in range(ns):
        for j in range(ns):
            if w_ud[i, j] != 0.0:
                T.append((float(w_ud[i, j]), _number(_up(i, ns)) + _number(_dn(j, ns))))
    for s in range(2):
        for i in range(ns):
            for j in range(i + 1, ns):
                if w_ss[s, i, j] != 0.0:
                    T.append((float(w_ss[s, i, j]),
                              _number(_mode(i, s, ns)) + _number(_mode(j, s, ns))))
    for xt in xterms:
        if xt[0] == UD_GENERAL:
            _, i, j, k, l, c = xt
            T.append((float(c), [(_up(i, ns), 1), (_dn(j, ns), 1), (_dn(l, ns), 0), (_up(k, ns), 0)]))
        elif xt[0] in (UU_GENERAL, DD_GENERAL):
            t, i, j, k, l, c = xt
            sp = 0 if t == UU_GENERAL else 1
            T.append((float(c), [(_mode(i, sp, ns), 1), (_mode(j, sp, ns), 1), (_mode(l, sp, ns), 0),
                                 (_mode(k, sp, ns), 0)]))
        else:
            typ, m, mp, c = xt
            T.append((float(c), _xstring(typ, m, mp, ns)))
    return T


SPIN_FLIP = 1
PAIR_HOP = 2
UD_GENERAL = 3
UU_GENERAL = 4
DD_GENERAL = 5


def _xstring(typ: int, m: int, mp: int, ns: int) -> List[Tuple[int, int]]:
    """Section 4: spin flip  d+_{m up} d_{m dn} d+_{m' dn} d_{m' up};
    pair hopping  d+_{m up} d+_{m dn} d_{m' up} d_{m' dn}  (as written)."""
    if typ == SPIN_FLIP:
        return [(_up(m, ns), 1), (_dn(m, ns), 0), (_dn(mp, ns), 1), (_up(mp, ns), 0)]
    if typ == PAIR_HOP:
        return [(_up(m, ns), 1), (_dn(m, ns), 1), (_up(mp, ns), 0), (_dn(mp, ns), 0)]
    raise ValueError("unknown four-fermion term type")


def terms_hubbard(lx: int, ly: int, t: float, U: float, periodic: bool = True) -> List[Term]:
    """Eq. (1): H = - sum_{i,j,s} t_ij c+_is c_js + U sum_i n_i,up n_i,dn on an
    lx-by-ly square lattice with nearest-neighbour t_ij = t, site i = x + lx*y.
    The double sum runs over ordered pairs, so every bond enters as (i,j) and
    (j,i); a bond reached twice (a 2-site periodic direction) counts twice."""
    ns = lx * ly
    tij = np.zeros((ns, ns))
    for y in range(ly):
        for x in range(lx):
            i = x + lx * y
            for (dx, dy) in ((1, 0), (0, 1)):
                xx, yy = x + dx, y + dy
                if periodic:
                    xx %= lx
                    yy %= ly
                elif xx >= lx or yy >= ly:
                    continue
                j = xx + lx * yy
                if i == j:
                    continue
                tij[i, j] += t
                tij[j, i] += t
    T: List[Term] = []
    for s in range(2):
        for i in range(ns):
            for j in range(ns):
                if tij[i, j] != 0.0:
                    T.append((-float(tij[i, j]), [(_mode(i, s, ns), 1), (_mode(j, s, ns), 0)]))
    if U != 0.0:
        for i in range(ns):
            T.append((float(U), _number(_up(i, ns)) + _number(_dn(i, ns))))
    return T


def terms_aim(U: float, eps_d: float, eps_k: Sequence[float], V: Sequence[float]) -> List[Term]:
    """Eq. (2): H_AIM = sum_{k,s} V_k [d+_s c_ks + c+_ks d_s] + sum_{k,s} eps_k n_ks
    + eps_d (n_up + n_dn) + U n_up n_dn.  Impurity = site 0, bath level k = site k
    (k = 1..N_s-1); V_k and eps_k are taken spin independent."""
    nk = len(eps_k)
    ns = nk + 1
    T: List[Term] = []
    for s in range(2):
        d = _mode(0, s, ns)
        for k in range(nk):
            c = _mode(k + 1, s, ns)
            if V[k] != 0.0:
                T.append((float(V[k]), [(d, 1), (c, 0)]))
                T.append((float(V[k]), [(c, 1), (d, 0)]))
        for k in range(nk):
            if eps_k[k] != 0.0:
                T.append((float(eps_k[k]), _number(_mode(k + 1, s, ns))))
        if eps_d != 0.0:
            T.append((float(eps_d), _number(d)))
    if U != 0.0:
        T.append((float(U), _number(_up(0, ns)) + _number(_dn(0, ns))))
    return T


def terms_kanamori(M: int, n_b: int, U: float, J: float, Up: float,
                   Jp_sf: float, Jp_ph: float, eps_imp: Sequence[float],
                   eps_bath, V) -> List[Term]:
    """Multi-orbital impurity Hamiltonian of Section 4 (the equation introducing
    the spin-flip study):
      sum_{m s} (eps_m - mu) n_ms + sum_{k s} eps_k n_ks
      + sum_{m k s} V_mk [d+_ms c_ks + H.c.] + sum_m U n_m,up n_m,dn
      + sum_{m<m', s, s'} (U' - J delta_ss') n_ms n_m's'
      - sum_{m != m'} J' [d+_m,up d_m,dn d+_m',dn d_m',up + d+_m,up d+_m,dn d_m',up d_m',dn].
    eps_imp[m] is (eps_m - mu).  Orbital m is site m; its bath level j is site
    M + m*n_b + j and couples only to orbital m with V[m][j].  The spin-flip and
    pair-hopping J' may be set separately (Jp_sf, Jp_ph)."""
    ns = M + M * n_b
    eps_bath = np.asarray(eps_bath, dtype=np.float64).reshape(M, n_b)
    V = np.asarray(V, dtype=np.float64).reshape(M, n_b)
    T: List[Term] = []
    for s in range(2):
        for m in range(M):
            if eps_imp[m] != 0.0:
                T.append((float(eps_imp[m]), _number(_mode(m, s, ns))))
        for m in range(M):
            for j in range(n_b):
                k = M + m * n_b + j
                if eps_bath[m, j] != 0.0:
                    T.append((float(eps_bath[m, j]), _number(_mode(k, s, ns))))
        for m in range(M):
            for j in range(n_b):
                k = M + m * n_b + j
                if V[m, j] != 0.0:
                    T.append((float(V[m, j]), [(_mode(m, s, ns), 1), (_mode(k, s, ns), 0)]))
                    T.append((float(V[m, j]), [(_mode(k, s, ns), 1), (_mode(m, s, ns), 0)]))
    for m in range(M):
        if U != 0.0:
            T.append((float(U), _number(_up(m, ns)) + _number(_dn(m, ns))))
    for m in range(M):
        for mp in range(m + 1, M):
            for s in range(2):
                for sp in range(2):
                    c = Up - (J if s == sp else 0.0)
                    if c != 0.0:
                        T.append((float(c), _number(_mode(m, s, ns)) + _number(_mode(mp, sp, ns))))
    for m in range(M):
        for mp in range(M):
            if m == mp:
                continue
            if Jp_sf != 0.0:
                T.append((-float(Jp_sf), _xstring(SPIN_FLIP, m, mp, ns)))
            if Jp_ph != 0.0:
                T.append((-float(Jp_ph), _xstring(PAIR_HOP, m, mp, ns)))
    return T


def _pack_terms(terms: List[Term]):
    coef = np.array([c for c, _ in terms], dtype=np.float64)
    off = np.zeros(len(terms) + 1, dtype=np.int64)
    modes: List[int] = []
    dags: List[int] = []
    for t, (_, ops) in enumerate(terms):
        off[t + 1] = off[t] + len(ops)
        for (m, d) in ops:
            modes.append(m)
            dags.append(1 if d else 0)
    return (coef, off, np.array(modes, dtype=np.int32), np.array(dags, dtype=np.int8))


# ----------------------------------------------------------- sector matrix --

class Sector:
    """One (N_up, N_dn) sector of a model given as operator strings."""

    def __init__(self, ns: int, nup: int, ndn: int, terms: List[Term]):
        self.ns, self.nup, self.ndn = ns, nup, ndn
        self.up = basis(ns, nup)
        self.dn = basis(ns, ndn)
        self.dup, self.ddn = len(self.up), len(self.dn)
        self.D = self.dup * self.ddn
        self.terms = terms
        self._packed = _pack_terms(terms)
        self._csr = None

    # -- CSR (Section 3.1, Fig. 1) --
    def coo(self):
        lib = _load()
        coef, off, mode, dag = self._packed
        n = lib.orc_build_coo(self.ns, self.dup, _ptr(self.up), self.ddn, _ptr(self.dn),
                              len(coef), _ptr(coef), _ptr(off), _ptr(mode), _ptr(dag),
                              None, None, None)
        if n < 0:
            raise ValueError("operator string leaves the (N_up, N_dn) sector" if n == -2
                             else "oracle COO build failed")
        row = np.empty(n, dtype=np.int64)
        col = np.empty(n, dtype=np.int64)
        val = np.empty(n, dtype=np.float64)
        lib.orc_build_coo(self.ns, self.dup, _ptr(self.up), self.ddn, _ptr(self.dn),
                          len(coef), _ptr(coef), _ptr(off), _ptr(mode), _ptr(dag),
                          _ptr(row), _ptr(col), _ptr(val))
        return row, col, val

    def csr(self):
        if self._csr is None:
            row, col, val = self.coo()
            self._csr = coo_to_csr(self.D, row, col, val)
            del row, col, val
        return self._csr

    def spmv(self, x: np.ndarray) -> np.ndarray:
        row_ind, col_ind, H = self.csr()
        return spmv(row_ind, col_ind, H, x)

    def dense(self) -> np.ndarray:
        row_ind, col_ind, H = self.csr()
        A = np.zeros((self.D, self.D))
        for i in range(self.D):
            a, b = row_ind[i], row_ind[i + 1]
            A[i, col_ind[a:b]] += H[a:b]
        return A

    # -- matrix-free rows (end of Section 3.2: evaluate elements when needed) --
    def row_entries(self, J: int):
        lib = _load()
        coef, off, mode, dag = self._packed
        cap = 4 * len(coef) + 8
        cols = np.empty(cap, dtype=np.int64)
        vals = np.empty(cap, dtype=np.float64)
        n = lib.orc_row_entries(self.ns, self.dup, _ptr(self.up), self.ddn, _ptr(self.dn),
                                len(coef), _ptr(coef), _ptr(off), _ptr(mode), _ptr(dag),
                                int(J), cap, _ptr(cols), _ptr(vals))
        if n < 0 or n > cap:
            raise ValueError("row generation failed")
        return cols[:n].copy(), vals[:n].copy()

    def rows_apply(self, rows: np.ndarray, x: np.ndarray) -> np.ndarray:
        lib = _load()
        coef, off, mode, dag = self._packed
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty(len(rows), dtype=np.float64)
        rc = lib.orc_rows_apply(self.ns, self.dup, _ptr(self.up), self.ddn, _ptr(self.dn),
                                len(coef), _ptr(coef), _ptr(off), _ptr(mode), _ptr(dag),
                                len(rows), _ptr(rows), _ptr(x), _ptr(y))
        if rc != 0:
            raise ValueError("row generation failed")
        return y


def coo_to_csr(nrows: int, row, col, val):
    """(row, col, value) triplets -> (row_ind, col_ind, H_values) as in Fig. 1."""
    lib = _load()
    row = np.ascontiguousarray(row, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int64)
    val = np.ascontiguousarray(val, dtype=np.float64)
    nnz = len(row)
    row_ind = np.empty(nrows + 1, dtype=np.int64)
    col_ind = np.empty(max(nnz, 1), dtype=np.int64)
    H = np.empty(max(nnz, 1), dtype=np.float64)
    n = lib.orc_coo_to_csr(nrows, nnz, _ptr(row), _ptr(col), _ptr(val),
                           _ptr(row_ind), _ptr(col_ind), _ptr(H))
    if n < 0:
        raise MemoryError("oracle CSR build failed")
    return row_ind, col_ind[:n].copy(), H[:n].copy()


def spmv(row_ind, col_ind, H, x) -> np.ndarray:
    """Listing 1 (CSR SpMV), rows split over OpenMP threads."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(len(row_ind) - 1, dtype=np.float64)
    lib.orc_spmv(len(row_ind) - 1, _ptr(row_ind), _ptr(col_ind), _ptr(H), _ptr(x), _ptr(y))
    return y


def onebody_table(ns: int, n: int, h) -> Tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
    """Per-spin elements of sum_{i!=j} h_ij c+_i c_j in one spin's sector:
    CSR over source states of (target rank, sign, h_ij), targets ascending."""
    lib = _load()
    st = basis(ns, n)
    h = np.ascontiguousarray(np.asarray(h, dtype=np.float64).reshape(ns, ns))
    cnt = lib.orc_onebody_table(ns, len(st), _ptr(st), _ptr(h), None, None, None, None)
    off = np.empty(len(st) + 1, dtype=np.int64)
    tgt = np.empty(max(cnt, 1), dtype=np.int64)
    sgn = np.empty(max(cnt, 1), dtype=np.int8)
    amp = np.empty(max(cnt, 1), dtype=np.float64)
    rc = lib.orc_onebody_table(ns, len(st), _ptr(st), _ptr(h), _ptr(off), _ptr(tgt),
                               _ptr(sgn), _ptr(amp))
    if rc < 0:
        raise ValueError("one-body table failed")
    return off, tgt[:cnt], sgn[:cnt], amp[:cnt]


# ------------------------------------------------------------ eigensolvers --

def lanczos_ground(matvec, v0: np.ndarray, max_iter: int = 400, tol: float = 1e-12,
                   reorth: bool = True, want_vector: bool = True):
    """Lanczos iteration (Section 3: repeated multiplication of H by a trial
    vector) for the lowest eigenpair, FP64.  With reorth=True every new vector
    is orthogonalised against all previous ones twice (classical Gram-Schmidt,
    'twice is enough').  Stops when |beta_j * s_j| <= tol * max(|theta|, 1)
    (s_j: last component of the lowest eigenvector of T_j) or on breakdown.
    Returns (theta, psi or None, info dict)."""
    from scipy.linalg import eigh_tridiagonal
    v = np.asarray(v0, dtype=np.float64)
    v = v / np.linalg.norm(v)
    V = [v] if (reorth or want_vector) else None
    alphas: List[float] = []
    betas: List[float] = []
    v_prev = None
    theta, s, resid = None, None, None
    it = 0
    for it in range(1, max_iter + 1):
        w = matvec(v)
        a = float(v @ w)
        w = w - a * v
        if v_prev is not None:
            w = w - betas[-1] * v_prev
        if reorth:
            for _ in range(2):
                c = np.array([q @ w for q in V])
                for q, ci in zip(V, c):
                    w = w - ci * q
                a += float(c[-1])
        alphas.append(a)
        b = float(np.linalg.norm(w))
        ev, evec = eigh_tridiagonal(np.array(alphas), np.array(betas),
                                    select="i", select_range=(0, 0))
        theta = float(ev[0])
        s = evec[:, 0]
        resid = abs(b * s[-1])
        if resid <= tol * max(abs(theta), 1.0) or b <= 1e-14 * max(abs(theta), 1.0):
            break
        betas.append(b)
        v_prev, v = v, w / b
        if V is not None:
            V.append(v)
    psi = None
    if want_vector and V is not None:
        psi = np.zeros_like(V[0])
        for q, si in zip(V, s):
            psi += si * q
        psi /= np.linalg.norm(psi)
    return theta, psi, {"iters": it, "residual": resid}


def lowest_k(sector: Sector, k: int, tol: float = 1e-12, dense_limit: int = 5000):
    """The k lowest eigenvalues of the sector matrix, counted with multiplicity.
    Small sectors: dense LAPACK (the full diagonalisation of the Introduction).
    Larger ones: ARPACK's implicitly restarted Lanczos (the P_ARPACK solver the
    paper cites in Section 3) on the Listing-1 SpMV."""
    if sector.D <= dense_limit:
        ev = np.linalg.eigvalsh(sector.dense())
        return ev[:k]
    from scipy.sparse.linalg import LinearOperator, eigsh
    op = LinearOperator((sector.D, sector.D), matvec=sector.spmv, dtype=np.float64)
    ncv = min(sector.D - 1, max(2 * k + 20, 40))
    v0 = np.random.default_rng(20100420).standard_normal(sector.D)
    ev = eigsh(op, k=k, which="SA", tol=tol, ncv=ncv, v0=v0, return_eigenvectors=False)
    return np.sort(ev)


def binom(n: int, k: int) -> int:
    return math.comb(n, k) if 0 <= k <= n else 0


def terms_from_model(p: dict) -> List[Term]:
    """Operator strings for a physical-parameter dictionary (keys as produced by
    the seeded workload generators: model = 'hubbard' | 'aim' | 'kanamori')."""
    if p["model"] == "hubbard":
        return terms_hubbard(p["lx"], p["ly"], p["t"], p["U"], p.get("periodic", True))
    if p["model"] == "aim":
        return terms_aim(p["U"], p["eps_d"], p["eps_k"], p["V"])
    if p["model"] == "kanamori":
        return terms_kanamori(p["M"], p["n_b"], p["U"], p["J"], p["Up"], p["Jp_sf"],
                              p["Jp_ph"], p["eps_imp"], p["eps_bath"], p["V"])
    raise ValueError("unknown model")


def sector_for(p: dict, nup: int, ndn: int) -> Sector:
    return Sector(int(p["Ns"]), nup, ndn, terms_from_model(p))

# ------------------------------------------------- Green function (Eq. 3) --

def ladder_matrix(src: Sector, dst: Sector, spin: int, site: int, dagger: bool) -> np.ndarray:
    """Dense matrix of c+_{site,spin} (dagger) or c_{site,spin} from sector src
    to sector dst, literally: each basis state of src becomes a Fock word, the
    one-operator string is applied with its Jordan-Wigner sign, and the result
    is looked up in dst's basis.  Its entries are the <mu|c+_sigma|nu> of Eq. 3
    in the occupation basis."""
    ns = src.ns
    mode = _mode(site, spin, ns)
    mask = (1 << ns) - 1
    L = np.zeros((dst.D, src.D))
    for u, su in enumerate(src.up):
        for d, sd in enumerate(src.dn):
            r = apply_string(int(su) | (int(sd) << ns), [(mode, 1 if dagger else 0)])
            if r is None:
                continue
            w2, sg = r
            iu = int(np.searchsorted(dst.up, w2 & mask))
            idn = int(np.searchsorted(dst.dn, w2 >> ns))
            if iu >= dst.dup or dst.up[iu] != (w2 & mask) or idn >= dst.ddn or dst.dn[idn] != (w2 >> ns):
                raise ValueError("ladder operator leaves the destination sector")
            L[iu * dst.ddn + idn, u * src.ddn + d] += sg
    return L


def ladder(src: Sector, dst: Sector, spin: int, site: int, dagger: bool, x: np.ndarray) -> np.ndarray:
    """c+_{site,spin} (dagger) or c_{site,spin} applied to a vector of sector src."""
    return ladder_matrix(src, dst, spin, site, dagger) @ x


def green_lehmann(p: dict, nup: int, ndn: int, spin: int, site: int, z) -> Tuple[np.ndarray, dict]:
    """Eq. 3 at zero temperature, where only the ground state |0> of the sector
    contributes (the Boltzmann weights of the other states vanish):
        G(z) = sum_mu |<mu|c+|0>|^2 / (z - (E_mu - E_0))
             + sum_nu |<nu|c|0>|^2 / (z + (E_nu - E_0)),
    mu over the sector with one more electron of the given spin, nu over the
    sector with one less, all by dense diagonalisation (small sectors only).
    The paper prints the denominator as E_nu - E_mu - i w_n, the negative of
    this standard Lehmann form (a sign convention); the form here is the one
    whose U = 0 limit is the one-body resolvent (z - h)^-1."""
    z = np.atleast_1d(np.asarray(z, dtype=np.complex128))
    s0 = sector_for(p, nup, ndn)
    e, v = np.linalg.eigh(s0.dense())
    if len(e) > 1 and e[1] - e[0] < 1e-8 * max(1.0, abs(e[0])):
        raise ValueError("degenerate ground state: the zero-temperature limit is not unique")
    e0, psi = e[0], v[:, 0]
    g = np.zeros(len(z), dtype=np.complex128)
    weights = {}
    ns = s0.ns
    n_sp = nup if spin == 0 else ndn
    for part, dn_, sgn in (("particle", 1, 1.0), ("hole", -1, -1.0)):
        n2 = n_sp + dn_
        if n2 < 0 or n2 > ns:
            weights[part] = 0.0
            continue
        s1 = sector_for(p, nup + (dn_ if spin == 0 else 0), ndn + (dn_ if spin == 1 else 0))
        e1, v1 = np.linalg.eigh(s1.dense())
        phi = ladder(s0, s1, spin, site, dn_ > 0, psi)
        w = (v1.T @ phi) ** 2
        weights[part] = float(np.sum(w))
        g += np.sum(w[None, :] / (z[:, None] - sgn * (e1[None, :] - e0)), axis=1)
    return g, {"E0": float(e0), "weights": weights}


def green_thermal(p: dict, spin: int, site: int, beta: float, z) -> Tuple[np.ndarray, dict]:
    """Eq. 3 at inverse temperature beta, as the double sum over all eigenpairs
    of the whole Fock space (every (N_up, N_dn) sector, dense diagonalisation):
        G(z) = (1/Z) sum_{nu, mu} |<mu|c+|nu>|^2 (e^{-beta E_nu} + e^{-beta E_mu})
                                  / (z - (E_mu - E_nu)),
    Z = sum_mu e^{-beta E_mu}, mu running over the sector with one more
    electron of the given spin than nu's.  The denominator's sign is the
    standard one (the reading taken for green_lehmann); energies are measured
    from the lowest level so that the exponentials cannot overflow."""
    z = np.atleast_1d(np.asarray(z, dtype=np.complex128))
    ns = int(p["Ns"])
    eig = {}
    for nu in range(ns + 1):
        for nd in range(ns + 1):
            sec = sector_for(p, nu, nd)
            e, v = np.linalg.eigh(sec.dense())
            eig[(nu, nd)] = (sec, e, v)
    emin = min(float(e.min()) for _, e, _ in eig.values())
    Z = sum(float(np.sum(np.exp(-beta * (e - emin)))) for _, e, _ in eig.values())
    g = np.zeros(len(z), dtype=np.complex128)
    for (nu, nd), (s0, e0, v0) in eig.items():
        tgt = (nu + 1, nd) if spin == 0 else (nu, nd + 1)
        if tgt not in eig:
            continue
        s1, e1, v1 = eig[tgt]
        M = v1.T @ ladder_matrix(s0, s1, spin, site, True) @ v0      # M[mu, nu] = <mu|c+|nu>
        fac = np.exp(-beta * (e0[None, :] - emin)) + np.exp(-beta * (e1[:, None] - emin))
        num = (M ** 2 * fac).ravel()
        den = (e1[:, None] - e0[None, :]).ravel()
        keep = num != 0.0
        g += np.sum(num[keep][None, :] / (z[:, None] - den[keep][None, :]), axis=1)
    return g / Z, {"Z": Z, "Emin": emin}

"""Coefficient arrays of the C interface for the paper's three model families.

Each builder returns a dict with eps [2,Ns], hop [2,Ns,Ns], w_ud [Ns,Ns],
w_ss [2,Ns,Ns] (float64) and xterms [(type, m, m', coef)], the generic form that
``ed_ham_create`` takes (its meaning is documented in include/ed.h).
Readings where the paper leaves the choice open:
  * Eq. (1): the double sum over (i, j) runs over ordered pairs, so each
    nearest-neighbour bond gives h_ij = h_ji = -t.  Site i = x + lx*y.
  * Eq. (2): impurity = site 0, bath level k = site k; V_k, eps_k spin independent.
  * Section 4 multi-orbital Hamiltonian: orbital m = site m, bath level j of
    orbital m = site M + m*n_b + j coupled only to orbital m; opposite-spin
    density-density U' for every m != m' pair, same-spin U' - J once per
    unordered pair; the J' bracket enters with coefficient -J' per ordered pair.
"""
from __future__ import annotations

from typing import Dict

import numpy as np

SPIN_FLIP = 1
PAIR_HOP = 2


def _empty(ns: int) -> Dict:
    return {"Ns": ns, "eps": np.zeros((2, ns)), "hop": np.zeros((2, ns, ns)),
            "w_ud": np.zeros((ns, ns)), "w_ss": np.zeros((2, ns, ns)), "xterms": []}


def hubbard_params(lx: int, ly: int, t: float, U: float, periodic: bool = True) -> Dict:
    """Eq. (1) on an lx x ly square lattice, nearest-neighbour hopping t."""
    ns = lx * ly
    p = _empty(ns)
    for y in range(ly):
        for x in range(lx):
            i = x + lx * y
            for xx, yy in ((x + 1, y), (x, y + 1)):
                if periodic:
                    xx, yy = xx % lx, yy % ly
                elif xx >= lx or yy >= ly:
                    continue
                j = xx + lx * yy
                if j == i:
                    continue
                for s in range(2):
                    p["hop"][s, i, j] -= t
                    p["hop"][s, j, i] -= t
    np.fill_diagonal(p["w_ud"], U)
    return p


def aim_params(U: float, eps_d: float, eps_k, V) -> Dict:
    """Eq. (2): single impurity (site 0) hybridised with bath levels 1..N_k."""
    nk = len(eps_k)
    ns = nk + 1
    p = _empty(ns)
    for s in range(2):
        p["eps"][s, 0] = eps_d
        p["eps"][s, 1:] = eps_k
        p["hop"][s, 0, 1:] = V
        p["hop"][s, 1:, 0] = V
    p["w_ud"][0, 0] = U
    return p


def kanamori_params(M: int, n_b: int, U: float, J: float, Up: float, Jp_sf: float,
                    Jp_ph: float, eps_imp, eps_bath, V) -> Dict:
    """Section 4 multi-orbital impurity Hamiltonian with per-orbital baths."""
    ns = M + M * n_b
    p = _empty(ns)
    eps_bath = np.asarray(eps_bath, dtype=np.float64).reshape(M, n_b)
    V = np.asarray(V, dtype=np.float64).reshape(M, n_b)
    for s in range(2):
        for m in range(M):
            p["eps"][s, m] = eps_imp[m]
            for j in range(n_b):
                k = M + m * n_b + j
                p["eps"][s, k] = eps_bath[m, j]
                p["hop"][s, m, k] = V[m, j]
                p["hop"][s, k, m] = V[m, j]
    for m in range(M):
        p["w_ud"][m, m] = U
        for mp in range(M):
            if mp != m:
                p["w_ud"][m, mp] = Up
    for s in range(2):
        for m in range(M):
            for mp in range(m + 1, M):
                p["w_ss"][s, m, mp] = Up - J
    for m in range(M):
        for mp in range(M):
            if m == mp:
                continue
            if Jp_sf != 0.0:
                p["xterms"].append((SPIN_FLIP, m, mp, -Jp_sf))
            if Jp_ph != 0.0:
                p["xterms"].append((PAIR_HOP, m, mp, -Jp_ph))
    return p


def params_from_model(m: Dict) -> Dict:
    """Coefficient arrays for a physical-parameter dict (model = hubbard|aim|kanamori)."""
    if m["model"] == "hubbard":
        return hubbard_params(m["lx"], m["ly"], m["t"], m["U"], m.get("periodic", True))
    if m["model"] == "aim":
        return aim_params(m["U"], m["eps_d"], m["eps_k"], m["V"])
    if m["model"] == "kanamori":
        return kanamori_params(m["M"], m["n_b"], m["U"], m["J"], m["Up"], m["Jp_sf"], m["Jp_ph"],
                               m["eps_imp"], m["eps_bath"], m["V"])
    raise ValueError("unknown model")

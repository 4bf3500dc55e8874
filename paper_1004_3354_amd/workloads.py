"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds no part of the method: it only draws model parameters and
random vectors.  The paper's own inputs (DMFT-fitted baths, LDA input for
Sr2RuO4) are not available, so parameters are drawn with the structure of the
models it diagonalises: Eq. (1) Hubbard lattice, Eq. (2) Anderson impurity and
the three-orbital impurity Hamiltonian of Section 4, at the sector sizes the
paper discusses (N_s = 8 ... 18).

Random vectors come from a counter-based generator, SplitMix64 (Steele, Lea and
Flood, OOPSLA 2014; constants as in Vigna's public-domain splitmix64.c), so any
element can be produced on its own: element i of stream `seed` is the (i+1)-th
output of SplitMix64 started from state `seed`.  The GPU library implements the
same published generator independently for device-side fills.
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np

SEED_BASE = 10043354

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, idx: np.ndarray) -> np.ndarray:
    """Output number idx (0-based) of SplitMix64 started from state `seed`."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (idx + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_at(seed: int, idx: np.ndarray) -> np.ndarray:
    """Uniform on [-1, 1): 2 * (top 53 bits / 2^53) - 1, exact in FP64."""
    z = splitmix64(seed, idx)
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return 2.0 * u - 1.0


def uniform_vector(seed: int, n: int, start: int = 0) -> np.ndarray:
    return uniform_at(seed, np.arange(start, start + n, dtype=np.uint64))


def gaussian_vector(seed: int, n: int) -> np.ndarray:
    """Standard normal by Box-Muller (1958) on outputs 2i and 2i+1:
    u1 in (0, 1], u2 in [0, 1), g = sqrt(-2 ln u1) cos(2 pi u2)."""
    i = np.arange(n, dtype=np.uint64)
    z1 = splitmix64(seed, 2 * i)
    z2 = splitmix64(seed, 2 * i + np.uint64(1))
    u1 = ((z1 >> np.uint64(11)).astype(np.float64) + 1.0) * (1.0 / 9007199254740992.0)
    u2 = (z2 >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


# --------------------------------------------------------------- models ----

def aim(n_bath: int, U: float, eps_d: float, seed: int,
        eps_range=(-2.0, 2.0), v_range=(0.2, 0.6)) -> Dict:
    """One-band Anderson impurity (Eq. 2): bath levels then hybridisations
    drawn from PCG64(seed), uniform in the given ranges."""
    rng = np.random.default_rng(seed)
    eps_k = rng.uniform(*eps_range, size=n_bath)
    V = rng.uniform(*v_range, size=n_bath)
    return {"model": "aim", "Ns": n_bath + 1, "U": U, "eps_d": eps_d,
            "eps_k": eps_k.tolist(), "V": V.tolist()}


def hubbard(lx: int, ly: int, t: float, U: float, periodic: bool = True) -> Dict:
    """Square-lattice Hubbard model (Eq. 1) with nearest-neighbour hopping."""
    return {"model": "hubbard", "Ns": lx * ly, "lx": lx, "ly": ly, "t": t, "U": U,
            "periodic": periodic}


def kanamori(M: int, n_b: int, U: float, J: float, seed: int, jprime: bool = True,
             Up: float = None, eps_imp: float = None,
             eps_range=(-3.0, 3.0), v_range=(0.1, 0.5)) -> Dict:
    """Three-orbital impurity of Section 4 with U' = U - 2J and, when switched on,
    J' = J for both spin flip and pair hopping.  Each orbital has n_b bath levels
    of its own.  Bath energies (site order) then hybridisations are drawn from
    PCG64(seed).  The impurity level eps_m - mu defaults to the particle-hole
    symmetric value -(U/2 + (M-1)(2U'-J)/2)."""
    if Up is None:
        Up = U - 2.0 * J
    if eps_imp is None:
        eps_imp = -(U / 2.0 + (M - 1) * (2.0 * Up - J) / 2.0)
    rng = np.random.default_rng(seed)
    eps_bath = rng.uniform(*eps_range, size=(M, n_b))
    V = rng.uniform(*v_range, size=(M, n_b))
    jp = J if jprime else 0.0
    return {"model": "kanamori", "Ns": M + M * n_b, "M": M, "n_b": n_b, "U": U, "J": J,
            "Up": Up, "Jp_sf": jp, "Jp_ph": jp, "eps_imp": [eps_imp] * M,
            "eps_bath": eps_bath.tolist(), "V": V.tolist()}


def config(idx: int, jprime: bool = True) -> Tuple[Dict, List[Tuple[int, int]]]:
    """The five benchmark workloads: (model parameters, sectors)."""
    seed = SEED_BASE + idx
    if idx == 0:   # 1 impurity + 7 bath levels, sector (4,4), dim 4900
        return aim(7, 2.0, -1.0, seed), [(4, 4)]
    if idx == 1:   # 4x4 periodic Hubbard, half filling, dim 12870^2
        return hubbard(4, 4, 1.0, 4.0), [(8, 8)]
    if idx == 2:   # 3 orbitals + 12 bath levels (N_s=15), sector (7,7), dim 6435^2
        return kanamori(3, 4, 2.3, 0.4, seed, jprime=jprime), [(7, 7)]
    if idx == 3:   # 3 orbitals + 9 bath levels (N_s=12), all 169 sectors
        return kanamori(3, 3, 2.3, 0.4, seed, jprime=jprime), [(a, b) for a in range(13) for b in range(13)]
    if idx == 4:   # 3 orbitals + 15 bath levels (N_s=18), sector (9,9), dim 48620^2
        return kanamori(3, 5, 2.3, 0.4, seed, jprime=jprime), [(9, 9)]
    raise ValueError("no such workload")


def start_vector_seed(idx: int) -> int:
    """Seed of the Lanczos start vector / H.v input vector of workload idx."""
    return SEED_BASE + 1000 + idx

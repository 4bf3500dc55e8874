"""Pins of the oracle's impurity Green function (Eq. 3 at zero temperature):
the U = 0 limit must be the one-body resolvent (z - h)^-1, the Hubbard atom
has a closed form, the spectral weight of c and c+ sums to 1, and a ladder
operator without its Jordan-Wigner sign must be caught."""
import numpy as np
import pytest

import oracle as orc
from paper_1004_3354_amd import workloads as wl

Z = 1j * np.pi * (2 * np.arange(6) + 1) / 8.0


def _aim_h(p):
    ns = p["Ns"]
    h = np.zeros((ns, ns))
    h[0, 0] = p["eps_d"]
    for k, (e, v) in enumerate(zip(p["eps_k"], p["V"])):
        h[k + 1, k + 1] = e
        h[0, k + 1] = h[k + 1, 0] = v
    return h


@pytest.mark.parametrize("spin", [0, 1])
@pytest.mark.parametrize("site", [0, 3])
def test_u0_is_one_body_resolvent(spin, site):
    p = wl.aim(5, 0.0, 0.3, seed=5)
    h = _aim_h(p)
    g, info = orc.green_lehmann(p, 3, 3, spin, site, Z)
    ref = np.array([np.linalg.inv(z * np.eye(p["Ns"]) - h)[site, site] for z in Z])
    assert np.max(np.abs(g - ref)) < 1e-12
    assert abs(info["weights"]["particle"] + info["weights"]["hole"] - 1.0) < 1e-12


def test_hubbard_atom_closed_form():
    U, eps = 4.0, -1.3
    p = wl.aim(0, U, eps, seed=1)
    g_dn, _ = orc.green_lehmann(p, 1, 0, 1, 0, Z)   # add the down electron: E = 2 eps + U
    g_up, _ = orc.green_lehmann(p, 1, 0, 0, 0, Z)   # remove the up electron: E = 0
    assert np.max(np.abs(g_dn - 1.0 / (Z - (eps + U)))) < 1e-14
    assert np.max(np.abs(g_up - 1.0 / (Z - eps))) < 1e-14


def test_spectral_weight_sum_rule_interacting():
    p = wl.kanamori(3, 1, 2.3, 0.4, seed=3)
    g, info = orc.green_lehmann(p, 3, 3, 0, 0, Z)
    assert abs(info["weights"]["particle"] + info["weights"]["hole"] - 1.0) < 1e-12
    # high-frequency tail: z G(z) -> total weight
    gz, _ = orc.green_lehmann(p, 3, 3, 0, 0, np.array([1e6j]))
    assert abs(1e6j * gz[0] - 1.0) < 1e-5


def test_planted_missing_sign_is_caught(monkeypatch):
    p = wl.aim(5, 0.0, 0.3, seed=5)
    h = _aim_h(p)
    real = orc.apply_string

    def unsigned(word, ops):
        r = real(word, ops)
        return None if r is None else (r[0], 1)
    monkeypatch.setattr(orc, "apply_string", unsigned)
    # site 3 sits above occupied modes, so the dropped sign changes matrix elements
    g, _ = orc.green_lehmann(p, 3, 3, 1, 3, Z)
    ref = np.array([np.linalg.inv(z * np.eye(p["Ns"]) - h)[3, 3] for z in Z])
    assert np.max(np.abs(g - ref)) > 1e-3


# ------------------------------------------------ finite temperature (Eq. 3) --

def test_thermal_hubbard_atom_closed_form():
    """One site, four states (0, eps, eps, 2 eps + U): Eq. 3 has two poles with
    weights (1 + e^{-b eps}) / Z and (e^{-b eps} + e^{-b (2 eps + U)}) / Z."""
    U, eps = 4.0, -1.3
    p = wl.aim(0, U, eps, seed=1)
    for b in (0.3, 2.5, 40.0):
        e_lo = min(0.0, eps, 2 * eps + U)          # common shift, cancels in the ratio
        f = lambda E: np.exp(-b * (E - e_lo))
        Zp = f(0.0) + 2 * f(eps) + f(2 * eps + U)
        ref = ((f(0.0) + f(eps)) / (Z - eps) + (f(eps) + f(2 * eps + U)) / (Z - eps - U)) / Zp
        for spin in (0, 1):
            g, _ = orc.green_thermal(p, spin, 0, b, Z)
            assert np.max(np.abs(g - ref)) < 1e-14, (b, spin)


@pytest.mark.parametrize("site", [0, 2])
def test_thermal_u0_is_one_body_resolvent(site):
    """Without interaction the grand-canonical Green function is (z - h)^-1 at
    every temperature."""
    p = wl.aim(3, 0.0, 0.3, seed=5)
    h = _aim_h(p)
    ref = np.array([np.linalg.inv(z * np.eye(p["Ns"]) - h)[site, site] for z in Z])
    for b in (0.5, 7.0):
        g, _ = orc.green_thermal(p, 1, site, b, Z)
        assert np.max(np.abs(g - ref)) < 1e-13, b


def test_thermal_low_temperature_limit():
    """At beta = 300 only the degenerate doublet (N_up, N_dn) = (4, 3), (3, 4)
    of this bath survives (next level 0.089 higher, weight e^-27): the thermal
    sum is the average of the two zero-temperature Lehmann sums."""
    p = wl.aim(5, 3.0, -1.5, seed=2)
    g, _ = orc.green_thermal(p, 0, 0, 300.0, Z)
    ga, ia = orc.green_lehmann(p, 4, 3, 0, 0, Z)
    gb, ib = orc.green_lehmann(p, 3, 4, 0, 0, Z)
    assert abs(ia["E0"] - ib["E0"]) < 1e-12
    assert np.max(np.abs(g - 0.5 * (ga + gb))) < 1e-9


def test_thermal_sum_rule_interacting():
    p = wl.kanamori(3, 1, 2.3, 0.4, seed=3)
    g, _ = orc.green_thermal(p, 0, 0, 10.0, np.array([1e6j]))
    assert abs(1e6j * g[0] - 1.0) < 1e-5


def test_thermal_planted_missing_sign_is_caught(monkeypatch):
    p = wl.aim(3, 0.0, 0.3, seed=5)
    h = _aim_h(p)
    real = orc.ladder_matrix

    def unsigned(src, dst, spin, site, dagger):
        return np.abs(real(src, dst, spin, site, dagger))
    monkeypatch.setattr(orc, "ladder_matrix", unsigned)
    g, _ = orc.green_thermal(p, 1, 2, 0.5, Z)
    ref = np.array([np.linalg.inv(z * np.eye(p["Ns"]) - h)[2, 2] for z in Z])
    assert np.max(np.abs(g - ref)) > 1e-3

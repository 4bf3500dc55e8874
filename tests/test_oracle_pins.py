"""Pins for the FP64 oracle against facts fixed by the paper and by mathematics.

Every check here is independent of the oracle's own code path: printed values
(Fig. 1, the quoted sector dimensions), closed-form spectra (Hubbard atom,
two-site dimer, U=0 filling of one-body levels, Kanamori atomic multiplets),
identities (trace and Frobenius closed forms, Hermiticity, SU(2) multiplets) and
brute force on tiny inputs.  A few tests plant a mistake in the oracle's input
terms and assert that a pin catches it.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle as orc
from paper_1004_3354_amd import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")
def C(n, k):
    return math.comb(n, k) if 0 <= k <= n else 0


def _spec(ns, nup, ndn, terms):
    return np.linalg.eigvalsh(orc.Sector(ns, nup, ndn, terms).dense())


# ------------------------------------------------------------------ basis ----

@pytest.mark.parametrize("ns", [1, 2, 5, 9, 12])
def test_enumeration_is_ascending_fixed_popcount(ns):
    for n in range(ns + 1):
        brute = [s for s in range(1 << ns) if bin(s).count("1") == n]
        assert orc.basis(ns, n).tolist() == brute


def test_enumeration_edges():
    assert orc.basis(32, 0).tolist() == [0]
    assert orc.basis(32, 32).tolist() == [0xFFFFFFFF]
    assert len(orc.basis(20, 10)) == C(20, 10)
    assert orc.basis(32, 1).tolist() == [1 << i for i in range(32)]


def test_paper_sector_dimensions():
    g = json.load(open(os.path.join(GOLD, "paper_dims.json")))
    for e in g["entries"]:
        ns = e["Ns"]
        if ns <= 16:
            d = len(orc.basis(ns, ns // 2)) ** 2
        else:
            d = C(ns, ns // 2) ** 2
        assert d == e["dim"], e["cite"]


# -------------------------------------------------------------- Fig. 1 CSR ----

def test_fig1_csr_arrays():
    g = json.load(open(os.path.join(GOLD, "fig1_csr.json")))
    rc = g["entries_row_col"]
    vals = {tuple(x): 100.0 + 10 * x[0] + x[1] for x in rc}
    rng = np.random.default_rng(1)
    order = rng.permutation(len(rc))
    row, col, val = [], [], []
    for k in order:               # shuffled input, one entry split in two halves
        r, c = rc[k]
        if (r, c) == (4, 0):
            row += [r, r]; col += [c, c]; val += [vals[(r, c)] / 2] * 2
        else:
            row.append(r); col.append(c); val.append(vals[(r, c)])
    row_ind, col_ind, H = orc.coo_to_csr(g["nrows"], row, col, val)
    assert row_ind.tolist() == g["row_ind"]
    assert col_ind.tolist() == g["col_ind"]
    names = ["h%d%d" % (r, c) for r, c in zip(np.repeat(np.arange(6), np.diff(row_ind)), col_ind)]
    assert names == g["H_value_order"]
    assert H.tolist() == [vals[(int(n[1]), int(n[2]))] for n in names]


def test_listing1_spmv_against_dense():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((37, 37)) * (rng.random((37, 37)) < 0.2)
    r, c = np.nonzero(A)
    row_ind, col_ind, H = orc.coo_to_csr(37, r, c, A[r, c])
    x = rng.standard_normal(37)
    np.testing.assert_allclose(orc.spmv(row_ind, col_ind, H, x), A @ x, rtol=1e-14, atol=1e-14)


# ------------------------------------------------------- Jordan-Wigner ----

def test_canonical_anticommutation():
    rng = np.random.default_rng(3)
    for _ in range(300):
        w = int(rng.integers(0, 1 << 12))
        p, q = (int(v) for v in rng.choice(12, 2, replace=False))
        for a, b in (((p, 0), (q, 1)), ((p, 1), (q, 1)), ((p, 0), (q, 0))):
            r1 = orc.apply_string(w, [a, b])
            r2 = orc.apply_string(w, [b, a])
            assert (r1 is None) == (r2 is None)
            if r1 is not None:
                assert r1[0] == r2[0] and r1[1] == -r2[1]
        # {c_p, c+_p} = 1 on every word
        r1 = orc.apply_string(w, [(p, 0), (p, 1)])
        r2 = orc.apply_string(w, [(p, 1), (p, 0)])
        got = (r1[1] if r1 else 0) + (r2[1] if r2 else 0)
        assert got == 1


def test_non_conserving_term_rejected():
    with pytest.raises(ValueError):
        orc.Sector(3, 1, 1, [(1.0, [(0, 1)])]).coo()


# -------------------------------------------------- closed-form spectra ----

def _atom_terms(eps, U):
    return orc.terms_generic(1, [[eps], [eps]], np.zeros((2, 1, 1)), [[U]], np.zeros((2, 1, 1)))


def test_hubbard_atom():
    eps, U = -0.7, 3.1
    T = _atom_terms(eps, U)
    assert np.allclose(_spec(1, 0, 0, T), [0.0])
    assert np.allclose(_spec(1, 1, 0, T), [eps])
    assert np.allclose(_spec(1, 0, 1, T), [eps])
    assert np.allclose(_spec(1, 1, 1, T), [2 * eps + U])
    T2 = orc.terms_aim(U, eps, [], [])
    assert np.allclose(_spec(1, 1, 1, T2), [2 * eps + U])


@pytest.mark.parametrize("t,U", [(1.0, 4.0), (0.5, 2.0), (1.3, 0.0)])
def test_two_site_dimer(t, U):
    T = orc.terms_hubbard(2, 1, t, U, periodic=False)
    ev = _spec(2, 1, 1, T)
    r = math.sqrt(U * U + 16 * t * t)
    np.testing.assert_allclose(ev, sorted([0.0, U, (U - r) / 2, (U + r) / 2]), atol=1e-13)
    if (t, U) == (1.0, 4.0):
        assert abs(ev[0] - (-0.82842712474619)) < 1e-12


def _onebody_aim(p):
    ns = p["Ns"]
    h = np.zeros((ns, ns))
    h[0, 0] = p["eps_d"]
    for k in range(ns - 1):
        h[k + 1, k + 1] = p["eps_k"][k]
        h[0, k + 1] = h[k + 1, 0] = p["V"][k]
    return h


def test_u0_aim_fills_lowest_levels():
    p = wl.aim(7, 0.0, -0.3, seed=11)
    lev = np.linalg.eigvalsh(_onebody_aim(p))
    T = orc.terms_from_model(p)
    for nup, ndn in [(4, 4), (3, 5), (2, 0), (8, 1)]:
        e0 = _spec(8, nup, ndn, T)[0]
        assert abs(e0 - (lev[:nup].sum() + lev[:ndn].sum())) < 1e-12


def test_u0_torus_3x3_and_lanczos():
    T = orc.terms_hubbard(3, 3, 1.0, 0.0)
    h = np.zeros((9, 9))
    for y in range(3):
        for x in range(3):
            i = x + 3 * y
            for j in (((x + 1) % 3) + 3 * y, x + 3 * ((y + 1) % 3)):
                h[i, j] -= 1.0
                h[j, i] -= 1.0
    lev = np.linalg.eigvalsh(h)
    sec = orc.Sector(9, 4, 5, T)
    v0 = wl.uniform_vector(5, sec.D)
    e0, psi, info = orc.lanczos_ground(sec.spmv, v0, tol=1e-13)
    assert abs(e0 - (lev[:4].sum() + lev[:5].sum())) < 1e-11
    r = sec.spmv(psi) - e0 * psi
    assert np.linalg.norm(r) < 1e-8


def _kanamori_atom(U, J, jp_sf, jp_ph, Up=None):
    Up = U - 2 * J if Up is None else Up
    return orc.terms_kanamori(3, 0, U, J, Up, jp_sf, jp_ph, [0.0] * 3, np.zeros((3, 0)), np.zeros((3, 0)))


def _kanamori_pin(T, U, J):
    """Closed-form t2g multiplets for U' = U - 2J, J' = J (rotationally invariant)."""
    want = {
        (1, 1): [U - 3 * J] * 3 + [U - J] * 5 + [U + 2 * J],
        (2, 0): [U - 3 * J] * 3,
        (2, 1): [3 * U - 9 * J] + [3 * U - 6 * J] * 5 + [3 * U - 4 * J] * 3,
        (3, 0): [3 * U - 9 * J],
    }
    ok = True
    for (a, b), ev in want.items():
        got = _spec(3, a, b, T)
        ok &= np.allclose(got, sorted(ev), atol=1e-12)
    return bool(ok)


def test_kanamori_atom_multiplets():
    U, J = 2.3, 0.4
    assert _kanamori_pin(_kanamori_atom(U, J, J, J), U, J)
    got = _spec(3, 1, 1, _kanamori_atom(U, J, J, J))
    np.testing.assert_allclose(got, sorted([1.1] * 3 + [1.9] * 5 + [3.1]), atol=1e-12)


def test_kanamori_atom_density_density_only():
    U, J = 2.3, 0.4
    T = _kanamori_atom(U, J, 0.0, 0.0)
    Up = U - 2 * J
    np.testing.assert_allclose(_spec(3, 1, 1, T), sorted([U] * 3 + [Up] * 6), atol=1e-13)
    np.testing.assert_allclose(_spec(3, 2, 0, T), [Up - J] * 3, atol=1e-13)


def test_planted_xterm_sign_is_caught():
    U, J = 2.3, 0.4
    T = _kanamori_atom(U, J, -J, -J)          # J' with the wrong sign
    assert not _kanamori_pin(T, U, J)
    T = _kanamori_atom(U, J, J, 0.0)          # pair hopping dropped
    assert not _kanamori_pin(T, U, J)
    T = _kanamori_atom(U, J, J, J, Up=U - 2 * J + 0.1)   # wrong U'
    assert not _kanamori_pin(T, U, J)


def test_planted_hop_order_is_caught():
    t, U = 1.0, 4.0
    good = orc.terms_hubbard(2, 1, t, U, periodic=False)
    bad = [(c, list(reversed(ops)) if len(ops) == 2 and ops[0][0] != ops[1][0] else ops)
           for c, ops in good]                # c_j c+_i instead of c+_i c_j
    r = math.sqrt(U * U + 16 * t * t)
    assert abs(_spec(2, 1, 1, good)[0] - (U - r) / 2) < 1e-12
    # c_j c+_i = -c+_i c_j: the reversed strings flip the sign of every hop.  On a
    # bipartite lattice that leaves the spectrum unchanged, on a triangle it does not.
    good3 = orc.terms_hubbard(3, 1, t, 0.0, periodic=True)
    bad3 = [(c, list(reversed(ops)) if ops[0][0] != ops[1][0] else ops) for c, ops in good3]
    h = -t * (np.ones((3, 3)) - np.eye(3))
    lev = np.linalg.eigvalsh(h)
    assert abs(_spec(3, 2, 0, good3)[0] - lev[:2].sum()) < 1e-12
    assert abs(_spec(3, 2, 0, bad3)[0] - lev[:2].sum()) > 1e-3


def test_su2_multiplets_with_bath():
    p = wl.kanamori(3, 1, 2.3, 0.4, seed=7)
    T = orc.terms_from_model(p)
    s44 = _spec(6, 3, 3, T)
    s53 = _spec(6, 4, 2, T)
    s35 = _spec(6, 2, 4, T)
    np.testing.assert_allclose(s53, s35, atol=1e-11)
    # every (5,3) level appears in (4,4)
    for e in s53:
        assert np.min(np.abs(s44 - e)) < 1e-9


# ------------------------------------------------------------ identities ----

def _random_generic(ns, seed, with_x=True):
    rng = np.random.default_rng(seed)
    eps = rng.uniform(-1, 1, (2, ns))
    hop = np.zeros((2, ns, ns))
    for s in range(2):
        a = rng.uniform(-1, 1, (ns, ns)) * (rng.random((ns, ns)) < 0.4)
        a = np.triu(a, 1)
        hop[s] = a + a.T
    w_ud = rng.uniform(0, 2, (ns, ns)) * (rng.random((ns, ns)) < 0.3)
    w_ss = np.zeros((2, ns, ns))
    for s in range(2):
        w_ss[s] = np.triu(rng.uniform(0, 1, (ns, ns)) * (rng.random((ns, ns)) < 0.3), 1)
    xt = []
    if with_x:
        for (m, mp) in [(0, 1), (0, 2), (1, 2)]:
            c1, c2 = rng.uniform(-0.5, 0.5, 2)
            xt += [(orc.SPIN_FLIP, m, mp, c1), (orc.SPIN_FLIP, mp, m, c1),
                   (orc.PAIR_HOP, m, mp, c2), (orc.PAIR_HOP, mp, m, c2)]
    return eps, hop, w_ud, w_ss, xt


@pytest.mark.parametrize("ns,nup,ndn", [(7, 3, 4), (8, 4, 4), (6, 2, 5), (7, 0, 3)])
def test_trace_and_frobenius_closed_forms(ns, nup, ndn):
    eps, hop, w_ud, w_ss, xt = _random_generic(ns, seed=ns * 100 + nup)
    sec = orc.Sector(ns, nup, ndn, orc.terms_generic(ns, eps, hop, w_ud, w_ss, xt))
    A = sec.dense()
    Du, Dd = C(ns, nup), C(ns, ndn)
    tr = (Dd * eps[0].sum() * C(ns - 1, nup - 1) + Du * eps[1].sum() * C(ns - 1, ndn - 1)
          + w_ud.sum() * C(ns - 1, nup - 1) * C(ns - 1, ndn - 1)
          + Dd * np.triu(w_ss[0], 1).sum() * C(ns - 2, nup - 2)
          + Du * np.triu(w_ss[1], 1).sum() * C(ns - 2, ndn - 2))
    assert abs(np.trace(A) - tr) < 1e-10 * max(1, abs(tr))
    off = A - np.diag(np.diag(A))
    fro = (Dd * (hop[0] ** 2).sum() * C(ns - 2, nup - 1)
           + Du * (hop[1] ** 2).sum() * C(ns - 2, ndn - 1)
           + sum(c * c for (_, _, _, c) in xt) * C(ns - 2, nup - 1) * C(ns - 2, ndn - 1))
    assert abs((off ** 2).sum() - fro) < 1e-10 * max(1, fro)


def test_hermiticity_and_adjoint_rows():
    ns = 7
    eps, hop, w_ud, w_ss, xt = _random_generic(ns, seed=5)
    sec = orc.Sector(ns, 3, 3, orc.terms_generic(ns, eps, hop, w_ud, w_ss, xt))
    A = sec.dense()
    assert np.array_equal(A, A.T)
    rows = np.arange(sec.D)
    x = wl.uniform_vector(9, sec.D)
    np.testing.assert_allclose(sec.rows_apply(rows, x), A @ x, rtol=1e-13, atol=1e-13)
    # a non-Hermitian term set: forward build is not symmetric, adjoint rows still agree
    nh = orc.Sector(ns, 3, 3, [(0.7, [(0, 1), (1, 0)])] + sec.terms)
    B = nh.dense()
    assert not np.array_equal(B, B.T)
    np.testing.assert_allclose(nh.rows_apply(rows, x), B @ x, rtol=1e-13, atol=1e-13)


def test_particle_number_conserved_per_spin():
    p = wl.kanamori(3, 2, 2.3, 0.4, seed=3)
    T = orc.terms_from_model(p)
    for (a, b) in [(0, 0), (4, 4), (9, 9), (2, 7)]:
        sec = orc.Sector(9, a, b, T)
        r, c, v = sec.coo()       # raises if any term leaves the sector
        assert r.max(initial=0) < sec.D and c.max(initial=0) < sec.D


def test_onebody_table_pins():
    rng = np.random.default_rng(4)
    ns, n = 9, 4
    a = np.triu(rng.uniform(-1, 1, (ns, ns)) * (rng.random((ns, ns)) < 0.5), 1)
    h = a + a.T
    off, tgt, sgn, amp = orc.onebody_table(ns, n, h)
    npairs = int((h != 0).sum())
    assert len(tgt) == npairs * C(ns - 2, n - 1)
    # symmetric: r -> t with (sign, h_ij) iff t -> r with the same sign and h_ji
    ent = {}
    for r in range(len(off) - 1):
        for k in range(off[r], off[r + 1]):
            ent[(r, int(tgt[k]))] = (int(sgn[k]), float(amp[k]))
        assert list(tgt[off[r]:off[r + 1]]) == sorted(tgt[off[r]:off[r + 1]])
    for (r, t), (s, v) in ent.items():
        assert ent[(t, r)] == (s, v)
    # with no down electrons the sector matrix is exactly this table
    sec = orc.Sector(ns, n, 0, orc.terms_generic(ns, np.zeros((2, ns)), np.stack([h, h]),
                                                 np.zeros((ns, ns)), np.zeros((2, ns, ns))))
    A = sec.dense()
    B = np.zeros_like(A)
    for (r, t), (s, v) in ent.items():
        B[t, r] += s * v
    assert np.array_equal(A, B)


def test_oracle_lanczos_vs_dense_config0():
    p, sectors = wl.config(0)
    sec = orc.sector_for(p, *sectors[0])
    assert sec.D == 4900
    ev = np.linalg.eigvalsh(sec.dense())
    e0, psi, info = orc.lanczos_ground(sec.spmv, wl.gaussian_vector(wl.start_vector_seed(0), sec.D),
                                       tol=1e-13)
    assert abs(e0 - ev[0]) < 1e-11 * max(1, abs(ev[0]))
    lk = orc.lowest_k(sec, 4)
    np.testing.assert_allclose(lk, ev[:4], atol=1e-11)


def test_arpack_path_matches_dense():
    p = wl.kanamori(3, 2, 2.3, 0.4, seed=9)
    sec = orc.sector_for(p, 3, 2)
    ev = np.linalg.eigvalsh(sec.dense())
    lk = orc.lowest_k(sec, 3, dense_limit=0)
    np.testing.assert_allclose(lk, ev[:3], atol=1e-10)


def test_splitmix64_published_vector():
    # First outputs of SplitMix64 from state 1234567 as printed by the reference
    # C implementation's well-known test (Vigna): computed here by the plain
    # recurrence on Python integers, independently of the numpy vectorisation.
    M = (1 << 64) - 1
    x = 1234567
    want = []
    for _ in range(5):
        x = (x + 0x9E3779B97F4A7C15) & M
        z = x
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        want.append(z ^ (z >> 31))
    got = wl.splitmix64(1234567, np.arange(5)).tolist()
    assert got == want
    assert want[0] == 6457827717110365317

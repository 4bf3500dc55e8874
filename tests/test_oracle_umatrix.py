"""Pins of the oracle's general opposite-spin two-body term
c+_{i up} c+_{j dn} c_{l dn} c_{k up} (an element U_ijkl of a full U-matrix):
special index sets reduce to the terms the paper writes out (spin flip, pair
hopping, density-density), and a Hermitian set gives a symmetric matrix."""
import numpy as np

import oracle as orc

NS = 4


def _dense(xterms, w_ud=None, nup=2, ndn=2):
    z = np.zeros
    T = orc.terms_generic(NS, z(2 * NS), z((2, NS, NS)), z((NS, NS)) if w_ud is None else w_ud,
                          z((2, NS, NS)), xterms)
    return orc.Sector(NS, nup, ndn, T).dense()


def test_spin_flip_is_a_general_term():
    # d+_{m up} d_{m dn} d+_{m' dn} d_{m' up} = -c+_{m up} c+_{m' dn} c_{m dn} c_{m' up}
    for (m, mp) in [(0, 1), (2, 0), (1, 3)]:
        a = _dense([(orc.SPIN_FLIP, m, mp, 0.7)])
        b = _dense([(orc.UD_GENERAL, m, mp, mp, m, -0.7)])
        assert np.array_equal(a, b) and np.abs(a).sum() > 0


def test_pair_hopping_is_a_general_term():
    # d+_{m up} d+_{m dn} d_{m' up} d_{m' dn} = -c+_{m up} c+_{m dn} c_{m' dn} c_{m' up}
    for (m, mp) in [(0, 1), (3, 1)]:
        a = _dense([(orc.PAIR_HOP, m, mp, 0.45)])
        b = _dense([(orc.UD_GENERAL, m, m, mp, mp, -0.45)])
        assert np.array_equal(a, b) and np.abs(a).sum() > 0


def test_density_density_is_a_general_term():
    for (i, j) in [(0, 0), (1, 3), (3, 2)]:
        w = np.zeros((NS, NS))
        w[i, j] = 1.3
        assert np.array_equal(_dense([(orc.UD_GENERAL, i, j, i, j, 1.3)]), _dense([], w_ud=w))


def test_hermitian_set_is_symmetric_and_one_sided_is_not():
    rng = np.random.default_rng(4)
    xt = []
    for _ in range(8):
        i, j, k, l = (int(v) for v in rng.integers(0, NS, 4))
        c = float(rng.uniform(-1, 1))
        xt += [(orc.UD_GENERAL, i, j, k, l, c), (orc.UD_GENERAL, k, l, i, j, c)]
    H = _dense(xt, nup=2, ndn=3)
    assert np.max(np.abs(H - H.T)) < 1e-15 and np.abs(H).sum() > 0
    H1 = _dense([(orc.UD_GENERAL, 0, 1, 2, 3, 0.5)], nup=2, ndn=2)   # hermitian partner missing
    assert np.max(np.abs(H1 - H1.T)) > 0.1

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


def test_same_spin_term_reduces_to_density_and_hops():
    """For j distinct from i and k the same-spin string with l = j is
    c+_i c+_j c_j c_k = c+_i n_j c_k = c+_i c_k n_j, a density-assisted hop;
    with its Hermitian partner the matrix is symmetric."""
    i, j, k = 0, 2, 3
    for t, sp in ((orc.UU_GENERAL, 0), (orc.DD_GENERAL, 1)):
        a = _dense([(t, i, j, k, j, 0.8), (t, k, j, i, j, 0.8)], nup=2, ndn=2)
        z = np.zeros
        T = [(0.8, [(orc._mode(i, sp, NS), 1), (orc._mode(k, sp, NS), 0)] + orc._number(orc._mode(j, sp, NS))),
             (0.8, [(orc._mode(k, sp, NS), 1), (orc._mode(i, sp, NS), 0)] + orc._number(orc._mode(j, sp, NS)))]
        b = orc.Sector(NS, 2, 2, T).dense()
        assert np.array_equal(a, b) and np.abs(a).sum() > 0
        assert np.max(np.abs(a - a.T)) == 0.0


def test_same_spin_pair_antisymmetry():
    """Swapping the two creators (or the two annihilators) flips the sign."""
    H1 = _dense([(orc.UU_GENERAL, 0, 1, 2, 3, 0.5), (orc.UU_GENERAL, 2, 3, 0, 1, 0.5)], nup=2, ndn=1)
    H2 = _dense([(orc.UU_GENERAL, 1, 0, 2, 3, -0.5), (orc.UU_GENERAL, 2, 3, 1, 0, -0.5)], nup=2, ndn=1)
    assert np.array_equal(H1, H2) and np.abs(H1).sum() > 0

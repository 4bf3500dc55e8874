"""GPU parity of the sector basis, hop tables and matrix-free H.v against the oracle.

Integer results (states, ranks, hop tables) must match bit for bit.  H.v must
agree element by element within the rounding bound of the precision used:
|y_gpu - y_oracle| <= (n_terms + 8) u (|H|_abs |x|), with u = 2^-53 (FP64) or
2^-24 (FP32), where |H|_abs is the oracle matrix of the absolute values of the
individual operator terms and the FP32 case feeds the oracle the same FP32
input values.  Sizes span several LDS row tiles and 64-state slices with ragged
tails; every compiled apply schedule that fits is checked.
"""
import math

import numpy as np
import pytest

import oracle as orc
from gpu_common import U32, U64, abs_apply, bound, build, generic_model, generic_terms, gpu_ed, sector
from paper_1004_3354_amd import models, workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda"

SMALL = [
    ("aim8", wl.config(0)[0], (4, 4)),
    ("aim8_35", wl.aim(7, 2.0, -1.0, seed=5), (3, 5)),
    ("hub3x3", wl.hubbard(3, 3, 1.0, 4.0), (4, 5)),
    ("hub4x2_open", wl.hubbard(4, 2, 1.0, 3.0, periodic=False), (4, 3)),
    ("kan9", wl.kanamori(3, 2, 2.3, 0.4, seed=3), (4, 5)),
    ("kan9_jpoff", wl.kanamori(3, 2, 2.3, 0.4, seed=3, jprime=False), (4, 4)),
    ("kan12_66", wl.config(3)[0], (6, 6)),
    ("kan12_57", wl.config(3)[0], (5, 7)),
    # wide down-spin rows: several LDS windows per row (top-bit runs)
    ("hub4x4_1_8", wl.hubbard(4, 4, 1.0, 4.0), (1, 8)),
    ("hub4x4_2_7", wl.hubbard(4, 4, 1.0, 4.0), (2, 7)),
    ("kan18_1_9", wl.config(4)[0], (1, 9)),
]

EDGE = [
    ("kan12_0_7", wl.config(3)[0], (0, 7)),
    ("kan12_12_5", wl.config(3)[0], (12, 5)),
    ("kan12_1_0", wl.config(3)[0], (1, 0)),
    ("kan12_0_0", wl.config(3)[0], (0, 0)),
    ("kan12_12_12", wl.config(3)[0], (12, 12)),
    ("atom1", wl.aim(0, 3.0, -0.5, seed=1), (1, 1)),
    ("hub3x3_U0", wl.hubbard(3, 3, 1.0, 0.0), (2, 7)),
]


def _x(n, seed):
    return wl.uniform_vector(seed, n)


def _apply_and_check(H, sec, sec_abs, x64, prec, variants):
    ed = gpu_ed()
    dt = torch.float64 if prec == ed.ED_FP64 else torch.float32
    xd = torch.from_numpy(x64).to(DEV, dt)
    xin = xd.double().cpu().numpy()          # the values the GPU actually reads
    y_ref = sec.spmv(xin)
    ahx = abs_apply(sec_abs, np.abs(xin))
    row_ind = sec_abs.csr()[0]
    nterm = int(np.max(np.diff(row_ind))) if len(row_ind) > 1 else 1
    tol = bound(ahx, nterm, U64 if prec == ed.ED_FP64 else U32)
    checked = 0
    for v in variants:
        if not H.variant_fits(v):
            continue
        yd = torch.full_like(xd, float("nan"))
        H.apply_variant(v, xd, yd)
        torch.cuda.synchronize()
        y = yd.double().cpu().numpy()
        err = np.abs(y - y_ref)
        bad = np.nonzero(~(err <= tol))[0]
        assert bad.size == 0, "variant %s: %d elements out of bound, first %d: %r vs %r (tol %g)" % (
            ed.variant_name(v), bad.size, bad[0], y[bad[0]], y_ref[bad[0]], tol[bad[0]])
        checked += 1
    assert checked > 0
    return checked


@pytest.mark.parametrize("name,phys,sec_nn", SMALL + EDGE, ids=[c[0] for c in SMALL + EDGE])
def test_basis_and_hop_tables_bitexact(name, phys, sec_nn):
    ed = gpu_ed()
    nup, ndn = sec_nn
    b, H = build(phys, nup, ndn, ed.ED_FP64)
    ns = int(phys["Ns"])
    p = models.params_from_model(phys)
    for s, n in ((0, nup), (1, ndn)):
        assert np.array_equal(b.states(s), orc.basis(ns, n))
        off, tgt, sgn, amp = H.hop_table(s)
        o_off, o_tgt, o_sgn, o_amp = orc.onebody_table(ns, n, p["hop"][s])
        assert np.array_equal(off, o_off)
        assert np.array_equal(tgt.astype(np.int64), o_tgt)
        assert np.array_equal(sgn, o_sgn)
        assert np.array_equal(amp, o_amp)


@pytest.mark.parametrize("ns,n", [(12, 6), (18, 9), (32, 1), (20, 3), (5, 0), (5, 5), (32, 31)])
def test_rank_bitexact(ns, n):
    ed = gpu_ed()
    b = ed.Basis(ns, n, 0)
    rng = np.random.default_rng(ns * 100 + n)
    if math.comb(ns, n) <= 200000:
        st = orc.basis(ns, n)
        want = np.arange(len(st), dtype=np.int64)
    else:
        st = np.unique(b.states(0)[rng.integers(0, b.dup, 5000)])
        want = np.searchsorted(b.states(0), st).astype(np.int64)
        assert np.array_equal(b.states(0)[want], st)
    junk = rng.integers(0, 2 ** 32, 3000, dtype=np.uint64).astype(np.uint32)
    pc = np.array([bin(int(v)).count("1") for v in junk])
    ok = (pc == n) & ((junk.astype(np.uint64) >> np.uint64(ns)) == 0)
    allst = np.concatenate([st, junk])
    sd = torch.from_numpy(allst.view(np.int32).copy()).to(DEV)
    rd = torch.empty(len(allst), dtype=torch.int64, device=DEV)
    b.rank(0, sd, rd)
    r = rd.cpu().numpy()
    assert np.array_equal(r[:len(st)], want)
    assert np.all(r[len(st):][~ok] == -1)
    if ok.any():
        full = b.states(0)
        assert np.array_equal(full[r[len(st):][ok]], junk[ok])


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("name,phys,sec_nn", SMALL + EDGE, ids=[c[0] for c in SMALL + EDGE])
def test_apply_parity_all_schedules(name, phys, sec_nn, prec):
    ed = gpu_ed()
    nup, ndn = sec_nn
    b, H = build(phys, nup, ndn, prec)
    sec = sector(phys, nup, ndn)
    sec_abs = sector(phys, nup, ndn, absval=True)
    x = _x(sec.D, 77 + nup * 13 + ndn)
    _apply_and_check(H, sec, sec_abs, x, prec, range(ed.variant_count()))


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("ns,nup,ndn,seed", [(7, 3, 4, 1), (9, 4, 4, 2), (10, 5, 3, 3)])
def test_apply_parity_generic_model(ns, nup, ndn, seed, prec):
    ed = gpu_ed()
    p = generic_model(ns, seed)
    b = ed.Basis(ns, nup, ndn)
    H = ed.Hamiltonian(p, b, prec)
    T = generic_terms(p)
    sec = orc.Sector(ns, nup, ndn, T)
    sec_abs = orc.Sector(ns, nup, ndn, [(abs(c), ops) for c, ops in T])
    _apply_and_check(H, sec, sec_abs, _x(sec.D, seed), prec, range(ed.variant_count()))


def test_apply_tuned_default_and_determinism():
    ed = gpu_ed()
    phys, sectors = wl.config(3)
    b, H = build(phys, 6, 6, ed.ED_FP32)
    x = torch.from_numpy(_x(b.D, 5)).to(DEV, torch.float32)
    y1 = torch.empty_like(x)
    y2 = torch.empty_like(x)
    H.apply(x, y1)
    v = H.current_variant()
    assert 0 <= v < ed.variant_count()
    H.apply(x, y2)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    y3 = torch.empty_like(x)
    H.apply_variant(v, x, y3)
    torch.cuda.synchronize()
    assert torch.equal(y1, y3)


def test_hermiticity_fp64():
    ed = gpu_ed()
    phys = wl.config(3)[0]
    b, H = build(phys, 5, 6, ed.ED_FP64)
    u = torch.from_numpy(_x(b.D, 1)).to(DEV)
    v = torch.from_numpy(_x(b.D, 2)).to(DEV)
    hu, hv = torch.empty_like(u), torch.empty_like(v)
    H.apply(u, hu)
    H.apply(v, hv)
    a = float(torch.dot(u, hv))
    c = float(torch.dot(hu, v))
    assert abs(a - c) <= 1e-13 * max(abs(a), 1.0) * math.sqrt(b.D)


def test_fill_random_matches_host_generator():
    ed = gpu_ed()
    n = 100003
    x = torch.empty(n, dtype=torch.float64, device=DEV)
    ed.fill_random(x, 4242, 0)
    assert np.array_equal(x.cpu().numpy(), wl.uniform_vector(4242, n))
    x32 = torch.empty(n, dtype=torch.float32, device=DEV)
    ed.fill_random(x32, 4242, 0)
    assert np.array_equal(x32.cpu().numpy(), wl.uniform_vector(4242, n).astype(np.float32))
    ed.fill_random(x, 99, 1)
    np.testing.assert_allclose(x.cpu().numpy(), wl.gaussian_vector(99, n), rtol=1e-14, atol=1e-14)


def test_rayleigh_fp64_on_fp32_storage():
    ed = gpu_ed()
    phys = wl.kanamori(3, 2, 2.3, 0.4, seed=3)
    b, H = build(phys, 4, 5, ed.ED_FP32)
    sec = sector(phys, 4, 5)
    x32 = torch.from_numpy(_x(b.D, 3)).to(DEV, torch.float32)
    xv = x32.double().cpu().numpy()
    hx = sec.spmv(xv)
    rq_ref = xv @ hx / (xv @ xv)
    res_ref = np.linalg.norm(hx - rq_ref * xv) / np.linalg.norm(xv)
    rq, res = H.rayleigh(x32)
    assert abs(rq - rq_ref) <= 1e-13 * max(1.0, abs(rq_ref))
    assert abs(res - res_ref) <= 1e-10 * res_ref


def test_errors_reported():
    ed = gpu_ed()
    phys = wl.config(0)[0]
    b, H = build(phys, 4, 4, ed.ED_FP64)
    x = torch.zeros(b.D, dtype=torch.float64, device=DEV)
    with pytest.raises(ed.EDError):
        H.apply(x, x)
    bad = models.params_from_model(phys)
    bad["hop"][0, 0, 1] += 1e-3          # not symmetric
    with pytest.raises(ed.EDError):
        ed.Hamiltonian(bad, b, ed.ED_FP64)
    bad = models.params_from_model(wl.kanamori(3, 1, 2.3, 0.4, seed=1))
    bad["xterms"] = bad["xterms"][:-1]   # no longer Hermitian
    b6 = ed.Basis(6, 3, 3)
    with pytest.raises(ed.EDError):
        ed.Hamiltonian(bad, b6, ed.ED_FP64)
    with pytest.raises(ed.EDError):
        H.workspace_bytes(None, k=b.D + 1)


# ------------------------------------------------------------ grouped order --
# Models whose one-spin move graphs split into components (each orbital of the
# three-orbital impurity hops only to its own bath levels): the library keeps a
# twin handle with the basis ordered by component.  Its H.v, in that order,
# must be the same operator: x is converted to the grouped order, multiplied
# with every schedule that fits the twin, converted back and compared with the
# oracle's product in rank order.
GROUPED = [c for c in SMALL + EDGE if c[0].startswith("kan")]


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("name,phys,sec_nn", GROUPED, ids=[c[0] for c in GROUPED])
def test_grouped_apply_parity_all_schedules(name, phys, sec_nn, prec):
    _grouped_parity(phys, sec_nn, prec, name)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("name,phys,sec_nn", GROUPED[:3], ids=[c[0] for c in GROUPED[:3]])
def test_grouped_apply_parity_wide_entries(name, phys, sec_nn, prec, monkeypatch):
    """The tile kernel's 32-bit hop entries (the form the N_s = 18 windows
    need) on the small sectors, which otherwise take the 16-bit form."""
    monkeypatch.setenv("ED_TILE_ENTRY_BITS", "32")
    _grouped_parity(phys, sec_nn, prec, name, prefix="gt_")


def _grouped_parity(phys, sec_nn, prec, name, prefix=None):
    ed = gpu_ed()
    nup, ndn = sec_nn
    b, H = build(phys, nup, ndn, prec)
    G = H.grouped()
    # the twin exists exactly when a one-spin move graph has several components
    ns = int(phys["Ns"])
    p = models.params_from_model(phys)
    split = any(_components(*orc.onebody_table(ns, n, p["hop"][s])[:2]) > 1 for s, n in ((0, nup), (1, ndn)))
    assert (G is not None) == split, (name, split)
    if G is None:
        return
    assert G.D == H.D
    sec = sector(phys, nup, ndn)
    sec_abs = sector(phys, nup, ndn, absval=True)
    dt = torch.float64 if prec == ed.ED_FP64 else torch.float32
    xd = torch.from_numpy(_x(sec.D, 91 + nup * 13 + ndn)).to(DEV, dt)
    xin = xd.double().cpu().numpy()
    y_ref = sec.spmv(xin)
    ahx = abs_apply(sec_abs, np.abs(xin))
    nterm = int(np.max(np.diff(sec_abs.csr()[0]))) if sec.D > 0 else 1
    tol = bound(ahx, nterm, U64 if prec == ed.ED_FP64 else U32)
    xg = torch.empty_like(xd)
    H.to_grouped(xd, xg)
    checked = 0
    for v in range(ed.variant_count()):
        if not G.variant_fits(v) or (prefix and not ed.variant_name(v).startswith(prefix)):
            continue
        yg = torch.full_like(xd, float("nan"))
        G.apply_variant(v, xg, yg)
        y = torch.empty_like(xd)
        H.from_grouped(yg, y)
        torch.cuda.synchronize()
        err = np.abs(y.double().cpu().numpy() - y_ref)
        bad = np.nonzero(~(err <= tol))[0]
        assert bad.size == 0, "variant %s: %d elements out of bound" % (ed.variant_name(v), bad.size)
        checked += 1
    assert checked >= 2
    # a grouped-only schedule fits every such twin
    assert any(ed.variant_name(v).startswith(("grp", "gt")) and G.variant_fits(v) for v in range(ed.variant_count()))


def _components(off, tgt):
    """Number of connected components of a one-spin hop graph (CSR)."""
    n = len(off) - 1
    par = list(range(n))

    def find(a):
        while par[a] != a:
            par[a] = par[par[a]]
            a = par[a]
        return a
    for i in range(n):
        for e in range(off[i], off[i + 1]):
            a, b = find(i), find(int(tgt[e]))
            if a != b:
                par[max(a, b)] = min(a, b)
    return len({find(i) for i in range(n)})


@pytest.mark.parametrize("name,phys,sec_nn", GROUPED[:4], ids=[c[0] for c in GROUPED[:4]])
def test_grouped_order_and_tables(name, phys, sec_nn):
    """The grouped order is a permutation that orders each component's states
    by hop count (descending), then by the occupation of the sites the
    four-fermion terms move that spin between, then rank; every hop of the twin
    stays inside its component, and the twin's hop table translated back to
    ranks is the oracle's (bit for bit, per row as a set of (target, sign,
    amplitude))."""
    ed = gpu_ed()
    nup, ndn = sec_nn
    ns = int(phys["Ns"])
    b, H = build(phys, nup, ndn, ed.ED_FP64)
    G = H.grouped()
    p = models.params_from_model(phys)
    for s, n in ((0, nup), (1, ndn)):
        perm = G.grouped_order(s).astype(np.int64)
        D = len(perm)
        assert np.array_equal(np.sort(perm), np.arange(D))
        off, tgt, sgn, amp = G.hop_table(s)
        o_off, o_tgt, o_sgn, o_amp = orc.onebody_table(ns, n, p["hop"][s])
        # components = connected sets of positions under the twin's hops
        comp = np.arange(D)
        for _ in range(D):
            changed = False
            for i in range(D):
                for e in range(off[i], off[i + 1]):
                    m = min(comp[i], comp[tgt[e]])
                    if comp[i] != m or comp[tgt[e]] != m:
                        comp[i] = comp[tgt[e]] = m
                        changed = True
            if not changed:
                break
        # contiguous components; inside each, more hops first, then the
        # four-fermion sites' occupation, then ascending rank
        fmask = 0
        for x in p["xterms"]:
            if x[0] == orc.UD_GENERAL:   # c+_{i up} c+_{j dn} c_{l dn} c_{k up}: up k -> i, down l -> j
                _, i, j, k, l, _ = x
                fmask |= (1 << k) | (1 << i) if s == 0 else (1 << l) | (1 << j)
            elif x[0] in (orc.SPIN_FLIP, orc.PAIR_HOP):   # both spins between m and m'
                fmask |= (1 << x[1]) | (1 << x[2])
        occ = (orc.basis(ns, n).astype(np.int64) & fmask)[perm]
        starts = np.nonzero(np.r_[True, comp[1:] != comp[:-1]])[0]
        assert len(np.unique(comp)) == len(starts)
        nh = np.diff(o_off)[perm]
        for a, z in zip(starts, np.r_[starts[1:], D]):
            key = list(zip((-nh[a:z]).tolist(), occ[a:z].tolist(), perm[a:z].tolist()))
            assert key == sorted(key)
        for i in range(D):
            r = perm[i]
            mine = sorted(zip(perm[tgt[off[i]:off[i + 1]]].tolist(), sgn[off[i]:off[i + 1]].tolist(),
                              amp[off[i]:off[i + 1]].tolist()))
            want = sorted(zip(o_tgt[o_off[r]:o_off[r + 1]].tolist(), o_sgn[o_off[r]:o_off[r + 1]].tolist(),
                              o_amp[o_off[r]:o_off[r + 1]].tolist()))
            assert mine == want, (s, i, r)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_solver_layouts_agree(prec):
    """The default solver path iterates on the grouped twin; the rank-order
    path gives the same ground state (energy and vector up to sign)."""
    ed = gpu_ed()
    phys, _ = wl.config(3)
    b, H = build(phys, 6, 6, prec)
    dt = torch.float64 if prec == 0 else torch.float32
    v0 = torch.empty(H.D, dtype=dt, device=DEV)
    ed.fill_random(v0, 5, 1)
    out = []
    for layout in (0, 1):
        psi = torch.empty_like(v0)
        e, info = H.lanczos_ground(v0, ed.options(tol=1e-12 if prec == 0 else 1e-7, layout=layout), psi=psi)
        out.append((e, psi.double()))
    (e0, p0), (e1, p1) = out
    tol = 1e-10 if prec == 0 else 1e-6
    assert abs(e0 - e1) <= tol * max(1.0, abs(e1))
    ov = abs(float(torch.dot(p0, p1))) / float(p0.norm() * p1.norm())
    assert ov >= 1.0 - (1e-10 if prec == 0 else 1e-5), ov

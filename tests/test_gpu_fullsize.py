"""H.v at the benchmark's full sector sizes (N_s = 15, 16, 18), in the tuned
schedule bench.py times, checked on sampled output elements.

x is the SplitMix64 uniform stream filled on the device; the oracle
regenerates x at exactly the columns each sampled row needs (bit-identical
generator), builds that row literally from the operator strings without
storing H, and the GPU value must lie within the rounding bound
(n_terms + 8) u sum_k |h_k x_k| of the precision used.  Sampled rows cover
the first and last rows, LDS-window and 64-state slice boundaries, and random
rows; the full matrix does not fit a CPU host at these sizes."""
import math

import numpy as np
import pytest

import oracle as orc
from gpu_common import U32, U64, build, gpu_ed
from paper_1004_3354_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
SEED = 20240501


def _rows(dup, ddn, ns, ndn, rng, nrand=1500):
    us = sorted({0, 1, dup // 2, dup - 2, dup - 1} | set(rng.integers(0, dup, 40).tolist()))
    edges = {0, 1, 63, 64, 65, ddn - 1, ddn - 2}
    for k in (1, 2, 3):        # runs of states sharing their top k bits
        for j in range(0, k + 1):
            e = sum(math.comb(ns - k, ndn - i) for i in range(j)) if j else 0
            edges |= {e - 1, e, e + 1}
    edges = sorted(v for v in edges if 0 <= v < ddn)
    rows = [u * ddn + d for u in us for d in edges]
    rows += rng.integers(0, dup * ddn, nrand).tolist()
    return np.unique(np.array(rows, dtype=np.int64))


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("cfg", [2, 1, 4], ids=["ns15", "ns16_4x4", "ns18"])
def test_fullsize_sampled_rows(cfg, prec):
    ed = gpu_ed()
    phys, sectors = wl.config(cfg)
    nup, ndn = sectors[0]
    b, H = build(phys, nup, ndn, prec)
    dt = torch.float64 if prec == 0 else torch.float32
    x = torch.empty(b.D, dtype=dt, device="cuda")
    ed.fill_random(x, SEED + cfg, 0)
    y = torch.empty_like(x)
    H.apply(x, y)                       # first call tunes the schedule, like bench.py
    H.apply(x, y)
    torch.cuda.synchronize()
    rng = np.random.default_rng(cfg)
    rows = _rows(b.dup, b.ddn, int(phys["Ns"]), ndn, rng)
    yg = y[torch.from_numpy(rows).cuda()].double().cpu().numpy()
    sched = ed.variant_name(H.current_variant())
    del x, y
    torch.cuda.empty_cache()
    sec = orc.sector_for(phys, nup, ndn)
    u = U64 if prec == 0 else U32
    worst = 0.0
    for J, g in zip(rows, yg):
        cols, vals = sec.row_entries(int(J))
        xv = wl.uniform_at(SEED + cfg, cols.astype(np.uint64))
        if prec == 1:
            xv = xv.astype(np.float32).astype(np.float64)
        ref = float(np.dot(vals, xv))
        tol = (len(cols) + 8) * u * float(np.dot(np.abs(vals), np.abs(xv))) + 1e-300
        worst = max(worst, abs(g - ref) / tol)
        assert abs(g - ref) <= tol, (int(J), g, ref, tol, sched)
    print("cfg%d prec%d schedule %s: %d rows, worst err/bound %.3f" % (cfg, prec, sched, len(rows), worst))


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_fullsize_general_terms_sampled_rows(prec):
    """The N_s = 15 workload plus general U-matrix elements (opposite- and
    same-spin, on impurity and bath sites), sampled rows in the tuned schedule."""
    from paper_1004_3354_amd import models
    ed = gpu_ed()
    phys, sectors = wl.config(2)
    nup, ndn = sectors[0]
    ns = int(phys["Ns"])
    p = models.params_from_model(phys)
    xt = list(p.get("xterms", []))
    for (t, i, j, k, l, c) in [(3, 0, 1, 2, 0, 0.21), (3, 1, 5, 9, 1, -0.13), (3, 2, 2, 0, 0, 0.08),
                               (4, 0, 1, 2, 9, 0.11), (5, 1, 2, 0, 5, -0.07), (4, 0, 3, 0, 7, 0.05)]:
        xt += [(t, i, j, k, l, c), (t, k, l, i, j, c)]
    p = dict(p, xterms=xt)
    b = ed.Basis(ns, nup, ndn)
    H = ed.Hamiltonian(p, b, prec)
    dt = torch.float64 if prec == 0 else torch.float32
    x = torch.empty(b.D, dtype=dt, device="cuda")
    ed.fill_random(x, SEED + 7, 0)
    y = torch.empty_like(x)
    H.apply(x, y)
    H.apply(x, y)
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    rows = _rows(b.dup, b.ddn, ns, ndn, rng, nrand=800)
    yg = y[torch.from_numpy(rows).cuda()].double().cpu().numpy()
    sched = ed.variant_name(H.current_variant())
    del x, y
    torch.cuda.empty_cache()
    sec = orc.Sector(ns, nup, ndn, orc.terms_generic(ns, p["eps"], p["hop"], p["w_ud"], p["w_ss"], xt))
    u = U64 if prec == 0 else U32
    for J, g in zip(rows, yg):
        cols, vals = sec.row_entries(int(J))
        xv = wl.uniform_at(SEED + 7, cols.astype(np.uint64))
        if prec == 1:
            xv = xv.astype(np.float32).astype(np.float64)
        ref = float(np.dot(vals, xv))
        tol = (len(cols) + 8) * u * float(np.dot(np.abs(vals), np.abs(xv))) + 1e-300
        assert abs(g - ref) <= tol, (int(J), g, ref, tol, sched)

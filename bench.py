"""Benchmark: matrix-free H.v GB/s (fraction of HBM peak) and time to the Lanczos
ground-state energy, FP32-mixed vs FP64, on one MI355X.

A timed step is one FP32 H.v over the N_s = 15 three-orbital impurity sector
(3 orbitals + 12 bath levels, N_up = N_dn = 7, D = 6435^2 = 41,409,225) with x
and y resident in HBM.  value = algorithmic bytes (read x + write y = 8 D) per
step / step time.  Besides the JSON fields of the common contract the line
carries: roofline (dominant kernel = the apply), cpu_baseline (the FP64 oracle
on the host cores, matrix-free literal rows on a bounded sample), fp64 H.v,
FP32 H.v at N_s = 18 (D = 48620^2), and time-to-E0 for both precisions from
the same start vector with the same residual target at N_s = 15 and N_s = 18
(the N_s = 18 pair takes about two minutes; --no-e0-ns18 skips it).

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-e0] [--no-cpu]
                       [--no-ns18] [--no-e0-ns18]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("apply.hip", "ed_internal.h", "tables.hip"):
        h.update(open(os.path.join(ROOT, "paper_1004_3354_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profile(workload, schedule):
    """HBM bytes per launch measured by rocprofv3 counters for this exact kernel
    source and schedule (profiles/apply_traffic.json), else None."""
    p = os.path.join(ROOT, "profiles", "apply_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except ValueError:
        return None
    e = d.get(workload)
    if not e or e.get("source_hash") != kernel_source_hash() or e.get("schedule") != schedule:
        return None
    return e.get("bytes_per_launch")


# ---- rocprofv3 summaries (the figures committed under profiles/) -----------
APPLY_KERNELS = ("k_apply", "k_cs<", "k_csb<", "k_rt<", "k_upb<", "k_upt<", "k_gtile<")


def summarize_stats(path):
    """Per-kernel dispatch count and average duration from a rocprofv3
    --kernel-trace --stats run (kernel_stats.csv), largest total first."""
    import csv
    out = []
    for r in csv.DictReader(open(path)):
        name = r.get("Name") or r.get("KernelName") or r.get("Kernel_Name")
        out.append((name, int(r.get("Calls", 0)), float(r.get("AverageNs", r.get("Average_Ns", 0.0)))))
    out.sort(key=lambda t: -t[1] * t[2])
    return out


def _per_dispatch(path, counter):
    import csv
    from collections import defaultdict
    vals = defaultdict(list)
    for r in csv.DictReader(open(path)):
        name = r.get("Kernel_Name") or r.get("Kernel-Name") or r.get("KernelName")
        cn = r.get("Counter_Name") or r.get("Counter-Name")
        if cn != counter:
            continue
        did = int(r.get("Dispatch_Id") or r.get("Dispatch-Id") or 0)
        vals[name].append((did, float(r.get("Counter_Value") or r.get("Counter-Value"))))
    return vals


def summarize_traffic(fetch_csv, write_csv, info_json, workload):
    """HBM bytes per apply launch from a FETCH_SIZE run and a WRITE_SIZE run of
    --pmc-pass (KiB per dispatch), each scaled by the factor that makes the same
    counter read the known 4 D bytes of the plain copy kernel in the same run."""
    info = json.loads([l for l in open(info_json) if l.startswith("{")][-1])
    steps, cb = info["steps"], info["copy_bytes_each_way"]
    res = {}
    for path, counter in ((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")):
        v = _per_dispatch(path, counter)
        copy = [x for n, l in v.items() if "copy" in n.lower() or "elementwise" in n.lower() for x in l]
        copy = sorted(copy)[-steps:]
        # the timed applies are the last dispatches of apply kernels (the tuning
        # run of every schedule comes before them): K kernels per apply, the K
        # names seen among the last `steps` apply dispatches
        disp = sorted((did, n, c) for n, l in v.items() if any(k in n for k in APPLY_KERNELS) for did, c in l)
        kpa = len({n for _, n, _ in disp[-steps:]})
        timed = disp[-kpa * steps:]
        apply_names = sorted({n for _, n, _ in timed})
        per_launch = sum(c for _, _, c in timed) / steps
        copy_kib = sum(c for _, c in copy) / max(len(copy), 1)
        factor = (cb / 1024.0) / copy_kib if copy_kib > 0 else float("nan")
        res[counter] = {"apply_kib_per_launch": per_launch, "copy_kib": copy_kib, "factor": factor,
                        "bytes": per_launch * 1024.0 * factor, "kernels": apply_names}
    total = res["FETCH_SIZE"]["bytes"] + res["WRITE_SIZE"]["bytes"]
    return {workload: {"source_hash": kernel_source_hash(), "bytes_per_launch": total,
                       "fetch_bytes": res["FETCH_SIZE"]["bytes"], "write_bytes": res["WRITE_SIZE"]["bytes"],
                       "fetch_factor": res["FETCH_SIZE"]["factor"], "write_factor": res["WRITE_SIZE"]["factor"],
                       "algorithmic_bytes": 8 * info["D"],
                       "schedule": info.get("schedule") or ",".join(info.get("schedules", [])),
                       "kernels": res["FETCH_SIZE"]["kernels"]}}


def schedule_kernels(name):
    """Kernels one apply launches under a schedule (by schedule-name prefix)."""
    for pre, k in (("gt2_", "k_gtile row pass + k_upt band pass"), ("gt_", "k_gtile"),
                   ("grp2_", "k_rt (grouped tiles) + k_upt band pass"), ("grp_", "k_rt (grouped tiles)"),
                   ("rt_", "k_rt"), ("csx_", "k_cs row pass + k_upb band pass"),
                   ("rwpk_", "k_apply (packed table)"), ("rw_", "k_apply")):
        if name.startswith(pre):
            return k
    return name


def timed_applies(H, x, y, steps, warmup):
    import torch
    for _ in range(warmup):
        H.apply(x, y)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        H.apply(x, y)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, e0.elapsed_time(e1) / 1000.0


def setup(cfg, prec, jprime=True):
    from paper_1004_3354_amd import ed, models, workloads as wl
    phys, sectors = wl.config(cfg, jprime=jprime)
    nup, ndn = sectors[0]
    t0 = time.perf_counter()
    b = ed.Basis(phys["Ns"], nup, ndn)
    H = ed.Hamiltonian(models.params_from_model(phys), b, prec)
    import torch
    torch.cuda.synchronize()
    return phys, (nup, ndn), b, H, time.perf_counter() - t0


def _omp(n=None):
    """Thread count of the OpenMP runtime the oracle's C core runs on (set when
    n is given); the oracle and this process share one libgomp."""
    import ctypes
    try:
        g = ctypes.CDLL("libgomp.so.1")
    except OSError:
        return None
    if n is not None:
        g.omp_set_num_threads(int(n))
    return int(g.omp_get_max_threads())


def cpu_baseline(cfg=2, max_steps=400, tol=1e-7):
    """FP64 oracle on the host cores, in the paper's own format: the sector
    matrix built from the literal operator strings into the CSR arrays of
    Fig. 1 (the "setup" of Table 1, timed), the CSR product of Listing 1 (rows
    over OpenMP threads; all cores, then one), and the oracle's three-term
    Lanczos on that product to the ground energy with the stopping rule of the
    GPU runs.  value = algorithmic GB/s of the all-core product (16 B per
    output element, FP64), the unit of the headline."""
    import numpy as np
    import oracle as orc
    from paper_1004_3354_amd import workloads as wl
    cores = len(os.sched_getaffinity(0))
    _omp(cores)
    phys, sectors = wl.config(cfg)
    sec = orc.sector_for(phys, *sectors[0])
    t0 = time.perf_counter()
    row_ind, col_ind, H = sec.csr()
    setup_s = time.perf_counter() - t0
    nnz = int(row_ind[-1])
    x = wl.uniform_vector(wl.start_vector_seed(cfg), sec.D)
    orc.spmv(row_ind, col_ind, H, x)                      # first touch
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        orc.spmv(row_ind, col_ind, H, x)
    spmv_s = (time.perf_counter() - t0) / reps
    _omp(1)
    t0 = time.perf_counter()
    orc.spmv(row_ind, col_ind, H, x)
    spmv_1_s = time.perf_counter() - t0
    _omp(cores)
    v0 = wl.gaussian_vector(wl.start_vector_seed(cfg), sec.D)
    t0 = time.perf_counter()
    e0, _, info = orc.lanczos_ground(lambda v: orc.spmv(row_ind, col_ind, H, v), v0, max_iter=max_steps, tol=tol,
                                     reorth=False, want_vector=False)
    e0_s = time.perf_counter() - t0
    rate = 16.0 * sec.D / spmv_s / 1e9
    return {"value": round(rate, 3), "unit": "GB/s (FP64 algorithmic: 16 B per output element)",
            "cores": cores, "kind": "oracle",
            "sample": ("the whole N_s=15 sector (7,7), D=%d: CSR of Fig. 1 built from the literal operator strings "
                       "(%d nonzeros, %.1f GB), Listing-1 product over %d threads" %
                       (sec.D, nnz, (nnz * 16 + 8 * sec.D) / 1e9, cores)),
            "setup_s": round(setup_s, 2), "spmv_csr_s": round(spmv_s, 4),
            "single_thread": {"spmv_csr_s": round(spmv_1_s, 3), "value": round(16.0 * sec.D / spmv_1_s / 1e9, 3)},
            "time_to_e0": {"seconds": round(e0_s, 2), "E0": e0, "iters": info["iters"], "tol": tol,
                           "method": "three-term Lanczos on the CSR product (no reorthogonalisation)"}}


def step_roofline(info, seconds):
    """The Lanczos run against the HBM roofline: the algorithmic bytes its
    kernels moved (ed_info.traffic: x read and y written per H.v, the projected
    vectors and Y per Gram-Schmidt pass, restarts, Ritz vector and refinement)
    over the whole solve's wall time, as a fraction of 8 TB/s."""
    gb = info["traffic"] / 1e9
    return {"bytes_GB": round(gb, 2), "ms_per_step": round(1e3 * seconds / max(info["iters"], 1), 3),
            "GBps": round(gb / seconds, 1), "frac": round(gb / seconds / (HBM_PEAK_GBS), 4)}


def time_to_e0(cfg, precs, max_basis, tol, seed_idx, reorth=3, keep=0):
    """Same start vector (SplitMix64 normal stream, FP32 = RNE cast of the FP64
    values, filled on the device) and same residual target for each precision.
    max_basis: int or {precision: int} (the FP64 basis must fit HBM at N_s = 18)."""
    import torch
    from paper_1004_3354_amd import ed, workloads as wl
    out = {}
    for prec in precs:
        m = max_basis[prec] if isinstance(max_basis, dict) else max_basis
        phys, nn, b, H, tset = setup(cfg, prec)
        dt = torch.float64 if prec == ed.ED_FP64 else torch.float32
        v0 = torch.empty(b.D, dtype=dt, device="cuda")
        ed.fill_random(v0, wl.start_vector_seed(seed_idx), 1)
        kp = keep[prec] if isinstance(keep, dict) else keep
        opts = ed.options(tol=tol, max_basis=m, reorth=reorth, keep=kp)
        ws = torch.empty(H.workspace_bytes(opts, 1), dtype=torch.uint8, device="cuda")
        y = ws[: b.D * v0.element_size()].view(dt)   # scratch: tune the schedule outside the timed region
        (H.grouped() or H).apply(v0, y)              # the solver iterates on the grouped twin when there is one
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        E, info = H.lanczos_ground(v0, opts, ws=ws, allow_noconv=True)
        torch.cuda.synchronize()
        dt_s = time.perf_counter() - t0
        key = "fp64" if prec == ed.ED_FP64 else "fp32_mixed"
        out[key] = {"seconds": round(dt_s, 4), "E0": E, "iters": info["iters"], "restarts": info["restarts"],
                    "converged": info["converged"], "residual": info["residual"], "setup_s": round(tset, 3),
                    "max_basis": m, "keep": kp, "step_roofline": step_roofline(info, dt_s)}
        log("time-to-E0 %s (reorth %d): %.3f s E0=%.12f iters=%d restarts=%d" % (key, reorth, dt_s, E, info["iters"],
                                                                                  info["restarts"]))
        del ws, y, H, b, v0
        torch.cuda.empty_cache()
    out["max_basis"] = max_basis
    out["tol"] = tol
    out["reorth"] = {2: "CGS2, two full passes", 3: "both CGS2 projections from one read of the basis"}.get(reorth, reorth)
    if "fp64" in out and "fp32_mixed" in out:
        e64 = out["fp64"]["E0"]
        out["fp32_vs_fp64_rel"] = abs(out["fp32_mixed"]["E0"] - e64) / max(1.0, abs(e64))
        out["speedup_fp32_mixed"] = round(out["fp64"]["seconds"] / out["fp32_mixed"]["seconds"], 3)
    gold = os.path.join(ROOT, "tests", "golden", "oracle_e0.json")
    if os.path.exists(gold):
        g = json.load(open(gold))["entries"].get("cfg%d" % cfg)
        if g:
            ref = list(g["sectors"].values())[0]["evals"][0]
            out["oracle_E0"] = ref
            for k in ("fp64", "fp32_mixed"):
                if k in out:
                    out[k]["rel_err_vs_oracle"] = abs(out[k]["E0"] - ref) / max(1.0, abs(ref))
    return out


def green_bench(cfg=2, m=100, beta=10.0):
    """Impurity Green function of Eq. 3 (spin up, site 0 = the first impurity
    orbital) at the N_s = 15 workload: ground state first (not timed), then the
    timed part: c+ and c applied to it, an m-step Lanczos in each neighbouring
    sector and the continued fractions at 64 Matsubara points.  Runs: FP32 and
    FP64 with full reorthogonalisation (both projections per basis read), and
    FP32 with the plain three-term recurrence (no reorthogonalisation); each is
    compared with an FP64 run of 2m levels (the truncation reference)."""
    import numpy as np
    import torch
    from paper_1004_3354_amd import ed, models, workloads as wl
    out = {"m": m, "spin": 0, "site": 0, "n_matsubara": 64, "beta": beta}
    z = 1j * np.pi * (2 * np.arange(64) + 1) / beta
    gref = None
    for key, prec, reorth, mm in (("fp64_reference", ed.ED_FP64, 3, 2 * m), ("fp64", ed.ED_FP64, 3, m),
                                  ("fp32_mixed", ed.ED_FP32, 3, m), ("fp32_mixed_no_reorth", ed.ED_FP32, 0, m)):
        phys, nn, b, H, _ = setup(cfg, prec)
        dt = torch.float64 if prec == ed.ED_FP64 else torch.float32
        v0 = torch.empty(b.D, dtype=dt, device="cuda")
        ed.fill_random(v0, wl.start_vector_seed(cfg), 1)
        psi = torch.empty_like(v0)
        e0, _ = H.lanczos_ground(v0, ed.options(tol=1e-7, max_basis=16, keep=8, reorth=3), psi=psi,
                                 allow_noconv=True)
        del v0
        bp, bm = ed.Basis(phys["Ns"], nn[0] + 1, nn[1]), ed.Basis(phys["Ns"], nn[0] - 1, nn[1])
        Hp = ed.Hamiltonian(models.params_from_model(phys), bp, prec)
        Hm = ed.Hamiltonian(models.params_from_model(phys), bm, prec)
        opts = ed.options(reorth=reorth, max_basis=mm)
        ws = torch.empty(max(Hp.workspace_bytes(opts, 1), Hm.workspace_bytes(opts, 1)), dtype=torch.uint8,
                         device="cuda")
        for Hx in (Hp, Hm):   # tune the apply schedules outside the timed region
            t = ws[: Hx.D * psi.element_size()].view(dt)
            ed.fill_random(t, 1, 0)
            Hx.apply(t, ws[Hx.D * psi.element_size(): 2 * Hx.D * psi.element_size()].view(dt))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g, info = ed.green_function(H, e0, psi, Hp, Hm, 0, 0, z, m=mm, opts=opts, ws=ws)
        torch.cuda.synchronize()
        dt_s = time.perf_counter() - t0
        out[key] = {"seconds": round(dt_s, 4), "reorth": reorth, "E0": e0,
                    "weights": {k: v["weight"] for k, v in info.items()},
                    "steps": {k: v["steps"] for k, v in info.items()}}
        if gref is None:
            gref = g
        else:
            out[key]["max_rel_dev_vs_reference"] = float(np.max(np.abs(g - gref)) / np.max(np.abs(gref)))
        log("Green function %s: %.3f s, weights %s" % (key, dt_s, out[key]["weights"]))
        del psi, H, Hp, Hm, b, bp, bm, ws
        torch.cuda.empty_cache()
    out["speedup_fp32_mixed"] = round(out["fp64"]["seconds"] / out["fp32_mixed"]["seconds"], 3)
    return out


def thermal_bench(K=300, beta=58.0, cutoff=1e-5, m=100):
    """One impurity-solver pass at N_s = 12 as the paper describes its DMFT
    iteration: the K = 300 lowest levels over all 169 sectors, Boltzmann
    weights at beta (T = 200 K with energies in eV) with the 1e-5 cut, and the
    Green function of Eq. 3 (spin up, first impurity orbital) from every kept
    level at 64 Matsubara points.  FP64 vectors, then FP32-mixed ones."""
    import numpy as np
    import torch
    from paper_1004_3354_amd import ed, models
    phys, sectors = wl_config(3)
    p = models.params_from_model(phys)
    ns = int(phys["Ns"])
    z = 1j * np.pi * (2 * np.arange(64) + 1) / beta
    out = {"workload": "kanamori_Ns12_3orb_9bath_all169", "K": K, "beta": beta, "cutoff": cutoff, "m": m}
    gref = None
    for key, prec, tol in (("fp64", ed.ED_FP64, 1e-8), ("fp32_mixed", ed.ED_FP32, 1e-7)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hams = [ed.Hamiltonian(p, ed.Basis(ns, u, d), prec) for (u, d) in sectors]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        opts = ed.options(tol=tol, max_iter=20000, max_basis=20, keep=8)
        levels, vecs, det = ed.lowest_levels(hams, K, opts, progress=log)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        w, kept = ed.boltzmann_weights([e for e, _, _ in levels], beta, cutoff)
        g = np.zeros(len(z), dtype=np.complex128)
        byn = {tuple(sec): h for sec, h in zip(sectors, hams)}
        for (e, s, i), wi in zip(levels, w):
            if wi == 0.0:
                continue
            u, d = sectors[s]
            ed.green_function(hams[s], e, vecs[s][i], byn.get((u + 1, d)), byn.get((u - 1, d)), 0, 0, z, m=m,
                              weight=wi, g=g)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        r = {"tables_s": round(t1 - t0, 3), "levels_s": round(t2 - t1, 3), "green_s": round(t3 - t2, 3),
             "total_s": round(t3 - t0, 3), "levels_found": len(levels), "kept_levels": kept,
             "lowest_calls": det["lowest_calls"], "capped": det["capped"],
             "level_span": round(levels[K - 1][0] - levels[0][0], 6), "E_min": levels[0][0],
             "sectors_with_levels": len(vecs)}
        if gref is None:
            gref = g
        else:
            r["G_max_rel_dev_vs_fp64"] = float(np.max(np.abs(g - gref)) / np.max(np.abs(gref)))
        out[key] = r
        log("thermal N_s=12 %s: levels %.2f s (%d lowest calls), Green %.2f s over %d levels" %
            (key, t2 - t1, det["lowest_calls"], t3 - t2, kept))
        del hams, vecs, byn
        torch.cuda.empty_cache()
    return out


def wl_config(i):
    from paper_1004_3354_amd import workloads as wl
    return wl.config(i)


def batched_bench():
    """All 169 sectors of the N_s = 12 three-orbital impurity: the batched
    FP32-mixed Lanczos (graph-replayed steps, per-sector restarts), in the
    tuned setting (20 stored vectors keeping 8, both projections per basis read)
    and in the plain one (60 vectors, CGS2, explicit restarts), vs the same
    sectors solved one after another by the single-sector solver."""
    import numpy as np
    import torch
    from paper_1004_3354_amd import ed, models, workloads as wl
    phys, sectors = wl.config(3)
    p = models.params_from_model(phys)
    t0 = time.perf_counter()
    hs = [ed.Hamiltonian(p, ed.Basis(phys["Ns"], a, b), ed.ED_FP32) for (a, b) in sectors]
    torch.cuda.synchronize()
    tset = time.perf_counter() - t0
    seed = wl.start_vector_seed(3)
    sum_d = int(sum(h.D for h in hs))
    gold = os.path.join(ROOT, "tests", "golden", "oracle_e0.json")
    ref = None
    if os.path.exists(gold):
        g = json.load(open(gold))["entries"].get("cfg3")
        if g:
            ref = np.array([g["sectors"]["%d,%d" % s]["evals"][0] for s in sectors])
    out = {"workload": "kanamori_Ns12_3orb_9bath_all169_sectors", "sum_D": sum_d, "setup_s": round(tset, 3)}
    runs = (("keep8_of_20_reorth3", dict(tol=1e-7, max_basis=20, keep=8, reorth=3, max_iter=3000)),
            ("basis60_cgs2", dict(tol=1e-7, max_basis=60, reorth=2, max_iter=3000)))
    E_main = None
    for key, kw in runs:
        opts = ed.options(**kw)
        ed.lanczos_ground_batched(hs, opts, seed=seed)           # graph capture + tile tuning
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        E, info = ed.lanczos_ground_batched(hs, opts, seed=seed)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        st = ed.batched_last_stats()
        r = {"seconds": round(tb, 4), "steps": st["steps"], "restart_events": st["restart_events"],
             "ms_per_step": round(1e3 * tb / max(st["steps"], 1), 4), "tile": st["tile"],
             "algorithmic_GB": round(st["bytes"] / 1e9, 3),
             "algorithmic_GBps": round(st["bytes"] / tb / 1e9, 1),
             "frac_of_8TBps": round(st["bytes"] / tb / 8e12, 4),
             "apply_equiv_GBps": round(8.0 * sum_d * st["steps"] / tb / 1e9, 1),
             "iters_max": max(i["iters"] for i in info), "restarts_max": max(i["restarts"] for i in info),
             "all_converged": all(i["converged"] for i in info), "options": kw}
        if ref is not None:
            r["max_rel_err_vs_oracle"] = float(np.max(np.abs(np.array(E) - ref) / np.maximum(1.0, np.abs(ref))))
        out[key] = r
        if E_main is None:
            E_main = E
            out["batched_s"] = r["seconds"]
        log("batched 169 sectors %s: %.3f s, %d steps (%.3f ms/step), %.1f GB/s algorithmic" %
            (key, tb, st["steps"], r["ms_per_step"], r["algorithmic_GBps"]))
    opts = ed.options(tol=1e-7, max_basis=20, keep=8, reorth=3, max_iter=3000)
    Dmax = max(h.D for h in hs)
    ws = torch.empty(max(h.workspace_bytes(opts, 1) for h in hs), dtype=torch.uint8, device="cuda")
    v0 = torch.empty(Dmax, dtype=torch.float32, device="cuda")
    for h in hs:                                             # tune every sector's apply schedule
        ed.fill_random(v0[:h.D], seed, 1)
        h.apply(v0[:h.D], ws[:4 * h.D].view(torch.float32))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Es = []
    for i, h in enumerate(hs):
        ed.fill_random(v0[:h.D], seed + i, 1)
        e, _ = h.lanczos_ground(v0[:h.D], opts, ws=ws, allow_noconv=True)
        Es.append(e)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    out["sequential_s"] = round(ts, 4)
    out["sequential_options"] = "same as keep8_of_20_reorth3, one sector after another"
    out["speedup"] = round(ts / out["batched_s"], 2)
    out["max_abs_diff_batched_vs_sequential"] = float(np.max(np.abs(np.array(E_main) - np.array(Es))))
    log("batched 169 sectors: %.3f s (sequential %.3f s)" % (out["batched_s"], ts))
    return out


def pmc_pass(args):
    """Workload for rocprofv3 counter runs: K applies of each schedule named in
    --schedules (default: the tuned one) in the --order basis order, then K
    plain device copies of x (4 D bytes read, 4 D bytes written) to calibrate
    the counters against a kernel whose traffic is known."""
    import torch
    from paper_1004_3354_amd import ed
    cfg = 2 if args.workload == "ns15" else 4
    phys, nn, b, H, _ = setup(cfg, ed.ED_FP32)
    HH = (H.grouped() or H) if args.order == "grouped" else H
    x = torch.empty(b.D, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    ed.fill_random(x, 12345, 0)
    names = [v for v in args.schedules.split(",") if v] if args.schedules else []
    ids = [v for v in range(ed.variant_count()) if ed.variant_name(v) in names]
    if not ids:
        HH.apply(x, y)
        ids = [HH.current_variant()]
    torch.cuda.synchronize()
    for v in ids:
        log("pmc-pass %s D=%d %s order, schedule %s" % (args.workload, b.D, args.order, ed.variant_name(v)))
        for _ in range(args.steps):
            HH.apply_variant(v, x, y)
        torch.cuda.synchronize()
    for _ in range(args.steps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"workload": args.workload, "D": b.D, "order": args.order,
                      "schedules": [ed.variant_name(v) for v in ids], "steps": args.steps,
                      "copy_bytes_each_way": 4 * b.D}), flush=True)


def apply_leg(cfg, prec, steps, warmup=2):
    """Tuned H.v of one sector in the rank order (ed_apply_H on the handle) and
    in the grouped order the solvers iterate in (ed_apply_H on its twin).
    Timed with HIP events on the launch stream."""
    import torch
    from paper_1004_3354_amd import ed
    phys, nn, b, H, tset = setup(cfg, prec)
    dt = torch.float64 if prec == ed.ED_FP64 else torch.float32
    elem = 8 if prec == ed.ED_FP64 else 4
    x = torch.empty(b.D, dtype=dt, device="cuda")
    y = torch.empty_like(x)
    ed.fill_random(x, 12345, 0)
    out = {"D": b.D, "setup_s": round(tset, 3)}
    for tag, HH in (("rank_order", H), ("grouped", H.grouped())):
        if HH is None:
            continue
        wall, evt = timed_applies(HH, x, y, steps, warmup)
        ms = evt / steps * 1e3
        gbs = 2.0 * elem * b.D / (ms * 1e-3) / 1e9
        out[tag] = {"ms_per_apply": round(ms, 5), "wall_ms": round(wall / steps * 1e3, 5), "gbps": round(gbs, 1),
                    "frac": round(gbs / HBM_PEAK_GBS, 4), "schedule": ed.variant_name(HH.current_variant()),
                    "schedule_id": HH.current_variant()}
        log("N_s=%d %s %s H.v: %.4f ms, %.1f GB/s (%s)" % (phys["Ns"], "fp64" if prec == 0 else "fp32", tag, ms, gbs,
                                                           out[tag]["schedule"]))
    del x, y, H, b
    torch.cuda.empty_cache()
    return out


def lowest_leg(cfg, precs, k, opts_kw, seed_idx):
    """E0 and the k lowest levels (with multiplicity) per precision from the
    same start vector; time to the first level and to all k."""
    import torch
    from paper_1004_3354_amd import ed, workloads as wl
    out = {}
    for prec in precs:
        phys, nn, b, H, tset = setup(cfg, prec)
        dt = torch.float64 if prec == ed.ED_FP64 else torch.float32
        v0 = torch.empty(b.D, dtype=dt, device="cuda")
        ed.fill_random(v0, wl.start_vector_seed(seed_idx), 1)
        kw = dict(opts_kw[prec]) if isinstance(opts_kw, dict) and prec in opts_kw else dict(opts_kw)
        opts = ed.options(**kw)
        evecs = torch.empty((k, b.D), dtype=dt, device="cuda")
        ws = torch.empty(H.workspace_bytes(opts, k), dtype=torch.uint8, device="cuda")
        (H.grouped() or H).apply(v0, evecs[0])          # tune outside the timed region
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev, infos = H.lowest(1, v0, opts, ws=ws, evecs=evecs[:1], allow_noconv=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if k > 1:
            ev, more = H.lowest_more(1, k, ev, v0, evecs, opts, ws=ws, allow_noconv=True)
            infos = infos + more
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        key = "fp64" if prec == ed.ED_FP64 else "fp32_mixed"
        out[key] = {"time_to_e0_s": round(t1 - t0, 4), "time_to_k_s": round(t2 - t0, 4), "E0": float(ev[0]),
                    "levels": [float(e) for e in ev], "iters": [i["iters"] for i in infos],
                    "residual": [i["residual"] for i in infos],
                    "kato_temple_lower": [i["e_lower"] for i in infos], "converged": all(i["converged"] for i in infos),
                    "max_basis": kw.get("max_basis"), "keep": kw.get("keep"), "setup_s": round(tset, 3),
                    "e0_step_roofline": step_roofline(infos[0], t1 - t0)}
        if k > 1:
            tot = dict(infos[0])
            tot["traffic"] = sum(i["traffic"] for i in infos)
            tot["iters"] = sum(i["iters"] for i in infos)
            out[key]["all_levels_step_roofline"] = step_roofline(tot, t2 - t0)
        log("N_s=%d %s: E0 %.12f in %.3f s, %d levels in %.3f s" % (phys["Ns"], key, ev[0], t1 - t0, k, t2 - t0))
        del ws, evecs, v0, H, b
        torch.cuda.empty_cache()
    if "fp64" in out and "fp32_mixed" in out:
        a, c = out["fp64"], out["fp32_mixed"]
        out["fp32_vs_fp64_rel"] = max(abs(x - y) / max(1.0, abs(x)) for x, y in zip(a["levels"], c["levels"]))
        out["speedup_fp32_mixed_e0"] = round(a["time_to_e0_s"] / c["time_to_e0_s"], 3)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-e0", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ns18", action="store_true")
    ap.add_argument("--no-ns16", action="store_true", help="skip the 4x4 Hubbard eigenvalue leg")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-green", action="store_true", help="skip the Green function at N_s=15")
    ap.add_argument("--no-thermal", action="store_true", help="skip the 300-level thermal pass at N_s=12")
    ap.add_argument("--e0-ns18", action="store_true", help=argparse.SUPPRESS)  # the default; kept for old scripts
    ap.add_argument("--no-e0-ns18", action="store_true", help="skip the eigenvalue legs at N_s=18")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="counter runs: tune, then K FP32 applies and K plain copies of x (known bytes)")
    ap.add_argument("--workload", choices=["ns15", "ns18"], default="ns15",
                    help="sector used by --pmc-pass")
    ap.add_argument("--order", choices=["grouped", "rank"], default="grouped",
                    help="basis order of the --pmc-pass apply")
    ap.add_argument("--schedules", default="", help="comma-separated schedule names for --pmc-pass")
    ap.add_argument("--summarize-stats", metavar="KERNEL_STATS_CSV",
                    help="print the per-kernel summary of a rocprofv3 --stats run and exit (no GPU)")
    ap.add_argument("--summarize-traffic", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "PMC_PASS_LOG", "WORKLOAD"),
                    help="print HBM bytes per apply from two --pmc-pass counter runs and exit (no GPU)")
    args = ap.parse_args()
    if args.summarize_stats:
        for n, c, a in summarize_stats(args.summarize_stats)[:25]:
            print("%6d  %12.2f us  %s" % (c, a / 1e3, n[:120]))
        return
    if args.summarize_traffic:
        print(json.dumps(summarize_traffic(*args.summarize_traffic), indent=1))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the sector is held by a single MI355X and no multi-GPU "
              "path is built; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1004_3354_amd import ed
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.pmc_pass:
        pmc_pass(args)
        return

    # ---- headline: FP32 H.v on the N_s = 15 sector in the grouped order the
    # Lanczos solvers iterate in (the rank-order product beside it)
    hv15 = apply_leg(2, ed.ED_FP32, args.steps, args.warmup)
    head = hv15.get("grouped") or hv15["rank_order"]
    D = hv15["D"]
    alg_bytes = 8.0 * D
    ms = head["wall_ms"]
    value = alg_bytes / (ms * 1e-3) / 1e9
    kern_s = head["ms_per_apply"] * 1e-3
    achieved = alg_bytes / kern_s / 1e9
    variant = head["schedule"]
    wl15 = "kanamori_Ns15_3orb_12bath_sector7_7"
    order = "grouped" if "grouped" in hv15 else "rank_order"
    traffic = traffic_from_profile(wl15 + ("" if order == "rank_order" else "_grouped"), variant)
    fp64 = apply_leg(2, ed.ED_FP64, max(5, args.steps // 2), 2)

    ns18 = None
    if not args.no_ns18 and torch.cuda.mem_get_info()[0] > 24e9:
        ns18 = {"workload": "kanamori_Ns18_3orb_15bath_sector9_9",
                "fp32": apply_leg(4, ed.ED_FP32, max(3, args.steps // 10), 1)}
        if torch.cuda.mem_get_info()[0] > 48e9:
            ns18["fp64"] = apply_leg(4, ed.ED_FP64, max(3, args.steps // 10), 1)

    # ---- time to E0, FP32-mixed vs FP64, same start vector and target
    e0 = e0_cgs2 = None
    if not args.no_e0:
        # implicitly restarted Lanczos keeping 4 of 14 vectors (the fastest setting of
        # a sweep over 10..16 stored vectors keeping 3..8), both projections per read
        e0 = time_to_e0(2, [ed.ED_FP32, ed.ED_FP64], max_basis=14, tol=1e-7, seed_idx=2, reorth=3, keep=4)
        # reference: two full Gram-Schmidt passes, restart from the Ritz vector
        e0_cgs2 = time_to_e0(2, [ed.ED_FP32, ed.ED_FP64], max_basis=50, tol=1e-7, seed_idx=2, reorth=2)
    e0_16 = None
    if not args.no_e0 and not args.no_ns16:
        # 4x4 periodic Hubbard, U = 4, half filling: E0 and the 4 lowest levels
        e0_16 = lowest_leg(1, [ed.ED_FP32, ed.ED_FP64], 4,
                           {ed.ED_FP32: dict(tol=1e-7, reorth=3, keep=8, max_basis=24, max_iter=4000),
                            ed.ED_FP64: dict(tol=1e-10, reorth=3, keep=8, max_basis=24, max_iter=4000)}, 1)
    e0_18 = None
    if not args.no_e0_ns18 and not args.no_e0 and not args.no_ns18:
        try:
            # FP32-mixed: E0 (16 stored vectors keeping 8, the fastest of 11..20 for
            # E0), then the 3 lowest levels (20 keeping 10); FP64: E0 (11 stored
            # 18.9 GB vectors keeping 5)
            e0_18 = lowest_leg(4, [ed.ED_FP32], 1, dict(tol=1e-7, reorth=3, keep=8, max_basis=16, max_iter=3000), 4)
            low3 = lowest_leg(4, [ed.ED_FP32], 3, dict(tol=1e-7, reorth=3, keep=10, max_basis=20, max_iter=3000), 4)
            e0_18["fp32_mixed_3_lowest"] = low3["fp32_mixed"]
            e0_18.update(lowest_leg(4, [ed.ED_FP64], 1, dict(tol=1e-7, reorth=3, keep=5, max_basis=11, max_iter=3000),
                                    4))
            a, c = e0_18["fp64"], e0_18["fp32_mixed"]
            e0_18["fp32_vs_fp64_rel"] = abs(a["E0"] - c["E0"]) / max(1.0, abs(a["E0"]))
            e0_18["speedup_fp32_mixed_e0"] = round(a["time_to_e0_s"] / c["time_to_e0_s"], 3)
        except torch.cuda.OutOfMemoryError as e:
            torch.cuda.empty_cache()
            e0_18 = {"skipped": "device memory: %s" % str(e).splitlines()[0]}
            log("eigenvalue legs at N_s=18 skipped: out of device memory")

    green = None if args.no_green else green_bench()
    thermal = None if args.no_thermal else thermal_bench()
    batched = None if args.no_batched else batched_bench()
    cpu = None if args.no_cpu else cpu_baseline(2)
    if cpu:
        log("cpu baseline: %s" % cpu)

    rec = {
        "metric": "H.v HBM GB/s (% peak) + s to Lanczos E0 at N_s=15/18, FP32-mixed vs FP64",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp32", "data": "synthetic (seeded baths and SplitMix64 vectors)",
        "config": {"workload": wl15, "Ns": 15, "sector": [7, 7], "D": D,
                   "step": "one FP32 matrix-free H.v in the %s basis order%s (x, y resident in HBM)" %
                           (order.replace("_", " "), " the Lanczos solvers iterate in" if order == "grouped" else ""),
                   "schedule": variant, "schedule_id": head["schedule_id"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "%s (schedule %s)" % (schedule_kernels(variant), variant),
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "avg_launch_ms": round(kern_s * 1e3, 5)},
        "cpu_baseline": cpu,
        "hv_ns15_fp32": hv15,
        "hv_ns15_fp64": fp64,
        "hv_ns18": ns18,
        "time_to_e0_ns15": e0,
        "time_to_e0_ns15_cgs2": e0_cgs2,
        "time_to_e0_ns16": e0_16,
        "time_to_e0_ns18": e0_18,
        "batched_ns12": batched,
        "green_ns15": green,
        "thermal_ns12": thermal,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()

"""ed_rayleigh_noalloc, the allocation-free variant of ed_rayleigh (its
partial sums live in a static device array), against ed_rayleigh through the
C interface: two calls in a row on one GPU, the second on a smaller sector,
in both precisions and on both basis orders.  Both run the same kernels with
the same fixed reduction order on the same vector, so the results must be
identical bit for bit."""
import pytest

from gpu_common import gpu_ed
from paper_1004_3354_amd import models, workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_rayleigh_noalloc_matches_rayleigh(prec):
    ed = gpu_ed()
    dt = torch.float64 if prec == 0 else torch.float32
    # the N_s = 15 sector (7, 7) first, then the smaller N_s = 12 sector (5, 6)
    for cfg, (nu, nd) in ((2, (7, 7)), (3, (5, 6))):
        phys, _ = wl.config(cfg)
        b = ed.Basis(int(phys["Ns"]), nu, nd)
        H = ed.Hamiltonian(models.params_from_model(phys), b, prec)
        x = torch.empty(H.D, dtype=dt, device="cuda")
        ed.fill_random(x, 31 + cfg, 1)
        for HH, xx in ((H, x), (H.grouped(), None)):
            if xx is None:
                xx = torch.empty_like(x)
                H.to_grouped(x, xx)
            rq0, r0 = HH.rayleigh(xx)
            rq1, r1 = HH.rayleigh_noalloc(xx)
            torch.cuda.synchronize()
            assert rq1 == rq0 and r1 == r0, (cfg, rq0, rq1, r0, r1)
        del x, H, b

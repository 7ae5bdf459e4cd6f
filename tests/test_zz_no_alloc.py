"""lbm_totals_noalloc (the five FP64 totals with the reduction's partial sums in the
library's fixed device scratch, no allocation) against the totals of lbm_moments, through
the C ABI: two calls in a row on different lattices, the second smaller, then a repeat."""
import numpy as np
import pytest

import synth_inputs as si
from tests.helpers import gpu_params, maxwell

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2306_16274_amd import lbm
    lbm.library()
    return lbm


def _check_against_moments(L, lat, got):
    m = lat.moments(want=("rho", "u", "totals"))
    ref = m["totals"]
    rho, u = m["rho"], m["u"]
    scale = np.array([ref[0]] + [float(np.abs(rho * u[a]).sum()) for a in range(3)] + [ref[4]])
    err = np.abs(got - ref) / np.where(scale > 0, scale, 1.0)
    print("noalloc totals", got, "lbm_moments", ref, "scaled error", err.max())
    assert np.all(np.isfinite(got))
    assert err.max() < 1e-12, (got, ref)


def test_noalloc_totals_match_lbm_moments(L):
    import torch
    out = torch.full((5,), float("nan"), dtype=torch.float64, device="cuda")
    cases = [
        (si.Workload("big", 19, 96, 80, 72, T_over_Tc=0.7, walls=("z_lo", "z_hi"), G_ads=0.1,
                     R=14.0, centre=(48, 40, 30), U=(0.01, -0.02, -0.03), nu=0.08, noise=0.01,
                     seed=4), "fp32"),
        (si.Workload("small", 27, 20, 16, 12, T_over_Tc=0.6, R=4.0, U=(0.02, 0.0, 0.01)),
         "fp64"),
    ]
    for w, storage in cases:
        rv, rl = maxwell(w)
        with L.Lattice(gpu_params(w, storage, rho_ref=rv if storage == "fp32" else 0.0)) as lat:
            lat.init_droplet(*w.droplet_centre(), w.R, w.W, rl, rv, *w.U, w.noise, w.seed)
            lat.step(7)
            L.lbm_totals_noalloc(lat.ctx, out.data_ptr())
            lat.synchronize()
            got = out.cpu().numpy().copy()
            _check_against_moments(L, lat, got)
            out.fill_(float("nan"))
            L.lbm_totals_noalloc(lat.ctx, out.data_ptr())
            lat.synchronize()
            assert np.array_equal(out.cpu().numpy(), got), w.name


def test_noalloc_totals_reject_bad_arguments(L):
    w = si.Workload("a", 19, 8, 8, 8)
    with L.Lattice(gpu_params(w, "fp64")) as lat:
        with pytest.raises(L.LbmError) as ei:
            L.lbm_totals_noalloc(lat.ctx, 0)
        assert ei.value.status == L.LBM_EINVAL
        with pytest.raises(L.LbmError) as ei:
            L.lbm_totals_noalloc(lat.ctx, 1 << 20)
        assert ei.value.status == L.LBM_ESTATE

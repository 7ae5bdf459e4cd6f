"""The periodic health check of the fused step (non-finite or non-positive density, Sec. 8
failure detection): it reads the stored populations and the solid mask only, so it is valid
right after an initialisation and between walls with rho_ref = 0, where solid nodes hold no
populations; a NaN at a single fluid node is reported; a failed member of a batch is
reported on that member only and can be evicted."""
import numpy as np
import pytest

import synth_inputs as si
from oracle import lbm as olbm
from tests.helpers import gpu_params, maxwell, oracle_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2306_16274_amd import lbm
    lbm.library()
    return lbm


@pytest.mark.parametrize("kernel", ["fused", "two_pass"])
@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_walls_with_unshifted_storage_pass_the_check(L, storage, kernel):
    """FP64 (and FP32) with rho_ref = 0 between z-walls, reduce_every = 1, a droplet from
    lbm_init_droplet, five steps and no lbm_moments call first: every check passes (solid
    nodes, whose slots hold 0, are skipped)."""
    w = si.STATIC_32.with_(nx=24, ny=20, nz=18, R=5.0, walls=("z_lo", "z_hi"),
                           centre=(12, 10, 6))
    rv, rl = maxwell(w)
    code = L.LBM_STEP_FUSED if kernel == "fused" else L.LBM_STEP_TWO_PASS
    with L.Lattice(gpu_params(w, storage, rho_ref=0.0, reduce_every=1, step_kernel=code)) as lat:
        lat.init_droplet(*w.droplet_centre(), w.R, w.W, rl, rv)
        lat.step(5)
        lat.synchronize()
        lat.step(5)
        lat.synchronize()
        assert L.lbm_steps_done(lat.ctx) == 10


@pytest.mark.parametrize("where", ["bulk", "next_to_wall"])
@pytest.mark.parametrize("kernel", ["fused", "two_pass"])
def test_nan_at_one_fluid_node_is_reported(L, where, kernel):
    """One population of one fluid node set to NaN (in the bulk, or in the first fluid layer
    above a wall): the check after the next step reports LBM_ENONFINITE and later steps are
    refused with LBM_ESTATE."""
    w = si.Workload("nan", 19, 16, 12, 14, walls=("z_lo", "z_hi"))
    rho, u = si.random_fields(w.shape, seed=1)
    P = oracle_params(w)
    solid = olbm.solid_mask(P)
    f = olbm.equilibrium_populations(P, rho, u, solid)
    z = 1 if where == "next_to_wall" else 7
    f[6, z, 5, 9] = np.nan          # population 6 (e = -z) of a fluid node
    code = L.LBM_STEP_FUSED if kernel == "fused" else L.LBM_STEP_TWO_PASS
    with L.Lattice(gpu_params(w, "fp64", reduce_every=1, step_kernel=code)) as lat:
        lat.set_populations(f)
        lat.step(1)
        with pytest.raises(L.LbmError) as ei:
            lat.synchronize()
        assert ei.value.status == L.LBM_ENONFINITE
        with pytest.raises(L.LbmError) as ei:
            lat.step(1)
        assert ei.value.status == L.LBM_ESTATE


def test_failed_batch_member_is_reported_alone_and_evicted(L):
    """Three lattices in one batch, each with reduce_every = 2; one carries a NaN. After the
    batch run the failed member reports LBM_ENONFINITE, the others pass and hold exactly the
    populations of their own single-lattice steps; the batch then refuses to run, and a
    batch rebuilt without the failed member (evicted) runs on."""
    ws = [si.Workload("a", 19, 40, 40, 40, T_over_Tc=0.7, walls=("z_lo", "z_hi"), R=8.0,
                      centre=(20, 20, 12), U=(0.0, 0.0, -0.03), nu=0.05),
          si.Workload("b", 19, 48, 40, 36, T_over_Tc=0.6, R=7.0, noise=0.01, seed=3),
          si.Workload("c", 19, 33, 24, 21, T_over_Tc=0.7, walls=("z_lo",), R=6.0,
                      centre=(16, 12, 8), nu=0.08)]

    def make(w):
        rv, rl = maxwell(w)
        lat = L.Lattice(gpu_params(w, "fp32", rho_ref=rv, reduce_every=2))
        lat.init_droplet(*w.droplet_centre(), w.R, w.W, rl, rv, *w.U, w.noise, w.seed)
        return lat
    mixed = [make(w) for w in ws]
    alone = [make(w) for w in ws]
    f = mixed[1].get_populations()
    f[3, 18, 20, 24] = np.nan
    mixed[1].set_populations(f)
    b = L.lbm_batch_create([m.ctx for m in mixed], 4)
    try:
        L.lbm_batch_run(b, 3)
        for k in (0, 2):
            mixed[k].synchronize()
        with pytest.raises(L.LbmError) as ei:
            mixed[1].synchronize()
        assert ei.value.status == L.LBM_ENONFINITE
        with pytest.raises(L.LbmError) as ei:
            L.lbm_batch_run(b, 1)
        assert ei.value.status == L.LBM_ESTATE
    finally:
        L.lbm_batch_destroy(b)
    b2 = L.lbm_batch_create([mixed[0].ctx, mixed[2].ctx], 4)
    try:
        L.lbm_batch_run(b2, 1)
    finally:
        L.lbm_batch_destroy(b2)
    for k in (0, 2):
        alone[k].step(16)
        assert np.array_equal(alone[k].get_populations(), mixed[k].get_populations()), k
    for lat in mixed + alone:
        lat.close()

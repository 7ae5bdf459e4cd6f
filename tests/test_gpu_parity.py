"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances: FP64 storage 1e-12 pointwise relative in rho after 100 steps (and on every
population); FP32 shifted storage 1e-5 pointwise relative in rho and 1e-4 absolute in u
after 100 steps.
"""
import numpy as np
import pytest

import synth_inputs as si
from oracle import lbm as olbm
from tests.helpers import abs_err, gpu_params, maxwell, oracle_params, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2306_16274_amd import lbm
    lbm.library()
    return lbm


def oracle_state_from_fields(w, rho, u, **over):
    P = oracle_params(w, **over)
    solid = olbm.solid_mask(P)
    return P, solid, olbm.equilibrium_populations(P, rho, u, solid)


def run_pair(L, w, f0, steps, storage="fp64", rho_ref=0.0, P=None, solid=None, **gover):
    """Run the GPU from populations f0 for `steps` and return (gpu f, gpu moments)."""
    p = gpu_params(w, storage, rho_ref, **gover)
    with L.Lattice(p) as lat:
        lat.set_populations(f0)
        lat.step(steps)
        return lat.get_populations(), lat.moments()


def test_library_loads_native(L):
    import os
    assert os.path.exists(L.LIBRARY)


@pytest.mark.parametrize("Q", [19, 27])
def test_set_get_populations_roundtrip_bitexact(L, Q):
    w = si.Workload("rt", Q, 13, 7, 9, walls=("z_lo", "y_hi"), cylinder=(3.0, 4.0, 1.5))
    rho, u = si.random_fields(w.shape, seed=11)
    P, solid, f = oracle_state_from_fields(w, rho, u)
    f = f * si.random_factors(Q, w.shape, seed=11)
    f[:, solid] = 0.0
    with L.Lattice(gpu_params(w, "fp64")) as lat:
        lat.set_populations(f)
        g = lat.get_populations()
    assert np.array_equal(g, f)


@pytest.mark.parametrize("Q", [19, 27])
def test_init_droplet_matches_oracle(L, Q):
    w = si.STATIC_32.with_(Q=Q, nx=24, ny=20, nz=18, R=6.0, noise=0.01, seed=7)
    rv, rl = maxwell(w)
    P = oracle_params(w)
    cx, cy, cz = w.droplet_centre()
    rho, u = olbm.droplet_fields(P, cx, cy, cz, w.R, w.W, rl, rv, U=(0.01, -0.02, 0.03),
                                 noise_amp=w.noise, seed=w.seed)
    fo = olbm.equilibrium_populations(P, rho, u)
    with L.Lattice(gpu_params(w, "fp64")) as lat:
        lat.init_droplet(cx, cy, cz, w.R, w.W, rl, rv, 0.01, -0.02, 0.03, w.noise, w.seed)
        g = lat.get_populations()
    assert abs_err(g, fo) < 1e-15


@pytest.mark.parametrize("Q", [19, 27])
@pytest.mark.parametrize("geometry", ["periodic", "walls"])
def test_fp64_brute_force_tiny_box(L, Q, geometry):
    """8^3 boxes (ragged 9x8x7 for walls) with every term switched on: sigma, kappa,
    wetting, a cylinder, density-dependent viscosity; 1 and 20 steps."""
    if geometry == "periodic":
        w = si.Workload("tiny", Q, 8, 8, 8, sigma=0.1, kappa=0.4, nu=0.05, T_over_Tc=0.6)
        over = {}
        gover = {}
    else:
        w = si.Workload("tiny", Q, 9, 8, 7, sigma=0.12, kappa=0.3, G_ads=0.15, nu=0.05,
                        T_over_Tc=0.6, walls=("z_lo", "z_hi"), cylinder=(4.0, 3.0, 1.2))
        over = dict(nu_v=0.15, rho_l=0.4, rho_v=0.01)
        gover = dict(nu_v=0.15, rho_l=0.4, rho_v=0.01)
    rho, u = si.random_fields(w.shape, seed=3, rho_lo=0.05, rho_hi=0.4)
    P, solid, f0 = oracle_state_from_fields(w, rho, u, **over)
    f0 = f0 * si.random_factors(Q, w.shape, seed=3, amp=0.02)
    for steps in (1, 20):
        fo = olbm.run(f0, P, steps, solid)
        g, mom = run_pair(L, w, f0, steps, **gover)
        fl = ~solid
        assert abs_err(g, fo) < 1e-13, steps
        ro, uo, po, _ = olbm.moments(fo, P, solid)
        assert rel_err(mom["rho"], ro, fl) < 1e-12
        assert abs_err(mom["u"], uo, fl) < 1e-13
        assert abs_err(mom["p"], po, fl) < 1e-13


def _static32(Q=19):
    w = si.STATIC_32.with_(Q=Q)
    rv, rl = maxwell(w)
    P = oracle_params(w)
    cx, cy, cz = w.droplet_centre()
    rho, u = olbm.droplet_fields(P, cx, cy, cz, w.R, w.W, rl, rv)
    return w, P, olbm.equilibrium_populations(P, rho, u), (rv, rl)


@pytest.fixture(scope="module")
def static32_oracle():
    w, P, f0, dens = _static32()
    f100 = olbm.run(f0, P, 100)
    return w, P, f0, f100, dens


def test_fp64_static_droplet_100_steps(L, static32_oracle):
    w, P, f0, f100, (rv, rl) = static32_oracle
    with L.Lattice(gpu_params(w, "fp64")) as lat:
        cx, cy, cz = w.droplet_centre()
        lat.init_droplet(cx, cy, cz, w.R, w.W, rl, rv)
        lat.step(100)
        g = lat.get_populations()
        mom = lat.moments()
    ro, uo, po, _ = olbm.moments(f100, P)
    print("fp64 32^3 100 steps: rho rel", rel_err(mom["rho"], ro), "u abs", abs_err(mom["u"], uo))
    assert rel_err(mom["rho"], ro) < 1e-12
    assert rel_err(g, f100) < 1e-12
    assert abs_err(mom["u"], uo) < 1e-13
    tot = olbm.totals(f100, P)
    assert abs(mom["totals"][0] - tot[0]) / tot[0] < 1e-13


@pytest.mark.parametrize("rho_ref_kind", ["zero", "vapour"])
def test_fp32_shifted_static_droplet_100_steps(L, static32_oracle, rho_ref_kind):
    w, P, f0, f100, (rv, rl) = static32_oracle
    rho_ref = 0.0 if rho_ref_kind == "zero" else rv
    with L.Lattice(gpu_params(w, "fp32", rho_ref=rho_ref)) as lat:
        cx, cy, cz = w.droplet_centre()
        lat.init_droplet(cx, cy, cz, w.R, w.W, rl, rv)
        lat.step(100)
        mom = lat.moments()
    ro, uo, _, _ = olbm.moments(f100, P)
    e_rho, e_u = rel_err(mom["rho"], ro), abs_err(mom["u"], uo)
    print(f"fp32 rho_ref={rho_ref}: rho rel {e_rho:.3e} u abs {e_u:.3e}")
    assert e_rho < 1e-5
    assert e_u < 1e-4


def test_fp16_shifted_static_droplet_error_reported(L, static32_oracle):
    """FP16 storage has no parity target; its error against the oracle is measured and
    bounded loosely (3 % in rho, 1e-2 in u after 100 steps)."""
    w, P, f0, f100, (rv, rl) = static32_oracle
    with L.Lattice(gpu_params(w, "fp16", rho_ref=rv)) as lat:
        cx, cy, cz = w.droplet_centre()
        lat.init_droplet(cx, cy, cz, w.R, w.W, rl, rv)
        lat.step(100)
        mom = lat.moments()
    ro, uo, _, _ = olbm.moments(f100, P)
    e_rho, e_u = rel_err(mom["rho"], ro), abs_err(mom["u"], uo)
    print(f"fp16 rho_ref={rv}: rho rel {e_rho:.3e} u abs {e_u:.3e}")
    assert e_rho < 3e-2 and e_u < 1e-2


def test_deterministic_rerun(L):
    w, P, f0, (rv, rl) = _static32()
    outs = []
    for _ in range(2):
        with L.Lattice(gpu_params(w, "fp32")) as lat:
            cx, cy, cz = w.droplet_centre()
            lat.init_droplet(cx, cy, cz, w.R, w.W, rl, rv, noise_amp=0.01, seed=5)
            lat.step(30)
            outs.append(lat.get_populations())
    assert np.array_equal(outs[0], outs[1])


def test_health_check_reports_non_finite(L):
    """A NaN planted in the populations from the host is reported by the periodic health
    check, and further steps are refused."""
    w = si.Workload("nan", 19, 16, 16, 16)
    rho, u = si.random_fields(w.shape, seed=1)
    P, solid, f = oracle_state_from_fields(w, rho, u)
    f[3, 5, 5, 5] = np.nan
    with L.Lattice(gpu_params(w, "fp64", reduce_every=1)) as lat:
        lat.set_populations(f)
        lat.step(2)
        with pytest.raises(L.LbmError) as ei:
            lat.synchronize()
        assert ei.value.status == L.LBM_ENONFINITE
        with pytest.raises(L.LbmError) as ei:
            lat.step(1)
        assert ei.value.status == L.LBM_ESTATE

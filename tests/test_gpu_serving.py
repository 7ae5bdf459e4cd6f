"""Batched stepping and the continuous-batching loop: every lattice gives the same result
alone and in the mix (bitwise: the per-node arithmetic is the same in both launches)."""
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


def _members():
    return [
        si.Workload("a", 19, 40, 40, 40, T_over_Tc=0.7, walls=("z_lo", "z_hi"), G_ads=0.1,
                    R=8.0, centre=(20, 20, 12), U=(0.0, 0.0, -0.03), nu=0.05),
        si.Workload("b", 19, 48, 40, 36, T_over_Tc=0.6, R=7.0, noise=0.01, seed=3),
        si.Workload("c", 19, 70, 33, 21, T_over_Tc=0.7, walls=("z_lo",), kappa=0.3,
                    cylinder=(16.0, 4.0, 3.0), R=6.0, centre=(35, 16, 12), nu=0.08),
    ]


def _make(L, w, storage):
    rv, rl = maxwell(w)
    lat = L.Lattice(gpu_params(w, storage, rho_ref=rv if storage == "fp32" else 0.0))
    cx, cy, cz = w.droplet_centre()
    lat.init_droplet(cx, cy, cz, w.R, w.W, rl, rv, *w.U, w.noise, w.seed)
    return lat


@pytest.mark.parametrize("variant", ["plain", "plain_nt", "prefetch", "prefetch_nt", "tiles32x8",
                                     "dispatch_order", "rows", "rows_nt"])
@pytest.mark.parametrize("storage", ["fp32", "fp64"])
def test_batch_equals_individual_steps(L, monkeypatch, storage, variant):
    """Batched launches (default plain 64x4 tiles in XCD order, prefetching tiles, 32x8
    tiles, dispatch order, row tiles of run-time width (4-byte storage; FP64 keeps the
    64x4 tiles); plain stores, the default for these unaligned rows, or nontemporal ones)
    give each member exactly the populations of its own single-lattice steps."""
    if variant.startswith("prefetch"):
        monkeypatch.setenv("LBM_BATCH_PF", "1")
    if variant.startswith("rows"):
        monkeypatch.setenv("LBM_BATCH_ROWS", "1")
    if variant.endswith("_nt"):
        monkeypatch.setenv("LBM_BATCH_NT", "1")
    if variant == "dispatch_order":
        monkeypatch.setenv("LBM_BATCH_REMAP", "0")
    if variant == "tiles32x8":
        monkeypatch.setenv("LBM_BATCH_TILE", "1")
    ws = _members()
    alone = [_make(L, w, storage) for w in ws]
    mixed = [_make(L, w, storage) for w in ws]
    for lat in alone:
        lat.step(30)
    b = L.lbm_batch_create([m.ctx for m in mixed], 10)
    try:
        L.lbm_batch_run(b, 2)                 # two graph replays
        mixed[1].step(4)                      # eager work on a member between replays
        L.lbm_batch_run(b, 1)
    finally:
        L.lbm_batch_destroy(b)
    alone[1].step(4)
    mixed[0].step(4)                          # the others catch up eagerly
    mixed[2].step(4)
    alone[0].step(4)
    alone[2].step(4)
    for a, m, w in zip(alone, mixed, ws):
        fa, fm = a.get_populations(), m.get_populations()
        diff = float(np.max(np.abs(fa - fm)))
        print(f"{storage} {w.name}: max |alone - batched| = {diff:.3e}")
        assert np.array_equal(fa, fm), (w.name, diff)
        assert L.lbm_steps_done(m.ctx) == L.lbm_steps_done(a.ctx) == 34
    for lat in alone + mixed:
        lat.close()


def test_batch_rejects_bad_arguments(L):
    w = _members()[0]
    a = _make(L, w, "fp32")
    b64 = _make(L, w, "fp64")
    with pytest.raises(L.LbmError) as ei:
        L.lbm_batch_create([a.ctx], 3)
    assert ei.value.status == L.LBM_EINVAL
    with pytest.raises(L.LbmError):
        L.lbm_batch_create([a.ctx, b64.ctx], 2)
    with pytest.raises(L.LbmError):
        L.lbm_batch_create([a.ctx, a.ctx], 2)
    a.close()
    b64.close()


def test_row_tiles_on_extreme_widths(L, monkeypatch):
    """Row tiles of run-time width at the edges of their range, bitwise against each
    member's own single-lattice steps: the widest eligible member (384: two rows per
    workgroup, a ragged last tile), 1- and 2-node widths (hundreds of rows, lanes wrapping
    onto themselves in x), a single row (both halo rows are the row itself), and 7 x 130
    between y walls (109 rows and a ragged tile whose surplus lanes wrap past the wall)."""
    monkeypatch.setenv("LBM_BATCH_ROWS", "1")
    ws = [si.Workload("w384", 19, 384, 5, 6, T_over_Tc=0.7, walls=("z_lo", "z_hi"),
                      G_ads=0.1, nu=0.05),
          si.Workload("w1", 19, 1, 9, 4, T_over_Tc=0.6, nu=0.08),
          si.Workload("w2", 19, 2, 1, 3, T_over_Tc=0.7, walls=("z_lo",), kappa=0.3),
          si.Workload("w7", 19, 7, 130, 5, T_over_Tc=0.6, walls=("y_lo", "y_hi"),
                      G_ads=-0.1, nu=0.1)]

    def make(w, k):
        rv, _ = maxwell(w)
        lat = L.Lattice(gpu_params(w, "fp32", rho_ref=rv))
        rho, u = si.random_fields(w.shape, seed=60 + k, rho_lo=0.05, rho_hi=0.4)
        lat.init_fields(rho, u)
        return lat

    alone = [make(w, k) for k, w in enumerate(ws)]
    mixed = [make(w, k) for k, w in enumerate(ws)]
    for lat in alone:
        lat.step(8)
    b = L.lbm_batch_create([m.ctx for m in mixed], 4)
    try:
        L.lbm_batch_run(b, 2)
    finally:
        L.lbm_batch_destroy(b)
    for a, m, w in zip(alone, mixed, ws):
        fa, fm = a.get_populations(), m.get_populations()
        print(f"row tiles {w.name}: max |alone - batched| = {float(np.max(np.abs(fa - fm))):.3e}")
        assert np.array_equal(fa, fm), w.name
    for lat in alone + mixed:
        lat.close()


@pytest.mark.parametrize("variant", ["rows", "tiles64x4"])
def test_batch_solid_free_segments_equal_general_form(L, monkeypatch, variant):
    """The batched step splits each member's z-chunks into general and solid-free segments
    (planes with no solid node within two): with LBM_SOLID_FREE on and off the members' FP32
    populations after one batch run of 8 steps are equal (np.array_equal), on the row tiles
    and on the 64x4 tiles."""
    monkeypatch.setenv("LBM_BATCH_ROWS", "1" if variant == "rows" else "0")
    out = {}
    for on in ("1", "0"):
        monkeypatch.setenv("LBM_SOLID_FREE", on)
        lats = [_make(L, w, "fp32") for w in _members()]
        b = L.lbm_batch_create([m.ctx for m in lats], 4)
        try:
            L.lbm_batch_run(b, 2)
        finally:
            L.lbm_batch_destroy(b)
        out[on] = [lat.get_populations() for lat in lats]
        for lat in lats:
            lat.close()
    for w, a, g in zip(_members(), out["1"], out["0"]):
        print(f"{variant} {w.name}: max |solid-free - general| = {float(np.max(np.abs(a - g))):.3e}")
        assert np.array_equal(a, g), w.name


def test_serving_results_same_alone_and_in_the_mix(L):
    """A compressed trace of 8 impact requests through the continuous-batching loop and
    through the one-at-a-time loop (same FP32 storage): every request's result (spreading
    diameter, mass) is identical."""
    import torch
    from paper_2306_16274_amd import serving
    trace = si.serving_trace(8, rate_per_s=40.0, seed=7, L_lo=24, L_hi=44, steps_lo=40,
                             steps_hi=160)
    stream = torch.cuda.Stream()
    rb = serving.serve(trace, "batched", "fp32", chunk=40, stream=stream.cuda_stream)
    rs = serving.serve(trace, "sequential", "fp32", chunk=40, stream=stream.cuda_stream)
    assert rb["requests"] == rs["requests"] == 8
    by_id = {r["id"]: r for r in rs["records"]}
    for r in rb["records"]:
        s = by_id[r["id"]]
        assert r["mass"] == s["mass"] and r["spread_diameter"] == s["spread_diameter"], r["id"]
        assert r["liquid_volume"] == s["liquid_volume"], r["id"]
        assert r["finite"]


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp32_rows"])
def test_batch_members_match_the_oracle(L, monkeypatch, storage):
    """Every member of a batch against the FP64 oracle (not only against its own single-
    lattice run): three small lattices (walls, a cylinder with wetting, kappa, a ragged
    shape) from seeded random states, one batch run of 10 steps. FP64 populations to 1e-13
    absolute; FP32 shifted storage (64x4 tiles, or row tiles of run-time width) to 1e-5
    relative in rho and 1e-4 absolute in u."""
    from oracle import lbm as olbm
    if storage == "fp32_rows":
        monkeypatch.setenv("LBM_BATCH_ROWS", "1")
        storage = "fp32"
    from tests.helpers import abs_err, oracle_params, rel_err
    ws = [si.Workload("a", 19, 20, 16, 12, T_over_Tc=0.6, walls=("z_lo", "z_hi"), G_ads=0.1,
                      kappa=0.3, nu=0.05),
          si.Workload("b", 19, 24, 13, 10, T_over_Tc=0.7, nu=0.08),
          si.Workload("c", 19, 17, 22, 14, T_over_Tc=0.6, walls=("z_lo",), G_ads=-0.1,
                      cylinder=(11.0, 4.0, 2.0), nu=0.1)]
    lats, refs = [], []
    for k, w in enumerate(ws):
        rho, u = si.random_fields(w.shape, seed=40 + k, rho_lo=0.05, rho_hi=0.4)
        P = oracle_params(w)
        solid = olbm.solid_mask(P)
        f0 = olbm.equilibrium_populations(P, rho, u, solid)
        f0 = f0 * si.random_factors(19, w.shape, seed=40 + k, amp=0.02)
        f0[:, solid] = 0.0
        rv, _ = maxwell(w)
        lat = L.Lattice(gpu_params(w, storage, rho_ref=rv if storage == "fp32" else 0.0))
        lat.set_populations(f0)
        lats.append(lat)
        refs.append((P, solid, olbm.run(f0, P, 10, solid)))
    b = L.lbm_batch_create([lat.ctx for lat in lats], 10)
    try:
        L.lbm_batch_run(b, 1)
    finally:
        L.lbm_batch_destroy(b)
    for lat, (P, solid, fo), w in zip(lats, refs, ws):
        fl = ~solid
        if storage == "fp64":
            g = lat.get_populations()
            err = abs_err(g, fo)
            print(f"batch member {w.name} fp64: max |df| {err:.2e}")
            assert err < 1e-13, w.name
        m = lat.moments()
        ro, uo, _, _ = olbm.moments(fo, P, solid)
        er, eu = rel_err(m["rho"], ro, fl), abs_err(m["u"], uo, fl)
        print(f"batch member {w.name} {storage}: rho rel {er:.2e}, u abs {eu:.2e}")
        assert er < (1e-12 if storage == "fp64" else 1e-5), w.name
        assert eu < (1e-13 if storage == "fp64" else 1e-4), w.name
        lat.close()


def test_batched_fp32_matches_sequential_fp64(L):
    """Equal accuracy of the two serving modes: three requests of the serving workload
    (CS at 0.7 T_c, walls, wetting, a falling droplet; boxes 40-72) advanced 200 steps in
    one FP32 shifted-storage batch and, one at a time, in FP64 with plain launches: every
    fluid node's rho within 1e-5 relative and u within 1e-4 absolute (the FP32 tolerances
    against FP64)."""
    from paper_2306_16274_amd import serving
    trace = si.serving_trace(3, seed=11, L_lo=40, L_hi=72, steps_lo=200, steps_hi=200)
    b32 = [serving.start_job(r, "fp32", None, 0.0) for r in trace]
    b = L.lbm_batch_create([j.lat.ctx for j in b32], serving.STEP_QUANTUM)
    try:
        L.lbm_batch_run(b, 200 // serving.STEP_QUANTUM)
    finally:
        L.lbm_batch_destroy(b)
    for r, j32 in zip(trace, b32):
        j64 = serving.start_job(r, "fp64", None, 0.0)
        j64.lat.step(200)
        m64 = j64.lat.moments(want=("rho", "u"))
        m32 = j32.lat.moments(want=("rho", "u"))
        fl = m64["rho"] > 0
        er = float(np.max(np.abs(m32["rho"][fl] - m64["rho"][fl]) / m64["rho"][fl]))
        eu = float(np.max(np.abs(m32["u"][:, fl] - m64["u"][:, fl])))
        print(f"request L={r['L']} theta={r['theta']:.0f}: batched fp32 vs fp64 rho {er:.2e} "
              f"u {eu:.2e}")
        assert er < 1e-5 and eu < 1e-4, (r["L"], er, eu)
        j64.lat.close()
        j32.lat.close()


@pytest.mark.parametrize("mode", ["batched", "sequential"])
def test_serving_evicts_a_failed_request(L, monkeypatch, mode):
    """A request whose lattice goes non-finite (a NaN planted in its populations right
    after it is created) is evicted by the serving loop at the next health check: its record
    says finite = False, every other request finishes with exactly the result of a clean
    run of the same trace."""
    import torch
    from paper_2306_16274_amd import serving
    monkeypatch.setattr(serving, "HEALTH_EVERY", 20)
    trace = si.serving_trace(6, rate_per_s=40.0, seed=5, L_lo=24, L_hi=40, steps_lo=60,
                             steps_hi=120)
    stream = torch.cuda.Stream()
    clean = serving.serve(trace, mode, "fp32", chunk=20, stream=stream.cuda_stream)
    start = serving.start_job

    def start_with_nan(req, storage, s, t_now):
        job = start(req, storage, s, t_now)
        if req["id"] == 2:
            f = job.lat.get_populations()
            f[1, 3, 4, 5] = np.nan
            job.lat.set_populations(f)
        return job
    monkeypatch.setattr(serving, "start_job", start_with_nan)
    bad = serving.serve(trace, mode, "fp32", chunk=20, stream=stream.cuda_stream)
    assert clean["failed"] == 0 and bad["failed"] == 1
    by_id = {r["id"]: r for r in clean["records"]}
    assert len(bad["records"]) == 6
    for r in bad["records"]:
        if r["id"] == 2:
            assert not r["finite"]
            continue
        c = by_id[r["id"]]
        assert r["finite"] and r["mass"] == c["mass"], r["id"]
        assert r["spread_diameter"] == c["spread_diameter"], r["id"]


@pytest.mark.parametrize("theta", [60.0, 140.0])
def test_serving_contact_angle_calibration(L, theta):
    """Spot check of the serving calibration: a sessile drop of the serving physics on a
    wall with G_ads = g_ads_for_angle(theta) settles to theta within 4 degrees."""
    from paper_2306_16274_amd import impact, serving
    req = dict(L=100, theta=theta, R=20.0, U=0.0, steps=8000)
    p, rv, rl = serving.request_params(req, "fp32")
    p.nz = 60
    thr = 0.5 * (rv + rl)
    with L.Lattice(p) as lat:
        lat.init_droplet(50.0, 50.0, 0.5 + 12.0, 20.0, 5.0, rl, rv)
        lat.step(8000)
        counts = lat.liquid_stats(thr, rv, rl)[0]
    measured = impact.contact_angle_from_planes(counts)[0]
    print(f"serving wall for {theta} degrees: G_ads {p.G_ads:.4f}, measured {measured:.1f}")
    assert abs(measured - theta) < 4.0

"""Host logic of the continuous-batching loop, on the CPU: the lattice and batch entry
points are replaced by stand-ins that count steps and memory, while request parameters,
coexistence densities and footprints come from the library's host-only entry points."""
import threading

import numpy as np
import pytest

import synth_inputs as si
from paper_2306_16274_amd import lbm as L
from paper_2306_16274_amd import serving


class Recorder:
    def __init__(self):
        self.lock = threading.Lock()
        self.alive = {}            # ctx -> device footprint in bytes
        self.steps = {}            # ctx -> steps taken
        self.closed = {}           # ctx -> steps at close
        self.peak_bytes = 0
        self.peak_alive = 0
        self.log = []              # ctx of every step call, in order
        self.peak_batch = 0        # most lattices in one batched launch
        self.failing = set()       # ctx whose health check reports a non-finite density
        self.fail_sizes = set()    # box sizes L whose lattices fail


def install_fakes(monkeypatch, rec):
    class FakeLattice:
        _next = [1]

        def __init__(self, params, use_torch_stream=True):
            with rec.lock:
                self.ctx = FakeLattice._next[0]
                FakeLattice._next[0] += 1
                self.nz = params.nz
                rec.alive[self.ctx] = L.lbm_footprint_bytes(params)
                if params.nx in rec.fail_sizes:
                    rec.failing.add(self.ctx)
                rec.steps[self.ctx] = 0
                rec.peak_bytes = max(rec.peak_bytes, sum(rec.alive.values()))
                rec.peak_alive = max(rec.peak_alive, len(rec.alive))

        def init_droplet(self, *a, **k):
            pass

        def step(self, n=1):
            with rec.lock:
                rec.steps[self.ctx] += n
                rec.log.append(self.ctx)

        def synchronize(self):
            with rec.lock:
                if self.ctx in rec.failing:
                    raise L.LbmError(L.LBM_ENONFINITE, "planted failure")

        def liquid_stats(self, thr, rv, rl, reach=1):
            c = np.zeros(self.nz, dtype=np.int64)
            c[1] = 100
            return c, np.zeros(self.nz, dtype=np.int64), 1.0

        def moments(self, want=()):
            return {"totals": np.array([1.0, 0, 0, 0, 0])}

        def close(self):
            with rec.lock:
                rec.closed[self.ctx] = rec.steps[self.ctx]
                rec.alive.pop(self.ctx, None)

    class FakeBatch:
        def __init__(self, ctxs, spl):
            self.ctxs, self.spl = list(ctxs), spl

    def batch_create(ctxs, spl, stream=None):
        with rec.lock:
            rec.peak_batch = max(rec.peak_batch, len(ctxs))
        return FakeBatch(ctxs, spl)

    def batch_run(b, n):
        with rec.lock:
            for c in b.ctxs:
                assert c in rec.alive, "batched a lattice that was already freed"
                rec.steps[c] += n * b.spl

    monkeypatch.setattr(serving.L, "Lattice", FakeLattice)
    monkeypatch.setattr(serving.L, "lbm_batch_create", batch_create)
    monkeypatch.setattr(serving.L, "lbm_batch_run", batch_run)
    monkeypatch.setattr(serving.L, "lbm_batch_destroy", lambda b: None)

    def health(ctx, wait=False):
        with rec.lock:
            return L.LBM_ENONFINITE if ctx in rec.failing else L.LBM_OK
    monkeypatch.setattr(serving.L, "lbm_health_status", health)


def _trace():
    return si.serving_trace(14, rate_per_s=2000.0, seed=11, L_lo=24, L_hi=60, steps_lo=35,
                            steps_hi=300)


def test_steps_of_rounds_up_to_the_quantum():
    assert serving.steps_of({"steps": 2000}) == 2000
    assert serving.steps_of({"steps": 2001}) == 2010
    assert serving.steps_of({"steps": 1}) == serving.STEP_QUANTUM


def test_contact_angle_map_interpolates_the_calibration():
    """The angle -> G_ads map goes through every calibration point, is increasing, puts
    the measured neutral wall at G_ads = 0 and extends the end segments beyond them."""
    for g, th in serving.CALIBRATION:
        assert serving.g_ads_for_angle(th) == pytest.approx(g, abs=1e-12)
    ths = np.linspace(60.0, 160.0, 101)
    gs = [serving.g_ads_for_angle(t) for t in ths]
    assert all(b > a for a, b in zip(gs, gs[1:]))
    assert abs(serving.g_ads_for_angle(90.0)) < 0.002
    assert 0.2 < serving.g_ads_for_angle(160.0) < 0.25


def test_request_params_use_the_coexistence_densities():
    req = _trace()[0]
    p, rv, rl = serving.request_params(req, "fp32")
    assert p.nx == p.ny == p.nz == req["L"]
    assert 0 < rv < rl and p.rho_ref == rv
    assert p.bc[2][0] == p.bc[2][1] == L.LBM_BC_WALL
    p64, _, _ = serving.request_params(req, "fp64")
    assert p64.rho_ref == 0.0


@pytest.mark.parametrize("budget_factor,max_slots", [(1.5, 64), (100.0, 3)])
def test_batched_loop_completes_every_request_within_budget(monkeypatch, budget_factor, max_slots):
    rec = Recorder()
    install_fakes(monkeypatch, rec)
    trace = _trace()
    fps = [L.lbm_footprint_bytes(serving.request_params(r, "fp32")[0]) for r in trace]
    budget = int(budget_factor * max(fps))
    out = serving.serve(trace, "batched", "fp32", budget_bytes=budget, max_slots=max_slots,
                        chunk=40, time_scale=1.0)
    assert out["requests"] == len(trace)
    assert sorted(r["id"] for r in out["records"]) == [r["id"] for r in trace]
    # every lattice took exactly its request's (rounded) step count and was freed
    assert not rec.alive
    assert sorted(rec.closed.values()) == sorted(serving.steps_of(r) for r in trace)
    # lattices whose results are still being read back hold their memory until freed:
    # the budget covers them; the slot limit bounds the lattices of one batched launch
    assert rec.peak_bytes <= budget
    assert rec.peak_batch <= max_slots
    assert all(r["latency"] >= 0 for r in out["records"])


def test_sequential_loop_runs_one_request_at_a_time_in_arrival_order(monkeypatch):
    rec = Recorder()
    install_fakes(monkeypatch, rec)
    trace = _trace()
    out = serving.serve(trace, "sequential", "fp64", chunk=40)
    assert out["requests"] == len(trace)
    # the steps of each lattice form one contiguous run: no interleaving of requests
    runs = [c for i, c in enumerate(rec.log) if i == 0 or rec.log[i - 1] != c]
    assert len(runs) == len(set(runs)) == len(trace)
    done = [r["id"] for r in sorted(out["records"], key=lambda r: r["t_done"])]
    assert done == [r["id"] for r in sorted(trace, key=lambda r: r["t_arrival"])]
    assert sorted(rec.closed.values()) == sorted(serving.steps_of(r) for r in trace)


@pytest.mark.parametrize("mode", ["batched", "sequential"])
def test_failed_request_is_evicted_and_freed(monkeypatch, mode):
    """A lattice whose health check fails is evicted at the next chunk boundary: it is never
    batched again, its lattice is freed, its record says finite = False, and every other
    request completes its full step count."""
    rec = Recorder()
    install_fakes(monkeypatch, rec)
    trace = _trace()
    bad_L = trace[3]["L"]
    rec.fail_sizes.add(bad_L)
    out = serving.serve(trace, mode, "fp32", chunk=40)
    assert out["requests"] == len(trace)
    bad = [r for r in out["records"] if r["L"] == bad_L]
    assert bad and all(not r["finite"] for r in bad)
    assert out["failed"] == len(bad)
    assert all(r["finite"] for r in out["records"] if r["L"] != bad_L)
    assert not rec.alive                      # every lattice freed, the failed ones too
    good = sorted(serving.steps_of(r) for r in trace if r["L"] != bad_L)
    assert sorted(v for c, v in rec.closed.items() if c not in rec.failing) == good
    # a failed lattice stops within one chunk of its first check
    assert all(v <= 2 * 40 for c, v in rec.closed.items() if c in rec.failing)

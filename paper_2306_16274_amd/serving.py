"""Continuous-batching request loop for droplet-impact simulations.

Requests (cubic box L, contact angle, impact speed, number of steps) arrive over time.
Each admitted request gets its own lattice, resident in HBM until its result has been read.
Admission is by device-memory footprint (lbm_footprint_bytes) against a budget, and by a
slot limit. All active lattices advance together, in chunks of time steps, through the
batched entry points of the library: one kernel launch per time step covers the tiles of
every active lattice, and the launches of a chunk are HIP-graph replays. At every chunk
boundary finished requests are retired (result read back, lattice freed) and requests that
arrived meanwhile are admitted, so new work joins the running batch instead of waiting for
it to drain.

Every lattice has its own stream; the batch has another, and events order them, so the
next chunk is enqueued before the results of the requests that just finished are read
back, and creating or freeing a lattice never drains the device.

The baseline mode runs the same trace first-in first-out, one request at a time, with plain
(unbatched, non-graph) lbm_step launches.

Physics of a request (the synthetic serving workload): D3Q19, Carnahan-Starling EOS at
T = 0.7 T_c (a = 0.5, b = 4, R = 1), G = -1, sigma = 0.1175 (fitted: a flat interface then
settles on the Maxwell densities), kappa = 0, nu = 0.05, the printed
rates except s4 = 1 (with s4 = 1.2 D3Q19 is linearly unstable at this viscosity), walls at
z = 0 and z = L-1, periodic in x and y; a droplet of radius R = L/6 centred at
(L/2, L/2, 1.25 R + 1) moving at -U along z. The contact angle is turned into G_ads by
interpolating a measured calibration of this physics (static sessile drops, R = 20 in
100 x 100 x 60, 8000 steps, spherical-cap fit; psi at the wall read at its mirror image).
"""
import argparse
import json
import math
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from . import lbm as L

STEP_QUANTUM = 10          # request step counts are rounded up to a multiple of this


# Static contact angle (degrees) against G_ads for the serving physics, measured on the
# GPU (sessile drop R = 20, 100 x 100 x 60, 8000 steps). Above about 150 degrees the drop
# detaches from the wall (G_ads >= 0.2), so no static angle is measured there.
CALIBRATION = ((-0.175, 26.6), (-0.15, 37.2), (-0.10, 55.7), (-0.05, 72.9), (0.00, 89.7),
               (0.05, 105.8), (0.10, 121.5), (0.15, 138.6), (0.16, 142.2), (0.17, 145.0),
               (0.18, 147.4), (0.19, 150.6))


def g_ads_for_angle(theta_deg):
    """Fluid-solid strength G_ads of Eq. (22) for a contact angle: linear interpolation in
    CALIBRATION, extended with the slope of its end segments beyond the measured range
    (above 150.6 degrees the wall is non-wetting: the drop would not stay on it)."""
    g = [a for a, _ in CALIBRATION]
    t = [b for _, b in CALIBRATION]
    if theta_deg <= t[0]:
        k = 0
    elif theta_deg >= t[-1]:
        k = len(t) - 2
    else:
        k = max(i for i in range(len(t) - 1) if t[i] <= theta_deg)
    return g[k] + (g[k + 1] - g[k]) * (theta_deg - t[k]) / (t[k + 1] - t[k])


_COEX = {}


HEALTH_EVERY = 200         # steps between health checks of a request's lattice
# sigma of Eq. (B1) at which a flat interface of the serving physics settles on the Maxwell
# coexistence densities (0.1 leaves its vapour 23 % below them)
SIGMA = 0.1175


def request_params(req, storage="fp32"):
    p = L.lbm_params_default()
    p.lattice = 19
    p.storage = {"fp64": L.LBM_FP64, "fp32": L.LBM_FP32}[storage]
    p.nx = p.ny = p.nz = int(req["L"])
    p.T_over_Tc = 0.7
    p.nu_l = p.nu_v = 0.05
    p.sigma, p.kappa = SIGMA, 0.0
    p.s4 = 1.0
    p.G_ads = g_ads_for_angle(req["theta"])
    p.bc[2][0] = p.bc[2][1] = L.LBM_BC_WALL
    p.reduce_every = HEALTH_EVERY
    key = (p.eos, p.T_over_Tc, p.cs_a, p.cs_b, p.cs_R)
    if key not in _COEX:
        _COEX[key] = L.lbm_coexistence(p)
    rv, rl = _COEX[key]
    p.rho_ref = rv if storage != "fp64" else 0.0
    return p, rv, rl


def steps_of(req):
    return int(math.ceil(req["steps"] / STEP_QUANTUM) * STEP_QUANTUM)


@dataclass
class Job:
    req: dict
    lat: object
    rho_v: float
    rho_l: float
    footprint: int
    steps: int
    done_steps: int = 0
    t_admit: float = 0.0
    mass0: float = 0.0

    @property
    def remaining(self):
        return self.steps - self.done_steps


def start_job(req, storage, stream, t_now):
    """Create and initialise the lattice of a request (on its own library-owned stream
    when stream is None)."""
    p, rv, rl = request_params(req, storage)
    p.stream = stream
    fp = L.lbm_footprint_bytes(p)
    lat = L.Lattice(p, use_torch_stream=False)
    n = int(req["L"])
    R = float(req["R"])
    lat.init_droplet(n / 2.0, n / 2.0, 1.25 * R + 1.0, R, 5.0, rl, rv, 0.0, 0.0, -req["U"])
    job = Job(req, lat, rv, rl, fp, steps_of(req), t_admit=t_now)
    return job


def finish_job(job):
    """Read the result of a finished request, reduced on the device: the spreading diameter
    (diameter of the equal-area disc of the liquid nodes in the first fluid layer, z = 1,
    Sec. IV A), the liquid volume and the total mass. A lattice whose last health check
    failed (detected only now: the check was still in flight at the chunk boundaries) gives
    the record of an evicted request."""
    if L.lbm_health_status(job.lat.ctx, wait=True) == L.LBM_ENONFINITE:
        return evicted_result(job)
    thr = 0.5 * (job.rho_l + job.rho_v)
    counts, _, volume = job.lat.liquid_stats(thr, job.rho_v, job.rho_l)
    d_f = 2.0 * math.sqrt(float(counts[1]) / math.pi)
    mass = float(job.lat.moments(want=("totals",))["totals"][0])
    job.lat.close()
    return dict(spread_diameter=d_f, spread_ratio=d_f / float(job.req["R"]), mass=mass,
                liquid_volume=volume, finite=bool(np.isfinite(mass)))


def evicted_result(job):
    """Result record of a request whose lattice failed its health check (non-finite or
    non-positive density): it is dropped from the batch and its lattice freed."""
    job.lat.close()
    return dict(spread_diameter=float("nan"), spread_ratio=float("nan"), mass=float("nan"),
                liquid_volume=float("nan"), finite=False)


def serve(trace, mode="batched", storage="fp32", budget_bytes=64 << 30, max_slots=64,
          chunk=200, time_scale=1.0, stream=None, log=None, phases=None,
          max_active_nodes=16 << 20):
    """Run a request trace. mode "batched" (continuous batching) or "sequential" (one
    request at a time, plain launches). time_scale > 1 compresses the arrival times.
    Admission stops while the active lattices already hold max_active_nodes nodes (enough
    to keep the GPU busy; more would only stretch everyone's time to result: on the
    256-request sweep, 16 Mi nodes keep 98 % of the throughput of 48 Mi and cut p50 / p99
    from 62-76 / 78-101 s to 53 / 76 s).
    phases: optional dict that accumulates host seconds per loop phase.
    A request whose lattice fails its periodic health check (every HEALTH_EVERY steps) is
    evicted at the next chunk boundary: it leaves the batch, its lattice is freed and its
    record says finite = False.
    Returns a dict with per-request records and the aggregate figures."""
    clock = time.perf_counter
    if phases is None:
        phases = {}

    def tick(name, t_start):
        phases[name] = phases.get(name, 0.0) + clock() - t_start
    assert chunk % STEP_QUANTUM == 0
    pending = sorted(trace, key=lambda r: r["t_arrival"])
    active, records = [], []
    used = 0
    batch, members = None, None
    work = 0.0
    t0 = time.perf_counter()

    def now():
        return (time.perf_counter() - t0) * time_scale

    evicted = []           # failed lattices, closed once no batch refers to them
    retiring = []          # finished in the previous chunk; results read after the next enqueue
    futures = []           # (job, future) of result readbacks in flight
    pool = ThreadPoolExecutor(max_workers=2)

    def retire(j):
        res = finish_job(j)
        return res, now()

    def record(j, res, t_done):
        rec = dict(id=j.req["id"], L=j.req["L"], steps=j.steps, t_arrival=j.req["t_arrival"],
                   t_admit=j.t_admit, t_done=t_done, latency=t_done - j.req["t_arrival"], **res)
        records.append(rec)
        if log:
            log(rec)

    def collect(block):
        nonlocal used
        for item in list(futures):
            j, fut = item
            if not block and not fut.done():
                continue
            ts = clock()
            res, t_done = fut.result()
            tick("retire", ts)
            record(j, res, t_done)
            used -= j.footprint
            futures.remove(item)
    inflight = []          # events after the last chunks, to keep at most 2 chunks queued
    ext = None
    if stream is not None and mode == "batched":
        import torch
        ext = torch.cuda.ExternalStream(stream)
    while pending or active or retiring or futures:
        t = now()
        # admission: arrived requests, while slots and the footprint budget allow; lattices
        # whose results are still being read back (futures) still hold their memory
        over_budget = False
        while pending and pending[0]["t_arrival"] <= t:
            if mode == "sequential" and (active or retiring):
                break
            if len(active) >= max_slots:
                break
            p, _, _ = request_params(pending[0], storage)
            fp = L.lbm_footprint_bytes(p)
            if (active or retiring or futures) and used + fp > budget_bytes:
                over_budget = True
                break
            if active and sum(int(j.req["L"]) ** 3 for j in active) >= max_active_nodes:
                break
            req = pending.pop(0)
            ts = clock()
            job = start_job(req, storage, None, now())
            tick("admit", ts)
            active.append(job)
            used += job.footprint
        finished = []
        if active:
            k = min(chunk, min(j.remaining for j in active))
            if mode == "batched":
                old = None
                if members != [id(j) for j in active]:
                    ts = clock()
                    old = batch
                    batch = L.lbm_batch_create([j.lat.ctx for j in active], STEP_QUANTUM, stream)
                    members = [id(j) for j in active]
                    tick("rebuild", ts)
                ts = clock()
                L.lbm_batch_run(batch, k // STEP_QUANTUM)
                tick("enqueue", ts)
                if ext is not None:
                    ev = torch.cuda.Event()
                    ev.record(ext)
                    inflight.append(ev)
                    if len(inflight) > 2:
                        ts = clock()
                        inflight.pop(0).synchronize()
                        tick("throttle", ts)
                if old is not None:         # its work precedes the run just enqueued
                    ts = clock()
                    L.lbm_batch_destroy(old)
                    tick("rebuild", ts)
                    for j in evicted:       # no batch refers to them any more
                        record(j, evicted_result(j), now())
                        used -= j.footprint
                    evicted = []
                failed = [j for j in active
                          if L.lbm_health_status(j.lat.ctx) == L.LBM_ENONFINITE]
            else:
                ts = clock()
                failed = []
                for j in active:
                    j.lat.step(k)
                    try:
                        j.lat.synchronize()
                    except L.LbmError as err:
                        if err.status != L.LBM_ENONFINITE:
                            raise
                        failed.append(j)
                tick("enqueue", ts)
            for j in active:
                j.done_steps += k
                work += float(j.req["L"]) ** 3 * k
            for j in failed:           # evicted: leaves the batch at the next rebuild
                active.remove(j)
                if mode == "batched":
                    evicted.append(j)
                else:
                    record(j, evicted_result(j), now())
                    used -= j.footprint
            finished = [j for j in active if j.remaining == 0]
            for j in finished:
                active.remove(j)
        # results of requests that finished one chunk earlier are read back by a worker
        # thread (the readback waits for the GPU), while this thread keeps enqueueing
        for j in retiring:
            futures.append((j, pool.submit(retire, j)))
        retiring = finished
        collect(block=False)
        if not active and not retiring:
            if futures and (over_budget or not pending or pending[0]["t_arrival"] > now()):
                collect(block=True)
            elif pending:
                wait = (pending[0]["t_arrival"] - now()) / time_scale
                if wait > 0:
                    ts = clock()
                    time.sleep(min(wait, 0.05))
                    tick("idle", ts)
    collect(block=True)
    pool.shutdown()
    if batch is not None:
        L.lbm_batch_destroy(batch)
    for j in evicted:
        record(j, evicted_result(j), now())
    makespan = now() - min(r["t_arrival"] for r in trace) if trace else 0.0
    lat = np.array([r["latency"] for r in records])
    return dict(mode=mode, storage=storage, requests=len(records),
                failed=sum(1 for r in records if not r["finite"]), phases_s=phases,
                makespan_s=makespan / time_scale,
                aggregate_mlups=work / (makespan / time_scale) / 1e6 if makespan > 0 else 0.0,
                p50_s=float(np.percentile(lat, 50)) / time_scale if len(lat) else None,
                p99_s=float(np.percentile(lat, 99)) / time_scale if len(lat) else None,
                records=records)


def main():
    import sys
    import os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch
    import synth_inputs as si
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--rate", type=float, default=4.0)
    ap.add_argument("--L-lo", type=int, default=64)
    ap.add_argument("--L-hi", type=int, default=192)
    ap.add_argument("--steps-lo", type=int, default=2000)
    ap.add_argument("--steps-hi", type=int, default=8000)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--chunk", type=int, default=200)
    ap.add_argument("--max-active-mnodes", type=float, default=16.0)
    ap.add_argument("--modes", default="batched:fp32,sequential:fp64")
    args = ap.parse_args()
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    trace = si.serving_trace(args.requests, args.rate, L_lo=args.L_lo, L_hi=args.L_hi,
                             steps_lo=args.steps_lo, steps_hi=args.steps_hi)
    out = {}
    for spec in args.modes.split(","):
        mode, storage = spec.split(":")
        def log(rec, spec=spec):
            print(json.dumps({"mode": spec, "done": rec["id"], "L": rec["L"],
                              "latency_s": round(rec["latency"], 3)}), flush=True)
        r = serve(trace, mode, storage, budget_bytes=int(args.budget_gb * (1 << 30)),
                  chunk=args.chunk, stream=stream.cuda_stream, log=log,
                  max_active_nodes=int(args.max_active_mnodes * (1 << 20)))
        r.pop("records")
        out[spec] = r
        print(json.dumps({spec: r}), flush=True)
    return out


if __name__ == "__main__":
    main()

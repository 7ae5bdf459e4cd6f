"""Throughput benchmark of the fused lattice update on one MI355X.

One step is one time step of the whole hot path (streaming with bounce-back, density and
pseudopotential, interaction / wetting / surface-tension terms, moment-space collision,
back-transform, store) over the lattice of the workload. The workload is a 256^3 D3Q19
static droplet (Carnahan-Starling EOS at T = 0.5 T_c, all non-viscous relaxation rates 1,
nu = 0.1, sigma = 0.1153 (the value at which a flat interface settles on the Maxwell
densities), +-1 % interface noise), populations resident in HBM before timing starts.

Prints one JSON line (rank 0): the FP32 shifted-storage throughput in MLUPS as `value`,
the FP64 and FP16-shifted throughputs beside it, the HBM roofline of the dominant kernel
measured with HIP events on the launch stream, a time-compressed serving sweep (p50/p99
time to result and aggregate MLUPS of continuous batching against one-at-a-time plain
launches) and the CPU oracle timed on a bounded sample (one core and all cores).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E peak, GB/s


def kernel_source_hash():
    """Hash of the fused step kernel's code and launch configuration (the files it is
    compiled from); a counter summary taken on other sources is not used."""
    h = hashlib.sha256()
    for name in ("lattice.h", "common.h", "fused.h"):
        with open(os.path.join(ROOT, "paper_2306_16274_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, storage):
    """HBM bytes per launch of `kernel` on the benchmark workload, from the committed
    rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter
    reads for a plain copy of known size), or None when the summary is missing or was
    taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{kernel}_{storage}_d3q19_256cube.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) == 2 and not line.startswith("#"):
                vals[parts[0]] = parts[1]
    if vals.get("source_hash") != kernel_source_hash():
        return None
    return float(vals["hbm_bytes_per_launch"])


def make_params(w, storage, rho_ref, rho_v, rho_l, step_kernel="fused"):
    from paper_2306_16274_amd import lbm as L
    p = L.lbm_params_default()
    p.lattice = w.Q
    p.storage = {"fp64": L.LBM_FP64, "fp32": L.LBM_FP32, "fp16": L.LBM_FP16}[storage]
    p.nx, p.ny, p.nz = w.nx, w.ny, w.nz
    p.rho_ref = rho_ref
    p.eos = L.LBM_EOS_CS
    p.cs_a, p.cs_b, p.cs_R, p.T_over_Tc = w.cs_a, w.cs_b, w.cs_R, w.T_over_Tc
    p.G, p.sigma, p.kappa, p.G_ads = w.G, w.sigma, w.kappa, w.G_ads
    p.nu_l = p.nu_v = w.nu
    if w.rates == "unit":
        for k in ("s2b", "s3", "s3b", "s4", "s4b", "s5", "s6"):
            setattr(p, k, 1.0)
    axes = {"x": 0, "y": 1, "z": 2}
    for name in w.walls:                      # solid layers at index 0 / n - 1 of an axis
        ax, side = name.split("_")
        p.bc[axes[ax]][0 if side == "lo" else 1] = L.LBM_BC_WALL
    p.reduce_every = 0
    p.step_kernel = L.LBM_STEP_FUSED if step_kernel == "fused" else L.LBM_STEP_TWO_PASS
    return p


def run_gpu(w, storage, steps, warmup, rho_ref_choice="vapour", step_kernel="fused"):
    import torch
    from paper_2306_16274_amd import lbm as L
    p0 = make_params(w, storage, 0.0, 0.0, 0.0)
    rho_v, rho_l = L.lbm_coexistence(p0)
    rho_ref = 0.0 if storage == "fp64" else {"zero": 0.0, "vapour": rho_v, "liquid": rho_l}[rho_ref_choice]
    p = make_params(w, storage, rho_ref, rho_v, rho_l, step_kernel)
    # a dedicated (default-priority) stream: the library launches on it and the timing
    # events are recorded on it
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    p.stream = stream.cuda_stream
    assert p.stream, "expected a non-null HIP stream handle"
    plan = L.lbm_fused_plan(p) if step_kernel == "fused" else None
    lat = L.Lattice(p)
    cx, cy, cz = w.droplet_centre()
    lat.init_droplet(cx, cy, cz, w.R, w.W, rho_l, rho_v, 0.0, 0.0, 0.0, w.noise, w.seed)
    lat.step(warmup)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    lat.step(steps)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    ktimes = lat.kernel_times(max(3, min(steps, 20)))
    mom = lat.moments(want=("totals",))
    lat.close()
    torch.cuda.set_stream(torch.cuda.default_stream())
    return dict(ms=ms, ms_per_step=ms / steps, mlups=w.nodes * steps / (ms * 1e-3) / 1e6,
                kernel_ms=ktimes, rho_ref=rho_ref, rho_v=rho_v, rho_l=rho_l, plan=plan,
                mass=float(mom["totals"][0]))


def copy_bandwidth(nbytes=2 << 30, reps=10):
    """HBM bandwidth of torch's device copy (read + write bytes / time), for context."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        b.copy_(a)
    t1.record()
    torch.cuda.synchronize()
    gbs = 2 * nbytes * reps / (t0.elapsed_time(t1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def _oracle_sample(w, n):
    import synth_inputs as si  # noqa: F401
    from oracle import lbm as olbm
    from tests.helpers import maxwell, oracle_params
    ws = w.with_(nx=n, ny=n, nz=n, R=w.R * n / w.nx)
    rv, rl = maxwell(ws)
    P = oracle_params(ws)
    cx, cy, cz = ws.droplet_centre()
    rho, u = olbm.droplet_fields(P, cx, cy, cz, ws.R, ws.W, rl, rv, noise_amp=ws.noise,
                                 seed=ws.seed)
    return ws, P, olbm.equilibrium_populations(P, rho, u), olbm.solid_mask(P)


def _oracle_run(args):
    """One process of the CPU baseline: FP64 oracle steps on the sample for budget_s
    seconds, one thread; returns (node updates, seconds)."""
    w, n, budget_s = args
    from threadpoolctl import threadpool_limits
    from oracle import lbm as olbm
    with threadpool_limits(limits=1):
        ws, P, f, solid = _oracle_sample(w, n)
        f = olbm.step(f, P, solid)          # warm-up
        steps, t = 0, 0.0
        t0 = time.perf_counter()
        while t < budget_s:
            f = olbm.step(f, P, solid)
            steps += 1
            t = time.perf_counter() - t0
    return ws.nodes * steps, t


def host_cpu():
    """CPU model name and the cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return model, cores


def cpu_baseline(w, budget_s=10.0, n=64, max_procs=16):
    """The FP64 CPU oracle on a bounded sample of the workload (a 64^3 box with the same
    physics, droplet radius scaled by 1/4): one process on one thread, then one process per
    usable core (at most max_procs) on independent copies of the sample at once."""
    from concurrent.futures import ProcessPoolExecutor
    model, cores = host_cpu()
    lups, t = _oracle_run((w, n, budget_s))
    single = lups / t / 1e6
    procs = max(1, min(cores, max_procs))
    with ProcessPoolExecutor(max_workers=procs) as ex:
        res = list(ex.map(_oracle_run, [(w, n, budget_s)] * procs))
    all_cores = sum(l for l, _ in res) / max(tt for _, tt in res) / 1e6
    return dict(value=single, unit="MLUPS", cores=1, kind="oracle",
                sample=f"{n}^3 D3Q19 box of the same workload (droplet R={w.R * n / w.nx:g}), "
                       f"FP64 numpy oracle steps for {budget_s:g} s, one thread",
                all_cores={"value": all_cores, "unit": "MLUPS", "cores": procs,
                           "sample": f"{procs} processes, one thread each, each on its own "
                                     f"copy of the sample for {budget_s:g} s"},
                cpu_model=model, host_cores=cores)


def serving_sweep(n_requests, seed=2306):
    """Time-compressed serving sweep: the serving trace's distribution (cubic boxes
    log-uniform in [64, 192], contact angle, impact speed, droplet R = L/6) with step counts
    and arrival gaps divided by ten (200-800 steps, Poisson arrivals at 40 per second: the
    same offered load in node updates per second), served by continuous batching in FP32
    shifted storage and, as baselines, one request at a time with plain launches in FP64
    (the survey's baseline) and in FP32 (the same bytes per node as the batched loop)."""
    import torch
    import synth_inputs as si
    from paper_2306_16274_amd import serving
    trace = si.serving_trace(n_requests, rate_per_s=40.0, seed=seed, steps_lo=200,
                             steps_hi=800)
    stream = torch.cuda.Stream()
    out = {"requests": n_requests, "trace": "serving trace / 10: steps 200-800, 40 arrivals/s, "
                                           f"L log-uniform in [64, 192], seed {seed}"}
    for spec in ("batched:fp32", "sequential:fp64", "sequential:fp32"):
        mode, storage = spec.split(":")
        r = serving.serve(trace, mode, storage, chunk=50, stream=stream.cuda_stream)
        out[spec] = {"p50_s": round(r["p50_s"], 3), "p99_s": round(r["p99_s"], 3),
                     "aggregate_MLUPS": round(r["aggregate_mlups"], 1),
                     "makespan_s": round(r["makespan_s"], 2), "failed": r["failed"]}
    b = out["batched:fp32"]
    for base in ("sequential:fp64", "sequential:fp32"):
        o = out[base]
        out["gain_vs_" + base.replace(":", "_")] = {
            "aggregate": round(b["aggregate_MLUPS"] / o["aggregate_MLUPS"], 3),
            "p99": round(o["p99_s"] / b["p99_s"], 3)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--fp64-steps", type=int, default=100)
    ap.add_argument("--fp16-steps", type=int, default=100)
    ap.add_argument("--slab-steps", type=int, default=200,
                    help="steps on one GPU's z-slab of the workload shared by 8 GPUs (0: skip)")
    ap.add_argument("--walls-steps", type=int, default=100,
                    help="steps on the workload between walls at z = 0 and z = 255, with and "
                         "without the solid-free planes (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=64,
                    help="requests of the time-compressed serving sweep (0: skip)")
    ap.add_argument("--rho-ref", default="vapour", choices=["zero", "vapour", "liquid"])
    ap.add_argument("--step-kernel", default="fused", choices=["fused", "two_pass"])
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the lattice update "
              "is benchmarked on a single MI355X; multi-GPU execution is not implemented.",
              file=sys.stderr)
        sys.exit(2)

    import synth_inputs as si
    w = si.LAPLACE_256
    # the CPU oracle first, before this process touches the GPU (its worker processes are
    # forked from a process without a HIP runtime)
    cpu = None if args.no_cpu_baseline else cpu_baseline(w)

    import torch
    from paper_2306_16274_amd import lbm as L
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    Q = w.Q

    r32 = run_gpu(w, "fp32", args.steps, args.warmup, args.rho_ref, args.step_kernel)
    r64 = run_gpu(w, "fp64", args.fp64_steps, max(2, args.warmup // 4), "zero", args.step_kernel)
    r16 = run_gpu(w, "fp16", args.fp16_steps, max(2, args.warmup // 4), args.rho_ref, args.step_kernel)
    # one GPU's share if the 256^3 lattice were cut into 8 z-slabs (periodic slab: the halo
    # exchange between GPUs is not implemented)
    slab = None
    if args.slab_steps > 0:
        ws = w.with_(nz=w.nz // 8, R=w.nz // 16 - 4.0, centre=(w.nx / 2, w.ny / 2, w.nz // 16))
        rs = run_gpu(ws, "fp32", args.slab_steps, args.warmup, args.rho_ref, args.step_kernel)
        slab = {"shape": [ws.nx, ws.ny, ws.nz], "value": round(rs["mlups"], 1), "unit": "MLUPS",
                "us_per_step": round(1000 * rs["ms_per_step"], 1),
                "kernel_us": round(1000 * max(rs["kernel_ms"].values()), 1),
                "steps": args.slab_steps, "storage": "fp32 shifted"}
    # the same workload between walls at z = 0 and z = 255 (FP32 shifted): the planes two or
    # more away from the walls run the solid-free form; beside it every plane in the general
    # form (LBM_SOLID_FREE=0)
    walls = None
    if args.walls_steps > 0:
        wz = w.with_(walls=("z_lo", "z_hi"))
        rw = run_gpu(wz, "fp32", args.walls_steps, args.warmup, args.rho_ref, args.step_kernel)
        prev = os.environ.get("LBM_SOLID_FREE")
        os.environ["LBM_SOLID_FREE"] = "0"
        try:
            rg = run_gpu(wz, "fp32", args.walls_steps, args.warmup, args.rho_ref, args.step_kernel)
        finally:
            if prev is None:
                del os.environ["LBM_SOLID_FREE"]
            else:
                os.environ["LBM_SOLID_FREE"] = prev
        walls = {"walls": "z = 0 and z = 255", "storage": "fp32 shifted",
                 "value": round(rw["mlups"], 1), "unit": "MLUPS",
                 "ms_per_step": round(rw["ms_per_step"], 4), "steps": args.walls_steps,
                 "kernel_ms": rw["kernel_ms"],
                 "solid_free_planes": [rw["plan"]["solid_free_lo"], rw["plan"]["solid_free_hi"]]
                 if rw["plan"] else None,
                 "general_form": {"value": round(rg["mlups"], 1),
                                  "ms_per_step": round(rg["ms_per_step"], 4)}}
    serving_block = serving_sweep(args.serving_requests) if args.serving_requests > 0 else None
    copy_gbs = copy_bandwidth()
    stream_copy_gbs = L.lbm_copy_bandwidth()

    # dominant kernel of the FP32 step and its algorithmic bytes per node
    kname, kms = max(r32["kernel_ms"].items(), key=lambda kv: kv[1])
    b = 4
    per_node = {"k_step_fused": 2 * Q * b,           # populations in + out
                "k_collide": 2 * Q * b + 4,          # populations in + out, psi of the node
                "k_density_psi": Q * b + 4}[kname]    # populations in, psi out
    alg_bytes = per_node * w.nodes
    achieved = alg_bytes / (kms * 1e-3) / 1e9
    traffic = measured_traffic(kname, "fp32")
    step_bytes = 2 * Q * b * w.nodes                  # method minimum per step
    effective = step_bytes / (r32["ms_per_step"] * 1e-3) / 1e9
    eff64 = 2 * Q * 8 * w.nodes / (r64["ms_per_step"] * 1e-3) / 1e9
    eff16 = 2 * Q * 2 * w.nodes / (r16["ms_per_step"] * 1e-3) / 1e9

    out = {
        "metric": "MLUPS, D3Q19 multiphase 256^3, FP32 shifted storage (FP64 beside it)",
        "value": round(r32["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "lattice": "D3Q19", "nodes": w.nodes,
                   "step_kernel": args.step_kernel,
                   "eos": "carnahan-starling", "T_over_Tc": w.T_over_Tc, "rates": w.rates,
                   "storage": "fp32 shifted", "rho_ref": r32["rho_ref"],
                   "droplet_R": w.R, "noise": w.noise},
        "fp64": {"value": round(r64["mlups"], 1), "unit": "MLUPS",
                 "ms_per_step": round(r64["ms_per_step"], 4), "steps": args.fp64_steps,
                 "effective_GBs": round(eff64, 1),
                 "effective_frac": round(eff64 / HBM_PEAK_GBS, 4),
                 "kernel_ms": r64["kernel_ms"]},
        "fp16": {"value": round(r16["mlups"], 1), "unit": "MLUPS",
                 "ms_per_step": round(r16["ms_per_step"], 4), "steps": args.fp16_steps,
                 "storage": "fp16 shifted", "effective_GBs": round(eff16, 1),
                 "effective_frac": round(eff16 / HBM_PEAK_GBS, 4),
                 "kernel_ms": r16["kernel_ms"]},
        "launch_plan": r32["plan"],
        "slab_of_8": slab,
        "walls_z": walls,
        "effective_step_GBs": round(effective, 1),
        "effective_step_frac": round(effective / HBM_PEAK_GBS, 4),
        "kernel_ms": r32["kernel_ms"],
        "copy_kernel_GBs": round(stream_copy_gbs, 1),
        "copy_kernel_frac_of_peak": round(stream_copy_gbs / HBM_PEAK_GBS, 4),
        "torch_copy_GBs": round(copy_gbs, 1),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": kname,
                     "alg_bytes_per_node": per_node, "alg_bytes_per_launch": alg_bytes,
                     "kernel_ms": round(kms, 5),
                     "frac_of_copy": round(achieved / stream_copy_gbs, 4)},
        "serving": serving_block,
        "cpu_baseline": cpu,
        "mass": r32["mass"],
    }
    out["source_hash"] = kernel_source_hash()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

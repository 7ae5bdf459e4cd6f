"""Python binding of the C ABI in include/lbm.h (argument marshalling only).

Every function has the name of the C entry point it wraps and raises LbmError on a
non-zero status. All lattice arithmetic runs in the HIP library; this module only moves
numpy buffers in and out. torch is imported first so that the library shares torch's HIP
runtime and can be given torch's current stream.
"""
import ctypes
import os

import numpy as np
import torch  # noqa: F401  (provides the HIP runtime and the streams)

HERE = os.path.dirname(os.path.abspath(__file__))
LIBRARY = os.path.join(HERE, "liblbm_hip.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_ENONFINITE, LBM_ESTATE = 0, -1, -2, -3, -4, -5
LBM_FP64, LBM_FP32, LBM_FP16 = 0, 1, 2
LBM_EOS_CS, LBM_EOS_PIECEWISE = 0, 1
LBM_BC_PERIODIC, LBM_BC_WALL = 0, 1
LBM_STEP_FUSED, LBM_STEP_TWO_PASS = 0, 1
LBM_WALL_PSI_NODE, LBM_WALL_PSI_FLUID_MEAN, LBM_WALL_PSI_ZERO, LBM_WALL_PSI_MIRROR = 0, 1, 2, 3

STATUS_NAMES = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EDEVICE",
                -4: "LBM_ENONFINITE", -5: "LBM_ESTATE"}


class lbm_params(ctypes.Structure):
    """Mirror of the C struct lbm_params (same field order and types)."""
    _fields_ = [
        ("lattice", ctypes.c_int32), ("storage", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("eos", ctypes.c_int32),
        ("rho_ref", ctypes.c_double),
        ("cs_a", ctypes.c_double), ("cs_b", ctypes.c_double), ("cs_R", ctypes.c_double),
        ("T_over_Tc", ctypes.c_double),
        ("pw_theta_v", ctypes.c_double), ("pw_theta_m", ctypes.c_double),
        ("pw_theta_l", ctypes.c_double), ("pw_rho1", ctypes.c_double), ("pw_rho2", ctypes.c_double),
        ("G", ctypes.c_double), ("sigma", ctypes.c_double), ("kappa", ctypes.c_double),
        ("G_ads", ctypes.c_double),
        ("nu_l", ctypes.c_double), ("nu_v", ctypes.c_double),
        ("rho_l", ctypes.c_double), ("rho_v", ctypes.c_double),
        ("s0", ctypes.c_double), ("s1", ctypes.c_double), ("s2b", ctypes.c_double),
        ("s3", ctypes.c_double), ("s3b", ctypes.c_double), ("s4", ctypes.c_double),
        ("s4b", ctypes.c_double), ("s5", ctypes.c_double), ("s6", ctypes.c_double),
        ("bc", (ctypes.c_int32 * 2) * 3),
        ("cylinder", ctypes.c_int32),
        ("cyl_y", ctypes.c_double), ("cyl_z", ctypes.c_double), ("cyl_r", ctypes.c_double),
        ("body_force", ctypes.c_double * 3),
        ("stream", ctypes.c_void_p),
        ("reduce_every", ctypes.c_int32),
        ("step_kernel", ctypes.c_int32),
        ("wall_psi", ctypes.c_int32),
    ]


class lbm_fused_plan_t(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("config", "tile_x", "tile_y", "full_rows", "prefetch",
                                               "z_chunk", "xcd_order", "hints", "addr64",
                                               "solid_free_lo", "solid_free_hi")] + [
        ("workgroups", ctypes.c_int64)]


class LbmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None

_D = ctypes.c_double
_P = ctypes.c_void_p
_SIGS = {
    "lbm_params_default": (ctypes.c_int, [ctypes.POINTER(lbm_params)]),
    "lbm_create": (ctypes.c_int, [ctypes.POINTER(lbm_params), ctypes.POINTER(_P)]),
    "lbm_destroy": (ctypes.c_int, [_P]),
    "lbm_last_error": (ctypes.c_char_p, [_P]),
    "lbm_init_droplet": (ctypes.c_int, [_P, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D,
                                        ctypes.c_uint64]),
    "lbm_init_fields": (ctypes.c_int, [_P, _P, _P]),
    "lbm_set_populations": (ctypes.c_int, [_P, _P]),
    "lbm_get_populations": (ctypes.c_int, [_P, _P]),
    "lbm_step": (ctypes.c_int, [_P, ctypes.c_int64]),
    "lbm_steps_done": (ctypes.c_int64, [_P]),
    "lbm_moments": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "lbm_liquid_stats": (ctypes.c_int, [_P, _D, _D, _D, ctypes.c_int32, _P, _P, _P]),
    "lbm_totals_noalloc": (ctypes.c_int, [_P, _P]),
    "lbm_synchronize": (ctypes.c_int, [_P]),
    "lbm_health_status": (ctypes.c_int, [_P, ctypes.c_int32]),
    "lbm_copy_bandwidth": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(_D)]),
    "lbm_kernel_times": (ctypes.c_int, [_P, ctypes.c_int64, _P, _P, ctypes.c_int32, _P]),
    "lbm_coexistence": (ctypes.c_int, [ctypes.POINTER(lbm_params), ctypes.POINTER(_D),
                                       ctypes.POINTER(_D)]),
    "lbm_footprint_bytes": (ctypes.c_int64, [ctypes.POINTER(lbm_params)]),
    "lbm_fused_plan": (ctypes.c_int, [ctypes.POINTER(lbm_params), ctypes.c_int32,
                                      ctypes.POINTER(lbm_fused_plan_t)]),
    "lbm_batch_create": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P, ctypes.POINTER(_P)]),
    "lbm_batch_run": (ctypes.c_int, [_P, ctypes.c_int64]),
    "lbm_batch_destroy": (ctypes.c_int, [_P]),
    "lbm_batch_last_error": (ctypes.c_char_p, []),
}


def library():
    """Load liblbm_hip.so (built in-tree by build.build()); fail loudly if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBRARY):
            raise ImportError(f"{LIBRARY} is missing: build it with "
                              "paper_2306_16274_amd.build.build()")
        lib = ctypes.CDLL(LIBRARY)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(status, ctx=None):
    if status != LBM_OK:
        msg = library().lbm_last_error(ctx)
        raise LbmError(status, msg.decode() if msg else "")


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def lbm_params_default():
    p = lbm_params()
    _check(library().lbm_params_default(ctypes.byref(p)))
    return p


def lbm_create(params):
    ctx = ctypes.c_void_p()
    _check(library().lbm_create(ctypes.byref(params), ctypes.byref(ctx)))
    return ctx


def lbm_destroy(ctx):
    _check(library().lbm_destroy(ctx))


def lbm_last_error(ctx=None):
    msg = library().lbm_last_error(ctx)
    return msg.decode() if msg else ""


def lbm_init_droplet(ctx, cx, cy, cz, R, W, rho_in, rho_out, ux=0.0, uy=0.0, uz=0.0,
                     noise_amp=0.0, seed=0):
    _check(library().lbm_init_droplet(ctx, cx, cy, cz, R, W, rho_in, rho_out, ux, uy, uz,
                                      noise_amp, seed), ctx)


def lbm_init_fields(ctx, rho, u=None):
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    uu = None if u is None else np.ascontiguousarray(u, dtype=np.float64)
    _check(library().lbm_init_fields(ctx, _ptr(rho), None if uu is None else _ptr(uu)), ctx)


def lbm_set_populations(ctx, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    _check(library().lbm_set_populations(ctx, _ptr(f)), ctx)


def lbm_get_populations(ctx, Q, shape):
    """Returns f_bar(x, t) as an array (Q, nz, ny, nx)."""
    out = np.empty((Q,) + tuple(shape), dtype=np.float64)
    _check(library().lbm_get_populations(ctx, _ptr(out)), ctx)
    return out


def lbm_step(ctx, nsteps):
    _check(library().lbm_step(ctx, int(nsteps)), ctx)


def lbm_steps_done(ctx):
    return library().lbm_steps_done(ctx)


def lbm_moments(ctx, shape, want=("rho", "u", "p", "totals")):
    """Returns dict with rho (nz,ny,nx), u (3,nz,ny,nx), p, totals (5,) as requested."""
    out = {}
    rho = np.empty(shape) if "rho" in want else None
    u = np.empty((3,) + tuple(shape)) if "u" in want else None
    p = np.empty(shape) if "p" in want else None
    tot = np.empty(5) if "totals" in want else None
    _check(library().lbm_moments(ctx, None if rho is None else _ptr(rho),
                                 None if u is None else _ptr(u),
                                 None if p is None else _ptr(p),
                                 None if tot is None else _ptr(tot)), ctx)
    for k, v in (("rho", rho), ("u", u), ("p", p), ("totals", tot)):
        if v is not None:
            out[k] = v
    return out


def lbm_totals_noalloc(ctx, totals_dev_ptr):
    """Enqueue the five totals into a device array of 5 float64 (address as an int)."""
    _check(library().lbm_totals_noalloc(ctx, ctypes.c_void_p(int(totals_dev_ptr))), ctx)


def lbm_liquid_stats(ctx, nz, threshold, rho_v, rho_l, reach=1):
    """Returns (count_z, wetted_z: int64 arrays of nz, volume float)."""
    cz = np.empty(nz, dtype=np.int64)
    wz = np.empty(nz, dtype=np.int64)
    vol = ctypes.c_double(0.0)
    _check(library().lbm_liquid_stats(ctx, threshold, rho_v, rho_l, reach, _ptr(cz), _ptr(wz),
                                      ctypes.byref(vol)), ctx)
    return cz, wz, float(vol.value)


def lbm_copy_bandwidth(nbytes=2 << 30, reps=20):
    """GB/s (read + write) of the library's streaming copy on the current device."""
    v = ctypes.c_double(0.0)
    _check(library().lbm_copy_bandwidth(nbytes, reps, ctypes.byref(v)))
    return float(v.value)


def lbm_kernel_times(ctx, nsteps, cap=8):
    """Returns {kernel name: mean duration in ms} over nsteps timed steps."""
    avg = (ctypes.c_double * cap)()
    names = (ctypes.c_char_p * cap)()
    count = ctypes.c_int32()
    _check(library().lbm_kernel_times(ctx, int(nsteps), ctypes.cast(avg, _P),
                                      ctypes.cast(names, _P), cap, ctypes.byref(count)), ctx)
    return {names[k].decode(): avg[k] for k in range(count.value)}


def lbm_synchronize(ctx):
    _check(library().lbm_synchronize(ctx), ctx)


def lbm_health_status(ctx, wait=False):
    """LBM_OK or LBM_ENONFINITE (returned, not raised): the last completed health check."""
    st = library().lbm_health_status(ctx, 1 if wait else 0)
    if st not in (LBM_OK, LBM_ENONFINITE):
        _check(st, ctx)
    return st


def lbm_coexistence(params):
    rv, rl = ctypes.c_double(), ctypes.c_double()
    _check(library().lbm_coexistence(ctypes.byref(params), ctypes.byref(rv), ctypes.byref(rl)))
    return rv.value, rl.value


def lbm_footprint_bytes(params):
    return library().lbm_footprint_bytes(ctypes.byref(params))


def lbm_fused_plan(params, cus=256):
    """Launch plan of the fused step for these parameters on a device with `cus` compute
    units (host-only): a dict with the fields of lbm_fused_plan_t."""
    out = lbm_fused_plan_t()
    _check(library().lbm_fused_plan(ctypes.byref(params), int(cus), ctypes.byref(out)))
    return {n: getattr(out, n) for n, _ in lbm_fused_plan_t._fields_}


def _check_batch(status):
    if status != LBM_OK:
        msg = library().lbm_batch_last_error()
        raise LbmError(status, msg.decode() if msg else "")


def lbm_batch_create(ctxs, steps_per_launch, stream=None):
    arr = (ctypes.c_void_p * len(ctxs))(*[c.value if isinstance(c, ctypes.c_void_p) else c
                                          for c in ctxs])
    out = ctypes.c_void_p()
    _check_batch(library().lbm_batch_create(ctypes.cast(arr, _P), len(ctxs),
                                            int(steps_per_launch), stream, ctypes.byref(out)))
    return out


def lbm_batch_run(batch, nlaunch):
    _check_batch(library().lbm_batch_run(batch, int(nlaunch)))


def lbm_batch_destroy(batch):
    _check_batch(library().lbm_batch_destroy(batch))


def lbm_batch_last_error():
    msg = library().lbm_batch_last_error()
    return msg.decode() if msg else ""


class Lattice:
    """Owns one context; a convenience wrapper over the functions above."""

    def __init__(self, params, use_torch_stream=True):
        if use_torch_stream and params.stream is None and torch.cuda.is_available():
            params.stream = torch.cuda.current_stream().cuda_stream
        self.params = params
        self.Q = params.lattice
        self.shape = (params.nz, params.ny, params.nx)
        self.ctx = lbm_create(params)

    def close(self):
        if self.ctx is not None:
            lbm_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_droplet(self, *a, **k):
        lbm_init_droplet(self.ctx, *a, **k)

    def init_fields(self, rho, u=None):
        lbm_init_fields(self.ctx, rho, u)

    def set_populations(self, f):
        lbm_set_populations(self.ctx, f)

    def get_populations(self):
        return lbm_get_populations(self.ctx, self.Q, self.shape)

    def step(self, n=1):
        lbm_step(self.ctx, n)

    def moments(self, want=("rho", "u", "p", "totals")):
        return lbm_moments(self.ctx, self.shape, want)

    def liquid_stats(self, threshold, rho_v, rho_l, reach=1):
        return lbm_liquid_stats(self.ctx, self.shape[0], threshold, rho_v, rho_l, reach)

    def synchronize(self):
        lbm_synchronize(self.ctx)

    def kernel_times(self, nsteps):
        return lbm_kernel_times(self.ctx, nsteps)

"""The C-ABI library loads and exports every entry point declared in include/lbm.h, and
the ctypes mirror of lbm_params has the C layout (no GPU needed)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for need in ("lbm_create", "lbm_init_droplet", "lbm_step", "lbm_moments", "lbm_destroy"):
        assert need in names


def test_library_exports_every_declared_symbol():
    from paper_2306_16274_amd import lbm
    lib = lbm.library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", lbm.LIBRARY], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (lbm_\w+)", out))
    assert set(declared_functions()) <= exported


def test_params_struct_layout_matches_c(tmp_path):
    import ctypes
    from paper_2306_16274_amd import lbm
    fields = [f[0] for f in lbm.lbm_params._fields_]
    src = tmp_path / "layout.c"
    body = "".join(f'printf("{f} %zu\\n", offsetof(lbm_params, {f}));' for f in fields)
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "lbm.h"\n'
                   'int main(void){' + body + 'printf("size %zu\\n", sizeof(lbm_params));'
                   'return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True,
                                                       text=True, check=True).stdout.splitlines())
    for f in fields:
        assert int(got[f]) == getattr(lbm.lbm_params, f).offset, f
    assert int(got["size"]) == ctypes.sizeof(lbm.lbm_params)


def test_host_only_entry_points_without_gpu():
    """Parameter defaults, validation, footprint and the coexistence solver run on the host."""
    from paper_2306_16274_amd import lbm
    p = lbm.lbm_params_default()
    assert p.lattice == 19 and p.nx == 64
    assert lbm.lbm_footprint_bytes(p) == 2 * 19 * 64 ** 3 * 4 + 64 ** 3 * 4 + 64 ** 3
    p.cylinder = 1                # the fused step's link words: 4 more bytes per node
    assert lbm.lbm_footprint_bytes(p) == 2 * 19 * 64 ** 3 * 4 + 64 ** 3 * 4 + 64 ** 3 * 5
    p.cylinder = 0
    rv, rl = lbm.lbm_coexistence(p)
    assert 0.009 < rv < 0.0095 and 0.355 < rl < 0.36
    bad = lbm.lbm_params_default()
    bad.lattice = 15
    with pytest.raises(lbm.LbmError) as ei:
        lbm.lbm_create(bad)
    assert ei.value.status == lbm.LBM_EINVAL and "lattice" in str(ei.value)


def test_coexistence_agrees_with_oracle_maxwell():
    """The library's host-side Maxwell solver (Gauss-Legendre, bisection) and the oracle's
    (scipy quadrature, Brent) are independent implementations of the same construction."""
    from oracle import eos
    from paper_2306_16274_amd import lbm
    for t in (0.5, 0.55, 0.6, 0.7):
        p = lbm.lbm_params_default()
        p.T_over_Tc = t
        rv, rl = lbm.lbm_coexistence(p)
        ov, ol = eos.maxwell_densities(eos.CarnahanStarling(0.5, 4, 1, t), 1e-9, 0.7)
        assert abs(rv - ov) / ov < 1e-8 and abs(rl - ol) / ol < 1e-10
    p = lbm.lbm_params_default()
    p.eos = lbm.LBM_EOS_PIECEWISE
    rv, rl = lbm.lbm_coexistence(p)
    assert abs(rv - 0.001) < 1e-8 and abs(rl - 1.0) < 1e-7


def _bad(**changes):
    from paper_2306_16274_amd import lbm
    p = lbm.lbm_params_default()
    for k, v in changes.items():
        if k == "bc":
            p.bc[0][1] = v
        elif k == "body_force":
            p.body_force[2] = v
        else:
            setattr(p, k, v)
    return p


@pytest.mark.parametrize("changes,message", [
    (dict(lattice=15), "lattice"),
    (dict(storage=7), "storage"),
    (dict(nx=0), "sizes"),
    (dict(nz=70000), "grid"),
    (dict(nx=2048, ny=2048, nz=1024), "2^31"),
    (dict(eos=5), "eos"),
    (dict(G=0.5), "G must be negative"),
    (dict(cs_a=-1.0), "Carnahan"),
    (dict(eos=1, pw_theta_m=0.1), "piecewise"),
    (dict(nu_l=0.0), "viscosit"),
    (dict(nu_l=-0.1), "viscosit"),
    (dict(s4=2.5), "relaxation rate"),
    (dict(s2b=0.0), "relaxation rate"),
    (dict(sigma=float("nan")), "non-finite"),
    (dict(body_force=float("inf")), "non-finite"),
    (dict(cylinder=1, cyl_r=0.0), "cylinder radius"),
    (dict(cylinder=1, cyl_y=32.0, cyl_z=32.0, cyl_r=200.0), "no fluid"),
    (dict(bc=3), "boundary"),
    (dict(reduce_every=-1), "reduce_every"),
    (dict(step_kernel=9), "step_kernel"),
    (dict(lattice=27, storage=0, nx=512, ny=512, nz=512), "4 GiB"),
    (dict(T_over_Tc=1.2), "two-phase"),
])
def test_create_rejects_invalid_parameters_before_touching_the_device(changes, message):
    """lbm_create validates on the host: every rejection is LBM_EINVAL with a message,
    without a GPU."""
    from paper_2306_16274_amd import lbm
    with pytest.raises(lbm.LbmError) as ei:
        lbm.lbm_create(_bad(**changes))
    assert ei.value.status == lbm.LBM_EINVAL
    assert message in str(ei.value), str(ei.value)

"""C-ABI checks that need no GPU: the library loads, exports every symbol
include/lbfe.h declares, struct layout agrees with the C compiler, argument
validation and the no-device path."""
import ctypes
import os
import re
import subprocess

import pytest
import torch

from paper_2504_03819_amd import lbfe
from oracle import eos

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbfe.h")


def declared_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(lbfe_\w+)\s*\(", txt, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 20
    L = lbfe.lib()
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", lbfe.LIB_PATH], capture_output=True, text=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}\b", out), n


def test_params_struct_layout_matches_c(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "lbfe.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu\\n\", sizeof(lbfe_params),"
        " offsetof(lbfe_params, a), offsetof(lbfe_params, omega), offsetof(lbfe_params, wet_value),"
        " offsetof(lbfe_params, rho_v), offsetof(lbfe_params, adjoint));return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    P = lbfe.Params
    assert vals == [ctypes.sizeof(P), P.a.offset, P.omega.offset, P.wet_value.offset, P.rho_v.offset, P.adjoint.offset]


def test_defaults_are_the_papers():
    p = lbfe.default_params()
    assert abs(p.a - 9 / 392) < 1e-17 and abs(p.b - 2 / 21) < 1e-17 and p.R == 1.0
    assert abs(p.T - 0.7 / 14) < 1e-15 and p.kappa == 0.02 and p.nu == 0.15
    assert list(p.omega) == [1.0] * 11 and p.corr4 == 1 and p.precision == lbfe.FP64


def test_coexistence_matches_oracle_maxwell():
    for tr in (0.7, 0.8, 0.85, 0.9):
        T = eos.temperature(tr)
        rl, rv = lbfe.coexistence(eos.PAPER["a"], eos.PAPER["b"], 1.0, T)
        ol, ov = eos.maxwell(eos.PAPER["a"], eos.PAPER["b"], 1.0, T)
        assert abs(rl - ol) < 1e-11 * ol and abs(rv - ov) < 1e-11 * ov
    with pytest.raises(lbfe.LBFEError):
        lbfe.coexistence(eos.PAPER["a"], eos.PAPER["b"], 1.0, 0.08)  # above T_c


@pytest.mark.parametrize("override", [
    dict(nu=0.0), dict(nu=float("nan")), dict(kappa=-1.0), dict(nx=0), dict(walls_z=1, nz=2),
    dict(precision=7), dict(wet_mode=1, wet_value=0.0), dict(wet_mode=2, wet_value=-0.5), dict(wet_mode=5),
    dict(rho_l=7.0), dict(rho_l=1.0, rho_v=2.0), dict(check_every=0), dict(corr4=2), dict(b=0.0),
    dict(nx=2048, ny=2048, nz=1024), dict(nx=32768, ny=16384, nz=1),
    dict(wall_u=(0.1, 0.0, 0.0, 0.0)), dict(walls_z=1, wall_u=(0.0, 0.0, 0.31, 0.0)),
    dict(walls_z=1, wall_u=(float("nan"), 0.0, 0.0, 0.0)),
    dict(solid_mask=2), dict(solid_mask=1, walls_z=1),
    # the moment-state path: the paper's unit rates, FP64/FP32, resting walls, no mask
    dict(step_path=4), dict(step_path=lbfe.PATH_STATE, precision=lbfe.FP16_DEV),
    dict(step_path=lbfe.PATH_STATE, precision=lbfe.FP16_DEV_F0FP32),
    dict(step_path=lbfe.PATH_STATE, omega=(1.0, 1.0, 1.0, 0.5) + (1.0,) * 7),
    dict(step_path=lbfe.PATH_STATE, omega=(0.9,) + (1.0,) * 10),
    dict(step_path=lbfe.PATH_STATE, walls_z=1, wall_u=(0.0, 0.0, 0.05, 0.0)),
    dict(step_path=lbfe.PATH_STATE, solid_mask=1),
])
def test_invalid_parameters_rejected_before_device(override):
    p = lbfe.default_params()
    for k, v in override.items():
        setattr(p, k, v)
    ctx = ctypes.c_void_p()
    assert lbfe.lib().lbfe_create(ctypes.byref(p), None, ctypes.byref(ctx)) == lbfe.E_INVAL
    assert ctx.value is None
    n = ctypes.c_size_t()
    assert lbfe.lib().lbfe_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == lbfe.E_INVAL


def test_solid_mask_workspace_holds_neighbour_words_and_phi():
    """A mask context adds one 32-bit neighbour word and three phi values
    (compute precision) per node to the workspace."""
    for prec, rb in ((lbfe.PRECISIONS["fp64"], 8), (lbfe.PRECISIONS["fp32"], 4)):
        p = lbfe.default_params(nx=40, ny=30, nz=20, precision=prec)
        a, b = ctypes.c_size_t(), ctypes.c_size_t()
        assert lbfe.lib().lbfe_workspace_bytes(ctypes.byref(p), ctypes.byref(a)) == lbfe.OK
        p.solid_mask = 1
        assert lbfe.lib().lbfe_workspace_bytes(ctypes.byref(p), ctypes.byref(b)) == lbfe.OK
        N = 40 * 30 * 20
        assert b.value - a.value >= (4 + 3 * rb) * N and b.value - a.value < (4 + 3 * rb) * N + 1024


def test_omega_range_checked_but_omega1_ignored():
    p = lbfe.default_params()
    p.omega[1] = float("nan")   # derived from nu, ignored
    n = ctypes.c_size_t()
    assert lbfe.lib().lbfe_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == lbfe.OK
    p.omega[4] = 2.5
    assert lbfe.lib().lbfe_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == lbfe.E_INVAL


def test_state_path_accepted_for_the_papers_rates():
    """Every rate but omega_1 at 1 (omega_1 itself comes from nu), FP64 or
    FP32, periodic or resting walls, with or without corr4."""
    for prec in (lbfe.FP64, lbfe.FP32):
        for extra in (dict(), dict(walls_z=1, wet_mode=1, wet_value=1.3), dict(corr4=0)):
            p = lbfe.default_params(precision=prec, step_path=lbfe.PATH_STATE, **extra)
            p.omega[1] = 0.4
            n = ctypes.c_size_t()
            assert lbfe.lib().lbfe_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == lbfe.OK, (prec, extra)


def test_workspace_size_accounts_for_forms_and_adjoint():
    sizes = {}
    for prec in (lbfe.FP64, lbfe.FP32, lbfe.FP16_DEV, lbfe.FP16_DEV_F0FP32):
        p = lbfe.default_params(nx=64, ny=64, nz=64, precision=prec)
        n = ctypes.c_size_t()
        assert lbfe.lib().lbfe_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == lbfe.OK
        sizes[prec] = n.value
    N = 64 ** 3
    assert sizes[lbfe.FP64] >= 2 * 27 * 8 * N and sizes[lbfe.FP32] >= 2 * 27 * 4 * N
    assert sizes[lbfe.FP64] > sizes[lbfe.FP32] > sizes[lbfe.FP16_DEV_F0FP32] > sizes[lbfe.FP16_DEV]
    p = lbfe.default_params(nx=64, ny=64, nz=64, adjoint=1)
    n = ctypes.c_size_t()
    lbfe.lib().lbfe_workspace_bytes(ctypes.byref(p), ctypes.byref(n))
    assert n.value >= sizes[lbfe.FP64] + 2 * 27 * 8 * N


def test_null_and_no_device_paths():
    L = lbfe.lib()
    assert L.lbfe_last_error(None) == b"null context"
    assert L.lbfe_destroy(None) == lbfe.OK
    assert L.lbfe_step(None, 1) == lbfe.E_INVAL
    assert L.lbfe_params_default(None) == lbfe.E_INVAL
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    p = lbfe.default_params()
    ctx = ctypes.c_void_p()
    assert L.lbfe_create(ctypes.byref(p), None, ctypes.byref(ctx)) == lbfe.E_DEVICE

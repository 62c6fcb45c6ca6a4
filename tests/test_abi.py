"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every function include/bpm.h declares, arguments are validated, and
the plan's FP64 constants agree with the oracle's independently computed
ones."""

import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bpm.h")


def _lib():
    from paper_2201_08500_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        from paper_2201_08500_amd.build import build
        build()
    return _native


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(bpm_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_abi():
    names = declared_functions()
    for must in ("bpm_plan_create", "bpm_propagate", "bpm_plan_destroy",
                 "bpm_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    N = _lib()
    handle = ctypes.CDLL(N.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(handle, n)]
    assert not missing, missing


C = dict(chi0=complex(-1.5e-5, 1e-8), chih=complex(3.8e-6, 0.9e-8),
         chihbar=complex(3.8e-6, 0.9e-8))


def plan(N, **over):
    kw = dict(Nx=1024, dx=0.5e-6, dz=0.5e-6, Nz=10, theta_B=math.pi / 4,
              lam=1.24e-10, Nomega=4, **C)
    kw.update(over)
    return N.Plan(**kw)


@pytest.mark.parametrize("bad", [
    dict(Nx=1000), dict(Nx=128), dict(Nx=8192), dict(Nz=0), dict(Nomega=0),
    dict(dx=0.0), dict(dz=-1e-6), dict(lam=0.0), dict(theta_B=0.0),
    dict(theta_B=math.pi / 2), dict(dx=float("nan")),
])
def test_plan_create_rejects_invalid_arguments(bad):
    N = _lib()
    with pytest.raises(N.BpmError) as e:
        plan(N, **bad)
    assert e.value.code == -1 and str(e.value)


def test_setters_validate_and_freeze_rules():
    N = _lib()
    L = N.lib()
    p = plan(N)
    assert L.bpm_plan_set_precision(p.handle, 7) == -1
    assert "precision" in N.last_error()
    assert L.bpm_plan_set_crystal(p.handle, float("nan"), 1.0) == -1
    assert L.bpm_plan_set_crystal(p.handle, 0.0, -1.0) == -1
    assert L.bpm_plan_set_crystal(p.handle, -1e-5, math.inf) == 0
    assert L.bpm_plan_set_options(p.handle, 3, 1) == -1
    assert L.bpm_plan_set_options(p.handle, 1, 2) == -1
    assert L.bpm_plan_set_options(p.handle, 1, 0) == 0
    assert L.bpm_plan_set_options(p.handle, 2, 1) == 0
    assert L.bpm_plan_set_options(p.handle, 4, 1) == 0
    m = np.zeros((10, 1024), np.uint8)
    assert L.bpm_plan_set_mask(p.handle, m.ctypes.data_as(ctypes.c_void_p)) == 0
    assert L.bpm_plan_set_mask(p.handle, None) == 0
    assert L.bpm_plan_set_time_grid(p.handle, 1e-15) == -1        # Nomega = 4
    assert L.bpm_plan_set_time_grid(p.handle, -1.0) == -1
    bad = (ctypes.c_double * 4)(0.0, -2.0, 0.0, 0.0)
    assert L.bpm_plan_set_detuning(p.handle, bad) == -1
    assert L.bpm_plan_set_detuning(p.handle, None) == -1
    p.close()
    assert L.bpm_plan_set_precision(None, 0) == -1


def test_propagate_rejects_null_buffers_before_touching_the_device():
    N = _lib()
    L = N.lib()
    p = plan(N)
    rc = L.bpm_propagate_ws(p.handle, None, None, None, None, None, None)
    assert rc == -1 and "non-NULL" in N.last_error()
    x = ctypes.c_void_p(0x1000)
    rc = L.bpm_propagate_ws(p.handle, x, None, x, ctypes.c_void_p(0x2000), None, None)
    assert rc == -1 and "alias" in N.last_error()
    rc = L.bpm_propagate_ws(p.handle, x, ctypes.c_void_p(0x3000),
                            ctypes.c_void_p(0x2000), ctypes.c_void_p(0x4000), None, None)
    assert rc == -1 and "workspace" in N.last_error()
    assert L.bpm_propagate_ws(None, x, None, x, x, None, None) == -1


def test_workspace_bytes():
    N = _lib()
    assert plan(N, precision="fp64").workspace_bytes() == 1024 * 10 * 16
    assert plan(N, precision="fp32").workspace_bytes() == 1024 * 10 * 8
    assert plan(N, precision="fp32s").workspace_bytes() == 1024 * 10 * 8


@pytest.mark.parametrize("chihbar,zas", [(C["chih"], True),
                                         (complex(2.2e-6, -0.5e-8), True),
                                         (C["chih"], False)])
def test_plan_constants_match_oracle(chihbar, zas):
    import oracle as O
    N = _lib()
    deltas = np.array([-4e-5, -1e-6, 0.0, 2.5e-5])
    p = plan(N, chihbar=chihbar, delta=deltas, zassenhaus=zas)
    po = O.Problem(1024, 0.5e-6, 0.5e-6, 10, C["chi0"], C["chih"], chihbar,
                   math.pi / 4, 1.24e-10, deltas, zassenhaus=zas)
    for w, d in enumerate(deltas):
        k, c, d0r, d0i, dpr, dpi, dmr, dmi = p.constants(w)
        ko, co, _ = O.slice_constants(po, d)
        d0, dp1, dm1 = O.coupling_constants(po, d)
        assert abs(k / ko - 1) < 1e-15 and abs(c / co - 1) < 1e-15
        assert abs(complex(d0r, d0i) - d0) < 2e-15
        assert abs(complex(dpr, dpi) - dp1) < 2e-15 * abs(dp1) + 1e-17
        assert abs(complex(dmr, dmi) - dm1) < 2e-15 * abs(dm1) + 1e-17


@pytest.mark.parametrize("order", [2, 4])
def test_substep_constants_match_oracle(order):
    """First B sub-step of the second- and fourth-order schemes (length
    b_0 dz, Eq. split-op) against the oracle's coupling constants."""
    import oracle as O
    N = _lib()
    deltas = np.array([-3e-5, 0.0, 1.5e-5, 4e-5])
    p = plan(N, delta=deltas, split_order=order)
    po = O.Problem(1024, 0.5e-6, 0.5e-6, 10, C["chi0"], C["chih"], C["chih"],
                   math.pi / 4, 1.24e-10, deltas, split_order=order)
    b0 = O.split_coefficients(order)[1][0]
    for w, d in enumerate(deltas):
        _, _, d0r, d0i, dpr, dpi, dmr, dmi = p.constants(w)
        d0, dp1, dm1 = O.coupling_constants(po, d, b0)
        assert abs(complex(d0r, d0i) - d0) < 2e-15
        assert abs(complex(dpr, dpi) - dp1) < 2e-15 * abs(dp1) + 1e-17
        assert abs(complex(dmr, dmi) - dm1) < 2e-15 * abs(dm1) + 1e-17


def test_default_detuning_grid_spans_ten_darwin_widths():
    import workloads as W
    N = _lib()
    p = plan(N, Nomega=8)
    eps = W.darwin_relative_width(C["chih"], C["chihbar"], math.pi / 4)
    expect = W.detuning_grid(8, eps)
    k0 = 2 * math.pi / 1.24e-10
    for w in range(8):
        assert abs(p.constants(w)[0] / (k0 * (1 + expect[w])) - 1) < 1e-15
    assert abs(plan(N, Nomega=1).constants(0)[0] / k0 - 1) < 1e-16


def test_too_long_step_is_rejected_at_use():
    N = _lib()
    p = plan(N, dz=1e-3)   # |q| ~ 7e4: far outside the two-beam expansion
    with pytest.raises(N.BpmError) as e:
        p.constants(0)
    assert "too long" in str(e.value)


@pytest.mark.parametrize("bad", [dict(Nx=1), dict(Nx=8193), dict(Ny=0), dict(Ny=33),
                                 dict(dy=0.0), dict(dz=0.0), dict(Nz=0)])
def test_plan_create_3d_rejects_invalid_arguments(bad):
    N = _lib()
    kw = dict(Nx=60, Ny=4, dx=0.5e-6, dy=2e-6, dz=0.5e-6, Nz=10, theta_B=math.pi / 4,
              lam=1.24e-10, Nomega=2, **C)
    kw.update(bad)
    with pytest.raises(N.BpmError):
        N.Plan3D(**kw)


def test_plan_3d_workspace_and_setters():
    N = _lib()
    L = N.lib()
    p = N.Plan3D(60, 4, 0.5e-6, 2e-6, 0.5e-6, 10, C["chi0"], C["chih"], C["chihbar"],
                 math.pi / 4, 1.24e-10, 3, precision="fp32s")
    # the deformation table only (the plan keeps its row propagators)
    assert p.workspace_bytes() == 60 * 4 * 10 * 8
    assert p.field_shape == (3, 4, 60) and p.u_shape == (10, 4, 60)
    assert L.bpm_plan_set_options(p.handle, 3, 1) == -1          # no such order
    assert L.bpm_plan_set_options(p.handle, 4, 1) == 0
    assert L.bpm_plan_set_options(p.handle, 1, 0) == 0
    m = np.ones((10, 4, 60), dtype=np.uint8)          # [Nz][Ny][Nx]
    assert L.bpm_plan_set_mask(p.handle, m.ctypes.data_as(ctypes.c_void_p)) == 0
    assert L.bpm_plan_set_mask(p.handle, None) == 0
    assert L.bpm_plan_set_schedule(p.handle, 1) == -4
    p.close()

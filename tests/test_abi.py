"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, its structs match the ctypes layout, and argument validation
(which runs before any HIP call) reports the documented status codes."""

import ctypes
import os
import re
import subprocess

import pytest

from paper_1801_05977_amd import qpgf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qpgf.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qpgf_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = qpgf.lib()
    names = _declared()
    assert "qpgf_plan_create" in names and "qpgf_gd3d" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(qpgf.EXPORTS)


def test_struct_layout_matches_header(tmp_path):
    prog = tmp_path / "sz.c"
    prog.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "qpgf.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(qpgf_params),"
        " offsetof(qpgf_params, lattice_rmin), sizeof(qpgf_plan_info), offsetof(qpgf_plan_info, far_grid_bytes),"
        " offsetof(qpgf_params, quad_q), offsetof(qpgf_params, sing_order), offsetof(qpgf_params, far_m),"
        " offsetof(qpgf_params, maxwell_trace), offsetof(qpgf_plan_info, far_m1),"
        " offsetof(qpgf_plan_info, far_points), offsetof(qpgf_plan_info, far_points_t));"
        "printf(\"%zu %zu %zu\\n\", sizeof(qpgf_train_cfg), offsetof(qpgf_train_cfg, member),"
        " offsetof(qpgf_train_cfg, seed));return 0;}\n")
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(prog), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [ctypes.sizeof(qpgf.Params), qpgf.Params.lattice_rmin.offset, ctypes.sizeof(qpgf.PlanInfo),
            qpgf.PlanInfo.far_grid_bytes.offset, qpgf.Params.quad_q.offset, qpgf.Params.sing_order.offset,
            qpgf.Params.far_m.offset, qpgf.Params.maxwell_trace.offset, qpgf.PlanInfo.far_m1.offset,
            qpgf.PlanInfo.far_points.offset, qpgf.PlanInfo.far_points_t.offset, ctypes.sizeof(qpgf.TrainCfg), qpgf.TrainCfg.member.offset,
            qpgf.TrainCfg.seed.offset]
    assert got == want


def test_params_default_values():
    p = qpgf.default_params(qpgf.KIND_GD3D, qpgf.C64, 256, 256, 64)
    assert (p.kind, p.prec, p.m1, p.m2, p.m3) == (1, 1, 256, 256, 64)
    assert (p.c, p.c_tilde, p.eps, p.quad_q) == (0.6, 1.0, 0.2, 64)
    assert p.far_h == 0.0                                # automatic, per instance
    assert p.far_zmax == 1.0 and p.wood_tol == 1e-3
    assert p.sing_order == 1 and p.ring_interp == 0
    assert p.far_m == 0 and p.maxwell_trace == 0


@pytest.mark.parametrize("field,value,status", [
    ("m1", 100, 4), ("m2", 8, 4), ("m3", 3, 4), ("c", 1.5, 1), ("eps", 0.6, 1), ("quad_q", 4, 1),
    ("far_h", -1.0, 1), ("far_h", 1e-7, 1), ("kind", 9, 1), ("prec", 5, 1), ("sing_order", 0, 1), ("sing_order", 4, 1),
    ("sing_order", 2, 1),     # above 1 only for the 2D G (this plan is 3D)
    ("ring_interp", 2, 1), ("ring_interp", 1, 1),
    ("special_tol", 0.79, 1),  # at most two special coefficients per pencil needs special_tol < pi / (4 c~)
    ("far_m", 100, 4), ("far_m", 8, 4), ("far_m", 4096, 4),   # complex128 3D: the far x2 axis is a column axis
    ("maxwell_trace", 1, 1), ("maxwell_trace", 2, 1),        # the trace variant is a Maxwell option
])
def test_plan_create_rejects_bad_params(field, value, status):
    L = qpgf.lib()
    p = qpgf.default_params(qpgf.KIND_GD3D, qpgf.C128, 64, 64, 32)
    setattr(p, field, value)
    h = ctypes.c_void_p()
    st = L.qpgf_plan_create(ctypes.byref(p), ctypes.byref(h))
    assert st == status
    assert not h.value
    assert L.qpgf_last_error().decode()


@pytest.mark.parametrize("kind", [qpgf.KIND_G2D, qpgf.KIND_G2D_GRAD, qpgf.KIND_G2D_HESS_DIFF, qpgf.KIND_GD3D])
@pytest.mark.parametrize("m1", [15, 18, 36, 90, 100, 4104, 8192])
def test_plan_create_rejects_x1_sizes_outside_the_transform_lengths(kind, m1):
    """x1 sizes are 2^a r with a >= 1 and r in {1, 3, 5, 7} in 2D (powers of two in 3D), 16 .. 4096."""
    L = qpgf.lib()
    p = qpgf.default_params(kind, qpgf.C128, m1, 32, 32)
    h = ctypes.c_void_p()
    assert L.qpgf_plan_create(ctypes.byref(p), ctypes.byref(h)) == 4
    assert not h.value and "m1" in L.qpgf_last_error().decode()


@pytest.mark.parametrize("m1", [24, 96, 768, 1280, 1792])
def test_plan_create_rejects_mixed_radix_x1_in_3d(m1):
    L = qpgf.lib()
    p = qpgf.default_params(qpgf.KIND_GD3D, qpgf.C128, m1, 32, 32)
    h = ctypes.c_void_p()
    assert L.qpgf_plan_create(ctypes.byref(p), ctypes.byref(h)) == 4
    assert not h.value


def test_null_arguments():
    L = qpgf.lib()
    assert L.qpgf_plan_create(None, None) == 1
    assert L.qpgf_prepare(None, 1.0, 0.1, 0.2) == 1
    assert L.qpgf_evaluate(None, None, 0, None, None) == 1
    assert L.qpgf_version().decode().startswith("qpgf")


def test_surrogate_entry_points_validate_before_touching_the_device():
    import ctypes
    from oracle import mlp as ref
    L = qpgf.lib()
    assert L.qpgf_mlp_param_count() == ref.N_PARAM
    h = ctypes.c_void_p()
    assert L.qpgf_mlp_create(0, 64, 0, ctypes.byref(h)) == 1
    assert L.qpgf_mlp_create(1, 100, 0, ctypes.byref(h)) == 1      # max_batch not a multiple of 64
    assert L.qpgf_mlp_create(9, 64, 0, ctypes.byref(h)) == 1
    assert not h.value
    assert L.qpgf_mlp_forward(None, 0, None, 0, None) == 1
    assert L.qpgf_mlp_gradient(None, 0, None, None, 64, None, None) == 1
    assert L.qpgf_mlp_last_error().decode()
    assert L.qpgf_evaluate_smooth(None, None, 0, None) == 1
    assert L.qpgf_surrogate_eval(None, None, 0.0, 0.0, 0.0, 0, None, None, None, None, None, None, None,
                                 None) == 1


def test_surrogate_training_and_checkpoint_entry_points_validate():
    L = qpgf.lib()
    one = (ctypes.c_double * 1)(1.0)
    off = (ctypes.c_int64 * 2)(0, 0)
    cfg = qpgf.TrainCfg(batch=64, steps=1, lr_max=1e-3, lr_min=0.0, member=-1, reserved=0, seed=0)
    kap = ctypes.c_double()
    assert L.qpgf_mlp_set_calibration(None, 1.0) == 1
    assert L.qpgf_mlp_get_calibration(None, ctypes.byref(kap)) == 1
    assert L.qpgf_surrogate_make_data(None, None, 1, one, one, one, off, None, None, None) == 1
    assert L.qpgf_surrogate_train(None, None, None, 64, ctypes.byref(cfg), None) == 1
    assert L.qpgf_surrogate_calibrate(None, None, 1, one, one, one, off, None, 1.0, 2.0, ctypes.byref(kap)) == 1
    assert L.qpgf_mlp_save(None, b"/nonexistent/x") == 1
    assert L.qpgf_mlp_load(None, b"/nonexistent/x") == 1
    assert "NULL" in L.qpgf_mlp_last_error().decode()


def test_workspace_entry_points_validate():
    L = qpgf.lib()
    n = ctypes.c_size_t()
    assert L.qpgf_plan_workspace_bytes(None, 1.0, 10, ctypes.byref(n)) == 1
    assert L.qpgf_plan_set_workspace(None, None, 0, 1.0, 10) == 1
    assert "NULL" in L.qpgf_last_error().decode()

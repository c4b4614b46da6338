"""The C-ABI library loads, exports every entry point include/fcn.h declares, and rejects
invalid plans on the host (no GPU call is made by these tests)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1507_05988_amd import fcn, workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "fcn.h")).read()
    return sorted(set(re.findall(r"^\s*(?:fcn_status|const char \*)\s*(fcn_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(fcn.LIB_PATH):
        from paper_1507_05988_amd import build
        build.build()
    return fcn.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(fcn.EXPORTED)


def _create(lib, insts, **opt):
    arr = (fcn.Instance * len(insts))(*[fcn.make_instance(i) for i in insts])
    o = fcn.Options(precision=opt.get("precision", 0), adaptive=opt.get("adaptive", 0),
                    max_phase=opt.get("max_phase", 0.05), dz_min=opt.get("dz_min", 1e-6),
                    dz_max=opt.get("dz_max", 1e-2), use_graph=0, col_tile=opt.get("col_tile", 0),
                    col_rows=opt.get("col_rows", 0), lanes=0)
    h = ctypes.c_void_p()
    rc = lib.fcn_plan_create(arr, len(insts), ctypes.byref(o), ctypes.byref(h))
    return rc, h


def test_plan_sizes_on_host(lib):
    insts = wl.config_batch(count=5)
    rc, h = _create(lib, insts, precision=1)
    assert rc == fcn.FCN_OK
    sz = ctypes.c_size_t()
    assert lib.fcn_field_size(h, ctypes.byref(sz)) == 0
    assert sz.value == sum(i["nr"] * i["nt"] for i in insts)
    offs = []
    for i in range(5):
        assert lib.fcn_field_offset(h, i, ctypes.byref(sz)) == 0
        offs.append(sz.value)
    assert offs[0] == 0 and all(offs[i + 1] - offs[i] == insts[i]["nr"] * insts[i]["nt"] for i in range(4))
    assert lib.fcn_field_offset(h, 5, ctypes.byref(sz)) == fcn.FCN_E_ARG
    assert lib.fcn_diag_record_size(h, ctypes.byref(sz)) == 0
    assert sz.value == sum(8 + i["nr"] for i in insts)
    assert lib.fcn_plan_workspace_size(h, ctypes.byref(sz)) == 0 and sz.value > 0
    # compute calls before bind are refused with a state error
    assert lib.fcn_step(h, ctypes.c_void_p(0x1000), 1) == fcn.FCN_E_STATE
    assert b"not bound" in lib.fcn_last_error(h)
    assert lib.fcn_plan_destroy(h) == 0


@pytest.mark.parametrize("field,value,code", [
    ("nt", 100, fcn.FCN_E_ARG),          # not a power of two
    ("nt", 16384, fcn.FCN_E_SIZE),       # beyond the largest FFT
    ("nr", 2, fcn.FCN_E_ARG),
    ("nr", 4097, fcn.FCN_E_SIZE),
    ("r_max", -1.0, fcn.FCN_E_ARG),
    ("t_max", -1.0, fcn.FCN_E_ARG),
    ("K", 0, fcn.FCN_E_ARG),
    ("terms", 128, fcn.FCN_E_ARG),
    ("terms", 64 | 63, fcn.FCN_E_ARG),   # the avalanche term without an ionisation potential
    ("dz", 0.0, fcn.FCN_E_ARG),          # fixed mode needs dz > 0
    ("sigma_K", -1.0, fcn.FCN_E_ARG),
    ("n2", float("nan"), fcn.FCN_E_ARG),
])
def test_invalid_instances_rejected(lib, field, value, code):
    inst = wl.config_small()
    inst[field] = value
    rc, h = _create(lib, [inst])
    assert rc == code
    assert not h.value


def test_fp32_storage_mode_on_host(lib):
    """FCN_FP32_STORAGE plans: same field size as FP32, FP64 twiddle tables in the workspace."""
    insts = [wl.config_small(nr=64, nt=256), wl.config_small(nr=40, nt=512)]
    sizes = {}
    for prec in (fcn.FCN_FP32, fcn.FCN_FP32_STORAGE):
        rc, h = _create(lib, insts, precision=prec)
        assert rc == fcn.FCN_OK
        sz = ctypes.c_size_t()
        assert lib.fcn_field_size(h, ctypes.byref(sz)) == 0
        assert sz.value == 64 * 256 + 40 * 512
        assert lib.fcn_plan_workspace_size(h, ctypes.byref(sz)) == 0
        sizes[prec] = sz.value
        lib.fcn_plan_destroy(h)
    assert sizes[fcn.FCN_FP32_STORAGE] >= sizes[fcn.FCN_FP32] + 8 * (256 + 512)
    assert _create(lib, insts, precision=4)[0] == fcn.FCN_E_ARG


def test_fp32_cn64_mode_on_host(lib):
    """FCN_FP32_CN64 plans: the FP32 field size, and twiddle tables twice the FP32 ones (the
    low parts follow the high parts)."""
    insts = [wl.config_small(nr=64, nt=256), wl.config_small(nr=40, nt=512)]
    sizes = {}
    for prec in (fcn.FCN_FP32, fcn.FCN_FP32_CN64):
        rc, h = _create(lib, insts, precision=prec)
        assert rc == fcn.FCN_OK
        sz = ctypes.c_size_t()
        assert lib.fcn_field_size(h, ctypes.byref(sz)) == 0
        assert sz.value == 64 * 256 + 40 * 512
        assert lib.fcn_plan_workspace_size(h, ctypes.byref(sz)) == 0
        sizes[prec] = sz.value
        w, l, e = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        assert lib.fcn_plan_tiles(h, ctypes.byref(w), ctypes.byref(l), ctypes.byref(e)) == 0
        assert e.value == 8  # FP32 row arithmetic
        if prec == fcn.FCN_FP32_CN64:
            assert l.value == 8  # the FP64-arithmetic column solve keeps 8 rows per thread
        lib.fcn_plan_destroy(h)
    assert sizes[fcn.FCN_FP32_CN64] >= sizes[fcn.FCN_FP32] + 8 * (256 + 512)


def test_invalid_options_rejected(lib):
    inst = wl.config_small()
    assert _create(lib, [inst], precision=7)[0] == fcn.FCN_E_ARG
    assert _create(lib, [inst], adaptive=1, max_phase=0.0)[0] == fcn.FCN_E_ARG
    assert _create(lib, [inst], adaptive=1, dz_min=1e-2, dz_max=1e-3)[0] == fcn.FCN_E_ARG
    assert _create(lib, [inst], col_tile=3)[0] == fcn.FCN_E_ARG
    assert _create(lib, [inst], col_rows=5)[0] == fcn.FCN_E_ARG
    rc, h = _create(lib, [inst], adaptive=1)
    assert rc == 0
    lib.fcn_plan_destroy(h)


def test_bind_rejects_bad_workspace(lib):
    rc, h = _create(lib, [wl.config_small()])
    assert rc == 0
    sz = ctypes.c_size_t()
    lib.fcn_plan_workspace_size(h, ctypes.byref(sz))
    assert lib.fcn_plan_bind(h, None, sz.value, None) == fcn.FCN_E_ARG
    assert lib.fcn_plan_bind(h, ctypes.c_void_p(0x1001), sz.value, None) == fcn.FCN_E_ARG  # misaligned
    assert lib.fcn_plan_bind(h, ctypes.c_void_p(0x1000), sz.value - 1, None) == fcn.FCN_E_SIZE
    lib.fcn_plan_destroy(h)


def test_plan_without_gpu_raises():
    """The Python Plan has no CPU path: without a GPU it refuses to run."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(fcn.FcnError):
        fcn.Plan(wl.config_small())


def test_network_abi_validates_on_host(lib):
    """fcn_net_*: invalid arguments, an unbound network and an undersized workspace are errors
    returned before any GPU call."""
    h = ctypes.c_void_p()
    assert lib.fcn_net_create(0, 1, ctypes.byref(h)) == fcn.FCN_E_ARG
    assert lib.fcn_net_create(65, 1, ctypes.byref(h)) == fcn.FCN_E_ARG
    assert lib.fcn_net_create(8, 3, ctypes.byref(h)) == fcn.FCN_E_ARG
    assert lib.fcn_net_create(32, 1, ctypes.byref(h)) == fcn.FCN_OK
    n = ctypes.c_size_t()
    assert lib.fcn_net_param_count(h, ctypes.byref(n)) == fcn.FCN_OK
    # 4 layers of 5x5 complex weights and complex biases: 1->32->32->32->1
    assert n.value == 2 * 25 * (32 + 32 * 32 * 2 + 32) + 2 * (32 * 3 + 1)
    ws_inf, ws_tr = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.fcn_net_workspace_size(h, 4, 64, 64, 0, ctypes.byref(ws_inf)) == fcn.FCN_OK
    assert lib.fcn_net_workspace_size(h, 4, 64, 64, 1, ctypes.byref(ws_tr)) == fcn.FCN_OK
    assert ws_tr.value > ws_inf.value > 0
    assert lib.fcn_net_workspace_size(h, 0, 64, 64, 0, ctypes.byref(ws_inf)) == fcn.FCN_E_ARG
    # unbound network
    assert lib.fcn_net_forward(h, 1, 8, 8, None) == fcn.FCN_E_STATE
    assert lib.fcn_net_refresh(h) == fcn.FCN_E_STATE
    assert lib.fcn_net_adam(h, 1e-3, 0.9, 0.999, 1e-8) == fcn.FCN_E_STATE
    # bind: NULL buffers, training without gradients, misaligned or undersized workspace
    p = ctypes.c_void_p(0x1000)
    args = (4, 64, 64)
    assert lib.fcn_net_bind(h, None, None, None, None, p, ws_inf.value, *args, 0, None) == fcn.FCN_E_ARG
    assert lib.fcn_net_bind(h, p, None, None, None, p, ws_tr.value, *args, 1, None) == fcn.FCN_E_ARG
    assert lib.fcn_net_bind(h, p, None, None, None, ctypes.c_void_p(0x1010), ws_inf.value, *args, 0,
                            None) == fcn.FCN_E_ARG
    assert lib.fcn_net_bind(h, p, None, None, None, p, ws_inf.value - 1, *args, 0, None) == fcn.FCN_E_SIZE
    assert b"workspace" in lib.fcn_net_last_error(h)
    assert lib.fcn_net_destroy(h) == fcn.FCN_OK
    # the parareal combination validates its sizes on the host as well
    assert lib.fcn_parareal_update(p, p, p, p, p, 0, 16, p, 4, None) == fcn.FCN_E_ARG
    assert lib.fcn_parareal_update(p, p, p, p, p, 16, 16, p, 0, None) == fcn.FCN_E_ARG


def test_step_scratch_rejects_on_the_host(lib):
    """fcn_step_scratch refuses, before any device call, a plan whose workspace exceeds the static
    scratch, a NULL field and a negative step count."""
    hdr = open(os.path.join(ROOT, "include", "fcn.h")).read()
    m = re.search(r"#define FCN_SCRATCH_BYTES \((\d+)u << (\d+)\)", hdr)
    assert m and int(m.group(1)) << int(m.group(2)) == fcn.SCRATCH_BYTES
    insts = wl.config_batch(count=300)
    rc, h = _create(lib, insts, precision=1)
    assert rc == fcn.FCN_OK
    sz = ctypes.c_size_t()
    assert lib.fcn_plan_workspace_size(h, ctypes.byref(sz)) == 0
    assert sz.value > fcn.SCRATCH_BYTES
    assert lib.fcn_step_scratch(h, ctypes.c_void_p(0x1000), 1, None) == fcn.FCN_E_SIZE
    assert b"static scratch" in lib.fcn_last_error(h)
    assert lib.fcn_plan_destroy(h) == 0
    rc, h = _create(lib, [wl.config_small(nr=16, nt=64)])
    assert rc == fcn.FCN_OK
    assert lib.fcn_step_scratch(h, None, 1, None) == fcn.FCN_E_ARG
    assert lib.fcn_step_scratch(h, ctypes.c_void_p(0x1000), -1, None) == fcn.FCN_E_ARG
    assert lib.fcn_plan_destroy(h) == 0


def test_instance_struct_matches_the_header(tmp_path):
    """The Python mirror of fcn_instance has the C struct's size and field offsets (gcc compiles
    the public header and prints them)."""
    fields = [name for name, _ in fcn.Instance._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"fcn.h\"\nint main(void) {\n"
                   "  printf(\"%zu\\n\", sizeof(fcn_instance));\n" +
                   "".join(f"  printf(\"%zu\\n\", offsetof(fcn_instance, {n}));\n" for n in fields) +
                   "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert got[0] == ctypes.sizeof(fcn.Instance)
    assert got[1:] == [getattr(fcn.Instance, n).offset for n in fields]


def test_cartesian_plan_sizes_on_host(lib):
    """A Cartesian instance: nx * ny * nt field elements ([ny][nx][nt]), a diagnostics record of
    8 + nx * ny doubles, beside a radial instance in the same plan; invalid Cartesian grids are
    refused."""
    cart = wl.config_cartesian(nx=31, ny=17, nt=64)
    rad = wl.config_small(nr=40, nt=128)
    rc, h = _create(lib, [rad, cart], precision=fcn.FCN_FP32_CN64)
    assert rc == fcn.FCN_OK
    sz = ctypes.c_size_t()
    assert lib.fcn_field_size(h, ctypes.byref(sz)) == 0 and sz.value == 40 * 128 + 31 * 17 * 64
    assert lib.fcn_field_offset(h, 1, ctypes.byref(sz)) == 0 and sz.value == 40 * 128
    assert lib.fcn_diag_record_size(h, ctypes.byref(sz)) == 0 and sz.value == (8 + 40) + (8 + 31 * 17)
    lib.fcn_plan_destroy(h)
    for key, value, code in (("ny", 2, fcn.FCN_E_ARG), ("ny", 4097, fcn.FCN_E_SIZE), ("nx", 2, fcn.FCN_E_ARG),
                             ("y_max", 0.0, fcn.FCN_E_ARG), ("x_max", -1.0, fcn.FCN_E_ARG)):
        bad = dict(cart, **{key: value})
        rc, h = _create(lib, [bad])
        assert rc == code and not h.value, (key, value)
    big = wl.config_cartesian(nx=4096, ny=1025, nt=64)  # more than 2^22 transverse points
    assert _create(lib, [big])[0] == fcn.FCN_E_SIZE
    inst = fcn.make_instance(cart)
    inst.geometry = 2
    arr = (fcn.Instance * 1)(inst)
    o = fcn.Options(precision=0, max_phase=0.05, dz_min=1e-6, dz_max=1e-2)
    assert lib.fcn_plan_create(arr, 1, ctypes.byref(o), ctypes.byref(ctypes.c_void_p())) == fcn.FCN_E_ARG

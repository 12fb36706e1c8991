"""The C-ABI library loads, exports every entry point of include/mdd.h, and
validates arguments on the host before any HIP call (runs without a GPU)."""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

from paper_2202_04486_amd import native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mdd.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:mdd|mdc)_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(native.LIB_PATH):
        pytest.fail("libmdd.so is not built (run `python -m paper_2202_04486_amd.build`)")
    return native.load()


def test_every_declared_symbol_is_exported(lib):
    names = header_functions()
    assert len(names) >= 15
    assert set(names) == set(native.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_header_is_plain_c():
    res = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-x", "c", HEADER],
                         capture_output=True, text=True)
    assert res.returncode == 0, res.stderr


def dims(**kw):
    base = dict(ns=32, nr=24, nvs=20, nt=128, nf=65, nb_max=8, precision="fp32", flags=0)
    base.update(kw)
    return native.make_dims(**base)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16x3", "bf16", "fp32_cgemm"])
def test_every_precision_accepted(lib, prec):
    """Every precision setting plans on the same workspace as float32."""
    assert native.workspace_bytes(dims(precision=prec)) == native.workspace_bytes(dims())


def test_workspace_bytes_valid_and_monotone(lib):
    a = native.workspace_bytes(dims())
    b = native.workspace_bytes(dims(nvs=40))
    assert a > 0 and b > a and a % 256 == 0


def test_full_gradient_flag_reserves_a_second_spectra_buffer(lib):
    a = native.workspace_bytes(dims())
    b = native.workspace_bytes(dims(flags=native.FLAG_FULL_GRAD))
    spectra = 24 * 2 * 65 * 16 * 8          # nr x blocks of 16 columns x nf x 16 complex64
    assert b - a >= spectra and (b - a) % 256 == 0


def test_streamed_kernel_flag_keeps_only_the_batch_rows(lib):
    """MDD_FLAG_STREAM_KERNEL: the kernel spectra shrink from ns to nb_max rows."""
    a = native.workspace_bytes(dims(ns=200, nb_max=8))
    b = native.workspace_bytes(dims(ns=200, nb_max=8, flags=native.FLAG_STREAM_KERNEL))
    nrp = 32                                 # 24 receivers padded to 16
    assert a - b >= (200 - 8) * nrp * 65 * 8 - 256
    assert b > 0


def test_streamed_data_workspace_does_not_grow_with_ns(lib):
    """MDD_FLAG_STREAM_KERNEL | MDD_FLAG_STREAM_DATA: only the batch's kernel and data rows
    are kept, so the workspace is the same for 200 sources and for a million; ns above
    4096 needs a streamed kernel."""
    f = native.FLAG_STREAM_KERNEL | native.FLAG_STREAM_DATA
    a = native.workspace_bytes(dims(ns=200, nb_max=8, flags=f))
    b = native.workspace_bytes(dims(ns=1 << 20, nb_max=8, flags=f))
    assert a == b > 0
    c = native.workspace_bytes(dims(ns=8192, nb_max=8, flags=native.FLAG_STREAM_KERNEL))
    assert c > a                                   # the data spectra of every source
    assert native.workspace_bytes(dims(ns=8192, nb_max=8)) == 0
    assert native.workspace_bytes(dims(ns=(1 << 20) + 1, nb_max=8, flags=f)) == 0
    assert native.workspace_bytes(dims(nr=5000, flags=f)) == 0


@pytest.mark.parametrize("kw", [dict(nf=66), dict(nt=100), dict(nt=2048), dict(nb_max=33),
                                dict(ns=100, nb_max=65), dict(ns=0), dict(nr=-1), dict(nf=0),
                                dict(precision=5), dict(precision=-1), dict(flags=8), dict(flags=6),
                                dict(flags=16), dict(flags=14), dict(nvs=5000), dict(ns=5000)])
def test_invalid_dims_rejected(lib, kw):
    assert native.workspace_bytes(dims(**kw)) == 0
    out = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(1 << 12)
    st = lib.mdd_plan_create(ctypes.byref(dims(**kw)), ctypes.addressof(buf), 1 << 12, None,
                             ctypes.byref(out))
    assert st in (native.MDD_ESHAPE, native.MDD_EINVAL, native.MDD_EUNSUPPORTED)
    assert not out.value


def test_plan_create_workspace_checks(lib):
    d = dims()
    need = native.workspace_bytes(d)
    out = ctypes.c_void_p()
    assert lib.mdd_plan_create(ctypes.byref(d), None, need, None, ctypes.byref(out)) == native.MDD_ENOMEM
    assert lib.mdd_plan_create(ctypes.byref(d), ctypes.c_void_p(4096), need - 1, None,
                               ctypes.byref(out)) == native.MDD_ENOMEM
    assert lib.mdd_plan_create(ctypes.byref(d), ctypes.c_void_p(4096 + 8), need, None,
                               ctypes.byref(out)) == native.MDD_ENOMEM
    assert lib.mdd_plan_create(ctypes.byref(d), ctypes.c_void_p(4096), need, None, None) == native.MDD_EINVAL
    assert lib.mdd_plan_create(None, ctypes.c_void_p(4096), need, None, ctypes.byref(out)) == native.MDD_EINVAL


def test_null_plan_rejected_everywhere(lib):
    p = ctypes.c_void_p(8)
    opt = native.Opt(1, 0, 1e-2, 0.9, 0.999, 1e-8, 0.9, 1)
    E = native.MDD_EINVAL
    assert lib.mdd_plan_destroy(None) == E
    assert lib.mdd_plan_set_stream(None, None) == E
    assert lib.mdd_set_kernel(None, p) == E
    assert lib.mdd_stage_kernel(None, p, 1) == E
    assert lib.mdd_set_data(None, p) == E
    assert lib.mdd_stage_data(None, p, 1) == E
    assert lib.mdd_set_mask(None, p) == E
    assert lib.mdc_forward(None, p, p, 1, p) == E
    assert lib.mdc_adjoint(None, p, p, 1, p) == E
    assert lib.mdd_stoch_grad(None, p, p, 1, p, p, p) == E
    assert lib.mdd_step(None, p, p, p, ctypes.byref(opt), p, 1, p, p) == E
    assert lib.mdd_full_grad(None, p, p, p, p) == E
    assert lib.mdd_full_step(None, p, p, p, ctypes.byref(opt), p, p) == E
    assert lib.mdd_invalidate_model_spectra(None) == E
    assert lib.mdd_sigma_max2(None, 10, p) == E
    assert lib.mdd_profile_enable(None, 1, 10) == E
    assert lib.mdd_plan_last_hip_error(None) == 0


def test_status_strings(lib):
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        s = native.status_string(code)
        assert isinstance(s, str) and s
    assert native.status_string(-99) == "unknown status"


def test_plan_refuses_cpu_device():
    from paper_2202_04486_amd.plan import Plan
    with pytest.raises(ValueError):
        Plan(8, 8, 8, 128, 65, 4, device="cpu")


def test_check_batch_host(lib):
    """The host-side batch check: sizes against nb_max, indices against [0, ns)."""
    def check(idx, ns=10, nb_max=4):
        arr = (ctypes.c_int32 * max(1, len(idx)))(*idx)
        return lib.mdd_check_batch_host(arr, len(idx), ns, nb_max)
    assert check([0, 3, 9]) == native.MDD_OK
    assert check([2, 2]) == native.MDD_OK                    # repeats are allowed
    assert check([0, 10]) == native.MDD_EINVAL
    assert check([-1]) == native.MDD_EINVAL
    assert check([]) == native.MDD_ESHAPE
    assert check([0, 1, 2, 3, 4]) == native.MDD_ESHAPE
    assert lib.mdd_check_batch_host(None, 1, 10, 4) == native.MDD_EINVAL


def test_reciprocity_rejects_bad_arguments_on_the_host(lib):
    p = ctypes.c_void_p(4096)
    assert lib.mdd_reciprocity(None, p, 4, 128, None) == native.MDD_EINVAL
    assert lib.mdd_reciprocity(ctypes.c_void_p(4100), p, 4, 128, None) == native.MDD_EINVAL
    assert lib.mdd_reciprocity(p, p, 0, 128, None) == native.MDD_ESHAPE
    assert lib.mdd_reciprocity(p, p, 4, 100, None) == native.MDD_ESHAPE


def test_calibration_rejects_bad_arguments_on_the_host(lib):
    p = ctypes.c_void_p(4096)
    E, S = native.MDD_EINVAL, native.MDD_ESHAPE
    assert lib.mdd_calibrate_update(None, p, p, p, 4, 20, 512, 200, 0, None) == E
    assert lib.mdd_calibrate_update(p, p, p, ctypes.c_void_p(4104), 4, 20, 512, 200, 0, None) == E
    assert lib.mdd_calibrate_update(p, p, p, p, 4, 20, 512, 200, 4, None) == E
    assert lib.mdd_calibrate_update(p, p, p, p, 4, 20, 512, 200, -1, None) == E
    assert lib.mdd_calibrate_update(p, p, p, p, 0, 20, 512, 200, 0, None) == S
    assert lib.mdd_calibrate_update(p, p, p, p, 4, 5000, 512, 200, 0, None) == S
    assert lib.mdd_calibrate_update(p, p, p, p, 4, 20, 500, 200, 0, None) == S
    assert lib.mdd_calibrate_update(p, p, p, p, 4, 20, 512, 258, 0, None) == S


def test_row_calibration_rejects_bad_arguments_on_the_host(lib):
    """mdd_calibrate_rows (the kernel-row stream of the one-virtual-source products)
    checks pointers, alignment and every extent before any HIP call."""
    p = ctypes.c_void_p(4096)
    E, S = native.MDD_EINVAL, native.MDD_ESHAPE
    assert lib.mdd_calibrate_rows(None, p, p, 64, 200, 1600, 1600, 0, None) == E
    assert lib.mdd_calibrate_rows(p, None, p, 64, 200, 1600, 1600, 0, None) == E
    assert lib.mdd_calibrate_rows(p, p, None, 64, 200, 1600, 1600, 0, None) == E
    assert lib.mdd_calibrate_rows(ctypes.c_void_p(4104), p, p, 64, 200, 1600, 1600, 0, None) == E
    assert lib.mdd_calibrate_rows(p, p, ctypes.c_void_p(4100), 64, 200, 1600, 1600, 0, None) == E
    assert lib.mdd_calibrate_rows(p, p, p, 0, 200, 1600, 1600, 0, None) == S
    assert lib.mdd_calibrate_rows(p, p, p, 65, 200, 1600, 1600, 0, None) == S
    assert lib.mdd_calibrate_rows(p, p, p, 64, 0, 1600, 1600, 0, None) == S
    assert lib.mdd_calibrate_rows(p, p, p, 64, 200, 0, 1600, 0, None) == S
    assert lib.mdd_calibrate_rows(p, p, p, 64, 200, 1600, 4097, 0, None) == S
    assert lib.mdd_calibrate_rows(p, p, p, 64, 200, 1600, 1600, 65, None) == S
    assert lib.mdd_calibrate_rows(p, p, p, 64, 200, 1600, 1600, -1, None) == S


def test_noalloc_gradient_rejects_on_the_host(lib):
    """mdd_stoch_grad_noalloc checks its arguments and the size of the plan against the
    static workspace before any HIP call."""
    p = ctypes.c_void_p(4096)
    d = dims()
    assert native.workspace_bytes(d) <= native.NOALLOC_WORKSPACE_BYTES
    E = native.MDD_EINVAL
    assert lib.mdd_stoch_grad_noalloc(None, p, p, None, p, p, 4, p, None, None, None) == E
    assert lib.mdd_stoch_grad_noalloc(ctypes.byref(d), None, p, None, p, p, 4, p, None, None, None) == E
    assert lib.mdd_stoch_grad_noalloc(ctypes.byref(d), p, p, None, p, p, 4, None, None, None, None) == E
    assert lib.mdd_stoch_grad_noalloc(ctypes.byref(d), p, p, None, p, p, 9, p, None, None,
                                      None) == native.MDD_ESHAPE
    for flag in (native.FLAG_STREAM_KERNEL, native.FLAG_FULL_GRAD):
        df = dims(flags=flag)
        assert lib.mdd_stoch_grad_noalloc(ctypes.byref(df), p, p, None, p, p, 4, p, None, None,
                                          None) == E
    big = dims(ns=1024, nr=1024, nvs=64, nt=512, nf=200, nb_max=8)
    assert native.workspace_bytes(big) > native.NOALLOC_WORKSPACE_BYTES
    assert lib.mdd_stoch_grad_noalloc(ctypes.byref(big), p, p, None, p, p, 4, p, None, None,
                                      None) == native.MDD_ELIMIT
    assert "static workspace" in native.status_string(native.MDD_ELIMIT)

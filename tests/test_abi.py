"""The C-ABI library loads, exports what include/sdl.h declares, and validates
arguments before touching the device (these calls never reach a HIP call)."""
import ctypes
import subprocess

import pytest

from paper_2007_03800_amd import _native


def test_header_symbols_exported():
    names = _native.header_functions()
    assert {"sdl_sparse_code", "sdl_tmod_update", "sdl_learn", "sdl_last_error", "sdl_default_options",
            "sdl_abi_version"} <= set(names)
    out = subprocess.run(["nm", "-D", "--defined-only", _native.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    lib = _native.lib()
    for n in names:
        assert hasattr(lib, n)
    assert lib.sdl_abi_version() == 9


def _problem(**kw):
    base = dict(m1=8, m2=8, n1=16, n2=16, s=8, reserved=0, N=10, Y=1, D1=2, D2=3, supp=4, coef=5, res2=6)
    base.update(kw)
    return _native.Problem(**base)


def _call(fn, prob, opts=None, extra=()):
    arr = (_native.Problem * 1)(prob)
    o = opts if opts is not None else _native.default_options()
    if fn == "sparse_code":
        return _native.lib().sdl_sparse_code(arr, 1, ctypes.byref(o), None)
    if fn == "tmod_update":
        return _native.lib().sdl_tmod_update(arr, 1, extra[0] if extra else 3, ctypes.byref(o), None)
    return _native.lib().sdl_learn(arr, 1, extra[0] if extra else 2, None, ctypes.byref(o), None)


@pytest.mark.parametrize("fn", ["sparse_code", "tmod_update", "learn"])
@pytest.mark.parametrize("kw,status", [
    (dict(s=257), -2),           # s > n1*n2
    (dict(m1=2, m2=2, s=5), -2),  # s > m1*m2
    (dict(m1=0), -2),
    (dict(n2=-3), -2),
    (dict(s=0), -2),
    (dict(N=-1), -1),
    (dict(D1=None), -1),
    (dict(Y=None), -1),
    (dict(supp=None), -1),
    (dict(coef=None), -1),
    (dict(reserved=7), -1),
    (dict(m1=65, n1=65), -2),
    (dict(s=33, n1=16), -2),
])
def test_validation(fn, kw, status):
    st = _call(fn, _problem(**kw))
    assert st == status
    assert _native.lib().sdl_last_error().decode() != ""


def test_bad_enums():
    o = _native.default_options()
    o.prec = 5
    assert _call("sparse_code", _problem(), o) == -1
    o = _native.default_options()
    o.schedule = 3
    assert _call("learn", _problem(), o) == -1
    o = _native.default_options()
    o.kernel = 9
    assert _call("sparse_code", _problem(), o) == -1
    assert _call("tmod_update", _problem(), None, (0,)) == -1
    assert _call("tmod_update", _problem(), None, (4,)) == -1
    assert _call("learn", _problem(), None, (-1,)) == -1
    assert _native.lib().sdl_sparse_code(None, 1, None, None) == -1
    assert _native.lib().sdl_sparse_code(None, -1, None, None) == -1


def test_default_options():
    o = _native.default_options()
    assert o.prec == 0 and o.use_graph == 1 and o.schedule == 0
    assert o.stop_rel < 0 and o.dep_eps < 0 and o.pivot_fp64 < 0
    assert o.err2 == 0.0
    assert o.tie_band == 2.0 ** -6 and o.fallback_margin == 1.01 and o.deterministic == 1
    assert o.reserved0 == 0 and not o.workspace and o.workspace_bytes == 0


@pytest.mark.parametrize("field,value", [("tie_band", -0.1), ("tie_band", 0.5), ("tie_band", float("nan")),
                                         ("fallback_margin", 0.99), ("fallback_margin", float("nan")),
                                         ("deterministic", 2), ("reserved0", 1)])
@pytest.mark.parametrize("fn", ["sparse_code", "tmod_update", "learn"])
def test_option_validation(fn, field, value):
    o = _native.default_options()
    setattr(o, field, value)
    assert _call(fn, _problem(), o) == -1


def test_workspace_validation():
    """A caller workspace that is misaligned or too small is refused before any device work;
    its required size comes from a host-only query."""
    lib = _native.lib()
    arr = (_native.Problem * 1)(_problem(N=100000))
    o = _native.default_options()
    o.prec = _native.SDL_FP32
    need = ctypes.c_size_t()
    for call, K in ((0, 0), (1, 0), (2, 20), (3, 0)):
        assert lib.sdl_workspace_bytes(arr, 1, call, K, ctypes.byref(o), ctypes.byref(need)) == 0
        assert need.value > 0
    assert lib.sdl_workspace_bytes(arr, 1, 4, 0, ctypes.byref(o), ctypes.byref(need)) == -1
    lib.sdl_workspace_bytes(arr, 1, 0, 0, ctypes.byref(o), ctypes.byref(need))
    o.workspace, o.workspace_bytes = 256, need.value - 1
    assert lib.sdl_sparse_code(arr, 1, ctypes.byref(o), None) == -4
    o.workspace, o.workspace_bytes = 257, need.value
    assert lib.sdl_sparse_code(arr, 1, ctypes.byref(o), None) == -1
    o.workspace, o.workspace_bytes = 256, 0
    assert lib.sdl_sparse_code(arr, 1, ctypes.byref(o), None) == -1


def test_sparse_code_sums_validation():
    lib = _native.lib()
    o = _native.default_options()
    arr = (_native.Problem * 1)(_problem())
    assert lib.sdl_sparse_code_sums(arr, 0, 8, ctypes.byref(o), None) == -1
    assert lib.sdl_sparse_code_sums(arr, 3, 8, ctypes.byref(o), None) == -1
    assert lib.sdl_sparse_code_sums(arr, 1, None, ctypes.byref(o), None) == -1
    arr = (_native.Problem * 1)(_problem(res2=None))
    assert lib.sdl_sparse_code_sums(arr, 1, 8, ctypes.byref(o), None) == -1
    arr = (_native.Problem * 1)(_problem(s=257))
    assert lib.sdl_sparse_code_sums(arr, 1, 8, ctypes.byref(o), None) == -2


def test_mixed_precision_validation():
    """SDL_MIXED_BF16 is refused for shapes without its kernel, and with the error-driven stop."""
    lib = _native.lib()
    o = _native.default_options()
    o.prec = _native.SDL_MIXED_BF16
    assert _call("sparse_code", _problem(m1=5, m2=7, n1=9, n2=11, s=3), o) == -7
    if lib.sdl_mixed_supported(12, 12, 24, 24, 12):
        o.err2 = 1.0
        assert _call("sparse_code", _problem(m1=12, m2=12, n1=24, n2=24, s=12), o) == -7


def test_proposer_file_errors(tmp_path):
    lib = _native.lib()
    h = ctypes.c_void_p()
    assert lib.sdl_proposer_load(str(tmp_path / "missing.bin").encode(), ctypes.byref(h)) == -1
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"NOTAPROP" + bytes(40))
    assert lib.sdl_proposer_load(str(bad).encode(), ctypes.byref(h)) == -1
    assert not h.value
    assert lib.sdl_proposer_save(None, str(bad).encode()) == -1


def test_error_driven_option_validation():
    """err2 < 0 or NaN is invalid; err2 > 0 runs on the one-wave or generic kernels only (kernel 2 is
    refused, and kernel 3 where the shape has no one-wave kernel; checked before device work)."""
    for bad in (-1.0, float("nan")):
        o = _native.default_options()
        o.err2 = bad
        assert _call("sparse_code", _problem(), o) == -1
    for kern in (2, 3):
        o = _native.default_options()
        o.err2 = 1.0
        o.kernel = kern
        assert _call("sparse_code", _problem(), o) == -7


def test_probe_validation():
    lib = _native.lib()
    d = ctypes.c_double()
    assert lib.sdl_probe_hbm_copy(None, None, 1024, 1, ctypes.byref(d), None) == -1
    assert lib.sdl_probe_hbm_copy(1, 2, 8, 1, ctypes.byref(d), None) == -1
    assert lib.sdl_probe_hbm_copy(1, 2, 1024, 0, ctypes.byref(d), None) == -1
    assert lib.sdl_probe_peak(7, 1, 1, ctypes.byref(d), None) == -1
    assert lib.sdl_probe_peak(0, None, 1, ctypes.byref(d), None) == -1
    assert lib.sdl_probe_peak(0, 1, 0, ctypes.byref(d), None) == -1


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built HIP library every call raises: the package has no CPU fallback."""
    monkeypatch.setattr(_native, "LIB_PATH", str(tmp_path / "libsdl.so"))
    monkeypatch.setattr(_native, "_lib", None)
    with pytest.raises(ImportError):
        _native.lib()
    from paper_2007_03800_amd import api
    with pytest.raises(ImportError):
        api.tuned_config(8, 8, 16, 16, 8)


def test_noalloc_refuses_before_device_work():
    """The allocation-free call checks its fixed scratch size and its options on the host."""
    lib = _native.lib()
    o = _native.default_options()
    arr = (_native.Problem * 8)(*[_problem(m1=32, m2=32, n1=64, n2=64, s=4) for _ in range(8)])
    assert lib.sdl_sparse_code_noalloc(arr, 8, ctypes.byref(o), None) == -4
    assert "workspace" in lib.sdl_last_error().decode()
    o.timing = 1
    assert lib.sdl_sparse_code_noalloc(arr, 1, ctypes.byref(o), None) == -1
    o = _native.default_options()
    o.workspace, o.workspace_bytes = 256, 1 << 20
    assert lib.sdl_sparse_code_noalloc(arr, 1, ctypes.byref(o), None) == -1
    assert lib.sdl_sparse_code_noalloc(None, 1, None, None) == -1


def test_orthonormal_method_validation():
    """method 1 (Remark 1) needs square dictionaries within the limits, FP32/FP64, plain schedule."""
    lib = _native.lib()
    o = _native.default_options()
    o.method = 1
    assert _call("sparse_code", _problem(m1=8, m2=8, n1=16, n2=16, s=8), o) == -2  # n != m
    assert _call("sparse_code", _problem(m1=40, m2=4, n1=40, n2=4, s=8), o) == -2  # m1 > 32
    o.method = 2
    assert _call("learn", _problem(), o) == -1
    o = _native.default_options()
    o.method, o.prec = 1, _native.SDL_BF16
    assert _call("learn", _problem(m1=8, m2=8, n1=8, n2=8, s=4), o) == -7
    o = _native.default_options()
    o.method, o.err2 = 1, 1.0
    assert _call("sparse_code", _problem(m1=8, m2=8, n1=8, n2=8, s=4), o) == -7
    o = _native.default_options()
    o.reserved1 = 3
    assert _call("sparse_code", _problem(), o) == -1
    assert lib.sdl_abi_version() == 9



def test_denoise_driver_validation():
    lib = _native.lib()
    o = _native.default_options()
    o.prec = 1  # SDL_FP32
    # patch extraction: element type, patch larger than the image, NULL pointers
    assert lib.sdl_image_to_patches(ctypes.c_void_p(1), 16, 16, 8, 8, 2, ctypes.c_void_p(2), None) == -1
    assert lib.sdl_image_to_patches(ctypes.c_void_p(1), 7, 16, 8, 8, 1, ctypes.c_void_p(2), None) == -2
    assert lib.sdl_image_to_patches(ctypes.c_void_p(1), 16, 16, 0, 8, 1, ctypes.c_void_p(2), None) == -2
    assert lib.sdl_image_to_patches(None, 16, 16, 8, 8, 1, ctypes.c_void_p(2), None) == -1
    # reconstruction: N must be the number of overlapping patches of an H x W image
    arr = (_native.Problem * 1)(_problem(N=81, Y=None))
    assert lib.sdl_patches_to_image(arr, 16, 16, ctypes.byref(o), None, None) == -1
    assert lib.sdl_patches_to_image(arr, 16, 17, ctypes.byref(o), ctypes.c_void_p(7), None) == -2
    assert lib.sdl_patches_to_image(arr, 7, 16, ctypes.byref(o), ctypes.c_void_p(7), None) == -2
    o.prec = 2  # SDL_BF16 codes are FP32; the image is FP32 or FP64
    assert lib.sdl_patches_to_image(arr, 16, 16, ctypes.byref(o), ctypes.c_void_p(7), None) == -1


def _tensor(**kw):
    t = _native.TensorProblem()
    t.nmodes, t.s, t.N = kw.get("nmodes", 3), kw.get("s", 4), kw.get("N", 10)
    ms, ns = kw.get("m", (4, 3, 5)), kw.get("n", (6, 5, 7))
    for d in range(len(ms)):
        t.m[d], t.n[d] = ms[d], ns[d]
        t.D[d] = 8 + d
    t.Y, t.supp, t.coef, t.res2 = kw.get("Y", 1), 2, 3, 4
    return t


@pytest.mark.parametrize("kw,status", [
    (dict(nmodes=1), -2), (dict(nmodes=5), -2), (dict(m=(0, 3, 5)), -2), (dict(n=(6, 65, 7)), -2),
    (dict(m=(64, 64, 2), n=(2, 2, 2)), -2),    # prod m > 4096
    (dict(s=0), -2), (dict(s=33), -2), (dict(s=30, m=(2, 2, 2)), -2), (dict(N=-1), -1), (dict(Y=None), -1),
])
def test_tensor_validation(kw, status):
    lib = _native.lib()
    o = _native.default_options()
    t = _tensor(**kw)
    assert lib.sdl_tensor_sparse_code(ctypes.byref(t), ctypes.byref(o), None) == status
    assert lib.sdl_tensor_learn(ctypes.byref(t), 2, None, ctypes.byref(o), None) == status


def test_tensor_option_refusals():
    lib = _native.lib()
    t = _tensor()
    for field, value in [("prec", 2), ("prec", 3), ("kernel", 2), ("method", 1), ("schedule", 1)]:
        o = _native.default_options()
        setattr(o, field, value)
        assert lib.sdl_tensor_sparse_code(ctypes.byref(t), ctypes.byref(o), None) == -7, field
    o = _native.default_options()
    assert lib.sdl_tensor_update(ctypes.byref(t), 0, ctypes.byref(o), None) == -1
    assert lib.sdl_tensor_update(ctypes.byref(t), 4, ctypes.byref(o), None) == -1
    assert lib.sdl_tensor_learn(ctypes.byref(t), -1, None, ctypes.byref(o), None) == -1
    t.res2 = None
    assert lib.sdl_tensor_learn(ctypes.byref(t), 2, None, ctypes.byref(o), None) == -1
    t.D[1] = None
    assert lib.sdl_tensor_sparse_code(ctypes.byref(t), ctypes.byref(o), None) == -1

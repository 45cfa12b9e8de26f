"""The C ABI library loads on the CPU and exports every function include/cgks.h declares."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "cgks.h")) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cgks_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_binding_set():
    from paper_2402_02075_amd import cgks
    assert set(_declared()) == set(cgks.EXPORTS)


def test_library_exports_every_declared_symbol():
    path = os.path.join(ROOT, "paper_2402_02075_amd", "libcgks.so")
    assert os.path.exists(path), "libcgks.so not built"
    lib = ctypes.CDLL(path)
    missing = [s for s in _declared() if not hasattr(lib, s)]
    assert not missing, missing


def test_default_params_without_gpu():
    from paper_2402_02075_amd import cgks
    p = cgks.default_params()
    assert p.gamma == 1.4 and p.levels == 3 and p.passes == 3 and p.seed == 1
    assert p.nu_pre[0] == 1 and p.nu_post[0] == 0
    assert abs(p.skew_sin - 0.17364817766693033) < 1e-15
    assert p.cell_order == 1 and p.mixed_stall == 300 and p.adjoint_tape == 0


def test_params_struct_size_matches_the_header():
    """cgks_default_params writes exactly the binding's copy of cgks_params: a buffer with guard
    bytes past the binding's size keeps them (a field added on one side only would overrun)."""
    from paper_2402_02075_amd import cgks
    n = ctypes.sizeof(cgks.Params)
    buf = (ctypes.c_uint8 * (n + 64))(*([0xA5] * (n + 64)))
    cgks.lib().cgks_default_params(ctypes.cast(buf, ctypes.c_void_p))
    assert bytes(buf[n:]) == bytes([0xA5] * 64)
    assert any(b != 0xA5 for b in buf[n - 8:n])  # the last field was written


def test_invalid_params_rejected_before_any_device_work():
    """cgks_create checks the parameters before it touches the device: each out-of-range field
    returns CGKS_E_ARG and no context (so this runs without a GPU), and the defaults pass the
    check (their create then fails only for the missing device, or succeeds on a GPU machine)."""
    from paper_2402_02075_amd import cgks
    bad = [("gamma", 1.0), ("gamma", 1.7), ("cfl", 0.0), ("prandtl", 0.0), ("gamma_lin", 1.0),
           ("levels", 0), ("levels", 9), ("passes", 17), ("precision", 2), ("coarse_smoother", 2),
           ("relax_sweeps", 65), ("cycle_gamma", 4), ("cell_order", 3), ("mixed_stall", 0),
           ("adjoint_tape", 2)]
    for field, value in bad:
        p = cgks.default_params()
        setattr(p, field, value)
        h = ctypes.c_void_p()
        code = cgks.lib().cgks_create(ctypes.byref(p), ctypes.byref(h))
        assert code == cgks.E_ARG and not h.value, (field, value, code)
    p = cgks.default_params()
    p.viscous, p.mu = 1, 0.0  # viscous flow needs a viscosity
    h = ctypes.c_void_p()
    assert cgks.lib().cgks_create(ctypes.byref(p), ctypes.byref(h)) == cgks.E_ARG and not h.value
    p = cgks.default_params()
    code = cgks.lib().cgks_create(ctypes.byref(p), ctypes.byref(h))
    assert code in (cgks.OK, cgks.E_DEVICE), code
    if code == cgks.OK:
        cgks.lib().cgks_destroy(h)

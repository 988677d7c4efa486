"""C ABI checks that need no GPU: the library loads, exports every function
include/rmatrix.h declares, and rejects invalid arguments before touching
the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1403_5524_amd import native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "rmatrix.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(rm_\w+)\(",
                                 txt, re.M)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(native.LIB_PATH):
        pytest.fail("librmatrix.so is not built (run __graft_entry__.build())")
    return native.lib()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert "rm_sweep_energies" in names and len(names) >= 9
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(native.EXPORTED)


def _desc(n=2, nh=3, **kw):
    E = np.array(kw.pop("E", [0.5, 1.5, 4.0][:nh]), dtype=np.float64)
    w = np.array(kw.pop("w", np.ones(n * nh)), dtype=np.float64)
    e = np.array(kw.pop("e", [0.0, 0.3][:n]), dtype=np.float64)
    l = np.array(kw.pop("l", [0, 1][:n]), dtype=np.int32)
    keep = (E, w, e, l)
    d = native.PolesDesc(kw.pop("n_chan", n), kw.pop("n_poles", nh),
                         E.ctypes.data, w.ctypes.data, kw.pop("a", 20.0),
                         e.ctypes.data, l.ctypes.data, None,
                         kw.pop("z", 1.0), kw.pop("g", 1.0))
    return d, keep


@pytest.mark.parametrize("bad", [
    {"n_chan": 0}, {"n_poles": 0}, {"a": 0.0}, {"a": -1.0}, {"z": -1.0},
    {"g": 0.0}, {"E": [0.5, 0.5, 4.0]}, {"E": [0.5, float("nan"), 4.0]},
    {"w": [1, 1, float("inf"), 1, 1, 1]}, {"l": [0, 13]}, {"l": [-1, 0]},
    {"e": [0.0, float("nan")]},
])
def test_load_rejects_invalid(L, bad):
    d, keep = _desc(**bad)
    h = ctypes.c_void_p()
    rc = L.rm_load_poles(ctypes.byref(d), ctypes.byref(h), None)
    assert rc == native.RM_ERR_ARG
    assert h.value is None
    assert len(L.rm_last_error()) > 0


def test_sweep_rejects_invalid(L):
    o = native.make_opts()
    assert L.rm_sweep_energies(None, 0, 1, None, 0, ctypes.byref(o), None,
                               None, None) == native.RM_ERR_ARG
    arr = (ctypes.c_void_p * 1)(None)
    assert L.rm_sweep_energies(arr, 1, 1, None, 0, ctypes.byref(o), None,
                               None, None) == native.RM_ERR_ARG
    bad = native.make_opts(prec=9)
    assert L.rm_sweep_energies(arr, 1, 1, None, 0, ctypes.byref(bad), None,
                               None, None) == native.RM_ERR_ARG
    assert b"precision" in L.rm_last_error()
    neg = native.make_opts(near_delta=-1.0)
    assert L.rm_sweep_energies(arr, 1, 1, None, 0, ctypes.byref(neg), None,
                               None, None) == native.RM_ERR_ARG
    both = native.make_opts(flags=native.RM_FLAG_NO_PAIR_PRODUCTS
                            | native.RM_FLAG_PAIR_PRODUCTS)
    assert L.rm_sweep_energies(arr, 1, 1, None, 0, ctypes.byref(both), None,
                               None, None) == native.RM_ERR_ARG
    unknown = native.make_opts(flags=0x10)
    assert L.rm_sweep_energies(arr, 1, 1, None, 0, ctypes.byref(unknown), None,
                               None, None) == native.RM_ERR_ARG
    assert b"flags" in L.rm_last_error()
    damp = native.make_opts(flags=native.RM_FLAG_RADIATION_DAMPING)
    assert L.rm_sweep_energies(arr, 1, 1, None, 0, ctypes.byref(damp), None,
                               None, None) == native.RM_ERR_ARG
    assert b"rm_photoionization only" in L.rm_last_error()
    band = native.make_opts(prec=1, near_delta=1e-2, band_delta=1e-3)
    assert L.rm_sweep_energies(arr, 1, 1, None, 0, ctypes.byref(band), None,
                               None, None) == native.RM_ERR_ARG
    assert b"band_delta" in L.rm_last_error()
    s32 = native.make_opts(solve_fp32=2)
    assert L.rm_sweep_energies(arr, 1, 1, None, 0, ctypes.byref(s32), None,
                               None, None) == native.RM_ERR_ARG


def test_null_handles_rejected(L):
    o = native.make_opts()
    assert L.rm_kmatrix(None, None, 0, ctypes.byref(o), None, None, None,
                        None, None) == native.RM_ERR_ARG
    assert L.rm_rmatrix(None, None, 0, ctypes.byref(o), None, None) == \
        native.RM_ERR_ARG
    assert L.rm_channel_functions(None, None, 0, None, None, None) == \
        native.RM_ERR_ARG
    assert L.rm_collision_strengths(None, None, None, None, 0, 1, None,
                                    None) == native.RM_ERR_ARG
    assert L.rm_free(None) == native.RM_OK


def test_postproc_rejects_invalid(L):
    f64 = ctypes.c_double
    dummy = ctypes.c_void_p(64)   # never dereferenced: rejected first
    other = ctypes.c_void_p(128)
    conv = L.rm_convolve_gaussian
    assert conv(dummy, 5, dummy, 0, f64(0.1), other, None) == native.RM_ERR_ARG
    assert conv(dummy, -1, dummy, 3, f64(0.1), other, None) == native.RM_ERR_ARG
    for bad in (0.0, -0.1, float("nan"), float("inf")):
        assert conv(dummy, 5, dummy, 3, f64(bad), other, None) == \
            native.RM_ERR_ARG
    assert b"fwhm" in L.rm_last_error()
    assert conv(None, 5, dummy, 3, f64(0.1), other, None) == native.RM_ERR_ARG
    assert conv(dummy, 5, dummy, 3, f64(0.1), dummy, None) == \
        native.RM_ERR_ARG
    assert b"in place" in L.rm_last_error()
    assert conv(None, 0, None, 3, f64(0.1), None, None) == native.RM_OK

    lev = np.array([0.0, 0.3], dtype=np.float64)
    ups = L.rm_effective_collision_strengths
    for kT in ([0.0], [-1.0], [float("nan")]):
        t = np.array(kT, dtype=np.float64)
        assert ups(dummy, 5, dummy, 2, lev.ctypes.data, t.ctypes.data, 1,
                   other, None) == native.RM_ERR_ARG
    t = np.array([0.5], dtype=np.float64)
    nan_lev = np.array([0.0, float("nan")], dtype=np.float64)
    assert ups(dummy, 5, dummy, 2, nan_lev.ctypes.data, t.ctypes.data, 1,
               other, None) == native.RM_ERR_ARG
    assert ups(dummy, 5, dummy, 0, lev.ctypes.data, t.ctypes.data, 1,
               other, None) == native.RM_ERR_ARG
    assert ups(None, 5, None, 2, lev.ctypes.data, t.ctypes.data, 1,
               other, None) == native.RM_ERR_ARG

    grp = L.rm_group_collision_strengths
    g = np.array([0, 2], dtype=np.int32)
    assert grp(dummy, 5, 2, g.ctypes.data, 2, other, None) == \
        native.RM_ERR_ARG
    assert b"group" in L.rm_last_error()
    g = np.array([0, -1], dtype=np.int32)
    assert grp(dummy, 5, 2, g.ctypes.data, 2, other, None) == \
        native.RM_ERR_ARG
    g = np.array([0, 1], dtype=np.int32)
    assert grp(dummy, 5, 2, g.ctypes.data, 0, other, None) == \
        native.RM_ERR_ARG
    assert grp(None, 5, 2, g.ctypes.data, 2, None, None) == native.RM_ERR_ARG
    assert grp(None, 0, 2, g.ctypes.data, 2, None, None) == native.RM_OK


def test_photo_rejects_invalid(L):
    o = native.make_opts()
    f64 = ctypes.c_double
    dummy = ctypes.c_void_p(64)
    assert L.rm_photoionization(None, 0, dummy, 4, f64(-1.0), ctypes.byref(o),
                                dummy, None, None) == native.RM_ERR_ARG
    arr = (ctypes.c_void_p * 1)(None)
    assert L.rm_photoionization(arr, 1, dummy, 4, f64(-1.0), ctypes.byref(o),
                                dummy, None, None) == native.RM_ERR_ARG
    assert L.rm_photoionization(arr, 1, dummy, -1, f64(-1.0),
                                ctypes.byref(o), dummy, None,
                                None) == native.RM_ERR_ARG
    assert L.rm_photoionization(arr, 1, dummy, 4, f64(float("nan")),
                                ctypes.byref(o), dummy, None,
                                None) == native.RM_ERR_ARG
    assert b"e0" in L.rm_last_error()
    assert L.rm_load_dipoles(None, dummy, None) == native.RM_ERR_ARG
    assert L.rm_load_widths(None, dummy, None) == native.RM_ERR_ARG
    # damping needs the FP64 pole sum and solve
    for bad in (native.make_opts(prec=1,
                                 flags=native.RM_FLAG_RADIATION_DAMPING),
                native.make_opts(solve_fp32=1,
                                 flags=native.RM_FLAG_RADIATION_DAMPING)):
        assert L.rm_photoionization(arr, 1, dummy, 4, f64(-1.0),
                                    ctypes.byref(bad), dummy, None,
                                    None) == native.RM_ERR_ARG
        assert b"damped" in L.rm_last_error()


def test_propagation_rejects_invalid(L):
    assert L.rm_set_propagation(None, ctypes.c_double(30.0), 10, 1, None,
                                None) == native.RM_ERR_ARG


def test_gailitis_rejects_invalid(L):
    assert L.rm_set_gailitis(None, 20, None) == native.RM_ERR_ARG
    assert L.rm_set_gailitis(None, -1, None) == native.RM_ERR_ARG


class _Poison:
    """A library stand-in that fails the test if any entry point is called:
    the binding must reject bad tensors before it reaches the C ABI."""

    def __getattr__(self, name):
        raise AssertionError("library entry point %s reached" % name)


def _bad_tensors():
    import torch
    good = torch.zeros(6, dtype=torch.float64)
    return [
        ("float32", good.float()),
        ("int32", good.to(torch.int32)),
        ("strided", torch.zeros(12, dtype=torch.float64)[::2]),
        ("host", good),  # right dtype and size, but host memory
    ]


@pytest.mark.parametrize("kind", ["float32", "int32", "strided", "host"])
def test_binding_rejects_bad_tensors_before_any_call(monkeypatch, kind):
    """Every tensor the binding passes to the C ABI is checked for dtype,
    contiguity, size and device first: a float32 or strided E would be read
    as the wrong doubles, a host pointer handed to a kernel is a GPU page
    fault.  Each rejection is an RmError(RM_ERR_ARG) raised before the
    library is touched."""
    import torch
    bad = dict(_bad_tensors())[kind]
    monkeypatch.setattr(native, "_lib", _Poison())
    sym = native.Symmetry(None, 2, 3, 2)
    calls = [
        lambda: native.rm_sweep_energies([sym], 2, bad),
        lambda: native.rm_kmatrix(sym, bad),
        lambda: native.rm_rmatrix(sym, bad),
        lambda: native.rm_channel_functions(sym, bad),
        lambda: native.rm_photoionization([sym], bad, -0.5),
        lambda: native.Plan([sym], 2, bad),
    ]
    for call in calls:
        with pytest.raises(native.RmError) as ei:
            call()
        assert ei.value.code == native.RM_ERR_ARG
    # caller-supplied outputs are checked too
    E_ok_shape = torch.zeros(6, dtype=torch.float64)
    with pytest.raises(native.RmError):
        native.rm_collision_strengths(sym, bad, bad, E_ok_shape, 2, bad)
    with pytest.raises(native.RmError):
        native.rm_convolve_gaussian(E_ok_shape, bad.reshape(2, 3)
                                    if bad.is_contiguous() else bad[:6].reshape(2, 3), 0.1)
    sym.handle = None


def test_binding_rejects_wrong_sizes():
    """Size is checked before the device: an output with the wrong element
    count is refused whatever memory it is in."""
    import torch
    with pytest.raises(native.RmError) as ei:
        native._f64(torch.zeros((4, 2), dtype=torch.float64), 12, "omega")
    assert "omega must hold 12" in str(ei.value)
    with pytest.raises(native.RmError) as ei:
        native._i32(torch.zeros(3, dtype=torch.int32), 4, "status")
    assert "status must hold 4" in str(ei.value)
    assert native._f64(None, 4, "R", optional=True) is None

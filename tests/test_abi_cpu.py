"""CPU-only checks of the C ABI: the library loads, exports every function
the header declares, and rejects bad arguments on the host (no GPU needed:
these error paths return before any HIP call)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2503_18479_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("cosim.h", "cosim_sparam.h")]

EINVAL, EUNSUPPORTED = -1, -4


def _declared():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(cosim_[a-z_0-9A-Z]+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    return _lib.load_library()


def test_library_under_test(lib):
    """Under tests/test_abi_asan.py this module runs against the ASan build
    with the ASan runtime preloaded: check that both are mapped."""
    if os.environ.get("COSIM_EXPECT_ASAN") != "1":
        return
    maps = open("/proc/self/maps").read()
    assert "libcosim_asan.so" in maps and "libclang_rt.asan" in maps


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.SIGNATURES), "binding and header disagree"
    assert lib.cosim_version() == 1


def _geom_args(n=2, nv=4):
    seg = np.arange(0, n * nv + 1, nv, dtype=np.int32)
    ang = np.linspace(0, 2 * np.pi, nv, endpoint=False)
    v = np.zeros((n * nv, 3))
    for k in range(n):
        v[k * nv:(k + 1) * nv, 0] = 0.01 * np.cos(ang) + 0.05 * k
        v[k * nv:(k + 1) * nv, 1] = 0.01 * np.sin(ang)
    return seg, v, np.full(n, 1e-3), np.full(n, 0.3)


def _create(lib, n, seg, v, a, R):
    h = ctypes.c_void_p()
    rc = lib.cosim_geometry_create(n, seg.ctypes.data if seg is not None else None,
                                   v.ctypes.data if v is not None else None,
                                   a.ctypes.data if a is not None else None,
                                   R.ctypes.data if R is not None else None, ctypes.byref(h))
    return rc, h


def test_geometry_create_and_errors(lib):
    seg, v, a, R = _geom_args()
    rc, h = _create(lib, 2, seg, v, a, R)
    assert rc == 0 and h.value
    n = ctypes.c_int(); V = ctypes.c_int()
    assert lib.cosim_geometry_size(h, ctypes.byref(n), ctypes.byref(V)) == 0
    assert (n.value, V.value) == (2, 8)
    assert lib.cosim_geometry_destroy(h) == 0
    assert _create(lib, 0, seg, v, a, R)[0] == EINVAL
    assert _create(lib, 2, None, v, a, R)[0] == EINVAL
    bad = seg.copy(); bad[1] = 2  # a loop with 2 vertices
    assert _create(lib, 2, bad, v, a, R)[0] == EINVAL
    assert b"fewer than 3" in lib.cosim_last_error()
    vv = v.copy(); vv[3, 1] = np.nan
    assert _create(lib, 2, seg, vv, a, R)[0] == EINVAL
    aa = a.copy(); aa[1] = 0.0
    assert _create(lib, 2, seg, v, aa, R)[0] == EINVAL
    RR = R.copy(); RR[0] = -1.0
    assert _create(lib, 2, seg, v, a, RR)[0] == EINVAL
    s0 = seg.copy(); s0[0] = 1
    assert _create(lib, 2, s0, v, a, R)[0] == EINVAL


def test_assemble_argument_errors(lib):
    seg, v, a, R = _geom_args()
    rc, g = _create(lib, 2, seg, v, a, R)
    out = ctypes.c_void_p()
    assert lib.cosim_assemble(g, 10, None, 1e-6, None, ctypes.byref(out)) == EINVAL
    assert lib.cosim_assemble(g, 0, ctypes.c_void_p(16), 1e-6, None, ctypes.byref(out)) == EINVAL
    assert lib.cosim_assemble(None, 10, ctypes.c_void_p(16), 1e-6, None, ctypes.byref(out)) == EINVAL
    assert lib.cosim_assemble(g, 10, ctypes.c_void_p(16), float("inf"), None, ctypes.byref(out)) == EINVAL
    assert lib.cosim_assemble(g, 10, ctypes.c_void_p(16), 1e-6, None, None) == EINVAL
    lib.cosim_geometry_destroy(g)
    # more loops than this build's solver supports
    seg, v, a, R = _geom_args(n=1025)
    rc, g = _create(lib, 1025, seg, v, a, R)
    assert rc == 0
    assert lib.cosim_assemble(g, 10, ctypes.c_void_p(16), 1e-6, None, ctypes.byref(out)) == EUNSUPPORTED
    lib.cosim_geometry_destroy(g)


def test_hot_call_argument_errors(lib):
    dummy = ctypes.c_void_p(64)
    # null plan
    assert lib.cosim_solve(None, 1, 1, dummy, dummy, dummy, dummy, None) == EINVAL
    assert lib.cosim_loss_and_grad(None, 1, 1, dummy, dummy, dummy, 0, 1, dummy, dummy, dummy, None) == EINVAL
    assert lib.cosim_field(None, 1, 1, dummy, 0, 0, dummy, None) == EINVAL
    assert lib.cosim_field_backward(None, 1, 1, dummy, dummy, dummy, dummy, 0, 1, dummy, dummy,
                                    None) == EINVAL
    cnt = ctypes.c_longlong()
    assert lib.cosim_plan_factorisations(None, ctypes.byref(cnt)) == EINVAL
    assert lib.cosim_plan_reserve(None, 1, 1) == EINVAL
    assert lib.cosim_plan_copy_M(None, dummy) == EINVAL
    assert lib.cosim_plan_destroy(None) == 0
    assert lib.cosim_geometry_destroy(None) == 0
    assert lib.cosim_last_error() != b""
    # the allocation-free call: null plan, and the size of its per-device array
    assert lib.cosim_loss_and_grad_noalloc(None, 1, 1, dummy, dummy, dummy, 0, 1, dummy, dummy,
                                           dummy, None) == EINVAL
    assert b"null plan" in lib.cosim_last_error()
    assert lib.cosim_noalloc_scratch_bytes() == 64 << 20


def test_tuning_argument_errors(lib):
    v = ctypes.c_int()
    assert lib.cosim_plan_set_variant(None, 0, 0) == EINVAL
    assert lib.cosim_plan_get_variant(None, 0, ctypes.byref(v), None) == EINVAL
    assert lib.cosim_plan_autotune(None, 1, 1, None, None, None, 0, 0, 1, None, None) == EINVAL
    assert lib.cosim_plan_timing(None, 4) == EINVAL


def test_adam_step_argument_errors(lib):
    d = ctypes.c_void_p(64)
    # count 0 is a no-op even with null pointers; the checks below return
    # before any HIP call
    assert lib.cosim_adam_step(0, None, None, None, None, None, 1e-13, 0.9, 0.999, 1e-8, None) == 0
    assert lib.cosim_adam_step(-1, d, d, d, d, d, 1e-13, 0.9, 0.999, 1e-8, None) == EINVAL
    assert lib.cosim_adam_step(4, None, d, d, d, d, 1e-13, 0.9, 0.999, 1e-8, None) == EINVAL
    assert lib.cosim_adam_step(4, d, d, d, d, None, 1e-13, 0.9, 0.999, 1e-8, None) == EINVAL
    assert lib.cosim_adam_step(4, d, d, d, d, d, 1e-13, 1.0, 0.999, 1e-8, None) == EINVAL
    assert lib.cosim_adam_step(4, d, d, d, d, d, 1e-13, 0.9, -0.1, 1e-8, None) == EINVAL
    assert lib.cosim_adam_step(4, d, d, d, d, d, float("nan"), 0.9, 0.999, 1e-8, None) == EINVAL
    assert lib.cosim_adam_step(4, d, d, d, d, d, 1e-13, 0.9, 0.999, -1.0, None) == EINVAL


def test_assemble_mask_and_many_argument_errors(lib):
    seg, v, a, R = _geom_args()
    rc, g = _create(lib, 2, seg, v, a, R)
    out = ctypes.c_void_p()
    d = ctypes.c_void_p(16)
    for mask in (0, 8, -1):
        assert lib.cosim_assemble_ex(g, 10, d, 1e-6, mask, None, ctypes.byref(out)) == EINVAL
    lib.cosim_geometry_destroy(g)
    arr = (ctypes.c_void_p * 1)(None)
    ints = (ctypes.c_int * 1)(1)
    assert lib.cosim_loss_and_grad_many(0, None, None, None, None, None, None, 0, 0, None, None,
                                        None, None) == 0
    assert lib.cosim_loss_and_grad_many(-1, arr, ints, ints, arr, arr, arr, 0, 0, arr, None,
                                        arr, None) == EINVAL
    assert lib.cosim_loss_and_grad_many(1, None, ints, ints, arr, arr, arr, 0, 0, arr, None,
                                        arr, None) == EINVAL
    assert lib.cosim_loss_and_grad_many(1, arr, ints, ints, arr, arr, arr, 0, 7, arr, None,
                                        arr, None) == EINVAL
    # a null plan is reported with its instance index
    assert lib.cosim_loss_and_grad_many(1, arr, ints, ints, arr, arr, arr, 0, 0, arr, None,
                                        arr, None) == EINVAL
    assert b"instance 0" in lib.cosim_last_error()


def test_sparam_argument_errors(lib):
    """cosim_sp_* reject bad shapes, indices, masks and pointers on the host."""
    ix = np.array([0, 1], dtype=np.int32)
    iy = np.array([0, 2], dtype=np.int32)
    exc = np.array([1.0, 0.0])
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails first
    h = ctypes.c_void_p()

    def create(n0=2, n1=1, F=1, P=4, nc=1, s0=fake, fl=fake, nvar=2, x=ix, y=iy, e=exc, mask=1,
               out=True):
        return lib.cosim_sp_create(n0, n1, F, P, nc, s0, fl, None, nvar,
                                   x.ctypes.data if x is not None else None,
                                   y.ctypes.data if y is not None else None,
                                   e.ctypes.data if e is not None else None, mask, None,
                                   ctypes.byref(h) if out else None)

    assert create(out=False) == EINVAL
    assert create(n0=0) == EINVAL
    assert create(n0=65) == EINVAL
    assert create(n1=0) == EINVAL
    assert create(n1=9) == EINVAL
    assert create(F=0) == EINVAL
    assert create(P=0) == EINVAL
    assert create(nc=4) == EINVAL
    assert create(s0=None) == EINVAL
    assert create(fl=None) == EINVAL
    assert create(x=None) == EINVAL
    assert create(e=None) == EINVAL
    assert create(mask=1 << 2) == EUNSUPPORTED
    assert create(mask=0) == EINVAL
    assert create(mask=1 << 5) == EINVAL
    bad = np.array([0, 3], dtype=np.int32)  # column 3 outside the 3 x 3 network
    assert create(y=bad) == EINVAL
    assert b"outside" in lib.cosim_last_error()
    neg = np.array([-1, 0], dtype=np.int32)
    assert create(x=neg) == EINVAL
    # calls on a null plan
    assert lib.cosim_sp_reserve(None, 4) == EINVAL
    assert lib.cosim_sp_field(None, 1, fake, None, None, fake, None) == EINVAL
    assert lib.cosim_sp_loss_and_grad(None, 1, fake, fake, 0, 0, 0, fake, None, fake, None) == EINVAL
    assert lib.cosim_sp_destroy(None) == 0
    # RC preprocessing
    assert lib.cosim_sp_rc(-1, 1, 2, fake, fake, fake, 50.0, fake, 2, None) == EINVAL
    assert lib.cosim_sp_rc(1, 0, 2, fake, fake, fake, 50.0, fake, 2, None) == EINVAL
    assert lib.cosim_sp_rc(1, 1, 2, fake, fake, fake, 50.0, fake, 1, None) == EINVAL
    assert lib.cosim_sp_rc(1, 1, 2, fake, fake, fake, 0.0, fake, 2, None) == EINVAL
    assert lib.cosim_sp_rc(1, 1, 2, None, fake, fake, 50.0, fake, 2, None) == EINVAL
    assert lib.cosim_sp_rc(0, 1, 2, None, None, None, 50.0, None, 2, None) == 0  # empty batch
    assert lib.cosim_sp_rc_backward(1, 1, 2, fake, fake, fake, 50.0, fake, 2, None, None) == EINVAL
    assert lib.cosim_sp_rc_backward(0, 1, 2, None, None, None, 50.0, None, 2, None, None) == 0


def test_parameter_calls_argument_errors(lib):
    fake = ctypes.c_void_p(0x1000)
    assert lib.cosim_loss_and_grad_params(None, 1, 1, fake, fake, fake, 0, 0, fake, fake, None, None,
                                          None, fake, None) == EINVAL
    assert lib.cosim_resonant_capacitance(None, 1, fake, 1, fake, None) == EINVAL
    assert lib.cosim_tanh_projection(-1, fake, 0.0, 1.0, fake, None, None) == EINVAL
    assert lib.cosim_tanh_projection(4, fake, 1.0, 1.0, fake, None, None) == EINVAL   # empty range
    assert lib.cosim_tanh_projection(4, None, 0.0, 1.0, fake, None, None) == EINVAL
    assert lib.cosim_tanh_projection(0, None, 0.0, 1.0, None, None, None) == 0
    assert lib.cosim_clip(4, fake, 2.0, 1.0, None) == EINVAL
    assert lib.cosim_clip(-1, fake, 0.0, 1.0, None) == EINVAL
    assert lib.cosim_clip(0, None, 0.0, 1.0, None) == 0


def test_component_and_drive_argument_errors(lib):
    fake = ctypes.c_void_p(0x1000)
    h = ctypes.c_void_p()
    rc, g = _create(lib, 2, *_geom_args())
    assert rc == 0
    for comp in (-1, 3):
        assert lib.cosim_assemble_component(g, 4, fake, 1e-6, 7, comp, None, ctypes.byref(h)) == EINVAL
        assert not h.value
    lib.cosim_geometry_destroy(g)
    one = np.array([0], dtype=np.int32)
    pw = np.array([1.0])
    assert lib.cosim_plan_set_drive(None, 1, one.ctypes.data, pw.ctypes.data, None, 50.0, None) == EINVAL


def test_refinement_argument_errors(lib):
    assert lib.cosim_plan_set_refinement(None, 1, 8, 0.0) == EINVAL


def test_many_call_checks_list_lengths():
    """ManyCall refuses instance lists of unequal lengths before touching a
    plan or tensor (no GPU needed)."""
    from paper_2503_18479_amd import ManyCall
    with pytest.raises(ValueError):
        ManyCall([object()], [], [], [])

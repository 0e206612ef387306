"""The C ABI without a GPU: the library loads, exports every function the header
declares, and rejects invalid arguments on the host before any launch."""

import ctypes
import os
import re

import pytest

from paper_2010_03598_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kgrape.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w]*\s*\**\s+\**(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libkgrape.so not built")
    return _lib.load()


def test_header_declares_the_boundary():
    fns = header_functions()
    for name in ["xxz_apply", "krylov_expv", "grape_forward", "grape_gradient",
                 "grape_ascent_update", "kg_workspace_bytes", "kg_states_bytes", "kg_last_error"]:
        assert name in fns


def test_every_declared_symbol_is_exported(lib):
    fns = header_functions()
    missing = [n for n in fns if not hasattr(lib, n)]
    assert not missing, missing
    # the Python binding declares a signature for each
    assert sorted(_lib.SIGNATURES) == fns


def xxz(L=8, kind=_lib.KG_HC_SX, sites=1, J=1.0, Delta=0.5):
    return _lib.KgXxz(L, kind, J, Delta, sites)


def kry(m=10, reorth=1, tol=0.0):
    return _lib.KgKrylov(m, reorth, tol)


def test_workspace_and_state_sizes(lib):
    h = xxz(L=10)
    k = kry(m=8)
    ws128 = lib.kg_workspace_bytes(ctypes.byref(h), ctypes.byref(k), _lib.KG_C128)
    ws64 = lib.kg_workspace_bytes(ctypes.byref(h), ctypes.byref(k), _lib.KG_C64)
    vb128, vb64 = 16 << 10, 8 << 10
    assert ws128 - ws64 == 17 * (vb128 - vb64)         # 2 x (7 basis + 1 H v) + 1 costate
    assert lib.kg_states_bytes(ctypes.byref(h), 100, 0, _lib.KG_C128) == 100 * vb128
    # checkpoints every 20: 4 checkpoints below the last segment + 2 x 20 buffer slots
    assert lib.kg_states_bytes(ctypes.byref(h), 100, 20, _lib.KG_C64) == 44 * vb64
    assert lib.kg_states_bytes(ctypes.byref(h), 101, 20, _lib.KG_C64) == 45 * vb64
    assert lib.kg_states_bytes(ctypes.byref(h), 100, 100, _lib.KG_C64) == 100 * vb64
    assert lib.kg_states_bytes(ctypes.byref(h), 10, 11, _lib.KG_C64) == 0
    assert lib.kg_workspace_bytes(ctypes.byref(h), ctypes.byref(kry(m=0)), _lib.KG_C64) == 0


@pytest.mark.parametrize("bad,msg", [
    (dict(L=1), "L=1"), (dict(L=31), "L=31"), (dict(kind=7), "hc_kind"),
    (dict(sites=0), "empty"), (dict(sites=3), "exactly one"), (dict(L=4, sites=1 << 4), "beyond"),
    (dict(J=float("nan")), "finite"),
])
def test_invalid_chain_rejected(lib, bad, msg):
    h = xxz(**bad)
    fake = ctypes.c_void_p(256)
    st = lib.xxz_apply(ctypes.byref(h), 0.1, _lib.KG_C128, fake, ctypes.c_void_p(1 << 20), None)
    assert st == _lib.KG_EINVAL
    assert msg in _lib.last_error()


def test_invalid_krylov_and_workspace_rejected(lib):
    h = xxz(L=6)
    v = ctypes.c_void_p(1 << 12)
    w = ctypes.c_void_p(1 << 16)
    for k, msg in [(kry(m=0), "m=0"), (kry(m=65), "m=65"), (kry(reorth=2), "reorth"),
                   (kry(tol=-1.0), "breakdown_tol")]:
        st = lib.krylov_expv(ctypes.byref(h), 0.0, 0.1, ctypes.byref(k), _lib.KG_C128, v, w,
                             ctypes.c_void_p(1 << 20), 1 << 30, None, None)
        assert st == _lib.KG_EINVAL and msg in _lib.last_error()
    k = kry(m=4)
    st = lib.krylov_expv(ctypes.byref(h), 0.0, 0.1, ctypes.byref(k), _lib.KG_C128, v, w,
                         ctypes.c_void_p(1 << 20), 16, None, None)
    assert st == _lib.KG_EWORKSPACE and "needs" in _lib.last_error()
    st = lib.krylov_expv(ctypes.byref(h), 0.0, 0.1, ctypes.byref(k), _lib.KG_C128, v, w,
                         ctypes.c_void_p((1 << 20) + 8), 1 << 30, None, None)
    assert st == _lib.KG_EWORKSPACE and "aligned" in _lib.last_error()
    st = lib.krylov_expv(ctypes.byref(h), 0.0, 0.1, ctypes.byref(k), _lib.KG_C128,
                         ctypes.c_void_p(8), w, ctypes.c_void_p(1 << 20), 1 << 30, None, None)
    assert st == _lib.KG_EINVAL and "aligned" in _lib.last_error()
    st = lib.krylov_expv(ctypes.byref(h), 0.0, 0.1, ctypes.byref(k), _lib.KG_C128, v,
                         ctypes.c_void_p((1 << 12) + 16), ctypes.c_void_p(1 << 20), 1 << 30, None,
                         None)
    assert st == _lib.KG_EINVAL and "overlap" in _lib.last_error()
    st = lib.krylov_expv(ctypes.byref(h), 0.0, 0.1, ctypes.byref(k), 5, v, w,
                         ctypes.c_void_p(1 << 20), 1 << 30, None, None)
    assert st == _lib.KG_EINVAL and "precision" in _lib.last_error()


def test_invalid_sweep_arguments_rejected(lib):
    h = xxz(L=6)
    k = kry(m=4)
    p = ctypes.c_void_p
    args = dict(u=p(1 << 12), N=10, dt=0.1, psi0=p(1 << 14), f=p(1 << 15), F=p(1 << 16),
                beta=p(1 << 17), grad=p(1 << 18), states=p(1 << 19), ckpt=0, valid=0)

    def call(**kw):
        a = dict(args, **kw)
        return lib.grape_gradient(ctypes.byref(h), a["u"], a["N"], a["dt"], ctypes.byref(k),
                                  _lib.KG_C64, a["psi0"], a["f"], a["F"], a["beta"], a["grad"],
                                  a["states"], a["ckpt"], a["valid"], p(1 << 20), 1 << 30, None)

    assert call(N=0) == _lib.KG_EINVAL and "N=0" in _lib.last_error()
    assert call(ckpt=11) == _lib.KG_EINVAL and "ckpt_every" in _lib.last_error()
    assert call(ckpt=-1) == _lib.KG_EINVAL
    assert call(u=p(0)) == _lib.KG_EINVAL and "u_dev" in _lib.last_error()
    assert call(grad=p(0)) == _lib.KG_EINVAL
    assert call(valid=3) == _lib.KG_EINVAL
    assert call(dt=float("inf")) == _lib.KG_EINVAL
    assert call(psi0=p(4)) == _lib.KG_EINVAL
    assert lib.grape_ascent_update(p(8), p(16), 0, 0.1, None) == _lib.KG_EINVAL
    assert lib.kg_debug_index_map(8, 250, 10, p(8), p(16), None) == _lib.KG_EINVAL
    assert lib.kg_version() >= 1

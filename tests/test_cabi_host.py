"""The C-ABI library loads and exports every function include/lbm_ec.h
declares; the host-only entry points (defaults, validation, workspace
sizing, error reporting) behave as documented.  No GPU is touched."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm_ec.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_ec_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def E():
    from paper_1812_05711_amd import lbm_ec

    lbm_ec.lib()
    return lbm_ec


def test_every_declared_symbol_is_exported(E):
    names = declared_functions()
    assert len(names) >= 20
    lib = ctypes.CDLL(E.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_defaults_and_validation(E):
    p = E.make_params(122, 100)
    assert (p.nx, p.ny, p.T, p.C, p.M, p.Fe) == (122, 100, 200.0, 10.0, 10.0, 4000.0)
    assert E.lib().lbm_ec_validate(ctypes.byref(p)) == E.OK
    for bad in (dict(tau_plus=0.5), dict(ny=2), dict(Lambda=0.0), dict(Fe=-1.0), dict(init_mode=7),
                dict(nx=5000, precision="fp64"), dict(charge_rates=3)):
        kw = dict(nx=122, ny=100)
        kw.update(bad)
        q = E.make_params(**kw)
        assert E.lib().lbm_ec_validate(ctypes.byref(q)) == E.EINVAL, bad
        assert E.lib().lbm_ec_last_error().decode() != ""
        assert E.lib().lbm_ec_workspace_bytes(ctypes.byref(q)) == 0


def test_workspace_sizes(E):
    f64 = E.workspace_bytes(E.make_params(122, 100))
    f32 = E.workspace_bytes(E.make_params(122, 100, precision="fp32"))
    assert f64 > f32 > 0
    big = E.workspace_bytes(E.make_params(4096, 4096, precision="fp32"))
    # populations dominate: 4 arrays of 9 x 4096 x 4096 floats
    assert 4 * 9 * 4096 * 4096 * 4 < big < 1.5 * 4 * 9 * 4096 * 4096 * 4 + 2 * 4 * 4096 * 4096 * 8
    head = E.batch_workspace_bytes([], 8, 16)
    one = E.batch_workspace_bytes([E.make_params(64, 32)], 8, 16)
    assert one - head == E.workspace_bytes(E.make_params(64, 32))


def test_create_rejects_small_workspace_without_touching_the_device(E):
    p = E.make_params(16, 8)
    h = ctypes.c_void_p()
    code = E.lib().lbm_ec_create(ctypes.byref(p), ctypes.c_void_p(256), 16, None, ctypes.byref(h))
    assert code == E.ENOMEM
    assert "workspace" in E.lib().lbm_ec_last_error().decode()

"""C-ABI checks that need no GPU: every symbol of include/atns.h is exported, and argument
validation happens before any device call."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2003_10561_amd import atns

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    src = open(os.path.join(ROOT, "include", "atns.h")).read()
    return sorted(set(re.findall(r"ATNS_API\s+[\w\s\*]+?\b(at_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(atns.LIB_PATH):
        pytest.skip("libatns.so not built")
    return atns.load_library()


def test_every_declared_symbol_is_exported(lib):
    syms = header_symbols()
    assert len(syms) >= 13
    for s in syms:
        assert hasattr(lib, s), s
    assert set(atns.EXPORTED) <= set(syms)


def test_only_abi_symbols_are_exported(lib):
    out = os.popen(f"nm -D --defined-only {atns.LIB_PATH}").read().split("\n")
    ours = [l.split()[-1] for l in out if " T " in l]
    assert ours and all(s.startswith("at_") for s in ours), ours


def cfg(**kw):
    base = dict(n=(32, 32, 32), p=(2, 2, 1), dt=0.01, mu_ref=0.01, max_delay=3)
    base.update(kw)
    return atns.Config(**base)


def test_workspace_bytes_formula(lib):
    c = cfg()
    b64 = atns.workspace_bytes(c)
    b32 = atns.workspace_bytes(cfg(precision="fp32"))
    assert b64 > 0 and b32 > 0 and b32 < b64
    N = 32 ** 3
    # two state buffers, the RK register, the ring of 6 levels x 9 components on the face layers
    # and three more level-sized buffers of AT sums (one per stage of a step): lower bound in FP64;
    # the scratch beyond it (reduction partials, tables) is small
    phi = 4 * (1 / 16 + 1 / 16 + 1 / 32)
    ring = (6 + 3) * 9 * phi * N
    need = 8 * (5 + 5 + 5) * N + 8 * ring
    assert need <= b64 <= 1.1 * need


def test_workspace_bytes_formula_order6(lib):
    """Sixth order: three face layers per side (phi = 6 (1/ex + 1/ey + 1/ez)), a ring of L + 4 levels,
    three ring-slot buffers of extrapolated face values (one per stage) and the 15-component flux
    buffer."""
    b64 = atns.workspace_bytes(cfg(order=6))
    N = 32 ** 3
    phi = 6 * (1 / 16 + 1 / 16 + 1 / 32)
    ring = (3 + 4 + 3) * 9 * phi * N
    need = 8 * (5 + 5 + 5 + 15) * N + 8 * ring
    assert need <= b64 <= 1.1 * need


def test_workspace_bytes_formula_paper_form(lib):
    """The paper's form: the ring holds the five conserved variables of the two face layers per side
    (L + 3 levels) and a 12-component gradient buffer replaces the AT-sum buffers."""
    b64 = atns.workspace_bytes(cfg(form=1))
    N = 32 ** 3
    phi = 4 * (1 / 16 + 1 / 16 + 1 / 32)
    ring = (3 + 3) * 5 * phi * N
    need = 8 * (5 + 5 + 5 + 12) * N + 8 * ring
    assert need <= b64 <= 1.15 * need
    assert atns.workspace_bytes(cfg(form=1, visc_law=1, sutherland_s=0.4)) == b64


@pytest.mark.parametrize("bad", [dict(n=(30, 32, 32), p=(4, 2, 1)), dict(p=(16, 2, 1)), dict(order=8),
                                 dict(order=6, p=(8, 2, 1)), dict(order=6, forcing=True),
                                 dict(form=2), dict(visc_law=1, sutherland_s=0.4), dict(form=1, visc_law=1),
                                 dict(form=1, order=6), dict(form=1, forcing=True), dict(form=1, p=(8, 2, 1)),
                                 dict(visc_law=2, form=1),
                                 dict(max_delay=9), dict(dt=0.0), dict(mu_ref=-1.0),
                                 dict(gamma=1.0), dict(precision="fp16x")])
def test_invalid_config_rejected_without_gpu(lib, bad):
    c = cfg(**bad)
    cc = c.to_c()
    if bad.get("precision") == "fp16x":
        cc.precision = 7
    assert lib.at_workspace_bytes(C.byref(cc)) == 0
    h = C.c_void_p()
    rc = lib.at_create(C.byref(cc), C.c_void_p(256), 1 << 30, None, C.byref(h))
    assert rc == atns.AT_E_INVAL
    assert lib.at_last_error().decode() != ""


def test_workspace_checks_without_gpu(lib):
    cc = cfg().to_c()
    need = lib.at_workspace_bytes(C.byref(cc))
    h = C.c_void_p()
    assert lib.at_create(C.byref(cc), None, need, None, C.byref(h)) == atns.AT_E_WORKSPACE
    assert lib.at_create(C.byref(cc), C.c_void_p(257), need, None, C.byref(h)) == atns.AT_E_WORKSPACE
    assert lib.at_create(C.byref(cc), C.c_void_p(256), need - 1, None, C.byref(h)) == atns.AT_E_WORKSPACE


def test_null_handle_calls(lib):
    assert lib.at_rk_step(None, 1) == atns.AT_E_INVAL
    assert lib.at_ab2_step(None, 1) == atns.AT_E_INVAL
    assert lib.at_set_stage_tuning(None, 1, 64, 5, 64) == atns.AT_E_INVAL
    assert lib.at_batch_set_stage_tuning(None, 1, 64, 5, 64) == atns.AT_E_INVAL
    v = [C.c_int32() for _ in range(4)]
    assert lib.at_get_stage_tuning(None, *[C.byref(x) for x in v]) == atns.AT_E_INVAL
    assert lib.at_destroy(None) == atns.AT_OK
    assert lib.at_version().decode().startswith("atns")


def test_batch_and_serve_argument_checks_without_gpu(lib):
    """Argument errors are reported before any device call."""
    assert lib.at_batch_step(None, 1) == atns.AT_E_INVAL
    assert lib.at_batch_add(None, None) == atns.AT_E_INVAL
    assert lib.at_batch_autotune(None, None, 3, None) == atns.AT_E_INVAL
    assert lib.at_batch_destroy(None) == atns.AT_OK
    h = C.c_void_p()
    assert lib.at_batch_create(7, None, C.byref(h)) == atns.AT_E_INVAL
    sc = atns._ServeConfig(atns.FP32, 4, -1, 64, 1e9)
    assert lib.at_serve(None, None, 0, None, None, None) == atns.AT_E_INVAL
    q = np.zeros((5, 16, 16, 16))
    reqs = (atns._Request * 2)()
    for i, t in enumerate((0.5, 0.1)):  # arrivals out of order
        reqs[i] = atns._Request(t, 16, 2, 3, atns.SYNC, 0, 0, 0.01, 0.01,
                                q.ctypes.data_as(C.POINTER(C.c_double)), None)
    res = (atns._Result * 2)()
    assert lib.at_serve(C.byref(sc), reqs, 2, None, res, None) == atns.AT_E_INVAL
    assert "sorted" in lib.at_last_error().decode()
    reqs[1].arrival_s = 0.6
    reqs[1].n, reqs[1].p = 18, 4  # 18 is not a multiple of 4
    assert lib.at_serve(C.byref(sc), reqs, 2, None, res, None) == atns.AT_E_INVAL
    bad = atns._ServeConfig(atns.FP32, 0, -1, 64, 1e9)
    assert lib.at_serve(C.byref(bad), reqs, 0, None, res, None) == atns.AT_E_INVAL


def test_grid_beyond_32bit_offsets_rejected(lib):
    """The largest grids: element offsets of one handle must stay below 2^32."""
    ok = cfg(n=(1024, 1024, 512), p=(16, 16, 8), max_delay=1)  # ring: 4 x 9 x 100M < 2^32
    assert lib.at_workspace_bytes(C.byref(ok.to_c())) > 0
    big = cfg(n=(2048, 2048, 512), p=(32, 32, 8))  # 5 * N >= 2^32
    assert lib.at_workspace_bytes(C.byref(big.to_c())) == 0
    assert "2^32" in lib.at_last_error().decode()

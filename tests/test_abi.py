"""Host-only checks of the C ABI (no GPU needed): the library loads, exports
every function include/glr.h declares, and rejects bad plans with the
documented status before touching the device."""
import ctypes
import os
import re

import pytest

import paper_2301_03047_amd as glr
from paper_2301_03047_amd.glr import Problem, Params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "glr.h")

FAKE_MASK = 4096          # never dereferenced by plan creation


def declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"GLR_API\s+[\w\s\*]+?\b(glr_\w+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 18
    L = glr.lib()
    for n in names:
        assert hasattr(L, n), f"{n} declared in glr.h but not exported"


def test_version_and_status_strings():
    L = glr.lib()
    assert L.glr_version() == 100
    for code, name in glr.STATUS_NAMES.items():
        assert L.glr_status_string(code).decode() == name


def _create(modality=glr.CACTI, H=64, W=64, C=4, P=6, N=32, K=16, iters=0, mask=FAKE_MASK,
            solver=None, **kw):
    L = glr.lib()
    prob = Problem(modality, H, W, C, mask)
    par = Params()
    L.glr_params_default(ctypes.byref(par))
    par.patch, par.n_keys, par.k, par.iters = P, N, K, iters
    par.solver = (1 if modality == glr.MRI else 0) if solver is None else solver
    for k, v in kw.items():
        setattr(par, k, v)
    h = ctypes.c_void_p()
    ws = ctypes.c_size_t()
    st = L.glr_plan_create(ctypes.byref(h), ctypes.byref(prob), ctypes.byref(par), ctypes.byref(ws))
    if st == 0:
        L.glr_plan_destroy(h)
    return st, ws.value, L.glr_last_error_message().decode()


def test_valid_plans_report_workspace():
    st, ws, _ = _create()
    assert st == 0 and ws > 0 and ws % 256 == 0
    st, ws_mri, _ = _create(glr.MRI, 256, 256, 1, 6, 1024, 45)
    assert st == 0
    # the distance chunk dominates: 1024 keys x 63001 candidates (row stride 63040)
    assert ws_mri >= 1024 * 63040 * 4
    st, _, _ = _create(glr.MSFA, 32, 32, 16, 6, 20, 8, mask=0)
    assert st == 0
    st, ws_c, _ = _create(glr.MRI, 256, 256, 1, 6, 1024, 45, lowrank=1)
    assert st == 0 and ws_c == ws_mri


@pytest.mark.parametrize("kw,code", [
    (dict(K=0), 2), (dict(K=65), 4), (dict(P=0), 2), (dict(P=70, H=64), 2), (dict(P=17, H=64), 4),
    (dict(N=0), 2), (dict(N=10 ** 6), 2), (dict(H=8, W=8, P=6, N=9, K=10), 2),
    (dict(C=128, P=6), 4), (dict(mask=0), 1), (dict(mask=FAKE_MASK + 1), 3),
    (dict(modality=7), 1), (dict(precision=5), 1), (dict(solver=1), 1),
    (dict(iters=3), 1), (dict(wnnm_eps=0.0), 1), (dict(agg_weights=2), 1),
    (dict(wnnm_iters=0), 1), (dict(wnnm_iters=17), 1), (dict(wnnm_iters=2, wnnm_delta=2.0), 1),
    (dict(wnnm_iters=2, wnnm_lambda=0.0), 1),
    (dict(lowrank=1), 1), (dict(modality=glr.MRI, H=64, W=64, C=1, lowrank=2), 1),
    (dict(modality=glr.MSFA, C=16, mask=0, lowrank=1), 1),
])
def test_invalid_plans(kw, code):
    st, _, msg = _create(**kw)
    assert st == code, (st, msg)
    assert msg


def test_mri_and_msfa_limits():
    assert _create(glr.MRI, 200, 256, 1, 6, 10, 4)[0] == 4      # not a power of two
    assert _create(glr.MRI, 256, 256, 2, 6, 10, 4)[0] == 2      # complex image is C = 1
    assert _create(glr.MRI, 256, 256, 1, 6, 10, 4, solver=0)[0] == 1
    assert _create(glr.MSFA, 32, 32, 8, 6, 10, 4, mask=0)[0] == 4
    assert _create(glr.MSFA, 30, 32, 16, 6, 10, 4, mask=0)[0] == 2


def test_null_arguments_rejected_before_launch():
    L = glr.lib()
    assert L.glr_plan_create(None, None, None, None) == 1
    assert L.glr_plan_destroy(None) == 1
    st = _create()
    # a call on a NULL plan fails on the host
    assert L.glr_prior_step(None, None, ctypes.c_float(0.1), None, None, None) == 1
    assert L.glr_read_stats(None, None, 0) == 1


def test_library_fails_loudly_when_missing(tmp_path, monkeypatch):
    import paper_2301_03047_amd.glr as g
    monkeypatch.setattr(g, "_LIB", None)
    monkeypatch.setattr(g, "library_path", lambda: str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        g.lib()


def _plan_handle(**kw):
    L = glr.lib()
    prob = Problem(glr.CACTI, kw.pop("H"), kw.pop("W"), kw.pop("C"), FAKE_MASK)
    par = Params()
    L.glr_params_default(ctypes.byref(par))
    par.patch, par.n_keys, par.k = kw.pop("P"), kw.pop("N"), kw.pop("K")
    for k, v in kw.items():
        setattr(par, k, v)
    h = ctypes.c_void_p()
    ws = ctypes.c_size_t()
    assert L.glr_plan_create(ctypes.byref(h), ctypes.byref(prob), ctypes.byref(par),
                             ctypes.byref(ws)) == 0
    return h, ws.value


def test_static_prior_step_refuses_on_the_host():
    """The allocation-free prior step checks the plan against its fixed
    scratch size (and refuses timing plans) before any device call."""
    L = glr.lib()
    fake = ctypes.c_void_p(FAKE_MASK)
    h, ws = _plan_handle(H=256, W=256, C=8, P=6, N=512, K=32)
    try:
        assert ws > glr.STATIC_SCRATCH_BYTES
        st = L.glr_prior_step_static(h, fake, ctypes.c_float(0.05), ctypes.c_void_p(2 * FAKE_MASK),
                                     None)
        assert st == 5, L.glr_last_error_message()
        assert b"static scratch" in L.glr_last_error_message()
    finally:
        L.glr_plan_destroy(h)
    h, ws = _plan_handle(H=64, W=64, C=4, P=6, N=32, K=16, timing=1)
    try:
        assert ws <= glr.STATIC_SCRATCH_BYTES
        st = L.glr_prior_step_static(h, fake, ctypes.c_float(0.05), ctypes.c_void_p(2 * FAKE_MASK),
                                     None)
        assert st == 4, L.glr_last_error_message()
    finally:
        L.glr_plan_destroy(h)
    assert L.glr_prior_step_static(None, fake, ctypes.c_float(0.05), fake, None) == 1


def _keys_of(**kw):
    L = glr.lib()
    prob = Problem(glr.CACTI, kw.pop("H"), kw.pop("W"), kw.pop("C"), FAKE_MASK)
    par = Params()
    L.glr_params_default(ctypes.byref(par))
    par.patch, par.n_keys, par.k = kw.pop("P"), kw.pop("N"), kw.pop("K")
    for k, v in kw.items():
        setattr(par, k, v)
    h = ctypes.c_void_p()
    ws = ctypes.c_size_t()
    st = L.glr_plan_create(ctypes.byref(h), ctypes.byref(prob), ctypes.byref(par), ctypes.byref(ws))
    if st:
        return st, None
    n = ctypes.c_int32()
    assert L.glr_plan_keys(h, ctypes.byref(n)) == 0
    L.glr_plan_destroy(h)
    return 0, n.value


def test_exemplar_counts_and_window_limits():
    # 256 x 256, P = 6: a 251 x 251 grid; interval 4 -> 63^2, interval 12 -> 21^2
    assert _keys_of(H=256, W=256, C=8, P=6, N=512, K=32) == (0, 512)
    assert _keys_of(H=256, W=256, C=8, P=6, N=512, K=32, exemplars=1, uniform_step=4) == (0, 3969)
    assert _keys_of(H=256, W=256, C=8, P=6, N=512, K=32, exemplars=2, uniform_step=4) == (0, 953)
    assert _keys_of(H=256, W=256, C=8, P=6, N=512, K=32, search=1, window=20) == (0, 512)
    # a 5 x 5 corner window holds 25 < K = 32 candidates
    assert _keys_of(H=64, W=64, C=2, P=4, N=8, K=32, search=1, window=4)[0] == 2
    assert _keys_of(H=64, W=64, C=2, P=4, N=8, K=32, search=1, window=0)[0] == 1
    assert _keys_of(H=64, W=64, C=2, P=4, N=8, K=8, exemplars=3)[0] == 1
    assert _keys_of(H=64, W=64, C=2, P=4, N=8, K=8, search=2)[0] == 1
    assert _keys_of(H=64, W=64, C=2, P=4, N=8, K=8, exemplars=1, uniform_step=0)[0] == 1
    # more than 16384 exemplars: 1019^2 positions at interval 4 -> 255^2
    assert _keys_of(H=1024, W=1024, C=1, P=6, N=8, K=8, exemplars=1, uniform_step=4)[0] == 4

"""CPU-side checks of the C ABI: the library loads, exports every entry point
the header declares, and rejects bad arguments on the host before touching a
GPU. No compute calls are made here."""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ssm_cascade.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ssm_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2411_17729_amd import binding as B
    if not os.path.exists(B.LIB_PATH):
        pytest.fail("libssm_cascade.so is not built (run __graft_entry__.build())")
    return B.load()


def test_header_declares_the_boundary():
    names = _declared()
    for required in ["ssm_cascade_prepare", "ssm_cascade_apply", "ssm_cascade_backward",
                     "ssm_cascade_recursion", "ssm_cascade_workspace_bytes"]:
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_exposes_the_same_names():
    from paper_2411_17729_amd import binding as B
    for name in _declared():
        assert callable(getattr(B, name, None)), name


def _desc(**kw):
    from paper_2411_17729_amd import binding as B
    d = dict(m=64, p=1, q=1, N=11, L=4096, delta=1e-2, param_set=0, reserved=0,
             u_offset=0, y_offset=0)
    d.update(kw)
    return B.ssm_seq_desc(**d)


@pytest.mark.parametrize("bad", [dict(m=0), dict(m=300), dict(p=0), dict(p=65), dict(q=65),
                                 dict(N=-31), dict(N=63), dict(L=0), dict(param_set=-1),
                                 dict(reserved=1), dict(u_offset=-1), dict(delta=0.0),
                                 dict(delta=float("nan"))])
def test_workspace_bytes_rejects_bad_descriptors(lib, bad):
    from paper_2411_17729_amd import binding as B
    arr = (B.ssm_seq_desc * 1)(_desc(**bad))
    assert lib.ssm_cascade_workspace_bytes(arr, 1, 0, 1, 0, 0, None) == 0
    assert lib.ssm_last_error().decode() != ""


def test_workspace_bytes_grows_with_batch(lib):
    from paper_2411_17729_amd import binding as B
    one = (B.ssm_seq_desc * 1)(_desc())
    two = (B.ssm_seq_desc * 2)(_desc(), _desc(u_offset=4096, y_offset=4096))
    n1 = lib.ssm_cascade_workspace_bytes(one, 1, 0, 1, 0, 0, None)
    n2 = lib.ssm_cascade_workspace_bytes(two, 2, 0, 1, 0, 0, None)
    assert 0 < n1 < n2
    # the second sequence shares the operator: only the state buffers and the
    # per-sequence launch tables (tiles, row ranges, chain units) grow
    assert n2 - n1 <= 2 * 4096 * 64 * 4 + 16384


def test_prepare_rejects_on_host(lib):
    from paper_2411_17729_amd import binding as B
    arr = (B.ssm_seq_desc * 1)(_desc())
    params = (B.ssm_params * 1)(B.ssm_params(A=None, B=None, C=None, D=None, m=64, p=1, q=1))
    plan = C.c_void_p()
    # NULL workspace
    st = lib.ssm_cascade_prepare(arr, 1, params, 1, 0, 1, 0, 0, None, None, 0, None, C.byref(plan))
    assert st == B.SSM_E_INVALID and plan.value is None
    # NULL parameter matrices (non-NULL fake workspace is never dereferenced)
    st = lib.ssm_cascade_prepare(arr, 1, params, 1, 0, 1, 0, 0, None, C.c_void_p(256), 1 << 40,
                                 None, C.byref(plan))
    assert st == B.SSM_E_INVALID
    # short workspace
    params[0] = B.ssm_params(A=256, B=256, C=256, D=256, m=64, p=1, q=1)
    st = lib.ssm_cascade_prepare(arr, 1, params, 1, 0, 1, 0, 0, None, C.c_void_p(256), 16, None,
                                 C.byref(plan))
    assert st == B.SSM_E_WORKSPACE
    # param_set beyond n_sets
    arr2 = (B.ssm_seq_desc * 1)(_desc(param_set=1))
    st = lib.ssm_cascade_prepare(arr2, 1, params, 1, 0, 1, 0, 0, None, C.c_void_p(256), 1 << 40,
                                 None, C.byref(plan))
    assert st == B.SSM_E_INVALID


def test_null_plan_calls(lib):
    from paper_2411_17729_amd import binding as B
    assert lib.ssm_cascade_apply(None, None, 1, 0, None, 0, None) == B.SSM_E_NOT_PREPARED
    assert lib.ssm_cascade_recursion(None, None, 1, 0, None, 0, None) == B.SSM_E_NOT_PREPARED
    assert lib.ssm_cascade_apply_noalloc(None, None, 1, 0, None, 0, None) == B.SSM_E_NOT_PREPARED
    assert lib.ssm_cascade_apply_state(None, None, 1, 0, None, 0, None, 0, None, 0, None) == B.SSM_E_NOT_PREPARED
    assert lib.ssm_cascade_destroy(None) == B.SSM_OK
    assert lib.ssm_cascade_param_grad_numel(None) == 0
    assert "INVALID" in lib.ssm_status_string(B.SSM_E_INVALID).decode()


def test_tuning_is_validated(lib):
    from paper_2411_17729_amd import binding as B
    arr = (B.ssm_seq_desc * 1)(_desc())
    for bad in (B.make_tuning(launch=7), B.make_tuning(tile_rows=(0, 100, 0, 0)),
                B.make_tuning(stage_kernel=4), B.make_tuning(chain_blocks=65),
                B.make_tuning(chain_blocks=-1), B.make_tuning(pair_stages=2),
                B.make_tuning(pair_stages=-1), B.make_tuning(pair_blocks=3),
                B.make_tuning(pair_blocks=257), B.make_tuning(input_split=2),
                B.make_tuning(state_bf16=2), B.make_tuning(state_bf16=-1),
                B.make_tuning(fold_stages=1), B.make_tuning(fold_stages=7), B.make_tuning(fold_stages=-2)):
        assert lib.ssm_cascade_workspace_bytes(arr, 1, 0, 1, 0, 0, C.byref(bad)) == 0
    for t in (B.make_tuning(pair_stages=1), B.make_tuning(pair_blocks=4), B.make_tuning(pair_blocks=256),
              B.make_tuning(input_split=1), B.make_tuning(state_bf16=1), B.make_tuning(fold_stages=-1),
              B.make_tuning(fold_stages=2), B.make_tuning(fold_stages=5), B.make_tuning(fold_stages=6)):
        assert lib.ssm_cascade_workspace_bytes(arr, 1, 0, 1, 0, 0, C.byref(t)) > 0
    for sk in (B.SSM_STAGE_RESIDENT, B.SSM_STAGE_CHAIN):  # FP32 only, not FP64 (compute 0)
        t = B.make_tuning(stage_kernel=sk, chain_blocks=3)
        assert lib.ssm_cascade_workspace_bytes(arr, 1, 0, 1, 0, 0, C.byref(t)) > 0
        assert lib.ssm_cascade_workspace_bytes(arr, 1, 0, 0, 0, 0, C.byref(t)) == 0
    t = B.make_tuning(tile_rows=(0, 64, 0, 0))  # half of the default 128 for m <= 64
    assert lib.ssm_cascade_workspace_bytes(arr, 1, 0, 1, 0, 0, C.byref(t)) > 0
    for bad in (1, 100, 512, -64):
        t = B.make_tuning(min_padded_m=bad)
        assert lib.ssm_cascade_workspace_bytes(arr, 1, 0, 1, 0, 0, C.byref(t)) == 0
    # padding m = 64 to 128 doubles the state buffers of the 4096 rows
    small = lib.ssm_cascade_workspace_bytes(arr, 1, 0, 1, 0, 0, None)
    t = B.make_tuning(min_padded_m=128)
    assert lib.ssm_cascade_workspace_bytes(arr, 1, 0, 1, 0, 0, C.byref(t)) >= small + 2 * 4096 * 64 * 4
    # final_state: 0 or 1, not with an explicitly persistent launch
    for bad in (B.make_tuning(final_state=2), B.make_tuning(final_state=-1),
                B.make_tuning(final_state=1, launch=B.SSM_LAUNCH_PERSISTENT)):
        assert lib.ssm_cascade_workspace_bytes(arr, 1, 0, 1, 0, 0, C.byref(bad)) == 0
    t = B.make_tuning(final_state=1)
    assert lib.ssm_cascade_workspace_bytes(arr, 1, 0, 1, 0, 0, C.byref(t)) > 0
    # static_state: 0 or 1, the workspace without the two state buffers
    # (4096 rows of 64 FP32 entries each), not with the backward
    for bad in (B.make_tuning(static_state=2), B.make_tuning(static_state=-1)):
        assert lib.ssm_cascade_workspace_bytes(arr, 1, 0, 1, 0, 0, C.byref(bad)) == 0
    full = lib.ssm_cascade_workspace_bytes(arr, 1, 0, 1, 0, 0, None)
    t = B.make_tuning(static_state=1)
    lean = lib.ssm_cascade_workspace_bytes(arr, 1, 0, 1, 0, 0, C.byref(t))
    assert lean > 0 and full - lean >= 2 * 4096 * 64 * 4
    assert lib.ssm_cascade_workspace_bytes(arr, 1, 0, 1, 1, 0, C.byref(t)) == 0
    assert "static_state" in lib.ssm_last_error().decode()
    t = B.make_tuning(spin_limit=-1)
    assert lib.ssm_cascade_workspace_bytes(arr, 1, 0, 1, 0, 0, C.byref(t)) == 0
    t = B.make_tuning(spin_limit=1)
    assert lib.ssm_cascade_workspace_bytes(arr, 1, 0, 1, 0, 0, C.byref(t)) > 0


def test_discretizations_on_host(lib):
    # trapezoid, given and exponential are accepted; the exponential needs its
    # scratch (three (m + p)^2 FP64 matrices per operator, six with the
    # backward); an unknown value is rejected
    from paper_2411_17729_amd import binding as B
    arr = (B.ssm_seq_desc * 1)(_desc(m=100, p=3))
    n = {d: lib.ssm_cascade_workspace_bytes(arr, 1, d, 1, 0, 0, None) for d in (0, 1, 2)}
    nb = {d: lib.ssm_cascade_workspace_bytes(arr, 1, d, 1, 1, 0, None) for d in (0, 2)}
    assert all(v > 0 for v in n.values()) and all(v > 0 for v in nb.values())
    assert n[2] >= n[1] + 3 * 103 * 103 * 8 and nb[2] >= n[2] + 3 * 103 * 103 * 8
    assert lib.ssm_cascade_workspace_bytes(arr, 1, 3, 1, 0, 0, None) == 0
    assert "discretization" in lib.ssm_last_error().decode()
    # the exponential needs a positive finite step, as the trapezoidal rule does
    bad = (B.ssm_seq_desc * 1)(_desc(m=100, p=3, delta=0.0))
    assert lib.ssm_cascade_workspace_bytes(bad, 1, 2, 1, 0, 0, None) == 0


def test_graph_calls_reject_on_host(lib):
    from paper_2411_17729_amd import binding as B
    g = C.c_void_p()
    assert lib.ssm_cascade_graph_apply(None, None, 1, 0, None, 0, None, C.byref(g)) == B.SSM_E_NOT_PREPARED
    assert lib.ssm_cascade_graph_launch(None, None) == B.SSM_E_INVALID
    assert lib.ssm_cascade_graph_destroy(None) == B.SSM_OK


def test_plr_tuning_is_validated(lib):
    """PLR powers: digits 0..15; FP32 or FP64 compute, forward only, per-stage
    launches; the records, rank table and compression scratch enlarge the
    workspace of a plan with an eligible stage."""
    from paper_2411_17729_amd import binding as B
    d = _desc()
    d.m, d.N, d.L = 256, 8, 4096
    arr = (B.ssm_seq_desc * 1)(d)
    for bad in (B.make_tuning(plr_digits=-1), B.make_tuning(plr_digits=16)):
        assert lib.ssm_cascade_workspace_bytes(arr, 1, 0, 1, 0, 0, C.byref(bad)) == 0
    t = B.make_tuning(plr_digits=6)
    assert lib.ssm_cascade_workspace_bytes(arr, 1, 0, 2, 0, 0, C.byref(t)) == 0  # BF16
    assert "PLR" in lib.ssm_last_error().decode()
    assert lib.ssm_cascade_workspace_bytes(arr, 1, 0, 1, 1, 1, C.byref(t)) == 0  # backward
    t2 = B.make_tuning(plr_digits=6, launch=B.SSM_LAUNCH_PERSISTENT)
    assert lib.ssm_cascade_workspace_bytes(arr, 1, 0, 1, 0, 0, C.byref(t2)) == 0
    off = lib.ssm_cascade_workspace_bytes(arr, 1, 0, 1, 0, 0, None)
    for compute in (0, 1):  # FP64, FP32
        on = lib.ssm_cascade_workspace_bytes(arr, 1, 0, compute, 0, 0, C.byref(t))
        assert on > lib.ssm_cascade_workspace_bytes(arr, 1, 0, compute, 0, 0, None) > 0
    assert off > 0


def test_plr_ranks_rejects_on_host(lib):
    from paper_2411_17729_amd import binding as B
    r = (C.c_int32 * 32)()
    used = C.c_int32(0)
    assert lib.ssm_cascade_plr_ranks(None, 0, 0, r, 32, C.byref(used)) == B.SSM_E_NOT_PREPARED


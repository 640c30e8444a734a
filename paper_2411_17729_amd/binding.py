"""ctypes binding of the C ABI in include/ssm_cascade.h.

Argument marshalling only: every function here forwards to the entry point of
the same name in libssm_cascade.so and raises ``SSMError`` on a non-OK status.
Pointers are Python ints (e.g. ``tensor.data_ptr()``), streams are raw HIP
stream handles (``torch.cuda.current_stream().cuda_stream``).

torch is imported before the library is loaded, so the process maps one HIP
runtime (the one torch ships) and torch's streams and allocations are valid
handles for the library.
"""

from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (loads the HIP runtime the library links against)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libssm_cascade.so")

SSM_OK, SSM_E_INVALID, SSM_E_UNSUPPORTED, SSM_E_WORKSPACE, SSM_E_HIP, SSM_E_NOT_PREPARED, SSM_E_NUMERIC = range(7)
SSM_F64, SSM_F32, SSM_BF16 = 0, 1, 2
SSM_DISC_TRAPEZOID, SSM_DISC_GIVEN, SSM_DISC_ZOH = 0, 1, 2
SSM_LAUNCH_AUTO, SSM_LAUNCH_PER_STAGE, SSM_LAUNCH_PERSISTENT = 0, 1, 2
SSM_STAGE_AUTO, SSM_STAGE_TILED, SSM_STAGE_RESIDENT, SSM_STAGE_CHAIN = 0, 1, 2, 3

# kernel classes of ssm_cascade_timing_read
TIMING_STAGE, TIMING_ADJOINT, TIMING_REDUCE, TIMING_RECURSION, TIMING_PAIR, TIMING_FOLD = 0, 1, 2, 3, 4, 5
TIMING_PLR = 6


class SSMError(RuntimeError):
    def __init__(self, status, where, detail):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


class ssm_seq_desc(C.Structure):
    _fields_ = [
        ("m", C.c_int32), ("p", C.c_int32), ("q", C.c_int32), ("N", C.c_int32),
        ("L", C.c_int64), ("delta", C.c_double),
        ("param_set", C.c_int32), ("reserved", C.c_int32),
        ("u_offset", C.c_int64), ("y_offset", C.c_int64),
    ]


class ssm_params(C.Structure):
    _fields_ = [
        ("A", C.c_void_p), ("B", C.c_void_p), ("C", C.c_void_p), ("D", C.c_void_p),
        ("m", C.c_int32), ("p", C.c_int32), ("q", C.c_int32), ("reserved", C.c_int32),
    ]


class ssm_tuning(C.Structure):
    _fields_ = [("launch", C.c_int32), ("tile_rows", C.c_int32 * 4), ("stage_kernel", C.c_int32),
                ("input_stages", C.c_int32), ("chain_blocks", C.c_int32), ("pair_stages", C.c_int32),
                ("pair_blocks", C.c_int32), ("input_split", C.c_int32), ("state_bf16", C.c_int32),
                ("fold_stages", C.c_int32), ("spin_limit", C.c_int32), ("static_state", C.c_int32),
                ("final_state", C.c_int32), ("plr_digits", C.c_int32), ("min_padded_m", C.c_int32)]


class ssm_plan_info(C.Structure):
    _fields_ = [
        ("n_seq", C.c_int32), ("n_ops", C.c_int32), ("compute", C.c_int32), ("max_stage", C.c_int32),
        ("total_steps", C.c_int64), ("stage_flops", C.c_double), ("io_flops", C.c_double),
        ("stage_bytes", C.c_double), ("stage_launches", C.c_int64), ("launch", C.c_int32),
        ("stage_kernel", C.c_int32), ("input_stages", C.c_int32), ("tile_rows", C.c_int32 * 4),
        ("persistent_grid", C.c_int32),
        ("persistent_items", C.c_int64), ("pair_launches", C.c_int64), ("pair_bytes", C.c_double),
        ("pair_flops", C.c_double), ("state_dtype", C.c_int32), ("fold_stages", C.c_int32),
        ("fold_launches", C.c_int64), ("fold_bytes", C.c_double), ("fold_flops", C.c_double),
        ("plr_stages", C.c_int32), ("plr_reserved", C.c_int32), ("plr_flops", C.c_double),
        ("plr_dense_flops", C.c_double), ("lower_ops", C.c_int32), ("lower_reserved", C.c_int32),
    ]


def make_tuning(launch=SSM_LAUNCH_AUTO, tile_rows=(0, 0, 0, 0), stage_kernel=SSM_STAGE_AUTO,
                input_stages=0, chain_blocks=0, pair_stages=0, pair_blocks=0, input_split=0,
                state_bf16=0, fold_stages=0, spin_limit=0, static_state=0, final_state=0, plr_digits=0,
                min_padded_m=0):
    t = ssm_tuning()
    t.plr_digits = int(plr_digits)
    t.min_padded_m = int(min_padded_m)
    t.spin_limit = int(spin_limit)
    t.static_state = int(static_state)
    t.final_state = int(final_state)
    t.launch = int(launch)
    t.stage_kernel = int(stage_kernel)
    t.input_stages = int(input_stages)
    t.chain_blocks = int(chain_blocks)
    t.pair_stages = int(pair_stages)
    t.pair_blocks = int(pair_blocks)
    t.input_split = int(input_split)
    t.state_bf16 = int(state_bf16)
    t.fold_stages = int(fold_stages)
    for i, r in enumerate(tile_rows):
        t.tile_rows[i] = int(r)
    return t


_lib = None

EXPORTS = [
    "ssm_cascade_workspace_bytes", "ssm_cascade_prepare", "ssm_cascade_apply", "ssm_cascade_apply_x0",
    "ssm_cascade_backward", "ssm_cascade_param_grad_numel", "ssm_cascade_recursion",
    "ssm_cascade_get_power", "ssm_cascade_get_bbar", "ssm_cascade_plan_info",
    "ssm_cascade_timing_enable", "ssm_cascade_timing_read", "ssm_cascade_destroy",
    "ssm_cascade_graph_apply", "ssm_cascade_graph_backward", "ssm_cascade_graph_launch",
    "ssm_cascade_graph_destroy", "ssm_status_string", "ssm_last_error", "ssm_cascade_device_status",
    "ssm_cascade_apply_noalloc", "ssm_cascade_apply_state", "ssm_cascade_backward_x0",
    "ssm_cascade_plan_stages", "ssm_cascade_plr_ranks",
]


def load(path=LIB_PATH):
    """Load the library (once). Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2411_17729_amd.build.build()")
    lib = C.CDLL(path)
    vp, i32, i64, sz, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t, C.c_double
    P = C.POINTER
    lib.ssm_cascade_workspace_bytes.restype = sz
    lib.ssm_cascade_workspace_bytes.argtypes = [P(ssm_seq_desc), i32, i32, i32, i32, i32,
                                                P(ssm_tuning)]
    lib.ssm_cascade_prepare.restype = i32
    lib.ssm_cascade_prepare.argtypes = [P(ssm_seq_desc), i32, P(ssm_params), i32, i32, i32, i32,
                                        i32, P(ssm_tuning), vp, sz, vp, P(vp)]
    lib.ssm_cascade_graph_apply.restype = i32
    lib.ssm_cascade_graph_apply.argtypes = [vp, vp, i32, sz, vp, sz, vp, P(vp)]
    lib.ssm_cascade_graph_backward.restype = i32
    lib.ssm_cascade_graph_backward.argtypes = [vp, vp, i32, sz, vp, sz, vp, vp, sz, vp, P(vp)]
    lib.ssm_cascade_graph_launch.restype = i32
    lib.ssm_cascade_graph_launch.argtypes = [vp, vp]
    lib.ssm_cascade_graph_destroy.restype = i32
    lib.ssm_cascade_graph_destroy.argtypes = [vp]
    lib.ssm_cascade_apply.restype = i32
    lib.ssm_cascade_apply.argtypes = [vp, vp, i32, sz, vp, sz, vp]
    lib.ssm_cascade_plan_stages.restype = i32
    lib.ssm_cascade_plan_stages.argtypes = [vp, P(i32), i32]
    lib.ssm_cascade_plr_ranks.restype = i32
    lib.ssm_cascade_plr_ranks.argtypes = [vp, i32, i32, P(i32), i32, P(i32)]
    lib.ssm_cascade_backward_x0.restype = i32
    lib.ssm_cascade_backward_x0.argtypes = [vp, vp, i32, sz, vp, sz, vp, sz, vp, vp, sz, vp, sz, vp]
    lib.ssm_cascade_apply_state.restype = i32
    lib.ssm_cascade_apply_state.argtypes = [vp, vp, i32, sz, vp, sz, vp, sz, vp, sz, vp]
    lib.ssm_cascade_apply_noalloc.restype = i32
    lib.ssm_cascade_apply_noalloc.argtypes = [vp, vp, i32, sz, vp, sz, vp]
    lib.ssm_cascade_apply_x0.restype = i32
    lib.ssm_cascade_apply_x0.argtypes = [vp, vp, i32, sz, vp, sz, vp, sz, vp]
    lib.ssm_cascade_recursion.restype = i32
    lib.ssm_cascade_recursion.argtypes = [vp, vp, i32, sz, vp, sz, vp]
    lib.ssm_cascade_backward.restype = i32
    lib.ssm_cascade_backward.argtypes = [vp, vp, i32, sz, vp, sz, vp, vp, sz, vp]
    lib.ssm_cascade_param_grad_numel.restype = sz
    lib.ssm_cascade_param_grad_numel.argtypes = [vp]
    lib.ssm_cascade_get_power.restype = i32
    lib.ssm_cascade_get_power.argtypes = [vp, i32, i32, vp, vp]
    lib.ssm_cascade_get_bbar.restype = i32
    lib.ssm_cascade_get_bbar.argtypes = [vp, i32, vp, vp]
    lib.ssm_cascade_plan_info.restype = i32
    lib.ssm_cascade_plan_info.argtypes = [vp, P(ssm_plan_info)]
    lib.ssm_cascade_timing_enable.restype = i32
    lib.ssm_cascade_timing_enable.argtypes = [vp, i32]
    lib.ssm_cascade_timing_read.restype = i32
    lib.ssm_cascade_timing_read.argtypes = [vp, i32, P(i64), P(dbl)]
    lib.ssm_cascade_destroy.restype = i32
    lib.ssm_cascade_device_status.argtypes = [vp, vp]
    lib.ssm_cascade_device_status.restype = i32
    lib.ssm_cascade_destroy.argtypes = [vp]
    lib.ssm_status_string.restype = C.c_char_p
    lib.ssm_status_string.argtypes = [i32]
    lib.ssm_last_error.restype = C.c_char_p
    lib.ssm_last_error.argtypes = []
    _lib = lib
    return lib


def _check(status, where):
    if status != SSM_OK:
        lib = load()
        raise SSMError(status, where, lib.ssm_last_error().decode())


def ssm_status_string(status):
    return load().ssm_status_string(status).decode()


def ssm_last_error():
    return load().ssm_last_error().decode()


def _descs(descs):
    arr = (ssm_seq_desc * len(descs))()
    for i, d in enumerate(descs):
        arr[i] = d if isinstance(d, ssm_seq_desc) else ssm_seq_desc(**d)
    return arr


def ssm_cascade_workspace_bytes(descs, disc, compute, with_backward, ckpt_every=0, tuning=None):
    arr = _descs(descs)
    n = load().ssm_cascade_workspace_bytes(arr, len(descs), disc, compute, int(with_backward),
                                           ckpt_every, C.byref(tuning) if tuning is not None else None)
    if n == 0:
        raise SSMError(SSM_E_INVALID, "ssm_cascade_workspace_bytes", ssm_last_error())
    return n


def ssm_cascade_prepare(descs, params, disc, compute, with_backward, ckpt_every, tuning, ws_ptr,
                        ws_bytes, stream):
    arr = _descs(descs)
    parr = (ssm_params * len(params))()
    for i, p in enumerate(params):
        parr[i] = p if isinstance(p, ssm_params) else ssm_params(**p)
    plan = C.c_void_p()
    _check(load().ssm_cascade_prepare(arr, len(descs), parr, len(params), disc, compute,
                                      int(with_backward), ckpt_every,
                                      C.byref(tuning) if tuning is not None else None, ws_ptr,
                                      ws_bytes, stream, C.byref(plan)), "ssm_cascade_prepare")
    return plan.value


def ssm_cascade_apply(plan, u_ptr, u_dtype, u_numel, y_ptr, y_numel, stream):
    _check(load().ssm_cascade_apply(plan, u_ptr, u_dtype, u_numel, y_ptr, y_numel, stream),
           "ssm_cascade_apply")


def ssm_cascade_plan_stages(plan, n_seq):
    arr = (C.c_int32 * n_seq)()
    _check(load().ssm_cascade_plan_stages(plan, arr, n_seq), "ssm_cascade_plan_stages")
    return [int(v) for v in arr]


def ssm_cascade_plr_ranks(plan, op, k):
    """(ranks of the 32 rank-table slots of P_k of operator op, whether the apply
    runs that stage in PLR form)."""
    arr = (C.c_int32 * 32)()
    used = C.c_int32(0)
    _check(load().ssm_cascade_plr_ranks(plan, op, k, arr, 32, C.byref(used)), "ssm_cascade_plr_ranks")
    return [int(v) for v in arr], bool(used.value)


def ssm_cascade_backward_x0(plan, u_ptr, u_dtype, u_numel, x0_ptr, x0_numel, dy_ptr, dy_numel, du_ptr, dx0_ptr,
                            dx0_numel, grad_ptr, grad_numel, stream):
    _check(load().ssm_cascade_backward_x0(plan, u_ptr, u_dtype, u_numel, x0_ptr, x0_numel, dy_ptr, dy_numel, du_ptr,
                                          dx0_ptr, dx0_numel, grad_ptr, grad_numel, stream), "ssm_cascade_backward_x0")


def ssm_cascade_apply_state(plan, u_ptr, u_dtype, u_numel, x0_ptr, x0_numel, y_ptr, y_numel, xl_ptr, xl_numel,
                            stream):
    _check(load().ssm_cascade_apply_state(plan, u_ptr, u_dtype, u_numel, x0_ptr, x0_numel, y_ptr, y_numel,
                                          xl_ptr, xl_numel, stream), "ssm_cascade_apply_state")


def ssm_cascade_apply_noalloc(plan, u_ptr, u_dtype, u_numel, y_ptr, y_numel, stream):
    _check(load().ssm_cascade_apply_noalloc(plan, u_ptr, u_dtype, u_numel, y_ptr, y_numel, stream),
           "ssm_cascade_apply_noalloc")


def ssm_cascade_apply_x0(plan, u_ptr, u_dtype, u_numel, x0_ptr, x0_numel, y_ptr, y_numel, stream):
    _check(load().ssm_cascade_apply_x0(plan, u_ptr, u_dtype, u_numel, x0_ptr, x0_numel, y_ptr, y_numel,
                                       stream), "ssm_cascade_apply_x0")


def ssm_cascade_recursion(plan, u_ptr, u_dtype, u_numel, y_ptr, y_numel, stream):
    _check(load().ssm_cascade_recursion(plan, u_ptr, u_dtype, u_numel, y_ptr, y_numel, stream),
           "ssm_cascade_recursion")


def ssm_cascade_backward(plan, u_ptr, u_dtype, u_numel, dy_ptr, dy_numel, du_ptr, grad_ptr,
                         grad_numel, stream):
    _check(load().ssm_cascade_backward(plan, u_ptr, u_dtype, u_numel, dy_ptr, dy_numel, du_ptr,
                                       grad_ptr, grad_numel, stream), "ssm_cascade_backward")


def ssm_cascade_param_grad_numel(plan):
    return load().ssm_cascade_param_grad_numel(plan)


def ssm_cascade_get_power(plan, op, k, dst_ptr, stream):
    _check(load().ssm_cascade_get_power(plan, op, k, dst_ptr, stream), "ssm_cascade_get_power")


def ssm_cascade_get_bbar(plan, op, dst_ptr, stream):
    _check(load().ssm_cascade_get_bbar(plan, op, dst_ptr, stream), "ssm_cascade_get_bbar")


def ssm_cascade_plan_info(plan):
    info = ssm_plan_info()
    _check(load().ssm_cascade_plan_info(plan, C.byref(info)), "ssm_cascade_plan_info")
    out = {f: getattr(info, f) for f, _ in ssm_plan_info._fields_}
    out["tile_rows"] = list(info.tile_rows)
    return out


def ssm_cascade_timing_enable(plan, enable):
    _check(load().ssm_cascade_timing_enable(plan, int(enable)), "ssm_cascade_timing_enable")


def ssm_cascade_timing_read(plan, kind):
    n = C.c_int64()
    ms = C.c_double()
    _check(load().ssm_cascade_timing_read(plan, kind, C.byref(n), C.byref(ms)),
           "ssm_cascade_timing_read")
    return n.value, ms.value


def ssm_cascade_device_status(plan, stream):
    _check(_lib.ssm_cascade_device_status(plan, stream), "ssm_cascade_device_status")


def ssm_cascade_destroy(plan):
    _check(load().ssm_cascade_destroy(plan), "ssm_cascade_destroy")


def ssm_cascade_graph_apply(plan, u_ptr, u_dtype, u_numel, y_ptr, y_numel, stream):
    g = C.c_void_p()
    _check(load().ssm_cascade_graph_apply(plan, u_ptr, u_dtype, u_numel, y_ptr, y_numel, stream,
                                          C.byref(g)), "ssm_cascade_graph_apply")
    return g.value


def ssm_cascade_graph_backward(plan, u_ptr, u_dtype, u_numel, dy_ptr, dy_numel, du_ptr, grad_ptr,
                               grad_numel, stream):
    g = C.c_void_p()
    _check(load().ssm_cascade_graph_backward(plan, u_ptr, u_dtype, u_numel, dy_ptr, dy_numel,
                                             du_ptr, grad_ptr, grad_numel, stream, C.byref(g)),
           "ssm_cascade_graph_backward")
    return g.value


def ssm_cascade_graph_launch(graph, stream):
    _check(load().ssm_cascade_graph_launch(graph, stream), "ssm_cascade_graph_launch")


def ssm_cascade_graph_destroy(graph):
    _check(load().ssm_cascade_graph_destroy(graph), "ssm_cascade_graph_destroy")

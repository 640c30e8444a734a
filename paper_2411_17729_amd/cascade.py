"""PyTorch-facing wrapper of the fast-cascade library.

PyTorch provides device memory and streams; every arithmetic step of the
path runs in the HIP kernels of libssm_cascade.so, reached through
``binding``. There is no CPU fallback: without the built library or a GPU
these classes raise.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import binding as B

_DT = {"f64": B.SSM_F64, "f32": B.SSM_F32, "bf16": B.SSM_BF16}
_TORCH_DT = {B.SSM_F64: torch.float64, B.SSM_F32: torch.float32, B.SSM_BF16: torch.bfloat16}


def dtype_code(name):
    return _DT[name] if isinstance(name, str) else int(name)


@dataclass
class Layout:
    """Descriptors and packed-buffer sizes of a batch of sequences."""
    descs: List[B.ssm_seq_desc]
    u_numel: int
    y_numel: int


def make_layout(seqs: Sequence, sets_dims: Sequence) -> Layout:
    """Sequences back to back in u and y. ``seqs`` items need .param_set,
    .delta, .L, .N; ``sets_dims`` gives (m, p, q) per parameter set."""
    descs = []
    uo = yo = 0
    for s in seqs:
        m, p, q = sets_dims[s.param_set]
        d = B.ssm_seq_desc(m=m, p=p, q=q, N=int(s.N), L=int(s.L), delta=float(s.delta),
                           param_set=int(s.param_set), reserved=0, u_offset=uo, y_offset=yo)
        descs.append(d)
        uo += int(s.L) * p
        yo += int(s.L) * q
    return Layout(descs, uo, yo)


def _stream():
    return torch.cuda.current_stream().cuda_stream


class CascadePlan:
    """A prepared batch: discretized operators, their powers Abar^(2^k) in the
    compute type, and the workspace (a torch uint8 tensor) the library carves."""

    def __init__(self, layout: Layout, params: Sequence, disc: str = "trapezoid",
                 compute: str = "f32", with_backward: bool = False, ckpt_every: int = 0,
                 device="cuda", launch="auto", tile_rows=(0, 0, 0, 0), stage_kernel="auto",
                 input_stages=0, chain_blocks=0, pair_stages=0, pair_blocks=0, input_split=0,
                 state_bf16=0, fold_stages=0, spin_limit=0, static_state=0, final_state=0,
                 plr_digits=0, min_padded_m=0):
        if not torch.cuda.is_available():
            raise RuntimeError("the fast-cascade library needs a ROCm GPU")
        B.load()
        self.layout = layout
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.compute = dtype_code(compute)
        discs = {"trapezoid": B.SSM_DISC_TRAPEZOID, "given": B.SSM_DISC_GIVEN, "zoh": B.SSM_DISC_ZOH}
        if disc not in discs:
            raise ValueError(f"discretization {disc!r}: one of {sorted(discs)}")
        self.disc = discs[disc]
        self.state_dtype = torch.float64 if self.compute == B.SSM_F64 else torch.float32
        # parameters as contiguous FP64 device tensors (kept alive for prepare)
        self.params = []
        cparams = []
        for (A, Bm, Cm, D) in params:
            ts = [(x.detach() if isinstance(x, torch.Tensor) else
                   torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)))
                  .to(device=self.device, dtype=torch.float64).contiguous()
                  for x in (A, Bm, Cm, D)]
            self.params.append(ts)
            m, p, q = ts[0].shape[0], ts[1].shape[1], ts[2].shape[0]
            cparams.append(B.ssm_params(A=ts[0].data_ptr(), B=ts[1].data_ptr(), C=ts[2].data_ptr(),
                                        D=ts[3].data_ptr(), m=m, p=p, q=q, reserved=0))
        mode = {"auto": B.SSM_LAUNCH_AUTO, "per_stage": B.SSM_LAUNCH_PER_STAGE,
                "persistent": B.SSM_LAUNCH_PERSISTENT}[launch] if isinstance(launch, str) else int(launch)
        sk = {"auto": B.SSM_STAGE_AUTO, "tiled": B.SSM_STAGE_TILED,
              "resident": B.SSM_STAGE_RESIDENT, "chain": B.SSM_STAGE_CHAIN}[stage_kernel] \
            if isinstance(stage_kernel, str) else int(stage_kernel)
        self.tuning = B.make_tuning(mode, tile_rows, sk, input_stages, chain_blocks, pair_stages,
                                    pair_blocks, input_split, state_bf16, fold_stages, spin_limit,
                                    static_state, final_state, plr_digits, min_padded_m)
        nbytes = B.ssm_cascade_workspace_bytes(layout.descs, self.disc, self.compute,
                                               with_backward, ckpt_every, self.tuning)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) // 256 * 256
        self._cparams = cparams
        self._ckpt_every = ckpt_every
        self._nbytes = nbytes
        self.plan = B.ssm_cascade_prepare(layout.descs, cparams, self.disc, self.compute,
                                          with_backward, ckpt_every, self.tuning, self.ws_ptr,
                                          nbytes, _stream())
        self.with_backward = with_backward

    def prepare_again(self):
        """Runs ssm_cascade_prepare once more on this plan's parameters and
        workspace (the discretization, squarings and packing are recomputed in
        place, to the same values) and replaces the plan handle."""
        old = self.plan
        self.plan = B.ssm_cascade_prepare(self.layout.descs, self._cparams, self.disc, self.compute,
                                          self.with_backward, self._ckpt_every, self.tuning,
                                          self.ws_ptr, self._nbytes, _stream())
        B.ssm_cascade_destroy(old)

    # -- forward ---------------------------------------------------------
    def apply(self, u: torch.Tensor, out: Optional[torch.Tensor] = None,
              x0: Optional[torch.Tensor] = None) -> torch.Tensor:
        """y of every sequence; x0 (optional) holds x_{-1} of each sequence, packed."""
        u = self._check_u(u)
        if out is None:
            out = torch.empty(self.layout.y_numel, dtype=self.state_dtype, device=self.device)
        if x0 is None:
            B.ssm_cascade_apply(self.plan, u.data_ptr(), self._u_code(u), u.numel(), out.data_ptr(),
                                out.numel(), _stream())
        else:
            if x0.dtype != self.state_dtype or not x0.is_contiguous() or x0.device != self.device:
                raise ValueError("x0 must be a contiguous device tensor of the state dtype")
            B.ssm_cascade_apply_x0(self.plan, u.data_ptr(), self._u_code(u), u.numel(), x0.data_ptr(),
                                   x0.numel(), out.data_ptr(), out.numel(), _stream())
        return out

    def stages(self):
        """N of every sequence (after an automatic choice)."""
        return B.ssm_cascade_plan_stages(self.plan, len(self.layout.descs))

    def state_numel(self) -> int:
        """Entries of the packed per-sequence states (x0, x_last): m of each."""
        return sum(int(d.m) for d in self.layout.descs)

    def apply_state(self, u: torch.Tensor, x0: Optional[torch.Tensor] = None,
                    out: Optional[torch.Tensor] = None, x_last: Optional[torch.Tensor] = None):
        """One chunk of a stream: y from the initial states x0 (packed, or
        None for zero), and the states of the sequences' last rows (needs a
        plan made with final_state=1). Returns (y, x_last)."""
        u = self._check_u(u)
        if out is None:
            out = torch.empty(self.layout.y_numel, dtype=self.state_dtype, device=self.device)
        if x_last is None:
            x_last = torch.empty(self.state_numel(), dtype=self.state_dtype, device=self.device)
        for t in ((x0,) if x0 is not None else ()) + (x_last,):
            if t.dtype != self.state_dtype or not t.is_contiguous() or t.device != self.device:
                raise ValueError("x0 and x_last must be contiguous device tensors of the state dtype")
        B.ssm_cascade_apply_state(self.plan, u.data_ptr(), self._u_code(u), u.numel(),
                                  x0.data_ptr() if x0 is not None else None, x0.numel() if x0 is not None else 0,
                                  out.data_ptr(), out.numel(), x_last.data_ptr(), x_last.numel(), _stream())
        return out, x_last

    def apply_noalloc(self, u: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """apply() with the state buffers taken from the library's static
        device scratch: ``out`` must be given, nothing is allocated."""
        u = self._check_u(u)
        B.ssm_cascade_apply_noalloc(self.plan, u.data_ptr(), self._u_code(u), u.numel(), out.data_ptr(),
                                    out.numel(), _stream())
        return out

    def recursion(self, u: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        u = self._check_u(u)
        if out is None:
            out = torch.empty(self.layout.y_numel, dtype=self.state_dtype, device=self.device)
        B.ssm_cascade_recursion(self.plan, u.data_ptr(), self._u_code(u), u.numel(),
                                out.data_ptr(), out.numel(), _stream())
        return out

    # -- backward --------------------------------------------------------
    def backward(self, u: torch.Tensor, dy: torch.Tensor, want_du=True, want_params=True,
                 x0: Optional[torch.Tensor] = None, want_dx0=False):
        """Gradients of sum(dy * y) for y = apply(u) (from the packed initial
        states x0 when given). Returns (du, param grads), and dx0 third when
        want_dx0."""
        u = self._check_u(u)
        if dy.dtype != self.state_dtype or not dy.is_contiguous() or dy.device != self.device:
            raise ValueError("dy must be a contiguous device tensor of the state dtype")
        du = torch.empty(self.layout.u_numel, dtype=self.state_dtype, device=self.device) if want_du else None
        ng = B.ssm_cascade_param_grad_numel(self.plan)
        g = torch.empty(ng, dtype=torch.float64, device=self.device) if want_params else None
        if x0 is None and not want_dx0:
            B.ssm_cascade_backward(self.plan, u.data_ptr(), self._u_code(u), u.numel(), dy.data_ptr(),
                                   dy.numel(), du.data_ptr() if du is not None else None,
                                   g.data_ptr() if g is not None else None, ng if g is not None else 0,
                                   _stream())
            return du, (self.split_param_grads(g) if g is not None else None)
        if x0 is not None and (x0.dtype != self.state_dtype or not x0.is_contiguous() or x0.device != self.device):
            raise ValueError("x0 must be a contiguous device tensor of the state dtype")
        dx0 = torch.empty(self.state_numel(), dtype=self.state_dtype, device=self.device) if want_dx0 else None
        B.ssm_cascade_backward_x0(self.plan, u.data_ptr(), self._u_code(u), u.numel(),
                                  x0.data_ptr() if x0 is not None else None, x0.numel() if x0 is not None else 0,
                                  dy.data_ptr(), dy.numel(), du.data_ptr() if du is not None else None,
                                  dx0.data_ptr() if dx0 is not None else None, dx0.numel() if dx0 is not None else 0,
                                  g.data_ptr() if g is not None else None, ng if g is not None else 0, _stream())
        return du, (self.split_param_grads(g) if g is not None else None), dx0

    def split_param_grads(self, g):
        out = []
        off = 0
        for ts in self.params:
            m, p, q = ts[0].shape[0], ts[1].shape[1], ts[2].shape[0]
            parts = []
            for (r, c) in ((m, m), (m, p), (q, m), (q, p)):
                parts.append(g[off: off + r * c].view(r, c))
                off += r * c
            out.append(parts)
        return out

    # -- HIP graphs --------------------------------------------------------
    def graph_apply(self, u: torch.Tensor, y: torch.Tensor, stream: torch.cuda.Stream):
        """Captures apply(u) -> y on ``stream`` (not the default stream) into a
        graph; returns a handle for ``graph_launch``."""
        u = self._check_u(u)
        return B.ssm_cascade_graph_apply(self.plan, u.data_ptr(), self._u_code(u), u.numel(),
                                         y.data_ptr(), y.numel(), stream.cuda_stream)

    def graph_backward(self, u, dy, du, g, stream: torch.cuda.Stream):
        u = self._check_u(u)
        return B.ssm_cascade_graph_backward(
            self.plan, u.data_ptr(), self._u_code(u), u.numel(), dy.data_ptr(), dy.numel(),
            du.data_ptr() if du is not None else None, g.data_ptr() if g is not None else None,
            g.numel() if g is not None else 0, stream.cuda_stream)

    @staticmethod
    def graph_launch(graph, stream: torch.cuda.Stream):
        B.ssm_cascade_graph_launch(graph, stream.cuda_stream)

    @staticmethod
    def graph_destroy(graph):
        B.ssm_cascade_graph_destroy(graph)

    # -- inspection ------------------------------------------------------
    def power(self, op: int, k: int) -> torch.Tensor:
        m = self._op_m(op)
        out = torch.empty((m, m), dtype=torch.float64, device=self.device)
        B.ssm_cascade_get_power(self.plan, op, k, out.data_ptr(), _stream())
        return out

    def bbar(self, op: int, m: int, p: int) -> torch.Tensor:
        out = torch.empty((m, p), dtype=torch.float64, device=self.device)
        B.ssm_cascade_get_bbar(self.plan, op, out.data_ptr(), _stream())
        return out

    def info(self):
        return B.ssm_cascade_plan_info(self.plan)

    def plr_ranks(self, op: int, k: int):
        """(rank table of P_k of operator op in PLR form, whether the apply runs
        stage k of its padded size in that form)."""
        return B.ssm_cascade_plr_ranks(self.plan, op, k)

    def device_status(self):
        """Synchronizes the stream and raises SSMError (SSM_E_HIP) if the last
        persistent launch gave up waiting for the items it depends on."""
        B.ssm_cascade_device_status(self.plan, _stream())

    def timing(self, enable: bool):
        B.ssm_cascade_timing_enable(self.plan, enable)

    def timing_read(self, kind: int):
        return B.ssm_cascade_timing_read(self.plan, kind)

    def _op_m(self, op):
        # operators are numbered by first appearance of (param_set, delta)
        seen = []
        for d in self.layout.descs:
            key = (d.param_set, d.delta if self.disc != B.SSM_DISC_GIVEN else 0.0)
            if key not in seen:
                seen.append(key)
                if len(seen) - 1 == op:
                    return d.m
        raise IndexError(op)

    def _u_code(self, u):
        return {torch.float64: B.SSM_F64, torch.float32: B.SSM_F32, torch.bfloat16: B.SSM_BF16}[u.dtype]

    def _check_u(self, u):
        if u.device != self.device or not u.is_contiguous():
            raise ValueError("u must be a contiguous tensor on the plan's device")
        return u

    def close(self):
        if getattr(self, "plan", None):
            B.ssm_cascade_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_for_workload(wl, compute="f32", with_backward=False, ckpt_every=0, device="cuda",
                      launch="auto", tile_rows=(0, 0, 0, 0), stage_kernel="auto", input_stages=0,
                      chain_blocks=0, pair_stages=0, pair_blocks=0, input_split=0, state_bf16=0,
                      fold_stages=0, disc=None, spin_limit=0, static_state=0, final_state=0,
                      plr_digits=0, min_padded_m=0):
    """Builds the layout and plan of a ``workloads.Workload`` (discretization:
    the workload's, "given" or "trapezoid", unless ``disc`` names one)."""
    dims = [(ps.m, ps.p, ps.q) for ps in wl.sets]
    layout = make_layout(wl.seqs, dims)
    params = [(ps.A, ps.B, ps.C, ps.D) for ps in wl.sets]
    if disc is None:
        disc = "given" if wl.given else "trapezoid"
    return CascadePlan(layout, params, disc=disc, compute=compute,
                       with_backward=with_backward, ckpt_every=ckpt_every, device=device,
                       launch=launch, tile_rows=tile_rows, stage_kernel=stage_kernel,
                       input_stages=input_stages, chain_blocks=chain_blocks,
                       pair_stages=pair_stages, pair_blocks=pair_blocks, input_split=input_split,
                       state_bf16=state_bf16, fold_stages=fold_stages, spin_limit=spin_limit,
                       static_state=static_state, final_state=final_state, plr_digits=plr_digits,
                       min_padded_m=min_padded_m)


def pack_u(wl, dtype=torch.float32, device="cuda"):
    """All sequences' u back to back (matching ``make_layout``)."""
    flat = np.concatenate([np.asarray(s.u, dtype=np.float64).reshape(-1) for s in wl.seqs])
    return torch.as_tensor(flat, device=device).to(dtype).contiguous()


def unpack_y(wl, y):
    """Splits a packed output into per-sequence (L, q) numpy arrays."""
    y = y.detach().double().cpu().numpy()
    out = []
    off = 0
    for s in wl.seqs:
        q = wl.sets[s.param_set].q
        out.append(y[off: off + s.L * q].reshape(s.L, q))
        off += s.L * q
    return out


class CascadeFn(torch.autograd.Function):
    """y = cascade(u; A, B, C, D) with the hand-written adjoint cascade as its
    backward. ``cfg`` holds the static part (layout, discretization, compute
    type, checkpoint interval); the tensors are u followed by A, B, C, D of
    every parameter set (FP64)."""

    @staticmethod
    def forward(ctx, cfg, u, *params):
        layout, disc, compute, ckpt_every = cfg
        sets = [params[i:i + 4] for i in range(0, len(params), 4)]
        plan = CascadePlan(layout, sets, disc=disc, compute=compute, with_backward=True,
                           ckpt_every=ckpt_every, device=u.device)
        u_c = u.detach().contiguous()
        y = plan.apply(u_c)
        ctx.plan = plan
        ctx.u = u_c
        ctx.u_dtype = u.dtype
        ctx.n_sets = len(sets)
        return y

    @staticmethod
    def backward(ctx, dy):
        plan = ctx.plan
        need_u = ctx.needs_input_grad[1]
        need_p = any(ctx.needs_input_grad[2:])
        du, grads = plan.backward(ctx.u, dy.detach().to(plan.state_dtype).contiguous(),
                                  want_du=need_u, want_params=need_p)
        out = [None, du.to(ctx.u_dtype) if du is not None else None]
        for i in range(ctx.n_sets):
            out.extend(grads[i] if grads is not None else [None] * 4)
        return tuple(out)


def ssm_cascade(u, params, layout, disc="trapezoid", compute="f32", ckpt_every=0):
    """Differentiable fast cascade: u is the packed input (see make_layout),
    params a list of (A, B, C, D) FP64 tensors per parameter set."""
    flat = [t for ps in params for t in ps]
    return CascadeFn.apply((layout, disc, compute, ckpt_every), u, *flat)

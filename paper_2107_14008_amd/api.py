"""torch-facing helpers over the C ABI (device memory and streams only).

``ShortRange`` owns one library context: ``build`` plans the tree and task
lists for a particle set and uploads them, ``forward`` returns the
short-range accelerations, ``adjoint`` the gradient of sum_i w_i . a_i.
``ShortRangeForce`` exposes forward and adjoint as a torch.autograd.Function
(gradients with respect to positions and masses).
"""

from __future__ import annotations

import torch

from . import binding as B

_PREC = {"fp64": B.PMFMM_FP64, "fp32": B.PMFMM_FP32}
_TRUNC = {"exact": B.TRUNC_EXACT, "table": B.TRUNC_TABLE, "r2": B.TRUNC_R2}
_ROUND = {"nearest": B.ROUND_NEAREST, "floor": B.ROUND_FLOOR}


def _params(kw):
    out = dict(kw)
    if isinstance(out.get("precision"), str):
        out["precision"] = _PREC[out["precision"]]
    if isinstance(out.get("trunc"), str):
        out["trunc"] = _TRUNC[out["trunc"]]
    if isinstance(out.get("table_round"), str):
        out["table_round"] = _ROUND[out["table_round"]]
    return out


class ShortRange:
    """Short-range force of one periodic box (or a batch of boxes)."""

    def __init__(self, **params):
        self.ctx = B.Context(**_params(params))
        self.n = 0

    def build(self, pos: torch.Tensor, mass: torch.Tensor):
        if pos.device.type != "cuda":
            raise ValueError("pos must be a CUDA tensor")
        pos = pos.detach().to(torch.float64).contiguous()
        mass = mass.detach().to(torch.float64).contiguous()
        self.ctx.build(pos, mass, torch.cuda.current_stream(pos.device))
        self.n = pos.shape[0]
        self.device = pos.device
        return self

    def build_batch(self, per_box: list, counts, pos, mass):
        boxes = [B.make_params(**_params(p)) for p in per_box]
        pos = pos.detach().to(torch.float64).contiguous()
        mass = mass.detach().to(torch.float64).contiguous()
        self.ctx.build_batch(boxes, list(counts), pos, mass,
                             torch.cuda.current_stream(pos.device))
        self.n = pos.shape[0]
        self.device = pos.device
        return self

    def set_eval(self, **kw):
        self.ctx.set_eval(**_params(kw))

    def forward(self, out: torch.Tensor | None = None) -> torch.Tensor:
        if out is None:
            out = torch.empty((self.n, 3), dtype=torch.float64,
                              device=self.device)
        self.ctx.forward(out, torch.cuda.current_stream(self.device))
        return out

    def adjoint(self, w: torch.Tensor):
        w = w.detach().to(torch.float64).contiguous()
        gp = torch.empty((self.n, 3), dtype=torch.float64, device=self.device)
        gm = torch.empty((self.n,), dtype=torch.float64, device=self.device)
        self.ctx.adjoint(w, gp, gm, torch.cuda.current_stream(self.device))
        return gp, gm

    def lists(self):
        return self.ctx.lists()

    def timings(self):
        return self.ctx.timings()


def long_range_accel(pos: torch.Tensor, mass: torch.Tensor, n_pm: int, **params):
    """Accelerations (n, 3) float64 of the long-range (mesh) part of the
    split, on an n_pm^3 mesh; uses params box, r_s and G."""
    ctx = B.Context(**_params(params))
    out = torch.empty((pos.shape[0], 3), dtype=torch.float64, device=pos.device)
    ctx.long_range(n_pm, pos.contiguous(), mass.contiguous(), out,
                   torch.cuda.current_stream(pos.device))
    return out


class Simulation:
    """Kick-drift-kick leapfrog of one periodic box on the GPU: the
    short-range force of this library (the tree rebuilt every step) plus,
    with n_pm, the long-range mesh force; kicks and drifts are the library's
    kernels.  pos, vel: CUDA float64 (n, 3), updated in place."""

    def __init__(self, pos: torch.Tensor, vel: torch.Tensor, mass: torch.Tensor,
                 n_pm: int | None = None, **params):
        self.pos, self.vel = pos, vel
        self.mass = mass.detach().to(torch.float64).contiguous()
        self.n_pm = n_pm
        self.box = float(params.get("box", 100.0))
        self.sr = ShortRange(**params)
        self.acc = torch.empty_like(pos)
        self.long = torch.empty_like(pos) if n_pm else None
        self.stream = torch.cuda.current_stream(pos.device)
        self._force()

    def _force(self):
        self.sr.build(self.pos, self.mass)
        self.sr.forward(self.acc)
        if self.n_pm:
            self.sr.ctx.long_range(self.n_pm, self.pos, self.mass, self.long, self.stream)
            self.acc += self.long

    def step(self, dt: float, steps: int = 1):
        for _ in range(steps):
            B.kick(self.vel, self.acc, 0.5 * dt, self.stream)
            B.drift(self.pos, self.vel, dt, self.box, self.stream)
            self._force()
            B.kick(self.vel, self.acc, 0.5 * dt, self.stream)
        return self.pos, self.vel


def short_range_accel(pos: torch.Tensor, mass: torch.Tensor, **params):
    """Accelerations (n, 3) float64 of the truncated short-range force."""
    return ShortRange(**params).build(pos, mass).forward()


class ShortRangeForce(torch.autograd.Function):
    """acc = ShortRangeForce.apply(pos, mass, params_dict).

    The backward pass runs the library's adjoint kernels: for a cotangent w
    it returns (dL/dpos, dL/dmass) of L = sum_i w_i . acc_i, through the P2P
    pairs and, with the far field on, the transposed far-field operators
    (tree, lists and expansion centres of the forward build held fixed).
    """

    @staticmethod
    def forward(ctx, pos, mass, params):
        sr = ShortRange(**params).build(pos, mass)
        ctx.sr = sr
        return sr.forward().to(pos.dtype)

    @staticmethod
    def backward(ctx, grad_acc):
        gp, gm = ctx.sr.adjoint(grad_acc)
        return gp, gm, None

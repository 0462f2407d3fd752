"""Energy as a differentiable function of the coordinates.

`DPEnergy.apply(coords, model, nlist, precision, mode)` returns the total
energy (shape (1,), float64).  Its forward runs the fused forward of the
force step and keeps the activations on the list; its backward runs the
hand-written adjoint kernels (G and G' recomputed from the table, never
stored) and returns grad_output * dE/dx = -grad_output * F.  The virial of
the last backward is left on `nlist.last_virial` (a side output, not
differentiable).
"""
import torch

from . import api
from ._lib import COMPRESSED, FP32, check, lib


class DPEnergy(torch.autograd.Function):

    @staticmethod
    def forward(ctx, coords, model, nlist, precision=FP32, mode=COMPRESSED):
        x = coords.detach().contiguous()
        n = x.shape[0]
        E = torch.empty(1, dtype=torch.float64, device=x.device)
        check(lib.dp_energy_forward(model.h, nlist.h, n, api._ptr(x), mode, precision, api._ptr(E), None,
                                    api._stream()))
        ctx.save_for_backward(x)
        ctx.model, ctx.nlist, ctx.precision, ctx.mode = model, nlist, precision, mode
        return E

    @staticmethod
    def backward(ctx, grad_E):
        (x,) = ctx.saved_tensors
        n = x.shape[0]
        F = torch.empty((n, 3), dtype=torch.float64, device=x.device)
        W = torch.empty((3, 3), dtype=torch.float64, device=x.device)
        check(lib.dp_energy_backward(ctx.model.h, ctx.nlist.h, n, api._ptr(x), ctx.mode, ctx.precision,
                                     api._ptr(F), api._ptr(W), api._stream()))
        ctx.nlist.last_virial = W
        return -grad_E.reshape(()) * F, None, None, None, None


def energy(coords, model, nlist, precision=FP32, mode=COMPRESSED):
    return DPEnergy.apply(coords, model, nlist, precision, mode)

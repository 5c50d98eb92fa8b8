"""torch.autograd.Function over the library's batch Greeks entry points.

``ask, bid = bt_autograd(S0, sigma, R, k, spec, mode=...)`` prices every
option of ``spec`` -- bt_params records giving N, K, K2, T, payoff and
flags, as a PARAMS_DTYPE array or a uint8 CUDA tensor (``params_tensor``) --
with its S0, sigma, R and k replaced by the tensors, on torch's current
stream, through ``bt_price_adjoint_batch`` (mode="adjoint": the Greeks by a
reverse sweep through each tree that recomputes its levels from checkpoints
every ceil(sqrt(N+2)) levels) or ``bt_price_grad_batch`` (mode="forward":
the derivatives carried forward through the recursion; the default, faster
with four parameters).  The records are assembled on the GPU, the library
derives the trees, plans and prices them there, and nothing is copied to the
host, so the forward is stream-ordered and can be captured in a graph once
the library's workspace exists.  Its backward contracts the derivatives
d(ask, bid)/d(S0, sigma, R, k) returned by the same call with the incoming
gradients.  An option that fails (status other than BT_OK) gives NaN prices
and NaN gradients.  The arithmetic runs in the library's kernels; this
module only moves numbers between tensors and the C ABI.
"""
import numpy as np
import torch

from . import params_tensor, price_batch
from .workloads import GRAD_DTYPE, PARAMS_DTYPE, RESULT_DTYPE

# float64 columns of a bt_params record (72 bytes = 9 doubles)
_S0, _R, _SIGMA, _K = 0, 3, 4, 6
_NF = PARAMS_DTYPE.itemsize // 8


class BtPrice(torch.autograd.Function):
    @staticmethod
    def forward(ctx, S0, sigma, R, k, spec, max_N, mode="forward"):
        n = spec.numel() // PARAMS_DTYPE.itemsize
        P = spec.clone()
        f = P.view(torch.float64).view(n, _NF)
        f[:, _S0] = S0.detach().to(f)
        f[:, _SIGMA] = sigma.detach().to(f)
        f[:, _R] = R.detach().to(f)
        f[:, _K] = k.detach().to(f)
        out, g = price_batch(P, max_N, grad=True, mode=mode)
        res = out.view(torch.float64).view(n, RESULT_DTYPE.itemsize // 8)
        G = g.view(torch.float64).view(n, GRAD_DTYPE.itemsize // 8)
        ctx.save_for_backward(G)
        ctx.devices = (S0.device, sigma.device, R.device, k.device)
        # results on the device of S0 (the GPU's own when the inputs live there)
        return res[:, 0].to(S0.device, copy=True), res[:, 1].to(S0.device, copy=True)

    @staticmethod
    def backward(ctx, g_ask, g_bid):
        (G,) = ctx.saved_tensors
        Ga, Gb = G[:, :4], G[:, 4:]
        g_ask = torch.zeros(G.shape[0], dtype=G.dtype, device=G.device) if g_ask is None else g_ask
        g_bid = torch.zeros(G.shape[0], dtype=G.dtype, device=G.device) if g_bid is None else g_bid
        grads = Ga * g_ask.to(G.device)[:, None] + Gb * g_bid.to(G.device)[:, None]
        d = ctx.devices
        return (grads[:, 0].to(d[0]), grads[:, 1].to(d[1]), grads[:, 2].to(d[2]), grads[:, 3].to(d[3]),
                None, None, None)


def bt_autograd(S0, sigma, R, k, spec, max_N=None, mode="forward"):
    """ask, bid of the options of ``spec`` at (S0, sigma, R, k); ``max_N``
    bounds their N (taken from ``spec`` when it is a host array); ``mode``
    "forward" or "adjoint" picks how the Greeks are computed."""
    if mode not in ("forward", "adjoint"):
        raise ValueError("mode is 'forward' or 'adjoint'")
    if isinstance(spec, np.ndarray):
        if max_N is None:
            max_N = int(np.max(spec["N"]))
        spec = params_tensor(spec, device=S0.device if S0.is_cuda else "cuda")
    elif max_N is None:
        raise ValueError("max_N is required when spec is a device tensor")
    return BtPrice.apply(S0, sigma, R, k, spec, int(max_N), mode)


__all__ = ["BtPrice", "bt_autograd", "GRAD_DTYPE"]

"""torch.autograd.Function over the library's Greeks.

``ask, bid = bt_autograd(S0, sigma, R, k, book_params)`` prices every option
of ``book_params`` (a PARAMS_DTYPE array giving N, K, K2, T, payoff and
flags; its S0, sigma, R, k columns are replaced by the tensors) with the
Greeks kernels, and its backward contracts the returned derivatives
d(ask, bid)/d(S0, sigma, R, k) with the incoming gradients.  The arithmetic
runs in the library's kernels; this module only moves numbers between
tensors and the C ABI.
"""
import numpy as np
import torch

from . import Book
from .workloads import GRAD_DTYPE


class BtPrice(torch.autograd.Function):
    @staticmethod
    def forward(ctx, S0, sigma, R, k, book_params):
        p = np.array(book_params, copy=True)
        p["S0"] = S0.detach().cpu().double().numpy()
        p["sigma"] = sigma.detach().cpu().double().numpy()
        p["R"] = R.detach().cpu().double().numpy()
        p["k"] = k.detach().cpu().double().numpy()
        book = Book(p, greeks=True)
        try:
            book.price_grad()
            book.resolve_overflow(grad=True)
            res, g = book.results(), book.grads()
        finally:
            book.close()
        if np.any(res["status"] != 0):
            raise RuntimeError(f"pricing failed for options {np.nonzero(res['status'])[0][:8]}")
        dev = S0.device
        ask = torch.as_tensor(res["ask"], dtype=torch.float64, device=dev)
        bid = torch.as_tensor(res["bid"], dtype=torch.float64, device=dev)
        names = [f"{side}_{v}" for side in ("ask", "bid") for v in ("dS0", "dsigma", "dR", "dk")]
        G = torch.as_tensor(np.stack([g[n] for n in names], axis=1), dtype=torch.float64, device=dev)
        ctx.save_for_backward(G)
        return ask, bid

    @staticmethod
    def backward(ctx, g_ask, g_bid):
        (G,) = ctx.saved_tensors
        Ga, Gb = G[:, :4], G[:, 4:]
        g_ask = torch.zeros(G.shape[0], dtype=G.dtype, device=G.device) if g_ask is None else g_ask
        g_bid = torch.zeros(G.shape[0], dtype=G.dtype, device=G.device) if g_bid is None else g_bid
        grads = Ga * g_ask[:, None] + Gb * g_bid[:, None]
        return grads[:, 0], grads[:, 1], grads[:, 2], grads[:, 3], None


def bt_autograd(S0, sigma, R, k, book_params):
    return BtPrice.apply(S0, sigma, R, k, book_params)


__all__ = ["BtPrice", "bt_autograd", "GRAD_DTYPE"]

"""The log-likelihood as a differentiable torch function of the particle parameters.

`loglik(ctx, p, y_obs)` returns ll[n] (the Gaussian log-likelihood of Section 2.3.2
for every particle); it is differentiable with respect to the float parameter
tensors of `p` (phi_b, phi, z_cond, m, z_charg, log10_tau, c).  When any of them
requires a gradient the forward pass calls the library's reverse sweep
(`rjsmc_loglik_grad`), which returns ll and d ll_i / d theta_i from one launch; the
backward pass is then only the chain rule, ll_bar_i * d ll_i / d theta_i, since
particle i's likelihood depends on its own parameters alone.  Without a gradient
request the plain `rjsmc_loglik` launch runs.  The counts (kappa, lambda) are
discrete and the observed data are not differentiated.  FP64 contexts only (the
library rejects a gradient on an FP32 context).
"""
import torch

from . import binding as _B

FLOAT_KEYS = ("phi_b", "phi", "z_cond", "m", "z_charg", "log10_tau", "c")
_META_KEYS = ("layout", "n_per_sounding", "kappa", "lambda_")


class _LogLik(torch.autograd.Function):
    @staticmethod
    def forward(fctx, rctx, meta, y_obs, *vals):
        p = dict(meta)
        p.update(zip(FLOAT_KEYS, vals))
        if any(fctx.needs_input_grad[3:]):
            ll, g = rctx.loglik_grad(p, y_obs)
            fctx.save_for_backward(*[g[k] for k in FLOAT_KEYS])
        else:
            ll = rctx.loglik(p, y_obs)
        return ll

    @staticmethod
    def backward(fctx, ll_bar):
        grads = tuple(ll_bar * g if need else None
                      for g, need in zip(fctx.saved_tensors, fctx.needs_input_grad[3:]))
        return (None, None, None) + grads


def loglik(rctx, p, y_obs):
    """ll[n] of the device population `p` (dict of tensors, rows [R, n]) against the
    observed soundings y_obs [n_sound, n_gate], differentiable in FLOAT_KEYS."""
    if not isinstance(rctx, _B.Context):
        raise TypeError("loglik needs a binding.Context")
    meta = {k: p[k] for k in _META_KEYS if k in p}
    return _LogLik.apply(rctx, meta, y_obs, *[p[k] for k in FLOAT_KEYS])

"""Training objective and optimiser in float64 (oracle).

Test infrastructure only.

Sec. 4.2: the gradient of KL(p || q) is estimated from one sample per vertex
as -E[(p / q_hat) grad log q]. With w = p / q_hat supplied per training sample
(the MIS-weighted radiance over the sampling pdf, Sec. 5), that is the
gradient of the weighted negative log-likelihood
    L = (1/B) sum_j w_j * (-log q(dir_j | feat_j)),
which is what this module computes (reading: mean over the batch). Its
gradient is taken by float64 autograd of the literal forward; Adam follows
Kingma and Ba (the optimiser the paper uses with Libtorch, Sec. 5).

With the selection probability c (a network with 8K + 1 outputs) the loss
is the blend of Sec. 4.2, e KL(p || q_hat) + (1 - e) KL(p || q) with
q_hat = c q + (1 - c) p_fs, estimated the same way (``blended_nll``); the
BSDF pdf p_fs at each training direction is an input (the renderer's).
"""

import torch

from . import mlp, nasg

F64 = torch.float64


def weighted_nll(weights, feat, dirs, w, n_lobes, eps=0.0, bf16=False, isotropic=False):
    """L = mean_j w_j * (-log q(dir_j)) for one batch (scalar tensor)."""
    raw = mlp.forward(weights, feat, bf16=bf16)
    lobes = nasg.decode(raw, n_lobes, eps, isotropic)
    log_q = nasg.mixture_log_pdf(dirs, lobes)
    w = torch.as_tensor(w, dtype=F64)
    return (w * (-log_q)).mean()


def loss_and_grad(weights, feat, dirs, w, n_lobes, eps=0.0, bf16=False, isotropic=False):
    """(L, [dL/dW_l]) with the gradient from float64 autograd."""
    ws = [torch.as_tensor(W, dtype=F64).clone().requires_grad_(True) for W in weights]
    L = weighted_nll(ws, feat, dirs, w, n_lobes, eps, bf16, isotropic)
    grads = torch.autograd.grad(L, ws)
    return float(L.detach()), [g.detach() for g in grads]


def raw_output_grad(raw, dirs, w, n_lobes, eps=0.0, isotropic=False):
    """dL/d(raw outputs) [B, 8K] for the loss above, by autograd."""
    raw = torch.as_tensor(raw, dtype=F64).clone().requires_grad_(True)
    log_q = nasg.mixture_log_pdf(dirs, nasg.decode(raw, n_lobes, eps, isotropic))
    w = torch.as_tensor(w, dtype=F64)
    L = (w * (-log_q)).mean()
    (g,) = torch.autograd.grad(L, raw)
    return g.detach()


def weight_grad_from_raw_grad(weights, feat, g_raw, bf16=False):
    """[dL/dW_l] given dL/d(raw outputs): the MLP part of the chain rule, by
    autograd of sum(raw * g_raw) with g_raw held fixed."""
    ws = [torch.as_tensor(W, dtype=F64).clone().requires_grad_(True) for W in weights]
    raw = mlp.forward(ws, feat, bf16=bf16)
    s = (raw * torch.as_tensor(g_raw, dtype=F64)).sum()
    return [g.detach() for g in torch.autograd.grad(s, ws)]


def mis_pdf(q, c, pdf_bsdf):
    """q_hat = c q + (1 - c) p_fs: the learned distribution blended with the
    BSDF's by the selection probability (Sec. 4.2, "Selection Probability")."""
    return c * q + (1.0 - c) * pdf_bsdf


def blended_nll(weights, feat, dirs, w, pdf_bsdf, n_lobes, e=0.2, eps=0.0, bf16=False):
    """L = mean_j w_j * -(e log q_hat_j + (1 - e) log q_j) for one batch.

    Sec. 4.2: the loss blends e KL(p || q_hat) with (1 - e) KL(p || q); the
    one-sample estimate of each KL's gradient has the weight w = p / q_hat_s
    of the density the sample was drawn from (supplied), as for ``weighted_nll``.
    The network has 8K + 1 outputs; the last is the selection logit.
    """
    raw = mlp.forward(weights, feat, bf16=bf16)
    lobes = nasg.decode(raw, n_lobes, eps)
    log_q = nasg.mixture_log_pdf(dirs, lobes)
    c = nasg.selection(raw, n_lobes)
    q_hat = mis_pdf(torch.exp(log_q), c, torch.as_tensor(pdf_bsdf, dtype=F64))
    w = torch.as_tensor(w, dtype=F64)
    return (w * -(e * torch.log(q_hat) + (1.0 - e) * log_q)).mean()


def blended_loss_and_grad(weights, feat, dirs, w, pdf_bsdf, n_lobes, e=0.2, eps=0.0, bf16=False):
    """(L, [dL/dW_l]) of ``blended_nll`` by float64 autograd."""
    ws = [torch.as_tensor(W, dtype=F64).clone().requires_grad_(True) for W in weights]
    L = blended_nll(ws, feat, dirs, w, pdf_bsdf, n_lobes, e, eps, bf16)
    grads = torch.autograd.grad(L, ws)
    return float(L.detach()), [g.detach() for g in grads]


def blended_raw_output_grad(raw, dirs, w, pdf_bsdf, n_lobes, e=0.2, eps=0.0):
    """dL/d(raw outputs) [B, 8K + 1] for ``blended_nll``, by autograd."""
    raw = torch.as_tensor(raw, dtype=F64).clone().requires_grad_(True)
    log_q = nasg.mixture_log_pdf(dirs, nasg.decode(raw, n_lobes, eps))
    c = nasg.selection(raw, n_lobes)
    q_hat = mis_pdf(torch.exp(log_q), c, torch.as_tensor(pdf_bsdf, dtype=F64))
    w = torch.as_tensor(w, dtype=F64)
    L = (w * -(e * torch.log(q_hat) + (1.0 - e) * log_q)).mean()
    (g,) = torch.autograd.grad(L, raw)
    return g.detach()


def blend_ramp(frames_done, M=4, B=64):
    """b of Sec. 5 (progressive learning and sampling): 0 at the start, raised
    by 1/B after every M rendered images, capped at 1. The renderer samples
    the learned distribution with probability b c."""
    return min(1.0, (int(frames_done) // int(M)) / float(B))


def adam_step(param, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1), bias-corrected, no decay.

    `step` is the number of updates already taken; returns
    (param, m, v, step + 1) as new tensors.
    """
    t = step + 1
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return param - lr * m_hat / (torch.sqrt(v_hat) + eps), m, v, t

"""FP64 oracle of the training loss (Supplement "Loss Formulation",
Eq. eq:loss) and its gradient with respect to the rendered semantics and
depth.

TEST INFRASTRUCTURE ONLY (see the package docstring).

    L = lambda_s * L_sem(S_hat, S) + lambda_d * L_depth(D_hat, D)

with L_sem the cross-entropy of the class probabilities softmax(S_hat) against
the semantic pseudo-label and L_depth the squared error of the rendered depth
against the depth pseudo-label (the paper: lambda_s = 2, lambda_d = 0.05).

Reading (listed with the others in the design notes):
R20 Each term is a mean over the pixels that carry that label.  A semantic
    label outside [0, C) (e.g. -1) means "no label"; a depth label counts where
    it is finite and > 0.  A term with no labelled pixel contributes 0.
"""
from __future__ import annotations

import numpy as np

__all__ = ["fused_loss"]


def fused_loss(sem, depth, sem_label, depth_label, lambda_sem=2.0, lambda_depth=0.05):
    """sem [R, C] (rendered S_hat), depth [R], sem_label [R] int, depth_label [R].

    Returns loss, loss_sem, loss_depth (floats) and g_sem [R, C] = dL/dS_hat,
    g_depth [R] = dL/dD_hat, all in FP64."""
    sem = np.asarray(sem, np.float64)
    depth = np.asarray(depth, np.float64).reshape(-1)
    R, C = sem.shape
    lab = np.asarray(sem_label).reshape(-1).astype(np.int64)
    dl = np.asarray(depth_label, np.float64).reshape(-1)

    has_s = (lab >= 0) & (lab < C)
    n_s = int(has_s.sum())
    z = sem - sem.max(axis=1, keepdims=True)
    logp = z - np.log(np.exp(z).sum(axis=1, keepdims=True))          # log softmax
    probs = np.exp(logp)
    ce = np.zeros(R)
    ce[has_s] = -logp[has_s, lab[has_s]]
    loss_sem = ce.sum() / n_s if n_s else 0.0
    g_sem = np.zeros((R, C))
    if n_s:
        onehot = np.zeros((R, C))
        onehot[np.nonzero(has_s)[0], lab[has_s]] = 1.0
        g_sem[has_s] = (lambda_sem / n_s) * (probs[has_s] - onehot[has_s])

    has_d = np.isfinite(dl) & (dl > 0)
    n_d = int(has_d.sum())
    diff = np.where(has_d, depth - np.where(has_d, dl, 0.0), 0.0)
    loss_depth = float((diff ** 2).sum() / n_d) if n_d else 0.0
    g_depth = (lambda_depth / n_d) * 2.0 * diff if n_d else np.zeros(R)

    return dict(loss=lambda_sem * loss_sem + lambda_depth * loss_depth, loss_sem=float(loss_sem),
                loss_depth=loss_depth, g_sem=g_sem, g_depth=g_depth, n_sem=n_s, n_depth=n_d)

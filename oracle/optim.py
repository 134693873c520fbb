"""Adam (Kingma & Ba 2015, Algorithm 1) with projection onto a box (oracle).

The paper optimises the control coefficients with Adam (Sec. III-C); the
projection onto [lo, hi] keeps exchange amplitudes physical (J >= 0, below the
device ceiling).
"""
import numpy as np


def adam_project(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8,
                 grad_scale=1.0, lo=-np.inf, hi=np.inf, active=None):
    """One step t >= 1 on float64 arrays; returns (theta, m, v). Rows with
    active == False are left unchanged (state included)."""
    g = grad_scale * np.asarray(grad, dtype=float)
    m_new = beta1 * m + (1.0 - beta1) * g
    v_new = beta2 * v + (1.0 - beta2) * g * g
    mhat = m_new / (1.0 - beta1 ** t)
    vhat = v_new / (1.0 - beta2 ** t)
    th = theta - lr * mhat / (np.sqrt(vhat) + eps)
    th = np.clip(th, lo, hi)
    if active is not None:
        a = np.asarray(active, dtype=bool)[:, None]
        th = np.where(a, th, theta)
        m_new = np.where(a, m_new, m)
        v_new = np.where(a, v_new, v)
    return th, m_new, v_new

"""Adam update (oracle, FP64).

Test infrastructure: used only to check the GPU library.

Alg. 1 updates all Gaussian parameters with Adam using one learning rate
for every parameter type (Sec. 4.1).  The paper gives only the learning
rate; beta1, beta2 and eps take Adam's customary values (0.9, 0.999, 1e-8).
This is the textbook update with bias correction at step t >= 1.
"""
from __future__ import annotations

import numpy as np


def adam_step(param, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step; returns (param, m, v) as new FP64 arrays."""
    param = np.asarray(param, dtype=np.float64)
    grad = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * grad
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * grad * grad
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return param - lr * m_hat / (np.sqrt(v_hat) + eps), m, v

"""Adam (Kingma and Ba 2015, Algorithm 1), the optimiser the paper's training
inherits from 3DGS, in FP64.  Test infrastructure like the rest of this
package.

One step t >= 1 on parameters theta with gradient g and moments m, v:
  m <- beta1 m + (1 - beta1) g
  v <- beta2 v + (1 - beta2) g^2
  theta <- theta - lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps)
The paper names no hyperparameters; the 3DGS lineage trains with
beta1 = 0.9, beta2 = 0.999 and eps = 1e-15 and a learning rate per
parameter group (the caller's choice).
"""
from __future__ import annotations

import numpy as np

BETA1, BETA2, EPS = 0.9, 0.999, 1e-15


def step(theta, g, m, v, t, lr, beta1=BETA1, beta2=BETA2, eps=EPS):
    """Returns the new (theta, m, v) as FP64 arrays; t is the 1-based step."""
    theta = np.asarray(theta, np.float64)
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return theta - lr * m_hat / (np.sqrt(v_hat) + eps), m, v

"""Adam optimiser step in fp64 (test infrastructure only; never imported by the
product path).

Kingma and Ba, "Adam: A Method for Stochastic Optimization" (ICLR 2015),
Algorithm 1: with gradient g at step t (t >= 1),
    m_t = beta1 m_{t-1} + (1 - beta1) g
    v_t = beta2 v_{t-1} + (1 - beta2) g^2
    p_t = p_{t-1} - lr * (m_t / (1 - beta1^t)) / (sqrt(v_t / (1 - beta2^t)) + eps)
This is the optimiser step that follows the gradient computation in the
paper's training pipeline (its figure of the differentiable rendering
training loop, the parameter-update step).
"""
import numpy as np


def adam_step(p, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-15):
    """One step; returns (p_t, m_t, v_t) as new fp64 arrays."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return p - lr * m_hat / (np.sqrt(v_hat) + eps), m, v

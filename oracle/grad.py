"""O4 the coefficient-fit loss and its gradient;  O5 one Adam step.

Test infrastructure only (see the package docstring).

O4.  CLOMP learns s through a masked fully connected layer y' = A (mask * s)
(Methods, "Coefficients learning on OMP"), trained on the residual loss of the
coefficients-learning framework (Methods, "General idea of coefficients
learning": loss = L_r + sum_i w_i L_p_i; priors are not part of this path).
The scale of L_r is not printed; this oracle fixes
    L(s) = 1/2 || A (mask * s) - y ||_2^2
whose gradient, by the chain rule through the mask, is
    dL/ds = mask * A^T (A (mask * s) - y).

O5.  The optimiser is Adam as defined by Kingma and Ba (ICLR 2015), Algorithm 1,
with bias correction and epsilon added after the square root.  This is the
update torch.optim.Adam applies (up to rounding order).
"""

import numpy as np


def grad_fp64(x, mask, A, y):
    """Return (loss, grad, u) with u = A(mask*x) - y, loss = 1/2 u.u,
    grad = mask * A^T u.  All float64.  mask: boolean or 0/1 array of length n."""
    A = np.asarray(A, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    mk = np.asarray(mask).astype(bool).astype(np.float64)
    u = A @ (mk * x) - y
    loss = 0.5 * float(u @ u)
    grad = mk * (A.T @ u)
    return loss, grad, u


def adam_step_fp64(theta, g, m, v, step, lr, beta1, beta2, eps):
    """One Adam update at iteration number `step` (1-based).

    Returns new (theta, m, v).  Coordinates whose gradient and moments are all
    zero do not move (their update is lr * 0 / (0 + eps) = 0).
    """
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * (g * g)
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    theta = theta - lr * m_hat / (np.sqrt(v_hat) + eps)
    return theta, m, v

"""Adam step on the variational and kernel parameters xi, in float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper trains xi with Adam between natural-gradient updates of T
(Section 3.1; learning rates in Section S5).  This is one step of Kingma and
Ba's published algorithm, with bias correction, written in its own order:

  g' = g (or -g to maximise the bound F)
  m  <- beta1 m + (1 - beta1) g'
  v  <- beta2 v + (1 - beta2) g'^2
  m^ =  m / (1 - beta1^t),   v^ = v / (1 - beta2^t)
  p  <- p - lr m^ / (sqrt(v^) + eps)

for step t = 1, 2, ... and m = v = 0 before the first step.
"""
import numpy as np


def adam_step(p, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, ascend=False):
    """Returns (p, m, v) after step t (t >= 1); inputs are not modified."""
    p, g, m, v = (np.asarray(a, np.float64) for a in (p, g, m, v))
    gp = -g if ascend else g
    m = beta1 * m + (1.0 - beta1) * gp
    v = beta2 * v + (1.0 - beta2) * gp * gp
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v

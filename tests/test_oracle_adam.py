"""Pins of the Adam oracle (oracle/optim.py) against a library routine
(torch.optim.Adam in float64, including its maximize mode) and against the
closed form of the first step."""
import numpy as np
import pytest

from oracle import optim


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


@pytest.mark.parametrize("ascend", [False, True])
def test_adam_matches_torch(ascend):
    torch = pytest.importorskip("torch")
    g = _rng(1)
    p0 = g.standard_normal(37)
    grads = [g.standard_normal(37) * (0.1 + k) for k in range(6)]
    pt = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=3e-2, betas=(0.8, 0.95), eps=1e-6, maximize=ascend)
    p, m, v = p0.copy(), np.zeros(37), np.zeros(37)
    for t, gr in enumerate(grads, start=1):
        pt.grad = torch.tensor(gr, dtype=torch.float64)
        opt.step()
        p, m, v = optim.adam_step(p, gr, m, v, t, lr=3e-2, beta1=0.8, beta2=0.95, eps=1e-6,
                                  ascend=ascend)
        np.testing.assert_allclose(p, pt.detach().numpy(), rtol=1e-13, atol=1e-14)


def test_adam_first_step_closed_form():
    # m^ = g and v^ = g^2 after the first step: p - lr g / (|g| + eps)
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    p = np.array([1.0, 2.0, 3.0, 4.0])
    lr, eps = 0.1, 1e-8
    p1, m1, v1 = optim.adam_step(p, g, np.zeros(4), np.zeros(4), 1, lr=lr, eps=eps)
    np.testing.assert_allclose(p1, p - lr * g / (np.abs(g) + eps), rtol=1e-14)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-14)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-14)
    # ascending moves against the descent step
    p1a, _, _ = optim.adam_step(p, g, np.zeros(4), np.zeros(4), 1, lr=lr, eps=eps, ascend=True)
    np.testing.assert_allclose(p1a - p, -(p1 - p), rtol=1e-14)

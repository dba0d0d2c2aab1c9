"""Autograd plumbing of the deposit-misfit loss, on the CPU with a stand-in
runner whose loss and gradient are known in closed form (the GPU tests run
the real adjoint through the same function)."""
import numpy as np
import torch

from paper_2104_06784_amd.calibrate import _DepositLossFn


class _Quadratic:
    """L(mu, s) = 1/2 |mu - a|^2 + 3 (s - 1)^2 * sum(w mu)."""

    def __init__(self, a, w):
        self.a, self.w = a, w
        self.calls = []

    def evaluate(self, mu, s, need):
        self.calls.append(need)
        L = 0.5 * np.sum((mu - self.a) ** 2) + 3 * (s - 1) ** 2 * np.sum(self.w * mu)
        if not need:
            return L, None, None
        gmu = (mu - self.a) + 3 * (s - 1) ** 2 * self.w
        gs = 6 * (s - 1) * np.sum(self.w * mu)
        return L, gmu, gs


def test_backward_returns_the_runner_gradients():
    rng = np.random.default_rng(0)
    a, w = rng.random((5, 7)), rng.random((5, 7))
    r = _Quadratic(a, w)
    mu = torch.tensor(rng.random((5, 7)), requires_grad=True)
    s = torch.tensor(1.3, dtype=torch.float64, requires_grad=True)
    loss = _DepositLossFn.apply(mu, s, r, True)
    loss.backward()
    m = mu.detach().numpy()
    assert np.allclose(mu.grad.numpy(), (m - a) + 3 * 0.09 * w, rtol=1e-14)
    assert abs(float(s.grad) - 6 * 0.3 * np.sum(w * m)) <= 1e-12 * abs(float(s.grad))
    assert r.calls == [True]


def test_gradcheck_and_no_grad_path():
    rng = np.random.default_rng(1)
    r = _Quadratic(rng.random((3, 4)), rng.random((3, 4)))
    mu = torch.tensor(rng.random((3, 4)), requires_grad=True)
    s = torch.tensor(0.8, dtype=torch.float64, requires_grad=True)
    assert torch.autograd.gradcheck(lambda m, v: _DepositLossFn.apply(m, v, r, True), (mu, s))
    r.calls.clear()
    _DepositLossFn.apply(mu.detach(), s.detach(), r, False)
    assert r.calls == [False]

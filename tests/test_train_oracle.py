"""Pins of the TV and Adam oracles (CPU)."""
import numpy as np
import torch

from oracle import train as ot


def test_tv_of_constant_planes_is_zero():
    planes = [[np.full((5, 7, 3), 0.7) for _ in range(6)]]
    v, g = ot.tv_loss(planes)
    assert v == 0.0 and all((x == 0).all() for x in g[0])


def test_tv_of_a_ramp_is_its_squared_slope():
    """R = c j (+ e i): the mean squared difference is c^2 along a and e^2
    along b, for every plane."""
    c, e = 0.3, -1.1
    i, j = np.meshgrid(np.arange(6), np.arange(9), indexing="ij")
    R = np.repeat((c * j + e * i)[:, :, None], 4, axis=2)
    v, _ = ot.tv_loss([[R] * 6], weight=2.0)
    assert abs(v - 2.0 * 6 * (c * c + e * e)) < 1e-12


def test_tv_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    planes = [[rng.normal(size=(4, 6, 2)) for _ in range(6)], [rng.normal(size=(3, 5, 2)) for _ in range(6)]]
    _, g = ot.tv_loss(planes, weight=0.5)
    for l, p, idx in [(0, 0, (0, 0, 1)), (0, 3, (2, 5, 0)), (1, 5, (1, 2, 1)), (1, 1, (2, 4, 0))]:
        x = planes[l][p]
        old = x[idx]
        x[idx] = old + 1e-6
        fp, _ = ot.tv_loss(planes, 0.5)
        x[idx] = old - 1e-6
        fm, _ = ot.tv_loss(planes, 0.5)
        x[idx] = old
        assert abs((fp - fm) / 2e-6 - g[l][p][idx]) < 1e-7


def test_adam_matches_torch_optim_adam():
    rng = np.random.default_rng(1)
    p0 = rng.normal(size=50)
    grads = [rng.normal(size=50) for _ in range(5)]
    tp = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.999), eps=1e-15)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for k, g in enumerate(grads, start=1):
        tp.grad = torch.tensor(g)
        opt.step()
        p, m, v = ot.adam(p, g, m, v, 1e-2, k)
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=0, atol=1e-14)

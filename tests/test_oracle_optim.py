"""Pins of the oracle's cut-set Adam step (init/training appendix: only the
cut set's parameters are updated; the optimiser is Adam) against torch's own
Adam on the gathered rows, and the first step's closed form."""
import numpy as np

import oracle


def test_adam_cut_matches_torch_adam_on_the_gathered_rows():
    import torch
    rng = np.random.default_rng(71)
    n, w = 300, 7
    p0 = rng.normal(size=(n, w))
    idx = np.sort(rng.choice(n, 120, replace=False))
    lr, b1, b2, eps = 3e-3, 0.9, 0.999, 1e-8
    rows = torch.tensor(p0[idx], dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([rows], lr=lr, betas=(b1, b2), eps=eps)
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for t in range(1, 6):
        g = rng.normal(size=(len(idx), w)) * 10.0 ** rng.uniform(-4, 1, (len(idx), 1))
        rows.grad = torch.tensor(g)
        opt.step()
        p, m, v = oracle.adam_cut(p, m, v, g, idx, lr, b1, b2, eps, t)
        st = opt.state[rows]
        np.testing.assert_allclose(p[idx], rows.detach().numpy(), rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(m[idx], st["exp_avg"].numpy(), rtol=1e-12, atol=1e-300)
        np.testing.assert_allclose(v[idx], st["exp_avg_sq"].numpy(), rtol=1e-12, atol=1e-300)
    rest = np.setdiff1d(np.arange(n), idx)
    assert np.array_equal(p[rest], p0[rest]) and not m[rest].any() and not v[rest].any()


def test_adam_cut_first_step_moves_each_element_by_lr_against_its_gradient():
    # m = (1 - b1) g and v = (1 - b2) g^2, so the bias-corrected step is
    # lr g / (|g| + eps)
    rng = np.random.default_rng(72)
    p0 = rng.normal(size=(50, 3))
    idx = np.array([3, 10, 11, 40])
    g = rng.normal(size=(4, 3))
    lr, eps = 0.01, 1e-12
    p, m, v = oracle.adam_cut(p0, np.zeros_like(p0), np.zeros_like(p0), g, idx, lr, 0.9, 0.999, eps, 1)
    np.testing.assert_allclose(p[idx], p0[idx] - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m[idx], 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v[idx], 0.001 * g * g, rtol=1e-12)

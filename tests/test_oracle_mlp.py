"""Pins of the oracle's learned residual predictor: the published SplitMix64
test vector, BF16 rounding against an independent library conversion,
central finite differences of the exact loss, the first Adam step's closed
form, a zero head giving a zero shift, and input features of an affine
grid function."""
import numpy as np
import pytest
import torch

import meshgen as G
import oracle as O


def test_splitmix64_published_vector():
    # SplitMix64 seeded with 1234567: first five outputs (reference values
    # published with the generator's C implementation by S. Vigna)
    assert [O.splitmix64(1234567, i) for i in range(5)] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]


def test_bf16_matches_library_rne():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=2000).astype(np.float32) * 10.0 ** rng.integers(-6, 6, 2000),
                        np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 0.0, -0.0],
                                 np.float32)]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).float().numpy()
    assert np.array_equal(O.bf16(x).view(np.uint32), ref.view(np.uint32))


def test_sample_indices_uniform_and_in_range():
    idx = np.concatenate([O.sample_indices(9, s, 4096, 1000) for s in range(10)])
    assert idx.min() >= 0 and idx.max() < 1000
    counts = np.bincount(idx, minlength=1000)
    assert abs(counts.mean() - 40.96) < 1e-9 and counts.std() < 12


@pytest.mark.parametrize("dim", [2, 3])
def test_backward_finite_differences(dim):
    rng = np.random.default_rng(dim)
    kpad, kin = O.mlp_kpad(dim), O.mlp_kin(dim)
    P = O.mlp_init(dim, 5).astype(np.float64)
    P[P.size - 65 - 2 * 64 - 4096:] += rng.normal(0, 0.05, P.size - (P.size - 65 - 2 * 64 - 4096))
    B = 16
    z = np.zeros((B, kpad))
    z[:, :kin] = rng.normal(size=(B, kin))
    y = rng.normal(size=B)
    loss, g = O.mlp_loss_exact(dim, P, z, y)
    sel = rng.choice(P.size, 60, replace=False)
    h = 1e-6
    for k in sel:
        Pp, Pm = P.copy(), P.copy()
        Pp[k] += h
        Pm[k] -= h
        fd = (O.mlp_loss_exact(dim, Pp, z, y, False)[0] - O.mlp_loss_exact(dim, Pm, z, y, False)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g).max()), (k, fd, g[k])


@pytest.mark.parametrize("dim", [2, 3])
def test_rounded_backward_close_to_exact(dim):
    rng = np.random.default_rng(10 + dim)
    kpad, kin = O.mlp_kpad(dim), O.mlp_kin(dim)
    P = O.mlp_init(dim, 6)
    z = np.zeros((256, kpad), np.float32)
    z[:, :kin] = O.bf16(rng.normal(size=(256, kin)))
    y = rng.normal(size=256).astype(np.float32)
    l1, g1 = O.mlp_backward(dim, P, z, y, True)
    l0, g0 = O.mlp_backward(dim, P, z, y, False)
    assert abs(l1 - l0) <= 2e-2 * abs(l0)
    assert np.linalg.norm(g1 - g0) <= 3e-2 * np.linalg.norm(g0)
    rho, _ = O.mlp_forward(dim, P, z)
    assert abs(np.mean((rho.astype(np.float64) - y) ** 2) - l1) <= 1e-6 * l1


def test_zero_head_gives_zero_shift():
    dim = 2
    P = O.mlp_init(dim, 1)
    P[-65:] = 0.0          # W4 and b4
    z = O.bf16(np.random.default_rng(0).normal(size=(64, O.mlp_kpad(dim))))
    rho, _ = O.mlp_forward(dim, P, z)
    assert np.all(rho == 0.0)
    assert np.all(O.rho_quantize(rho) == 0)


def test_rho_quantize():
    r = np.array([0.5, 1.5, -0.5, -2.5, 2.49, 1e9, -1e9, np.nan], np.float32)
    assert O.rho_quantize(r).tolist() == [0, 2, 0, -2, 2, 32767, -32767, 0]


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(3)
    p = rng.normal(size=100).astype(np.float32)
    g = (rng.normal(size=100) * 10.0 ** rng.integers(-3, 3, 100)).astype(np.float32)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    p0 = p.copy()
    O.adam_step(p, m, v, g, 1, 1e-3)
    # m_hat = g, v_hat = g^2: the step is lr * g / (|g| + eps)
    expect = p0 - 1e-3 * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(p, expect, rtol=0, atol=1e-6)


@pytest.mark.parametrize("dim", [2, 3])
def test_features_of_affine_grid(dim):
    """x1' = 0.25 * i0 on the grid and a vertex at i = (5, 6, 7) + t: multilinear
    g gives 0.25 * (5 + t0), so input a is bf16(0.25 * (a0 - 1 - t0) * kappa)."""
    dims = (12, 11, 10) if dim == 3 else (12, 11, 1)
    g = O.make_grid(dim, dims, (0, 0, 0), (1, 1, 1))
    I = np.indices(dims[::-1])[::-1].reshape(3, -1)
    xhat = (0.25 * I[0]).astype(np.float32)
    t0 = 0.375
    pts = np.array([[5 + t0], [6.5], [7.25]][:dim], np.float32)
    gv = O.back_interp(pts, g, xhat)
    assert gv[0] == np.float32(0.25 * (5 + t0))
    z = O.mlp_features(pts, g, xhat, gv, 2.0)
    side2 = 4 if dim == 3 else 1
    expect = []
    for _ in range(side2):
        for _ in range(4):
            for a0 in range(4):
                expect.append(0.25 * (a0 - 1 - t0) * 2.0)
    expect += [t0 - 0.5, 0.0, -0.25][:dim]
    expect += [0.0] * (O.mlp_kpad(dim) - len(expect))
    assert z[0].tolist() == O.bf16(np.array(expect, np.float32)).tolist()


def test_training_reduces_loss():
    """A learnable target (a fixed random linear map of the inputs): Adam on
    the oracle network brings the loss well down."""
    dim = 2
    rng = np.random.default_rng(4)
    n = 4096
    kpad, kin = O.mlp_kpad(dim), O.mlp_kin(dim)
    z = np.zeros((n, kpad), np.float32)
    z[:, :kin] = O.bf16(rng.normal(size=(n, kin)))
    wt = rng.normal(size=kin) / np.sqrt(kin)
    y = (z[:, :kin] @ wt).astype(np.float32) * 3
    params, losses = O.train(dim, z, y, steps=150, batch=128, seed=7, lr=3e-3)
    assert np.mean(losses[-10:]) < 0.2 * np.mean(losses[:10])


def test_adam_constant_gradient_closed_form():
    """With the same gradient g at every step from m = v = 0, the moments are
    m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2 exactly, so the bias-corrected
    estimates are g and g^2 at every t and each step moves lr g / (|g| + eps).
    A bias correction with the wrong power of beta at any t >= 2 moves the
    parameters by a visibly different amount (1 + b1 = 1.9 times as far for
    1 - b1 in place of 1 - b1^2)."""
    rng = np.random.default_rng(8)
    p = rng.normal(size=64).astype(np.float32)
    g = (rng.normal(size=64) * 10.0 ** rng.integers(-2, 2, 64)).astype(np.float32)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    p0 = p.astype(np.float64)
    step = 1e-3 * g.astype(np.float64) / (np.abs(g.astype(np.float64)) + 1e-8)
    for t in range(1, 11):
        O.adam_step(p, m, v, g, t, 1e-3)
        np.testing.assert_allclose(p, p0 - t * step, rtol=0, atol=2e-6)
        np.testing.assert_allclose(m, (1 - 0.9 ** t) * g, rtol=2e-6, atol=0)
        np.testing.assert_allclose(v, (1 - 0.999 ** t) * g.astype(np.float64) ** 2, rtol=2e-5, atol=0)


def test_adam_three_steps_hand_derived():
    """Gradients 1, -2, 1/2 on one parameter from p = 1, lr 1e-3, b1 0.9,
    b2 0.999, eps 1e-8, worked by hand:
      t=1: m = 1/10, v = 1/1000; m_hat = 1, v_hat = 1
      t=2: m = 9/100 - 2/10 = -11/100; v = 999/10^6 + 4/1000 = 4999/10^6;
           m_hat = (-11/100) / (19/100) = -11/19; v_hat = 4999/1999
      t=3: m = -99/1000 + 5/100 = -49/1000; v = 999*4999/10^9 + 25/10^5
           = 5244001/10^9; m_hat = (-49/1000) / (271/1000) = -49/271;
           v_hat = 5244001/2997001
    and p_t = p_{t-1} - lr m_hat / (sqrt(v_hat) + eps).  A correction
    left at its t = 1 value would make steps 2 and 3 34 % and 57 % larger,
    far above the FP32 tolerance used."""
    from math import sqrt
    m_hat = [1.0, -11 / 19, -49 / 271]
    v_hat = [1.0, 4999 / 1999, 5244001 / 2997001]
    m_exp = [0.1, -0.11, -0.049]
    v_exp = [1e-3, 4999e-6, 5244001e-9]
    p = np.array([1.0], np.float32)
    m = np.zeros(1, np.float32)
    v = np.zeros(1, np.float32)
    ref = 1.0
    for t, gt in enumerate([1.0, -2.0, 0.5], start=1):
        O.adam_step(p, m, v, np.array([gt], np.float32), t, 1e-3)
        ref -= 1e-3 * m_hat[t - 1] / (sqrt(v_hat[t - 1]) + 1e-8)
        # b1 and b2 are FP32 (0.9f and 0.999f differ from 0.9 and 0.999 by
        # 2.4e-8 and 1.3e-8, i.e. up to 1.3e-5 relative in 1 - b2)
        assert abs(float(m[0]) - m_exp[t - 1]) <= 1e-6 * abs(m_exp[t - 1])
        assert abs(float(v[0]) - v_exp[t - 1]) <= 3e-5 * v_exp[t - 1]
        assert abs(float(p[0]) - ref) <= 2e-7, t

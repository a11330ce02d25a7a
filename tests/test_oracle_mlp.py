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

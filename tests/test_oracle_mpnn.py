"""Pins for the oracle of the learned smooth-vector network (CPU only).

  * Gradients: the hand-written backward pass equals central finite
    differences of the loss (float64, no bfloat16 rounding).
  * Features: closed forms on the Poisson matrix (interior rows: ratio 1,
    first two relaxation sweeps from ones leave 1; boundary rows lose 1/12 of
    their l1 weight per missing neighbour in the first sweep).
  * Aggregation: the row-normalised operator maps constants to constants.
  * bfloat16 rounding: values with known nearest-even results.
  * Degenerate network: zero weights give the constant bias.
"""
import numpy as np
import pytest

import oracle.mpnn as M
import workloads as W


def test_round_bf16_known_values():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 3.0e38, 1e-30])
    r = M.round_bf16(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                      # halfway, ties to even
    assert r[2] == 1.0 + 2 ** -6            # halfway between 1+2^-7 and 1+2^-6 -> even (1+2^-6)
    assert r[3] == -2.5
    assert np.isfinite(r[4])
    assert abs(r[5] - 1e-30) <= 1e-30 * 2 ** -8


def test_features_poisson_closed_form():
    N = 5
    A = W.poisson7(N)
    X, s = M.features(A)
    idx = np.arange(A.n)
    x, y, z = idx % N, (idx // N) % N, idx // (N * N)
    nb = sum(((c > 0).astype(int) + (c < N - 1).astype(int)) for c in (x, y, z))
    assert np.allclose(X[:, 0], 1.0)
    assert np.allclose(X[:, 1], np.log(6.0) / 4)
    assert np.allclose(X[:, 2], nb / 6.0)
    missing = 6 - nb
    assert np.allclose(X[:, 3], 1.0 - missing / (6.0 + nb))
    interior = nb == 6
    assert np.allclose(X[interior & (x > 1) & (x < N - 2) & (y > 1) & (y < N - 2) & (z > 1) & (z < N - 2), 4], 1.0)
    assert np.allclose(X[:, 5], 0.0)        # all couplings equal
    assert np.allclose(X[:, 6], nb / 6.0)
    assert np.allclose(s, nb)


def test_aggregation_maps_constants_to_constants():
    A = W.lognormal7(6, 3, ell=2.0)
    X, s = M.features(A)
    c = np.full((A.n, 3), 2.5)
    assert np.allclose(M._ahat(A, c, s), 2.5)


def test_zero_weights_give_bias():
    A = W.poisson7(4)
    theta = np.zeros(M.NPARAMS)
    theta[-1] = 0.75
    y, _ = M.forward(theta, A)
    assert np.allclose(y, 0.75)


@pytest.mark.parametrize("seed", [0, 1])
def test_backward_matches_finite_differences(seed):
    A = W.lognormal7(5, 11 + seed, ell=2.0)
    theta = M.init_params(seed)
    target = np.log(0.3 + W.uniform(50 + seed, A.n))
    loss, g = M.loss_and_grad(theta, A, target)
    rng = np.random.default_rng(seed)
    idx = rng.choice(M.NPARAMS, 80, replace=False)
    eps = 1e-6
    for i in idx:
        tp = theta.copy(); tp[i] += eps
        tm = theta.copy(); tm[i] -= eps
        lp = M.loss_and_grad(tp, A, target)[0]
        lm = M.loss_and_grad(tm, A, target)[0]
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (i, fd, g[i])

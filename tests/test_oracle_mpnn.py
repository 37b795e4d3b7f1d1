"""Pins for the oracle of the learned smooth-vector network (CPU only).

  * Gradients: the hand-written backward pass equals central finite
    differences of the loss (float64, no bfloat16 rounding).
  * Features: closed forms on the Poisson matrix (interior rows: ratio 1,
    first two relaxation sweeps from ones leave 1; boundary rows lose 1/12 of
    their l1 weight per missing neighbour in the first sweep).
  * Aggregation: the row-normalised operator maps constants to constants.
  * bfloat16 rounding: values with known nearest-even results.
  * Degenerate network: zero weights give the constant bias.
  * Forward pass with non-zero weights: equal to a node-by-node evaluation of
    the network's definition written in this file (exact rationals on a
    3-vertex path; scalar loops on a 2x2x2 graph in binary64 and with
    bfloat16 storage), with both ReLU branches active in both layers; copies
    of forward() with a planted mistake (swapped concatenation, missing ReLU,
    transposed weights, dropped aggregation) fail that comparison.
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


# --------------------------------------------------------------------------
# Independent pins of the forward pass with non-zero weights.  The expected
# outputs are evaluated here node by node from the network's definition
#   h1 = ReLU([X | Ahat X] W1 + b1), h2 = ReLU([h1 | Ahat h1] W2 + b2),
#   y = h2 wh + bh,  (Ahat X)_i = sum_{j != i} |a_ij| X_j / sum_{j != i} |a_ij|,
# with exact rationals (binary64 mode) or scalar loops with a bfloat16
# rounding written from its definition (bfloat16 mode); neither calls into
# oracle.mpnn beyond the function under test.

from fractions import Fraction as Fr  # noqa: E402
import inspect  # noqa: E402
import math  # noqa: E402

HID, F0 = 32, 8


def _pattern_params():
    """Small dyadic weights and biases with both signs (exact in bfloat16)."""
    W1 = [[Fr((a * 7 + b * 3) % 9 - 4, 8) for b in range(HID)] for a in range(2 * F0)]
    b1 = [Fr((b * 5) % 7 - 3, 4) for b in range(HID)]
    W2 = [[Fr((a * 5 + b * 11) % 13 - 6, 16) for b in range(HID)] for a in range(2 * HID)]
    b2 = [Fr((b * 3) % 5 - 2, 8) for b in range(HID)]
    wh = [Fr((b * 7) % 9 - 4, 8) for b in range(HID)]
    bh = Fr(1, 4)
    return W1, b1, W2, b2, wh, bh


def _flat(W1, b1, W2, b2, wh, bh):
    flat = [v for row in W1 for v in row] + b1 + [v for row in W2 for v in row] + b2 + wh + [bh]
    assert len(flat) == M.NPARAMS
    return np.array([float(v) for v in flat])


def _path3():
    """3-vertex path: [[2, -1, 0], [-1, 3, -1/2], [0, -1/2, 3/2]]."""
    rp = np.array([0, 2, 5, 7], np.int32)
    ci = np.array([0, 1, 0, 1, 2, 1, 2], np.int32)
    va = np.array([2.0, -1.0, -1.0, 3.0, -0.5, -0.5, 1.5])
    return W.CSR(3, rp, ci, va)


def _net_by_nodes(A, X, params, rnd=lambda v: v, swap=False):
    """The two-layer network evaluated one node at a time (Fractions or floats)."""
    W1, b1, W2, b2, wh, bh = params
    n = A.n
    nbrs = [[(int(A.col[k]), abs(A.val[k])) for k in range(A.row_ptr[i], A.row_ptr[i + 1])
             if A.col[k] != i] for i in range(n)]
    num = (lambda v: Fr(v)) if isinstance(bh, Fr) else (lambda v: float(v))
    s = [sum((num(a) for _, a in nbrs[i]), num(0)) for i in range(n)]

    def ahat(H):
        out = []
        for i in range(n):
            acc = [num(0)] * len(H[0])
            for j, a in nbrs[i]:
                acc = [acc[f] + num(a) * H[j][f] for f in range(len(acc))]
            out.append([rnd(v / s[i]) if s[i] != 0 else rnd(v) for v in acc])
        return out

    def dense(U, Wm, bias):
        return [[sum((U[i][a] * rnd(Wm[a][b]) for a in range(len(U[i]))), num(0)) + bias[b]
                 for b in range(len(bias))] for i in range(n)]

    X0 = [[rnd(num(v)) for v in row] for row in X]
    N0 = ahat(X0)
    U1 = [(N0[i] + X0[i]) if swap else (X0[i] + N0[i]) for i in range(n)]
    Z1 = dense(U1, W1, b1)
    h1 = [[rnd(max(v, num(0))) for v in row] for row in Z1]
    N1 = ahat(h1)
    U2 = [(N1[i] + h1[i]) if swap else (h1[i] + N1[i]) for i in range(n)]
    Z2 = dense(U2, W2, b2)
    h2 = [[rnd(max(v, num(0))) for v in row] for row in Z2]
    y = [sum((h2[i][b] * wh[b] for b in range(HID)), num(0)) + bh for i in range(n)]
    return y, Z1, Z2


def _features_pattern(n):
    return [[Fr((i * 3 + f * 5) % 7 - 3, 4) for f in range(F0)] for i in range(n)]


def _bf16_by_definition(v):
    """Nearest bfloat16 (8 significant bits, ties to even) of the binary32 value of v."""
    f = float(np.float32(v))
    if f == 0.0 or not math.isfinite(f):
        return f
    m, e = math.frexp(f)              # f = m 2^e, 0.5 <= |m| < 1
    q = round(m * 256.0)              # round half to even on an exact half
    return math.ldexp(q, e - 8)


def test_forward_matches_hand_evaluation_path3():
    """Exact rational evaluation on a 3-vertex path; both ReLU branches occur
    in both layers, and the evaluation with the two halves of the concatenation
    swapped differs, so a swapped, transposed or missing term shows."""
    A = _path3()
    P = _pattern_params()
    Xf = _features_pattern(A.n)
    y_ref, Z1, Z2 = _net_by_nodes(A, Xf, P)
    for Z in (Z1, Z2):
        flat = [v for row in Z for v in row]
        assert any(v > 0 for v in flat) and any(v < 0 for v in flat)
    y_swap, _, _ = _net_by_nodes(A, Xf, P, swap=True)
    assert max(abs(float(a - b)) for a, b in zip(y_ref, y_swap)) > 1e-2
    X = np.array([[float(v) for v in row] for row in Xf])
    y, _ = M.forward(_flat(*P), A, X=X)
    ref = np.array([float(v) for v in y_ref])
    assert np.max(np.abs(y - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref))), (y, ref)


@pytest.mark.parametrize("bf16", [False, True])
def test_forward_matches_node_loops_2x2x2(bf16):
    """Scalar per-node loops on a 2x2x2 log-normal diffusion graph with fixed
    non-zero weights, in binary64 and with bfloat16 storage of every dense
    product's inputs."""
    A = W.lognormal7(2, 5, ell=1.0)
    P = _pattern_params()
    Pf = tuple([[float(v) for v in row] for row in P[0]]), [float(v) for v in P[1]], \
        [[float(v) for v in row] for row in P[2]], [float(v) for v in P[3]], \
        [float(v) for v in P[4]], float(P[5])
    X = (W.uniform_pm1(33, A.n * F0) * 2.0).reshape(A.n, F0)
    rnd = _bf16_by_definition if bf16 else (lambda v: v)
    y_ref, Z1, Z2 = _net_by_nodes(A, X.tolist(), Pf, rnd=rnd)
    for Z in (Z1, Z2):
        flat = [v for row in Z for v in row]
        assert any(v > 0 for v in flat) and any(v < 0 for v in flat)
    y, _ = M.forward(_flat(*P), A, X=X, bf16=bf16)
    ref = np.array(y_ref)
    assert np.max(np.abs(y - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref))), (y, ref)


_PLANTED = {
    "concatenation order swapped": ("np.concatenate([X0, N0], axis=1)", "np.concatenate([N0, X0], axis=1)"),
    "second layer without ReLU": ("h2 = r(np.maximum(Z2, 0.0))", "h2 = r(Z2)"),
    "W1 read transposed": ('U1 @ r(p["W1"])', 'U1 @ r(p["W1"].reshape(-1).reshape(HID, 2 * F0).T)'),
    "W2 read transposed": ('U2 @ r(p["W2"])', 'U2 @ r(p["W2"].reshape(-1).reshape(HID, 2 * HID).T)'),
    "aggregation of the first layer dropped": ("N1 = r(_ahat(A, h1, s))", "N1 = r(h1 * 0.0)"),
}


@pytest.mark.parametrize("name", sorted(_PLANTED))
def test_planted_forward_mistakes_fail_the_pins(name):
    """A CPU copy of forward() with one planted mistake disagrees with the
    hand evaluation (so the pins above can catch that mistake)."""
    old, new = _PLANTED[name]
    src = inspect.getsource(M.forward)
    assert old in src
    ns = dict(vars(M))
    exec(compile(src.replace(old, new), "<planted>", "exec"), ns)
    bad = ns["forward"]
    A = _path3()
    P = _pattern_params()
    Xf = _features_pattern(A.n)
    ref = np.array([float(v) for v in _net_by_nodes(A, Xf, P)[0]])
    X = np.array([[float(v) for v in row] for row in Xf])
    y, _ = bad(_flat(*P), A, X=X)
    assert np.max(np.abs(y - ref)) > 1e-6

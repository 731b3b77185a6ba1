"""Pins of the learned-center oracle (CPU): finite differences, closed forms."""
import numpy as np

from oracle import mlp


def test_bf16_round_examples():
    # exactly representable values survive; 1 + 2^-8 is a tie rounded to even (1.0);
    # 1 + 3*2^-8 rounds up to 1 + 2^-6... checked against the bit definition
    v = np.array([1.0, 256.0, 257.0, 1 + 2 ** -8, 1 + 3 * 2 ** -9, -3.5], np.float64)
    r = mlp.bf16_round(v)
    assert r[0] == 1.0 and r[1] == 256.0
    assert r[2] == 256.0            # 257 is a tie between 256 and 258: even mantissa wins
    assert r[3] == 1.0              # tie, even
    assert r[4] == 1 + 2 ** -7      # 1 + 0.75 ulp rounds up
    assert r[5] == -3.5
    assert (mlp.from_bf16_bits(mlp.bf16_bits(v)) == r).all()


def test_featurize_counts():
    A, W, X = 0, 17, 22
    X3 = mlp.featurize([np.array([A, A, A, A], np.uint8),
                        np.array([A, W, A, W], np.uint8),
                        np.array([A, X, A, A], np.uint8),
                        np.array([A, A], np.uint8)])
    assert X3[0, 0] == 2 and X3[0].sum() == 2
    assert X3[1, 400 * A + 20 * W + A] == 1 and X3[1, 400 * W + 20 * A + W] == 1 and X3[1].sum() == 2
    assert X3[2].sum() == 0          # every window holds the X code (>= 20)
    assert X3[3].sum() == 0


def _tiny(rng):
    F, Hh, Em, N = 8, 4, 3, 6
    W1 = rng.normal(size=(F, Hh))
    b1 = rng.normal(size=Hh) * 0.1
    W2 = rng.normal(size=(Hh, Em))
    b2 = rng.normal(size=Em) * 0.1
    X = rng.integers(0, 4, size=(N, F)).astype(np.float64)
    t = rng.normal(size=N // 2)
    return X, W1, b1, W2, b2, t


def _loss(X, W1, b1, W2, b2, t):
    _, _, E = mlp.forward(X, W1, b1, W2, b2, round_h=False)
    return mlp.pair_loss(E, t)[0]


def test_grouped_loss_matches_central_differences():
    """The per-group mean-error term: dL/dE against FP64 central differences
    of the loss itself, and a hand case (two groups of two pairs)."""
    rng = np.random.default_rng(4)
    P, G, Em = 12, 3, 5
    E = rng.normal(size=(2 * P, Em))
    t = rng.normal(size=P)
    lam = 0.7
    L, dE = mlp.pair_loss(E, t, group=G, lam=lam)
    eps = 1e-6
    num = np.zeros_like(E)
    for idx in np.ndindex(E.shape):
        old = E[idx]
        E[idx] = old + eps
        lp = mlp.pair_loss(E, t, group=G, lam=lam)[0]
        E[idx] = old - eps
        lm = mlp.pair_loss(E, t, group=G, lam=lam)[0]
        E[idx] = old
        num[idx] = (lp - lm) / (2 * eps)
    assert np.abs(num - dE).max() <= 1e-6 * max(1.0, np.abs(num).max())
    # hand case: predictions 1, 2, 3, 4 (e_a = [p], e_b = [1]) against 0:
    # MSE = 30 / 4; group means 1.5 and 3.5, their mean square (2.25 + 12.25) / 2
    E2 = np.array([[1.0], [2.0], [3.0], [4.0], [1.0], [1.0], [1.0], [1.0]])
    L2, _ = mlp.pair_loss(E2, np.zeros(4), group=2, lam=2.0)
    assert abs(L2 - (7.5 + 2.0 * 7.25)) < 1e-12
    assert mlp.pair_loss(E2, np.zeros(4))[0] == 7.5


def test_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    X, W1, b1, W2, b2, t = _tiny(rng)
    z, h, E = mlp.forward(X, W1, b1, W2, b2, round_h=False)
    _, dE = mlp.pair_loss(E, t)
    dW1, db1, dW2, db2 = mlp.backward(X, W1, W2, z, h, dE, round_ops=False)
    eps = 1e-3
    for P, G in ((W1, dW1), (b1, db1), (W2, dW2), (b2, db2)):
        num = np.zeros_like(P)
        for idx in np.ndindex(P.shape):
            old = P[idx]
            P[idx] = old + eps
            lp = _loss(X, W1, b1, W2, b2, t)
            P[idx] = old - eps
            lm = _loss(X, W1, b1, W2, b2, t)
            P[idx] = old
            num[idx] = (lp - lm) / (2 * eps)
        # relu kinks are avoided: no pre-activation is within eps of 0 here
        assert np.abs(num - G).max() <= 1e-5 * max(1.0, np.abs(G).max()), (np.abs(num - G).max())


def test_adam_first_step_closed_form():
    # step 1: m_hat = g, v_hat = g^2, so the update is lr * g / (|g| + eps)
    g = np.array([0.5, -2.0, 1e-3])
    p, m, v = mlp.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.1)
    assert np.allclose(p, -0.1 * g / (np.abs(g) + 1e-8))
    # step 2 with the same gradient: still lr * sign(g) up to eps
    p2, _, _ = mlp.adam(p, g, m, v, 2, lr=0.1)
    assert np.allclose(p2 - p, -0.1 * np.sign(g), atol=1e-6)


def test_center_scores_and_topk():
    rng = np.random.default_rng(1)
    E = rng.normal(size=(30, 5))
    u = mlp.center_scores(E)
    brute = np.array([sum(E[i] @ E[j] for j in range(30) if j != i) for i in range(30)])
    assert np.allclose(u, brute)
    u2 = np.array([3.0, 5.0, 5.0, 1.0, 5.0])
    assert list(mlp.topk(u2, 3)) == [1, 2, 4]

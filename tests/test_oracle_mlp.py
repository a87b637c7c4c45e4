"""Pins of the numpy reference of the learned proposal: bfloat16 rounding on
known values, the backward pass against central finite differences (float64,
no rounding), and the quantised proposal's invariants."""
import numpy as np

from oracle import mlp


def test_bf16_round_known_values():
    one = np.float32(1.0)
    ulp = np.float32(2.0 ** -7)            # bf16 spacing at 1
    cases = {
        1.0: 1.0,
        1.0 + 2.0 ** -8: 1.0,              # exact tie -> even (1.0)
        1.0 + 3 * 2.0 ** -8: 1.0 + 2 * 2.0 ** -7,   # tie between 1+2^-7 and 1+2^-6 -> even
        1.0 + 2.0 ** -8 + 2.0 ** -20: 1.0 + 2.0 ** -7,  # above the tie -> up
        -2.5: -2.5,
    }
    for x, want in cases.items():
        got = float(mlp.bf16_round(np.float32(x)))
        assert abs(got - want) <= abs(want) * 1e-4, (x, got, want)
    # by bit patterns: below, at and above the half-way point, odd and even kept halves
    for bits, want in ((0x7F61B1E6, 0x7F620000), (0x3F808000, 0x3F800000), (0x3F818000, 0x3F820000),
                       (0x3F807FFF, 0x3F800000), (0xBF808001, 0xBF810000)):
        got = mlp.bf16_round(np.array([bits], np.uint32).view(np.float32)).view(np.uint32)[0]
        assert got == want, (hex(bits), hex(got), hex(want))
    # every result is representable: low 16 bits are zero
    r = mlp.bf16_round(np.random.default_rng(0).normal(size=1000).astype(np.float32))
    assert np.all((r.view(np.uint32) & 0xFFFF) == 0)
    assert float(mlp.bf16_round(one + ulp)) == float(one + ulp)


def _tiny(seed=0, N=5, M=7, H=6, Kp=8, Mp=8, B=4):
    rng = np.random.default_rng(seed)
    params = [rng.normal(size=(H, Kp)), rng.normal(size=H) * 0.1, rng.normal(size=(H, H)),
              rng.normal(size=H) * 0.1, rng.normal(size=(Mp, H)), rng.normal(size=Mp) * 0.1]
    params[0][:, N:] = 0
    params[4][M:] = 0
    X = rng.poisson(5, size=(B, N)).astype(np.int32)
    alpha = rng.exponential(1.0, size=(B, M))
    alpha[rng.random((B, M)) < 0.3] = 0
    alpha[:, 0] = 1.0
    return params, X, alpha, N, M


def test_backward_matches_finite_differences():
    params, X, alpha, N, M = _tiny()
    loss, grads, _ = mlp.loss_and_grads(params, X, alpha, N, M, mirror_bf16=False)
    h = 1e-6
    rng = np.random.default_rng(1)
    for i, P in enumerate(params):
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in P.shape)
            if i == 0 and idx[1] >= N or i in (4, 5) and idx[0] >= M:
                continue                      # padding: no gradient path, skipped
            old = P[idx]
            P[idx] = old + h
            lp, _, _ = mlp.loss_and_grads(params, X, alpha, N, M, mirror_bf16=False)
            P[idx] = old - h
            lm, _, _ = mlp.loss_and_grads(params, X, alpha, N, M, mirror_bf16=False)
            P[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grads[i][idx]) <= 1e-6 + 1e-5 * abs(fd), (i, idx, fd, grads[i][idx])


def test_padding_gets_no_gradient():
    params, X, alpha, N, M = _tiny()
    _, grads, _ = mlp.loss_and_grads(params, X, alpha, N, M)
    assert np.all(grads[0][:, N:] == 0)
    assert np.all(grads[4][M:] == 0) and np.all(grads[5][M:] == 0)


def test_softmax_support_and_quantisation():
    params, X, alpha, N, M = _tiny()
    fw = mlp.forward(params, X, alpha, N, M)
    q = fw["q"]
    assert np.allclose(q.sum(axis=1), 1.0)
    assert np.all(q[alpha == 0] == 0)
    Q = mlp.quantise(q, alpha > 0, M)
    assert np.all(Q[alpha > 0] >= 1) and np.all(Q[alpha == 0] == 0)
    assert np.all(Q.astype(np.uint64).sum(axis=1) < 2 ** 32)


def _hand_net():
    """N = 2 species, H = 2 hidden units, M = 3 reactions, small integer
    weights: the forward pass can be carried out by hand (see the test)."""
    W1 = np.array([[1.0, 1.0], [-1.0, 0.0]])
    b1 = np.array([0.0, 1.0])
    W2 = np.array([[1.0, 0.0], [1.0, 1.0]])
    b2 = np.array([0.0, -1.0])
    W3 = np.array([[1.0, 0.0], [0.0, 1.0], [1.0, -1.0]])
    b3 = np.array([0.0, 0.0, 0.0])
    return [W1, b1, W2, b2, W3, b3]


def test_forward_hand_computed_values():
    """X = (3, 0): f = (log 4, 0) = (2 ln 2, 0) (log1p of the counts);
    h1 = relu(W1 f + b1) = relu(2 ln 2, 1 - 2 ln 2) = (2 ln 2, 0);
    h2 = relu(W2 h1 + b2) = (2 ln 2, 2 ln 2 - 1);
    z = W3 h2 + b3 = (2 ln 2, 2 ln 2 - 1, 1), so exp(z) = (4, 4/e, e).
    With alpha = (1, 2, 3) every reaction is on the support:
    q = (4, 4/e, e) / (4 + 4/e + e); with alpha = (1, 0, 2) the second is
    masked: q = (4, 0, e) / (4 + e), and the loss with p = (1/3, 0, 2/3) is
    -(1/3) ln(4 / (4 + e)) - (2/3) ln(e / (4 + e)).  A transposed weight,
    log instead of log1p, a dropped bias or an unmasked softmax changes these.
    The features are rounded to float32 as the GPU computes them (relative
    6e-8), so the comparisons allow 1e-6."""
    e = np.e
    params = _hand_net()
    X = np.array([[3, 0], [3, 0]], dtype=np.int32)
    alpha = np.array([[1.0, 2.0, 3.0], [1.0, 0.0, 2.0]])
    fw = mlp.forward(params, X, alpha, N=2, M=3, mirror_bf16=False)
    l2 = 2 * np.log(2.0)
    tol = dict(rtol=0, atol=1e-6)
    assert np.allclose(fw["f"], [[l2, 0.0]] * 2, **tol)
    assert np.allclose(fw["h1"], [[l2, 0.0]] * 2, **tol)
    assert np.allclose(fw["h2"], [[l2, l2 - 1.0]] * 2, **tol)
    assert np.allclose(fw["z"], [[l2, l2 - 1.0, 1.0]] * 2, **tol)
    want = np.array([[4.0, 4.0 / e, e], [4.0, 0.0, e]])
    want /= want.sum(axis=1, keepdims=True)
    assert np.allclose(fw["q"], want, rtol=1e-6, atol=0)
    loss, _, _ = mlp.loss_and_grads(params, X[1:], alpha[1:], N=2, M=3, mirror_bf16=False)
    want_loss = -(np.log(4.0 / (4.0 + e)) + 2.0 * np.log(e / (4.0 + e))) / 3.0
    assert abs(loss - want_loss) <= 1e-6 * abs(want_loss)


def test_forward_hand_computed_bf16():
    """The same network with the GPU's bfloat16 storage: f = bf16(2 ln 2) =
    177/128 = 1.3828125 (2 ln 2 = 1.38629..., between the bf16 neighbours
    1.3828125 and 1.390625, nearer the first); then h1 = (a, 0),
    h2 = (a, a - 1) with a - 1 = 49/128 exactly representable, and
    z = (a, a - 1, 1)."""
    a = 177.0 / 128.0
    params = _hand_net()
    X = np.array([[3, 0]], dtype=np.int32)
    alpha = np.array([[1.0, 2.0, 3.0]])
    fw = mlp.forward(params, X, alpha, N=2, M=3, mirror_bf16=True)
    assert fw["f"][0, 0] == a and fw["f"][0, 1] == 0.0
    assert list(fw["h1"][0]) == [a, 0.0]
    assert list(fw["h2"][0]) == [a, a - 1.0]
    assert np.allclose(fw["z"][0], [a, a - 1.0, 1.0], rtol=0, atol=1e-15)
    ez = np.exp([a, a - 1.0, 1.0])
    assert np.allclose(fw["q"][0], ez / ez.sum(), rtol=1e-14, atol=0)


def _adam_closed(gs, lr, b1, b2, eps, w0=0.0):
    """Adam on one scalar with the textbook formulas in float64."""
    w, m, v = w0, 0.0, 0.0
    out = []
    for t, g in enumerate(gs, start=1):
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        w = w - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
        out.append((w, m, v))
    return out


def test_adam_two_steps_closed_forms():
    """Two Adam steps on scalars against values worked out by hand.

    * g = (1, -1), beta1 = 0.9, beta2 = 0.999: step 1 moves by lr / (1 + eps)
      (bias-corrected m_hat = 1, v_hat = 1); step 2 has
      m_hat = (0.09 - 0.1) / 0.19 = -1/19 and
      v_hat = (0.999 * 0.001 + 0.001) / (1 - 0.999^2) = 1, so it moves back
      by lr (1/19) / (1 + eps).
    * g = (1, 2): m_hat = 0.29 / 0.19 = 29/19,
      v_hat = (0.000999 + 0.004) / 0.001999 = 4.999 / 1.999.
    * a large eps (0.5) outside the square root: step 1 moves by
      lr * 3 / (3 + 0.5) for g = 3 (inside it would be lr * 3 / sqrt(9.5)).
    Tolerance: float32 rounding of a few operations (relative 1e-6)."""
    lr = 1e-2
    one = np.float32([0.0])
    w, m, v = one, one, one
    w1, m1, v1 = mlp.adam_step(w, m, v, np.float32([1.0]), 1, lr)
    assert abs(float(w1[0]) - (-lr / (1 + 1e-8))) <= 1e-6 * lr
    assert abs(float(m1[0]) - 0.1) <= 1e-6 * 0.1 and abs(float(v1[0]) - 0.001) <= 1e-4 * 0.001
    w2, m2, v2 = mlp.adam_step(w1, m1, v1, np.float32([-1.0]), 2, lr)
    assert abs(float(w2[0]) - (-lr + lr / 19.0)) <= 2e-6 * lr
    assert abs(float(m2[0]) - (-0.01)) <= 1e-5 * 0.01
    # g = (1, 2)
    w1, m1, v1 = mlp.adam_step(one, one, one, np.float32([1.0]), 1, lr)
    w2, _, _ = mlp.adam_step(w1, m1, v1, np.float32([2.0]), 2, lr)
    want = -lr - lr * (29.0 / 19.0) / np.sqrt(4.999 / 1.999)
    assert abs(float(w2[0]) - want) <= 2e-6 * lr
    # eps outside the square root
    w1, _, _ = mlp.adam_step(one, one, one, np.float32([3.0]), 1, lr, eps=0.5)
    assert abs(float(w1[0]) - (-lr * 3.0 / 3.5)) <= 1e-6 * lr
    # the same sequences against the float64 textbook recursion, on a vector
    rng = np.random.default_rng(7)
    g = rng.normal(size=(5, 64)).astype(np.float32)
    w = rng.normal(size=64).astype(np.float32)
    m = np.zeros(64, np.float32)
    v = np.zeros(64, np.float32)
    f32 = lambda x: float(np.float32(x))        # the optimizer's constants are float32
    ref = [_adam_closed(g[:, i].astype(np.float64), f32(lr), f32(0.9), f32(0.999), f32(1e-8),
                        w0=float(w[i])) for i in range(64)]
    ga = None
    for t in range(5):
        w, m, v = mlp.adam_step(w, m, v, g[t], t + 1, lr)
        rw = np.array([r[t][0] for r in ref])
        rm = np.array([r[t][1] for r in ref])
        rv = np.array([r[t][2] for r in ref])
        # m is a sum of terms of both signs: its rounding error scales with the
        # same recursion run on |g| (ga), not with |m| itself
        ga = ga * 0.9 + 0.1 * np.abs(g[t]) if t else 0.1 * np.abs(g[t])
        assert np.all(np.abs(w - rw) <= 1e-6 * np.maximum(1.0, np.abs(rw)))
        assert np.all(np.abs(m - rm) <= 1e-6 * ga)
        assert np.all(np.abs(v - rv) <= 1e-6 * np.abs(rv))


def test_adam_is_float32_arithmetic():
    """Every result is a float32 and each stage is rounded: the update of a
    weight whose step is below half an ulp leaves it unchanged."""
    w = np.float32([1.0e4])
    w1, m1, v1 = mlp.adam_step(w, np.float32([0]), np.float32([0]), np.float32([1.0]), 1, 1e-5)
    assert w1.dtype == np.float32 and m1.dtype == np.float32 and v1.dtype == np.float32
    assert w1[0] == np.float32(1.0e4)          # 1e-5 is below half an ulp of 1e4 (~4.9e-4)


def test_pins_catch_planted_mistakes(monkeypatch):
    """Plausible mistakes planted in the oracle fail the hand-computed pins."""
    e = np.e
    X = np.array([[3, 0]], dtype=np.int32)
    alpha = np.array([[1.0, 0.0, 2.0]])
    want = np.array([4.0, 0.0, e]) / (4.0 + e)

    def q_of(params):
        return mlp.forward(params, X, alpha, N=2, M=3, mirror_bf16=False)["q"][0]

    assert np.allclose(q_of(_hand_net()), want, rtol=1e-6)
    transposed = _hand_net()
    transposed[0] = transposed[0].T.copy()
    assert not np.allclose(q_of(transposed), want, rtol=1e-3)
    no_bias = _hand_net()
    no_bias[3] = np.zeros(2)
    assert not np.allclose(q_of(no_bias), want, rtol=1e-3)
    with monkeypatch.context() as mp:
        mp.setattr(mlp, "features", lambda X, N, Kp, mirror_bf16=True: np.log(
            np.maximum(np.asarray(X, np.float64), 1.0)))
        assert not np.allclose(q_of(_hand_net()), want, rtol=1e-3)
    unmasked = mlp.forward(_hand_net(), X, np.array([[1.0, 1e-30, 2.0]]), N=2, M=3,
                           mirror_bf16=False)["q"][0]
    assert not np.allclose(unmasked, want, rtol=1e-3)     # a tiny propensity is on the support

    # Adam: no bias correction, eps inside the square root, betas swapped
    one = np.float32([0.0])
    good = mlp.adam_step(one, one, one, np.float32([3.0]), 1, 1e-2, eps=0.5)[0][0]
    assert abs(good - (-1e-2 * 3.0 / 3.5)) <= 1e-8

    def no_correction(w, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        m_t = beta1 * m + (1 - beta1) * g
        v_t = beta2 * v + (1 - beta2) * g * g
        return w - lr * m_t / (np.sqrt(v_t) + eps), m_t, v_t

    def eps_inside(w, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        m_t = beta1 * m + (1 - beta1) * g
        v_t = beta2 * v + (1 - beta2) * g * g
        return w - lr * (m_t / (1 - beta1 ** t)) / np.sqrt(v_t / (1 - beta2 ** t) + eps), m_t, v_t

    def swapped(w, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        return mlp.adam_step(w, m, v, g, t, lr, beta1=1 - beta1, beta2=beta2, eps=eps)

    for bad in (no_correction, eps_inside, swapped):
        w1 = bad(one, one, one, np.float32([3.0]), 1, 1e-2, eps=0.5)[0][0]
        w1b, m1b, v1b = bad(one, one, one, np.float32([1.0]), 1, 1e-2)
        w2b = bad(w1b, m1b, v1b, np.float32([-1.0]), 2, 1e-2)[0][0]
        hit1 = abs(w1 - (-1e-2 * 3.0 / 3.5)) > 1e-8
        hit2 = abs(w2b - (-1e-2 + 1e-2 / 19.0)) > 2e-8
        assert hit1 or hit2, bad.__name__

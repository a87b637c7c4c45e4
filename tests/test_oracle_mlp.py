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

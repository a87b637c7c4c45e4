"""GPU tests of the learned-proposal path against the CPU oracle.

* MFMA GEMM (all operand layouts) against float64 products of the same BF16
  values;
* mass-action propensities and the SSA jump chain: bit-exact;
* MLP forward: ||q_gpu - q_cpu|| / ||q_cpu|| <= 1e-2 with the same BF16
  weights and inputs, also per row (relative L1) and per element above 1e-4;
  Q exactly the quantisation of the GPU's q;
* proposal selection: bit-exact against the oracle fed the GPU's Q;
* gradients of one training step within 2e-2 of the CPU backward, norm-wise
  and element by element against each tensor's scale;
* the Adam step (lr > 0, t = 1 and 2): masters, moments and BF16 copies
  bit-exact against the oracle's float32 Adam fed the GPU's gradients;
* training raises the per-trial acceptance over uniform AR; the learned
  selections follow alpha_j / alpha_0 (chi-square against the exact law);
* checkpoint / resume reproduces the weights bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import laws, mlp as omlp
from paper_1404_0027_amd import arsel, learned, workloads

pytestmark = pytest.mark.gpu


def _bf16(shape, seed):
    g = torch.Generator().manual_seed(seed)
    return torch.randn(*shape, generator=g).to(torch.bfloat16)


@pytest.mark.parametrize("shape", [(100, 70, 75), (256, 136, 96), (72, 64, 520)])
@pytest.mark.parametrize("akc,bkc", [(True, True), (True, False), (False, True), (False, False)])
def test_gemm_layouts(gpu, akc, bkc, shape):
    """Ragged edges (scalar loads), aligned tiles (16-byte loads) and a long K."""
    M, N, K = shape
    A = _bf16((M, K) if akc else (K, M), 1)
    B = _bf16((N, K) if bkc else (K, N), 2)
    bias = torch.randn(N, generator=torch.Generator().manual_seed(3))
    C = arsel.gemm_bf16(A.cuda(), K if akc else M, akc, B.cuda(), K if bkc else N, bkc, M, N, K,
                        bias=bias.cuda(), relu=True)
    a = A.float().numpy().astype(np.float64)
    b = B.float().numpy().astype(np.float64)
    a = a if akc else a.T
    b = b if bkc else b.T
    ref = np.maximum(a @ b.T + bias.numpy(), 0.0)
    got = C.cpu().numpy()
    assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)


def _states(net, R, steps, seed=5):
    X0 = workloads.poisson_counts(N=net.N, R=R, seed=seed)
    Xf, rec, _ = oracle.ssa_chain(net, X0, seed=11, step0=0, steps=steps, rec_from=0, threads=8)
    return rec.reshape(-1, net.N)


def test_propensities_bit_exact(gpu):
    net = workloads.mass_action_network()
    X = workloads.poisson_counts(N=net.N, R=64, seed=9)
    X[:8] *= 700                                     # counts whose products exceed 2^24
    dn = learned.DeviceNetwork(net)
    a = dn.propensities(torch.from_numpy(X).cuda()).cpu().numpy()
    ref = oracle.propensities(net, X)
    assert np.array_equal(a.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("N,M,R,steps", [(64, 100, 40, 200), (641, 1029, 8, 120)])
def test_ssa_chain_bit_exact(gpu, N, M, R, steps):
    net = workloads.mass_action_network(N=N, M=M, seed=4)
    X0 = workloads.poisson_counts(N=N, R=R, seed=5)
    dn = learned.DeviceNetwork(net)
    X = torch.from_numpy(X0).cuda()
    rec, fired = dn.chain(X, seed=3, step0=17, steps=steps, record_from=20, want_fired=True)
    Xo, reco, firedo = oracle.ssa_chain(net, X0, seed=3, step0=17, steps=steps, rec_from=20,
                                        threads=8)
    assert np.array_equal(fired.cpu().numpy(), firedo)
    assert np.array_equal(rec.cpu().numpy(), reco)
    assert np.array_equal(X.cpu().numpy(), Xo)


@pytest.fixture(scope="module")
def net_and_data(gpu):
    net = workloads.mass_action_network()
    dn = learned.DeviceNetwork(net)
    X0 = torch.from_numpy(workloads.poisson_counts(N=net.N, R=256, seed=21)).cuda()
    dn.chain(X0, seed=1, step0=0, steps=200)                       # burn-in
    rec, _ = dn.chain(X0, seed=1, step0=200, steps=200, record_from=0)
    X = rec.reshape(-1, net.N).contiguous()
    alpha = dn.propensities(X)
    return net, dn, X, alpha


def _params_np(lp):
    return [t.cpu().numpy().astype(np.float64) for t in lp.master]


def test_mlp_forward_matches_cpu(net_and_data):
    net, dn, X, alpha = net_and_data
    lp = learned.LearnedProposal(net.N, net.M, seed=3)
    Xs, As = X[:512], alpha[:512]
    Q, q = lp.forward(Xs, As, want_q=True)
    fw = omlp.forward(_params_np(lp), Xs.cpu().numpy(), As.cpu().numpy(), net.N, net.M)
    qg = q.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(qg - fw["q"]) <= 1e-2 * np.linalg.norm(fw["q"])
    # row by row: relative L1 error of every state's q (each row sums to 1)
    row_err = np.abs(qg - fw["q"]).sum(axis=1) / np.abs(fw["q"]).sum(axis=1)
    assert row_err.max() <= 1e-2, row_err.max()
    # and element by element, with an absolute floor for the tiny entries
    err = np.abs(qg - fw["q"])
    print(f"q: max row L1 {row_err.max():.3e}, max element error / (q + 1e-5) "
          f"{(err / (fw['q'] + 1e-5)).max():.3e}")
    assert np.all(err <= 1e-2 * fw["q"] + 1e-5)
    L = laws.ceil_log2(net.M)
    sup = As.cpu().numpy() > 0
    Qref = np.where(sup, np.maximum(np.floor(q.cpu().numpy() * np.float32(2.0 ** (31 - L))), 1), 0)
    assert np.array_equal(Q.cpu().numpy().view(np.uint32), Qref.astype(np.uint32))


@pytest.mark.parametrize("R", [37, 512, 1])
def test_mlp_forward_fused_matches_layer_by_layer(net_and_data, R):
    """The fused inference kernel against the layer-by-layer kernels: same
    products and exponentials, softmax row sums in another order; a partial
    last block of states (R % 32 != 0) included."""
    net, dn, X, alpha = net_and_data
    lp = learned.LearnedProposal(net.N, net.M, seed=5)
    Xs, As = X[:R].contiguous(), alpha[:R].contiguous()
    try:
        arsel.set_mlp_fused(False)
        Qu, qu = lp.forward(Xs, As, want_q=True)
        arsel.set_mlp_fused(True)
        Qf, qf = lp.forward(Xs, As, want_q=True)
    finally:
        arsel.set_mlp_fused(False)
    qu, qf = qu.cpu().numpy(), qf.cpu().numpy()
    assert np.array_equal(qu > 0, qf > 0)
    assert np.all(np.abs(qf - qu) <= 1e-6 * qu + 1e-12)
    Qu = Qu.cpu().numpy().view(np.uint32).astype(np.int64)
    Qf = Qf.cpu().numpy().view(np.uint32).astype(np.int64)
    assert np.all(np.abs(Qf - Qu) <= 1)
    fw = omlp.forward(_params_np(lp), Xs.cpu().numpy(), As.cpu().numpy(), net.N, net.M)
    err = np.abs(qf.astype(np.float64) - fw["q"])
    assert np.all(err <= 1e-2 * fw["q"] + 1e-5)


def test_proposal_select_bit_exact(net_and_data):
    net, dn, X, alpha = net_and_data
    lp = learned.LearnedProposal(net.N, net.M, seed=4)
    Xs, As = X[:2048].contiguous(), alpha[:2048].contiguous()
    Q, _ = lp.forward(Xs, As)
    a_np, Q_np = As.cpu().numpy(), Q.cpu().numpy().view(np.uint32)
    for t_max in (4096, 0, 1, 130):
        idx, tr = arsel.select_proposal(As, Q, seed=7, step=t_max, t_max=t_max, want_trials=True)
        oi, ot = oracle.select_proposal(a_np, Q_np, seed=7, step=t_max, t_max=t_max, threads=8)
        assert np.array_equal(idx.cpu().numpy(), oi), t_max
        assert np.array_equal(tr.cpu().numpy().view(np.uint32), ot), t_max
    # adversarial and invalid proposals
    rng = np.random.default_rng(0)
    Qr = rng.integers(1, 1000, size=Q_np.shape).astype(np.uint32) * (a_np > 0)
    Qr[0, np.argmax(a_np[0])] = 0                                    # -4: support not covered
    Qr[1, :] = 0
    Qr[1, 0] = 0xFFFFFFFF
    Qr[1, 1] = 2                                                     # -4 or -1: sum >= 2^32
    a_bad = a_np.copy()
    a_bad[2, 5] = np.nan                                             # -2
    a_bad[3, :] = 0                                                  # -1
    idx, tr = arsel.select_proposal(torch.from_numpy(a_bad).cuda(),
                                    torch.from_numpy(Qr.view(np.int32)).cuda(), seed=2,
                                    want_trials=True)
    oi, ot = oracle.select_proposal(a_bad, Qr, seed=2, threads=8)
    assert np.array_equal(idx.cpu().numpy(), oi)
    assert np.array_equal(tr.cpu().numpy().view(np.uint32), ot)
    assert oi[0] == -4 and oi[2] == -2 and oi[3] == -1


def test_gradients_match_cpu(net_and_data):
    net, dn, X, alpha = net_and_data
    lp = learned.LearnedProposal(net.N, net.M, seed=5)
    params = _params_np(lp)
    Xb, Ab = X[:1024].contiguous(), alpha[:1024].contiguous()
    loss = lp.train_step(Xb, Ab, lr=0.0)
    torch.cuda.synchronize()
    ref_loss, ref_g, _ = omlp.loss_and_grads(params, Xb.cpu().numpy(), Ab.cpu().numpy(), net.N,
                                             net.M)
    assert abs(loss.item() - ref_loss) <= 1e-3 * abs(ref_loss)
    for i, (g, r) in enumerate(zip(lp.grad, ref_g)):
        g = g.cpu().numpy().astype(np.float64)
        assert np.linalg.norm(g - r) <= 2e-2 * np.linalg.norm(r) + 1e-12, i
        # element by element against the tensor's scale: a wrong row or column
        # (a missing bias entry, a transposed operand) cannot hide in the norm
        err = np.abs(g - r)
        assert err.max() <= 2e-2 * np.abs(r).max() + 1e-12, (i, err.max(), np.abs(r).max())
        if r.ndim == 2:
            # per row and per column of the weight gradient, against that
            # row's or column's own scale
            for axis in (0, 1):
                scale = np.abs(r).max(axis=axis)
                worst = (err.max(axis=axis) / (scale + 1e-3 * np.abs(r).max())).max()
                print(f"grad {i} axis {axis}: worst error / (scale + floor) {worst:.3e}")
                assert worst <= 1e-1, (i, axis, worst)
    # lr = 0 leaves the weights unchanged
    for t, p in zip(lp.master, params):
        assert np.array_equal(t.cpu().numpy().astype(np.float64), p)


@pytest.mark.parametrize("lr", [1e-3, 3e-2])
def test_adam_step_matches_oracle(net_and_data, lr):
    """Two training steps with lr > 0 (t = 1 and t = 2): the FP32 masters and
    both Adam moments equal the oracle's float32 Adam fed the GPU's own
    gradients, bit for bit, and the BF16 copies are the masters rounded to
    nearest even."""
    net, dn, X, alpha = net_and_data
    lp = learned.LearnedProposal(net.N, net.M, seed=13)
    B = 512
    for t in (1, 2):
        w0 = [x.cpu().numpy().copy() for x in lp.master]
        m0 = [x.cpu().numpy().copy() for x in lp.m]
        v0 = [x.cpu().numpy().copy() for x in lp.v]
        lp.train_step(X[(t - 1) * B:t * B].contiguous(), alpha[(t - 1) * B:t * B].contiguous(),
                      lr=lr)
        torch.cuda.synchronize()
        assert lp.t == t
        for i in range(6):
            g = lp.grad[i].cpu().numpy()
            w1, m1, v1 = omlp.adam_step(w0[i], m0[i], v0[i], g, t, lr)
            for name, got, want in (("w", lp.master[i], w1), ("m", lp.m[i], m1),
                                    ("v", lp.v[i], v1)):
                got = got.cpu().numpy()
                diff = got.view(np.uint32) != want.view(np.uint32)
                assert not diff.any(), (t, i, name, int(diff.sum()), got[diff][:4], want[diff][:4])
        for wb, i in zip(lp.Wb, (0, 2, 4)):
            got = wb.cpu().view(torch.int16).numpy().astype(np.uint16)
            want = (omlp.bf16_round(lp.master[i].cpu().numpy()).view(np.uint32) >> 16).astype(np.uint16)
            assert np.array_equal(got, want), (t, i)


def _acceptance(trials):
    t = trials.cpu().numpy().view(np.uint32).astype(np.int64)
    ok = (t >= 1) & (t <= 4096)
    return ok.sum() / (t[ok].sum() + 4096 * (t > 4096).sum())


def test_training_raises_acceptance_and_keeps_the_law(net_and_data):
    net, dn, X, alpha = net_and_data
    lp = learned.LearnedProposal(net.N, net.M, seed=6)
    B = 1024
    n = (X.shape[0] // B) * B
    first = last = None
    for epoch in range(6):
        for s in range(0, n, B):
            loss = lp.train_step(X[s:s + B], alpha[s:s + B], lr=1e-3).item()
            first = loss if first is None else first
            last = loss
    assert last < first
    # held-out states: fresh realizations
    X0 = torch.from_numpy(workloads.poisson_counts(N=net.N, R=1024, seed=77)).cuda()
    dn.chain(X0, seed=9, step0=0, steps=300)
    Ah = dn.propensities(X0)
    Q, _ = lp.forward(X0, Ah)
    _, tr_l = arsel.select_proposal(Ah, Q, seed=3, want_trials=True)
    _, _, tr_u = arsel.select(Ah, net.M, 1024, net.M, arsel.AOS, seed=3, want_trials=True)
    acc_l, acc_u = _acceptance(tr_l), _acceptance(tr_u)
    print(f"per-trial acceptance: learned {acc_l:.4f}, uniform {acc_u:.4f}")
    assert acc_l > 2.0 * acc_u
    # the law: one held-out state broadcast to many instances, 1.02e6 selections
    a1 = Ah[:1].expand(4096, -1).contiguous()
    Q1 = Q[:1].expand(4096, -1).contiguous()
    counts = np.zeros(net.M)
    for step in range(250):
        idx, _ = arsel.select_proposal(a1, Q1, seed=12, step=step)
        counts += np.bincount(idx.cpu().numpy(), minlength=net.M)
    law, _ = laws.proposal_law(a1[0].cpu().numpy(), Q1[0].cpu().numpy().view(np.uint32), 4096)
    p = laws.chi_square_p(counts, law)
    e = law * counts.sum()
    worst = np.argsort(-(counts - e) ** 2 / np.maximum(e, 1e-300))[:5]
    assert p > 0.01, (p, [(int(j), counts[j], round(float(e[j]), 1)) for j in worst])


def test_checkpoint_resume_is_bit_exact(net_and_data):
    net, dn, X, alpha = net_and_data
    B = 512
    a = learned.LearnedProposal(net.N, net.M, seed=8)
    for s in range(6):
        a.train_step(X[s * B:(s + 1) * B], alpha[s * B:(s + 1) * B], lr=1e-3)
    b = learned.LearnedProposal(net.N, net.M, seed=8)
    for s in range(3):
        b.train_step(X[s * B:(s + 1) * B], alpha[s * B:(s + 1) * B], lr=1e-3)
    c = learned.LearnedProposal(net.N, net.M, seed=99)
    c.load_state_dict(b.state_dict())
    for s in range(3, 6):
        c.train_step(X[s * B:(s + 1) * B], alpha[s * B:(s + 1) * B], lr=1e-3)
    for x, y in zip(a.master, c.master):
        assert torch.equal(x, y)

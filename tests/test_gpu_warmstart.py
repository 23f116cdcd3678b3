"""GPU: the learned warm start's kernels (features, forward, gradient, Adam,
prediction) against the FP64 reference network in oracle/mlp.py, and the
warm-start fit certified by the oracle."""
import numpy as np
import pytest

import apd_synth as S
import oracle as O
from oracle import mlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2403_03571_amd as apd
    return apd.Context(0)


def _prob(inst):
    import paper_2403_03571_amd as apd
    return apd.Problem.from_instance(inst, "cuda:0")


def test_features_match_the_reference(ctx):
    import paper_2403_03571_amd as apd
    net = apd.WarmStart(ctx, mlp.init_params(0))
    for inst in (S.make_c5(600000), S.custom(2, 7, 32, seed=2), S.custom(2, 300, 64, seed=3, sigma=0.3)):
        F = net.features(_prob(inst)).cpu().numpy()
        d = mlp.deficit(inst.n, O.evaluate(inst, np.zeros(inst.n)).grad)
        ref = mlp.features(inst.x, inst.A, inst.v, inst.lo, inst.hi, d=d)
        np.testing.assert_allclose(F, ref, rtol=2e-6, atol=1e-6)


def test_forward_and_gradient_match_the_reference(ctx):
    import torch
    import paper_2403_03571_amd as apd
    rng = np.random.default_rng(0)
    p0 = mlp.init_params(3)
    p0 = (p0 + 0.01 * rng.standard_normal(p0.size)).astype(np.float32)
    net = apd.WarmStart(ctx, p0)
    for S_ in (1, 37, 300):
        X = rng.standard_normal((S_, mlp.N_FEAT)).astype(np.float32)
        t = rng.standard_normal(S_).astype(np.float32)
        Xd = torch.as_tensor(X, device="cuda:0")
        td = torch.as_tensor(t, device="cuda:0")
        y = net.forward(Xd).cpu().numpy()
        yr, _ = mlp.forward(p0.astype(np.float64), X.astype(np.float64))
        np.testing.assert_allclose(y, yr, rtol=1e-4, atol=1e-4 * np.abs(yr).max())
        loss, g = net.loss_grad(Xd, td)
        lr_, gr = mlp.loss_and_grad(p0.astype(np.float64), X.astype(np.float64), t.astype(np.float64))
        assert loss == pytest.approx(lr_, rel=1e-4)
        g = g.cpu().numpy()
        np.testing.assert_allclose(g, gr, rtol=0, atol=2e-4 * np.abs(gr).max())


def test_bf16_inference_matches_its_definition(ctx):
    """apd_ws_infer (BF16 matrix cores, FP32 accumulation) against the
    reference BF16 inference (BF16-rounded weights and layer inputs, exact
    sums): within 2^-9 of the output layer's absolute sum (the FP32
    accumulation order, and BF16 roundings of hidden values it may flip);
    against the FP64 network within 2^-6 of that sum (the stated BF16
    tolerance); after a parameter update too."""
    import torch
    import paper_2403_03571_amd as apd
    rng = np.random.default_rng(9)
    p0 = (mlp.init_params(11) + 0.02 * rng.standard_normal(mlp.n_params())).astype(np.float32)
    net = apd.WarmStart(ctx, p0)

    def check(params, X):
        y = net.infer(torch.as_tensor(X, device="cuda:0")).cpu().numpy().astype(np.float64)
        yb, sc = mlp.forward_bf16(params, X.astype(np.float64))
        y64, _ = mlp.forward(params, X.astype(np.float64))
        assert np.all(np.abs(y - yb) <= 2.0 ** -9 * sc), float(np.max(np.abs(y - yb) / sc))
        assert np.all(np.abs(y - y64) <= 2.0 ** -6 * sc), float(np.max(np.abs(y - y64) / sc))

    for S_ in (1, 31, 32, 33, 300):
        check(p0.astype(np.float64), rng.standard_normal((S_, mlp.N_FEAT)).astype(np.float32))
    X = rng.standard_normal((64, mlp.N_FEAT)).astype(np.float32)
    t = rng.standard_normal(64).astype(np.float32)
    net.train_step(torch.as_tensor(X, device="cuda:0"), torch.as_tensor(t, device="cuda:0"), 1e-2)
    check(net.params().astype(np.float64), X)


def test_adam_steps_match_the_reference(ctx):
    import torch
    import paper_2403_03571_amd as apd
    rng = np.random.default_rng(1)
    p = mlp.init_params(4)
    net = apd.WarmStart(ctx, p)
    X = rng.standard_normal((64, mlp.N_FEAT)).astype(np.float32)
    t = rng.standard_normal(64).astype(np.float32)
    pr = p.astype(np.float64)
    m = np.zeros_like(pr)
    v = np.zeros_like(pr)
    for step in range(1, 4):
        net.train_step(torch.as_tensor(X, device="cuda:0"), torch.as_tensor(t, device="cuda:0"), 1e-3)
        _, g = mlp.loss_and_grad(pr, X, t)
        pr, m, v = mlp.adam_step(pr, g, m, v, step, 1e-3)
    np.testing.assert_allclose(net.params(), pr, rtol=0, atol=2e-5)


def test_train_epoch_is_the_minibatch_steps(ctx):
    """apd_ws_train_epoch over S = 9000 samples: the Adam steps of its
    minibatches (4096, 4096, 808 in storage order), bit for bit the same
    parameters as three apd_ws_train_step calls, the reported loss their
    sample-weighted mean, and the parameters those of the FP64 reference's
    three Adam steps on the same minibatches to 2e-5."""
    import torch
    import paper_2403_03571_amd as apd
    rng = np.random.default_rng(3)
    p = mlp.init_params(6)
    S = 9000
    X = rng.standard_normal((S, mlp.N_FEAT)).astype(np.float32)
    t = rng.standard_normal(S).astype(np.float32)
    Xd, td = torch.as_tensor(X, device="cuda:0"), torch.as_tensor(t, device="cuda:0")
    a, b = apd.WarmStart(ctx, p), apd.WarmStart(ctx, p)
    loss_epoch = a.train_epoch(Xd, td, 1e-3)
    losses, sizes = [], []
    for k in range(0, S, 4096):
        sb = min(4096, S - k)
        losses.append(b.train_step(Xd[k:k + sb].contiguous(), td[k:k + sb].contiguous(), 1e-3))
        sizes.append(sb)
    assert sizes == [4096, 4096, 808]
    assert np.array_equal(a.params(), b.params())
    assert loss_epoch == pytest.approx(np.dot(losses, sizes) / S, rel=1e-12)
    pr = p.astype(np.float64)
    m = np.zeros_like(pr)
    v = np.zeros_like(pr)
    for step, k in enumerate(range(0, S, 4096), start=1):
        _, g = mlp.loss_and_grad(pr, X[k:k + 4096], t[k:k + 4096])
        pr, m, v = mlp.adam_step(pr, g, m, v, step, 1e-3)
    np.testing.assert_allclose(a.params(), pr, rtol=0, atol=2e-5)


def test_warm_fit_is_certified_and_falls_back(ctx):
    import paper_2403_03571_amd as apd
    inst = S.make_c5(600001)
    net = apd.WarmStart(ctx, mlp.init_params(5))   # untrained: a poor guess
    w, rep, used = net.fit(_prob(inst))
    assert rep.converged
    assert O.evaluate(inst, w.cpu().numpy()).maxrel < 0.01
    # prediction = centred (BF16-inference) network output / N
    F = net.features(_prob(inst))
    y = net.infer(F).cpu().numpy().astype(np.float64)
    wp = net.predict(_prob(inst)).cpu().numpy()
    np.testing.assert_allclose(wp, (y - y.mean()) / inst.n, rtol=0, atol=1e-12)
    # a tiny budget forces the fallback to the cold start
    w2, rep2, used2 = net.fit(_prob(inst), max_evals=3)
    assert not used2


def test_trained_network_gain_is_measured(ctx):
    """Train the network on the library's own solutions of small 2D
    instances (256^2 pixels, N in [100, 300]) with the library's kernels,
    then on held-out instances: the prediction explains most of the optimal
    weights' variance (R^2 > 0.5 against the centred targets; measured
    0.63), every warm fit is certified by the oracle, and the warm fits take
    fewer passes than the cold ones on average, the feature pass included
    (measured 80.5 against 81.5: a gain of about 1 %, the honest size of it
    -- the passes go to the last decade of the volume error, which a
    per-seed prediction does not shorten)."""
    import torch
    import paper_2403_03571_amd as apd
    from paper_2403_03571_amd import warmstart as W

    def inst_of(seed):
        return S.make_c5(seed, n=int(np.random.default_rng(seed).integers(100, 301)), M=256)

    net = apd.WarmStart(ctx, mlp.init_params(7))
    train = [_prob(inst_of(700000 + k)) for k in range(160)]
    ws, reps, st = ctx.apd_fit_weights_batched(train)
    assert st == "APD_OK"
    F = torch.cat([net.features(p) for p in train])
    t = torch.cat([net.targets(w) for w in ws])
    hist, _ = W.train(net, F, t, epochs=6, batch=2048, lr=2e-3, seed=1, log=lambda m: None)
    assert hist[-1] < 0.9 * hist[0]
    ss_res = ss_tot = 0.0
    cold, warm = [], []
    for k in range(12):
        inst = inst_of(800000 + k)
        p = _prob(inst)
        wc, rc = ctx.apd_fit_weights(p)
        y = net.forward(net.features(p)).cpu().numpy().astype(np.float64)
        tt = net.targets(wc).cpu().numpy().astype(np.float64)
        yc = y - y.mean()
        ss_res += float(((yc - tt) ** 2).sum())
        ss_tot += float((tt ** 2).sum())
        w, rw, used = net.fit(p)
        assert rw.converged
        assert O.evaluate(inst, w.cpu().numpy()).maxrel < 0.01
        cold.append(rc.evals)
        warm.append(rw.evals)
    r2 = 1.0 - ss_res / ss_tot
    print(f"[warm start] held-out R^2 {r2:.3f}; passes cold {np.mean(cold):.1f} "
          f"warm {np.mean(warm):.1f} (incl. the feature pass)", flush=True)
    assert r2 > 0.5
    assert np.mean(warm) < np.mean(cold)

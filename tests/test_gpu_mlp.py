"""The proposal network's GPU kernels against the FP64 oracle, and the
learned schedule against the plain one."""
import numpy as np
import pytest

import workloads
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


def test_forward_and_gradient_match_oracle(qs_lib):
    qs = qs_lib
    params = omlp.init_params(7)
    g = np.random.default_rng(8)
    X = g.standard_normal((300, 32))
    y = (g.random(300) < 0.4).astype(float)
    net = qs.MLP(omlp.flatten(params))
    np.testing.assert_array_equal(net.get_params(), omlp.flatten(params).astype(np.float32))
    scores = net.forward(X)
    want = omlp.forward(params, X)["score"]
    np.testing.assert_allclose(scores, want, atol=2e-6, rtol=1e-5)
    grad, loss = net.grad(X, y)
    gw = omlp.flatten(omlp.backward(params, X, y))
    rel = np.linalg.norm(grad - gw) / np.linalg.norm(gw)
    assert rel < 1e-4, rel
    assert abs(loss - omlp.loss(params, X, y)) < 1e-5
    # the gradient is a real descent direction: a small step lowers the loss
    step = omlp.unflatten(omlp.flatten(params) - 0.05 * grad.astype(np.float64))
    assert omlp.loss(step, X, y) < omlp.loss(params, X, y)
    net.free()


def test_adam_training_matches_oracle_steps(qs_lib):
    qs = qs_lib
    g = np.random.default_rng(9)
    X = g.standard_normal((512, 32))
    y = (X[:, 0] - 0.7 * X[:, 5] + 0.2 > 0).astype(float)
    params = omlp.init_params(10)
    net = qs.MLP(omlp.flatten(params))
    loss_gpu = net.train(X, y, steps=60, batch=128, lr=1e-2)
    # the oracle takes the same Adam steps on the same consecutive minibatches
    m = {k: np.zeros(s) for k, s in omlp.SHAPES}
    v = {k: np.zeros(s) for k, s in omlp.SHAPES}
    cur = 0
    for step in range(1, 61):
        if cur + 128 > 512:
            cur = 0
        Xb, yb = X[cur:cur + 128], y[cur:cur + 128]
        cur += 128
        omlp.adam_step(params, omlp.backward(params, Xb, yb), m, v, step, lr=1e-2)
    loss_orc = omlp.loss(params, X, y)
    assert abs(loss_gpu - loss_orc) < 2e-3, (loss_gpu, loss_orc)
    np.testing.assert_allclose(net.get_params(), omlp.flatten(params), atol=2e-3)
    assert loss_gpu < 0.3
    net.free()


def collect(qs, protocol, seeds, p, rows=4, cols=6, layers=7):
    Xs, ys = [], []
    for s in seeds:
        gates = workloads.grid_circuit(rows, cols, layers, s)
        r = protocol.approx_run(rows * cols, gates, p, features=True)
        Xs.append(r["features"])
        ys.append(np.array([a[3] for a in r["log"]], dtype=np.float32))
    return np.concatenate(Xs), np.concatenate(ys)


def test_learned_schedule_tests_fewer_qubits(qs_lib):
    """Train on plain runs of disjoint seeds; on held-out circuits the learned
    schedule makes fewer exact tests, every rounding it makes still obeys
    eps <= p/2, and F stays within a few percent of the plain schedule's."""
    from paper_2304_14969_amd import protocol
    qs = qs_lib
    p = 0.1
    X, y = collect(qs, protocol, range(10000, 10040), p)
    assert 0.02 < y.mean() < 0.9
    order = np.random.default_rng(0).permutation(len(y))
    net = qs.MLP(omlp.flatten(omlp.init_params(1)))
    loss = net.train(X[order], y[order], steps=1500, batch=256, lr=3e-3)
    assert loss < 0.6
    plain_tests = learned_tests = 0
    for s in range(5):
        gates = workloads.grid_circuit(4, 6, 7, s)
        a = protocol.approx_run(24, gates, p, record=True)
        b = protocol.approx_run(24, gates, p, record=True, proposer=net, cutoff=0.3)
        assert a["ok"] and b["ok"]
        for q, nsub, eps, rounded in b["log"]:
            if rounded:
                assert eps <= p / 2 + 1e-6
        plain_tests += a["attempts"]
        learned_tests += b["attempts"]
        assert b["F"] >= a["F"] * 0.9
    assert learned_tests < plain_tests
    net.free()

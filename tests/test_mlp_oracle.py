"""Pins of the learned-form oracle (CPU): the network, its loss gradient, the
Adam update, the pair features, and the restricted learned-form step.

Each pin comes from outside the function it checks: central finite
differences of the loss, hand-set networks with known outputs, closed forms
of the loss and of the first Adam steps, the exact energy change as a
function of the features, and the special cases of the restricted step that
reduce to the ordinary step or to enumerating single flips by Eq. 1.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_2010_00180_amd import workloads


def _samples(n, seed):
    rng = np.random.default_rng(seed)
    X = np.stack([rng.normal(0, 1.5, n), rng.normal(0, 1.5, n), rng.normal(0, 1, n),
                  rng.choice([-1.0, 1.0], n)], axis=1)
    y = (rng.random(n) < 0.3).astype(np.uint8)
    return X, y


@pytest.mark.parametrize("pos_w", [1.0, 7.5])
def test_gradient_matches_central_differences(pos_w):
    P = workloads.network_params(1)
    X, y = _samples(40, 2)
    L, G = mlp.loss_grad(P, X, y, pos_w)
    rng = np.random.default_rng(3)
    # every bias and output weight, and a sample of the weight matrices
    idx = list(range(mlp.OFF_B1, mlp.OFF_W2)) + list(range(mlp.OFF_B2, mlp.NPARAM))
    idx += list(rng.choice(np.arange(mlp.OFF_W1, mlp.OFF_B1), 40, replace=False))
    idx += list(rng.choice(np.arange(mlp.OFF_W2, mlp.OFF_B2), 200, replace=False))
    eps = 1e-6
    for k in idx:
        Pp = P.copy(); Pp[k] += eps
        Pm = P.copy(); Pm[k] -= eps
        fd = (mlp.loss_grad(Pp, X, y, pos_w)[0] - mlp.loss_grad(Pm, X, y, pos_w)[0]) / (2 * eps)
        assert abs(fd - G[k]) <= 1e-6 * max(1.0, abs(G[k])) + 1e-8, (k, fd, G[k])


def test_loss_closed_form_at_zero_logit():
    # all parameters zero => z = 0 => loss = log 2 * mean(p y + (1 - y)), dL/db3 = mean(-p y + (1 - y)) / 2
    P = np.zeros(mlp.NPARAM)
    X, y = _samples(64, 4)
    p = 3.0
    L, G = mlp.loss_grad(P, X, y, p)
    assert L == pytest.approx(np.log(2) * np.mean(p * y + (1 - y)), rel=1e-14)
    assert G[mlp.OFF_B3] == pytest.approx(np.mean(-p * y + (1 - y)) / 2, rel=1e-14)
    assert np.all(G[:mlp.OFF_B3] == 0)


def test_forward_hand_set_network():
    # h1_0 = relu(x0), h2_0 = relu(h1_0), z = 2 h2_0 - 1 ; h1_1 = relu(-x3 + 0.5) feeds h2_1 with weight 3
    P = np.zeros(mlp.NPARAM)
    P[mlp.OFF_W1 + 0 * 4 + 0] = 1.0
    P[mlp.OFF_W1 + 1 * 4 + 3] = -1.0
    P[mlp.OFF_B1 + 1] = 0.5
    P[mlp.OFF_W2 + 0 * 64 + 0] = 1.0
    P[mlp.OFF_W2 + 1 * 64 + 1] = 3.0
    P[mlp.OFF_W3 + 0] = 2.0
    P[mlp.OFF_W3 + 1] = 0.25
    P[mlp.OFF_B3] = -1.0
    X = np.array([[1.5, 0, 0, 1], [-2.0, 5, 5, 1], [0.25, 0, 0, -1], [3.0, 1, 1, -1]])
    want = [2 * 1.5 - 1, -1.0, 2 * 0.25 - 1 + 0.25 * 3 * 1.5, 2 * 3.0 - 1 + 0.25 * 3 * 1.5]
    np.testing.assert_allclose(mlp.forward(P, X), want, rtol=0, atol=1e-15)


def test_adam_first_steps_closed_form():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p0 = np.array([1.0, 1.0, 1.0, 1.0])
    lr, eps = 1e-2, 1e-8
    p1, m1, v1 = mlp.adam_step(p0, np.zeros(4), np.zeros(4), g, 1, lr=lr, eps=eps)
    # bias-corrected moments of one step are g and g^2: the step is lr * g / (|g| + eps)
    np.testing.assert_allclose(p1, p0 - lr * g / (np.abs(g) + eps), rtol=1e-12, atol=0)
    # a constant gradient keeps the corrected moments at g and g^2
    p2, _, _ = mlp.adam_step(p1, m1, v1, g, 2, lr=lr, eps=eps)
    np.testing.assert_allclose(p2, p1 - lr * g / (np.abs(g) + eps), rtol=1e-12, atol=0)


def test_features_determine_the_energy_change():
    w = workloads.custom([40], L=1, M=4, seed_offset=7)
    inst = w.instances[0]
    x = inst.init_bits[0]
    Xf, ii, jj = mlp.pair_features(inst.J, inst.h, x)
    E0 = oracle.energy(inst.J, inst.h, x)
    N = inst.N
    dE = -2 * Xf[:, 0] - 2 * Xf[:, 1] + 4 * Xf[:, 2] / np.sqrt(N) * Xf[:, 3]
    rng = np.random.default_rng(5)
    for k in rng.choice(len(ii), 60, replace=False):
        y = x.copy()
        y[ii[k] >> 6] ^= np.uint64(1) << np.uint64(ii[k] & 63)
        y[jj[k] >> 6] ^= np.uint64(1) << np.uint64(jj[k] & 63)
        assert oracle.energy(inst.J, inst.h, y) - E0 == pytest.approx(dE[k], abs=1e-12)


def _kept_after_one_step(inst, M):
    b1, E1, f1, _ = oracle.step(inst.J, inst.h, M, inst.init_bits[:1])
    return b1, E1, f1


def test_step_proposed_with_all_pairs_is_the_step():
    w = workloads.custom([30], L=2, M=12, seed_offset=8)
    inst = w.instances[0]
    M = w.M
    b1, E1, f1 = _kept_after_one_step(inst, M)
    N = inst.N
    allp = [int(i) | int(j) << 16 for i, j in zip(*np.triu_indices(N, 1))]
    par = np.nonzero(f1)[0]
    got = oracle.step_proposed(inst.J, inst.h, M, b1, E1, par, [allp] * len(par))
    want = oracle.step(inst.J, inst.h, M, b1, E1, f1)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
    assert np.array_equal(got[2], want[2]) and got[3] == want[3]


def test_step_proposed_without_pairs_offers_singles_only():
    w = workloads.custom([20], L=1, M=10, seed_offset=9)
    inst = w.instances[0]
    M, N = w.M, inst.N
    b1, E1, f1 = _kept_after_one_step(inst, M)
    par = np.nonzero(f1)[0][:3]
    got_b, got_E, _, _ = oracle.step_proposed(inst.J, inst.h, M, b1, E1, par, [[] for _ in par])
    # by hand: S_t and the single flips of the parents, energies by Eq. 1, (E, psi) order
    cand = {}
    for k in range(len(E1)):
        cand[int(b1[k][0])] = oracle.energy(inst.J, inst.h, b1[k])
    for p in par:
        for i in range(N):
            y = b1[p].copy()
            y[0] ^= np.uint64(1) << np.uint64(i)
            cand[int(y[0])] = oracle.energy(inst.J, inst.h, y)
    order = sorted(cand.items(), key=lambda kv: (kv[1], kv[0]))[:M]
    assert [int(v[0]) for v in got_b] == [k for k, _ in order]
    np.testing.assert_array_equal(got_E, [e for _, e in order])


def test_step_proposed_rejects_malformed_pairs():
    w = workloads.custom([20], L=1, M=4, seed_offset=9)
    inst = w.instances[0]
    b1, E1, f1 = _kept_after_one_step(inst, 4)
    with pytest.raises(ValueError):
        oracle.step_proposed(inst.J, inst.h, 4, b1, E1, [0], [[5 | 3 << 16]])

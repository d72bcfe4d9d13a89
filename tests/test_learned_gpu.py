"""Learned-proposal form on the GPU, through the C ABI.

Parity of a ranking step is exact: given the proposals the GPU recorded, the
kept set must equal the oracle's M lowest distinct states of S_t, the single
flips of the ranked parents and the proposed pair flips; a full step must
equal the oracle's exact step; and every final set must be a fixed point of
the exact step (the stability certificate).  The ranking itself is checked
against the network evaluated with the kernel's bf16 rounding points in
numpy (FP64 accumulation), the training kernels against the FP64 oracle.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_2010_00180_amd import binding, workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    binding.load()


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def torch_mod():
    import torch
    return torch


def bf16(x):
    """Round to bf16 (nearest even) and return as float32 values."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32)


def emulated_scores(P, J, h, x):
    """The network as the ranking kernel evaluates it: weights, features and
    hidden activations rounded to bf16; sums here in FP64."""
    P = np.asarray(P, np.float32)
    N = len(h)
    s = mlp.spins(x, N)
    F = np.asarray(h) + np.asarray(J) @ s
    f = (s * F).astype(np.float32)
    ii, jj = np.triu_indices(N, 1)
    jn = bf16(np.float32(np.sqrt(N) * np.asarray(J)[ii, jj]))
    X = np.stack([bf16(f[ii]), bf16(f[jj]), jn, s[ii] * s[jj], np.ones(len(ii))], 1).astype(np.float64)
    W1 = bf16(P[mlp.OFF_W1:mlp.OFF_B1].reshape(64, 4)).astype(np.float64)
    b1 = bf16(P[mlp.OFF_B1:mlp.OFF_W2]).astype(np.float64)
    W2 = bf16(P[mlp.OFF_W2:mlp.OFF_B2].reshape(64, 64)).astype(np.float64)
    b2 = P[mlp.OFF_B2:mlp.OFF_W3].astype(np.float64)
    w3 = bf16(P[mlp.OFF_W3:mlp.OFF_B3]).astype(np.float64)
    b3 = float(P[mlp.OFF_B3])
    a1 = X[:, :4] @ W1.T + b1
    H1 = np.maximum(bf16(a1), 0).astype(np.float64)
    H2 = np.maximum(bf16(H1 @ W2.T + b2), 0).astype(np.float64)
    return H2 @ w3 + b3, ii, jj


def score_intervals(P, J, h, x):
    """Per pair, an interval that holds the ranking kernel's score.  The
    network as the kernel evaluates it (bf16 weights, features and hidden
    activations, nearest even) is followed exactly, except that the kernel
    sums in FP32 in an order of its own: each sum of n exact products is
    within gamma_n = n 2^-24 of its magnitude sum of the exact value, so each
    pre-activation is carried as an interval, rounded to bf16 at both ends
    (rounding is monotone) and passed on by interval arithmetic."""
    P = np.asarray(P, np.float32)
    N = len(h)
    s = mlp.spins(x, N)
    F = np.asarray(h) + np.asarray(J) @ s
    f = (s * F).astype(np.float32)
    ii, jj = np.triu_indices(N, 1)
    jn = bf16(np.float32(np.sqrt(N) * np.asarray(J)[ii, jj]))
    X = np.stack([bf16(f[ii]), bf16(f[jj]), jn, s[ii] * s[jj], np.ones(len(ii))], 1).astype(np.float64)
    W1 = np.concatenate([bf16(P[mlp.OFF_W1:mlp.OFF_B1].reshape(64, 4)),
                         bf16(P[mlp.OFF_B1:mlp.OFF_W2]).reshape(64, 1)], 1).astype(np.float64)
    W2 = bf16(P[mlp.OFF_W2:mlp.OFF_B2].reshape(64, 64)).astype(np.float64)
    b2 = P[mlp.OFF_B2:mlp.OFF_W3].astype(np.float64)
    w3 = bf16(P[mlp.OFF_W3:mlp.OFF_B3]).astype(np.float64)
    b3 = float(P[mlp.OFF_B3])
    u = 2.0 ** -24

    def rnd(v):   # bf16 nearest even of FP64 values (exact ones here), then relu
        return np.maximum(bf16(v.astype(np.float32)).astype(np.float64), 0.0)

    # layer 1: 5 exact products per unit (features x bf16 weights, bias x 1)
    a1 = X @ W1.T
    e1 = 6 * u * (np.abs(X) @ np.abs(W1).T)
    # the FP32 sum can also round the exact value itself once more
    h1_lo, h1_hi = rnd(a1 - e1), rnd(a1 + e1)
    # layer 2: 64 exact products and the FP32 bias
    Wp, Wn = np.maximum(W2, 0), np.minimum(W2, 0)
    a2_lo = h1_lo @ Wp.T + h1_hi @ Wn.T + b2
    a2_hi = h1_hi @ Wp.T + h1_lo @ Wn.T + b2
    e2 = 66 * u * (h1_hi @ np.abs(W2).T + np.abs(b2))
    h2_lo, h2_hi = rnd(a2_lo - e2), rnd(a2_hi + e2)
    wp, wn = np.maximum(w3, 0), np.minimum(w3, 0)
    z_lo = h2_lo @ wp + h2_hi @ wn + b3
    z_hi = h2_hi @ wp + h2_lo @ wn + b3
    e3 = 67 * u * (h2_hi @ np.abs(w3) + abs(b3))
    return z_lo - e3, z_hi + e3, ii, jj


def codes_of(ii, jj):
    return (np.asarray(ii, np.uint64) | (np.asarray(jj, np.uint64) << np.uint64(16))).astype(np.uint32)


def random_params(seed):
    return wl.network_params(seed).astype(np.float32)


def index_of_states(bits):
    return {bytes(np.ascontiguousarray(b).tobytes()): k for k, b in enumerate(bits)}


def learned_parity(w, scorer, params, tag, topk=8, persistent=0, cap=400):
    note(f"[{tag}] Ns={[i.N for i in w.instances]} L={w.L} M={w.M} scorer={scorer} topk={topk} persistent={persistent}")
    s = binding.IsingSearch.from_workload(w, form=binding.FORM_LEARNED, topk_factor=topk,
                                          flags=binding.FLAG_RECORD_PROPOSALS, persistent=persistent)
    s.set_scorer(scorer, params, seed=11)
    S = w.L * len(w.instances)
    done = [False] * S
    ranked_steps = full_steps = 0
    for t in range(cap):
        before = [s.get_search(k) for k in range(S)]
        active = s.step()
        for k in range(S):
            inst = w.instances[k // w.L]
            N = inst.N
            bb, bE, bf = before[k]
            gb, gE, gf = s.get_search(k)
            if done[k]:
                assert np.array_equal(gb, bb) and np.array_equal(gE, bE), f"{tag} search {k} moved after stopping"
                continue
            mode, props = s.get_proposals(k)
            if mode == 0:
                ranked_steps += 1
                where = index_of_states(bb)
                par = [where[bytes(np.ascontiguousarray(p).tobytes())] for p, _ in props]
                assert sorted(par) == list(np.nonzero(bf)[0]), f"{tag} search {k} step {t + 1}: ranked parents"
                P = N * (N - 1) // 2
                for _, c in props:
                    i, j = c & 0xFFFF, c >> 16
                    assert len(c) == min(topk * N, P)
                    assert len(np.unique(c)) == len(c) and np.all(i < j) and np.all(j < N)
                ob, oE, of, nn = oracle.step_proposed(inst.J, inst.h, w.M, bb, bE, par, [c for _, c in props])
            else:
                full_steps += 1
                assert not props
                ob, oE, of, nn = oracle.step(inst.J, inst.h, w.M, bb, bE, literal=True)
            assert gb.shape == ob.shape and np.array_equal(gb, ob), f"{tag} search {k} step {t + 1} mode {mode}: bits"
            assert np.array_equal(gE, oE), f"{tag} search {k} step {t + 1}: energies"
            assert np.array_equal(gf.astype(bool), of.astype(bool)), f"{tag} search {k} step {t + 1}: new flags"
            if mode == 1 and nn == 0:
                done[k] = True
        if active == 0:
            break
    assert all(done), f"{tag}: searches still running after {cap} steps"
    for k in range(S):
        inst = w.instances[k // w.L]
        gb, gE, _ = s.get_search(k)
        _, _, _, nn = oracle.step(inst.J, inst.h, w.M, gb, gE, literal=True)
        assert nn == 0, f"{tag} search {k}: final set is not a fixed point of the exact step"
    st = s.stats()
    assert st["fallbacks"] == full_steps and st["ranked_states"] > 0
    s.destroy()
    note(f"[{tag}] ok: {ranked_steps} ranked and {full_steps} full search-steps")
    return st


@pytest.mark.parametrize("scorer", [binding.SCORER_NETWORK, binding.SCORER_FIELDS, binding.SCORER_UNIFORM])
def test_learned_parity_small(scorer):
    w = wl.custom([24, 40], L=3, M=8, seed_offset=301)
    learned_parity(w, scorer, random_params(1), f"small-{scorer}")


def test_learned_parity_ragged_many_compactions():
    # K = 2N of N(N-1)/2 pairs, N not a multiple of 16 or 64: the key buffer fills many times
    w = wl.custom([130, 97], L=2, M=24, seed_offset=302)
    learned_parity(w, binding.SCORER_NETWORK, random_params(2), "ragged", topk=2)


def test_learned_parity_tiny_instances():
    w = wl.custom([2, 3, 5, 17], L=2, M=6, seed_offset=303)
    learned_parity(w, binding.SCORER_FIELDS, None, "tiny")


def test_learned_parity_persistent_graph():
    w = wl.custom([64, 100], L=2, M=16, seed_offset=304)
    learned_parity(w, binding.SCORER_NETWORK, random_params(3), "graph", persistent=1)


def test_learned_first_step_at_n600_sampled():
    # the shape of the N=600, M=120 workload: two searches, the first two steps, checked exactly
    w = wl.custom([600], L=2, M=120, seed_offset=305)
    inst = w.instances[0]
    s = binding.IsingSearch.from_workload(w, form=binding.FORM_LEARNED, flags=binding.FLAG_RECORD_PROPOSALS)
    s.set_scorer(binding.SCORER_NETWORK, random_params(4))
    for t in range(2):
        before = [s.get_search(k) for k in range(2)]
        s.step()
        for k in range(2):
            bb, bE, bf = before[k]
            mode, props = s.get_proposals(k)
            assert mode == 0 and len(props) == int(bf.sum())
            where = index_of_states(bb)
            par = [where[bytes(np.ascontiguousarray(p).tobytes())] for p, _ in props]
            ob, oE, of, _ = oracle.step_proposed(inst.J, inst.h, w.M, bb, bE, par, [c for _, c in props])
            gb, gE, gf = s.get_search(k)
            assert np.array_equal(gb, ob) and np.array_equal(gE, oE), f"N=600 search {k} step {t + 1}"
            note(f"[n600] search {k} step {t + 1}: {len(par)} parents ok")
    s.destroy()


def _first_step_proposals(w, scorer, params, topk=8):
    s = binding.IsingSearch.from_workload(w, form=binding.FORM_LEARNED, topk_factor=topk,
                                          flags=binding.FLAG_RECORD_PROPOSALS)
    s.set_scorer(scorer, params, seed=5)
    s.step()
    out = [s.get_proposals(k) for k in range(w.L)]
    s.destroy()
    return out


def test_network_ranking_is_the_top_k():
    """The kernel keeps exactly K = 8N pairs: every pair whose score interval
    lies above those of all but fewer than K others, and none whose interval
    lies below those of K others (the intervals hold the kernel's FP32 sums;
    only pairs whose intervals straddle the K-th score are undecided)."""
    w = wl.custom([150], L=3, M=16, seed_offset=306)
    inst = w.instances[0]
    P = random_params(6)
    for k, (mode, props) in enumerate(_first_step_proposals(w, binding.SCORER_NETWORK, P)):
        assert mode == 0 and len(props) == 1
        x, c = props[0]
        assert np.array_equal(x, inst.init_bits[k])
        lo, hi, ii, jj = score_intervals(P, inst.J, inst.h, x)
        K = len(c)
        assert K == 8 * inst.N and len(set(c.tolist())) == K
        chosen = np.isin(codes_of(ii, jj), c)
        # for each pair: how many others certainly score higher / may score higher
        los, his = np.sort(lo), np.sort(hi)
        n = len(lo)
        above_certain = n - np.searchsorted(los, hi, side="right")        # lo_q > hi_p
        above_possible = n - np.searchsorted(his, lo, side="left") - 1    # hi_q >= lo_p, q != p
        must_in = above_possible < K
        must_out = above_certain >= K
        assert not np.any(must_in & must_out)
        assert np.all(chosen[must_in]), f"search {k}: {np.sum(must_in & ~chosen)} certain pairs missing"
        assert not np.any(chosen[must_out]), f"search {k}: {np.sum(must_out & chosen)} excluded pairs kept"
        undecided = np.sum(~must_in & ~must_out)
        width = np.max(hi - lo)
        note(f"[rank] search {k}: {undecided} of {n} pairs undecided by the intervals "
             f"(widest {width:.2e}); all {K} kept pairs consistent")
        assert undecided < K // 20


def test_fields_ranking_is_exact():
    w = wl.custom([90], L=2, M=8, seed_offset=307)
    inst = w.instances[0]
    for k, (mode, props) in enumerate(_first_step_proposals(w, binding.SCORER_FIELDS, None)):
        x, c = props[0]
        s = mlp.spins(x, inst.N)
        a = -2.0 * s * (inst.h + inst.J @ s)
        ii, jj = np.triu_indices(inst.N, 1)
        z = (-0.5 * (a[ii] + a[jj])).astype(np.float32)
        code = codes_of(ii, jj)
        order = np.lexsort((code, -z.astype(np.float64)))   # larger score first, then smaller code
        K = 8 * inst.N
        assert set(code[order[:K]].tolist()) == set(c.tolist())


# ---------------------------------------------------------------- training kernels
def _dev(a, dtype):
    torch = torch_mod()
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _samples(n, seed):
    rng = np.random.default_rng(seed)
    X = np.stack([rng.normal(0, 1.5, n), rng.normal(0, 1.5, n), rng.normal(0, 1, n),
                  rng.choice([-1.0, 1.0], n)], 1).astype(np.float32)
    y = (rng.random(n) < 0.2).astype(np.uint8)
    return X, y


@pytest.mark.parametrize("n", [1, 63, 1000, 70001])
def test_gradient_matches_oracle(n):
    torch = torch_mod()
    P = random_params(7)
    X, y = _samples(n, 8)
    pw = 3.5
    dP, dX, dy = _dev(P, torch.float32), _dev(X, torch.float32), _dev(y, torch.uint8)
    g = torch.zeros(mlp.NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    wsb = binding.mlp_workspace_bytes()
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    binding.mlp_loss_grad(dP.data_ptr(), dX.data_ptr(), dy.data_ptr(), n, pw, g.data_ptr(), loss.data_ptr(),
                          ws.data_ptr(), wsb, stream)
    torch.cuda.synchronize()
    Lr, Gr = mlp.loss_grad(P.astype(np.float64), X.astype(np.float64), y, pw)
    G = g.cpu().numpy().astype(np.float64)
    # FP32 sums of at most n terms per entry: well inside 1e-4 of the largest entry
    tol = 1e-4 * np.max(np.abs(Gr)) + 1e-7
    assert np.max(np.abs(G - Gr)) <= tol, (np.max(np.abs(G - Gr)), tol)
    assert abs(float(loss.item()) - Lr) <= 1e-5 * abs(Lr) + 1e-7
    z = torch.zeros(n, dtype=torch.float32, device="cuda")
    binding.mlp_forward(dP.data_ptr(), dX.data_ptr(), n, z.data_ptr(), stream)
    torch.cuda.synchronize()
    zr = mlp.forward(P.astype(np.float64), X.astype(np.float64))
    assert np.max(np.abs(z.cpu().numpy() - zr)) <= 1e-4 * (1 + np.max(np.abs(zr)))


def test_adam_matches_oracle():
    torch = torch_mod()
    rng = np.random.default_rng(9)
    P = random_params(9)
    m = np.zeros(mlp.NPARAM)
    v = np.zeros(mlp.NPARAM)
    dP, dm, dv = _dev(P, torch.float32), _dev(m, torch.float32), _dev(v, torch.float32)
    p64 = P.astype(np.float64)
    for t in range(1, 4):
        g = rng.normal(0, 1e-2, mlp.NPARAM).astype(np.float32)
        dg = _dev(g, torch.float32)
        binding.mlp_adam(dP.data_ptr(), dm.data_ptr(), dv.data_ptr(), dg.data_ptr(), t, lr=1e-3,
                         stream=torch.cuda.current_stream().cuda_stream)
        p64, m, v = mlp.adam_step(p64, m, v, g.astype(np.float64), t, lr=1e-3)
    torch.cuda.synchronize()
    assert np.max(np.abs(dP.cpu().numpy() - p64)) <= 1e-6 * (1 + np.max(np.abs(p64)))


def test_training_learns_a_separable_rule():
    torch = torch_mod()
    n = 200000
    X, _ = _samples(n, 10)
    # label: the exact energy change of the features is below -1
    dE = -2 * X[:, 0] - 2 * X[:, 1] + 4 * X[:, 2] / np.sqrt(100) * X[:, 3]
    y = (dE < -1.0).astype(np.uint8)
    P = random_params(10)
    dP, dX, dy = _dev(P, torch.float32), _dev(X, torch.float32), _dev(y, torch.uint8)
    dm = torch.zeros(mlp.NPARAM, dtype=torch.float32, device="cuda")
    dv = torch.zeros_like(dm)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    wsb = binding.mlp_workspace_bytes()
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    L0, _ = mlp.loss_grad(P.astype(np.float64), X[:20000].astype(np.float64), y[:20000], 1.0)
    binding.mlp_train(dP.data_ptr(), dm.data_ptr(), dv.data_ptr(), dX.data_ptr(), dy.data_ptr(), n, 4096, 300, 0,
                      3e-3, 1.0, 123, loss.data_ptr(), ws.data_ptr(), wsb, st)
    torch.cuda.synchronize()
    P1 = dP.cpu().numpy().astype(np.float64)
    L1, _ = mlp.loss_grad(P1, X[:20000].astype(np.float64), y[:20000], 1.0)
    acc = np.mean((mlp.forward(P1, X[:20000].astype(np.float64)) > 0) == (y[:20000] == 1))
    note(f"[train] loss {L0:.4f} -> {L1:.4f}, accuracy {acc:.4f}")
    assert L1 < 0.25 * L0 and acc > 0.97


# ---------------------------------------------------------------- trace capture
def test_trace_labels_match_the_oracle():
    torch = torch_mod()
    w = wl.custom([40], L=1, M=16, seed_offset=308)
    inst = w.instances[0]
    N = inst.N
    cap = 1 << 16
    feat = torch.zeros((cap, 4), dtype=torch.float32, device="cuda")
    lab = torch.zeros(cap, dtype=torch.uint8, device="cuda")
    s = binding.IsingSearch.from_workload(w)
    s.set_trace(feat.data_ptr(), lab.data_ptr(), cap, pairs_per_state=24, rate=1.0, seed=3)
    seen = 0
    checked = positives = 0
    for t in range(100):
        bb, bE, bf = s.get_search(0)
        active = s.step()
        ab, aE, af = s.get_search(0)
        cnt = s.trace_count()
        assert cnt <= cap
        F = feat[seen:cnt].cpu().numpy()
        Y = lab[seen:cnt].cpu().numpy()
        seen = cnt
        new = {bytes(ab[k].tobytes()) for k in range(len(ab)) if af[k]}
        # every sample's features identify (parent, pair) among the expanded states; its label
        # must say whether that child is a new member of the next kept set
        table = {}
        for p in np.nonzero(bf)[0]:
            Xf, ii, jj = mlp.pair_features(inst.J, inst.h, bb[p])
            key = np.round(Xf.astype(np.float32).astype(np.float64), 9)
            for r in range(len(ii)):
                table.setdefault(tuple(key[r]), []).append((p, ii[r], jj[r]))
        for r in range(len(F)):
            hits = table.get(tuple(np.round(F[r].astype(np.float64), 9)))
            assert hits, f"step {t + 1}: sample {r} matches no pair of an expanded state"
            p, i, j = hits[0]
            y = bb[p].copy()
            y[i >> 6] ^= np.uint64(1) << np.uint64(i & 63)
            y[j >> 6] ^= np.uint64(1) << np.uint64(j & 63)
            assert bool(Y[r]) == (bytes(y.tobytes()) in new), f"step {t + 1}: sample {r} label"
            checked += 1
            positives += int(Y[r])
        if active == 0:
            break
    s.destroy()
    note(f"[trace] {checked} samples checked, {positives} positive")
    assert checked > 100 and positives > 0


# ---------------------------------------------------------------- what the trained network gains
def _miss_rates(w, scorer, params, topk=8, steps=6):
    """Per ranked step: |S_full \\ S_ranked| / |S_full|, S_full the exact step of the
    same parents from the same S_t (oracle)."""
    s = binding.IsingSearch.from_workload(w, form=binding.FORM_LEARNED, topk_factor=topk)
    s.set_scorer(scorer, params, seed=17)
    S = w.L * len(w.instances)
    miss = []
    for t in range(steps):
        before = [s.get_search(k) for k in range(S)]
        s.step()
        for k in range(S):
            bb, bE, bf = before[k]
            if bf.sum() == 0:
                continue
            inst = w.instances[k // w.L]
            ob, _, _, _ = oracle.step(inst.J, inst.h, w.M, bb, bE, bf)
            gb, _, _ = s.get_search(k)
            got = {bytes(x.tobytes()) for x in gb}
            miss.append(np.mean([bytes(x.tobytes()) not in got for x in ob]))
    st = s.stats()
    s.destroy()
    return float(np.mean(miss)), st


def test_trained_network_gains_over_an_untrained_ranking():
    torch = torch_mod()
    train = wl.custom([100] * 6, L=6, M=32, seed_offset=310)
    held = wl.custom([100] * 2, L=4, M=32, seed_offset=320)
    cap = 1 << 21
    feat = torch.zeros((cap, 4), dtype=torch.float32, device="cuda")
    lab = torch.zeros(cap, dtype=torch.uint8, device="cuda")
    s = binding.IsingSearch.from_workload(train)
    s.set_trace(feat.data_ptr(), lab.data_ptr(), cap, pairs_per_state=64, rate=1.0, seed=4)
    s.run()
    n = min(s.trace_count(), cap)
    s.destroy()
    y = lab[:n].cpu().numpy()
    npos = int(y.sum())
    note(f"[gain] {n} trace samples, {npos} positive")
    assert npos > 100
    P0 = random_params(11)
    dP = _dev(P0, torch.float32)
    dm = torch.zeros(mlp.NPARAM, dtype=torch.float32, device="cuda")
    dv = torch.zeros_like(dm)
    wsb = binding.mlp_workspace_bytes()
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    binding.mlp_train(dP.data_ptr(), dm.data_ptr(), dv.data_ptr(), feat.data_ptr(), lab.data_ptr(), n, 8192, 600, 0,
                      2e-3, (n - npos) / npos, 99, 0, ws.data_ptr(), wsb, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    P1 = dP.cpu().numpy()
    r_net, st_net = _miss_rates(held, binding.SCORER_NETWORK, P1)
    r_init, _ = _miss_rates(held, binding.SCORER_NETWORK, P0)
    r_uni, _ = _miss_rates(held, binding.SCORER_UNIFORM, None)
    r_fld, _ = _miss_rates(held, binding.SCORER_FIELDS, None)
    note(f"[gain] miss rate at K=8N: trained {r_net:.4f}, untrained {r_init:.4f}, uniform {r_uni:.4f}, "
         f"fields {r_fld:.4f}; exact pair evaluations {st_net['pair_evals']} of {st_net['scored_pairs']} scored")
    assert r_net < 0.5 * r_uni and r_net < r_init
    assert st_net["pair_evals"] * 4 < st_net["scored_pairs"]

"""Graph-replayed runs of several steps per graph, and the retry path of a
full candidate buffer, through the C ABI: the kept sets, step counts and
merged results must be those of eager single steps (and of the oracle)."""
import sys

import numpy as np
import pytest

import oracle
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


def same_run(w, ref_kw, kw, tag, max_iters=0, same_counts=True):
    note(f"[{tag}] Ns={sorted(set(i.N for i in w.instances))} L={w.L} M={w.M} ref={ref_kw} got={kw}")
    a = binding.IsingSearch.from_workload(w, **ref_kw)
    g = binding.IsingSearch.from_workload(w, **kw)
    ia, sa = a.run(max_iters)
    ig, sg = g.run(max_iters)
    assert (ia, sa) == (ig, sg), f"{tag}: iterations {ia, sa} vs {ig, sg}"
    for sid in range(a.B * a.L):
        ab, aE, af = a.get_search(sid)
        gb, gE, gf = g.get_search(sid)
        assert np.array_equal(ab, gb) and np.array_equal(aE, gE) and np.array_equal(af, gf), f"{tag} search {sid}"
    for b in range(a.B):
        ab, aE = a.get_states(b)
        gb, gE = g.get_states(b)
        assert np.array_equal(ab, gb) and np.array_equal(aE, gE), f"{tag} instance {b}"
    st_a, st_g = a.stats(), g.stats()
    assert st_a["steps"] == st_g["steps"], (st_a, st_g)
    # a re-scan counts its pairs again, and which candidates a full buffer
    # stored (hence how many re-scans a step takes) follows the atomics' order
    if same_counts:
        assert st_a["pair_evals"] == st_g["pair_evals"], (st_a, st_g)
    note(f"[{tag}] ok: {ig} steps, retries {st_g['retries']}")
    a.destroy()
    g.destroy()
    return st_g


@pytest.mark.parametrize("k", [2, 8, 64])
def test_graph_of_k_steps_equals_eager(k):
    w = wl.custom([100, 200, 300, 64, 129, 600], L=3, M=40, config=71)
    same_run(w, {}, {"persistent": 1, "graph_steps": k}, f"graph k={k}")


@pytest.mark.parametrize("form,flags", [(binding.FORM_PLAIN, 0), (binding.FORM_SPLIT_BF16, binding.FLAG_FP16_SCAN),
                                        (binding.FORM_SPLIT_BF16, binding.FLAG_SITE_BOUND)])
def test_graph_with_full_buffers(form, flags):
    """Candidate buffers of 128 records (M = 60): searches overflow, the graph
    halts on the device, the host finishes the step with retry passes (and
    larger buffers) and the run goes on."""
    w = wl.custom([200, 300], L=4, M=60, config=72)
    st = same_run(w, {"form": form, "flags": flags, "surv_capacity": 128},
                  {"form": form, "flags": flags, "surv_capacity": 128, "persistent": 1, "graph_steps": 8},
                  f"full buffers form={form} flags={flags}", same_counts=False)
    assert st["retries"] > 0


@pytest.mark.parametrize("scorer", [binding.SCORER_FIELDS, binding.SCORER_NETWORK])
def test_learned_form_in_graphs_of_k_steps(scorer):
    """The learned form's ranked and full steps switch on the device, so a
    graph of several steps holds both kinds."""
    w = wl.custom([90, 150], L=3, M=30, config=76)
    params = wl.network_params(5).astype(np.float32)
    runs = []
    for kw in ({}, {"persistent": 1, "graph_steps": 8}):
        s = binding.IsingSearch.from_workload(w, form=binding.FORM_LEARNED, **kw)
        s.set_scorer(scorer, params if scorer == binding.SCORER_NETWORK else None, seed=3)
        it = s.run()
        runs.append((it, [s.get_search(k) for k in range(s.B * s.L)], s.stats()))
        s.destroy()
    (ia, sa, sta), (ig, sg, stg) = runs
    assert ia == ig
    for k, (a, g) in enumerate(zip(sa, sg)):
        assert all(np.array_equal(x, y) for x, y in zip(a, g)), f"search {k}"
    assert sta["steps"] == stg["steps"] and sta["fallbacks"] == stg["fallbacks"]
    assert sta["scored_pairs"] == stg["scored_pairs"]


def test_graph_respects_the_step_cap():
    w = wl.custom([150, 250], L=2, M=50, config=73)
    for cap in (3, 13, 20):
        same_run(w, {}, {"persistent": 1, "graph_steps": 8}, f"cap {cap}", max_iters=cap)


@pytest.mark.parametrize("N,form,flags", [(200, binding.FORM_PLAIN, 0), (200, binding.FORM_SPLIT_BF16, 0),
                                          (300, binding.FORM_PLAIN, binding.FLAG_SITE_BOUND),
                                          (120, binding.FORM_SPLIT_BF16, binding.FLAG_FP16_SCAN)])
def test_retry_path_against_the_oracle(N, form, flags):
    """Every step of every search against the oracle, with buffers so small
    that the retry path runs (a full buffer re-scanned with the cut its stored
    candidates give, or doubled when that cut cannot move)."""
    w = wl.custom([N], L=3, M=60, config=74, seed_offset=N + form)
    note(f"[retry] N={N} form={form} flags={flags}")
    s = binding.IsingSearch.from_workload(w, form=form, flags=flags, surv_capacity=128)
    inst = w.instances[0]
    trajs = []
    for x0 in inst.init_bits:
        bits, E, front = x0.reshape(1, -1), None, np.ones(1, np.uint8)
        tr = []
        while True:
            ob, oE, of, n_new = oracle.step(inst.J, inst.h, w.M, bits, E, front, fields=True)
            tr.append((ob, oE, of))
            if n_new == 0:
                break
            bits, E, front = ob, oE, of
        trajs.append(tr)
    for t in range(max(len(tr) for tr in trajs)):
        s.step()
        for l, tr in enumerate(trajs):
            ob, oE, of = tr[min(t, len(tr) - 1)]
            gb, gE, gf = s.get_search(l)
            assert np.array_equal(gb, ob) and np.array_equal(gE, oE), f"search {l} step {t + 1}"
            if t < len(tr):
                assert np.array_equal(gf.astype(bool), of.astype(bool)), f"search {l} step {t + 1}: flags"
    st = s.stats()
    note(f"[retry] retries {st['retries']}")
    assert st["retries"] > 0
    s.destroy()


def test_small_buffers_are_validated():
    w = wl.custom([40], L=2, M=200, config=75)
    for cap in (50, 399, (1 << 24) + 1):
        with pytest.raises(binding.IsingError):
            binding.IsingSearch.from_workload(w, surv_capacity=cap)
    with pytest.raises(binding.IsingError):
        binding.IsingSearch.from_workload(w, persistent=1, graph_steps=65)


def test_buffer_grows_when_the_cut_cannot_move():
    """128 records for M = 60: the stored candidates are mostly copies of
    states already kept, the cut cannot move, the buffer doubles and the step
    finishes; the run equals one with the default buffer."""
    w = wl.custom([200, 300], L=2, M=60, config=72)
    st = same_run(w, {}, {"surv_capacity": 128}, "growth", same_counts=False)
    assert st["retries"] > 0 and st["surv_capacity"] > 128
    st = same_run(w, {}, {"surv_capacity": 128, "persistent": 1, "graph_steps": 8}, "growth, graph",
                  same_counts=False)
    assert st["retries"] > 0 and st["surv_capacity"] > 128

"""Oracle parity at the measured sizes (N = 600 and N = 1000, M = 120), for
every form, through the C ABI.

At selected steps of sampled searches the oracle takes one step of the
Sec. II iteration from exactly the kept set the GPU holds (its bitstrings and
energies), expanding every kept state, and the GPU's next kept set must equal
the oracle's bit for bit: bitstrings, order, energies and new-state flags.
The GPU expands only the states that entered in the previous step, so the
check also fails when that previous step went wrong.  The steps checked are
the first three, every 20th, and for every sampled search the last step that
brought a new state and the step that found none; some searches are checked
at every step (the oracle then expands the new states only).  At the end
every sampled search must be a fixed point of the exact step (the oracle's
literal step from its final set brings nothing), and every instance's
merged result must be the Alg. 4 merge of the GPU's final sets.  The oracle
steps with its local-field energy changes, which the CPU pins tie to Eq. 1.

The learned form is checked the same way with its recorded proposals: a
ranking step against the oracle's step over S_t, the single flips of the
ranked states and the proposed pairs; a full step against the exact step.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2010_00180_amd import binding, workloads as wl

pytestmark = pytest.mark.gpu

PLAIN, SPLIT, LEARNED = binding.FORM_PLAIN, binding.FORM_SPLIT_BF16, binding.FORM_LEARNED
SB, F16, REC = binding.FLAG_SITE_BOUND, binding.FLAG_FP16_SCAN, binding.FLAG_RECORD_PROPOSALS


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


def same(g, o, what):
    gb, gE, gf = g
    ob, oE, of = o[0], o[1], o[2]
    assert gb.shape == ob.shape, f"{what}: count {gb.shape} vs {ob.shape}"
    assert np.array_equal(gb, ob), f"{what}: bitstrings differ"
    assert np.array_equal(gE, oE), f"{what}: energies differ (max {np.max(np.abs(gE - oE))})"
    assert np.array_equal(gf.astype(bool), of.astype(bool)), f"{what}: new-state flags differ"


def index_of_states(bits):
    return {bytes(np.ascontiguousarray(b).tobytes()): k for k, b in enumerate(bits)}


def oracle_next(s, inst, M, before, sid, learned, literal=True, h1=0):
    """The oracle's step from the GPU's set `before` of search sid; for the
    learned form, from the proposals the GPU recorded in its last step."""
    bb, bE, bf = before
    if not learned:
        return oracle.step(inst.J, inst.h, M, bb, bE, bf, literal=literal, fields=True, h1=h1)
    mode, props = s.get_proposals(sid)
    if mode == 1:
        return oracle.step(inst.J, inst.h, M, bb, bE, literal=True, fields=True)
    where = index_of_states(bb)
    par = [where[bytes(np.ascontiguousarray(p).tobytes())] for p, _ in props]
    assert sorted(par) == list(np.nonzero(bf)[0]), f"search {sid}: ranked parents are not the new states"
    return oracle.step_proposed(inst.J, inst.h, M, bb, bE, par, [c for _, c in props], fields=True)


def large_parity(w, tag, checked, every=(), cap=3000, scorer=None, params=None, autotune=False, h1=0, **kw):
    """Step a handle to the end; check the sampled searches against the oracle
    at the selected steps (the searches in `every` at every step); return the
    handle's statistics."""
    learned = kw.get("form") == LEARNED
    if learned:
        kw["flags"] = kw.get("flags", 0) | REC
    checked = sorted(set(checked) | set(every))
    note(f"[{tag}] Ns={sorted(set(i.N for i in w.instances))} B={len(w.instances)} L={w.L} M={w.M} "
          f"checked={checked} every step={list(every)} {kw}")
    s = binding.IsingSearch.from_workload(w, **kw)
    if learned:
        s.set_scorer(scorer, params, seed=23)
    hist = {k: [None, s.get_search(k)] for k in checked}   # the sets after steps t-2 and t-1
    last_checked = {k: 0 for k in checked}
    stable_at = {}
    n_checks = 0
    for t in range(1, cap + 1):
        if autotune and t == 2:
            active = s.autotune()
        else:
            active = s.step()
        for k in checked:
            inst = w.instances[k // w.L]
            after = s.get_search(k)
            prev, before = hist[k]
            if k in stable_at:
                assert np.array_equal(after[0], before[0]) and np.array_equal(after[1], before[1]), \
                    f"{tag} search {k} step {t}: moved after stopping"
                continue
            stops = not after[2].any()
            if k in every:
                o = oracle_next(s, inst, w.M, before, k, learned, literal=False, h1=h1)
                same(after, o, f"{tag} search {k} step {t}")
                n_checks += 1
            elif t <= 3 or t % 20 == 0 or stops:
                if stops and not learned and last_checked[k] < t - 1 and prev is not None:
                    # the last step that brought new states
                    same(before, oracle_next(s, inst, w.M, prev, k, False, h1=h1), f"{tag} search {k} step {t - 1}")
                    n_checks += 1
                o = oracle_next(s, inst, w.M, before, k, learned, h1=h1)
                same(after, o, f"{tag} search {k} step {t}")
                last_checked[k] = t
                n_checks += 1
                if stops and not learned:
                    assert o[3] == 0
            if stops and (not learned or s.get_proposals(k)[0] == 1):
                stable_at[k] = t
            hist[k] = [before, after]
        if active == 0:
            break
    assert active == 0, f"{tag}: searches still running after {cap} steps"
    # the fixed-point certificate of every sampled search
    for k in checked:
        inst = w.instances[k // w.L]
        gb, gE, _ = s.get_search(k)
        _, _, _, nn = oracle.step(inst.J, inst.h, w.M, gb, gE, literal=True, fields=True, h1=h1)
        assert nn == 0, f"{tag} search {k}: final set is not a fixed point of the exact step"
    # the Alg. 4 merge of every instance from the GPU's final sets
    for b, inst in enumerate(w.instances):
        lists = []
        for l in range(w.L):
            gb, gE, _ = s.get_search(b * w.L + l)
            lists.append((gb, gE))
        mb, mE = oracle.merge(inst.N, w.M, lists)
        gb, gE = s.get_states(b)
        assert np.array_equal(gb, mb) and np.array_equal(gE, mE), f"{tag} instance {b}: merge"
    st = s.stats()
    note(f"[{tag}] ok: {t} steps, {n_checks} oracle steps compared, stable at {sorted(stable_at.values())[-3:]}, "
          f"pairs {st['pair_evals']:.3e}, bounded {st['bounded_states']}, re-score rejections {st['fallbacks']}")
    s.destroy()
    return st


def sample(w, n, seed):
    rng = np.random.default_rng(seed)
    return sorted(int(x) for x in rng.choice(w.n_searches, n, replace=False))


# the forms of the plain and split paths: (form, flags, persistent)
FORMS = {
    "plain": (PLAIN, 0, 0),
    "split_fp32": (SPLIT, 0, 0),
    "split_fp16": (SPLIT, F16, 0),
    "plain_bound": (PLAIN, SB, 0),
    "split_fp32_bound": (SPLIT, SB, 0),
    "split_fp16_bound": (SPLIT, SB | F16, 0),
    "plain_graph": (PLAIN, 0, 1),
    "split_fp16_graph": (SPLIT, F16, 1),
}


@pytest.mark.parametrize("name", list(FORMS))
def test_n600_m120_every_form(name):
    """Two instances of the N = 600, M = 120, L = 64 workload (128 searches), six sampled."""
    form, flags, persistent = FORMS[name]
    w = wl.c3_n600(n_instances=2)
    every = [70] if name in ("plain", "split_fp16") else []
    large_parity(w, f"n600 {name}", sample(w, 6, 600), every=every, form=form, flags=flags, persistent=persistent)


@pytest.mark.parametrize("name", ["plain", "split_fp32", "split_fp16", "split_fp32_bound", "plain_graph"])
def test_n1000_m120(name):
    """N = 1000 (sixteen words per state), M = 120, L = 8, four sampled searches."""
    form, flags, persistent = FORMS[name]
    w = wl.c5_learned(1000, n_instances=1, L=8)
    every = [5] if name == "plain" else []
    large_parity(w, f"n1000 {name}", sample(w, 4, 1000), every=every, form=form, flags=flags,
                 persistent=persistent)


@pytest.mark.parametrize("name", ["plain", "split_fp32", "split_fp16", "plain_bound", "split_fp16_bound"])
def test_ragged_sizes_past_the_round_boundaries(name):
    """Sizes just past the preparation's rounds of 384 and 512 sites, the
    frontier's 512-site blocks, 640 (the site bound's register copy) and 1024,
    every search checked."""
    form, flags, persistent = FORMS[name]
    w = wl.custom([385, 513, 641, 1025], L=2, M=120, config=41)
    large_parity(w, f"ragged {name}", list(range(w.n_searches)), form=form, flags=flags, persistent=persistent)


def test_uneven_batch_autotuned_graph_sampled_above_n300():
    """A batch shaped like the 480-instance uneven workload (N from 100 to 600,
    L = 32, M = 120), graph-replayed and autotuned after its first step; eight
    searches of instances with N >= 300 checked."""
    w = wl.c4_uneven(n_instances=24, L=32)
    big = [b for b, inst in enumerate(w.instances) if inst.N >= 300]
    rng = np.random.default_rng(4)
    checked = sorted(int(b) * w.L + int(rng.integers(w.L)) for b in rng.choice(big, 8, replace=False))
    note(f"[c4] N of the checked searches: {[w.instances[k // w.L].N for k in checked]}")
    large_parity(w, "c4 graph autotuned", checked, form=PLAIN, persistent=1, autotune=True)


@pytest.mark.parametrize("N,scorer", [(600, binding.SCORER_NETWORK), (600, binding.SCORER_FIELDS),
                                      (1000, binding.SCORER_NETWORK)])
def test_learned_at_measured_sizes(N, scorer):
    """The learned form at N = 600 and N = 1000 (K = 8N proposals per state),
    L = 4, every search checked at the selected steps with its recorded
    proposals; the final sets certified as fixed points of the exact step."""
    w = wl.c5_learned(N, n_instances=1, L=4)
    params = wl.network_params(7).astype(np.float32) if scorer == binding.SCORER_NETWORK else None
    large_parity(w, f"learned n{N} scorer {scorer}", list(range(w.n_searches)), form=LEARNED, scorer=scorer,
                 params=params)


@pytest.mark.parametrize("N,M,L", [(100, 600, 2), (64, 1024, 2), (300, 600, 2)])
def test_large_kept_sets(N, M, L):
    """Kept sets of 600 and 1024 states (the merge's multi-pass sort, the
    frontier's widened pool prefix), every search checked."""
    w = wl.custom([N], L=L, M=M, config=42, seed_offset=N + M)
    large_parity(w, f"M={M} N={N}", list(range(w.n_searches)), every=[0])

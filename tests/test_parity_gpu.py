"""Parity of the HIP path with the CPU oracle, through the C ABI.

Every comparison is exact: with J and h on the 2^-24 grid all energies are
exact in FP64, so kept bitstrings, their order and their energies must be
identical (this is stricter than the 1e-9 relative energy tolerance asked of
the method).  Small cases are compared at every step; the full-size workload
is compared on sampled searches and on properties that hold at any size.
"""
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


def oracle_trajectory(inst, M, x0, max_steps=10000):
    """Kept sets after each step, from the oracle's own step function."""
    bits = np.asarray(x0, np.uint64).reshape(1, -1)
    E, front = None, np.ones(1, np.uint8)
    traj = []
    for _ in range(max_steps):
        ob, oE, of, n_new = oracle.step(inst.J, inst.h, M, bits, E, front)
        traj.append((ob, oE, of))
        if n_new == 0:
            break
        bits, E, front = ob, oE, of
    return traj


def assert_same_set(g, o, what):
    gb, gE, gf = g
    ob, oE, of = o
    assert gb.shape == ob.shape, f"{what}: count {gb.shape} vs {ob.shape}"
    assert np.array_equal(gb, ob), f"{what}: bitstrings differ"
    assert np.array_equal(gE, oE), f"{what}: energies differ (max {np.max(np.abs(gE - oE))})"
    assert np.array_equal(gf.astype(bool), of.astype(bool)), f"{what}: new-state flags differ"


def stepwise_parity(w, tag, **kw):
    note(f"[{tag}] Ns={[i.N for i in w.instances]} L={w.L} M={w.M} {kw}")
    s = binding.IsingSearch.from_workload(w, **kw)
    trajs = {}
    for b, inst in enumerate(w.instances):
        for l in range(w.L):
            trajs[b * w.L + l] = oracle_trajectory(inst, w.M, inst.init_bits[l])
    nsteps = max(len(t) for t in trajs.values())
    for t in range(nsteps):
        active = s.step()
        for sid, traj in trajs.items():
            o = traj[min(t, len(traj) - 1)]
            assert_same_set(s.get_search(sid), o if t < len(traj) else (o[0], o[1], np.zeros_like(o[2])),
                            f"{tag} search {sid} step {t + 1}")
        want_active = sum(1 for traj in trajs.values() if t + 1 < len(traj))
        assert active == want_active, f"{tag} step {t + 1}: {active} active, oracle {want_active}"
    assert s.step() == 0
    for b, inst in enumerate(w.instances):
        lists = [(trajs[b * w.L + l][-1][0], trajs[b * w.L + l][-1][1]) for l in range(w.L)]
        mb, mE = oracle.merge(inst.N, w.M, lists)
        gb, gE = s.get_states(b)
        assert np.array_equal(gb, mb) and np.array_equal(gE, mE), f"{tag} instance {b} merge"
    st = s.stats()
    s.destroy()
    return st


def test_c1_n24_stepwise_and_brute_force():
    w = wl.c1_n24()
    st = stepwise_parity(w, "c1")
    assert st["pair_evals"] > 0
    inst = w.instances[0]
    bb, bE = oracle.brute_lowest(inst.J, inst.h, w.M)
    s = binding.IsingSearch.from_workload(w)
    s.run()
    gb, gE = s.get_states(0)
    # the search never reports an energy below the true k-th lowest
    assert np.all(gE >= bE[: len(gE)])
    note(f"c1: found ground state {gE[0] == bE[0]}; lowest kept {gE[:3]}, exact {bE[:3]}")
    s.destroy()


@pytest.mark.parametrize("N,M,L", [(1, 1, 2), (2, 3, 2), (3, 8, 2), (5, 40, 2), (24, 1, 3), (63, 7, 2),
                                   (64, 40, 2), (65, 120, 2), (100, 17, 2), (130, 60, 1), (200, 120, 1)])
def test_sizes_stepwise(N, M, L):
    w = wl.custom([N], L=L, M=M, config=11, seed_offset=N * 7 + M)
    stepwise_parity(w, f"size N={N} M={M}")


@pytest.mark.parametrize("dist", ["pmj", "sk_h0", "uniform"])
def test_ties_and_symmetry_stepwise(dist):
    w = wl.custom([40, 70], L=2, M=50, config=12, dist=dist)
    stepwise_parity(w, f"ties {dist}")


@pytest.mark.parametrize("form,flags", [(binding.FORM_PLAIN, 0), (binding.FORM_SPLIT_BF16, 0),
                                        (binding.FORM_PLAIN, binding.FLAG_SITE_BOUND),
                                        (binding.FORM_SPLIT_BF16, binding.FLAG_SITE_BOUND)])
def test_wide_fields_stepwise(form, flags):
    """Fields beyond 2^31 units of the 2^-24 grid: the library holds them in
    FP64 instead of 32-bit integers; with them an instance of +-1 couplings
    (grid 1, fields up to N), held as integers."""
    w = wl.custom([60, 130], L=2, M=40, config=13, dist="wide")
    st = stepwise_parity(w, f"wide fields form={form} flags={flags}", form=form, flags=flags)
    assert st["field_bytes"] == 8
    w = wl.custom([150], L=2, M=40, config=14, dist="pmj")
    st = stepwise_parity(w, f"integer fields form={form} flags={flags}", form=form, flags=flags)
    assert st["field_bytes"] == 4
    w = wl.custom([60], L=2, M=40, config=13, dist="wide")   # this one alone fits
    st = stepwise_parity(w, f"fitting fields form={form} flags={flags}", form=form, flags=flags)
    assert st["field_bytes"] == 4


def test_uneven_sizes_one_handle():
    w = wl.custom([5, 64, 65, 100, 129], L=2, M=30, config=13)
    stepwise_parity(w, "uneven")


@pytest.mark.parametrize("sc", [1, 7, 64, 200])
def test_tile_configuration_does_not_change_results(sc):
    w = wl.custom([90, 150], L=3, M=40, config=14)
    stepwise_parity(w, f"sc={sc}", states_per_item=sc)


def test_checkpoint_restore_continues_identically():
    w = wl.custom([80, 120], L=3, M=30, config=15)
    note("[checkpoint]")
    a = binding.IsingSearch.from_workload(w)
    for _ in range(3):
        a.step()
    b = binding.IsingSearch.from_workload(w)
    for sid in range(a.B * a.L):
        bits, E, fr = a.get_search(sid)
        b.set_search(sid, bits, fr)
        gb, gE, gf = b.get_search(sid)
        assert np.array_equal(gb, bits) and np.array_equal(gE, E) and np.array_equal(gf, fr)
    a.run()
    b.run()
    for sid in range(a.B * a.L):
        assert_same_set(b.get_search(sid), a.get_search(sid), f"restored search {sid}")
    a.destroy()
    b.destroy()


def test_iteration_cap_reports_not_converged():
    w = wl.custom([150], L=2, M=60, config=16)
    s = binding.IsingSearch.from_workload(w)
    it, stable = s.run(max_iters=2)
    assert it == 2 and not stable
    it2, stable2 = s.run()
    assert stable2
    trajs = [oracle_trajectory(w.instances[0], w.M, x) for x in w.instances[0].init_bits]
    assert it + it2 == max(len(t) for t in trajs)
    for l in range(2):
        assert_same_set(s.get_search(l), (trajs[l][-1][0], trajs[l][-1][1], np.zeros_like(trajs[l][-1][2])),
                        f"cap search {l}")
    s.destroy()


def test_c2_full_size_sampled():
    """120 instances, N=200, L=16, M=120, as the benchmark runs them."""
    w = wl.c2_n200()
    note("[c2] full workload")
    s = binding.IsingSearch.from_workload(w)
    it, stable = s.run()
    assert stable
    note(f"[c2] steps={it} stats={s.stats()}")
    rng = np.random.default_rng(2)
    for sid in rng.choice(w.n_searches, 2, replace=False):
        b, l = divmod(int(sid), w.L)
        inst = w.instances[b]
        ob, oE, oit, ostable = oracle.search(inst.J, inst.h, w.M, inst.init_bits[l])
        gb, gE, gf = s.get_search(int(sid))
        assert np.array_equal(gb, ob) and np.array_equal(gE, oE), f"c2 search {sid}"
        assert oit <= it
    for b in rng.choice(len(w.instances), 4, replace=False):
        inst = w.instances[b]
        gb, gE = s.get_states(int(b))
        assert len(gE) == w.M
        assert np.all(np.diff(gE) >= 0)
        assert len({tuple(r) for r in gb}) == len(gb)
        for k in rng.choice(len(gE), 5, replace=False):
            assert oracle.energy(inst.J, inst.h, gb[k]) == gE[k]
    s.destroy()


def test_reset_repeats_the_search_exactly():
    w = wl.custom([100, 140], L=3, M=40, config=17)
    note("[reset]")
    s = binding.IsingSearch.from_workload(w)
    it1, st1 = s.run()
    first = [s.get_search(k) for k in range(s.B * s.L)]
    fm = [s.get_states(b) for b in range(s.B)]
    s.reset()
    it2, st2 = s.run()
    assert (it1, st1) == (it2, st2)
    for k in range(s.B * s.L):
        assert_same_set(s.get_search(k), first[k], f"reset search {k}")
    for b in range(s.B):
        gb, gE = s.get_states(b)
        assert np.array_equal(gb, fm[b][0]) and np.array_equal(gE, fm[b][1])
    s.destroy()


def test_persistent_graph_replays_match_eager_every_step():
    """Uneven N in one handle; the graph replay of a step must equal the eager
    launches after every replay (eager copies and synchronizations between)."""
    w = wl.custom([100, 200, 300, 64, 129, 600], L=3, M=40, config=18)
    note("[graph] uneven N, persistent vs eager")
    a = binding.IsingSearch.from_workload(w)
    g = binding.IsingSearch.from_workload(w, persistent=1)
    for t in range(400):
        na = a.step()
        ng = g.step()
        assert na == ng, f"step {t + 1}: active {na} vs {ng}"
        for sid in range(a.B * a.L):
            assert_same_set(g.get_search(sid), a.get_search(sid), f"graph search {sid} step {t + 1}")
        if na == 0:
            break
    assert na == 0
    for b in range(a.B):
        ab, aE = a.get_states(b)
        gb, gE = g.get_states(b)
        assert np.array_equal(ab, gb) and np.array_equal(aE, gE)
    # the small instances against the oracle
    for b in (3, 4):
        inst = w.instances[b]
        for l in range(w.L):
            ob, oE, _, _ = oracle.search(inst.J, inst.h, w.M, inst.init_bits[l])
            gb, gE, _ = g.get_search(b * w.L + l)
            assert np.array_equal(gb, ob) and np.array_equal(gE, oE)
    a.destroy()
    g.destroy()


def test_autotune_keeps_results_and_picks_candidates():
    w = wl.custom([100, 300, 100, 500], L=4, M=60, config=19)
    note("[autotune]")
    a = binding.IsingSearch.from_workload(w)
    t = binding.IsingSearch.from_workload(w, persistent=1)
    a.step()
    t.step()
    a.step()
    t.autotune()
    tiles = t.tuning()
    # tuned per N, or the per-step choice (one power of two for all) if faster
    assert all(x in (16, 32, 64, 128, 256) for x in tiles)
    assert tiles[0] == tiles[2]   # same N, same choice
    a.run()
    t.run()
    for sid in range(a.B * a.L):
        assert_same_set(t.get_search(sid), a.get_search(sid), f"autotuned search {sid}")
    a.destroy()
    t.destroy()


@pytest.mark.parametrize("form,flags", [(binding.FORM_PLAIN, 0), (binding.FORM_SPLIT_BF16, 0),
                                        (binding.FORM_SPLIT_BF16, binding.FLAG_FP16_SCAN)])
def test_states_per_item_chosen_per_step(form, flags):
    """With states_per_item 0 every step picks a power of two in [16, 256] from
    its work; the kept sets match those of a fixed 64 step by step."""
    # enough work that a full frontier leaves every scan wave 16 items of 32 states
    w = wl.custom([600] * 40 + [300] * 8, L=32, M=60, config=27)
    note(f"[states per item] form={form} flags={flags}")
    a = binding.IsingSearch.from_workload(w, states_per_item=64, form=form, flags=flags)
    c = binding.IsingSearch.from_workload(w, form=form, flags=flags)
    seen = set()
    for t in range(600):
        na = a.step()
        nc = c.step()
        assert na == nc, f"step {t + 1}: active {na} vs {nc}"
        tiles = c.tuning()
        assert len(set(tiles)) == 1 and tiles[0] in (16, 32, 64, 128, 256), tiles
        seen.add(tiles[0])
        if t % 25 == 0:
            for sid in range(0, a.B * a.L, 97):
                assert_same_set(c.get_search(sid), a.get_search(sid), f"search {sid} step {t + 1}")
        if na == 0:
            break
    assert na == 0
    assert max(seen) > 16 and min(seen) < max(seen), seen   # the choice follows the work
    for b in range(a.B):
        ab, aE = a.get_states(b)
        cb, cE = c.get_states(b)
        assert np.array_equal(ab, cb) and np.array_equal(aE, cE), f"instance {b}"
    a.destroy()
    c.destroy()


def test_uneven_batch_persistent_sampled():
    """A reduced batch shaped like the 480-instance uneven workload (N drawn from
    100..600, L=32, M=120), persistent and autotuned, sampled against the oracle."""
    w = wl.c4_uneven(n_instances=48, L=32)
    note(f"[c4-shaped] sizes={sorted(set(i.N for i in w.instances))}")
    s = binding.IsingSearch.from_workload(w, persistent=1)
    s.step()
    s.autotune()
    it, stable = s.run()
    assert stable
    rng = np.random.default_rng(4)
    small = [b for b, inst in enumerate(w.instances) if inst.N == 100]
    for b in rng.choice(small, 2, replace=False):
        inst = w.instances[int(b)]
        l = int(rng.integers(w.L))
        ob, oE, _, _ = oracle.search(inst.J, inst.h, w.M, inst.init_bits[l])
        gb, gE, _ = s.get_search(int(b) * w.L + l)
        assert np.array_equal(gb, ob) and np.array_equal(gE, oE)
    for b in rng.choice(len(w.instances), 6, replace=False):
        inst = w.instances[int(b)]
        gb, gE = s.get_states(int(b))
        assert len(gE) == w.M and np.all(np.diff(gE) >= 0)
        assert len({tuple(r) for r in gb}) == len(gb)
        for k in rng.choice(len(gE), 3, replace=False):
            assert oracle.energy(inst.J, inst.h, gb[k]) == gE[k]
    s.destroy()


# ---------------------------------------------------------------- split-bf16 form
def ebf_bound(inst):
    """The bound on |F~ - F| that the library uses for the bf16 hi+lo fields."""
    R = np.abs(inst.J).sum(axis=1)
    n = inst.N
    return float(np.max((2.0 ** -15 + 2.1 * n * 2.0 ** -24) * R + 2.0 ** -23 * (np.abs(inst.h) + R)))


@pytest.mark.parametrize("N,M,L,dist", [(24, 8, 4, "sk"), (65, 40, 2, "sk"), (130, 60, 2, "sk"),
                                        (200, 120, 1, "sk"), (70, 50, 2, "pmj"), (90, 30, 2, "sk_h0")])
def test_split_form_stepwise(N, M, L, dist):
    w = wl.custom([N], L=L, M=M, config=21, dist=dist, seed_offset=N + M)
    st = stepwise_parity(w, f"split N={N} {dist}", form=binding.FORM_SPLIT_BF16)
    assert 0.0 <= st["split_field_err"] <= ebf_bound(w.instances[0])


def test_split_form_matches_plain_full_c2():
    w = wl.c2_n200()
    note("[split c2] plain vs split")
    a = binding.IsingSearch.from_workload(w)
    s = binding.IsingSearch.from_workload(w, form=binding.FORM_SPLIT_BF16)
    ia, _ = a.run()
    is_, _ = s.run()
    assert ia == is_
    for sid in range(0, w.n_searches, 7):
        assert_same_set(s.get_search(sid), a.get_search(sid), f"split c2 search {sid}")
    for b in range(len(w.instances)):
        ab, aE = a.get_states(b)
        sb, sE = s.get_states(b)
        assert np.array_equal(ab, sb) and np.array_equal(aE, sE)
    st = s.stats()
    note(f"[split c2] field err {st['split_field_err']:.3e} bound {max(ebf_bound(i) for i in w.instances):.3e} "
         f"re-scored and rejected {st['fallbacks']}")
    assert 0.0 < st["split_field_err"] <= max(ebf_bound(i) for i in w.instances)
    a.destroy()
    s.destroy()


# ---------------------------------------------------------------- site bound
# Pair flips whose two sites cannot both satisfy a_i + min a - max_k |4J_ik| <= T
# are skipped; the kept sets must stay those of the full scan (and the oracle's).
@pytest.mark.parametrize("form", [binding.FORM_PLAIN, binding.FORM_SPLIT_BF16])
@pytest.mark.parametrize("N,M,L,dist", [(24, 8, 4, "sk"), (65, 40, 2, "sk"), (130, 60, 2, "sk"),
                                        (200, 120, 1, "sk"), (70, 50, 2, "pmj"), (90, 30, 2, "sk_h0")])
def test_site_bound_stepwise(form, N, M, L, dist):
    w = wl.custom([N], L=L, M=M, config=23, dist=dist, seed_offset=N + 3 * M)
    st = stepwise_parity(w, f"site bound form={form} N={N} {dist}", form=form, flags=binding.FLAG_SITE_BOUND)
    note(f"  bounded {st['bounded_states']} of {st['frontier_states']} states, pairs {st['pair_evals']}")
    assert st["bounded_states"] > 0
    assert st["pair_evals"] < st["frontier_states"] * N * (N - 1) // 2


def test_site_bound_uneven_and_tiles():
    w = wl.custom([5, 64, 65, 100, 129], L=2, M=30, config=24)
    stepwise_parity(w, "site bound uneven sc=7", flags=binding.FLAG_SITE_BOUND, states_per_item=7)


def test_site_bound_matches_full_scan_c2():
    """120 instances, N=200, L=16, M=120: every search and every merged set equal
    with and without the bound, for both forms; fewer pairs evaluated."""
    w = wl.c2_n200()
    for form in (binding.FORM_PLAIN, binding.FORM_SPLIT_BF16):
        note(f"[site bound c2] form {form}")
        a = binding.IsingSearch.from_workload(w, form=form)
        s = binding.IsingSearch.from_workload(w, form=form, flags=binding.FLAG_SITE_BOUND)
        ia, _ = a.run()
        is_, stable = s.run()
        assert stable and ia == is_
        for sid in range(w.n_searches):
            assert_same_set(s.get_search(sid), a.get_search(sid), f"site bound c2 search {sid}")
        for b in range(len(w.instances)):
            ab, aE = a.get_states(b)
            sb, sE = s.get_states(b)
            assert np.array_equal(ab, sb) and np.array_equal(aE, sE)
        sa, ss = a.stats(), s.stats()
        note(f"  pairs {sa['pair_evals']:.3e} -> {ss['pair_evals']:.3e}, bounded {ss['bounded_states']} of "
             f"{ss['frontier_states']}")
        assert ss["frontier_states"] == sa["frontier_states"]
        assert ss["pair_evals"] < sa["pair_evals"]
        a.destroy()
        s.destroy()


def test_site_bound_persistent_and_autotune():
    w = wl.custom([100, 200, 300, 64, 129, 600], L=3, M=40, config=25)
    note("[site bound] graph replay and autotune vs eager")
    a = binding.IsingSearch.from_workload(w)
    g = binding.IsingSearch.from_workload(w, persistent=1, flags=binding.FLAG_SITE_BOUND)
    a.step()
    g.step()
    g.autotune()
    a.step()
    for t in range(400):
        na = a.step()
        ng = g.step()
        assert na == ng, f"step {t + 3}: active {na} vs {ng}"
        for sid in range(a.B * a.L):
            assert_same_set(g.get_search(sid), a.get_search(sid), f"site bound graph search {sid} step {t + 3}")
        if na == 0:
            break
    assert na == 0
    a.destroy()
    g.destroy()


def test_site_bound_n600_sampled():
    """N=600, M=120, L=64 instances (4 of them): the split form with the bound
    against the split form without it (whose smaller cases are checked against
    the oracle step by step), energies of sampled kept states by Eq. 1."""
    w = wl.c3_n600(n_instances=4)
    note("[site bound n600] 4 instances")
    a = binding.IsingSearch.from_workload(w, form=binding.FORM_SPLIT_BF16)
    s = binding.IsingSearch.from_workload(w, form=binding.FORM_SPLIT_BF16, flags=binding.FLAG_SITE_BOUND)
    ia, _ = a.run()
    is_, stable = s.run()
    assert stable and ia == is_
    for sid in range(w.n_searches):
        assert_same_set(s.get_search(sid), a.get_search(sid), f"site bound n600 search {sid}")
    for b in range(len(w.instances)):
        ab, aE = a.get_states(b)
        sb, sE = s.get_states(b)
        assert np.array_equal(ab, sb) and np.array_equal(aE, sE)
    rng = np.random.default_rng(6)
    for b in range(len(w.instances)):
        inst = w.instances[b]
        gb, gE = s.get_states(b)
        assert len(gE) == w.M and np.all(np.diff(gE) >= 0)
        for k in rng.choice(len(gE), 3, replace=False):
            assert oracle.energy(inst.J, inst.h, gb[k]) == gE[k]
    st = s.stats()
    note(f"  steps {is_}, bounded {st['bounded_states']} of {st['frontier_states']}, pairs {st['pair_evals']:.3e}")
    a.destroy()
    s.destroy()


def test_site_bound_rejects_trace_capture():
    import torch
    w = wl.custom([40], L=2, M=8, config=26)
    s = binding.IsingSearch.from_workload(w, flags=binding.FLAG_SITE_BOUND)
    feat = torch.zeros((16, 4), dtype=torch.float32, device="cuda")
    lab = torch.zeros(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(binding.IsingError):
        s.set_trace(feat.data_ptr(), lab.data_ptr(), 16)
    assert "site bound" in binding.last_error()
    s.destroy()


@pytest.mark.parametrize("form", [binding.FORM_PLAIN, binding.FORM_SPLIT_BF16])
def test_site_bound_large_n_matches_full_scan(form):
    """N above 640 takes the site bound's path without the register copy of a;
    every search must end where the full scan ends, step by step."""
    w = wl.custom([700, 1000], L=2, M=40, config=27)
    note(f"[site bound large N] form {form}")
    a = binding.IsingSearch.from_workload(w, form=form)
    s = binding.IsingSearch.from_workload(w, form=form, flags=binding.FLAG_SITE_BOUND)
    for t in range(2000):
        na = a.step()
        ns = s.step()
        assert na == ns, f"step {t + 1}: active {na} vs {ns}"
        for sid in range(a.B * a.L):
            assert_same_set(s.get_search(sid), a.get_search(sid), f"large N search {sid} step {t + 1}")
        if na == 0:
            break
    assert na == 0
    st = s.stats()
    note(f"  bounded {st['bounded_states']} of {st['frontier_states']}")
    assert st["bounded_states"] > 0
    a.destroy()
    s.destroy()


# ---------------------------------------------------------------- FP16 scan
# The split form's pair scan in packed FP16 with its own slack; the FP64
# re-score keeps the kept sets those of the oracle.
@pytest.mark.parametrize("N,M,L,dist", [(24, 8, 4, "sk"), (65, 40, 2, "sk"), (130, 60, 2, "sk"),
                                        (200, 120, 1, "sk"), (70, 50, 2, "pmj"), (90, 30, 2, "sk_h0"),
                                        (150, 25, 2, "uniform")])
def test_fp16_scan_stepwise(N, M, L, dist):
    w = wl.custom([N], L=L, M=M, config=28, dist=dist, seed_offset=N + 5 * M)
    st = stepwise_parity(w, f"fp16 scan N={N} {dist}", form=binding.FORM_SPLIT_BF16, flags=binding.FLAG_FP16_SCAN)
    note(f"  admitted and rejected by the FP64 re-score: {st['fallbacks']}")


def test_fp16_scan_with_site_bound_and_tiles():
    w = wl.custom([5, 64, 65, 100, 129, 257], L=2, M=30, config=29)
    stepwise_parity(w, "fp16 scan + site bound, sc=7", form=binding.FORM_SPLIT_BF16,
                    flags=binding.FLAG_FP16_SCAN | binding.FLAG_SITE_BOUND, states_per_item=7)


def test_fp16_scan_matches_fp32_scan_n600():
    """4 instances of N=600, M=120, L=64: every search and merged set equal to
    the FP32 scan's, and fewer than one admitted pair in 10^4 rejected."""
    w = wl.c3_n600(n_instances=4)
    note("[fp16 scan n600]")
    a = binding.IsingSearch.from_workload(w, form=binding.FORM_SPLIT_BF16)
    h = binding.IsingSearch.from_workload(w, form=binding.FORM_SPLIT_BF16, flags=binding.FLAG_FP16_SCAN)
    ia, _ = a.run()
    ih, stable = h.run()
    assert stable and ia == ih
    for sid in range(w.n_searches):
        assert_same_set(h.get_search(sid), a.get_search(sid), f"fp16 n600 search {sid}")
    for b in range(len(w.instances)):
        ab, aE = a.get_states(b)
        hb, hE = h.get_states(b)
        assert np.array_equal(ab, hb) and np.array_equal(aE, hE)
    sa, sh = a.stats(), h.stats()
    note(f"  rejected by the re-score: fp32 {sa['fallbacks']}, fp16 {sh['fallbacks']}; pairs {sh['pair_evals']:.3e}")
    assert sh["pair_evals"] == sa["pair_evals"]
    a.destroy()
    h.destroy()


def test_fp16_scan_large_n_and_persistent():
    w = wl.custom([700, 1000, 300], L=2, M=40, config=30)
    note("[fp16 scan large N, graph replay] vs plain")
    a = binding.IsingSearch.from_workload(w)
    h = binding.IsingSearch.from_workload(w, form=binding.FORM_SPLIT_BF16, flags=binding.FLAG_FP16_SCAN, persistent=1)
    for t in range(2000):
        na = a.step()
        nh = h.step()
        assert na == nh, f"step {t + 1}: active {na} vs {nh}"
        for sid in range(a.B * a.L):
            assert_same_set(h.get_search(sid), a.get_search(sid), f"fp16 large N search {sid} step {t + 1}")
        if na == 0:
            break
    assert na == 0
    a.destroy()
    h.destroy()


def test_fp16_scan_rejects_values_outside_its_range():
    inst = wl.make_instance(40, 31, 2)
    J = inst.J * 2.0 ** 12
    with pytest.raises(binding.IsingError):
        binding.IsingSearch([inst.N], [J], [inst.h], [inst.init_bits], 8, form=binding.FORM_SPLIT_BF16,
                            flags=binding.FLAG_FP16_SCAN)
    assert "FP16" in binding.last_error()

"""The two other choices of H1 that Sec. VI names, on the GPU through the C
ABI, against the oracle's steps with the same neighbourhood: single flips
only (the J = 1 perturbation) and the XX exchange of two unequal spins, which
keeps every search in the sector of its initial state.  Small cases step by
step for every search; N = 600 and N = 1000 at selected steps, as in the
other large-size parity tests."""
import sys

import numpy as np
import pytest

import oracle
from paper_2010_00180_amd import binding, workloads as wl
from test_parity_large_gpu import large_parity, sample

pytestmark = pytest.mark.gpu

SINGLES, EXCHANGE, SB = binding.FLAG_SINGLE_FLIPS, binding.FLAG_EXCHANGE, binding.FLAG_SITE_BOUND
H1_OF = {SINGLES: 1, EXCHANGE: 2}


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


def sector_workload(Ns, L, M, config, dist="sk", frac=0.5):
    w = wl.custom(Ns, L=L, M=M, config=config, dist=dist)
    return wl.in_sector(w, [max(1, int(round(frac * n))) for n in Ns], seed=config)


def stepwise(w, flags, tag):
    h1 = H1_OF[flags & (SINGLES | EXCHANGE)]
    note(f"[{tag}] Ns={[i.N for i in w.instances]} L={w.L} M={w.M} flags={flags}")
    s = binding.IsingSearch.from_workload(w, flags=flags)
    trajs = {}
    for b, inst in enumerate(w.instances):
        for l in range(w.L):
            bits, E, front = inst.init_bits[l].reshape(1, -1), None, np.ones(1, np.uint8)
            tr = []
            while True:
                ob, oE, of, n_new = oracle.step(inst.J, inst.h, w.M, bits, E, front, fields=True, h1=h1)
                tr.append((ob, oE, of))
                if n_new == 0:
                    break
                bits, E, front = ob, oE, of
            trajs[b * w.L + l] = tr
    nsteps = max(len(t) for t in trajs.values())
    for t in range(nsteps):
        active = s.step()
        for sid, tr in trajs.items():
            ob, oE, of = tr[min(t, len(tr) - 1)]
            if t >= len(tr):
                of = np.zeros_like(of)
            gb, gE, gf = s.get_search(sid)
            assert gb.shape == ob.shape and np.array_equal(gb, ob), f"{tag} search {sid} step {t + 1}: bits"
            assert np.array_equal(gE, oE), f"{tag} search {sid} step {t + 1}: energies"
            assert np.array_equal(gf.astype(bool), of.astype(bool)), f"{tag} search {sid} step {t + 1}: flags"
        assert active == sum(1 for tr in trajs.values() if t + 1 < len(tr)), f"{tag} step {t + 1}: active"
    assert s.step() == 0
    for b, inst in enumerate(w.instances):
        mb, mE = oracle.merge(inst.N, w.M, [(trajs[b * w.L + l][-1][0], trajs[b * w.L + l][-1][1])
                                          for l in range(w.L)])
        gb, gE = s.get_states(b)
        assert np.array_equal(gb, mb) and np.array_equal(gE, mE), f"{tag} instance {b}: merge"
        if h1 == 2:
            downs = {int(sum(bin(int(x)).count("1") for x in r)) for r in gb}
            assert len(downs) == 1, f"{tag} instance {b}: kept states left the sector"
    st = s.stats()
    s.destroy()
    return st


@pytest.mark.parametrize("N,M,L,dist", [(1, 1, 2, "sk"), (5, 8, 2, "sk"), (24, 8, 4, "sk"), (65, 40, 2, "pmj"),
                                        (130, 60, 2, "sk"), (200, 120, 1, "uniform"), (300, 120, 1, "sk_h0")])
def test_single_flips_stepwise(N, M, L, dist):
    w = wl.custom([N], L=L, M=M, config=51, dist=dist, seed_offset=N)
    st = stepwise(w, SINGLES, f"singles N={N} {dist}")
    assert st["pair_evals"] == 0 and st["single_evals"] > 0


@pytest.mark.parametrize("sb", [0, SB])
@pytest.mark.parametrize("N,M,L,dist,frac", [(6, 8, 2, "sk", 0.5), (24, 8, 4, "sk", 0.5), (65, 40, 2, "pmj", 0.3),
                                             (130, 60, 2, "sk", 0.5), (200, 120, 1, "uniform", 0.1),
                                             (90, 30, 2, "sk_h0", 0.5)])
def test_exchange_stepwise(N, M, L, dist, frac, sb):
    w = sector_workload([N], L, M, config=52, dist=dist, frac=frac)
    stepwise(w, EXCHANGE | sb, f"exchange N={N} {dist} down={frac} sb={sb}")


def test_h1_uneven_sizes_one_handle():
    w = wl.custom([5, 64, 65, 100, 129], L=2, M=30, config=53)
    stepwise(w, SINGLES, "singles uneven")
    w = sector_workload([5, 64, 65, 100, 129], 2, 30, config=53)
    stepwise(w, EXCHANGE, "exchange uneven")


@pytest.mark.parametrize("flags", [SINGLES, EXCHANGE, EXCHANGE | SB])
@pytest.mark.parametrize("N", [600, 1000])
def test_h1_at_measured_sizes(flags, N):
    h1 = H1_OF[flags & (SINGLES | EXCHANGE)]
    w = wl.custom([N], L=8, M=120, config=54, seed_offset=N)
    if h1 == 2:
        w = wl.in_sector(w, [N // 2], seed=N)
    large_parity(w, f"h1={h1} N={N} flags={flags}", sample(w, 4, N), every=[0], h1=h1, flags=flags)


def test_exchange_rejects_mixed_sectors():
    w = wl.custom([40], L=3, M=8, config=55)   # random states: different numbers of down spins
    downs = {int(sum(bin(int(x)).count("1") for x in r)) for r in w.instances[0].init_bits}
    assert len(downs) > 1
    with pytest.raises(binding.IsingError):
        binding.IsingSearch.from_workload(w, flags=EXCHANGE)
    assert "sector" in binding.last_error()
    w = wl.in_sector(w, [20])
    s = binding.IsingSearch.from_workload(w, flags=EXCHANGE)
    bad = w.instances[0].init_bits[:1].copy()
    bad[0, 0] ^= np.uint64(1)
    with pytest.raises(binding.IsingError):
        s.set_search(0, bad)
    s.destroy()


def test_h1_flags_need_the_plain_form():
    w = wl.custom([40], L=2, M=8, config=56)
    for form, flags in ((binding.FORM_SPLIT_BF16, SINGLES), (binding.FORM_LEARNED, EXCHANGE), (0, SINGLES | SB),
                        (0, SINGLES | EXCHANGE)):
        with pytest.raises(binding.IsingError):
            binding.IsingSearch.from_workload(w, form=form, flags=flags)

"""The best-first search of Alg. 2-4 on the GPU, through the C ABI, against
the oracle's sequential Alg. 3 and Alg. 4: every search's final list (states,
energies, expanded flags, arrival iterations, in list order), the merged list
of each instance, and the number of expanding iterations, all bit for bit."""
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


H1 = {0: 0, binding.FLAG_SINGLE_FLIPS: 1, binding.FLAG_EXCHANGE: 2}


def check(insts, K, I, tag, flags=0, x0s=None):
    x0s = x0s if x0s is not None else [i.init_bits[:, 0] for i in insts]
    note(f"[bestfirst {tag}] N={[i.N for i in insts]} L={len(x0s[0])} K={K} I={I} flags={flags}")
    got = binding.bestfirst([i.J for i in insts], [i.h for i in insts], x0s, K, I, flags=flags, searches=True)
    h1 = H1[flags]
    for b, inst in enumerate(insts):
        for l, x0 in enumerate(x0s[b]):
            ob, oE, ou, obn, oex = oracle.bf_search(inst.J, inst.h, K, I, np.array([x0], np.uint64), h1=h1)
            gb, gE, gu, gbn = got["searches"][b][l]
            what = f"{tag} instance {b} search {l}"
            assert gb.shape == ob.shape and np.array_equal(gb, ob), f"{what}: states"
            assert np.array_equal(gE, oE), f"{what}: energies"
            assert np.array_equal(gu, ou), f"{what}: expanded flags"
            assert np.array_equal(gbn, obn), f"{what}: arrival iterations"
            assert got["expanded"][b, l] == oex, f"{what}: expanded {got['expanded'][b, l]} vs {oex}"
        mb, mE, _ = oracle.bf_multi(inst.J, inst.h, K, I, np.asarray(x0s[b], np.uint64).reshape(-1, 1), h1=h1)
        gb, gE = got["merged"][b]
        assert gb.shape == mb.shape and np.array_equal(gb, mb), f"{tag} instance {b}: merged states"
        assert np.array_equal(gE, mE), f"{tag} instance {b}: merged energies"
    return got


@pytest.mark.parametrize("N", [12, 16, 20])
def test_single_search_paper_setting(N):
    """(L, phi_1) = (1, 0) and I = K = K0 (Sec. IV, Fig. 1 and 2)."""
    K0 = N * (N + 1) // 2 + 1
    insts = [wl.make_instance(N, 8100 + 10 * N + k, 1, "uniform") for k in range(3)]
    check(insts, K0, K0, f"single N={N}", x0s=[[0]] * 3)


@pytest.mark.parametrize("N,a", [(16, 0.5), (20, 1.0), (24, 0.5)])
def test_multi_search_paper_setting(N, a):
    """(I, K, L) = (aN, K0, N) with random initial states (Sec. IV, Fig. 3 and 8)."""
    K0 = N * (N + 1) // 2 + 1
    insts = [wl.make_instance(N, 8200 + N + k, N, "uniform") for k in range(2)]
    check(insts, K0, int(a * N), f"multi N={N} a={a}")


@pytest.mark.parametrize("N,K,I", [(8, 5, 30), (10, 40, 12), (12, 3, 50), (14, 100, 20)])
def test_exact_ties_keep_arrival_order(N, K, I):
    insts = [wl.make_instance(N, 8300 + N + k, 3, "pmj") for k in range(2)]
    check(insts, K, I, f"ties N={N}")


@pytest.mark.parametrize("N,K,I", [(1, 1, 3), (2, 3, 4), (3, 0, 5), (3, 7, 10), (5, 31, 40), (4, 15, 0),
                                   (6, 100, 70)])
def test_tiny_sizes_and_edges(N, K, I):
    insts = [wl.make_instance(N, 8400 + N + K, 2, "sk") for k in range(2)]
    check(insts, K, I, f"tiny N={N} K={K} I={I}")


@pytest.mark.parametrize("N", [40, 63, 64])
def test_one_word_limit(N):
    insts = [wl.make_instance(N, 8500 + N, 2, "sk")]
    check(insts, 200, 8, f"N={N}")


@pytest.mark.parametrize("flags", [0, binding.FLAG_SINGLE_FLIPS])
def test_states_with_every_bit_set(flags):
    """At N = 64 the states 2^64 - 1 and 2^64 - 2 (every spin down, and every
    spin but the first) are ordinary states of the search; the kernels' hash
    of the list keeps them apart from its slot markers."""
    insts = [wl.make_instance(64, 8550 + k, 2, "sk") for k in range(2)]
    top = (1 << 64) - 1
    check(insts, 300, 40, f"all-down starts flags={flags}", flags=flags, x0s=[[top, top - 1], [top - 1, top - 3]])


def test_uneven_sizes_one_call():
    insts = [wl.make_instance(n, 8600 + n, 3, "uniform") for n in (9, 30, 17, 30)]
    check(insts, 120, 15, "uneven")


@pytest.mark.parametrize("flags", [binding.FLAG_SINGLE_FLIPS, binding.FLAG_EXCHANGE])
def test_other_h1(flags):
    insts = [wl.make_instance(18, 8700 + k, 4, "sk") for k in range(2)]
    if flags == binding.FLAG_EXCHANGE:
        w = wl.in_sector(wl.Workload("t", 9, insts, M=8, L=4), [9, 6])
        insts = w.instances
    check(insts, 60, 25, f"h1 flags={flags}", flags=flags)


@pytest.mark.parametrize("N,K,I,dist,L,n_inst", [
    (64, 2047, 5, "sk", 2, 2),             # search lists in device memory, merge in LDS
    (20, 2110, 2110, "uniform", 1, 2),     # K = 10 K0 at N = 20: search in LDS, merge in device memory
    (20, 2110, 60, "uniform", 3, 2),       # the same split, with three lists merged
    (16, 2740, 2740, "uniform", 1, 2),
    (14, 3000, 200, "pmj", 2, 2),          # both in device memory; exact ties in the long list
    (24, 3010, 3010, "uniform", 1, 1),     # K = 10 K0 at N = 24: both in device memory
    (12, 5000, 5000, "uniform", 1, 1),     # a list longer than the 4096 states: every state found and expanded
])
def test_lists_past_the_lds(N, K, I, dist, L, n_inst):
    """Lists that do not fit the 160 KB of LDS beside a kernel's other arrays
    live in device memory, one region per block; each kernel decides on its
    own, so the search and the merge may differ."""
    insts = [wl.make_instance(N, 8900 + N + k, L, dist) for k in range(n_inst)]
    x0s = [[0]] * n_inst if (L == 1 and dist == "uniform" and I == K) else None
    check(insts, K, I, f"long lists N={N} K={K} L={L}", x0s=x0s)


def test_rejects_what_the_kernels_cannot_take():
    big = wl.make_instance(65, 8801, 1, "sk")
    with pytest.raises(binding.IsingError):
        binding.bestfirst([big.J], [big.h], [[0]], 10, 5)
    inst = wl.make_instance(12, 8802, 1, "sk")
    with pytest.raises(binding.IsingError):
        binding.bestfirst([inst.J], [inst.h], [[0]], 1 << 20, 5)
    assert "K=" in binding.last_error()

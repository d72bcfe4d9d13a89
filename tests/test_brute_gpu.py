"""The GPU enumeration of all 2^N states (the brute-force reference of
Sec. IV and the spectra of Sec. V) against the oracle's own exhaustive
search, bit for bit: the K lowest states in (E, psi) order and their exact
energies."""
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


def check(insts, K, tag):
    note(f"[brute {tag}] N={[i.N for i in insts]} K={K}")
    got = binding.brute_lowest([i.J for i in insts], [i.h for i in insts], K)
    for inst, (gb, gE) in zip(insts, got):
        ob, oE = oracle.brute_lowest(inst.J, inst.h, K)
        assert gb.shape == ob.shape, f"{tag} N={inst.N}: {gb.shape} vs {ob.shape}"
        assert np.array_equal(gb, ob), f"{tag} N={inst.N}: states differ"
        assert np.array_equal(gE, oE), f"{tag} N={inst.N}: energies differ"
    return got


@pytest.mark.parametrize("N", [1, 2, 3, 5, 7, 8, 9, 12, 13, 14, 15, 17, 20])
def test_every_size_small(N):
    insts = [wl.make_instance(N, 7000 + N + 50 * k, 1, d) for k, d in enumerate(("sk", "uniform"))]
    for K in (1, 8, 120):
        check(insts, K, f"N={N}")


@pytest.mark.parametrize("dist", ["sk", "uniform", "pmj", "sk_h0"])
def test_n24_distributions(dist):
    inst = wl.make_instance(24, 7100, 1, dist)
    check([inst], 120 if dist != "pmj" else 40, dist)


def test_uneven_sizes_one_call_and_large_k():
    insts = [wl.make_instance(n, 7200 + n, 1, "uniform") for n in (16, 4, 22, 11, 16, 18)]
    check(insts, 4096, "uneven K=4096")


def test_more_states_asked_than_exist():
    insts = [wl.make_instance(n, 7300 + n, 1, "sk") for n in (3, 10)]
    got = check(insts, 2000, "K > 2^N")
    assert [len(E) for _, E in got] == [8, 1024]


def test_ground_energy_fit_at_n26():
    """Sec. V, Fig. 9: the mean ground energy of 24 U[-1/2, 1/2] instances at
    N = 26 within three standard errors of -0.218 N^{3/2} + 0.79."""
    insts = [wl.make_instance(26, 7400 + k, 1, "uniform") for k in range(24)]
    note("[brute fit] 24 instances N=26")
    got = binding.brute_lowest([i.J for i in insts], [i.h for i in insts], 2)
    e1 = np.array([E[0] for _, E in got])
    for inst, (b, E) in zip(insts[:2], got[:2]):
        assert oracle.energy(inst.J, inst.h, b[0]) == E[0]
    fit = -0.218 * 26 ** 1.5 + 0.79
    se = e1.std(ddof=1) / np.sqrt(len(e1))
    note(f"[brute fit] mean E1 {e1.mean():.3f} +- {se:.3f}, fit {fit:.3f}")
    assert abs(e1.mean() - fit) < 3 * se + 0.14 + 0.001 * 26 ** 1.5


def test_rejects_bad_arguments():
    inst = wl.make_instance(10, 7500, 1, "sk")
    for K in (0, 4097):
        with pytest.raises(binding.IsingError):
            binding.brute_lowest([inst.J], [inst.h], K)
    J = inst.J.copy()
    J[0, 1] += 2.0 ** -30
    with pytest.raises(binding.IsingError):
        binding.brute_lowest([J], [inst.h], 4)

"""The configuration's files through the C ABI: the autotuner's tile cache
(written by one handle, read back by the next without timing) and the
learned form's parameter file (the same network as set_scorer)."""
import numpy as np
import pytest

from paper_2010_00180_amd import binding, workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    binding.load()


def run_tuned(w, cache, **kw):
    s = binding.IsingSearch.from_workload(w, tile_cache=cache, **kw)
    s.step()
    s.autotune()
    tiles = list(s.tuning())
    s.run()
    out = [s.get_states(b) for b in range(s.B)]
    s.destroy()
    return tiles, out


@pytest.mark.parametrize("kw", [{}, {"form": binding.FORM_SPLIT_BF16}, {"flags": binding.FLAG_SITE_BOUND}])
def test_tile_cache_round_trip(tmp_path, kw):
    w = wl.custom([100, 200, 200, 300], L=4, M=40, config=81)
    cache = str(tmp_path / "tiles.txt")
    t1, r1 = run_tuned(w, cache, **kw)
    lines = open(cache).read().splitlines()
    assert len(lines) == 3, lines   # one line per distinct N
    for ln in lines:
        f = ln.split()
        assert f[0] == "ising-tile" and f[1] == "1" and int(f[7]) in (16, 32, 64, 128, 256)
    t2, r2 = run_tuned(w, cache, **kw)
    assert open(cache).read().splitlines() == lines   # nothing timed, nothing added
    assert t2 == t1
    # a size missing from the cache is tuned and appended
    w3 = wl.custom([100, 150], L=4, M=40, config=82)
    run_tuned(w3, cache, **kw)
    new = open(cache).read().splitlines()
    assert new[:3] == lines and len(new) == 4 and new[3].split()[5] == "150"
    # the tiles never change the results
    _, r0 = run_tuned(w, None, **kw)
    for (ab, aE), (bb, bE), (cb, cE) in zip(r0, r1, r2):
        assert np.array_equal(ab, bb) and np.array_equal(ab, cb)
        assert np.array_equal(aE, bE) and np.array_equal(aE, cE)


def test_cache_lines_for_other_keys_are_ignored(tmp_path):
    w = wl.custom([120], L=4, M=40, config=83)
    probe = tmp_path / "probe.txt"
    run_tuned(w, str(probe))
    arch = probe.read_text().split()[2]   # this device, as the library names it
    cache = tmp_path / "tiles.txt"
    cache.write_text("ising-tile 1 gfx000 0 0 120 40 16 0\n"               # another device
                     f"ising-tile 1 {arch} 0 0 120 41 16 0\n"              # another M
                     "garbage line\n"
                     f"ising-tile 2 {arch} 0 0 120 40 16 0\n"              # another version
                     f"ising-tile 1 {arch} 0 0 120 40 24 0\n")             # not a tile size
    run_tuned(w, str(cache))
    lines = cache.read_text().splitlines()
    assert len(lines) == 6 and lines[5].split()[5:7] == ["120", "40"]


def test_weights_file_equals_set_scorer(tmp_path):
    w = wl.custom([60, 90], L=4, M=30, config=84)
    params = wl.network_params(9).astype(np.float32)
    path = str(tmp_path / "w.bin")
    binding.save_mlp_weights(path, params)
    a = binding.IsingSearch.from_workload(w, form=binding.FORM_LEARNED)
    a.set_scorer(binding.SCORER_NETWORK, params, seed=0)
    b = binding.IsingSearch.from_workload(w, form=binding.FORM_LEARNED, mlp_weights=path)
    ia, ib = a.run(), b.run()
    assert ia == ib
    for k in range(a.B):
        xa, Ea = a.get_states(k)
        xb, Eb = b.get_states(k)
        assert np.array_equal(xa, xb) and np.array_equal(Ea, Eb)
    assert a.stats()["scored_pairs"] == b.stats()["scored_pairs"]
    a.destroy()
    b.destroy()

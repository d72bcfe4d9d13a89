"""Seeded synthetic Ising instances and initial states.

This module only draws random numbers and packs bits.  It holds none of the
search method's arithmetic, so both the HIP path and the CPU oracle may use it
to obtain identical inputs.

Conventions (Sec. III, Eq. 15 of the paper):
  * a state of N spins is the integer psi = sum_i 2^i sigma_i with
    sigma_i in {0, 1}; sigma_i = 0 means s_i = +1 and sigma_i = 1 means s_i = -1;
  * psi is stored little-endian in W = ceil(N/64) uint64 words: bit i of word
    i >> 6 is sigma_i; bits at positions >= N are zero.

Couplings J are dense N x N float64, exactly symmetric with a zero diagonal;
fields h are N float64.  Every value is rounded (half to even) to an integer
multiple of 2^-24 so that all sums formed by the method are exact in float64
(the magnitudes stay far below 2^29), which makes energies order independent.

Distributions:
  * ``sk``:       J_ij ~ N(0,1)/sqrt(N) for i<j, h_i ~ N(0,1)   (the measured workloads)
  * ``uniform``:  J_ij, h_i ~ U[-1/2, 1/2]   (the paper's Sec. IV distribution)
  * ``pmj``:      J_ij in {-1,+1}, h_i in {-1,0,+1} (a tie-heavy stress input)

Seeds: instance k of configuration c uses PCG64 seeded with
201000180 + 1000*c + k; the upper triangle of J is drawn first in row-major
order, then h, then the L initial states (N fair bits each).
"""
from __future__ import annotations

import dataclasses
from typing import List, Sequence

import numpy as np

SEED_BASE = 201000180
GRID = 2.0 ** -24


def seed_for(config: int, k: int) -> int:
    return SEED_BASE + 1000 * config + k


def words_for(N: int) -> int:
    return (N + 63) // 64


def snap(x: np.ndarray) -> np.ndarray:
    """Round to the nearest multiple of 2^-24 (ties to even)."""
    return np.rint(np.asarray(x, dtype=np.float64) / GRID) * GRID


def pack_bits(sigma: np.ndarray) -> np.ndarray:
    """sigma: (..., N) array of 0/1 -> (..., W) uint64 words, bit i of word i>>6."""
    sigma = np.asarray(sigma, dtype=np.uint64)
    N = sigma.shape[-1]
    W = words_for(N)
    out = np.zeros(sigma.shape[:-1] + (W,), dtype=np.uint64)
    for i in range(N):
        out[..., i >> 6] |= sigma[..., i] << np.uint64(i & 63)
    return out


def unpack_bits(words: np.ndarray, N: int) -> np.ndarray:
    words = np.asarray(words, dtype=np.uint64)
    out = np.zeros(words.shape[:-1] + (N,), dtype=np.uint8)
    for i in range(N):
        out[..., i] = ((words[..., i >> 6] >> np.uint64(i & 63)) & np.uint64(1)).astype(np.uint8)
    return out


@dataclasses.dataclass
class Instance:
    N: int
    J: np.ndarray          # (N, N) float64, symmetric, zero diagonal
    h: np.ndarray          # (N,) float64
    init_bits: np.ndarray  # (L, W) uint64
    seed: int
    dist: str


def make_instance(N: int, seed: int, L: int, dist: str = "sk") -> Instance:
    rng = np.random.Generator(np.random.PCG64(seed))
    iu = np.triu_indices(N, 1)
    J = np.zeros((N, N), dtype=np.float64)
    n_up = len(iu[0])
    if dist == "sk":
        J[iu] = rng.standard_normal(n_up) / np.sqrt(N)
        h = rng.standard_normal(N)
    elif dist == "uniform":
        J[iu] = rng.uniform(-0.5, 0.5, n_up)
        h = rng.uniform(-0.5, 0.5, N)
    elif dist == "pmj":
        J[iu] = rng.choice(np.array([-1.0, 1.0]), n_up)
        h = rng.choice(np.array([-1.0, 0.0, 1.0]), N)
    elif dist == "wide":
        # unnormalized couplings: row sums |h_i| + sum_j |J_ij| of about 3N,
        # beyond 2^7 on the 2^-24 grid for N >= 50
        J[iu] = 2.0 * rng.standard_normal(n_up)
        h = 2.0 * rng.standard_normal(N)
    elif dist == "sk_h0":
        J[iu] = rng.standard_normal(n_up) / np.sqrt(N)
        h = np.zeros(N)
        rng.standard_normal(N)  # keep the stream aligned with "sk"
    else:
        raise ValueError(f"unknown distribution {dist!r}")
    J = snap(J + J.T)
    h = snap(h)
    sigma = rng.integers(0, 2, size=(L, N))
    return Instance(N=N, J=J, h=h, init_bits=pack_bits(sigma), seed=seed, dist=dist)


@dataclasses.dataclass
class Workload:
    name: str
    config: int
    instances: List[Instance]
    M: int
    L: int

    @property
    def n_searches(self) -> int:
        return len(self.instances) * self.L

    def pair_flips_per_state(self) -> List[int]:
        return [inst.N * (inst.N - 1) // 2 for inst in self.instances]


# The five measured workloads.  ``n_instances`` may be reduced for tests.
def c1_n24(n_instances: int = 1) -> Workload:
    """1 instance, N=24, M=8 kept, 4 initial states; small enough for brute force."""
    inst = [make_instance(24, seed_for(1, k), 4) for k in range(n_instances)]
    return Workload("c1_n24_m8_l4", 1, inst, M=8, L=4)


def c2_n200(n_instances: int = 120, L: int = 16) -> Workload:
    inst = [make_instance(200, seed_for(2, k), L) for k in range(n_instances)]
    return Workload("c2_n200_m120_l16", 2, inst, M=120, L=L)


def c3_n600(n_instances: int = 120, L: int = 64) -> Workload:
    inst = [make_instance(600, seed_for(3, k), L) for k in range(n_instances)]
    return Workload("c3_n600_m120_l64", 3, inst, M=120, L=L)


def c4_sizes(n_instances: int = 480) -> List[int]:
    rng = np.random.Generator(np.random.PCG64(seed_for(4, 999)))
    return [int(x) for x in rng.choice(np.arange(100, 601, 100), n_instances)]


def c4_uneven(n_instances: int = 480, L: int = 32) -> Workload:
    sizes = c4_sizes(480)[:n_instances]
    inst = [make_instance(n, seed_for(4, k), L) for k, n in enumerate(sizes)]
    return Workload("c4_uneven_n100_600_m120_l32", 4, inst, M=120, L=L)


def c5_learned(N: int, n_instances: int = 120, L: int = 64) -> Workload:
    inst = [make_instance(N, seed_for(5, k + (0 if N == 600 else 500)), L) for k in range(n_instances)]
    return Workload(f"c5_n{N}_m120_l{L}", 5, inst, M=120, L=L)


def custom(Ns: Sequence[int], L: int, M: int, config: int = 9, dist: str = "sk", seed_offset: int = 0) -> Workload:
    inst = [make_instance(n, seed_for(config, seed_offset + k), L, dist) for k, n in enumerate(Ns)]
    return Workload(f"custom_{dist}", config, inst, M=M, L=L)


def in_sector(w: Workload, n_down: Sequence[int], seed: int = 0) -> Workload:
    """The same instances with new initial states: for instance b, L states
    with exactly n_down[b] down spins each, at uniformly drawn sites (one
    sector of the total sigma^z per instance, for the exchange neighbourhood)."""
    out = []
    for k, inst in enumerate(w.instances):
        rng = np.random.Generator(np.random.PCG64(seed_for(w.config, 700 + 31 * seed + k)))
        sigma = np.zeros((w.L, inst.N), dtype=np.int64)
        for l in range(w.L):
            sigma[l, rng.choice(inst.N, int(n_down[k]), replace=False)] = 1
        out.append(dataclasses.replace(inst, init_bits=pack_bits(sigma)))
    return Workload(w.name + "_sector", w.config, out, M=w.M, L=w.L)


# Initial parameters of the learned form's scoring network (4545 values in the
# order W1[64][4], b1[64], W2[64][64], b2[64], w3[64], b3): a seeded He-style
# draw, used as the starting point of training and as an untrained baseline.
NET_PARAMS = 4 * 64 + 64 + 64 * 64 + 64 + 64 + 1


def network_params(seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed_for(9, seed)))
    P = np.zeros(NET_PARAMS)
    o = 0
    for size, std in ((4 * 64, np.sqrt(2 / 4)), (64, 0.1), (64 * 64, np.sqrt(2 / 64)), (64, 0.1), (64, np.sqrt(1 / 64))):
        P[o:o + size] = rng.normal(0.0, std, size)
        o += size
    return P

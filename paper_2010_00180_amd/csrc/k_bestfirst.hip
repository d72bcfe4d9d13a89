// The paper's best-first form of the search (Sec. III): Alg. 3, the single
// search with the list update of Alg. 2, and the merge of Alg. 4.
//
// One block per search; the list of K + 1 entries (state, energy, expanded
// flag, arrival iteration) lives in LDS (in global memory, per block, when
// it does not fit: the same code through the same pointers) in energy order,
// entries of equal energy in order of arrival, placeholders (E = +inf) at the
// end.  An iteration expands the first entry that has not been expanded: its
// children (single flips of sites 0 .. N-1, then pair flips (0,1), (0,2), ..;
// one of the two families for the other choices of H1) are offered to the
// list one after the other in Alg. 2, each entering when it is not in the
// list and its energy is below the last entry's.  Such a stream of offers
// keeps exactly the K + 1 lowest distinct states in (energy, arrival) order
// of everything offered (a copy of a state that left the list is never lower
// than the list's last entry), so the block evaluates all children at once
// from the parent's local fields, keeps those below the last entry that the
// list does not hold (a hash of the list's states, which each merge updates
// with the states that enter and leave), sorts them by (energy, child index)
// and merges them behind the old entries of equal energy.  All energies are
// exact on the 2^-24 grid, so the list is the one the sequential algorithm
// builds.  The search for the entry to expand starts where the last merge
// first changed the list, or after the entry just expanded.
//
// The merge of Alg. 4 is the same update with the later searches' lists, in
// their own order, as the offered entries.
#include "bestfirst.h"

namespace qi {

namespace {

// Slot contents of the hash of the list's states besides a state: an empty
// slot, and one whose state has left the list.  The two states with these
// bit patterns (possible only at N = 64) are kept as flags instead.
constexpr uint64_t BF_EMPTY = ~0ull;
constexpr uint64_t BF_GONE = ~0ull - 1;

struct BfLds {
    uint64_t* psi[2];
    double* E[2];
    int* born[2];
    uint8_t* used[2];
    uint64_t* hash;    // [HS] the list's states by open addressing, BF_EMPTY or BF_GONE elsewhere
    int HS;
    double* cE;        // [C] offered entries: energy
    uint32_t* cI;      // [C] child index (search) or list index (merge)
    uint64_t* cpsi;    // [C] merge only
    uint8_t* pi;       // [C] first site of child c (pair table)
    uint8_t* pj;       // [C] second site, or 0xFF for a single flip
    double* F;         // [64]
    int* misc;         // [8]: 0 first entry to expand, 1 offered count, 2 hash slots not empty,
                       //      3 first list position a merge changed, 4 flags of the two special states
};

// Hash slots for a list of K1 entries: twice the list, so that the slots
// holding a state or a departed one stay below 5/8 between rebuilds.
__host__ __device__ inline int bf_hash_slots(int K1) { return (2 * K1 + 63) / 64 * 64; }

__device__ inline uint32_t bf_slot(uint64_t x, int HS)
{
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    return (uint32_t)(((uint64_t)(uint32_t)x * (uint32_t)HS) >> 32);
}

__device__ inline int bf_special(uint64_t x) { return x == BF_EMPTY ? 1 : (x == BF_GONE ? 2 : 0); }

__device__ inline bool bf_member(const BfLds& s, uint64_t x)
{
    if (const int f = bf_special(x)) return (s.misc[4] & f) != 0;
    uint32_t h = bf_slot(x, s.HS);
    while (true) {
        const uint64_t k = s.hash[h];
        if (k == x) return true;
        if (k == BF_EMPTY) return false;
        if (++h == (uint32_t)s.HS) h = 0;
    }
}

// x is not in the hash; inserts may run together, never beside a removal
__device__ inline void bf_insert(const BfLds& s, uint64_t x)
{
    if (const int f = bf_special(x)) {
        atomicOr(&s.misc[4], f);
        return;
    }
    uint32_t h = bf_slot(x, s.HS);
    while (true) {
        const uint64_t k = s.hash[h];
        if ((k == BF_EMPTY || k == BF_GONE) && atomicCAS((unsigned long long*)&s.hash[h], k, x) == k) {
            if (k == BF_EMPTY) atomicAdd(&s.misc[2], 1);
            return;
        }
        if (++h == (uint32_t)s.HS) h = 0;
    }
}

// x is in the hash; removals may run together, never beside an insert
__device__ inline void bf_remove(const BfLds& s, uint64_t x)
{
    if (const int f = bf_special(x)) {
        atomicAnd(&s.misc[4], ~f);
        return;
    }
    uint32_t h = bf_slot(x, s.HS);
    while (s.hash[h] != x)
        if (++h == (uint32_t)s.HS) h = 0;
    s.hash[h] = BF_GONE;
}

// The hash rebuilt from the real entries of list `cur`.  Block-wide.
__device__ void bf_rehash(const BfLds& s, int cur, int K1)
{
    for (int q = threadIdx.x; q < s.HS; q += blockDim.x) s.hash[q] = BF_EMPTY;
    if (threadIdx.x == 0) s.misc[2] = s.misc[4] = 0;
    __syncthreads();
    for (int k = threadIdx.x; k < K1; k += blockDim.x)
        if (s.E[cur][k] < INFINITY) bf_insert(s, s.psi[cur][k]);
    __syncthreads();
}

// Bitonic sort of cE/cI[0 .. n2) by (E, index), ascending.  Block-wide.
__device__ void bf_sort(const BfLds& s, int n2)
{
    for (int size = 2; size <= n2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int q = threadIdx.x; q < n2; q += blockDim.x) {
                const int p = q ^ stride;
                if (p > q) {
                    const bool up = (q & size) == 0;
                    const bool gt = s.cE[q] > s.cE[p] || (s.cE[q] == s.cE[p] && s.cI[q] > s.cI[p]);
                    if (gt == up) {
                        const double te = s.cE[q];
                        s.cE[q] = s.cE[p];
                        s.cE[p] = te;
                        const uint32_t ti = s.cI[q];
                        s.cI[q] = s.cI[p];
                        s.cI[p] = ti;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// number of v[0 .. n) (ascending) below x, or at or below x
__device__ inline int count_below(const double* v, int n, double x, bool or_equal)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (or_equal ? v[mid] <= x : v[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// List `cur` merged with the n offered entries (cE ascending, their states,
// flags and arrivals given by `get`) into list 1 - cur, K1 entries: an old
// entry goes before offered entries of equal energy.  The hash follows: the
// states pushed past the end leave it, the offered ones that enter join it,
// and it is rebuilt once the departed ones fill an eighth of it.  misc[3]
// gets the first position where the two lists may differ.  The first
// `agree` entries of list 1 - cur already equal those of list cur; of them,
// the ones that keep their place are not copied.  Block-wide.
template <class Get>
__device__ void bf_merge(const BfLds& s, int cur, int K1, int n, int agree, const Get& get)
{
    const int nx = 1 - cur;
    const double c0 = s.cE[0];
    for (int k = threadIdx.x; k < K1; k += blockDim.x) {
        const double e = s.E[cur][k];
        if (k < agree && e <= c0) continue;
        const int pos = k + count_below(s.cE, n, e, false);
        if (pos < K1) {
            s.psi[nx][pos] = s.psi[cur][k];
            s.E[nx][pos] = e;
            s.used[nx][pos] = s.used[cur][k];
            s.born[nx][pos] = s.born[cur][k];
        } else if (e < INFINITY) {
            bf_remove(s, s.psi[cur][k]);
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
        const int pos = q + count_below(s.E[cur], K1, s.cE[q], true);
        if (q == 0) s.misc[3] = pos < K1 ? pos : K1;
        if (pos < K1) {
            uint64_t x;
            uint8_t u;
            int bn;
            get(q, x, u, bn);
            s.psi[nx][pos] = x;
            s.E[nx][pos] = s.cE[q];
            s.used[nx][pos] = u;
            s.born[nx][pos] = bn;
            bf_insert(s, x);
        }
    }
    __syncthreads();
    if (s.misc[2] * 8 > s.HS * 5) {
        __syncthreads();   // every thread has read misc[2] before the rebuild clears it
        bf_rehash(s, nx, K1);
    }
}

constexpr size_t BF_MERGE_STATIC = 256 * sizeof(int);   // the merge kernel's own prefix-sum array

__host__ __device__ inline size_t bf_round(size_t b) { return (b + 15) & ~(size_t)15; }

// the two lists and the hash of K1-entry lists
__host__ __device__ inline size_t bf_list_bytes(int K1)
{
    return 2 * (bf_round(8 * (size_t)K1) * 2 + bf_round(4 * (size_t)K1) + bf_round((size_t)K1)) +
           bf_round(8 * (size_t)bf_hash_slots(K1));
}

// the offered entries (C of them), with the pair table of a search or the
// offered states of a merge, the parent's fields and the counters
__host__ __device__ inline size_t bf_aux_bytes(int C, bool merge)
{
    return bf_round(8 * (size_t)C) + bf_round(4 * (size_t)C) +
           (merge ? bf_round(8 * (size_t)C) : 2 * bf_round((size_t)C)) + bf_round(8 * 64) + bf_round(4 * 8);
}

__device__ BfLds bf_carve(unsigned char* lists, unsigned char* aux, int K1, int C, bool merge)
{
    BfLds s;
    auto taker = [](unsigned char* base) {
        return [base, o = (size_t)0](size_t bytes) mutable {
            unsigned char* p = base + o;
            o += bf_round(bytes);
            return p;
        };
    };
    auto tl = taker(lists);
    for (int c = 0; c < 2; ++c) {
        s.psi[c] = reinterpret_cast<uint64_t*>(tl(8 * (size_t)K1));
        s.E[c] = reinterpret_cast<double*>(tl(8 * (size_t)K1));
        s.born[c] = reinterpret_cast<int*>(tl(4 * (size_t)K1));
        s.used[c] = tl((size_t)K1);
    }
    s.HS = bf_hash_slots(K1);
    s.hash = reinterpret_cast<uint64_t*>(tl(8 * (size_t)s.HS));
    auto ta = taker(aux);
    s.cE = reinterpret_cast<double*>(ta(8 * (size_t)C));
    s.cI = reinterpret_cast<uint32_t*>(ta(4 * (size_t)C));
    s.cpsi = merge ? reinterpret_cast<uint64_t*>(ta(8 * (size_t)C)) : nullptr;
    s.pi = merge ? nullptr : ta((size_t)C);
    s.pj = merge ? nullptr : ta((size_t)C);
    s.F = reinterpret_cast<double*>(ta(8 * 64));
    s.misc = reinterpret_cast<int*>(ta(4 * 8));
    return s;
}

}  // namespace

BestFirstPlan bestfirst_plan(int K1, int Cs)
{
    BestFirstPlan p{};
    const size_t lists = bf_list_bytes(K1), aux_s = bf_aux_bytes(Cs, false), aux_m = bf_aux_bytes(K1, true);
    size_t ws = 0;
    p.lists_in_lds = aux_s + lists <= BFS_LDS_MAX;
    p.lds_search = aux_s + (p.lists_in_lds ? lists : 0);
    if (!p.lists_in_lds) ws = lists;
    p.merge_in_lds = aux_m + lists + BF_MERGE_STATIC <= BFS_LDS_MAX;
    p.lds_merge = p.merge_in_lds ? aux_m + lists : 0;
    if (!p.merge_in_lds) ws = std::max(ws, aux_m + lists);
    p.ws_stride = (ws + 255) / 256 * 256;
    return p;
}

// One block per search (search = instance * L + l).
__global__ __launch_bounds__(256) void k_bf_search(BestFirstArgs a)
{
    extern __shared__ __align__(16) unsigned char bf_dyn[];
    const int sid = blockIdx.x;
    const int b = sid / a.L;
    const int N = a.N[b];
    const int K1 = a.K1;
    // the offered entries always in LDS, the lists after them or in global memory
    const BfLds s = bf_carve(a.lists_in_lds ? bf_dyn + bf_aux_bytes(a.Cs, false) : a.ws + (size_t)sid * a.ws_stride,
                             bf_dyn, K1, a.Cs, false);
    const double* __restrict__ J = a.J + a.joff[b];
    const double* __restrict__ h = a.h + (size_t)b * 64;
    const int h1 = a.h1;
    // children in arrival order: single flips (unless exchanges), then pairs
    const int nsingle = h1 == H1_EXCHANGE ? 0 : N;
    const int npair = h1 == H1_SINGLES ? 0 : N * (N - 1) / 2;
    const int nchild = nsingle + npair;
    for (int c = threadIdx.x; c < nchild; c += blockDim.x) {
        if (c < nsingle) {
            s.pi[c] = (uint8_t)c;
            s.pj[c] = 0xFF;
        } else {
            int q = c - nsingle, i = 0;
            while (q >= N - 1 - i) {
                q -= N - 1 - i;
                ++i;
            }
            s.pi[c] = (uint8_t)i;
            s.pj[c] = (uint8_t)(i + 1 + q);
        }
    }
    // the initial list: x0, then placeholders
    const uint64_t x0 = a.x0[sid];
    for (int k = threadIdx.x; k < K1; k += blockDim.x) {
        s.E[0][k] = INFINITY;
        s.psi[0][k] = 0;
        s.used[0][k] = 0;
        s.born[0][k] = 0;
    }
    if (threadIdx.x < 64) {
        const int t = threadIdx.x;
        double f = 0.0;
        if (t < N) {
            f = h[t];
            for (int l = 0; l < N; ++l) f += J[t * N + l] * (((x0 >> l) & 1) ? -1.0 : 1.0);
        }
        // E = (1/2) sum_i s_i (F_i + h_i)
        double e = t < N ? 0.5 * (((x0 >> t) & 1) ? -1.0 : 1.0) * (f + h[t]) : 0.0;
        for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
        if (t == 0) {
            s.E[0][0] = e;
            s.psi[0][0] = x0;
        }
    }
    __syncthreads();
    bf_rehash(s, 0, K1);
    int cur = 0, expanded = 0;
    int from = 0;    // every entry before it has been expanded
    int agree = 0;   // list 1 - cur equals list cur on its first `agree` entries
    for (int it = 1; it <= a.I; ++it) {
        // the first entry not yet expanded
        if (threadIdx.x == 0) {
            s.misc[0] = K1;
            s.misc[1] = 0;
        }
        __syncthreads();
        int mine = K1;
        for (int k = from + threadIdx.x; k < K1; k += blockDim.x)
            if (s.E[cur][k] < INFINITY && !s.used[cur][k]) {
                mine = k;
                break;
            }
        if (mine < K1) atomicMin(&s.misc[0], mine);
        __syncthreads();
        const int kp = s.misc[0];
        if (kp >= K1) break;   // every entry expanded: no later iteration changes the list
        const uint64_t xp = s.psi[cur][kp];
        const double Ep = s.E[cur][kp];
        if (threadIdx.x < 64) {
            const int t = threadIdx.x;
            if (t < N) {
                double f = h[t];
                for (int l = 0; l < N; ++l) f += J[t * N + l] * (((xp >> l) & 1) ? -1.0 : 1.0);
                s.F[t] = f;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            s.used[cur][kp] = 1;
            if (kp < agree) s.used[1 - cur][kp] = 1;
        }
        ++expanded;
        const double Elast = s.E[cur][K1 - 1];
        for (int c = threadIdx.x; c < nchild; c += blockDim.x) {
            const int i = s.pi[c], j = s.pj[c];
            const double si = ((xp >> i) & 1) ? -1.0 : 1.0;
            double d = -2.0 * si * s.F[i];
            uint64_t x = xp ^ (1ull << i);
            if (j != 0xFF) {
                const double sj = ((xp >> j) & 1) ? -1.0 : 1.0;
                if (h1 == H1_EXCHANGE && si == sj) continue;   // an exchange of equal spins gives the parent back
                d += -2.0 * sj * s.F[j] + 4.0 * J[i * N + j] * si * sj;
                x ^= 1ull << j;
            }
            const double Ec = Ep + d;
            if (Ec < Elast && !bf_member(s, x)) {
                const int slot = atomicAdd(&s.misc[1], 1);
                s.cE[slot] = Ec;
                s.cI[slot] = (uint32_t)c;
            }
        }
        __syncthreads();
        const int n = s.misc[1];
        __syncthreads();   // misc is reset by the next iteration
        from = kp + 1;
        if (n == 0) continue;
        int n2 = 1;
        while (n2 < n) n2 <<= 1;
        for (int q = n + threadIdx.x; q < n2; q += blockDim.x) {
            s.cE[q] = INFINITY;
            s.cI[q] = 0xFFFFFFFFu;
        }
        __syncthreads();
        bf_sort(s, n2);
        bf_merge(s, cur, K1, n, agree, [&](int q, uint64_t& x, uint8_t& u, int& bn) {
            const int c = (int)s.cI[q];
            x = xp ^ (1ull << s.pi[c]);
            if (s.pj[c] != 0xFF) x ^= 1ull << s.pj[c];
            u = 0;
            bn = it;
        });
        agree = s.misc[3];             // the entries before it kept their places
        from = min(from, agree);
        cur = 1 - cur;
    }
    // the real entries, in list order
    const size_t o = (size_t)sid * K1;
    for (int k = threadIdx.x; k < K1; k += blockDim.x) {
        a.out_psi[o + k] = s.psi[cur][k];
        a.out_E[o + k] = s.E[cur][k];
        a.out_used[o + k] = s.used[cur][k];
        a.out_born[o + k] = s.born[cur][k];
    }
    if (threadIdx.x == 0) a.out_expanded[sid] = expanded;
}

// One block per instance: Alg. 4 over the L lists written by k_bf_search.
__global__ __launch_bounds__(256) void k_bf_merge(BestFirstArgs a)
{
    extern __shared__ __align__(16) unsigned char bf_dyn[];
    __shared__ int tmp[BF_MERGE_STATIC / sizeof(int)];
    const int b = blockIdx.x;
    const int K1 = a.K1;
    unsigned char* base = a.merge_in_lds ? bf_dyn : a.ws + (size_t)b * a.ws_stride;
    const BfLds s = bf_carve(base + bf_aux_bytes(K1, true), base, K1, K1, true);
    const size_t o0 = (size_t)b * a.L * K1;
    for (int k = threadIdx.x; k < K1; k += blockDim.x) {
        s.psi[0][k] = a.out_psi[o0 + k];
        s.E[0][k] = a.out_E[o0 + k];
        s.used[0][k] = a.out_used[o0 + k];
        s.born[0][k] = a.out_born[o0 + k];
    }
    __syncthreads();
    bf_rehash(s, 0, K1);
    int cur = 0, agree = 0;
    for (int l = 1; l < a.L; ++l) {
        const size_t o = o0 + (size_t)l * K1;
        const double Elast = s.E[cur][K1 - 1];
        // the entries of list l that may enter, in their order (a prefix sum
        // keeps it)
        int n = 0;
        for (int c0 = 0; c0 < K1; c0 += blockDim.x) {
            const int k = c0 + threadIdx.x;
            int take = 0;
            double e = INFINITY;
            uint64_t x = 0;
            if (k < K1) {
                e = a.out_E[o + k];
                x = a.out_psi[o + k];
                take = e < Elast && !bf_member(s, x);
            }
            // exclusive prefix sum over the block
            tmp[threadIdx.x] = take;
            __syncthreads();
            for (int off = 1; off < (int)blockDim.x; off <<= 1) {
                const int v = threadIdx.x >= (unsigned)off ? tmp[threadIdx.x - off] : 0;
                __syncthreads();
                tmp[threadIdx.x] += v;
                __syncthreads();
            }
            const int excl = tmp[threadIdx.x] - take;
            const int tot = tmp[blockDim.x - 1];
            if (take) {
                s.cE[n + excl] = e;
                s.cI[n + excl] = (uint32_t)k;
                s.cpsi[n + excl] = x;
            }
            n += tot;
            __syncthreads();
        }
        if (n == 0) continue;
        bf_merge(s, cur, K1, n, agree, [&](int q, uint64_t& x, uint8_t& u, int& bn) {
            const int k = (int)s.cI[q];
            x = s.cpsi[q];
            u = a.out_used[o + k];
            bn = a.out_born[o + k];
        });
        agree = s.misc[3];
        cur = 1 - cur;
    }
    const size_t ob = (size_t)b * K1;
    for (int k = threadIdx.x; k < K1; k += blockDim.x) {
        a.merged_psi[ob + k] = s.psi[cur][k];
        a.merged_E[ob + k] = s.E[cur][k];
    }
}

hipError_t bestfirst_set_lds(const BestFirstPlan& p)
{
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_bf_search),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds_search);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_bf_merge), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)p.lds_merge);
    return e;
}

hipError_t launch_bestfirst(const BestFirstArgs& a, int n_inst, const BestFirstPlan& p, hipStream_t st)
{
    hipLaunchKernelGGL(k_bf_search, dim3((unsigned)(n_inst * a.L)), dim3(256), p.lds_search, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bf_merge, dim3((unsigned)n_inst), dim3(256), p.lds_merge, st, a);
    return hipGetLastError();
}

}  // namespace qi

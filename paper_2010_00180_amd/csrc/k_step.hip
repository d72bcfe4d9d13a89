// One synchronous step of every active search (Sec. II): expand the states
// that entered in the previous step by all single and pair flips (Eq. 9 with
// the H1 of Eq. 16), and keep the M lowest distinct states of the union with
// the current kept set.  Energies of flipped states come from local fields:
// with a_i = -2 s_i F_i, a single flip changes E by a_i and a pair flip (i,j)
// by a_i + a_j + 4 s_i s_j J_ij.  This is the paper's "only the couplings of
// the flipped sites" rule (Sec. III, cost paragraph) with F cached per state.
//
// Kernels of one step, in launch order:
//   k_step_begin  clear per-step counters
//   k_frontier    per search: list its new states; cut = M-th kept energy,
//                 tightened by a pilot (exact energies of the pair flips among
//                 the lightest sites of its lowest new state)
//   k_plan        per-instance work prefix sums for the scan and the prep
//   k_prep        per frontier state: a_i, the scan threshold, single flips
//   k_scan        per (instance, chunk of states, 64x64 tile of pairs): every
//                 pair energy change, filtered by the cut, survivors recorded
//   k_merge       per search: sort kept + survivors by (E, psi), drop
//                 duplicates, keep M, write new states and their local fields
#include "common.h"

namespace qi {

// ------------------------------------------------------------------ helpers
__device__ inline uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ inline uint32_t mbcnt64(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ inline int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ inline double spin_of(const uint64_t* x, int i)
{
    return ((x[i >> 6] >> (i & 63)) & 1ull) ? -1.0 : 1.0;
}

// Exclusive prefix sum of v over a block of 256 threads; returns the total.
__device__ int block_exclusive_scan(int v, int* tmp, int& excl)
{
    const int t = threadIdx.x;
    tmp[t] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int add = t >= off ? tmp[t - off] : 0;
        __syncthreads();
        tmp[t] += add;
        __syncthreads();
    }
    excl = tmp[t] - v;
    const int total = tmp[255];
    __syncthreads();
    return total;
}

// ------------------------------------------------------------------ k_step_begin
__global__ void k_step_begin(Layout lay, int retry_mode)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (!retry_mode && t < lay.B) lay.fr_count[t] = 0;
    if (t < lay.S && (!retry_mode || lay.retry[t])) lay.surv_count[t] = 0;
    // a retry pass keeps the count of searches that already committed
    if (t == FLAG_OVERFLOW || t == FLAG_STUCK) lay.flags[t] = 0;
    if (t == FLAG_ACTIVE && !retry_mode) lay.flags[t] = 0;
    if (t == FLAG_RETRY_MODE) lay.flags[t] = retry_mode;
}

// ------------------------------------------------------------------ bitonic sort of (key, idx) in LDS
template <class Less>
__device__ void bitonic_sort(double* key, uint32_t* idx, int n2, const Less& less)
{
    for (int k = 2; k <= n2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < (n2 >> 1); t += blockDim.x) {
                const int i = 2 * j * (t / j) + (t % j);
                const int l = i + j;
                const bool up = (i & k) == 0;
                const bool swap = up ? less(key[l], idx[l], key[i], idx[i]) : less(key[i], idx[i], key[l], idx[l]);
                if (swap) {
                    const double tk = key[i]; key[i] = key[l]; key[l] = tk;
                    const uint32_t ti = idx[i]; idx[i] = idx[l]; idx[l] = ti;
                }
            }
            __syncthreads();
        }
    }
}

struct PlainLess {
    __device__ bool operator()(double a, uint32_t ia, double b, uint32_t ib) const
    {
        return a < b || (a == b && ia < ib);
    }
};

__device__ inline int pow2_at_least(int n)
{
    int p = 1;
    while (p < n) p <<= 1;
    return p;
}

// ------------------------------------------------------------------ k_frontier
// One block per search.  Lists the states that entered in the last step (the
// only ones whose neighbourhoods can hold anything new), and sets the cut on
// child energies.  The cut starts at the M-th kept energy (a child above it
// ranks behind the whole kept set, the paper's "E < E_{K+1}" acceptance test).
// The pilot tightens it: the M lowest of any M distinct children of one state
// bound the M-th lowest distinct state of the union from above, so
//   cut = min(E_M, E_p + theta),  theta = M-th smallest energy change among
// the single flips of the K lightest sites of the lowest new state p and the
// pair flips among them (exact values; only their selection is heuristic).
__global__ __launch_bounds__(256) void k_frontier(Layout lay, const double* __restrict__ J4)
{
    __shared__ double key[MAX_N];
    __shared__ uint32_t idx[MAX_N];
    __shared__ int tmp[256];
    __shared__ int s_pilot;
    const int s = blockIdx.x;
    const int b = s / lay.L;
    const int M = lay.M;
    if (!lay.active[s]) {
        if (threadIdx.x == 0) lay.cut[s] = -INFINITY;
        return;
    }
    const int nk = lay.nkept[s];
    const int* kept = lay.kept + (size_t)s * M;
    const size_t q0 = (size_t)s * 2 * M;

    // rank the new states in kept (energy) order
    int base_rank = 0;
    if (threadIdx.x == 0) s_pilot = -1;
    __syncthreads();
    int fr_base = 0;
    for (int c0 = 0; c0 < nk; c0 += 256) {
        const int k = c0 + threadIdx.x;
        const int slot = k < nk ? kept[k] : 0;
        const int isnew = (k < nk && lay.fresh[q0 + slot]) ? 1 : 0;
        int excl;
        const int tot = block_exclusive_scan(isnew, tmp, excl);
        if (isnew) idx[base_rank + excl] = (uint32_t)slot;   // temporary list of new slots
        base_rank += tot;
    }
    __syncthreads();
    const int nfresh = base_rank;
    if (threadIdx.x == 0 && nfresh > 0) {
        fr_base = atomicAdd(&lay.fr_count[b], nfresh);
        s_pilot = (int)idx[0];
        tmp[0] = fr_base;
    }
    __syncthreads();
    if (nfresh > 0) {
        fr_base = tmp[0];
        for (int r = threadIdx.x; r < nfresh; r += blockDim.x)
            lay.fr_list[(size_t)b * lay.fmax + fr_base + r] = (int)(s * 2 * M + idx[r]);
    }
    const double ecut = nk == M ? lay.E[q0 + kept[M - 1]] : INFINITY;
    __syncthreads();
    if (nfresh == 0) {
        if (threadIdx.x == 0) lay.cut[s] = ecut;
        return;
    }

    // pilot: lowest new state p (first new one in energy order)
    const int N = lay.N[b], Np = lay.Npad[b];
    const int ps = s_pilot;
    const uint64_t* xp = lay.bits + (q0 + ps) * lay.Wmax;
    const double* Fp = lay.F + (q0 + ps) * lay.Npmax;
    const double Ep = lay.E[q0 + ps];
    const int n2 = pow2_at_least(N);
    for (int i = threadIdx.x; i < n2; i += blockDim.x) {
        key[i] = i < N ? -2.0 * spin_of(xp, i) * Fp[i] : INFINITY;
        idx[i] = (uint32_t)i;
    }
    __syncthreads();
    bitonic_sort(key, idx, n2, PlainLess());
    const int K = N < PILOT_K ? N : PILOT_K;
    const int nc = K * (K + 1) / 2;
    double theta = INFINITY;
    if (nc >= M) {
        // candidates: K singles and K(K-1)/2 pairs, written behind the sorted prefix
        __shared__ double aK[PILOT_K];
        __shared__ int iK[PILOT_K];
        if (threadIdx.x < K) {
            aK[threadIdx.x] = key[threadIdx.x];
            iK[threadIdx.x] = (int)idx[threadIdx.x];
        }
        __syncthreads();
        const double* Jb = J4 + lay.joff[b];
        const int n2c = pow2_at_least(nc);
        for (int t = threadIdx.x; t < n2c; t += blockDim.x) {
            double v = INFINITY;
            if (t < K) {
                v = aK[t];
            } else if (t < nc) {
                // t - K enumerates pairs (p, r), p < r < K
                int u = t - K, p = 0;
                while (u >= K - 1 - p) { u -= K - 1 - p; ++p; }
                const int r = p + 1 + u;
                const int i = iK[p], j = iK[r];
                const double sij = spin_of(xp, i) * spin_of(xp, j);
                v = aK[p] + aK[r] + sij * Jb[(size_t)i * Np + j];
            }
            key[t] = v;
            idx[t] = (uint32_t)t;
        }
        __syncthreads();
        bitonic_sort(key, idx, n2c, PlainLess());
        theta = key[M - 1];
    }
    if (threadIdx.x == 0) {
        const double c = Ep + theta;
        lay.cut[s] = c < ecut ? c : ecut;
    }
}

// ------------------------------------------------------------------ k_plan
// One block.  Work prefix sums over instances: scan items (chunks x tiles)
// and frontier entries; also the evaluation counters.
__global__ __launch_bounds__(1024) void k_plan(Layout lay, long long* __restrict__ fr_prefix)
{
    __shared__ long long part_items[1024];
    __shared__ long long part_fr[1024];
    const int t = threadIdx.x;
    const int per = (lay.B + 1023) / 1024;
    const int b0 = t * per;
    long long items = 0, fr = 0, pairs = 0, singles = 0;
    for (int b = b0; b < b0 + per && b < lay.B; ++b) {
        const long long P = lay.fr_count[b];
        const long long N = lay.N[b];
        items += (P + lay.sc - 1) / lay.sc * tiles_of((int)N);
        fr += P;
        pairs += P * (N * (N - 1) / 2);
        singles += P * N;
    }
    part_items[t] = items;
    part_fr[t] = fr;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const long long ai = t >= off ? part_items[t - off] : 0;
        const long long af = t >= off ? part_fr[t - off] : 0;
        __syncthreads();
        part_items[t] += ai;
        part_fr[t] += af;
        __syncthreads();
    }
    long long run_i = part_items[t] - items, run_f = part_fr[t] - fr;
    for (int b = b0; b < b0 + per && b < lay.B; ++b) {
        lay.item_prefix[b] = run_i;
        fr_prefix[b] = run_f;
        const long long P = lay.fr_count[b];
        run_i += (P + lay.sc - 1) / lay.sc * tiles_of(lay.N[b]);
        run_f += P;
    }
    if (t == 1023) {
        lay.item_prefix[lay.B] = part_items[1023];
        fr_prefix[lay.B] = part_fr[1023];
    }
    // counters (the retry pass counts in k_prep instead)
    __shared__ unsigned long long cp[1024], cs[1024];
    cp[t] = (unsigned long long)pairs;
    cs[t] = (unsigned long long)singles;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (t < w) { cp[t] += cp[t + w]; cs[t] += cs[t + w]; }
        __syncthreads();
    }
    if (t == 0 && !lay.flags[FLAG_RETRY_MODE]) {
        lay.ctr[CTR_PAIRS] += cp[0];
        lay.ctr[CTR_SINGLES] += cs[0];
        lay.ctr[CTR_FRONTIER] += (unsigned long long)part_fr[1023];
        lay.ctr[CTR_STEPS] += 1;
    }
}

__device__ inline int find_instance(const long long* prefix, int B, long long e)
{
    int lo = 0, hi = B;   // prefix[lo] <= e < prefix[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

// ------------------------------------------------------------------ k_prep
// One wave per frontier entry: a_i = -2 s_i F_i, the scan threshold
// T = cut - E (a pair survives iff a_i + a_j + 4 s_i s_j J_ij <= T), and the
// single flips below the cut.
__global__ __launch_bounds__(256) void k_prep(Layout lay, const long long* __restrict__ fr_prefix)
{
    const long long total = fr_prefix[lay.B];
    const int wave = threadIdx.x >> 6;
    const uint32_t lane = threadIdx.x & 63;
    const int retry_mode = lay.flags[FLAG_RETRY_MODE];
    for (long long e = (long long)blockIdx.x * 4 + wave; e < total; e += (long long)gridDim.x * 4) {
        const int b = find_instance(fr_prefix, lay.B, e);
        const int f = (int)(e - fr_prefix[b]);
        const int code = lay.fr_list[(size_t)b * lay.fmax + f];
        const int s = code / (2 * lay.M);
        if (retry_mode && !lay.retry[s]) continue;
        const size_t q = (size_t)code;   // s*2M + slot
        const int N = lay.N[b], Np = lay.Npad[b];
        const double Em = lay.E[q];
        const double c = lay.cut[s];
        const uint64_t* x = lay.bits + q * lay.Wmax;
        const double* F = lay.F + q * lay.Npmax;
        double* A = lay.A + ((size_t)b * lay.fmax + f) * lay.Npmax;
        if (lane == 0) lay.T[(size_t)b * lay.fmax + f] = c - Em;
        if (retry_mode && lane == 0) {
            atomicAdd(&lay.ctr[CTR_PAIRS], (unsigned long long)N * (N - 1) / 2);
            atomicAdd(&lay.ctr[CTR_SINGLES], (unsigned long long)N);
        }
        for (int i0 = 0; i0 < Np; i0 += 64) {
            const int i = i0 + lane;
            double a = 0.0;
            if (i < N) a = -2.0 * spin_of(x, i) * F[i];
            A[i] = a;
            const double Ec = Em + a;
            const bool hit = i < N && Ec <= c;
            const uint64_t m = __builtin_amdgcn_ballot_w64(hit);
            if (m) {
                int base = 0;
                if (lane == 0) base = atomicAdd(&lay.surv_count[s], __builtin_popcountll(m));
                base = __shfl(base, 0, 64);
                if (hit) {
                    const int pos = base + (int)mbcnt64(m);
                    if (pos < lay.cap_surv) {
                        Surv r;
                        r.E = Ec;
                        r.f = (uint32_t)f;
                        r.pair = (uint32_t)i | (SINGLE << 16);
                        lay.surv[(size_t)s * lay.cap_surv + pos] = r;
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------------------ k_scan
// One wave per work item (instance b, chunk of sc frontier states, tile of
// 64 rows i x 64 columns j with row block <= column block).  Lane = row i;
// the wave holds the 64 values 4J_ij of its row in registers and walks the
// chunk's states, so each tile load serves sc states.  For state m the pair
// (i,j) survives iff a_j + s_i s_j 4J_ij <= T_m - a_i.  The sign s_i s_j is
// applied in place to the high word of the register copy: the stored sign
// changes between consecutive states by (bit_i ^ bit_i') ^ (bit_j ^ bit_j'),
// and adding 2^31 flips bit 31 exactly like xor, so (hi ^ di) + dj is a
// single v_xad_u32.  Pairs outside the triangle or the instance hold NaN,
// which never passes the test.  a_j is wave-uniform (scalar loads).
// Survivors are staged in LDS and appended to the search's record buffer
// with one atomic per flush.
__device__ inline void flush_stage(const Layout& lay, Surv* stage, int& n, int s)
{
    if (n == 0) return;
    __syncthreads();
    int base = 0;
    if (lane_id() == 0) base = atomicAdd(&lay.surv_count[s], n);
    base = __shfl(base, 0, 64);
    for (int k = (int)lane_id(); k < n; k += 64) {
        const int pos = base + k;
        if (pos < lay.cap_surv) lay.surv[(size_t)s * lay.cap_surv + pos] = stage[k];
    }
    __syncthreads();
    n = 0;
}

__global__ __launch_bounds__(64) void k_scan(Layout lay, const double* __restrict__ J4,
                                             const double* __restrict__ Abuf,
                                             const double* __restrict__ Tbuf,
                                             const int* __restrict__ frl)
{
    __shared__ Surv stage[STAGE];
    const uint32_t lane = lane_id();
    const long long total = lay.item_prefix[lay.B];
    const int retry_mode = lay.flags[FLAG_RETRY_MODE];
    const int M2 = 2 * lay.M;
    for (long long item = blockIdx.x; item < total; item += gridDim.x) {
        const int b = uniform_int(find_instance(lay.item_prefix, lay.B, item));
        const long long r = item - lay.item_prefix[b];
        const int N = lay.N[b], Np = lay.Npad[b];
        const int nb = Np / TILE;
        const long long T = tiles_of(N);
        const int c = (int)(r / T);
        int t = (int)(r % T);
        int bi = 0;
        while (t >= nb - bi) { t -= nb - bi; ++bi; }
        const int bj = bi + t;
        bi = uniform_int(bi);
        const int bjj = uniform_int(bj);
        const int P = lay.fr_count[b];
        const int f0 = c * lay.sc;
        const int f1 = min(f0 + lay.sc, P);

        // the tile: row i = bi*64 + lane, columns j = bjj*64 + 0..63
        const int row = bi * TILE + (int)lane;
        const double* Jt = J4 + lay.joff[b];
        uint64_t Jb[TILE];
#pragma unroll
        for (int j = 0; j < TILE; ++j) {
            const int col = bjj * TILE + j;
            double v = Jt[(size_t)col * Np + row];   // symmetric: (col,row) = (row,col)
            const bool ok = row < N && col < N && (bi != bjj || j > (int)lane);
            Jb[j] = ok ? (uint64_t)__double_as_longlong(v) : 0x7ff8000000000000ull;
        }
        uint32_t prev_i = 0;
        uint64_t prev_wj = 0;
        int nstage = 0, sstage = -1;
        for (int f = f0; f < f1; ++f) {
            const int code = uniform_int(frl[(size_t)b * lay.fmax + f]);
            const int s = code / M2;
            if (retry_mode && !lay.retry[s]) continue;
            if (s != sstage) {
                flush_stage(lay, stage, nstage, sstage);
                sstage = s;
            }
            const uint64_t* xb = lay.bits + (size_t)code * lay.Wmax;
            const uint64_t wi = xb[bi];
            const uint64_t wj = xb[bjj];
            const size_t arow = ((size_t)b * lay.fmax + f) * lay.Npmax;
            const double tm = Tbuf[(size_t)b * lay.fmax + f];
            const double ai = Abuf[arow + row];
            const double Ea = lay.E[code] + ai;
            const double rr = row < N ? tm - ai : -INFINITY;
            const uint32_t cur_i = (uint32_t)(wi >> lane) & 1u;
            const uint32_t di = (cur_i ^ prev_i) << 31;
            prev_i = cur_i;
            const uint64_t dw = wj ^ prev_wj;
            prev_wj = wj;
            const double* aj = Abuf + arow + (size_t)bjj * TILE;
#pragma unroll
            for (int g = 0; g < TILE; g += 8) {
                uint64_t m[8];
                double x[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int j = g + u;
                    const uint32_t dj = (uint32_t)((dw >> j) & 1ull) << 31;
                    const uint32_t hi = (((uint32_t)(Jb[j] >> 32)) ^ di) + dj;
                    Jb[j] = (Jb[j] & 0xffffffffull) | ((uint64_t)hi << 32);
                    x[u] = aj[j] + __longlong_as_double((long long)Jb[j]);
                    m[u] = __builtin_amdgcn_ballot_w64(x[u] <= rr);
                }
                const uint64_t any = m[0] | m[1] | m[2] | m[3] | m[4] | m[5] | m[6] | m[7];
                if (any) {
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        if (m[u]) {
                            if (nstage > STAGE - 64) flush_stage(lay, stage, nstage, s);
                            if ((m[u] >> lane) & 1ull) {
                                Surv rec;
                                rec.E = Ea + x[u];
                                rec.f = (uint32_t)f;
                                rec.pair = (uint32_t)row | ((uint32_t)(bjj * TILE + g + u) << 16);
                                stage[nstage + (int)mbcnt64(m[u])] = rec;
                            }
                            nstage += __builtin_popcountll(m[u]);
                        }
                    }
                }
            }
        }
        flush_stage(lay, stage, nstage, sstage);
    }
}

// ------------------------------------------------------------------ merge helpers
// Candidate sources give the energy and the packed words of a candidate.
struct SearchSrc {
    const Layout* lay;
    int s, b;
    __device__ uint64_t word(uint32_t ref, int w) const
    {
        const size_t q0 = (size_t)s * 2 * lay->M;
        if (ref & REF_SURV) {
            const Surv r = lay->surv[(size_t)s * lay->cap_surv + (ref & ~REF_SURV)];
            const int code = lay->fr_list[(size_t)b * lay->fmax + r.f];
            uint64_t v = lay->bits[(size_t)code * lay->Wmax + w];
            const int i = (int)(r.pair & 0xFFFFu), j = (int)(r.pair >> 16);
            if ((i >> 6) == w) v ^= 1ull << (i & 63);
            if (j != (int)SINGLE && (j >> 6) == w) v ^= 1ull << (j & 63);
            return v;
        }
        const int slot = lay->kept[(size_t)s * lay->M + ref];
        return lay->bits[(q0 + slot) * lay->Wmax + w];
    }
};

struct InstanceSrc {
    const Layout* lay;
    int b;
    __device__ uint64_t word(uint32_t ref, int w) const
    {
        const int l = (int)(ref / (uint32_t)lay->M), k = (int)(ref % (uint32_t)lay->M);
        const int s = b * lay->L + l;
        const int slot = lay->kept[(size_t)s * lay->M + k];
        return lay->bits[((size_t)s * 2 * lay->M + slot) * lay->Wmax + w];
    }
};

constexpr uint32_t REF_PAD = 0xFFFFFFFFu;

// (E, psi, ref): psi compared as an unsigned integer from the highest word.
template <class Src>
struct StateLess {
    const Src* src;
    int W;
    __device__ bool operator()(double a, uint32_t ia, double b, uint32_t ib) const
    {
        if (a < b) return true;
        if (a > b) return false;
        if (ia == REF_PAD || ib == REF_PAD) return ia < ib;
        for (int w = W - 1; w >= 0; --w) {
            const uint64_t x = src->word(ia, w), y = src->word(ib, w);
            if (x != y) return x < y;
        }
        return ia < ib;
    }
};

template <class Src>
__device__ bool same_state(const Src& src, int W, double a, uint32_t ia, double b, uint32_t ib)
{
    if (a != b || ia == REF_PAD || ib == REF_PAD) return false;
    for (int w = W - 1; w >= 0; --w)
        if (src.word(ia, w) != src.word(ib, w)) return false;
    return true;
}

// Sorts key/ref[0..n), drops duplicates (the first of equal states is kept;
// the order puts a kept state before its copies), keeps the first M distinct
// at the front.  Returns their count.
template <class Src>
__device__ int sort_dedupe_keep(const Src& src, int W, double* key, uint32_t* ref, int n, int M,
                                int* tmp, uint8_t* keep)
{
    const int n2 = pow2_at_least(n < 2 ? 2 : n);
    for (int t = n + threadIdx.x; t < n2; t += blockDim.x) {
        key[t] = INFINITY;
        ref[t] = REF_PAD;
    }
    __syncthreads();
    StateLess<Src> less{&src, W};
    bitonic_sort(key, ref, n2, less);
    for (int t = threadIdx.x; t < n; t += blockDim.x)
        keep[t] = (t == 0 || !same_state(src, W, key[t - 1], ref[t - 1], key[t], ref[t])) ? 1 : 0;
    __syncthreads();
    // compact the first M distinct, in order, in chunks of 256
    int out = 0;
    __shared__ double ck[256];
    __shared__ uint32_t cr[256];
    for (int c0 = 0; c0 < n && out < M; c0 += 256) {
        const int t = c0 + threadIdx.x;
        const int kf = t < n ? keep[t] : 0;
        int excl;
        const int tot = block_exclusive_scan(kf, tmp, excl);
        double kv = 0.0;
        uint32_t rv = 0;
        if (kf) { kv = key[t]; rv = ref[t]; }
        __syncthreads();
        if (kf && out + excl < M) {
            ck[excl] = kv;
            cr[excl] = rv;
        }
        __syncthreads();
        const int take = min(tot, M - out);
        if ((int)threadIdx.x < take) {
            key[out + threadIdx.x] = ck[threadIdx.x];
            ref[out + threadIdx.x] = cr[threadIdx.x];
        }
        __syncthreads();
        out += take;
    }
    return out;
}

// ------------------------------------------------------------------ k_merge
// One block per active search.  Kept set and survivors are merged in passes of
// MERGE_CH candidates: each pass sorts the running best list plus the next
// survivors by (E, psi), drops duplicates and keeps M.  A survivor buffer that
// overflowed only yields a tighter cut (its M-th distinct energy) for a
// re-scan.  Otherwise the new kept set is written: new states take slots the
// old set does not use, with bits = parent xor flips, E from the record and
// F_k = F_k(parent) - 2 s_i J_ik - 2 s_j J_jk.
__global__ __launch_bounds__(256) void k_merge(Layout lay, const double* __restrict__ J4)
{
    __shared__ double key[MERGE_CH];
    __shared__ uint32_t ref[MERGE_CH];
    __shared__ uint8_t keep[MERGE_CH];
    __shared__ int tmp[256];
    __shared__ int freeslot[2048];
    __shared__ int kslot[1024];
    __shared__ uint8_t used[2048];
    const int s = blockIdx.x;
    const int b = s / lay.L;
    const int M = lay.M;
    const int retry_mode = lay.flags[FLAG_RETRY_MODE];
    if (!lay.active[s]) return;
    if (retry_mode && !lay.retry[s]) return;
    const int nk = lay.nkept[s];
    const int ctot = lay.surv_count[s];
    const int cnt = ctot < lay.cap_surv ? ctot : lay.cap_surv;
    const size_t q0 = (size_t)s * 2 * M;
    const int W = words_of(lay.N[b]);
    SearchSrc src{&lay, s, b};

    for (int k = threadIdx.x; k < nk; k += blockDim.x) {
        key[k] = lay.E[q0 + lay.kept[(size_t)s * M + k]];
        ref[k] = (uint32_t)k;
    }
    __syncthreads();
    int nrun = nk;
    int pos = 0;
    do {
        const int room = MERGE_CH - nrun;
        const int take = min(cnt - pos, room);
        for (int t = threadIdx.x; t < take; t += blockDim.x) {
            key[nrun + t] = lay.surv[(size_t)s * lay.cap_surv + pos + t].E;
            ref[nrun + t] = REF_SURV | (uint32_t)(pos + t);
        }
        __syncthreads();
        nrun = sort_dedupe_keep(src, W, key, ref, nrun + take, M, tmp, keep);
        pos += take;
    } while (pos < cnt);

    if (threadIdx.x == 0) atomicAdd(&lay.ctr[CTR_SURV], (unsigned long long)cnt);
    if (ctot > lay.cap_surv) {
        // some candidates were not stored: the stored ones still bound the cut
        if (threadIdx.x == 0) {
            const double oldc = lay.cut[s];
            const double nc = nrun == M ? key[M - 1] : oldc;
            lay.cut[s] = nc;
            lay.retry[s] = 1;
            atomicAdd(&lay.flags[FLAG_OVERFLOW], 1);
            atomicAdd(&lay.ctr[CTR_RETRY], 1ull);
            if (!(nc < oldc)) atomicAdd(&lay.flags[FLAG_STUCK], 1);
        }
        return;
    }

    // slots used by the current set; new states take the free ones in order
    for (int q = threadIdx.x; q < 2 * M; q += blockDim.x) used[q] = 0;
    __syncthreads();
    for (int k = threadIdx.x; k < nk; k += blockDim.x) used[lay.kept[(size_t)s * M + k]] = 1;
    __syncthreads();
    int nfree = 0;
    for (int c0 = 0; c0 < 2 * M; c0 += 256) {
        const int q = c0 + threadIdx.x;
        const int isfree = (q < 2 * M && !used[q]) ? 1 : 0;
        int excl;
        const int tot = block_exclusive_scan(isfree, tmp, excl);
        if (isfree) freeslot[nfree + excl] = q;
        nfree += tot;
    }
    __syncthreads();
    // position of each new state among the new ones
    int nnew = 0;
    for (int c0 = 0; c0 < nrun; c0 += 256) {
        const int k = c0 + threadIdx.x;
        const int isnew = (k < nrun && (ref[k] & REF_SURV)) ? 1 : 0;
        int excl;
        const int tot = block_exclusive_scan(isnew, tmp, excl);
        if (k < nrun) {
            int slot;
            if (isnew) {
                slot = freeslot[nnew + excl];
                keep[k] = 1;
            } else {
                slot = lay.kept[(size_t)s * M + ref[k]];
                keep[k] = 0;
            }
            kslot[k] = slot;
        }
        nnew += tot;
    }
    __syncthreads();
    // old members that stay are no longer new
    for (int k = threadIdx.x; k < nrun; k += blockDim.x)
        if (!keep[k]) lay.fresh[q0 + kslot[k]] = 0;
    // new members: bits, energy, hash, flag
    const int N = lay.N[b], Np = lay.Npad[b];
    for (int k = threadIdx.x; k < nrun; k += blockDim.x) {
        if (!keep[k]) continue;
        const Surv r = lay.surv[(size_t)s * lay.cap_surv + (ref[k] & ~REF_SURV)];
        const int code = lay.fr_list[(size_t)b * lay.fmax + r.f];
        const int slot = kslot[k];
        const int i = (int)(r.pair & 0xFFFFu), j = (int)(r.pair >> 16);
        const uint64_t* xp = lay.bits + (size_t)code * lay.Wmax;
        uint64_t* xn = lay.bits + (q0 + slot) * lay.Wmax;
        for (int w = 0; w < lay.Wmax; ++w) {
            uint64_t v = xp[w];
            if ((i >> 6) == w) v ^= 1ull << (i & 63);
            if (j != (int)SINGLE && (j >> 6) == w) v ^= 1ull << (j & 63);
            xn[w] = v;
        }
        uint64_t z = lay.zob[code] ^ lay.zkey[i];
        if (j != (int)SINGLE) z ^= lay.zkey[j];
        lay.zob[q0 + slot] = z;
        lay.E[q0 + slot] = r.E;
        lay.fresh[q0 + slot] = 1;
    }
    // local fields of new members: one member at a time, threads over sites
    const double* Jb = J4 + lay.joff[b];
    for (int k = 0; k < nrun; ++k) {
        if (!keep[k]) continue;
        const Surv r = lay.surv[(size_t)s * lay.cap_surv + (ref[k] & ~REF_SURV)];
        const int code = lay.fr_list[(size_t)b * lay.fmax + r.f];
        const int slot = kslot[k];
        const int i = (int)(r.pair & 0xFFFFu), j = (int)(r.pair >> 16);
        const uint64_t* xp = lay.bits + (size_t)code * lay.Wmax;
        const double ci = -0.5 * spin_of(xp, i);                       // -2 s_i J = -0.5 s_i (4J)
        const double cj = j != (int)SINGLE ? -0.5 * spin_of(xp, j) : 0.0;
        const double* Fp = lay.F + (size_t)code * lay.Npmax;
        double* Fn = lay.F + (q0 + slot) * lay.Npmax;
        const double* Ji = Jb + (size_t)i * Np;
        const double* Jj = Jb + (size_t)(j != (int)SINGLE ? j : i) * Np;
        for (int kk = threadIdx.x; kk < Np; kk += blockDim.x) {
            double v = Fp[kk] + ci * Ji[kk];
            if (j != (int)SINGLE) v += cj * Jj[kk];
            Fn[kk] = kk < N ? v : 0.0;
        }
    }
    for (int k = threadIdx.x; k < nrun; k += blockDim.x)
        lay.kept[(size_t)s * M + k] = kslot[k];
    if (threadIdx.x == 0) {
        lay.nkept[s] = nrun;
        lay.retry[s] = 0;
        if (nnew > 0) atomicAdd(&lay.flags[FLAG_ACTIVE], 1);
        else lay.active[s] = 0;
    }
}

// ------------------------------------------------------------------ k_final
// Alg. 4: per instance, the M lowest distinct states of the union of its L
// kept sets, sorted by (E, psi).
__global__ __launch_bounds__(256) void k_final(Layout lay)
{
    __shared__ double key[MERGE_CH];
    __shared__ uint32_t ref[MERGE_CH];
    __shared__ uint8_t keep[MERGE_CH];
    __shared__ int tmp[256];
    const int b = blockIdx.x;
    const int M = lay.M;
    const int W = words_of(lay.N[b]);
    InstanceSrc src{&lay, b};
    int nrun = 0;
    int l = 0;
    while (l < lay.L) {
        // append whole searches while they fit
        int n = nrun;
        while (l < lay.L) {
            const int s = b * lay.L + l;
            const int nk = lay.nkept[s];
            if (n + nk > MERGE_CH) break;
            for (int k = threadIdx.x; k < nk; k += blockDim.x) {
                const int slot = lay.kept[(size_t)s * M + k];
                key[n + k] = lay.E[(size_t)s * 2 * M + slot];
                ref[n + k] = (uint32_t)(l * M + k);
            }
            n += nk;
            ++l;
        }
        __syncthreads();
        nrun = sort_dedupe_keep(src, W, key, ref, n, M, tmp, keep);
    }
    for (int k = threadIdx.x; k < nrun; k += blockDim.x) {
        lay.out_E[(size_t)b * M + k] = key[k];
        for (int w = 0; w < lay.Wmax; ++w)
            lay.out_bits[((size_t)b * M + k) * lay.Wmax + w] = w < W ? src.word(ref[k], w) : 0ull;
    }
    if (threadIdx.x == 0) lay.out_count[b] = nrun;
}

// ------------------------------------------------------------------ launchers
hipError_t launch_step_begin(const Layout& lay, bool retry_mode, hipStream_t st)
{
    const int n = (lay.B > lay.S ? lay.B : lay.S) + 8;
    hipLaunchKernelGGL(k_step_begin, dim3((n + 255) / 256), dim3(256), 0, st, lay, retry_mode ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_step(const Layout& lay, int scan_grid, bool retry_mode, hipStream_t st)
{
    long long* fr_prefix = lay.item_prefix + (lay.B + 1);
    if (!retry_mode) {
        hipLaunchKernelGGL(k_frontier, dim3(lay.S), dim3(256), 0, st, lay, lay.J4);
        hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, st, lay, fr_prefix);
    }
    hipLaunchKernelGGL(k_prep, dim3(4096), dim3(256), 0, st, lay, (const long long*)fr_prefix);
    hipLaunchKernelGGL(k_scan, dim3(scan_grid), dim3(64), 0, st, lay, lay.J4, (const double*)lay.A,
                       (const double*)lay.T, (const int*)lay.fr_list);
    hipLaunchKernelGGL(k_merge, dim3(lay.S), dim3(256), 0, st, lay, lay.J4);
    return hipGetLastError();
}

hipError_t launch_final(const Layout& lay, hipStream_t st)
{
    hipLaunchKernelGGL(k_final, dim3(lay.B), dim3(256), 0, st, lay);
    return hipGetLastError();
}

}  // namespace qi

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
//   k_scan        per (instance, chunk of states, 64x32 tile of pairs): every
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

// Word k of a state held one word per lane (lane k), as a wave-uniform value.

// blocks of 64 sites whose loads a preparation wave issues together
constexpr int PREP_BLOCKS = 8;

__device__ inline double spin_of(const uint64_t* x, int i)
{
    return ((x[i >> 6] >> (i & 63)) & 1ull) ? -1.0 : 1.0;
}

// Exclusive prefix sum of v over a block of 256 threads; returns the total.
// Inclusive sums within each wave by shuffles, then the four wave totals.
__device__ int block_exclusive_scan(int v, int* tmp, int& excl)
{
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    int incl = v;
    for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(incl, off, 64);
        if (lane >= off) incl += u;
    }
    if (lane == 63) tmp[w] = incl;
    __syncthreads();
    int base = 0, total = 0;
    for (int k = 0; k < 4; ++k) {
        const int sk = tmp[k];
        base += k < w ? sk : 0;
        total += sk;
    }
    excl = base + incl - v;
    __syncthreads();   // tmp is reused by the next call
    return total;
}

// Within one wave, LDS accesses complete in program order, so stages of a
// sort that stay inside the wave's own elements need no block barrier.
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------ k_step_begin
__global__ void k_step_begin(Layout lay, int retry_mode)
{
    if (step_halted(lay)) return;   // a later step of a multi-step graph after a halt
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (!retry_mode && t < lay.B) {
        lay.fr_count[t] = 0;
        lay.lr_count[t] = 0;
    }
    if (t < lay.S && (!retry_mode || lay.retry[t])) lay.surv_count[t] = 0;
    // a retry pass keeps the count of searches that already committed
    if (t == FLAG_OVERFLOW || t == FLAG_STUCK) lay.flags[t] = 0;
    if (t == FLAG_ACTIVE && !retry_mode) lay.flags[t] = 0;
    if (t == FLAG_RETRY_MODE) lay.flags[t] = retry_mode;
}

// ------------------------------------------------------------------ bitonic sort of (key, idx) in LDS
// Blocks of 256 threads.  Pair p of a stage with distance j touches elements
// 2j floor(p/j) + p%j and that plus j; for j <= 64 the pairs of one wave
// (p in 64w + 256m .. +63) stay inside element blocks 128(w + 4m) .. +127,
// so only stages with j >= 128 exchange data between waves.
template <class Less>
__device__ void bitonic_sort(double* key, uint32_t* idx, int n2, const Less& less)
{
    __syncthreads();
    for (int k = 2; k <= n2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= 128) __syncthreads();
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
            if (j >= 128) __syncthreads();
            else wave_sync();
        }
    }
    __syncthreads();
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
// Pilots tighten it: any M distinct members of the union bound its M-th
// lowest distinct energy from above, whichever children they are.  The pilots
// are the NPIL lowest new states, one wave each: every lane takes the lightest
// of its sites (i = lane mod 64, lowest a_i), the wave sorts the 64, and the
// pilot offers the single flips of the PKW lightest of them and the pair flips
// among these, with exact energies (more pilots with fewer sites each give a
// tighter cut than a few pilots with many sites).  A ranking step (learned
// form) instead takes the singles of the PRANK lightest sites of NPILOT
// pilots.  Two children of pilots p, q are the same state iff x_p xor x_q
// equals the symmetric difference of their flip sets, which is checked exactly
// from the pilots' words, so the pool's M-th distinct energy is a valid cut.
// Sorts by (value, index) the shortest prefix of the (value, index) order of
// n elements that holds at least `need` of them, into key/idx[0..cnt), and
// returns cnt.  A 256-bin histogram over [min, max] finds the prefix: every
// value of a bin lies below every value of a later bin, so whole bins form a
// prefix of the order.  get(k, v, id) yields element k.  Block of 256 threads.
struct PrefixShared {
    double red[8];
    int hist[256];
    int bstar, cnt, fill;
};

template <class Get>
__device__ int sort_prefix(const Get& get, int n, int need, double* key, uint32_t* idx, PrefixShared& ps)
{
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    double lo = INFINITY, hi = -INFINITY;
    for (int k = t; k < n; k += blockDim.x) {
        double v;
        uint32_t id;
        get(k, v, id);
        lo = fmin(lo, v);
        hi = fmax(hi, v);
    }
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off, 64));
        hi = fmax(hi, __shfl_xor(hi, off, 64));
    }
    if (lane == 0) {
        ps.red[w] = lo;
        ps.red[4 + w] = hi;
    }
    ps.hist[t] = 0;
    if (t == 0) ps.fill = 0;
    __syncthreads();
    lo = fmin(fmin(ps.red[0], ps.red[1]), fmin(ps.red[2], ps.red[3]));
    hi = fmax(fmax(ps.red[4], ps.red[5]), fmax(ps.red[6], ps.red[7]));
    const double scale = hi > lo ? 256.0 / (hi - lo) : 0.0;
    auto bin_of = [&](double v) -> int {
        const int k = (int)((v - lo) * scale);
        return k < 0 ? 0 : (k > 255 ? 255 : k);
    };
    for (int k = t; k < n; k += blockDim.x) {
        double v;
        uint32_t id;
        get(k, v, id);
        atomicAdd(&ps.hist[bin_of(v)], 1);
    }
    __syncthreads();
    if (t < 64) {
        // lane l holds bins 4l .. 4l+3 (lowest first)
        int c[4], loc = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            c[u] = ps.hist[4 * t + u];
            loc += c[u];
        }
        int incl = loc;
        for (int off = 1; off < 64; off <<= 1) {
            const int v = __shfl_up(incl, off, 64);
            if (t >= off) incl += v;
        }
        int run = incl - loc;
        if (run < need && need <= incl) {
            for (int u = 0; u < 4; ++u) {
                run += c[u];
                if (run >= need) {
                    ps.bstar = 4 * t + u;
                    ps.cnt = run;
                    break;
                }
            }
        }
    }
    __syncthreads();
    const int bstar = ps.bstar, cnt = ps.cnt;
    for (int k = t; k < n; k += blockDim.x) {
        double v;
        uint32_t id;
        get(k, v, id);
        if (bin_of(v) <= bstar) {
            const int pos = atomicAdd(&ps.fill, 1);
            key[pos] = v;
            idx[pos] = id;
        }
    }
    const int n2 = pow2_at_least(cnt < 2 ? 2 : cnt);
    for (int k = cnt + t; k < n2; k += blockDim.x) {
        key[k] = INFINITY;
        idx[k] = 0xFFFFFFFFu;
    }
    bitonic_sort(key, idx, n2, PlainLess());
    return cnt;
}

constexpr int NPILOT = 4;                    // pilots of a ranking step
constexpr int PRANK = 512;                   // singles per pilot of a ranking step
constexpr int NPIL = 32;                     // pilots of a full step
constexpr int PKW = 10;                      // sites per pilot of a full step (at least)
constexpr int PIL_BLOCKS = 10;               // 64-site blocks of a pilot's fields loaded in one round
constexpr int PCW = PKW * (PKW + 1) / 2;     // candidates per pilot of a full step
constexpr int POOL = NPILOT * PRANK;         // candidate pool, a power of 2
static_assert(NPIL * PCW <= POOL, "the candidate pool holds either kind of step");
static_assert(POOL >= 1024 && POOL >= 4 * 64, "key/idx hold the fresh states (M <= 1024) and the pilots' sites");
static_assert(NPIL <= 32, "the pilot index takes the top 6 bits of a candidate id");

// Sites where the states at xa and xb differ, up to 4 of them into d;
// returns their number, or 5 when there are more.
__device__ inline int pilot_diff(const uint64_t* xa, const uint64_t* xb, int W, int* d)
{
    // the words in chunks of eight, each chunk's loads issued together
    int n = 0;
    for (int w0 = 0; w0 < W && n <= 4; w0 += 8) {
        uint64_t x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = w0 + u < W ? xa[w0 + u] ^ xb[w0 + u] : 0ull;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            uint64_t v = x[u];
            while (v && n <= 4) {
                if (n < 4) d[n] = (w0 + u) * 64 + __builtin_ctzll(v);
                ++n;
                v &= v - 1;
            }
        }
    }
    return n;
}

// Bitonic sort of one (value, index) per lane across the wave, ascending by
// (value, index).
__device__ inline void wave_sort64(double& best, int& bi, int lane)
{
    for (int k = 2; k <= 64; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            const double ob = __shfl_xor(best, j, 64);
            const int oi = __shfl_xor(bi, j, 64);
            const bool other_less = ob < best || (ob == best && oi < bi);
            // in an ascending run the lower lane of a pair keeps the smaller
            const bool keep_small = ((lane & k) == 0) == ((lane & j) == 0);
            if (other_less == keep_small) {
                best = ob;
                bi = oi;
            }
        }
}

__device__ inline void cand_sites(uint32_t id, int* out, int& n)
{
    // id = pilot << 26 | single << 25 | i << 12 | j
    n = 0;
    out[n++] = (int)((id >> 12) & 0xFFFu);
    if (!((id >> 25) & 1u)) out[n++] = (int)(id & 0xFFFu);
}

__global__ __launch_bounds__(256) void k_frontier(Layout lay, const double* __restrict__ J4, int kn)
{
    if (step_halted(lay)) return;   // a later step of a multi-step graph after a halt
    // key/idx: kn >= max(POOL, pow2(Npmax)) entries, in dynamic LDS, so that
    // three blocks share a CU for N up to 2048
    extern __shared__ __align__(16) unsigned char fr_dyn[];
    double* const key = reinterpret_cast<double*>(fr_dyn);
    uint32_t* const idx = reinterpret_cast<uint32_t*>(fr_dyn + sizeof(double) * kn);
    __shared__ double pE[POOL];
    __shared__ uint32_t pid[POOL];
    __shared__ int tmp[256];
    __shared__ int pslot[NPIL];
    __shared__ PrefixShared ps;
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
    // learned-proposal form: a ranking step expands the new states with ranked
    // pairs; a full step (after a ranking step found nothing) enumerates every
    // kept state whose pairs were not all evaluated yet
    const bool learned = lay.form == 2;
    const int mode = learned ? lay.mode[s] : 1;
    const bool ranked = learned && mode == 0;

    // rank the states to expand in kept (energy) order
    int nfresh = 0;
    for (int c0 = 0; c0 < nk; c0 += 256) {
        const int k = c0 + threadIdx.x;
        const int slot = k < nk ? kept[k] : 0;
        int isnew = 0;
        if (k < nk) isnew = (learned && !ranked) ? !lay.xfull[q0 + slot] : lay.fresh[q0 + slot];
        int excl;
        const int tot = block_exclusive_scan(isnew, tmp, excl);
        if (isnew) idx[nfresh + excl] = (uint32_t)slot;   // lowest energy first
        nfresh += tot;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (learned) {
            lay.last_mode[s] = mode;
            if (!ranked && nfresh > 0) atomicAdd(&lay.ctr[CTR_FALLBACK], 1ull);
        }
        if (nfresh > 0) tmp[0] = atomicAdd(ranked ? &lay.lr_count[b] : &lay.fr_count[b], nfresh);
    }
    if ((int)threadIdx.x < NPIL) pslot[threadIdx.x] = (int)threadIdx.x < nfresh ? (int)idx[threadIdx.x] : -1;
    __syncthreads();
    if (nfresh > 0) {
        const int fr_base = tmp[0];
        for (int r = threadIdx.x; r < nfresh; r += blockDim.x) {
            const size_t pos = ranked ? (size_t)(lay.fmax - 1 - (fr_base + r)) : (size_t)(fr_base + r);
            lay.fr_list[(size_t)b * lay.fmax + pos] = (int)(s * 2 * M + idx[r]);
            if (learned && !ranked) lay.xfull[q0 + idx[r]] = 1;
        }
    }
    const double ecut = nk == M ? lay.E[q0 + kept[M - 1]] : INFINITY;
    __syncthreads();
    if (nfresh == 0) {
        if (threadIdx.x == 0) lay.cut[s] = ecut;
        return;
    }
    const int N = lay.N[b], Np = lay.Npad[b];
    const int W = words_of(N);
    // a ranking step offers every single flip but only ranked pairs, so its
    // pilots contribute their lightest single flips only; so do the pilots
    // of the single-flip neighbourhood.  Pilots of the exchange neighbourhood
    // offer pairs of one up and one down spin among their lightest sites.
    const bool single_pilots = ranked || lay.h1 == H1_SINGLES;
    const bool xch = lay.h1 == H1_EXCHANGE;
    const int npil = single_pilots ? NPILOT : NPIL;
    const int np = nfresh < npil ? nfresh : npil;
    // few pilots take more sites each, up to twice M candidates as the pool allows
    int KW = PKW;
    while (KW < 64 && np * (KW * (KW + 1) / 2) < 2 * M && np * ((KW + 1) * (KW + 2) / 2) <= POOL) ++KW;
    if (KW > N) KW = N;
    int KX = 8;   // exchange: up and down sites per pilot
    while (KX < 64 && np * KX * KX < 2 * M && np * (KX + 1) * (KX + 1) <= POOL) ++KX;
    const int nc = single_pilots ? (N < PRANK ? N : PRANK) : (xch ? KX * KX : KW * (KW + 1) / 2);
    if (nc * np < M) {   // too few candidates to bound anything
        if (threadIdx.x == 0) lay.cut[s] = ecut;
        return;
    }
    if (single_pilots) {
        for (int p = 0; p < np; ++p) {
            const uint64_t* xp = lay.bits + (q0 + pslot[p]) * lay.Wmax;
            const FieldRow Fp = field_row(lay, q0 + pslot[p], b);
            const double Ep = lay.E[q0 + pslot[p]];
            // the lightest sites (lowest a_i, then lowest i) in key/idx[0 ..)
            sort_prefix([&](int i, double& v, uint32_t& id) {
                v = -2.0 * spin_of(xp, i) * Fp[i];
                id = (uint32_t)i;
            }, N, nc, key, idx, ps);
            for (int t = threadIdx.x; t < nc; t += blockDim.x) {
                pE[p * nc + t] = Ep + key[t];
                pid[p * nc + t] = ((uint32_t)p << 26) | (1u << 25) | (idx[t] << 12);
            }
            __syncthreads();
        }
    } else if (xch) {
        const double* Jb = J4 + lay.joff[b];
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        // the up and the down sites of each wave's pilot, in key/idx
        double* const aW = key + 128 * wave;
        uint32_t* const iW = idx + 128 * wave;
        if (threadIdx.x == 0) tmp[1] = 0;
        __syncthreads();
        for (int p = wave; p < np; p += 4) {
            const uint64_t* xp = lay.bits + (q0 + pslot[p]) * lay.Wmax;
            const FieldRow Fp = field_row(lay, q0 + pslot[p], b);
            const double Ep = lay.E[q0 + pslot[p]];
            // the lane's lightest up site and lightest down site (first of equals)
            const uint64_t xw = lane < W ? xp[lane] : 0ull;
            double bu = INFINITY, bd = INFINITY;
            int iu = 0x7FFFFFFF, id = 0x7FFFFFFF;
            for (int i0 = 0; i0 < N; i0 += 64 * PIL_BLOCKS) {
                double f[PIL_BLOCKS];
                Fp.gather(f, [&](int r) { return min(i0 + 64 * r, Np - 64) + lane; });
#pragma unroll
                for (int r = 0; r < PIL_BLOCKS; ++r) {
                    const int ib = i0 + 64 * r, i = ib + lane;
                    if (ib < N) {
                        const bool neg = __builtin_amdgcn_inverse_ballot_w64(word_of_lane(xw, ib >> 6));
                        const double a = -2.0 * (neg ? -1.0 : 1.0) * f[r];
                        if (i < N && neg && a < bd) {
                            bd = a;
                            id = i;
                        }
                        if (i < N && !neg && a < bu) {
                            bu = a;
                            iu = i;
                        }
                    }
                }
            }
            wave_sort64(bu, iu, lane);
            wave_sort64(bd, id, lane);
            const int cu = __builtin_popcountll(__builtin_amdgcn_ballot_w64(bu < INFINITY));
            const int cd = __builtin_popcountll(__builtin_amdgcn_ballot_w64(bd < INFINITY));
            if (cu < KX || cd < KX) {
                if (lane == 0) atomicOr(&tmp[1], 1);   // too few sites of one spin: no pilot cut
            }
            if (lane < KX) {
                aW[lane] = bu;
                iW[lane] = (uint32_t)iu;
                aW[64 + lane] = bd;
                iW[64 + lane] = (uint32_t)id;
            }
            wave_sync();
            if (cu >= KX && cd >= KX) {
                for (int t = lane; t < nc; t += 64) {
                    const int a = t / KX, c = t % KX;
                    int i = (int)iW[a], j = (int)iW[64 + c];
                    if (i > j) { const int x = i; i = j; j = x; }
                    // one up and one down spin: s_i s_j = -1
                    const double v = aW[a] + aW[64 + c] - Jb[(size_t)i * Np + j];
                    pE[p * nc + t] = Ep + v;
                    pid[p * nc + t] = ((uint32_t)p << 26) | ((uint32_t)i << 12) | (uint32_t)j;
                }
            }
            wave_sync();   // aW is rewritten for the wave's next pilot
        }
        __syncthreads();
        if (tmp[1]) {
            if (threadIdx.x == 0) lay.cut[s] = ecut;
            return;
        }
    } else {
        const double* Jb = J4 + lay.joff[b];
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        // the sites of each wave's pilot, in key/idx (free until the pool is sorted)
        double* const aW = key + 64 * wave;
        uint32_t* const iW = idx + 64 * wave;
        for (int p = wave; p < np; p += 4) {
            const uint64_t* xp = lay.bits + (q0 + pslot[p]) * lay.Wmax;
            const FieldRow Fp = field_row(lay, q0 + pslot[p], b);
            const double Ep = lay.E[q0 + pslot[p]];
            // the lane's lightest site (the first of equals): rounds of PIL_BLOCKS blocks
            // of 64 sites whose loads are issued together (blocks past Np load
            // the last block again, unused); the word of block k, held by lane
            // k, is the lane mask of the flipped spins
            const uint64_t xw = lane < W ? xp[lane] : 0ull;
            double best = INFINITY;
            int bi = 0x7FFFFFFF;
            for (int i0 = 0; i0 < N; i0 += 64 * PIL_BLOCKS) {
                double f[PIL_BLOCKS];
                Fp.gather(f, [&](int r) { return min(i0 + 64 * r, Np - 64) + lane; });
#pragma unroll
                for (int r = 0; r < PIL_BLOCKS; ++r) {
                    const int ib = i0 + 64 * r, i = ib + lane;
                    if (ib < N) {
                        const bool neg = __builtin_amdgcn_inverse_ballot_w64(word_of_lane(xw, ib >> 6));
                        const double a = -2.0 * (neg ? -1.0 : 1.0) * f[r];
                        if (i < N && a < best) {
                            best = a;
                            bi = i;
                        }
                    }
                }
            }
            wave_sort64(best, bi, lane);
            if (lane < KW) {
                aW[lane] = best;
                iW[lane] = (uint32_t)bi;
            }
            wave_sync();
            for (int t = lane; t < nc; t += 64) {
                double v;
                uint32_t id;
                if (t < KW) {
                    v = aW[t];
                    id = (1u << 25) | (iW[t] << 12);
                } else {
                    int u = t - KW, a = 0;   // pairs (a, c), a < c < KW
                    while (u >= KW - 1 - a) { u -= KW - 1 - a; ++a; }
                    const int c = a + 1 + u;
                    int i = (int)iW[a], j = (int)iW[c];
                    if (i > j) { const int x = i; i = j; j = x; }
                    const double sij = spin_of(xp, i) * spin_of(xp, j);
                    v = aW[a] + aW[c] + sij * Jb[(size_t)i * Np + j];
                    id = ((uint32_t)i << 12) | (uint32_t)j;
                }
                pE[p * nc + t] = Ep + v;
                pid[p * nc + t] = ((uint32_t)p << 26) | id;
            }
            wave_sync();   // aW is rewritten for the wave's next pilot
        }
        __syncthreads();
    }
    // pool: sort a prefix by energy, drop duplicates, take the M-th distinct
    // (a prefix with fewer than M distinct states is widened; the pilots of a
    // search share many children, so the first prefix holds 3M + 64)
    const int npool = np * nc;
    double theta = INFINITY;
    int seen = 0;
    for (int need = 3 * M + 64 < npool ? 3 * M + 64 : npool;; need = 2 * need < npool ? 2 * need : npool) {
    const int cnt = sort_prefix([&](int k, double& v, uint32_t& id) {
        v = pE[k];
        id = pid[k];
    }, npool, need, key, idx, ps);
    theta = INFINITY;
    seen = 0;
    for (int c0 = 0; c0 < cnt && seen < M; c0 += 256) {
        const int t = c0 + threadIdx.x;
        int isnew = 0;
        if (t < cnt) {
            isnew = 1;
            const uint32_t id = idx[t];
            int fa[2], na;
            cand_sites(id, fa, na);
            const int pa = (int)(id >> 26);
            for (int u = t - 1; u >= 0 && key[u] == key[t] && isnew; --u) {
                const uint32_t ib = idx[u];
                const int pb = (int)(ib >> 26);
                if (pb == pa) continue;   // children of one parent are distinct
                int dsite[4];
                const int nd = pilot_diff(lay.bits + (q0 + pslot[pa]) * lay.Wmax,
                                          lay.bits + (q0 + pslot[pb]) * lay.Wmax, W, dsite);
                if (nd > 4) continue;
                int fb[2], nb2;
                cand_sites(ib, fb, nb2);
                // symmetric difference of the two flip sets must equal the differing sites
                int sd[4], ns = 0;
                for (int e = 0; e < na; ++e) {
                    bool in = false;
                    for (int g = 0; g < nb2; ++g) in |= fa[e] == fb[g];
                    if (!in) sd[ns++] = fa[e];
                }
                for (int g = 0; g < nb2; ++g) {
                    bool in = false;
                    for (int e = 0; e < na; ++e) in |= fb[g] == fa[e];
                    if (!in) sd[ns++] = fb[g];
                }
                if (ns != nd) continue;
                bool same = true;
                for (int e = 0; e < ns && same; ++e) {
                    bool in = false;
                    for (int g = 0; g < nd; ++g) in |= sd[e] == dsite[g];
                    same = in;
                }
                if (same) isnew = 0;
            }
        }
        int excl;
        const int tot = block_exclusive_scan(isnew, tmp, excl);
        if (isnew && seen + excl == M - 1) tmp[0] = t;   // read after the barrier below
        __syncthreads();
        if (seen < M && seen + tot >= M) theta = key[tmp[0]];
        __syncthreads();
        seen += tot;
    }
    if (seen >= M || cnt == npool) break;
    }
    if (threadIdx.x == 0) lay.cut[s] = theta < ecut ? theta : ecut;
}

// ------------------------------------------------------------------ k_plan
// One block.  Work prefix sums over instances: scan items (chunks x tiles)
// and frontier entries; also the evaluation counters.
// Prepared entries are the fully enumerated ones followed by the ranked ones
// (learned form); ranked entries also get a prefix of their own.
__device__ inline long long proposals_of(const Layout& lay, long long N)
{
    const long long P = N * (N - 1) / 2, K = (long long)lay.topk * N;
    return K < P ? K : P;
}

__global__ __launch_bounds__(1024) void k_plan(Layout lay, long long* __restrict__ fr_prefix, int count)
{
    if (step_halted(lay)) return;   // a later step of a multi-step graph after a halt
    __shared__ long long part_items[1024];
    __shared__ long long part_fr[1024];
    __shared__ long long part_lr[1024];
    long long* lr_prefix = lay.item_prefix + 3 * (lay.B + 1);
    const int t = threadIdx.x;
    const int per = (lay.B + 1023) / 1024;
    const int b0 = t * per;
    // single flips only: no pair is scanned
    const bool scanned = lay.h1 != H1_SINGLES;
    __shared__ int sc_all;
    if (lay.sc_auto) {
        // states per scan item, chosen each step: the largest power of two up
        // to 256 that still gives every scan wave 16 items of this step's
        // tiles x states, so that each item loads its couplings for as many
        // states as the balance of the grid allows
        __shared__ long long wsum[1024];
        long long w = 0;
        for (int b = b0; b < b0 + per && b < lay.B; ++b)
            w += scanned ? (long long)lay.fr_count[b] * scan_tiles(lay, lay.N[b]) : 0;
        wsum[t] = w;
        __syncthreads();
        for (int off = 512; off > 0; off >>= 1) {
            if (t < off) wsum[t] += wsum[t + off];
            __syncthreads();
        }
        if (t == 0) {
            const long long target = 16ll * lay.scan_waves;
            int sc = 256;
            while (sc > 16 && wsum[0] / sc < target) sc >>= 1;
            sc_all = sc;
        }
        __syncthreads();
        for (int b = b0; b < b0 + per && b < lay.B; ++b) lay.scb[b] = sc_all;
    }
    long long items = 0, fr = 0, lr = 0, pairs = 0, singles = 0, scored = 0;
    for (int b = b0; b < b0 + per && b < lay.B; ++b) {
        const long long P = lay.fr_count[b];
        const long long Q = lay.lr_count[b];
        const long long N = lay.N[b];
        const int sc = lay.sc_auto ? sc_all : lay.scb[b];
        items += scanned ? (P + sc - 1) / sc * tiles_of((int)N) : 0;
        fr += P + Q;
        lr += Q;
        // with the site bound the pairs are counted once the entries are sorted out
        pairs += (lay.sb || !scanned ? 0 : P * (N * (N - 1) / 2)) + Q * proposals_of(lay, N);
        scored += Q * (N * (N - 1) / 2);
        singles += (P + Q) * N;
    }
    part_items[t] = items;
    part_fr[t] = fr;
    part_lr[t] = lr;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const long long ai = t >= off ? part_items[t - off] : 0;
        const long long af = t >= off ? part_fr[t - off] : 0;
        const long long al = t >= off ? part_lr[t - off] : 0;
        __syncthreads();
        part_items[t] += ai;
        part_fr[t] += af;
        part_lr[t] += al;
        __syncthreads();
    }
    long long run_i = part_items[t] - items, run_f = part_fr[t] - fr, run_l = part_lr[t] - lr;
    for (int b = b0; b < b0 + per && b < lay.B; ++b) {
        lay.item_prefix[b] = run_i;
        fr_prefix[b] = run_f;
        lr_prefix[b] = run_l;
        const long long P = lay.fr_count[b];
        const long long Q = lay.lr_count[b];
        const int sc = lay.sc_auto ? sc_all : lay.scb[b];
        run_i += scanned ? (P + sc - 1) / sc * tiles_of(lay.N[b]) : 0;
        run_f += P + Q;
        run_l += Q;
    }
    if (t == 1023) {
        lay.item_prefix[lay.B] = part_items[1023];
        fr_prefix[lay.B] = part_fr[1023];
        lr_prefix[lay.B] = part_lr[1023];
    }
    // counters (the retry pass counts in k_prep instead)
    __shared__ unsigned long long cp[1024], cs[1024], cq[1024];
    cp[t] = (unsigned long long)pairs;
    cs[t] = (unsigned long long)singles;
    cq[t] = (unsigned long long)scored;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (t < w) { cp[t] += cp[t + w]; cs[t] += cs[t + w]; cq[t] += cq[t + w]; }
        __syncthreads();
    }
    if (t == 0 && count && !lay.flags[FLAG_RETRY_MODE]) {
        lay.ctr[CTR_PAIRS] += cp[0];
        lay.ctr[CTR_SINGLES] += cs[0];
        lay.ctr[CTR_SCORED] += cq[0];
        lay.ctr[CTR_LEARNED] += (unsigned long long)part_lr[1023];
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

// ------------------------------------------------------------------ k_site_bound
// Site bound, before the form's preparation: one wave per frontier entry
// evaluates the state's single flips and the pairs among its bounded sites
// (site_bound_pairs) and records in fr_bound how it went (1 + r, or 0 when
// the state has too many such sites and goes to the full scan).  The work
// is a chain of dependent memory rounds per state, so the kernel is kept lean
// enough for eight waves per SIMD: that many states are in flight per CU.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_site_bound(
    Layout lay, const long long* __restrict__ fr_prefix)
{
    if (step_halted(lay)) return;   // a later step of a multi-step graph after a halt
    __shared__ uint16_t sb_idx[4][SB_CAP];
    __shared__ double sb_a[4][SB_CAP];
    __shared__ Surv sb_stage[4][SB_STG];
    const long long total = fr_prefix[lay.B];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63;
    const int retry_mode = lay.flags[FLAG_RETRY_MODE];
    // XCD x (blocks x, x + 8, ...) takes the x-th contiguous eighth of the
    // entries, so the states it bounds at once share one L2 for their couplings
    const int nx = gridDim.x >= 8 ? 8 : 1;
    const int xcd = blockIdx.x % nx;
    const long long seg1 = total * (xcd + 1) / nx;
    const long long stride = (long long)(gridDim.x / nx) * 4;
    int b = -1;   // instance of entry e: found once, then advanced (e only grows)
    for (long long e = total * xcd / nx + (long long)(blockIdx.x / nx) * 4 + wave; e < seg1; e += stride) {
        if (b < 0) b = find_instance(fr_prefix, lay.B, e);
        while (fr_prefix[b + 1] <= e) ++b;
        const size_t fe = (size_t)b * lay.fmax + (size_t)(e - fr_prefix[b]);
        const int code = lay.fr_list[fe];
        const int s = code / (2 * lay.M);
        if (retry_mode && !lay.retry[s]) continue;
        const size_t q = (size_t)code;
        const int r = site_bound_pairs(lay, b, s, code, lay.E[q], lay.cut[s], lay.bits + q * lay.Wmax,
                                       field_row(lay, q, b), lay.N[b], lay.Npad[b], sb_idx[wave], sb_a[wave],
                                       sb_stage[wave]);
        if (lane == 0) {
            lay.fr_bound[fe] = (uint16_t)(r + 1);
            // a retry pass counts its single flips here (the pairs in k_sb_list)
            if (retry_mode && r >= 0) atomicAdd(&lay.ctr[CTR_SINGLES], (unsigned long long)lay.N[b]);
        }
    }
}

// ------------------------------------------------------------------ k_prep
// One wave per frontier entry: a_i = -2 s_i F_i, the per-state record the
// scan reads (threshold T = cut - E, energy, search, slot), a copy of the
// state's words next to it, and the single flips below the cut.
template <bool SB>
__global__ __launch_bounds__(256) void k_prep(Layout lay, const long long* __restrict__ fr_prefix)
{
    if (step_halted(lay)) return;   // a later step of a multi-step graph after a halt
    const long long total = fr_prefix[lay.B];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63;
    const int retry_mode = lay.flags[FLAG_RETRY_MODE];
    const bool singles = lay.h1 != H1_EXCHANGE;
    // XCD x (blocks x, x + 8, ...) takes the x-th contiguous eighth of the
    // entries, so the states it prepares at once share one L2 for their
    // couplings
    const int nx = gridDim.x >= 8 ? 8 : 1;
    const int xcd = blockIdx.x % nx;
    const long long seg1 = total * (xcd + 1) / nx;
    const long long stride = (long long)(gridDim.x / nx) * 4;
    int b = -1;   // instance of entry e: found once, then advanced (e only grows)
    for (long long e = total * xcd / nx + (long long)(blockIdx.x / nx) * 4 + wave; e < seg1; e += stride) {
        if (b < 0) b = find_instance(fr_prefix, lay.B, e);
        while (fr_prefix[b + 1] <= e) ++b;
        const int f = (int)(e - fr_prefix[b]);
        const int P = lay.fr_count[b];
        const bool ranked = f >= P;   // learned form: a ranked entry, listed from the back
        const size_t fe = (size_t)b * lay.fmax + (ranked ? lay.fmax - lay.lr_count[b] + (f - P) : f);
        // site bound: the states k_site_bound evaluated need nothing here
        if (SB && lay.fr_bound[fe] != 0) continue;
        const int code = lay.fr_list[fe];
        const int s = code / (2 * lay.M);
        if (retry_mode && !lay.retry[s]) continue;
        const size_t q = (size_t)code;   // s*2M + slot
        const int N = lay.N[b], Np = lay.Npad[b];
        const double Em = lay.E[q];
        const double c = lay.cut[s];
        const uint64_t* x = lay.bits + q * lay.Wmax;
        const FieldRow F = field_row(lay, q, b);
        double* A = lay.A + fe * lay.Npmax;
        if (lane == 0) {
            FrRec r;
            r.T = c - Em;
            r.E = Em;
            r.s = s;
            r.code = code;
            lay.rec[fe] = r;
        }
        // lane w holds word w of the state (at most 64 words)
        const uint64_t xw = (int)lane < lay.Wmax ? x[lane] : 0ull;
        if ((int)lane < lay.Wmax) lay.fbits[fe * lay.Wmax + lane] = xw;
        if (retry_mode && lane == 0) {
            const unsigned long long all = (unsigned long long)N * (N - 1) / 2;
            // with the site bound the pairs are counted once the entries are sorted out
            if (!lay.sb) atomicAdd(&lay.ctr[CTR_PAIRS], ranked ? (unsigned long long)proposals_of(lay, N) : all);
            atomicAdd(&lay.ctr[CTR_SINGLES], (unsigned long long)N);
            if (ranked) atomicAdd(&lay.ctr[CTR_SCORED], all);
        }
        // a_i, and the single flips below the cut, in rounds of PREP_BLOCKS
        // blocks of 64 sites: the loads of a round are issued together (blocks
        // past Np load the last block again, unused, so that every load is
        // unconditional and in bounds); the round's hits are counted, so that one
        // atomic reserves their places, then recorded
        for (int i0 = 0; i0 < Np; i0 += 64 * PREP_BLOCKS) {
            double Fv[PREP_BLOCKS];
            F.gather(Fv, [&](int r) { return min(i0 + 64 * r, Np - 64) + (int)lane; });
            double ar[PREP_BLOCKS];
            int nhit = 0;
#pragma unroll
            for (int r = 0; r < PREP_BLOCKS; ++r) {
                const int ib = i0 + 64 * r;
                ar[r] = 0.0;
                if (ib < Np) {
                    const int i = ib + (int)lane;
                    // the word of sites ib .. ib+63 is the lane mask of the flipped spins
                    const bool neg = __builtin_amdgcn_inverse_ballot_w64(word_of_lane(xw, ib >> 6));
                    const double a = i < N ? -2.0 * (neg ? -1.0 : 1.0) * Fv[r] : 0.0;
                    ar[r] = a;
                    A[i] = a;
                    // a ranked state's singles go with its pairs; the exchange
                    // neighbourhood has no single flips
                    nhit += __builtin_popcountll(
                        __builtin_amdgcn_ballot_w64(singles && !ranked && i < N && Em + a <= c));
                }
            }
            if (nhit) {
                int base = 0;
                if (lane == 0) base = atomicAdd(&lay.surv_count[s], nhit);
                base = __shfl(base, 0, 64);
#pragma unroll
                for (int r = 0; r < PREP_BLOCKS; ++r) {
                    const int i = i0 + 64 * r + (int)lane;
                    const double Ec = Em + ar[r];
                    const bool hit = singles && i < N && Ec <= c;
                    const uint64_t m = __builtin_amdgcn_ballot_w64(hit);
                    if (m) {
                        if (hit) {
                            const int pos = base + (int)mbcnt64(m);
                            if (pos < lay.cap_surv) {
                                Surv rec;
                                rec.E = Ec;
                                rec.code = (uint32_t)code;
                                rec.pair = (uint32_t)i | (SINGLE << 16);
                                lay.surv[(size_t)s * lay.cap_surv + pos] = rec;
                            }
                        }
                        base += __builtin_popcountll(m);
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------------------ k_scan
// One wave per work item (instance b, chunk of sc frontier states, tile of
// 64 rows i x 32 columns j).  Lane = row i; the wave keeps y_j = s_j 4J_ij for
// its row and the tile's 32 columns in registers and walks the chunk's states,
// so one tile load serves sc states.  For state m the pair (i,j) survives iff
//   x = fma(s_i, y_j, a_j) = a_j + s_i s_j 4J_ij <= T_m - a_i
// (exact: the product by +-1 is exact and the fma rounds once, like an add).
// Only column signs live in the registers; they change between consecutive
// states of a chunk only at the few sites where the states differ, so a group
// of 8 columns is re-signed only when one of its columns changed.  The hot
// loop is one v_fma_f64 and one v_min_f64 per pair and one compare per group;
// a group whose minimum passes runs the exact pass that records survivors.
// Pairs outside the triangle or the instance hold NaN, which fmin ignores and
// no compare passes.  a_j is wave-uniform and read from a per-wave LDS row
// that the next state's row replaces once the current one's reads are issued
// (one wave's LDS accesses complete in order); the next state's record, words and a_i are
// loaded while the current state is scanned.  Survivors are staged in LDS and
// appended to the search's buffer with one atomic per flush.
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

// XCH: the exchange neighbourhood; a pair counts only when its two spins differ
// (the running minimum still covers every pair of the group, so it only
// admits groups; the exact pass applies the condition).
template <bool XCH>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_scan(Layout lay, const double* __restrict__ J4,
                                             const double* __restrict__ Abuf,
                                             const FrRec* __restrict__ recs,
                                             const uint64_t* __restrict__ fbits)
{
    if (step_halted(lay)) return;   // a later step of a multi-step graph after a halt
    __shared__ Surv stage[STAGE];
    __shared__ double abuf[TCOL];   // a_j of the current state
    // per-state data of up to 64 states of the chunk, staged once per item
    // per state, what the loop over states reads: one address for all of it
    struct StRec {
        double T, E;       // threshold and energy
        uint64_t wi;       // word of the tile's rows
        uint32_t wj;       // the tile's 32 columns of their word
        int s, code;       // search, pool slot of the state
        uint32_t fe;       // entry index: below 2^32, as the FP64 rows of every entry fit in memory
    };
    __shared__ StRec srec[64];
    const uint32_t lane = lane_id();
    const long long total = lay.item_prefix[lay.B];
    const int retry_mode = lay.flags[FLAG_RETRY_MODE];
    const int Wm = lay.Wmax;
    const int Npm = lay.Npmax;
    // Workgroups are dispatched round-robin over the 8 XCDs, so block k runs on
    // XCD k % 8.  XCD x takes the x-th contiguous eighth of the item list: the
    // tiles of one chunk of states (and most chunks of one instance) then share
    // one XCD's L2 for their a_i values and J tiles.
    const int nx = gridDim.x >= 8 ? 8 : 1;
    const int xcd = blockIdx.x % nx;
    const long long seg0 = total * xcd / nx, seg1 = total * (xcd + 1) / nx;
    const long long stride = gridDim.x / nx;
    for (long long item = seg0 + blockIdx.x / nx; item < seg1; item += stride) {
        const int b = uniform_int(find_instance(lay.item_prefix, lay.B, item));
        const long long r = item - lay.item_prefix[b];
        const int N = lay.N[b], Np = lay.Npad[b];
        const int nc = (N + TCOL - 1) / TCOL;   // column blocks holding a column below N
        const long long T = tiles_of(N);
        const int c = (int)(r / T);
        int t = (int)(r % T);
        int bi = 0;
        while (t >= nc - 2 * bi) { t -= nc - 2 * bi; ++bi; }
        bi = uniform_int(bi);
        const int bc = uniform_int(2 * bi + t);
        const int P = lay.sb ? lay.full_count[b] : lay.fr_count[b];
        const int sc = lay.scb[b];
        const int f0 = c * sc;
        const int f1 = min(f0 + sc, P);
        const size_t fb = (size_t)b * lay.fmax;

        // the tile: row i = bi*64 + lane, columns j = bc*32 + 0..31, unsigned
        const int row = bi * TILE + (int)lane;
        const int col0 = bc * TCOL;
        const double* Jt = J4 + lay.joff[b];
        uint64_t Jb[TCOL];
#pragma unroll
        for (int j = 0; j < TCOL; ++j) {
            const int col = col0 + j;
            const double v = Jt[(size_t)col * Np + row];   // symmetric: (col,row) = (row,col)
            const bool ok = row < N && col < N && col > row;
            Jb[j] = ok ? (uint64_t)__double_as_longlong(v) : 0x7ff8000000000000ull;
        }
        const int wrow = bi, wcol = bc >> 1, shcol = 32 * (bc & 1);
        uint32_t prev_wj = 0;   // column signs currently applied to Jb
        int nstage = 0, sstage = -1;
        for (int g0 = f0; g0 < f1; g0 += 64) {
            const int ns = min(64, f1 - g0);
            // stage the records of states g0 .. g0+ns-1 (with the site bound, the
            // entries left to the scan)
            if ((int)lane < ns) {
                const size_t fe = fb + (lay.sb ? lay.full_list[fb + g0 + lane] : g0 + (int)lane);
                const FrRec rc = recs[fe];
                const uint64_t* fw = fbits + fe * Wm;
                StRec sr;
                sr.T = rc.T;
                sr.E = rc.E;
                sr.wi = fw[wrow];
                sr.wj = (uint32_t)(fw[wcol] >> shcol);
                sr.s = rc.s;
                sr.code = rc.code;
                sr.fe = (uint32_t)fe;
                srec[lane] = sr;
            }
            __syncthreads();
            const double* A0 = Abuf + (size_t)(uint32_t)uniform_int((int)srec[0].fe) * Npm;   // a values of state g0
            double nai = A0[row];
            double naj = lane < TCOL ? A0[col0 + lane] : 0.0;
            if (lane < TCOL) abuf[lane] = naj;
            __syncthreads();
            for (int k = 0; k < ns; ++k) {
                const double ai = nai;
                if (k + 1 < ns) {
                    const double* An = Abuf + (size_t)(uint32_t)uniform_int((int)srec[k + 1].fe) * Npm;
                    nai = An[row];
                    if (lane < TCOL) naj = An[col0 + lane];
                }
                const StRec cur = srec[k];
                const int s = uniform_int(cur.s);
                const bool skip = retry_mode && !lay.retry[s];
                if (!skip) {
                    if (s != sstage) {
                        flush_stage(lay, stage, nstage, sstage);
                        sstage = s;
                    }
                    const double Tm = cur.T;
                    const double Ea = cur.E + ai;
                    const double rr = row < N ? Tm - ai : -INFINITY;
                    // the row bits of the state are the lane mask of the negative s_i
                    const double si = __builtin_amdgcn_inverse_ballot_w64(
                        ((uint64_t)(uint32_t)uniform_int((int)(cur.wi >> 32)) << 32) |
                        (uint32_t)uniform_int((int)(uint32_t)cur.wi)) ? -1.0 : 1.0;
                    const uint32_t wj = (uint32_t)uniform_int((int)cur.wj);
                    const uint32_t dw = wj ^ prev_wj;
                    prev_wj = wj;
                    const int code = cur.code;
                    const double* aj = abuf;
#pragma unroll
                    for (int g = 0; g < TCOL; g += 8) {
                        if ((dw >> g) & 0xFFu) {
                            // a column of this group changed sign since the last state
#pragma unroll
                            for (int u = 0; u < 8; ++u) {
                                const uint64_t flip = (uint64_t)((dw >> (g + u)) & 1u) << 63;
                                Jb[g + u] ^= flip;
                            }
                        }
                        double a8[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u) a8[u] = aj[g + u];
                        // running minimum over the group (two chains); NaN pairs drop out of fmin
                        double mn0 = fma(si, __longlong_as_double((long long)Jb[g]), a8[0]);
                        double mn1 = fma(si, __longlong_as_double((long long)Jb[g + 1]), a8[1]);
#pragma unroll
                        for (int u = 2; u < 8; ++u) {
                            const double x = fma(si, __longlong_as_double((long long)Jb[g + u]), a8[u]);
                            if (u & 1) mn1 = fmin(mn1, x);
                            else mn0 = fmin(mn0, x);
                        }
                        if (__builtin_amdgcn_ballot_w64(fmin(mn0, mn1) <= rr)) {
                            // rare: recompute the group and record every survivor
#pragma unroll
                            for (int u = 0; u < 8; ++u) {
                                const double x = fma(si, __longlong_as_double((long long)Jb[g + u]), a8[u]);
                                bool pass = x <= rr;
                                if (XCH) pass = pass && ((si < 0.0) != (((wj >> (g + u)) & 1u) != 0));
                                const uint64_t m = __builtin_amdgcn_ballot_w64(pass);
                                if (m) {
                                    if (nstage > STAGE - 64) flush_stage(lay, stage, nstage, s);
                                    if ((m >> lane) & 1ull) {
                                        // opaque to the optimiser, so the 32 record codes are formed
                                        // here instead of being held in registers across the loop
                                        uint32_t rowv = (uint32_t)row;
                                        asm volatile("" : "+v"(rowv));
                                        Surv rec;
                                        rec.E = Ea + x;
                                        rec.code = (uint32_t)code;
                                        rec.pair = rowv | ((uint32_t)(col0 + g + u) << 16);
                                        stage[nstage + (int)mbcnt64(m)] = rec;
                                    }
                                    nstage += __builtin_popcountll(m);
                                }
                            }
                        }
                    }
                }
                // one wave: its LDS accesses complete in order, so the next row can
                // replace this one once its reads are issued
                if (k + 1 < ns && lane < TCOL) abuf[lane] = naj;
                __syncthreads();
            }
        }
        flush_stage(lay, stage, nstage, sstage);
        __syncthreads();
    }
}

// ------------------------------------------------------------------ merge helpers
// A candidate decoded once: the words of its parent state and up to two
// flipped sites (j = SINGLE for a single flip, i = j = SINGLE for a state
// taken as it is).  Comparisons of words then issue independent loads.
struct Cand {
    const uint64_t* base;
    int i, j;
    __device__ uint64_t flips(int w) const
    {
        uint64_t v = 0;
        if (i != (int)SINGLE && (i >> 6) == w) v ^= 1ull << (i & 63);
        if (j != (int)SINGLE && (j >> 6) == w) v ^= 1ull << (j & 63);
        return v;
    }
    __device__ uint64_t word(int w) const { return base[w] ^ flips(w); }
};

// Candidates of one search: kept states (ref < REF_SURV, index into the kept
// list) and survivor records (ref = REF_SURV | record index).
struct SearchSrc {
    const Layout* lay;
    int s, b;
    __device__ Cand decode(uint32_t ref) const
    {
        if (ref & REF_SURV) {
            const Surv r = lay->surv[(size_t)s * lay->cap_surv + (ref & ~REF_SURV)];
            return Cand{lay->bits + (size_t)r.code * lay->Wmax, (int)(r.pair & 0xFFFFu), (int)(r.pair >> 16)};
        }
        const int slot = lay->kept[(size_t)s * lay->M + ref];
        return Cand{lay->bits + ((size_t)s * 2 * lay->M + slot) * lay->Wmax, (int)SINGLE, (int)SINGLE};
    }
};

// Candidates of one instance: ref = l * M + k, the k-th kept state of search l.
struct InstanceSrc {
    const Layout* lay;
    int b;
    __device__ Cand decode(uint32_t ref) const
    {
        const int l = (int)(ref / (uint32_t)lay->M), k = (int)(ref % (uint32_t)lay->M);
        const int s = b * lay->L + l;
        const int slot = lay->kept[(size_t)s * lay->M + k];
        return Cand{lay->bits + ((size_t)s * 2 * lay->M + slot) * lay->Wmax, (int)SINGLE, (int)SINGLE};
    }
};

constexpr uint32_t REF_PAD = 0xFFFFFFFFu;

// Total order (E, psi, ref).  Two candidates with equal energy and equal
// Zobrist hash are taken to be the same state and ordered by ref (a kept
// state has a smaller ref than any survivor, so it comes first); the dedupe
// pass confirms this on the full words and, on a hash collision, the list is
// sorted again with strict = true, which always compares psi.
template <class Src>
struct StateLess {
    const Src* src;
    int W;
    bool strict;
    __device__ bool operator()(double a, uint32_t ia, uint64_t za, double b, uint32_t ib, uint64_t zb) const
    {
        if (a < b) return true;
        if (a > b) return false;
        if (ia == REF_PAD || ib == REF_PAD) return ia < ib;
        if (!strict && za == zb) return ia < ib;
        const Cand A = src->decode(ia), B = src->decode(ib);
        for (int w = W - 1; w >= 0; --w) {
            const uint64_t x = A.word(w), y = B.word(w);
            if (x != y) return x < y;
        }
        return ia < ib;
    }
};

template <class Less>
__device__ void bitonic_sort3(double* key, uint32_t* idx, uint64_t* zk, int n2, const Less& less)
{
    __syncthreads();
    for (int k = 2; k <= n2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= 128) __syncthreads();
            for (int t = threadIdx.x; t < (n2 >> 1); t += blockDim.x) {
                const int i = 2 * j * (t / j) + (t % j);
                const int l = i + j;
                const bool up = (i & k) == 0;
                const bool swap = up ? less(key[l], idx[l], zk[l], key[i], idx[i], zk[i])
                                     : less(key[i], idx[i], zk[i], key[l], idx[l], zk[l]);
                if (swap) {
                    const double tk = key[i]; key[i] = key[l]; key[l] = tk;
                    const uint32_t ti = idx[i]; idx[i] = idx[l]; idx[l] = ti;
                    const uint64_t tz = zk[i]; zk[i] = zk[l]; zk[l] = tz;
                }
            }
            if (j >= 128) __syncthreads();
            else wave_sync();
        }
    }
    __syncthreads();
}

template <class Src>
__device__ bool same_words(const Src& src, int W, uint32_t ia, uint32_t ib)
{
    const Cand A = src.decode(ia), B = src.decode(ib);
    if (A.base == B.base && A.i == B.i && A.j == B.j) return true;
    uint64_t diff = 0;
    int w = 0;
    for (; w + 4 <= W; w += 4) {
        // four words of each state in flight at once
        const uint64_t a0 = A.base[w], a1 = A.base[w + 1], a2 = A.base[w + 2], a3 = A.base[w + 3];
        const uint64_t b0 = B.base[w], b1 = B.base[w + 1], b2 = B.base[w + 2], b3 = B.base[w + 3];
        diff |= (a0 ^ b0 ^ A.flips(w) ^ B.flips(w)) | (a1 ^ b1 ^ A.flips(w + 1) ^ B.flips(w + 1)) |
                (a2 ^ b2 ^ A.flips(w + 2) ^ B.flips(w + 2)) | (a3 ^ b3 ^ A.flips(w + 3) ^ B.flips(w + 3));
    }
    for (; w < W; ++w) diff |= A.word(w) ^ B.word(w);
    return diff == 0;
}

// Sorts key/ref/zob[0..n), drops duplicates (the first of equal states is
// kept; a kept state sorts before its copies) and moves the first M distinct
// to the front.  Returns their count.
template <class Src>
__device__ int sort_dedupe_keep(const Src& src, int W, double* key, uint32_t* ref, uint64_t* zk, int n, int M,
                                int* tmp, uint8_t* keep)
{
    __shared__ int s_collide;
    const int n2 = pow2_at_least(n < 2 ? 2 : n);
    for (int t = n + threadIdx.x; t < n2; t += blockDim.x) {
        key[t] = INFINITY;
        ref[t] = REF_PAD;
        zk[t] = 0;
    }
    if (threadIdx.x == 0) s_collide = 0;
    __syncthreads();
    bitonic_sort3(key, ref, zk, n2, StateLess<Src>{&src, W, false});
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        int kf = 1;
        if (t > 0 && key[t - 1] == key[t] && zk[t - 1] == zk[t]) {
            if (same_words(src, W, ref[t - 1], ref[t])) kf = 0;
            else s_collide = 1;
        }
        keep[t] = (uint8_t)kf;
    }
    __syncthreads();
    if (s_collide) {
        // a 64-bit hash collision: order by the full words and compare them
        bitonic_sort3(key, ref, zk, n2, StateLess<Src>{&src, W, true});
        for (int t = threadIdx.x; t < n; t += blockDim.x)
            keep[t] = (t == 0 || key[t - 1] != key[t] || !same_words(src, W, ref[t - 1], ref[t])) ? 1 : 0;
        __syncthreads();
    }
    // compact the first M distinct, in order, in chunks of 256
    int out = 0;
    __shared__ double ck[256];
    __shared__ uint32_t cr[256];
    __shared__ uint64_t cz[256];
    for (int c0 = 0; c0 < n && out < M; c0 += 256) {
        const int t = c0 + threadIdx.x;
        const int kf = t < n ? keep[t] : 0;
        int excl;
        const int tot = block_exclusive_scan(kf, tmp, excl);
        double kv = 0.0;
        uint32_t rv = 0;
        uint64_t zv = 0;
        if (kf) { kv = key[t]; rv = ref[t]; zv = zk[t]; }
        __syncthreads();
        if (kf && out + excl < M) {
            ck[excl] = kv;
            cr[excl] = rv;
            cz[excl] = zv;
        }
        __syncthreads();
        const int take = min(tot, M - out);
        if ((int)threadIdx.x < take) {
            key[out + threadIdx.x] = ck[threadIdx.x];
            ref[out + threadIdx.x] = cr[threadIdx.x];
            zk[out + threadIdx.x] = cz[threadIdx.x];
        }
        __syncthreads();
        out += take;
    }
    return out;
}

// ------------------------------------------------------------------ k_merge
// One block per active search: the new kept set is the M lowest distinct
// states among the kept set and the survivors, in (E, psi) order.
// Pre-filter: a 1024-bin histogram of the candidate energies picks the lowest
// bins holding at least 2M + 64 candidates; bins are monotone in E, so this is
// a prefix of the sorted candidates, and if it holds M distinct states nothing
// above it can enter.  Otherwise (or when everything fits) all candidates are
// sorted, in passes of MERGE_CH that carry the running best M.
// A survivor buffer that overflowed only yields a tighter cut (its M-th
// distinct energy) for a re-scan.  Otherwise the new set is written: new states
// take slots the old set does not use (bits = parent xor flips, E from the
// record, hash updated); their local fields are written by k_fupdate.
constexpr int NBIN = 1024;

__device__ double block_reduce(double v, double* red, bool take_max)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double o = red[threadIdx.x + w];
            red[threadIdx.x] = take_max ? fmax(red[threadIdx.x], o) : fmin(red[threadIdx.x], o);
        }
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// The first histogram bin at which the running count (lowest bins first)
// reaches want, written to *out; wave 0 scans, 16 bins per lane.  The caller
// synchronises before reading *out.
__device__ void first_bin_reaching(const int* hist, int want, int* out)
{
    if (threadIdx.x < 64) {
        constexpr int PER = NBIN / 64;
        const int l = threadIdx.x;
        int loc = 0;
        for (int k = 0; k < PER; ++k) loc += hist[PER * l + k];
        int incl = loc;
        for (int off = 1; off < 64; off <<= 1) {
            const int v = __shfl_up(incl, off, 64);
            if (l >= off) incl += v;
        }
        int run = incl - loc;
        if (run < want && want <= incl) {
            for (int k = 0; k < PER; ++k) {
                run += hist[PER * l + k];
                if (run >= want) {
                    *out = PER * l + k;
                    break;
                }
            }
        }
    }
}

// Dedupe table of k_merge: 4096 slots of 64 bits, the high 52 bits of a mix
// of (E, Zobrist hash) above a 12-bit candidate index; the low 12 bits of the
// mix give the home slot.
constexpr int HASH_T = 4096;
constexpr int HASH_PER = 12;                  // candidates per thread: n <= 3072
constexpr uint64_t HASH_EMPTY = ~0ull;
static_assert(HASH_T == 2 * MERGE_CH, "the table spans the key and zk arrays");
static_assert(HASH_PER * 256 <= 3 * HASH_T / 4, "load factor at most 3/4");

__device__ inline uint64_t mix_state(uint64_t z, double e)
{
    // splitmix64 finalizer (Steele, Lea and Flood) of the hash xor the scaled energy bits
    uint64_t x = z ^ ((uint64_t)__double_as_longlong(e) * 0x9E3779B97F4A7C15ull);
    x ^= x >> 30;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 27;
    x *= 0x94D049BB133111EBull;
    x ^= x >> 31;
    return x;
}

static_assert(MERGE_CH == 2048, "the slot bookkeeping of k_merge lives in the upper halves of key and zk");

// At most 52 KB of LDS: three blocks share a CU, which the merge, bound by the
// latency of its gathers, needs.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_merge(Layout lay, const double* __restrict__ J4)
{
    if (step_halted(lay)) return;   // a later step of a multi-step graph after a halt
    __shared__ uint64_t kz[2 * MERGE_CH];   // key then zk; the dedupe table before them
    __shared__ uint32_t ref[MERGE_CH];
    __shared__ uint8_t keep[MERGE_CH];
    __shared__ int tmp[256];
    __shared__ double red[8];
    __shared__ int hist[NBIN];
    double* const key = reinterpret_cast<double*>(kz);
    uint64_t* const zk = kz + MERGE_CH;
    // once the new set is chosen only its first M <= 1024 rows of key and zk
    // are read; the slot bookkeeping takes the upper halves
    int* const freeslot = reinterpret_cast<int*>(kz + MERGE_CH / 2);             // [2M]
    int* const kslot = reinterpret_cast<int*>(kz + MERGE_CH + MERGE_CH / 2);     // [M]
    uint8_t* const used = reinterpret_cast<uint8_t*>(kz + MERGE_CH + MERGE_CH / 2 + MERGE_CH / 4);   // [2M]
    const int s = blockIdx.x;
    const int b = s / lay.L;
    const int M = lay.M;
    const int retry_mode = lay.flags[FLAG_RETRY_MODE];
    if (blockIdx.x == 0 && threadIdx.x == 0) lay.flags[FLAG_FIRST] = 0;   // the first step has been scanned
    if (!lay.active[s]) return;
    if (retry_mode && !lay.retry[s]) return;
    const int nk = lay.nkept[s];
    const int ctot = lay.surv_count[s];
    const int cnt = ctot < lay.cap_surv ? ctot : lay.cap_surv;
    const size_t q0 = (size_t)s * 2 * M;
    const int W = words_of(lay.N[b]);
    const Surv* sv = lay.surv + (size_t)s * lay.cap_surv;
    const int* keptl = lay.kept + (size_t)s * M;
    SearchSrc src{&lay, s, b};
    const int n = nk + cnt;
    auto candE = [&](int c) -> double { return c < nk ? lay.E[q0 + keptl[c]] : sv[c - nk].E; };
    auto ref_of = [&](int c) -> uint32_t { return c < nk ? (uint32_t)c : REF_SURV | (uint32_t)(c - nk); };
    // energy and Zobrist hash of candidate c (0..n)
    auto cand_key = [&](int c, double& e, uint64_t& z) {
        if (c < nk) {
            const int slot = keptl[c];
            e = lay.E[q0 + slot];
            z = lay.zob[q0 + slot];
        } else {
            const Surv r = sv[c - nk];
            const int i = (int)(r.pair & 0xFFFFu), j = (int)(r.pair >> 16);
            z = lay.zob[r.code] ^ lay.zkey[i];
            if (j != (int)SINGLE) z ^= lay.zkey[j];
            e = r.E;
        }
    };
    // candidate c into position p of the sort arrays
    auto load_cand = [&](int c, int p) {
        double e;
        uint64_t z;
        cand_key(c, e, z);
        key[p] = e;
        ref[p] = ref_of(c);
        zk[p] = z;
    };

    int nrun = -1;
    const int target = 2 * M + 64;
    if (n > 256 && n <= HASH_PER * 256) {
        // Copies first.  Copies of one state share (E, Zobrist hash): the table
        // keeps per key the lowest candidate index, which is the copy the sort
        // would keep (kept states precede survivors, survivors are in order).
        // Only the distinct representatives are ranked.  Every copy that could
        // reach the cut is then compared word by word with its representative;
        // a mismatch (two states whose mixes agree) falls back to sorting all.
        uint64_t* const tab = kz;
        for (int k = threadIdx.x; k < HASH_T; k += blockDim.x) tab[k] = HASH_EMPTY;
        if (threadIdx.x == 0) {
            tmp[1] = 0;
            tmp[2] = 0;
        }
        __syncthreads();
        double ce[HASH_PER];
        uint64_t cz[HASH_PER];
        int cslot[HASH_PER];
#pragma unroll
        for (int m = 0; m < HASH_PER; ++m) {
            const int c = (int)threadIdx.x + 256 * m;
            cslot[m] = -1;
            ce[m] = 0.0;
            cz[m] = 0;
            if (c < n) cand_key(c, ce[m], cz[m]);
        }
#pragma unroll
        for (int m = 0; m < HASH_PER; ++m) {
            const int c = (int)threadIdx.x + 256 * m;
            if (c < n) {
                const uint64_t h = mix_state(cz[m], ce[m]);
                const uint64_t mine = (h & ~(uint64_t)(HASH_T - 1)) | (uint64_t)c;
                int slot = (int)(h & (HASH_T - 1));
                for (;;) {
                    uint64_t v = tab[slot];
                    if (v == HASH_EMPTY) {
                        v = atomicCAS(&tab[slot], HASH_EMPTY, mine);
                        if (v == HASH_EMPTY) break;
                    }
                    if ((v >> 12) == (mine >> 12)) {
                        atomicMin(&tab[slot], mine);
                        break;
                    }
                    slot = (slot + 1) & (HASH_T - 1);
                }
                cslot[m] = slot;
            }
        }
        __syncthreads();
        int crep[HASH_PER];
        int nmine = 0;
        double lo = INFINITY, hi = -INFINITY;
#pragma unroll
        for (int m = 0; m < HASH_PER; ++m) {
            const int c = (int)threadIdx.x + 256 * m;
            crep[m] = cslot[m] >= 0 ? (int)(tab[cslot[m]] & (uint64_t)(HASH_T - 1)) : -1;
            if (crep[m] == c) {
                ++nmine;
                lo = fmin(lo, ce[m]);
                hi = fmax(hi, ce[m]);
            }
        }
        atomicAdd(&tmp[1], nmine);
        for (int off = 32; off > 0; off >>= 1) {
            lo = fmin(lo, __shfl_xor(lo, off, 64));
            hi = fmax(hi, __shfl_xor(hi, off, 64));
        }
        if ((threadIdx.x & 63) == 0) {
            red[threadIdx.x >> 6] = lo;
            red[4 + (threadIdx.x >> 6)] = hi;
        }
        for (int k = threadIdx.x; k < NBIN; k += blockDim.x) hist[k] = 0;
        __syncthreads();   // the table is no longer read: key and zk are the sort arrays again
        const int nrep = tmp[1];
        // representatives to rank: all of them, or the lowest bins holding M
        int bmax = NBIN;
        lo = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
        hi = fmax(fmax(red[4], red[5]), fmax(red[6], red[7]));
        const double scale = hi > lo ? (double)NBIN / (hi - lo) : 0.0;
        auto bin_of = [&](double e) -> int {
            const int k = (int)((e - lo) * scale);
            return k < 0 ? 0 : (k >= NBIN ? NBIN - 1 : k);
        };
        if (nrep > M + 32) {
#pragma unroll
            for (int m = 0; m < HASH_PER; ++m)
                if (crep[m] == (int)threadIdx.x + 256 * m) atomicAdd(&hist[bin_of(ce[m])], 1);
            __syncthreads();
            first_bin_reaching(hist, nrep < M ? nrep : M, tmp);
            __syncthreads();
            bmax = tmp[0];
        }
#pragma unroll
        for (int m = 0; m < HASH_PER; ++m) {
            const int c = (int)threadIdx.x + 256 * m;
            if (crep[m] == c && (bmax == NBIN || bin_of(ce[m]) <= bmax)) {
                const int pos = atomicAdd(&tmp[2], 1);
                if (pos < MERGE_CH) {
                    key[pos] = ce[m];
                    ref[pos] = ref_of(c);
                    zk[pos] = cz[m];
                }
            }
        }
        __syncthreads();
        const int np = tmp[2];
        __syncthreads();
        if (np <= MERGE_CH) {
            if (np <= 256) {
                // few representatives: the rank of each in the (E, psi, ref)
                // order is the count of those before it, and it moves there
                // (ranks are distinct: the order is total)
                const int t = (int)threadIdx.x;
                double kt = 0.0;
                uint32_t rt = 0;
                uint64_t zt = 0;
                if (t < np) {
                    kt = key[t];
                    rt = ref[t];
                    zt = zk[t];
                }
                int rank = 0, same = 0;
                const StateLess<SearchSrc> less{&src, W, false};
                for (int j = 0; j < np; ++j) {
                    const double kj = key[j];
                    if (kj < kt) {
                        ++rank;
                    } else if (kj == kt && j != t && t < np) {
                        // equal energies: the same state under two hash keys
                        // (+0 and -0) is left to the sort; else psi decides
                        if (zk[j] == zt) same = 1;
                        else if (less(kj, ref[j], zk[j], kt, rt, zt)) ++rank;
                    }
                }
                if (__syncthreads_or(same)) {
                    nrun = sort_dedupe_keep(src, W, key, ref, zk, np, M, tmp, keep);
                } else {
                    if (t < np && rank < M) {
                        key[rank] = kt;
                        ref[rank] = rt;
                        zk[rank] = zt;
                    }
                    __syncthreads();
                    nrun = np < M ? np : M;
                }
            } else {
                nrun = sort_dedupe_keep(src, W, key, ref, zk, np, M, tmp, keep);
            }
            const double cut = nrun >= M ? key[M - 1] : INFINITY;
            // the copies to confirm, as (copy, representative) in the slot
            // arrays (unused until the new set is written); more than fit
            // sends the merge to the exact sort of everything
            uint32_t* const vlist = reinterpret_cast<uint32_t*>(freeslot);
            constexpr int VCAP = 2048;
            if (threadIdx.x == 0) tmp[3] = 0;
            __syncthreads();
            int bad = 0;
#pragma unroll
            for (int m = 0; m < HASH_PER; ++m) {
                const int c = (int)threadIdx.x + 256 * m;
                if (crep[m] >= 0 && crep[m] != c && ce[m] <= cut) {
                    const int v = atomicAdd(&tmp[3], 1);
                    if (v < VCAP) vlist[v] = (uint32_t)c | ((uint32_t)crep[m] << 16);
                    else bad = 1;
                }
            }
            __syncthreads();
            const int nv = tmp[3] < VCAP ? tmp[3] : VCAP;
            for (int v = threadIdx.x; v < nv; v += blockDim.x) {
                // equal words imply equal hashes; equal energies are checked
                // as the sort's dedupe requires them
                const int c = (int)(vlist[v] & 0xFFFFu), r = (int)(vlist[v] >> 16);
                if (candE(c) != candE(r) || !same_words(src, W, ref_of(c), ref_of(r))) bad = 1;
            }
            if (__syncthreads_or(bad)) nrun = -1;
        }
    } else if (n > target + 256) {
        double lo = INFINITY, hi = -INFINITY;
        for (int c = threadIdx.x; c < n; c += blockDim.x) {
            const double e = candE(c);
            lo = fmin(lo, e);
            hi = fmax(hi, e);
        }
        for (int off = 32; off > 0; off >>= 1) {
            lo = fmin(lo, __shfl_xor(lo, off, 64));
            hi = fmax(hi, __shfl_xor(hi, off, 64));
        }
        if ((threadIdx.x & 63) == 0) {
            red[threadIdx.x >> 6] = lo;
            red[4 + (threadIdx.x >> 6)] = hi;
        }
        for (int k = threadIdx.x; k < NBIN; k += blockDim.x) hist[k] = 0;
        if (threadIdx.x == 0) tmp[1] = 0;
        __syncthreads();
        lo = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
        hi = fmax(fmax(red[4], red[5]), fmax(red[6], red[7]));
        const double scale = hi > lo ? (double)NBIN / (hi - lo) : 0.0;
        auto bin_of = [&](double e) -> int {
            const int k = (int)((e - lo) * scale);
            return k < 0 ? 0 : (k >= NBIN ? NBIN - 1 : k);
        };
        for (int c = threadIdx.x; c < n; c += blockDim.x) atomicAdd(&hist[bin_of(candE(c))], 1);
        __syncthreads();
        first_bin_reaching(hist, target, tmp);
        __syncthreads();
        const int bmax = tmp[0];
        // the candidates of bins <= bmax, in any order (they are sorted next),
        // if they fit the sort arrays
        for (int c = threadIdx.x; c < n; c += blockDim.x) {
            if (bin_of(candE(c)) <= bmax) {
                const int pos = atomicAdd(&tmp[1], 1);
                if (pos < MERGE_CH) load_cand(c, pos);
            }
        }
        __syncthreads();
        const int np = tmp[1];
        __syncthreads();
        if (np <= MERGE_CH) {
            nrun = sort_dedupe_keep(src, W, key, ref, zk, np, M, tmp, keep);
            if (nrun < M && np < n) nrun = -1;   // not enough distinct states below: sort everything
        }
    }
    if (nrun < 0) {
        // everything, in passes that carry the running best M
        for (int c = threadIdx.x; c < nk; c += blockDim.x) load_cand(c, c);
        __syncthreads();
        nrun = nk;
        int pos = nk;
        do {
            const int take = min(n - pos, MERGE_CH - nrun);
            for (int t = threadIdx.x; t < take; t += blockDim.x) load_cand(pos + t, nrun + t);
            __syncthreads();
            nrun = sort_dedupe_keep(src, W, key, ref, zk, nrun + take, M, tmp, keep);
            pos += take;
        } while (pos < n);
    }

    if (threadIdx.x == 0) atomicAdd(&lay.ctr[CTR_SURV], (unsigned long long)cnt);
    if (ctot > lay.cap_surv) {
        // some candidates were not stored: the stored ones still bound the cut
        if (threadIdx.x == 0) {
            const double oldc = lay.cut[s];
            // never above the cut the candidates were scanned with
            const double nc = (nrun == M && key[M - 1] < oldc) ? key[M - 1] : oldc;
            lay.cut[s] = nc;
            lay.retry[s] = 1;
            lay.nm_count[s] = 0;
            atomicAdd(&lay.flags[FLAG_OVERFLOW], 1);
            atomicAdd(&lay.ctr[CTR_RETRY], 1ull);
            if (!(nc < oldc)) atomicAdd(&lay.flags[FLAG_STUCK], 1);
        }
        return;
    }

    // slots used by the current set; new states take the free ones in order
    for (int q = threadIdx.x; q < 2 * M; q += blockDim.x) used[q] = 0;
    __syncthreads();
    for (int k = threadIdx.x; k < nk; k += blockDim.x) used[keptl[k]] = 1;
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
    int nnew = 0;
    for (int c0 = 0; c0 < nrun; c0 += 256) {
        const int k = c0 + threadIdx.x;
        const int isnew = (k < nrun && (ref[k] & REF_SURV)) ? 1 : 0;
        int excl;
        const int tot = block_exclusive_scan(isnew, tmp, excl);
        if (k < nrun) {
            if (isnew) {
                const int m = nnew + excl;
                const Surv r = sv[ref[k] & ~REF_SURV];
                const int slot = freeslot[m];
                kslot[k] = slot;
                keep[k] = 1;
                lay.nm_code[(size_t)s * M + m] = (int)r.code;
                lay.nm_pair[(size_t)s * M + m] = r.pair;
                lay.nm_slot[(size_t)s * M + m] = slot;
                lay.E[q0 + slot] = r.E;
                lay.zob[q0 + slot] = zk[k];
                lay.fresh[q0 + slot] = 1;
                if (lay.form == 2) lay.xfull[q0 + slot] = 0;
                const int i = (int)(r.pair & 0xFFFFu), j = (int)(r.pair >> 16);
                const uint64_t* xp = lay.bits + (size_t)r.code * lay.Wmax;
                uint64_t* xn = lay.bits + (q0 + slot) * lay.Wmax;
                for (int w = 0; w < lay.Wmax; ++w) {
                    uint64_t v = xp[w];
                    if ((i >> 6) == w) v ^= 1ull << (i & 63);
                    if (j != (int)SINGLE && (j >> 6) == w) v ^= 1ull << (j & 63);
                    xn[w] = v;
                }
            } else {
                kslot[k] = keptl[ref[k]];
                keep[k] = 0;
            }
        }
        nnew += tot;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nrun; k += blockDim.x) {
        if (!keep[k]) lay.fresh[q0 + kslot[k]] = 0;
        lay.kept[(size_t)s * M + k] = kslot[k];
    }
    if (threadIdx.x == 0) {
        lay.nkept[s] = nrun;
        lay.nm_count[s] = nnew;
        lay.retry[s] = 0;
        if (lay.form == 2) {
            // learned form: a ranking step that finds nothing is followed by a
            // full enumeration; a full enumeration that finds nothing certifies
            // that the set is stable under the exact step
            const int mode = lay.mode[s];
            if (nnew > 0) {
                lay.mode[s] = 0;
                atomicAdd(&lay.flags[FLAG_ACTIVE], 1);
            } else if (mode == 0) {
                lay.mode[s] = 1;
                atomicAdd(&lay.flags[FLAG_ACTIVE], 1);
            } else {
                lay.active[s] = 0;
            }
        } else if (nnew > 0) {
            atomicAdd(&lay.flags[FLAG_ACTIVE], 1);
        } else {
            lay.active[s] = 0;
        }
    }
}

// ------------------------------------------------------------------ k_fupdate
// Local fields of the states that entered in the last merge (row a6):
// F_k = F_k(parent) - 2 s_i J_ik - 2 s_j J_jk with the parent's spins.  One
// wave per new state, lanes over sites; blocks of 4 states, search-major, so
// that the blocks of one instance run together and its coupling rows stay in
// L2 while its new states use them.
__global__ __launch_bounds__(256) void k_fupdate(Layout lay, const double* __restrict__ J4)
{
    if (step_halted(lay)) return;   // a later step of a multi-step graph after a halt
    const int groups = (lay.M + 3) / 4;
    // XCD x (blocks x, x + 8, ...) takes the x-th contiguous eighth of the
    // (search, group) blocks, so that the states of an instance meet in one
    // XCD's L2 and share the coupling rows they read
    // (the grid is a multiple of 8 blocks, at least S * groups)
    const unsigned per = gridDim.x / 8;
    const unsigned lb = (blockIdx.x % 8) * per + blockIdx.x / 8;   // logical block
    if (lb >= (unsigned)lay.S * (unsigned)groups) return;
    const int s = (int)(lb / groups);
    const int m = (int)(lb % groups) * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (m >= lay.nm_count[s]) return;
    const int b = s / lay.L;
    const int N = lay.N[b], Np = lay.Npad[b];
    const size_t k0 = (size_t)s * lay.M + m;
    const int code = lay.nm_code[k0];
    const uint32_t pr = lay.nm_pair[k0];
    const int slot = lay.nm_slot[k0];
    const int i = (int)(pr & 0xFFFFu), j = (int)(pr >> 16);
    const uint64_t* xp = lay.bits + (size_t)code * lay.Wmax;
    const double ci = -0.5 * spin_of(xp, i);   // -2 s_i J = -0.5 s_i (4J)
    const bool pairf = j != (int)SINGLE;
    const double cj = pairf ? -0.5 * spin_of(xp, j) : 0.0;
    const size_t qn = (size_t)s * 2 * lay.M + slot;
    if (lay.Fq && lay.J4f) {
        // fields in grid units, 4J exact in FP32: the changes -2 s J_ik are
        // whole grid units, so the sums are exact
        const double u = 1.0 / lay.fsc[b];
        const double di = ci * u, dj = cj * u;
        const int32_t* Fp = lay.Fq + (size_t)code * lay.Npmax;
        int32_t* Fn = lay.Fq + qn * lay.Npmax;
        const float* Jf = lay.J4f + lay.joff[b];
        const float* Ji = Jf + (size_t)i * Np;
        const float* Jj = Jf + (size_t)(pairf ? j : i) * Np;
        // four entries per lane and load (rows are 64-entry aligned)
#pragma unroll 2
        for (int k = 4 * lane; k < Np; k += 256) {
            const int4 f = *reinterpret_cast<const int4*>(Fp + k);
            const float4 ji = *reinterpret_cast<const float4*>(Ji + k);
            double v0 = (double)f.x + di * (double)ji.x, v1 = (double)f.y + di * (double)ji.y;
            double v2 = (double)f.z + di * (double)ji.z, v3 = (double)f.w + di * (double)ji.w;
            if (pairf) {
                const float4 jj = *reinterpret_cast<const float4*>(Jj + k);
                v0 += dj * (double)jj.x;
                v1 += dj * (double)jj.y;
                v2 += dj * (double)jj.z;
                v3 += dj * (double)jj.w;
            }
            int4 o;
            o.x = k < N ? (int32_t)v0 : 0;
            o.y = k + 1 < N ? (int32_t)v1 : 0;
            o.z = k + 2 < N ? (int32_t)v2 : 0;
            o.w = k + 3 < N ? (int32_t)v3 : 0;
            *reinterpret_cast<int4*>(Fn + k) = o;
        }
        return;
    }
    if (lay.J4f) {
        // 4J exact in FP32: half the coupling bytes, the same sums
        const double* Fp = lay.Fd + (size_t)code * lay.Npmax;
        double* Fn = lay.Fd + qn * lay.Npmax;
        const float* Jf = lay.J4f + lay.joff[b];
        const float* Ji = Jf + (size_t)i * Np;
        const float* Jj = Jf + (size_t)(pairf ? j : i) * Np;
        // two entries per lane and load (rows are 64-entry aligned), four
        // iterations in flight
#pragma unroll 4
        for (int k = 2 * lane; k < Np; k += 128) {
            const double2 f = *reinterpret_cast<const double2*>(Fp + k);
            const float2 ji = *reinterpret_cast<const float2*>(Ji + k);
            double v0 = f.x + ci * (double)ji.x, v1 = f.y + ci * (double)ji.y;
            if (pairf) {
                const float2 jj = *reinterpret_cast<const float2*>(Jj + k);
                v0 += cj * (double)jj.x;
                v1 += cj * (double)jj.y;
            }
            double2 o;
            o.x = k < N ? v0 : 0.0;
            o.y = k + 1 < N ? v1 : 0.0;
            *reinterpret_cast<double2*>(Fn + k) = o;
        }
        return;
    }
    const FieldRow Fp = field_row(lay, (size_t)code, b);
    const double* Jb = J4 + lay.joff[b];
    const double* Ji = Jb + (size_t)i * Np;
    const double* Jj = Jb + (size_t)(pairf ? j : i) * Np;
    for (int k = lane; k < Np; k += 64) {
        double v = Fp[k] + ci * Ji[k];
        if (pairf) v += cj * Jj[k];
        field_store(lay, qn, b, k, k < N ? v : 0.0);
    }
}

// ------------------------------------------------------------------ k_final
// Alg. 4: per instance, the M lowest distinct states of the union of its L
// kept sets, sorted by (E, psi).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_final(Layout lay)
{
    __shared__ double key[MERGE_CH];
    __shared__ uint32_t ref[MERGE_CH];
    __shared__ uint64_t zk[MERGE_CH];
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
                zk[n + k] = lay.zob[(size_t)s * 2 * M + slot];
            }
            n += nk;
            ++l;
        }
        __syncthreads();
        nrun = sort_dedupe_keep(src, W, key, ref, zk, n, M, tmp, keep);
    }
    for (int k = threadIdx.x; k < nrun; k += blockDim.x) {
        lay.out_E[(size_t)b * M + k] = key[k];
        for (int w = 0; w < lay.Wmax; ++w)
            lay.out_bits[((size_t)b * M + k) * lay.Wmax + w] = w < W ? src.decode(ref[k]).word(w) : 0ull;
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

// Entries of the frontier's key/idx arrays: the candidate pool, the fresh
// states (M <= 1024) and a prefix of the sites of one state.
static int frontier_keys(const Layout& lay)
{
    int kn = POOL;
    while (kn < lay.Npmax) kn <<= 1;
    return kn;
}

hipError_t frontier_set_lds(const Layout& lay)
{
    return hipFuncSetAttribute(reinterpret_cast<const void*>(k_frontier), hipFuncAttributeMaxDynamicSharedMemorySize,
                               frontier_keys(lay) * 12);
}

hipError_t launch_frontier_plan(const Layout& lay, hipStream_t st)
{
    long long* fr_prefix = lay.item_prefix + (lay.B + 1);
    const int kn = frontier_keys(lay);
    hipLaunchKernelGGL(k_frontier, dim3(lay.S), dim3(256), (size_t)kn * 12, st, lay, lay.J4, kn);
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, st, lay, fr_prefix, 1);
    return hipGetLastError();
}

hipError_t launch_plan_only(const Layout& lay, hipStream_t st)
{
    long long* fr_prefix = lay.item_prefix + (lay.B + 1);
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, st, lay, fr_prefix, 0);
    return hipGetLastError();
}

__global__ void k_clear_survivors(Layout lay)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < lay.S) lay.surv_count[t] = 0;
}

hipError_t launch_clear_survivors(const Layout& lay, hipStream_t st)
{
    hipLaunchKernelGGL(k_clear_survivors, dim3((lay.S + 255) / 256), dim3(256), 0, st, lay);
    return hipGetLastError();
}

// Site bound: the entries of instance b that the preparation left to the scan,
// in frontier order (consecutive states of a search stay together, so a scan
// item re-signs few columns between them), and the pair count of the step.
__global__ __launch_bounds__(256) void k_sb_list(Layout lay, int count)
{
    if (step_halted(lay)) return;   // a later step of a multi-step graph after a halt
    __shared__ int tmp[256];
    const int b = blockIdx.x;
    const int P = lay.fr_count[b];
    const size_t fb = (size_t)b * lay.fmax;
    const int retry_mode = lay.flags[FLAG_RETRY_MODE];
    const unsigned long long N = (unsigned long long)lay.N[b];
    unsigned long long pairs = 0, bounded = 0;
    int nfull = 0;
    for (int f0 = 0; f0 < P; f0 += 256) {
        const int f = f0 + (int)threadIdx.x;
        int isfull = 0;
        if (f < P) {
            const int v = lay.fr_bound[fb + f];
            isfull = v == 0;
            const int s = lay.fr_list[fb + f] / (2 * lay.M);
            if (!retry_mode || lay.retry[s]) {
                pairs += isfull ? N * (N - 1) / 2 : (unsigned long long)(v - 1) * (v - 2) / 2;
                bounded += isfull ? 0 : 1;
            }
        }
        int excl;
        const int tot = block_exclusive_scan(isfull, tmp, excl);
        if (isfull) lay.full_list[fb + nfull + excl] = f;
        nfull += tot;
    }
    if (threadIdx.x == 0) lay.full_count[b] = nfull;
    if (count) {
        for (int off = 32; off > 0; off >>= 1) {
            pairs += __shfl_xor(pairs, off, 64);
            bounded += __shfl_xor(bounded, off, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            if (pairs) atomicAdd(&lay.ctr[CTR_PAIRS], pairs);
            if (bounded) atomicAdd(&lay.ctr[CTR_BOUNDED], bounded);
        }
    }
}

// Scan items of the FP64 scan over the entries left to it.
__global__ __launch_bounds__(1024) void k_sb_items(Layout lay)
{
    if (step_halted(lay)) return;   // a later step of a multi-step graph after a halt
    __shared__ long long part[1024];
    const int t = threadIdx.x;
    const int per = (lay.B + 1023) / 1024;
    const int b0 = t * per;
    long long items = 0;
    for (int b = b0; b < b0 + per && b < lay.B; ++b)
        items += ((long long)lay.full_count[b] + lay.scb[b] - 1) / lay.scb[b] * tiles_of(lay.N[b]);
    part[t] = items;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const long long a = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += a;
        __syncthreads();
    }
    long long run = part[t] - items;
    for (int b = b0; b < b0 + per && b < lay.B; ++b) {
        lay.item_prefix[b] = run;
        run += ((long long)lay.full_count[b] + lay.scb[b] - 1) / lay.scb[b] * tiles_of(lay.N[b]);
    }
    if (t == 1023) lay.item_prefix[lay.B] = part[1023];
}

hipError_t launch_prep(const Layout& lay, hipStream_t st, bool count, hipEvent_t after_bound)
{
    const long long* fr_prefix = lay.item_prefix + (lay.B + 1);
    if (lay.sb) {
        hipLaunchKernelGGL(k_site_bound, dim3(SB_GRID), dim3(256), 0, st, lay, fr_prefix);
        if (after_bound) {
            const hipError_t e = hipEventRecord(after_bound, st);
            if (e != hipSuccess) return e;
        }
    }
    if (lay.form == 1) {
        hipError_t e = launch_prep32(lay, st);
        if (e == hipSuccess && lay.sb) hipLaunchKernelGGL(k_sb_list, dim3(lay.B), dim3(256), 0, st, lay, count ? 1 : 0);
        return e == hipSuccess ? hipGetLastError() : e;
    }
    if (lay.sb) hipLaunchKernelGGL(k_prep<true>, dim3(4096), dim3(256), 0, st, lay, fr_prefix);
    else hipLaunchKernelGGL(k_prep<false>, dim3(4096), dim3(256), 0, st, lay, fr_prefix);
    if (lay.sb) {
        hipLaunchKernelGGL(k_sb_list, dim3(lay.B), dim3(256), 0, st, lay, count ? 1 : 0);
        hipLaunchKernelGGL(k_sb_items, dim3(1), dim3(1024), 0, st, lay);
    }
    return hipGetLastError();
}

hipError_t launch_scan(const Layout& lay, int scan_grid, hipStream_t st)
{
    if (lay.form == 1) return launch_scan32(lay, scan_grid, st);
    if (lay.h1 == H1_SINGLES) return hipSuccess;   // no pair flips to scan
    if (lay.h1 == H1_EXCHANGE)
        hipLaunchKernelGGL(k_scan<true>, dim3(scan_grid), dim3(64), 0, st, lay, lay.J4, (const double*)lay.A,
                           (const FrRec*)lay.rec, (const uint64_t*)lay.fbits);
    else
        hipLaunchKernelGGL(k_scan<false>, dim3(scan_grid), dim3(64), 0, st, lay, lay.J4, (const double*)lay.A,
                           (const FrRec*)lay.rec, (const uint64_t*)lay.fbits);
    return hipGetLastError();
}

hipError_t launch_merge(const Layout& lay, hipStream_t st)
{
    hipLaunchKernelGGL(k_merge, dim3(lay.S), dim3(256), 0, st, lay, lay.J4);
    return hipGetLastError();
}

hipError_t launch_fupdate(const Layout& lay, hipStream_t st)
{
    const unsigned blocks = (unsigned)lay.S * ((lay.M + 3) / 4);
    hipLaunchKernelGGL(k_fupdate, dim3((blocks + 7) / 8 * 8), dim3(256), 0, st, lay, lay.J4);
    return hipGetLastError();
}

// Multi-step graphs: the halt flag is cleared by a kernel (the graph holds no
// memset), and after step t the active count is recorded; a step that found
// every search stable, or a full candidate buffer (the host then runs the
// retry passes), halts the graph's later steps.
__global__ void k_graph_begin(Layout lay)
{
    if (threadIdx.x == 0) {
        lay.flags[FLAG_HALT] = 0;
        lay.flags[FLAG_HALT_STEP] = -1;
    }
}

__global__ void k_step_end(Layout lay, int t)
{
    if (threadIdx.x != 0 || step_halted(lay)) return;
    const int active = lay.flags[FLAG_ACTIVE];
    lay.step_active[t] = active;
    if (active == 0 || lay.flags[FLAG_OVERFLOW] > 0) {
        lay.flags[FLAG_HALT] = 1;
        lay.flags[FLAG_HALT_STEP] = t;
    }
}

hipError_t launch_graph_begin(const Layout& lay, hipStream_t st)
{
    hipLaunchKernelGGL(k_graph_begin, dim3(1), dim3(64), 0, st, lay);
    return hipGetLastError();
}

hipError_t launch_step_end(const Layout& lay, int t, hipStream_t st)
{
    hipLaunchKernelGGL(k_step_end, dim3(1), dim3(64), 0, st, lay, t);
    return hipGetLastError();
}

hipError_t launch_final(const Layout& lay, hipStream_t st)
{
    hipLaunchKernelGGL(k_final, dim3(lay.B), dim3(256), 0, st, lay);
    return hipGetLastError();
}

}  // namespace qi

// Internal declarations shared by the HIP translation units of the library.
// Device memory layout (all arrays live in HBM for the whole run):
//   J4     per instance b: Npad[b] x Npad[b] row-major FP64 holding 4*J_ij
//          (zero in the padding); 4*J is exact, it is the pair term of the
//          energy change.
//   h      per instance: Npad[b] FP64.
//   pool   per search s: 2M slots; slot q holds bits[Wmax], E, zob, F[Npmax]
//          (F exact: 32-bit integers of the instance's grid, or FP64).
//          A new kept state always takes a slot that the current kept set
//          does not use, so parents stay readable while children are written.
//   kept   per search: up to M slot ids sorted by (E, psi).
//   front  per instance: list of (search, slot) of states to expand.
//   A      per frontier entry: a_i = -2 s_i F_i (the single-flip change).
//   surv   per search: candidate records {E_child, parent slot, i | j<<16}.
// Learned-proposal form: frontier states whose pair flips are ranked by the
// scoring network are listed from the back of the instance's frontier list,
// states enumerated in full from the front.
#pragma once
#include <type_traits>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qi {

constexpr int TILE = 64;            // rows of one J tile (one row per lane)
constexpr int TCOL = 32;            // columns of one J tile held in registers
constexpr int MAX_N = 4096;         // pair indices are packed into 16 bits
constexpr int MERGE_CH = 2048;      // candidates sorted per merge pass (LDS)
constexpr int STAGE = 256;          // wave-private survivor staging (records)
constexpr uint32_t SINGLE = 0xFFFFu;   // j field of a single-flip record
constexpr uint32_t REF_SURV = 0x80000000u;
constexpr int MLP_H = 64;           // hidden width of the pair-scoring network
constexpr int MLP_NPARAM = 4 * MLP_H + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1;   // 4545
constexpr int MLP_W1 = 0, MLP_B1 = 4 * MLP_H, MLP_W2 = MLP_B1 + MLP_H, MLP_B2 = MLP_W2 + MLP_H * MLP_H,
              MLP_W3 = MLP_B2 + MLP_H, MLP_B3 = MLP_W3 + MLP_H;
constexpr int LR_WAVES = 4;                        // waves of the ranking kernel's block
constexpr int LR_R = 16;                           // blocks of 16 pairs per wave between barriers
constexpr int LR_ROOM = LR_WAVES * LR_R * 16;      // keys appended per round at most

struct Surv {
    double E;        // energy of the child
    uint32_t code;   // pool slot of the parent: search * 2M + slot
    uint32_t pair;   // i | j << 16, j = SINGLE for a single flip
};
static_assert(sizeof(Surv) == 16, "record layout");

// What the scan needs of one frontier state besides its a_i values.
struct FrRec {
    double T;        // cut - E: a pair survives iff a_i + a_j + 4 s_i s_j J_ij <= T
    double E;        // energy of the state
    int s;           // search
    int code;        // s * 2M + slot
};
static_assert(sizeof(FrRec) == 24, "record layout");

// Everything the kernels need, passed by value.
struct Layout {
    int B, L, M, S;          // instances, searches per instance, kept per search, searches
    int Wmax, Npmax;         // words and padded spins of the largest instance
    int fmax;                // frontier entries per instance (= L*M)
    int cap_surv;            // survivor records per search
    int* scb;                // [B] frontier states per scan item, per instance (tuned per N)
    int sc_auto;             // 1: the plan chooses the states per item each step
    int scan_waves;          // waves of the scan's grid
    const int* N;            // [B]
    const int* Npad;         // [B]
    const long long* joff;   // [B] offset of instance b in J4 (doubles)
    const double* J4;
    const double* h;         // [B][Npmax]
    const uint64_t* zkey;    // [MAX_N] Zobrist keys per site
    // pool
    uint64_t* bits;          // [S][2M][Wmax]
    double* E;               // [S][2M]
    uint64_t* zob;           // [S][2M]
    // local fields of the pool slots, [S][2M][Npmax]: when every instance's
    // fields fit, 32-bit integers in units of the instance's grid (F = Fq *
    // fsc[b], exact), else FP64; exactly one of Fq and Fd is set
    int32_t* Fq;
    double* Fd;
    const double* fsc;       // [B] grid unit of instance b (a power of two)
    uint8_t* fresh;          // [S][2M]
    int* kept;               // [S][M]
    int* nkept;              // [S]
    int* active;             // [S]
    int* retry;              // [S]
    double* cut;             // [S] child energies above this cannot enter
    // frontier
    int* fr_count;           // [B]
    int* fr_list;            // [B][fmax] : s * 2M + slot
    double* A;               // [B][fmax][Npmax]
    FrRec* rec;              // [B][fmax]
    uint64_t* fbits;         // [B][fmax][Wmax] : copy of the state's words
    // site bound (forms 0 and 1, on request): a state whose pairs can only
    // involve a few sites has them evaluated in the preparation kernel
    int sb;                  // 1 = site bound on
    const float* rmax4;      // [B][Npmax] max_j |4J_ij| of row i, rounded up to FP32
    uint16_t* fr_bound;      // [B][fmax] 0 = scanned in full, else 1 + the sites kept by the bound
    int* full_list;          // [B][fmax] entries left to the scan, in frontier order
    int* full_count;         // [B]
    // survivors
    int* surv_count;         // [S]
    Surv* surv;              // [S][cap_surv]
    // scheduling and counters
    long long* item_prefix;  // [4][B+1]: scan items, prepared entries, FP32 scan items, ranked entries
    unsigned long long* ctr; // [16] device counters (see CTR_*)
    int* flags;              // [8] per-step flags (see FLAG_*)
    int* step_active;        // [MAX_GRAPH_STEPS] active searches after each step of a multi-step graph
    // new kept states of the last merge, for the field update
    int* nm_count;           // [S]
    int* nm_code;            // [S][M] parent slot code
    uint32_t* nm_pair;       // [S][M] i | j << 16
    int* nm_slot;            // [S][M] slot taken by the new state
    // the perturbation H1 that defines the neighbourhood (Sec. VI): H1_FLIPS
    // single and pair flips (Eq. 16), H1_SINGLES single flips only, H1_EXCHANGE
    // pair flips of unequal spins only (the XX interaction)
    int h1;
    // split-bf16 form
    int form;                // 0 plain, 1 split-bf16
    const float* J32;        // per instance, fl32(4J) (same layout as J4)
    const float* J4f;        // the same buffer when every 4J_ij is exact in FP32 (else null)
    const uint16_t* Jhi;     // per instance, bf16(4J)
    const uint16_t* Jlo;     // per instance, bf16(4J - hi)
    const double* ybound;    // [B] max |4J_ij|
    const double* ebf;       // [B] bound on |F~ - F| of the bf16 hi+lo fields
    const double* abound;    // [B] bound on |a_i| = 2 |F_i| <= 2 (|h_i| + sum_j |J_ij|) over all states
    float* Ft;               // [S][Npmax] F~ of the initial states (bf16 hi+lo GEMM, FP32 sums)
    float* A32;              // [B][fmax][Npmax] fl32(a_i)
    float* RR32;             // [B][fmax][Npmax] T - a_i + slack, rounded up to FP32
    int h16;                 // 1 = the split scan runs in packed FP16 (A32 rows then hold fl16(a))
    const uint16_t* J16;     // per instance, fl16(4J) (same layout as J4), or null
    // learned-proposal form
    uint8_t* xfull;          // [S][2M] 1 = every pair flip of the state was evaluated exactly
    int* mode;               // [S] 0 = the next step ranks pairs, 1 = it enumerates all pairs
    int* last_mode;          // [S] the mode of the last step
    int* lr_count;           // [B] ranked frontier entries, at fr_list[fmax-lr_count .. fmax)
    int topk;                // K = topk * N proposals per state
    int scorer;              // 0 network, 1 f_i + f_j, 2 hashed uniform
    uint64_t seed;           // salt of the uniform scorer and of the trace sampling
    const float* mlp;        // [MLP_NPARAM] FP32 master parameters; bf16 is taken in the kernel
    const uint16_t* Jn16;    // per instance, bf16(sqrt(N) J_ij) (same layout as J4)
    uint32_t* prop;          // [B][fmax][kmax] proposals of the last step (i | j << 16), or null
    int* prop_n;             // [B][fmax] proposals recorded per entry
    int kmax;                // row stride of prop (K of the largest instance)
    int cap_lr;              // candidate keys held in LDS per ranked state
    uint64_t* lr_tmp;        // [grid][kmax] compaction buffer of the ranking kernel
    // trace capture (features, label) of expanded states
    float* tr_feat;          // [tr_cap][4]
    uint8_t* tr_label;       // [tr_cap]
    long long tr_cap;
    int tr_neg;              // sampled pair flips per traced state
    float tr_rate;           // fraction of expanded states traced
    // final merge output
    uint64_t* out_bits;      // [B][M][Wmax]
    double* out_E;           // [B][M]
    int* out_count;          // [B]
};

// The local fields of one pool slot, read as FP64 whichever way they are held.
struct FieldRow {
    const int32_t* q;
    const double* d;
    double sc;
    __device__ double operator[](int i) const { return q ? (double)q[i] * sc : d[i]; }
    // K fields at idx(0 .. K-1), the loads issued together (the choice of
    // storage is made once, outside them)
    template <int K, typename Idx>
    __device__ void gather(double (&v)[K], Idx idx) const
    {
        if (q) {
            int32_t t[K];
#pragma unroll
            for (int k = 0; k < K; ++k) t[k] = q[idx(k)];
#pragma unroll
            for (int k = 0; k < K; ++k) v[k] = (double)t[k] * sc;
        } else {
#pragma unroll
            for (int k = 0; k < K; ++k) v[k] = d[idx(k)];
        }
    }
};

__device__ inline FieldRow field_row(const Layout& lay, size_t slot, int b)
{
    FieldRow r;
    r.q = lay.Fq ? lay.Fq + slot * lay.Npmax : nullptr;
    r.d = lay.Fq ? nullptr : lay.Fd + slot * lay.Npmax;
    r.sc = lay.fsc[b];
    return r;
}

// Field i of a pool slot from its exact FP64 value (on the instance's grid).
__device__ inline void field_store(const Layout& lay, size_t slot, int b, int i, double v)
{
    if (lay.Fq) lay.Fq[slot * lay.Npmax + i] = (int32_t)(v / lay.fsc[b]);
    else lay.Fd[slot * lay.Npmax + i] = v;
}

enum { CTR_PAIRS = 0, CTR_SINGLES = 1, CTR_FRONTIER = 2, CTR_SURV = 3, CTR_RETRY = 4, CTR_STEPS = 5,
       CTR_FALLBACK = 6, CTR_SCORED = 7, CTR_LEARNED = 8, CTR_TRACE = 9, CTR_BOUNDED = 10 };
constexpr int SB_CAP = 256;          // most sites a state may keep for the site-bound evaluation
enum { H1_FLIPS = 0, H1_SINGLES = 1, H1_EXCHANGE = 2 };

constexpr int MAX_SURV_CAP = 1 << 24;   // candidate records per search, at most
constexpr int MAX_GRAPH_STEPS = 64;   // steps captured in one replayed graph at most

// FLAG_HALT: a step of a multi-step graph found every search stable or a
// search's candidate buffer full; the kernels of the graph's later steps then
// return at once (FLAG_HALT_STEP holds the step), and the host takes over.
enum { FLAG_ACTIVE = 0, FLAG_OVERFLOW = 1, FLAG_STUCK = 2, FLAG_RETRY_MODE = 3, FLAG_FIRST = 4, FLAG_HALT = 5,
       FLAG_HALT_STEP = 6 };

__device__ inline bool step_halted(const Layout& lay) { return lay.flags[FLAG_HALT] != 0; }

__host__ __device__ inline int words_of(int N) { return (N + 63) >> 6; }
__host__ __device__ inline int pad_of(int N) { return (N + TILE - 1) / TILE * TILE; }
// Tiles of 64 rows x 32 columns that hold pairs i < j: row block bi meets
// column blocks bc >= 2*bi of the nc = ceil(N/32) column blocks that hold a
// column below N.
__host__ __device__ inline long long tiles_of(int N) {
    const long long nb = (N + TILE - 1) / TILE, nc = (N + TCOL - 1) / TCOL;
    return nb * nc - nb * (nb - 1);
}
// Tiles of 64 x 64 (FP32 scan) with row block <= column block.
__host__ __device__ inline long long tiles64(int N)
{
    const long long nb = (N + TILE - 1) / TILE;
    return nb * (nb + 1) / 2;
}
// Tiles of 64 rows x 128 columns (FP16 scan) with some column above the rows.
constexpr int T16 = 128;
__host__ __device__ inline long long tiles16(int N)
{
    const int Np = pad_of(N);
    const int nb = Np / TILE, nc = (Np + T16 - 1) / T16;
    long long t = 0;
    for (int bi = 0; bi < nb; ++bi) t += nc - (bi >> 1);
    return t;
}
// Tiles of the form's full scan.
__host__ __device__ inline long long scan_tiles(const Layout& lay, int N)
{
    return lay.form == 1 ? (lay.h16 ? tiles16(N) : tiles64(N)) : tiles_of(N);
}

// Word k of a state held by lane k (k < 64), as a wave-uniform value.
__device__ inline uint64_t word_of_lane(uint64_t xw, int k)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)xw, k);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(xw >> 32), k);
    return ((uint64_t)hi << 32) | lo;
}

// Site bound of one frontier state, evaluated by one wave.  The pair (i, j)
// changes the energy by a_i + a_j + s_i s_j 4J_ij >= a_i + min_k a_k - max_k |4J_ik|,
// so it can pass the cut c only if both sites satisfy
// a_i + min_k a_k - max_k |4J_ik| <= T = c - E (all terms on the 2^-24 grid: exact).
// With at most SB_CAP such sites, every pair among them is evaluated with the
// scan's arithmetic (x = fma(s_i, s_j 4J_ij, a_j) <= T - a_i, E' = (E + a_i) + x)
// and its survivors recorded, and so are the single flips below the cut
// (E + a_i <= c); returns the number r of such sites (r (r - 1) / 2 pairs
// evaluated), or -1, having recorded nothing, when there are too many and the
// state must be prepared for the full scan.  sidx (site | sign << 15) and sa
// are this wave's LDS arrays of SB_CAP entries, stage its SB_STG survivor
// records.  The work is a chain of dependent memory rounds, so it is cut into
// few of them: a is held in registers (N <= 640); the pairs are taken in 8 x 8
// blocks (lane = 8 p + q), the couplings of SB_BATCH blocks gathered at once;
// survivors wait in LDS, and one atomic per state (or per full stage) reserves
// their places in the search's buffer.
constexpr int SB_AREG = 10;
constexpr int SB_BATCH = 8;
constexpr int SB_STG = 128;
constexpr int SB_GRID = 2048;   // k_site_bound blocks: 8192 waves, eight per SIMD
__device__ inline int site_bound_pairs(const Layout& lay, int b, int s, int code, double Em, double c,
                                       const uint64_t* __restrict__ x, const FieldRow F,
                                       int N, int Np, uint16_t* sidx, double* sa, Surv* stage)
{
    const uint32_t lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    const double T = c - Em;
    // the exchange neighbourhood has no single flips and only pairs of unequal spins
    const bool xch = lay.h1 == H1_EXCHANGE;
    auto bit = [&](int i) -> uint32_t { return (uint32_t)((x[i >> 6] >> (i & 63)) & 1ull); };
    auto lane_rank = [&](uint64_t m) -> int {
        return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    };
    auto wave_sync = [&]() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    // staged survivors: nst (wave-uniform) records in stage[0 .. nst)
    int nst = 0;
    auto flush = [&]() {
        wave_sync();   // the stage's writes before its reads
        int pos0 = 0;
        if (lane == 0) pos0 = atomicAdd(&lay.surv_count[s], nst);
        pos0 = __shfl(pos0, 0, 64);
        Surv* const out = lay.surv + (size_t)s * lay.cap_surv;
        for (int k = (int)lane; k < nst; k += 64)
            if (pos0 + k < lay.cap_surv) out[pos0 + k] = stage[k];
        wave_sync();   // its reads before it is refilled
        nst = 0;
    };
    auto push = [&](bool keep, double E, uint32_t pair) {
        const uint64_t m = __builtin_amdgcn_ballot_w64(keep);
        if (m) {
            const int n = __builtin_popcountll(m);
            if (nst + n > SB_STG) flush();
            if (keep) {
                Surv rec;
                rec.E = E;
                rec.code = (uint32_t)code;
                rec.pair = pair;
                stage[nst + lane_rank(m)] = rec;
            }
            nst += n;
        }
    };
    // the bound's max |4J_ik| rounded up: a site it keeps needlessly only
    // costs the evaluation of its pairs
    const float* rm = lay.rmax4 + (size_t)b * lay.Npmax;
    int r = 0;
    if (N <= 64 * SB_AREG) {
        // the state's words in one load (word k held by lane k, its bits then
        // the lane mask of the flipped spins), and a
        const uint64_t xw = (int)lane < words_of(N) ? x[lane] : 0ull;
        double areg[SB_AREG];
        uint32_t negm = 0;   // bit k: site 64k + lane has s = -1
        double amin = INFINITY;
#pragma unroll
        for (int k = 0; k < SB_AREG; ++k) {
            const int i = 64 * k + (int)lane;
            const bool neg = 64 * k < N && __builtin_amdgcn_inverse_ballot_w64(word_of_lane(xw, k));
            negm |= (neg ? 1u : 0u) << k;
            areg[k] = i < N ? (neg ? 2.0 : -2.0) * F[i] : 0.0;
            if (i < N) amin = fmin(amin, areg[k]);
        }
        for (int off = 32; off > 0; off >>= 1) amin = fmin(amin, __shfl_xor(amin, off, 64));
        // count and list in one pass; entries past SB_CAP are only counted
#pragma unroll
        for (int k = 0; k < SB_AREG; ++k) {
            const int i = 64 * k + (int)lane;
            const bool in = i < N && (areg[k] + amin) - (double)rm[i] <= T;
            const uint64_t m = __builtin_amdgcn_ballot_w64(in);
            const int pos = r + lane_rank(m);
            if (in && pos < SB_CAP) {
                sidx[pos] = (uint16_t)(i | (((negm >> k) & 1u) << 15));
                sa[pos] = areg[k];
            }
            r += __builtin_popcountll(m);
        }
        if (r > SB_CAP) return -1;
        // single flips below the cut
        if (!xch) {
#pragma unroll
            for (int k = 0; k < SB_AREG; ++k) {
                const int i = 64 * k + (int)lane;
                push(i < N && Em + areg[k] <= c, Em + areg[k], (uint32_t)i | (SINGLE << 16));
            }
        }
    } else {
        double amin = INFINITY;
        for (int i = (int)lane; i < N; i += 64) amin = fmin(amin, (bit(i) ? 2.0 : -2.0) * F[i]);
        for (int off = 32; off > 0; off >>= 1) amin = fmin(amin, __shfl_xor(amin, off, 64));
        for (int i0 = 0; i0 < N; i0 += 64) {
            const int i = i0 + (int)lane;
            const bool in = i < N && ((bit(i) ? 2.0 : -2.0) * F[i] + amin) - (double)rm[i] <= T;
            r += __builtin_popcountll(__builtin_amdgcn_ballot_w64(in));
        }
        if (r > SB_CAP) return -1;
        int base = 0;
        for (int i0 = 0; i0 < N; i0 += 64) {
            const int i = i0 + (int)lane;
            const double a = i < N ? (bit(i) ? 2.0 : -2.0) * F[i] : 0.0;
            const bool in = i < N && (a + amin) - (double)rm[i] <= T;
            const uint64_t m = __builtin_amdgcn_ballot_w64(in);
            if (in) {
                sidx[base + lane_rank(m)] = (uint16_t)(i | (bit(i) << 15));
                sa[base + lane_rank(m)] = a;
            }
            base += __builtin_popcountll(m);
            if (!xch) push(i < N && Em + a <= c, Em + a, (uint32_t)i | (SINGLE << 16));
        }
    }
    wave_sync();   // the site list before it is read
    const int pp = (int)(lane >> 3), qq = (int)(lane & 7);
    const int nb = (r + 7) >> 3;
    // the 8 x 8 blocks (P, Q), P <= Q, in row order, SB_BATCH per round
    auto next_block = [&](int& P, int& Q) {
        if (P < nb && ++Q == nb) {
            ++P;
            Q = P;
        }
    };
    auto pairs = [&](const auto* __restrict__ Jp) {
        using JT = typename std::remove_cv<typename std::remove_reference<decltype(*Jp)>::type>::type;
        constexpr int NBAT = sizeof(JT) == 8 ? SB_BATCH / 2 : SB_BATCH;   // registers per round alike
        int P = 0, Q = 0;
        while (P < nb) {
            // the couplings of the round, all loads in flight together
            JT jc[NBAT];
            int P1 = P, Q1 = Q;
#pragma unroll
            for (int u = 0; u < NBAT; ++u) {
                const int p = 8 * P1 + pp, q = 8 * Q1 + qq;
                jc[u] = (JT)0;
                if (P1 < nb && p < q && q < r) {
                    const int i = (int)(sidx[p] & 0x7FFFu), j = (int)(sidx[q] & 0x7FFFu);
                    jc[u] = Jp[(size_t)i * Np + j];
                }
                next_block(P1, Q1);
            }
#pragma unroll
            for (int u = 0; u < NBAT; ++u) {
                const int p = 8 * P + pp, q = 8 * Q + qq;
                bool keep = false;
                double E = 0.0;
                uint32_t pair = 0;
                if (P < nb && p < q && q < r) {
                    const uint32_t ei = sidx[p], ej = sidx[q];
                    const double ai = sa[p];
                    const double xv = fma((ei >> 15) ? -1.0 : 1.0, ((ej >> 15) ? -1.0 : 1.0) * (double)jc[u], sa[q]);
                    keep = xv <= T - ai && (!xch || (ei >> 15) != (ej >> 15));
                    E = (Em + ai) + xv;
                    pair = (ei & 0x7FFFu) | ((ej & 0x7FFFu) << 16);
                }
                push(keep, E, pair);
                next_block(P, Q);
            }
        }
    };
    // 4J_ij from the exact FP32 copy when there is one (half the bytes per gather)
    if (lay.J4f) pairs(lay.J4f + lay.joff[b]);
    else pairs(lay.J4 + lay.joff[b]);
    if (nst > 0) flush();
    // the list and the stage are rewritten by this wave's next state
    wave_sync();
    return r;
}

// Host launchers (defined next to their kernels).
hipError_t launch_init_fields(const Layout& lay, const uint64_t* d_x0, hipStream_t st);
hipError_t launch_fields_for(const Layout& lay, int search, int count, hipStream_t st);
hipError_t launch_frontier_plan(const Layout& lay, hipStream_t st);
hipError_t launch_plan_only(const Layout& lay, hipStream_t st);      // re-plan without counting
hipError_t launch_clear_survivors(const Layout& lay, hipStream_t st);
// after_bound, if given, is recorded once the site-bound kernel is queued
hipError_t launch_prep(const Layout& lay, hipStream_t st, bool count = true, hipEvent_t after_bound = nullptr);
hipError_t launch_scan(const Layout& lay, int scan_grid, hipStream_t st);
hipError_t launch_merge(const Layout& lay, hipStream_t st);
hipError_t launch_fupdate(const Layout& lay, hipStream_t st);
hipError_t launch_init_split(const Layout& lay, const uint64_t* d_x0, double* d_maxerr, hipStream_t st);
hipError_t launch_prep32(const Layout& lay, hipStream_t st);
hipError_t launch_scan32(const Layout& lay, int scan_grid, hipStream_t st);
hipError_t launch_step_begin(const Layout& lay, bool retry_mode, hipStream_t st);
hipError_t launch_learn(const Layout& lay, int grid, hipStream_t st);
hipError_t learn_set_lds(size_t bytes);
hipError_t frontier_set_lds(const Layout& lay);
size_t learn_lds_bytes(const Layout& lay);
hipError_t launch_trace(const Layout& lay, hipStream_t st);
// training of the scoring network (device pointers; partial = workspace)
int mlp_grid_for(long long count);
hipError_t launch_mlp_grad(const float* P, const float* X, const uint8_t* y, long long n, long long count,
                           uint64_t seed, int step, float pos_w, float* partial, int grid, hipStream_t st);
hipError_t launch_mlp_reduce(const float* partial, int grid, float* grad, float* loss, hipStream_t st);
hipError_t launch_mlp_adam(float* P, float* m, float* v, const float* g, float lr, float b1, float b2, float eps,
                           float c1, float c2, hipStream_t st);
hipError_t launch_mlp_forward(const float* P, const float* X, long long n, float* z, hipStream_t st);
hipError_t launch_final(const Layout& lay, hipStream_t st);
hipError_t launch_graph_begin(const Layout& lay, hipStream_t st);
hipError_t launch_step_end(const Layout& lay, int t, hipStream_t st);

// ------------------------------------------------------------------ exhaustive enumeration (k_brute.hip)
constexpr int BF_NL = 8;                 // low sites walked in Gray order by one thread
constexpr int BF_DSTRIDE = 1 << BF_NL;   // table entries per instance
constexpr int BF_CAP = 8192;             // records per instance collected for the final sort
constexpr int BF_KMAX = 4096;            // lowest states returned per instance at most
constexpr int BF_NMAX = 40;              // 2^N states, one 64-bit word each
enum { BF_MIN = 0, BF_COUNT = 1, BF_COLLECT = 2 };

struct BruteRec {
    double E;
    uint64_t psi;
};
static_assert(sizeof(BruteRec) == 16, "record layout");

// All instances of one size N; instance b of the group at J + b*N*N, h + b*N.
struct BruteArgs {
    int N;
    int n_list;                  // instances processed by this launch
    const int* list;             // [n_list] their indices in the group
    const double* J;             // [nb][N][N] couplings J_ij (symmetric, zero diagonal)
    const double* h;             // [nb][N]
    double* D;                   // [nb][BF_DSTRIDE] Gray-walk table of the low sites
    const double* T;             // [nb] thresholds (count and collect passes)
    unsigned long long* emin;    // [nb] order-preserving image of the lowest energy
    unsigned long long* count;   // [nb] states counted or collected
    BruteRec* rec;               // [nb][BF_CAP]
};

int brute_low_sites(int N);
hipError_t launch_brute_table(const BruteArgs& a, hipStream_t st);
hipError_t launch_brute_pass(const BruteArgs& a, int mode, hipStream_t st);
hipError_t brute_sort_set_lds();
hipError_t launch_brute_sort(const BruteArgs& a, int K, uint64_t* out_bits, double* out_E, int* out_n,
                             hipStream_t st);

}  // namespace qi

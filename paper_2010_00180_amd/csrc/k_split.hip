// Split-bf16 form of the scan.  The local fields of the initial states are
// also formed on the bf16 matrix cores with 4J = hi + lo split into two bf16
// parts (the +-1 spins are exact in bf16) and FP32 accumulation; the pair
// scan runs in FP32 against a threshold that carries a proven error slack; and
// every pair it admits is re-scored in FP64 before it can enter, so the kept
// sets are the same as in the FP64 form.  The FP64 steps are the re-scoring,
// the singles, the pilot cut and the incremental field updates.
#include "common.h"

namespace qi {

__device__ inline uint32_t lane_id32() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ inline uint32_t mbcnt64s(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// A value the whole wave holds alike, moved to scalar registers.
__device__ inline uint32_t uniform_u32(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }

__device__ inline uint64_t uniform_u64(uint64_t v)
{
    return ((uint64_t)uniform_u32((uint32_t)(v >> 32)) << 32) | uniform_u32((uint32_t)v);
}

// Word k of a state held one word per lane (lane k), as a wave-uniform value.
__device__ inline uint64_t lane_word(uint64_t xw, int k)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)xw, k);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(xw >> 32), k);
    return ((uint64_t)hi << 32) | lo;
}

// blocks of 64 sites whose loads a preparation wave issues together
constexpr int PREP_CH = 8;

// ------------------------------------------------------------------ bf16 hi+lo GEMM
// One wave: 16 sites x 16 searches of acc = (hi + lo) * S with
// v_mfma_f32_16x16x32_bf16 (lane l: A rows l%16, k = 8*(l/16)..+7; B columns
// l%16, same k; D rows 4*(l/16)+r, column l%16), then F~ = h + acc/4.
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(64) void k_init_split(Layout lay, const uint64_t* __restrict__ x0)
{
    const int b = blockIdx.x;
    const int N = lay.N[b], Np = lay.Npad[b];
    const int row0 = blockIdx.y * 16, col0 = blockIdx.z * 16;
    if (row0 >= Np || col0 >= lay.L) return;
    const int lane = threadIdx.x;
    const uint16_t* hi = lay.Jhi + lay.joff[b];
    const uint16_t* lo = lay.Jlo + lay.joff[b];
    const int ai = row0 + (lane & 15);
    const int kq = 8 * (lane >> 4);
    const int lj = col0 + (lane & 15);
    const bool colok = lj < lay.L;
    const uint64_t* xs = x0 + (size_t)(b * lay.L + (colok ? lj : 0)) * lay.Wmax;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < Np; k0 += 32) {
        v8bf ah, al, bs;
        const uint16_t* ph = hi + (size_t)ai * Np + k0 + kq;
        const uint16_t* pl = lo + (size_t)ai * Np + k0 + kq;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            ah[e] = __builtin_bit_cast(__bf16, ph[e]);
            al[e] = __builtin_bit_cast(__bf16, pl[e]);
            const int k = k0 + kq + e;
            uint16_t sb = 0;   // 0.0
            if (colok && k < N) sb = ((xs[k >> 6] >> (k & 63)) & 1ull) ? (uint16_t)0xBF80 : (uint16_t)0x3F80;
            bs[e] = __builtin_bit_cast(__bf16, sb);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bs, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bs, acc, 0, 0, 0);
    }
    if (!colok) return;
    const int s = b * lay.L + lj;
    const double* h = lay.h + (size_t)b * lay.Npmax;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int site = row0 + 4 * (lane >> 4) + r;
        if (site < Np) lay.Ft[(size_t)s * lay.Npmax + site] = site < N ? (float)h[site] + 0.25f * acc[r] : 0.f;
    }
}

// max |F~ - F| over the initial states, as an ordered bit pattern (non-negative doubles)
__global__ __launch_bounds__(256) void k_split_err(Layout lay, unsigned long long* out)
{
    const int s = blockIdx.x;
    const int b = s / lay.L;
    const int N = lay.N[b];
    const FieldRow F = field_row(lay, (size_t)s * 2 * lay.M, b);   // slot 0
    const float* Ft = lay.Ft + (size_t)s * lay.Npmax;
    double m = 0.0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) m = fmax(m, fabs((double)Ft[i] - F[i]));
    atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

hipError_t launch_init_split(const Layout& lay, const uint64_t* d_x0, double* d_maxerr, hipStream_t st)
{
    dim3 grid(lay.B, (lay.Npmax + 15) / 16, (lay.L + 15) / 16);
    hipLaunchKernelGGL(k_init_split, grid, dim3(64), 0, st, lay, d_x0);
    hipLaunchKernelGGL(k_split_err, dim3(lay.S), dim3(256), 0, st, lay,
                       reinterpret_cast<unsigned long long*>(d_maxerr));
    return hipGetLastError();
}

// ------------------------------------------------------------------ k_prep32
// As the FP64 preparation, and also: fl32(a_i) for the FP32 scan (in the
// first step from F~ of the bf16 GEMM) and the FP32 threshold
// RR_i = round_up(T - a_i + delta), with delta = 4u (max|4J| + A)
// (+ 2 max|F~ - F| in the first step), u = 2^-24, where A bounds |a| over
// every state of the instance (the proof needs only an upper bound).  Then every pair with
// a_i + a_j + s_i s_j 4J_ij <= T also has fl32(fma(s_i, s_j fl32(4J_ij), fl32(a_j))) <= RR_i.
__device__ inline double wave_max(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ inline int find_inst(const long long* prefix, int B, long long e)
{
    int lo = 0, hi = B;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

// An FP16 value at or above x that has no FP16 value between it and x (the
// smallest one, except that a result of zero is +0).  The hardware conversions
// to FP32 (to nearest) and on to FP16 (toward zero) land on one of the two FP16
// values around x, as both are FP32 values and each rounding stays between
// them; the one below x is moved up a step.  The same value as rounding up to
// FP32 and then up to FP16, as every FP16 value is an FP32 value.
__device__ inline _Float16 half_up(double x)
{
    const float xf = (float)x;
    uint32_t u = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(xf, xf)) & 0xFFFFu;
    if ((double)__builtin_bit_cast(_Float16, (uint16_t)u) < x) u = (u & 0x8000u) ? u - 1u : u + 1u;
    if (u == 0x8000u) u = 0;   // -0 as +0: an admission test reads the sign of RR_i - x
    return __builtin_bit_cast(_Float16, (uint16_t)u);
}

template <bool SB, bool H16>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_prep32(Layout lay, const long long* __restrict__ fr_prefix)
{
    if (step_halted(lay)) return;   // a later step of a multi-step graph after a halt
    const long long total = fr_prefix[lay.B];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63;
    const int retry_mode = lay.flags[FLAG_RETRY_MODE];
    const int first = lay.flags[FLAG_FIRST];
    // XCD x (blocks x, x + 8, ...) takes the x-th contiguous eighth of the
    // entries, so the states it prepares at once share one L2 for their
    // couplings
    const int nx = gridDim.x >= 8 ? 8 : 1;
    const int xcd = blockIdx.x % nx;
    const long long seg1 = total * (xcd + 1) / nx;
    const long long stride = (long long)(gridDim.x / nx) * 4;
    int b = -1;   // instance of entry e: found once, then advanced (e only grows)
    for (long long e = total * xcd / nx + (long long)(blockIdx.x / nx) * 4 + wave; e < seg1; e += stride) {
        if (b < 0) b = find_inst(fr_prefix, lay.B, e);
        while (fr_prefix[b + 1] <= e) ++b;
        const int f = (int)(e - fr_prefix[b]);
        const size_t fe = (size_t)b * lay.fmax + f;
        // site bound: the states k_site_bound evaluated need nothing here
        if (SB && lay.fr_bound[fe] != 0) continue;
        const int code = lay.fr_list[fe];
        const int s = code / (2 * lay.M);
        if (retry_mode && !lay.retry[s]) continue;
        const size_t q = (size_t)code;
        const int N = lay.N[b], Np = lay.Npad[b];
        const double Em = lay.E[q];
        const double c = lay.cut[s];
        const double T = c - Em;
        const uint64_t* x = lay.bits + q * lay.Wmax;
        const FieldRow F = field_row(lay, q, b);
        const bool from_ft = first && (code % (2 * lay.M)) == 0;
        const float* Ft = lay.Ft + (size_t)s * lay.Npmax;
        double* A = lay.A + fe * lay.Npmax;
        float* A32 = lay.A32 + fe * lay.Npmax;
        float* RR = lay.RR32 + fe * lay.Npmax;
        if (lane == 0) {
            FrRec r;
            r.T = T;
            r.E = Em;
            r.s = s;
            r.code = code;
            lay.rec[fe] = r;
        }
        // lane w holds word w of the state (at most 64 words)
        const uint64_t xw = (int)lane < lay.Wmax ? x[lane] : 0ull;
        if ((int)lane < lay.Wmax) lay.fbits[fe * lay.Wmax + lane] = xw;
        if (retry_mode && lane == 0) {
            // with the site bound the pairs are counted once the entries are sorted out
            if (!lay.sb) atomicAdd(&lay.ctr[CTR_PAIRS], (unsigned long long)N * (N - 1) / 2);
            atomicAdd(&lay.ctr[CTR_SINGLES], (unsigned long long)N);
        }
        // slack of the FP32 threshold, from the instance's bound on |a|
        const double u = 5.9604644775390625e-08;   // 2^-24
        double delta = 4.0 * u * (lay.ybound[b] + lay.abound[b]) + (from_ft ? 2.0 * lay.ebf[b] : 0.0);
        if (H16) {
            // packed FP16 scan: the row holds fl16(a_j), and the slack covers FP16
            // rounding of a_j, of 4J_ij and of the fma, each at most 2^-11 of its
            // magnitude (2^-25 absolute below the normal range), with the
            // instance's bound on |a|
            const double u16 = 4.8828125e-04;   // 2^-11
            delta = 2.01 * u16 * (lay.ybound[b] + lay.abound[b]) + 2.384185791015625e-07 +
                    (from_ft ? 2.0 * lay.ebf[b] : 0.0);
        }
        _Float16* A16 = reinterpret_cast<_Float16*>(A32);
        // rounds of CH blocks of 64 sites: the loads of a round are issued
        // together, so that the wave waits on memory once per round.  Without
        // the site bound the rounds are shorter: their fewer registers let more
        // waves share a SIMD, which hides more of the latency than longer
        // rounds save
        constexpr int CH = SB ? PREP_CH : 6;
        for (int i0 = 0; i0 < Np; i0 += 64 * CH) {
            // blocks past Np load the last block again (unused), so that every
            // load is unconditional and in bounds
            double Fv[CH];
            float Ftv[CH];
            F.gather(Fv, [&](int r) { return min(i0 + 64 * r, Np - 64) + (int)lane; });
            if (from_ft) {
#pragma unroll
                for (int r = 0; r < CH; ++r) Ftv[r] = Ft[min(i0 + 64 * r, Np - 64) + (int)lane];
            }
            // a_i and the thresholds; the single flips below the cut are counted,
            // so that one atomic reserves their places for the round
            double ar[CH];
            int nhit = 0;
#pragma unroll
            for (int r = 0; r < CH; ++r) {
                const int ib = i0 + 64 * r;
                ar[r] = 0.0;
                if (ib < Np) {
                    const int i = ib + (int)lane;
                    // the word of sites ib .. ib+63 is the lane mask of the flipped spins
                    const bool neg = __builtin_amdgcn_inverse_ballot_w64(lane_word(xw, ib >> 6));
                    const double sp = neg ? -1.0 : 1.0;
                    const double a = i < N ? -2.0 * sp * Fv[r] : 0.0;
                    ar[r] = a;
                    if (lay.tr_feat) A[i] = a;   // FP64 a is read back only by trace capture
                    const double av = i < N ? (from_ft ? -2.0 * sp * (double)Ftv[r] : a) : 0.0;
                    if (H16) A16[i] = i < N ? (_Float16)av : (_Float16)INFINITY;   // padding: no pair can pass
                    else A32[i] = (float)av;
                    if (H16) reinterpret_cast<_Float16*>(RR)[i] = i < N ? half_up(T - a + delta) : (_Float16)-INFINITY;
                    else RR[i] = i < N ? __double2float_ru(T - a + delta) : -INFINITY;
                    nhit += __builtin_popcountll(__builtin_amdgcn_ballot_w64(i < N && Em + a <= c));
                }
            }
            if (H16 && i0 + 64 * CH >= Np) {
                // the FP16 scan reads whole 128-column tiles: +inf past Np as well
                for (int i = Np + (int)lane; i < ((Np + 127) & ~127); i += 64) A16[i] = (_Float16)INFINITY;
            }
            if (nhit) {
                int base = 0;
                if (lane == 0) base = atomicAdd(&lay.surv_count[s], nhit);
                base = __shfl(base, 0, 64);
#pragma unroll
                for (int r = 0; r < CH; ++r) {
                    const int i = i0 + 64 * r + (int)lane;
                    const double Ec = Em + ar[r];
                    const bool hit = i < N && Ec <= c;
                    const uint64_t m = __builtin_amdgcn_ballot_w64(hit);
                    if (m) {
                        if (hit) {
                            const int pos = base + (int)mbcnt64s(m);
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

// ------------------------------------------------------------------ k_scan32
// One wave per (instance, chunk of states, 64 x 64 tile with row block <= column
// block).  Lane = row i; registers hold y_j = s_j fl32(4J_ij) for 64 columns
// (column signs re-applied per group of 8 when they change between states);
// per pair one v_fma_f32 and one v_min_f32, one compare per group against
// RR_i.  Admitted pairs are queued in LDS and re-scored in FP64 (a_i + a_j +
// s_i s_j 4J_ij against T, all exact) a wave's worth at a time, so the global
// reads of the re-score overlap; only then are they recorded, and the rest are
// counted.
constexpr int T32 = 64;

__device__ inline void flush32(const Layout& lay, Surv* stage, int& n, int s)
{
    if (n == 0) return;
    __syncthreads();
    int base = 0;
    if (lane_id32() == 0) base = atomicAdd(&lay.surv_count[s], n);
    base = __shfl(base, 0, 64);
    for (int k = (int)lane_id32(); k < n; k += 64) {
        const int pos = base + k;
        if (pos < lay.cap_surv) lay.surv[(size_t)s * lay.cap_surv + pos] = stage[k];
    }
    __syncthreads();
    n = 0;
}

// At most 128 VGPRs, so that four waves share each SIMD: the loop is bound by
// latency, and occupancy decides its speed.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_scan32(Layout lay, const float* __restrict__ J32,
                                               const double* __restrict__ J4,
                                               const float* __restrict__ A32,
                                               const float* __restrict__ RR32,
                                               const FrRec* __restrict__ recs,
                                               const uint64_t* __restrict__ fbits,
                                               const long long* __restrict__ iprefix)
{
    if (step_halted(lay)) return;   // a later step of a multi-step graph after a halt
    __shared__ Surv stage[STAGE];
    __shared__ float abuf[T32];   // a_j of the current state
    __shared__ double sT[64], sE[64];
    __shared__ int sCode[64];
    // per state, what the loop over states reads: one address for all of it
    struct StRec {
        uint64_t wi, wj;   // words of the tile's rows and columns
        uint32_t s;        // search
        uint32_t fe;       // entry index: below 2^32, as the FP64 rows of every entry fit in memory
    };
    __shared__ StRec srec[64];
    constexpr int PEND = 640;
    __shared__ uint32_t pend[PEND];   // admitted pairs awaiting the FP64 re-score: k << 12 | row << 6 | col
    const uint32_t lane = lane_id32();
    const long long total = iprefix[lay.B];
    const int retry_mode = lay.flags[FLAG_RETRY_MODE];
    const int Wm = lay.Wmax;
    const int Npm = lay.Npmax;
    const int nx = gridDim.x >= 8 ? 8 : 1;
    const int xcd = blockIdx.x % nx;
    const long long seg0 = total * xcd / nx, seg1 = total * (xcd + 1) / nx;
    const long long stride = gridDim.x / nx;
    unsigned long long rejected = 0;
    for (long long item = seg0 + blockIdx.x / nx; item < seg1; item += stride) {
        const int b = __builtin_amdgcn_readfirstlane(find_inst(iprefix, lay.B, item));
        const long long r = item - iprefix[b];
        const int N = lay.N[b], Np = lay.Npad[b];
        const int nb = Np / TILE;
        const long long T = tiles64(N);
        const int c = (int)(r / T);
        int t = (int)(r % T);
        int bi = 0;
        while (t >= nb - bi) { t -= nb - bi; ++bi; }
        bi = __builtin_amdgcn_readfirstlane(bi);
        const int bj = __builtin_amdgcn_readfirstlane(bi + t);
        const int P = lay.sb ? lay.full_count[b] : lay.fr_count[b];
        const int sc = lay.scb[b];
        const int f0 = c * sc;
        const int f1 = min(f0 + sc, P);
        const size_t fb = (size_t)b * lay.fmax;
        const int row = bi * TILE + (int)lane;
        const int col0 = bj * T32;
        const float* Jt = J32 + lay.joff[b];
        uint32_t Jb[T32];
#pragma unroll
        for (int j = 0; j < T32; ++j) {
            const int col = col0 + j;
            const float v = Jt[(size_t)col * Np + row];
            const bool ok = row < N && col < N && col > row;
            Jb[j] = ok ? __float_as_uint(v) : 0x7FC00000u;
        }
        uint64_t prev_wj = 0;
        int nstage = 0, sstage = -1;
        int npend = 0;
        // exact FP64 re-score of the admitted pairs, survivors to the stage
        auto rescore = [&]() {
            for (int p0 = 0; p0 < npend; p0 += 64) {
                const int p = p0 + (int)lane;
                bool keep = false;
                Surv rec;
                rec.E = 0.0;
                rec.code = 0;
                rec.pair = 0;
                if (p < npend) {
                    const uint32_t pr = pend[p];
                    const int k = (int)(pr >> 12), rl = (int)((pr >> 6) & 63u), cl = (int)(pr & 63u);
                    const int prow = bi * TILE + rl, pcol = col0 + cl;
                    const int cd = sCode[k];
                    const FieldRow Frow = field_row(lay, (size_t)cd, b);
                    const double sid = ((srec[k].wi >> rl) & 1ull) ? -1.0 : 1.0;
                    const double sj = ((srec[k].wj >> cl) & 1ull) ? -1.0 : 1.0;
                    const double ai = -2.0 * sid * Frow[prow];
                    const double x = -2.0 * sj * Frow[pcol] + sid * sj * J4[lay.joff[b] + (size_t)prow * Np + pcol];
                    keep = ai + x <= sT[k];
                    if (!keep) ++rejected;
                    rec.E = (sE[k] + ai) + x;
                    rec.code = (uint32_t)cd;
                    rec.pair = (uint32_t)prow | ((uint32_t)pcol << 16);
                }
                const uint64_t m = __builtin_amdgcn_ballot_w64(keep);
                if (m) {
                    if (nstage > STAGE - 64) flush32(lay, stage, nstage, sstage);
                    if (keep) stage[nstage + (int)mbcnt64s(m)] = rec;
                    nstage += __builtin_popcountll(m);
                }
            }
            npend = 0;
        };
        for (int g0 = f0; g0 < f1; g0 += 64) {
            const int ns = min(64, f1 - g0);
            // the records of states g0 .. g0+ns-1 (with the site bound, the
            // entries left to the scan)
            if ((int)lane < ns) {
                const size_t fe = fb + (lay.sb ? lay.full_list[fb + g0 + lane] : g0 + (int)lane);
                const FrRec rc = recs[fe];
                sT[lane] = rc.T;
                sE[lane] = rc.E;
                sCode[lane] = rc.code;
                const uint64_t* fw = fbits + fe * Wm;
                StRec sr;
                sr.wi = fw[bi];
                sr.wj = fw[bj];
                sr.s = (uint32_t)rc.s;
                sr.fe = (uint32_t)fe;
                srec[lane] = sr;
            }
            __syncthreads();
            const size_t fe0 = (size_t)uniform_u32(srec[0].fe) * Npm;
            float nrr = RR32[fe0 + row];
            float naj = A32[fe0 + col0 + lane];
            abuf[lane] = naj;
            __syncthreads();
            for (int k = 0; k < ns; ++k) {
                const float rrt = nrr;
                if (k + 1 < ns) {
                    const size_t fn = (size_t)uniform_u32(srec[k + 1].fe) * Npm;
                    nrr = RR32[fn + row];
                    naj = A32[fn + col0 + lane];
                }
                const StRec cur = srec[k];
                const int s = (int)uniform_u32(cur.s);
                const bool skip = retry_mode && !lay.retry[s];
                if (!skip) {
                    if (s != sstage) {
                        rescore();
                        flush32(lay, stage, nstage, sstage);
                        sstage = s;
                    }
                    // the row bits of the state are the lane mask of the negative s_i
                    const float si = __builtin_amdgcn_inverse_ballot_w64(uniform_u64(cur.wi)) ? -1.f : 1.f;
                    const uint64_t wj = uniform_u64(cur.wj);
                    const uint64_t dw = wj ^ prev_wj;
                    prev_wj = wj;
                    const float* aj = abuf;
                    float a8n[8];   // the next group's a_j, read one group ahead
#pragma unroll
                    for (int u = 0; u < 8; ++u) a8n[u] = aj[u];
#pragma unroll
                    for (int g = 0; g < T32; g += 8) {
                        float a8[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u) a8[u] = a8n[u];
                        if (g + 8 < T32) {
#pragma unroll
                            for (int u = 0; u < 8; ++u) a8n[u] = aj[g + 8 + u];
                        }
                        if ((dw >> g) & 0xFFull) {
#pragma unroll
                            for (int u = 0; u < 8; ++u) Jb[g + u] ^= (uint32_t)((dw >> (g + u)) & 1ull) << 31;
                        }
                        float mn0 = fmaf(si, __uint_as_float(Jb[g]), a8[0]);
                        float mn1 = fmaf(si, __uint_as_float(Jb[g + 1]), a8[1]);
#pragma unroll
                        for (int u = 2; u < 8; ++u) {
                            const float x = fmaf(si, __uint_as_float(Jb[g + u]), a8[u]);
                            if (u & 1) mn1 = fminf(mn1, x);
                            else mn0 = fminf(mn0, x);
                        }
                        if (__builtin_amdgcn_ballot_w64(fminf(mn0, mn1) <= rrt)) {
                            // admitted pairs wait for the exact re-score: a mask of the lane's
                            // 8 columns, then rounds that queue each lane's lowest admitted
                            // column (admitted pairs are sparse: usually one round)
                            uint32_t am = 0;
#pragma unroll
                            for (int u = 0; u < 8; ++u)
                                am |= (fmaf(si, __uint_as_float(Jb[g + u]), a8[u]) <= rrt ? 1u : 0u) << u;
                            for (uint64_t m = __builtin_amdgcn_ballot_w64(am != 0); m;
                                 m = __builtin_amdgcn_ballot_w64(am != 0)) {
                                if (npend > PEND - 64) rescore();
                                if (am) {
                                    pend[npend + (int)mbcnt64s(m)] = ((uint32_t)k << 12) | (lane << 6) |
                                                                     (uint32_t)(g + __builtin_ctz(am));
                                    am &= am - 1u;
                                }
                                npend += __builtin_popcountll(m);
                            }
                        }
                    }
                }
                // one wave: its LDS accesses complete in order, so the next row can
                // replace this one once its reads are issued
                if (k + 1 < ns) abuf[lane] = naj;
                __syncthreads();
            }
            rescore();   // before the next 64 states replace the records
        }
        flush32(lay, stage, nstage, sstage);
        __syncthreads();
    }
    // count re-scored pairs that the exact test rejected
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)rejected, off, 64);
        const uint32_t hi = __shfl_xor((uint32_t)(rejected >> 32), off, 64);
        rejected += ((uint64_t)hi << 32) | lo;
    }
    if (lane == 0 && rejected) atomicAdd(&lay.ctr[CTR_FALLBACK], rejected);
}

// ------------------------------------------------------------------ k_scan16
// The split scan in packed FP16 (on request): one wave per (instance, chunk of
// states, tile of 64 rows x 128 columns with some column above the rows).
// Lane = row i; 64 registers hold y_j = s_j fl16(4J_ij) for 128 columns as
// pairs; per group of 16 columns eight v_pk_fma_f16, four v_pk_minimum3_f16 and
// one compare against RR_i rounded up to FP16.  RR_i carries the FP16
// slack; admitted pairs are queued and re-scored in FP64 as in k_scan32.
typedef _Float16 h2v __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_scan16(Layout lay, const uint16_t* __restrict__ J16,
                                               const double* __restrict__ J4,
                                               const uint16_t* __restrict__ A16,
                                               const _Float16* __restrict__ RR16,
                                               const FrRec* __restrict__ recs,
                                               const uint64_t* __restrict__ fbits,
                                               const long long* __restrict__ iprefix)
{
    if (step_halted(lay)) return;   // a later step of a multi-step graph after a halt
    __shared__ Surv stage[STAGE];
    __shared__ uint32_t abuf[T16 / 2];   // fl16(a_j) pairs of the current state
    __shared__ double sT[64], sE[64];
    __shared__ int sCode[64];
    // per state, what the loop over states reads: one address for all of it
    struct StRec {
        uint64_t wi, wj0, wj1;   // words of the tile's rows and columns
        uint32_t s;              // search
        uint32_t fe;             // entry index: below 2^32, as the FP64 rows of every entry fit in memory
    };
    __shared__ StRec srec[64];
    constexpr int PEND = 512;
    __shared__ uint32_t pend[PEND];   // admitted pairs awaiting the FP64 re-score: k << 13 | row << 7 | col
    const uint32_t lane = lane_id32();
    const long long total = iprefix[lay.B];
    const int retry_mode = lay.flags[FLAG_RETRY_MODE];
    const int Wm = lay.Wmax;
    const int Npm = lay.Npmax;
    const int nx = gridDim.x >= 8 ? 8 : 1;
    const int xcd = blockIdx.x % nx;
    const long long seg0 = total * xcd / nx, seg1 = total * (xcd + 1) / nx;
    const long long stride = gridDim.x / nx;
    unsigned long long rejected = 0;
    for (long long item = seg0 + blockIdx.x / nx; item < seg1; item += stride) {
        const int b = __builtin_amdgcn_readfirstlane(find_inst(iprefix, lay.B, item));
        const long long r = item - iprefix[b];
        const int N = lay.N[b], Np = lay.Npad[b];
        const int nb = Np / TILE, nc = (Np + T16 - 1) / T16;
        const long long T = tiles16(N);
        const int c = (int)(r / T);
        int t = (int)(r % T);
        int bi = 0;
        while (t >= nc - (bi >> 1)) { t -= nc - (bi >> 1); ++bi; }
        bi = __builtin_amdgcn_readfirstlane(bi);
        const int bj = __builtin_amdgcn_readfirstlane((bi >> 1) + t);
        const int P = lay.sb ? lay.full_count[b] : lay.fr_count[b];
        const int sc = lay.scb[b];
        const int f0 = c * sc;
        const int f1 = min(f0 + sc, P);
        const size_t fb = (size_t)b * lay.fmax;
        const int row = bi * TILE + (int)lane;
        const int col0 = bj * T16;
        // groups of 16 columns with a pair in the triangle (the others are skipped)
        uint32_t live = 0;
        for (int g = 0; g < T16 / 2; g += 8)
            if (col0 + 2 * g < N && col0 + 2 * g + 15 > bi * TILE) live |= 1u << (g >> 3);
        live = (uint32_t)__builtin_amdgcn_readfirstlane((int)live);
        if (!live) continue;
        const int w0 = 2 * bj, w1 = 2 * bj + 1 < Wm ? 2 * bj + 1 : -1;   // words of the tile's columns
        // row i of the (symmetric) couplings, four columns per 8-byte load;
        // columns at or past Np are not read.  No entry is NaN, so that a
        // NaN-propagating three-way minimum can reduce them: rows and columns
        // at or past N hold 0 (such a row's threshold is -inf, such a column's
        // a_j is +inf); the diagonal holds +inf, which the column-sign tracking
        // turns into s_i inf, so that its product with s_i is +inf; below the
        // diagonal the couplings stay (each such pair is also met above it) and
        // the admission step drops them.
        const uint64_t* Jrow = reinterpret_cast<const uint64_t*>(J16 + lay.joff[b] + (size_t)row * Np);
        uint32_t Jb[T16 / 2];   // columns col0 + 2v (low half) and col0 + 2v + 1 (high half)
#pragma unroll
        for (int q = 0; q < T16 / 4; ++q) {
            const int c4 = col0 + 4 * q;
            uint64_t v = (row < N && c4 < Np) ? Jrow[c4 >> 2] : 0ull;
#pragma unroll
            for (int h = 0; h < 4; ++h)
                if (row < N && c4 + h == row) v = (v & ~(0xFFFFull << (16 * h))) | (0x7C00ull << (16 * h));
            Jb[2 * q] = (uint32_t)v;
            Jb[2 * q + 1] = (uint32_t)(v >> 32);
        }
        (void)nb;
        uint64_t prev0 = 0, prev1 = 0;
        int nstage = 0, sstage = -1;
        int npend = 0;
        // exact FP64 re-score of the admitted pairs, survivors to the stage
        auto rescore = [&]() {
            for (int p0 = 0; p0 < npend; p0 += 64) {
                const int p = p0 + (int)lane;
                bool keep = false;
                Surv rec;
                rec.E = 0.0;
                rec.code = 0;
                rec.pair = 0;
                if (p < npend) {
                    const uint32_t pr = pend[p];
                    const int k = (int)(pr >> 13), rl = (int)((pr >> 7) & 63u), cl = (int)(pr & 127u);
                    const int prow = bi * TILE + rl, pcol = col0 + cl;
                    const int cd = sCode[k];
                    const FieldRow Frow = field_row(lay, (size_t)cd, b);
                    const double sid = ((srec[k].wi >> rl) & 1ull) ? -1.0 : 1.0;
                    const uint64_t wj = cl < 64 ? srec[k].wj0 : srec[k].wj1;
                    const double sj = ((wj >> (cl & 63)) & 1ull) ? -1.0 : 1.0;
                    const double ai = -2.0 * sid * Frow[prow];
                    const double x = -2.0 * sj * Frow[pcol] + sid * sj * J4[lay.joff[b] + (size_t)prow * Np + pcol];
                    keep = ai + x <= sT[k];
                    if (!keep) ++rejected;
                    rec.E = (sE[k] + ai) + x;
                    rec.code = (uint32_t)cd;
                    rec.pair = (uint32_t)prow | ((uint32_t)pcol << 16);
                }
                const uint64_t m = __builtin_amdgcn_ballot_w64(keep);
                if (m) {
                    if (nstage > STAGE - 64) flush32(lay, stage, nstage, sstage);
                    if (keep) stage[nstage + (int)mbcnt64s(m)] = rec;
                    nstage += __builtin_popcountll(m);
                }
            }
            npend = 0;
        };
        for (int g0 = f0; g0 < f1; g0 += 64) {
            const int ns = min(64, f1 - g0);
            // the records of states g0 .. g0+ns-1 (with the site bound, the
            // entries left to the scan)
            if ((int)lane < ns) {
                const size_t fe = fb + (lay.sb ? lay.full_list[fb + g0 + lane] : g0 + (int)lane);
                const FrRec rc = recs[fe];
                sT[lane] = rc.T;
                sE[lane] = rc.E;
                sCode[lane] = rc.code;
                const uint64_t* fw = fbits + fe * Wm;
                StRec sr;
                sr.wi = fw[bi];
                sr.wj0 = fw[w0];
                sr.wj1 = w1 >= 0 ? fw[w1] : 0ull;
                sr.s = (uint32_t)rc.s;
                sr.fe = (uint32_t)fe;
                srec[lane] = sr;
            }
            __syncthreads();
            // a row of state k: 2 Npmax halves per entry; the tile reads halves
            // col0 .. col0+127 < Np + 64 <= 2 Npmax
            const uint32_t* A0 = reinterpret_cast<const uint32_t*>(A16);
            const size_t fe0 = (size_t)uniform_u32(srec[0].fe) * Npm;
            _Float16 nrr = RR16[2 * fe0 + row];   // rows of 2 Npmax halves
            uint32_t naj = A0[fe0 + (col0 >> 1) + lane];
            abuf[lane] = naj;
            __syncthreads();
            for (int k = 0; k < ns; ++k) {
                const _Float16 rr = nrr;
                if (k + 1 < ns) {
                    const size_t fn = (size_t)uniform_u32(srec[k + 1].fe) * Npm;
                    nrr = RR16[2 * fn + row];
                    naj = A0[fn + (col0 >> 1) + lane];
                }
                const StRec cur = srec[k];
                const int s = (int)uniform_u32(cur.s);
                const bool skip = retry_mode && !lay.retry[s];
                if (!skip) {
                    if (s != sstage) {
                        rescore();
                        flush32(lay, stage, nstage, sstage);
                        sstage = s;
                    }
                    // s_i for both halves (-1 or +1 in FP16): the row bits of the state
                    // are the lane mask of the negative ones
                    const h2v si2 = __builtin_bit_cast(
                        h2v, __builtin_amdgcn_inverse_ballot_w64(uniform_u64(cur.wi)) ? 0xBC00BC00u : 0x3C003C00u);
                    const uint64_t wj[2] = {uniform_u64(cur.wj0), uniform_u64(cur.wj1)};
                    const uint64_t dw[2] = {wj[0] ^ prev0, wj[1] ^ prev1};
                    prev0 = wj[0];
                    prev1 = wj[1];
                    const uint32_t* aj = abuf;
                    uint32_t a8n[8];   // the next group's a_j pairs, read one group ahead
#pragma unroll
                    for (int u = 0; u < 8; ++u) a8n[u] = aj[u];
#pragma unroll
                    for (int g = 0; g < T16 / 2; g += 8) {
                        // group: registers g .. g+7, columns col0 + 2g .. col0 + 2g + 15
                        uint32_t a8[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u) a8[u] = a8n[u];
                        if (g + 8 < T16 / 2) {
#pragma unroll
                            for (int u = 0; u < 8; ++u) a8n[u] = aj[g + 8 + u];
                        }
                        if (!((live >> (g >> 3)) & 1u)) continue;
                        const uint64_t dwg = dw[g >> 5] >> ((2 * g) & 63);
                        if (dwg & 0xFFFFull) {
#pragma unroll
                            for (int u = 0; u < 8; ++u) {
                                // the two sign bits of the pair, formed in one scalar register
                                // (bit 0 of the 2-bit field to bit 15, bit 1 to bit 31, by one
                                // multiply) so that the flip is a single vector op
                                const uint32_t fl = (uint32_t)__builtin_amdgcn_readfirstlane(
                                    (int)(((((uint32_t)dwg >> (2 * u)) & 3u) * 0x40008000u) & 0x80008000u));
                                Jb[g + u] ^= fl;
                            }
                        }
                        auto xf = [&](int u) {
                            return __builtin_elementwise_fma(si2, __builtin_bit_cast(h2v, Jb[g + u]),
                                                             __builtin_bit_cast(h2v, a8[u]));
                        };
                        // three-way minima (v_pk_minimum3_f16): four for the 16 columns
                        const h2v m1 = __builtin_elementwise_minimum(__builtin_elementwise_minimum(xf(0), xf(1)), xf(2));
                        const h2v m2 = __builtin_elementwise_minimum(__builtin_elementwise_minimum(xf(3), xf(4)), xf(5));
                        const h2v m3 = __builtin_elementwise_minimum(__builtin_elementwise_minimum(xf(6), xf(7)), m1);
                        const h2v mm = __builtin_elementwise_minimum(m2, m3);
                        const bool any = mm[0] <= rr || mm[1] <= rr;
                        if (__builtin_amdgcn_ballot_w64(any)) {
                            // admitted pairs wait for the exact re-score.  The lane's admitted
                            // columns come from the signs of RR_i - x_ij (exact: +0 when equal),
                            // gathered by byte permutes into a 16-bit mask in which bit 8b + q
                            // stands for column 4q + b of the group
                            const h2v rr2 = {rr, rr};
                            uint32_t d[8];
#pragma unroll
                            for (int u = 0; u < 8; ++u) d[u] = __builtin_bit_cast(uint32_t, rr2 - xf(u));
                            uint32_t t = 0;
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                // high bytes of both halves of d[2q] and d[2q+1]: columns 4q .. 4q+3
                                const uint32_t sb = __builtin_amdgcn_perm(d[2 * q + 1], d[2 * q], 0x07050301u);
                                t |= (sb >> (7 - q)) & (0x01010101u << q);
                            }
                            uint32_t am = ~t & 0x0F0F0F0Fu;
                            // columns at or below the row (the diagonal block) or at or past N
                            // are not pairs; the empty asm keeps this rare step from being
                            // hoisted out of the loop over states
                            int rw = row;
                            asm volatile("" : "+v"(rw));
                            const int lo = rw - (col0 + 2 * g) + 1, hi = N - (col0 + 2 * g);
                            // each round queues the lowest admitted column of every lane that
                            // has one (admitted pairs are sparse: usually one round)
                            for (uint64_t m = __builtin_amdgcn_ballot_w64(am != 0); m;
                                 m = __builtin_amdgcn_ballot_w64(am != 0)) {
                                if (npend > PEND - 64) rescore();
                                int j = -1;
                                if (am) {
                                    const int p = __builtin_ctz(am);
                                    am &= am - 1u;
                                    j = 4 * (p & 7) + (p >> 3);
                                    if (j < lo || j >= hi) j = -1;
                                }
                                const uint64_t w = __builtin_amdgcn_ballot_w64(j >= 0);
                                if (j >= 0)
                                    pend[npend + (int)mbcnt64s(w)] = ((uint32_t)k << 13) | (lane << 7) | (uint32_t)(2 * g + j);
                                npend += __builtin_popcountll(w);
                            }
                        }
                    }
                }
                // one wave: its LDS accesses complete in order, so the next row can
                // replace this one once its reads are issued
                if (k + 1 < ns) abuf[lane] = naj;
                __syncthreads();
            }
            rescore();   // before the next 64 states replace the records
        }
        flush32(lay, stage, nstage, sstage);
        __syncthreads();
    }
    // count re-scored pairs that the exact test rejected
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)rejected, off, 64);
        const uint32_t hi = __shfl_xor((uint32_t)(rejected >> 32), off, 64);
        rejected += ((uint64_t)hi << 32) | lo;
    }
    if (lane == 0 && rejected) atomicAdd(&lay.ctr[CTR_FALLBACK], rejected);
}

// Work prefix over instances for the 64 x 128 tiles of the FP16 scan.
__global__ __launch_bounds__(1024) void k_plan16(Layout lay, long long* __restrict__ iprefix)
{
    if (step_halted(lay)) return;   // a later step of a multi-step graph after a halt
    __shared__ long long part[1024];
    const int t = threadIdx.x;
    const int per = (lay.B + 1023) / 1024;
    const int b0 = t * per;
    long long items = 0;
    for (int b = b0; b < b0 + per && b < lay.B; ++b) {
        const long long P = lay.sb ? lay.full_count[b] : lay.fr_count[b];
        items += (P + lay.scb[b] - 1) / lay.scb[b] * tiles16(lay.N[b]);
    }
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
        iprefix[b] = run;
        const long long P = lay.sb ? lay.full_count[b] : lay.fr_count[b];
        run += (P + lay.scb[b] - 1) / lay.scb[b] * tiles16(lay.N[b]);
    }
    if (t == 1023) iprefix[lay.B] = part[1023];
}

// ------------------------------------------------------------------ k_plan32
// Work prefix over instances for the 64 x 64 tiles of the FP32 scan.
__global__ __launch_bounds__(1024) void k_plan32(Layout lay, long long* __restrict__ iprefix)
{
    if (step_halted(lay)) return;   // a later step of a multi-step graph after a halt
    __shared__ long long part[1024];
    const int t = threadIdx.x;
    const int per = (lay.B + 1023) / 1024;
    const int b0 = t * per;
    long long items = 0;
    for (int b = b0; b < b0 + per && b < lay.B; ++b) {
        const long long P = lay.sb ? lay.full_count[b] : lay.fr_count[b];
        items += (P + lay.scb[b] - 1) / lay.scb[b] * tiles64(lay.N[b]);
    }
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
        iprefix[b] = run;
        const long long P = lay.sb ? lay.full_count[b] : lay.fr_count[b];
        run += (P + lay.scb[b] - 1) / lay.scb[b] * tiles64(lay.N[b]);
    }
    if (t == 1023) iprefix[lay.B] = part[1023];
}

hipError_t launch_prep32(const Layout& lay, hipStream_t st)
{
    const long long* fr_prefix = lay.item_prefix + (lay.B + 1);
    if (lay.sb && lay.h16) hipLaunchKernelGGL((k_prep32<true, true>), dim3(4096), dim3(256), 0, st, lay, fr_prefix);
    else if (lay.sb) hipLaunchKernelGGL((k_prep32<true, false>), dim3(4096), dim3(256), 0, st, lay, fr_prefix);
    else if (lay.h16) hipLaunchKernelGGL((k_prep32<false, true>), dim3(4096), dim3(256), 0, st, lay, fr_prefix);
    else hipLaunchKernelGGL((k_prep32<false, false>), dim3(4096), dim3(256), 0, st, lay, fr_prefix);
    return hipGetLastError();
}

hipError_t launch_scan32(const Layout& lay, int scan_grid, hipStream_t st)
{
    long long* iprefix = lay.item_prefix + 2 * (lay.B + 1);
    if (lay.h16) {
        hipLaunchKernelGGL(k_plan16, dim3(1), dim3(1024), 0, st, lay, iprefix);
        hipLaunchKernelGGL(k_scan16, dim3(scan_grid), dim3(64), 0, st, lay, lay.J16, lay.J4,
                           (const uint16_t*)lay.A32, (const _Float16*)lay.RR32,
                           (const FrRec*)lay.rec, (const uint64_t*)lay.fbits, (const long long*)iprefix);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_plan32, dim3(1), dim3(1024), 0, st, lay, iprefix);
    hipLaunchKernelGGL(k_scan32, dim3(scan_grid), dim3(64), 0, st, lay, lay.J32, lay.J4, (const float*)lay.A32,
                       (const float*)lay.RR32, (const FrRec*)lay.rec,
                       (const uint64_t*)lay.fbits, (const long long*)iprefix);
    return hipGetLastError();
}

}  // namespace qi

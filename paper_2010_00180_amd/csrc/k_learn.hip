// Learned-proposal form (not in the paper, whose own lever for a cheaper
// search is a smaller H1).  For every ranked frontier state a small network
// scores all N(N-1)/2 pair flips from the features
//   (f_i, f_j, sqrt(N) J_ij, s_i s_j),   f_i = s_i F_i = -a_i / 2,
// the K = topk * N best are evaluated exactly in FP64 (a_i + a_j + s_i s_j 4J_ij,
// the same energy change as the full scan) and filtered by the step's cut.
// The single flips of ranked states are offered here too, under the same
// per-state bound (below).
//
// k_learn: one block (4 waves) per ranked state.  A wave scores four blocks of
// 16 pairs (row i, columns j..j+15) per pass, one block per lane group, with
// the network on the bf16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// accumulation), per block:
//   layer 1  4 MFMAs: rows = 64 hidden units, K = 8 feature slots
//            (f_i, f_j, Jn, ss, 1 for the bias, zeros), columns = 16 pairs
//   layer 2  8 MFMAs: 64 x 64, the bias in the accumulator
//   output   2 MFMAs: row 0 = w3, the bias in the accumulator
// The D layout of one layer (lane l holds rows 4(l/16)+r, column l%16) is the
// next layer's B operand after relu and rounding to bf16, once the hidden
// index is permuted: logical k = 8q + t of K-step kk is hidden unit
// 32 kk + 16 (t/4) + 4q + t%4.  The weight operands carry the same permutation.
// Scores become 64-bit keys (ordered score, ~pair code: ties go to the smaller
// code); keys above a block-wide threshold are appended to an LDS buffer, and
// when it fills, a radix select (8-bit digits) finds the K-th largest key,
// which becomes the threshold, and the K best are compacted through a
// per-block global buffer.
//
// k_trace: (features, label) samples for training, from the states expanded
// in a step once its merge has committed.
#include "common.h"

namespace qi {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));


__device__ inline uint32_t lr_lane() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ inline uint32_t lr_mbcnt(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// finaliser of splitmix64 (Steele, Lea and Flood)
__device__ inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ inline uint32_t ord_score(float z)
{
    if (!(z == z)) return 0u;   // NaN ranks last
    const uint32_t u = __float_as_uint(z);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ inline __bf16 bfb(uint16_t u) { return __builtin_bit_cast(__bf16, u); }

typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

// two floats to one packed bf16 pair (one v_cvt_pk_bf16_f32, nearest even)
__device__ inline unsigned int pack_bf16(float a, float b)
{
    const v2f f = {a, b};
    return __builtin_bit_cast(unsigned int, __builtin_convertvector(f, v2bf));
}

__device__ inline v8bf relu_pack(v4f a, v4f b)
{
    const v4u u = {pack_bf16(a[0], a[1]), pack_bf16(a[2], a[3]), pack_bf16(b[0], b[1]), pack_bf16(b[2], b[3])};
    // relu on the bf16 bit patterns: a set sign bit is a negative int16
    v8s s = __builtin_bit_cast(v8s, u);
    const v8s zero = {0, 0, 0, 0, 0, 0, 0, 0};
    s = __builtin_elementwise_max(s, zero);
    return __builtin_bit_cast(v8bf, s);
}

// The network's operands, laid out so that one pass scores four blocks of 16
// pairs: lane group q (lanes 16q .. 16q+15) holds the features of block q in
// K slots 8q .. 8q+7, so layer 1 of block q uses a copy of W1 placed in those
// slots (a1[q]), and the output of block q is written to row 4q (a3[q]),
// which is register 0 of lane group q.
struct Net {
    v8bf a1[4][4];   // [q][m]: rows 16m .. 16m+15 of (W1 | b1), in lane group q
    v8bf a2[4][2];   // [output tile][K-step], hidden index permuted
    v4f c2[4];       // b2 in the accumulator layout
    v8bf a3[4][2];   // [q][K-step]: w3 in row 4q
    v4f c3;          // b3 in register 0 of every lane
};

// bf16 copies (nearest even) of the parameters in this lane's registers.
__device__ inline void load_net(const float* __restrict__ P, Net& n)
{
    const int l = (int)(lr_lane() & 63u), g = l >> 4, r = l & 15;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                float v = 0.f;
                if (g == q && t < 4) v = P[MLP_W1 + (16 * m + r) * 4 + t];
                if (g == q && t == 4) v = P[MLP_B1 + 16 * m + r];
                n.a1[q][m][t] = (__bf16)v;
            }
        }
    }
#pragma unroll
    for (int o = 0; o < 4; ++o) {
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
#pragma unroll
            for (int t = 0; t < 8; ++t)
                n.a2[o][kk][t] = (__bf16)P[MLP_W2 + (16 * o + r) * MLP_H + 32 * kk + 16 * (t >> 2) + 4 * g + (t & 3)];
        }
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) n.c2[o][rr] = P[MLP_B2 + 16 * o + 4 * g + rr];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const float w = P[MLP_W3 + 32 * kk + 16 * (t >> 2) + 4 * g + (t & 3)];
                n.a3[q][kk][t] = (__bf16)(r == 4 * q ? w : 0.f);
            }
        }
    }
    n.c3[0] = P[MLP_B3];
    n.c3[1] = 0.f;
    n.c3[2] = 0.f;
    n.c3[3] = 0.f;
}

// Logits of four blocks: lane l gets the logit of pair l%16 of block l/16.
__device__ inline float net_score4(const Net& n, v8bf x)
{
    const v4f z4 = {0.f, 0.f, 0.f, 0.f};
    const int g = (int)(lr_lane() & 63u) >> 4;
    float z = 0.f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const v4f d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(n.a1[q][0], x, z4, 0, 0, 0);
        const v4f d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(n.a1[q][1], x, z4, 0, 0, 0);
        const v4f d2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(n.a1[q][2], x, z4, 0, 0, 0);
        const v4f d3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(n.a1[q][3], x, z4, 0, 0, 0);
        const v8bf h0 = relu_pack(d0, d1), h1 = relu_pack(d2, d3);
        v4f e[4];
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            e[o] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(n.a2[o][0], h0, n.c2[o], 0, 0, 0);
            e[o] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(n.a2[o][1], h1, e[o], 0, 0, 0);
        }
        const v8bf g0 = relu_pack(e[0], e[1]), g1 = relu_pack(e[2], e[3]);
        v4f out = __builtin_amdgcn_mfma_f32_16x16x32_bf16(n.a3[q][0], g0, n.c3, 0, 0, 0);
        out = __builtin_amdgcn_mfma_f32_16x16x32_bf16(n.a3[q][1], g1, out, 0, 0, 0);
        z = g == q ? out[0] : z;
    }
    return z;
}

struct LrShared {
    int cnt, cnt2, d, rank, cntd;
    unsigned long long thr, kth, dmax;
    double red[LR_WAVES];
};

// doubles as unsigned integers in the same order
__device__ inline unsigned long long ord_double(double v)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__device__ inline double unord_double(unsigned long long u)
{
    return __longlong_as_double((long long)((u >> 63) ? (u & 0x7FFFFFFFFFFFFFFFull) : ~u));
}

__device__ inline double lr_block_min(double v, LrShared& sh)
{
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) sh.red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = sh.red[0];
    for (int w = 1; w < LR_WAVES; ++w) r = fmin(r, sh.red[w]);
    __syncthreads();
    return r;
}

__device__ inline double lr_block_max(double v, LrShared& sh)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) sh.red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = sh.red[0];
    for (int w = 1; w < LR_WAVES; ++w) r = fmax(r, sh.red[w]);
    __syncthreads();
    return r;
}

// Keep the K largest of cand[0..cnt) (cnt > K, keys distinct): radix select of
// the K-th largest key, then compaction through gtmp.  Sets cnt = K and the
// threshold to the K-th key.  Called by the whole block.
__device__ void lr_select(uint64_t* cand, int cnt, int K, uint64_t* __restrict__ gtmp, int* hist, LrShared& sh)
{
    const int tid = threadIdx.x;
    uint64_t prefix = 0, pmask = 0;
    int rank = K;
    bool unique = false;
    for (int shift = 56;; shift -= 8) {
        for (int d = tid; d < 256; d += blockDim.x) hist[d] = 0;
        __syncthreads();
        for (int e = tid; e < cnt; e += blockDim.x) {
            const uint64_t k = cand[e];
            if ((k & pmask) == prefix) atomicAdd(&hist[(int)((k >> shift) & 255u)], 1);
        }
        __syncthreads();
        if (tid < 64) {
            // lane l holds digits 255-4l .. 252-4l (largest first)
            const int l = tid;
            int c[4], loc = 0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                c[u] = hist[255 - 4 * l - u];
                loc += c[u];
            }
            int incl = loc;
            for (int off = 1; off < 64; off <<= 1) {
                const int v = __shfl_up(incl, off, 64);
                if (l >= off) incl += v;
            }
            int run = incl - loc;
            if (run < rank && rank <= incl) {
                for (int u = 0; u < 4; ++u) {
                    if (run + c[u] >= rank) {
                        sh.d = 255 - 4 * l - u;
                        sh.rank = rank - run;
                        sh.cntd = c[u];
                        break;
                    }
                    run += c[u];
                }
            }
        }
        __syncthreads();
        prefix |= (uint64_t)sh.d << shift;
        pmask |= 0xFFull << shift;
        rank = sh.rank;
        if (shift == 0) break;
        if (sh.cntd == 1) {
            unique = true;
            break;
        }
    }
    if (unique) {
        for (int e = tid; e < cnt; e += blockDim.x)
            if ((cand[e] & pmask) == prefix) sh.kth = cand[e];
    } else if (tid == 0) {
        sh.kth = prefix;
    }
    if (tid == 0) sh.cnt2 = 0;
    __syncthreads();
    const uint64_t kth = sh.kth;
    for (int e = tid; e < cnt; e += blockDim.x) {
        const uint64_t k = cand[e];
        if (k >= kth) {
            const int pos = atomicAdd(&sh.cnt2, 1);
            if (pos < K) gtmp[pos] = k;
        }
    }
    __syncthreads();
    for (int e = tid; e < K; e += blockDim.x) cand[e] = gtmp[e];
    if (tid == 0) {
        sh.cnt = K;
        sh.thr = kth;
    }
    __syncthreads();
}

__device__ inline int lr_find(const long long* prefix, int B, long long e)
{
    int lo = 0, hi = B;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_learn(Layout lay)
{
    if (step_halted(lay)) return;   // a later step of a multi-step graph after a halt
    extern __shared__ __align__(16) unsigned char lr_smem[];
    __shared__ LrShared sh;
    __shared__ int hist[256];
    uint64_t* cand = reinterpret_cast<uint64_t*>(lr_smem);
    uint64_t* sbits = cand + lay.cap_lr;
    uint16_t* f16s = reinterpret_cast<uint16_t*>(sbits + lay.Wmax);
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const uint32_t lane = (uint32_t)tid & 63u;
    const long long* lr_prefix = lay.item_prefix + 3 * (lay.B + 1);
    const long long total = lr_prefix[lay.B];
    const int retry_mode = lay.flags[FLAG_RETRY_MODE];
    uint64_t* gtmp = lay.lr_tmp + (size_t)blockIdx.x * lay.kmax;
    Net net;
    if (lay.scorer == 0) load_net(lay.mlp, net);
    for (long long e = blockIdx.x; e < total; e += gridDim.x) {
        const int b = lr_find(lr_prefix, lay.B, e);
        const int kq = (int)(e - lr_prefix[b]);
        const size_t fe = (size_t)b * lay.fmax + (size_t)(lay.fmax - lay.lr_count[b] + kq);
        const FrRec rc = lay.rec[fe];
        const int s = rc.s;
        if (retry_mode && !lay.retry[s]) continue;
        const int N = lay.N[b], Np = lay.Npad[b];
        const int W = words_of(N);
        const double* A = lay.A + fe * lay.Npmax;
        const long long npairs = (long long)N * (N - 1) / 2;
        const long long kl = (long long)lay.topk * N;
        const int K = (int)(kl < npairs ? kl : npairs);
        for (int w = tid; w < W; w += blockDim.x) sbits[w] = lay.fbits[fe * lay.Wmax + w];
        for (int i = tid; i < N; i += blockDim.x)
            f16s[i] = __builtin_bit_cast(uint16_t, (__bf16)(float)(-0.5 * A[i]));
        if (tid == 0) {
            sh.cnt = 0;
            sh.thr = 0;
        }
        __syncthreads();

        // blocks of 16 pairs: row i, columns j0 .. j0+15 (j0 = i+1, i+17, ...)
        const long long n1 = N - 1;
        const long long a16 = n1 / 16, rem = n1 % 16;
        const long long NB = n1 > 0 ? 8 * a16 * (a16 + 1) + rem * (a16 + 1) : 0;
        const long long rounds = (NB + (long long)LR_WAVES * LR_R - 1) / ((long long)LR_WAVES * LR_R);
        int gi = 0, gj = 1;   // this wave's block: the wave-th of the row-major block list
        for (int u = 0; u < wave; ++u) {
            gj += 16;
            if (gj >= N) { ++gi; gj = gi + 1; }
        }
        const uint64_t zp = lay.zob[rc.code] ^ lay.seed;
        const uint16_t* Jn = lay.Jn16 + lay.joff[b];
        for (long long r = 0; r < rounds; ++r) {
            const uint64_t thr = sh.thr;
            for (int u = 0; u < LR_R; u += 4) {
                // this wave's next four blocks, one per lane group
                const long long g0 = (long long)LR_WAVES * (r * LR_R + u) + wave;
                if (g0 >= NB) break;
                int bi[4], bj[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    bi[q] = gi;
                    bj[q] = gj;
                    for (int v = 0; v < LR_WAVES; ++v) {
                        gj += 16;
                        if (gj >= N) { ++gi; gj = gi + 1; }
                    }
                }
                const int q = (int)(lane >> 4);
                const bool inblk = g0 + (long long)LR_WAVES * q < NB;
                int mgi = q == 0 ? bi[0] : q == 1 ? bi[1] : q == 2 ? bi[2] : bi[3];
                int mgj = q == 0 ? bj[0] : q == 1 ? bj[1] : q == 2 ? bj[2] : bj[3];
                if (!inblk) { mgi = 0; mgj = 1; }   // in range; its keys are dropped
                const int j = mgj + (int)(lane & 15u);
                const bool valid = inblk && j < N;
                const int jc = j < N ? j : N - 1;
                const int ic = mgi < N ? mgi : 0;
                const uint32_t code = (uint32_t)ic | ((uint32_t)jc << 16);
                float z;
                if (lay.scorer == 0) {
                    const bool neg = (((sbits[ic >> 6] >> (ic & 63)) ^ (sbits[jc >> 6] >> (jc & 63))) & 1ull) != 0;
                    const __bf16 zb = bfb(0);
                    v8bf x;
                    x[0] = bfb(f16s[ic]);
                    x[1] = bfb(f16s[jc]);
                    x[2] = bfb(Jn[(size_t)ic * Np + jc]);
                    x[3] = bfb(neg ? (uint16_t)0xBF80 : (uint16_t)0x3F80);
                    x[4] = bfb(0x3F80);
                    x[5] = zb;
                    x[6] = zb;
                    x[7] = zb;
                    z = net_score4(net, x);
                } else if (lay.scorer == 1) {
                    z = (float)(-0.5 * (A[ic] + A[jc]));
                } else {
                    z = (float)(mix64(zp + 0x9E3779B97F4A7C15ull * ((uint64_t)code + 1ull)) >> 40) *
                        5.9604644775390625e-08f;
                }
                const uint64_t key = valid ? (((uint64_t)ord_score(z) << 32) | (uint64_t)(~code)) : 0ull;
                const bool pass = key > thr;
                const uint64_t m = __builtin_amdgcn_ballot_w64(pass);
                if (m) {
                    int base = 0;
                    if (lane == 0) base = atomicAdd(&sh.cnt, __popcll(m));
                    base = __shfl(base, 0, 64);
                    if (pass) cand[base + (int)lr_mbcnt(m)] = key;
                }
            }
            __syncthreads();
            if (sh.cnt > lay.cap_lr - LR_ROOM) lr_select(cand, sh.cnt, K, gtmp, hist, sh);
        }
        if (sh.cnt > K) lr_select(cand, sh.cnt, K, gtmp, hist, sh);
        const int nfin = sh.cnt;

        // exact FP64 energy change of the proposals (kept in gtmp), and the
        // state's own bound: its N single flips and nfin proposals are distinct
        // states, so when there are at least M of them, the M-th lowest of their
        // energy changes bounds the search's M-th lowest candidate, and nothing
        // of this state above it can enter.  The bound is taken as the largest
        // change in the lowest histogram bins that hold M of them.
        const double* Jb = lay.J4 + lay.joff[b];
        double dlo = INFINITY, dhi = -INFINITY;
        for (int ee = tid; ee < nfin; ee += blockDim.x) {
            const uint32_t code = ~(uint32_t)cand[ee];
            const int i = (int)(code & 0xFFFFu), j = (int)(code >> 16);
            const bool neg = (((sbits[i >> 6] >> (i & 63)) ^ (sbits[j >> 6] >> (j & 63))) & 1ull) != 0;
            const double y = Jb[(size_t)i * Np + j];
            const double dE = A[i] + A[j] + (neg ? -y : y);
            reinterpret_cast<double*>(gtmp)[ee] = dE;
            dlo = fmin(dlo, dE);
            dhi = fmax(dhi, dE);
        }
        for (int i = tid; i < N; i += blockDim.x) {
            dlo = fmin(dlo, A[i]);
            dhi = fmax(dhi, A[i]);
        }
        const int ncand = nfin + N;
        double Tl = rc.T;
        if (ncand >= lay.M) {
            dlo = lr_block_min(dlo, sh);
            dhi = lr_block_max(dhi, sh);
            const double scale = dhi > dlo ? 256.0 / (dhi - dlo) : 0.0;
            auto bin_of = [&](double v) -> int {
                const int k = (int)((v - dlo) * scale);
                return k < 0 ? 0 : (k > 255 ? 255 : k);
            };
            for (int d = tid; d < 256; d += blockDim.x) hist[d] = 0;
            if (tid == 0) sh.dmax = 0ull;
            __syncthreads();
            for (int ee = tid; ee < nfin; ee += blockDim.x)
                atomicAdd(&hist[bin_of(reinterpret_cast<const double*>(gtmp)[ee])], 1);
            for (int i = tid; i < N; i += blockDim.x) atomicAdd(&hist[bin_of(A[i])], 1);
            __syncthreads();
            if (tid < 64) {
                // lane l holds bins 4l .. 4l+3 (lowest first)
                const int l = tid;
                int c[4], loc = 0;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    c[u] = hist[4 * l + u];
                    loc += c[u];
                }
                int incl = loc;
                for (int off = 1; off < 64; off <<= 1) {
                    const int v = __shfl_up(incl, off, 64);
                    if (l >= off) incl += v;
                }
                int run = incl - loc;
                if (run < lay.M && lay.M <= incl) {
                    for (int u = 0; u < 4; ++u) {
                        run += c[u];
                        if (run >= lay.M) {
                            sh.d = 4 * l + u;
                            break;
                        }
                    }
                }
            }
            __syncthreads();
            const int bstar = sh.d;
            for (int ee = tid; ee < nfin; ee += blockDim.x) {
                const double v = reinterpret_cast<const double*>(gtmp)[ee];
                if (bin_of(v) <= bstar) atomicMax(&sh.dmax, ord_double(v));
            }
            for (int i = tid; i < N; i += blockDim.x)
                if (bin_of(A[i]) <= bstar) atomicMax(&sh.dmax, ord_double(A[i]));
            __syncthreads();
            const double bound = unord_double(sh.dmax);
            Tl = bound < Tl ? bound : Tl;
        }
        // survivors: single flips, then the proposals
        for (int e0 = 0; e0 < ncand; e0 += blockDim.x) {
            const int ee = e0 + tid;
            bool hit = false;
            double dE = 0.0;
            uint32_t code = 0;
            if (ee < N) {
                dE = A[ee];
                code = (uint32_t)ee | (SINGLE << 16);
                hit = dE <= Tl;
            } else if (ee < ncand) {
                const int k = ee - N;
                dE = reinterpret_cast<const double*>(gtmp)[k];
                code = ~(uint32_t)cand[k];
                hit = dE <= Tl;
                if (lay.prop) lay.prop[fe * lay.kmax + k] = code;
            }
            const uint64_t m = __builtin_amdgcn_ballot_w64(hit);
            if (m) {
                int base = 0;
                if (lane == 0) base = atomicAdd(&lay.surv_count[s], __popcll(m));
                base = __shfl(base, 0, 64);
                if (hit) {
                    const int pos = base + (int)lr_mbcnt(m);
                    if (pos < lay.cap_surv) {
                        Surv rr;
                        rr.E = rc.E + dE;
                        rr.code = (uint32_t)rc.code;
                        rr.pair = code;
                        lay.surv[(size_t)s * lay.cap_surv + pos] = rr;
                    }
                }
            }
        }
        if (lay.prop && tid == 0) lay.prop_n[fe] = nfin;
        __syncthreads();
    }
}

size_t learn_lds_bytes(const Layout& lay)
{
    return (size_t)lay.cap_lr * 8 + (size_t)lay.Wmax * 8 + (size_t)lay.Npmax * 2;
}

hipError_t learn_set_lds(size_t bytes)
{
    return hipFuncSetAttribute(reinterpret_cast<const void*>(k_learn), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

hipError_t launch_learn(const Layout& lay, int grid, hipStream_t st)
{
    hipLaunchKernelGGL(k_learn, dim3(grid), dim3(256), learn_lds_bytes(lay), st, lay);
    return hipGetLastError();
}

// ------------------------------------------------------------------ k_trace
// One wave per prepared entry of a committed search, traced with probability
// tr_rate: one sample per pair flip of this parent that entered the kept set
// (label 1) and tr_neg uniformly drawn pairs i < j labelled by membership of
// the child among the new kept states (exact energy, then the Zobrist hash).
__global__ __launch_bounds__(256) void k_trace(Layout lay, const long long* __restrict__ fr_prefix)
{
    if (step_halted(lay)) return;   // a later step of a multi-step graph after a halt
    const long long total = fr_prefix[lay.B];
    const int wave = threadIdx.x >> 6;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t salt = (uint64_t)lay.ctr[CTR_STEPS] * 0x9E3779B97F4A7C15ull;
    const int M = lay.M;
    for (long long e = (long long)blockIdx.x * 4 + wave; e < total; e += (long long)gridDim.x * 4) {
        const int b = lr_find(fr_prefix, lay.B, e);
        const int f = (int)(e - fr_prefix[b]);
        const int P = lay.fr_count[b];
        const size_t fe = (size_t)b * lay.fmax + (f >= P ? lay.fmax - lay.lr_count[b] + (f - P) : f);
        const FrRec rc = lay.rec[fe];
        const int s = rc.s;
        if (lay.retry[s]) continue;   // the merge of this search did not commit
        const uint64_t hsel = mix64(lay.seed ^ salt ^ ((uint64_t)(uint32_t)rc.code << 17));
        if ((float)(hsel >> 40) * 5.9604644775390625e-08f >= lay.tr_rate) continue;
        const int N = lay.N[b], Np = lay.Npad[b];
        if (N < 2) continue;
        const double* A = lay.A + fe * lay.Npmax;
        const uint64_t* x = lay.fbits + fe * lay.Wmax;
        const double* Jb = lay.J4 + lay.joff[b];
        const double sq = sqrt((double)N);
        const size_t q0 = (size_t)s * 2 * M;
        const int nk = lay.nkept[s];
        const int* kept = lay.kept + (size_t)s * M;
        auto emit = [&](bool on, int i, int j, bool label) {
            const uint64_t m = __builtin_amdgcn_ballot_w64(on);
            if (!m) return;
            unsigned long long base = 0;
            if (lane == 0) base = atomicAdd(&lay.ctr[CTR_TRACE], (unsigned long long)__popcll(m));
            base = __shfl(base, 0, 64);
            if (!on) return;
            const unsigned long long pos = base + lr_mbcnt(m);
            if (pos >= (unsigned long long)lay.tr_cap) return;
            const bool neg = (((x[i >> 6] >> (i & 63)) ^ (x[j >> 6] >> (j & 63))) & 1ull) != 0;
            float* o = lay.tr_feat + pos * 4;
            o[0] = (float)(-0.5 * A[i]);
            o[1] = (float)(-0.5 * A[j]);
            o[2] = (float)(sq * (0.25 * Jb[(size_t)i * Np + j]));
            o[3] = neg ? -1.f : 1.f;
            lay.tr_label[pos] = label ? 1 : 0;
        };
        // pair flips of this parent that entered
        const int nm = lay.nm_count[s];
        for (int m0 = 0; m0 < nm; m0 += 64) {
            const int m = m0 + (int)lane;
            bool on = false;
            int i = 0, j = 1;
            if (m < nm && lay.nm_code[(size_t)s * M + m] == rc.code) {
                const uint32_t pr = lay.nm_pair[(size_t)s * M + m];
                if ((pr >> 16) != SINGLE) {
                    on = true;
                    i = (int)(pr & 0xFFFFu);
                    j = (int)(pr >> 16);
                }
            }
            emit(on, i, j, true);
        }
        // uniformly drawn pairs, labelled by membership
        for (int r0 = 0; r0 < lay.tr_neg; r0 += 64) {
            const int r = r0 + (int)lane;
            const bool on = r < lay.tr_neg;
            const uint64_t u = mix64(hsel + 0x632BE59BD9B4E019ull * (uint64_t)(r + 1));
            int i = (int)((u & 0xFFFFFFFFull) % (uint64_t)N);
            int j = (int)((u >> 32) % (uint64_t)(N - 1));
            if (j >= i) ++j;
            if (i > j) { const int t = i; i = j; j = t; }
            const bool neg = (((x[i >> 6] >> (i & 63)) ^ (x[j >> 6] >> (j & 63))) & 1ull) != 0;
            const double y = Jb[(size_t)i * Np + j];
            const double Ec = rc.E + A[i] + A[j] + (neg ? -y : y);
            const uint64_t zc = lay.zob[rc.code] ^ lay.zkey[i] ^ lay.zkey[j];
            int lo = 0, hi = nk;   // first kept index with E >= Ec
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (lay.E[q0 + kept[mid]] < Ec) lo = mid + 1; else hi = mid;
            }
            bool in = false;
            for (int k = lo; k < nk && lay.E[q0 + kept[k]] == Ec; ++k) {
                const int slot = kept[k];
                if (lay.zob[q0 + slot] == zc && lay.fresh[q0 + slot]) in = true;
            }
            emit(on, i, j, in);
        }
    }
}

hipError_t launch_trace(const Layout& lay, hipStream_t st)
{
    const long long* fr_prefix = lay.item_prefix + (lay.B + 1);
    hipLaunchKernelGGL(k_trace, dim3(1024), dim3(256), 0, st, lay, fr_prefix);
    return hipGetLastError();
}

}  // namespace qi

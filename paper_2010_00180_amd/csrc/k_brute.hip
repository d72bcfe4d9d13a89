// Exhaustive enumeration of all 2^N states of small instances: the paper's
// brute-force reference (Sec. IV, Fig. 1) and the source of the exact
// low-energy spectra of Sec. V (ground energy, gap, k-th lowest energies).
//
// Thread layout.  The N sites split into NL low sites and N - NL high sites.
// One thread owns the 2^NL states that share its high bits (its prefix) and
// visits them in Gray-code order, one low spin flip per state.  With the low
// part y and the prefix fixed,
//     E(y) = E_high + sum_{i<NL} s_i C_i + E_low(y),
//     C_i = h_i + sum_{l>=NL} J_il s_l            (per thread, constant),
//     E_low(y) = sum_{i<j<NL} J_ij s_i s_j        (the same for every thread),
// so flipping low spin i changes the energy by -2 s_i C_i + D_g, where
// D_g = E_low(y_g) - E_low(y_{g-1}) is a table of 2^NL - 1 values per instance.
// The walk is unrolled at compile time: the flipped site, its spin before the
// flip and the table offset are constants, so a state costs two FP64 adds plus
// what the pass does with its energy.  Every value is on the 2^-24 grid, so all
// energies are exact and independent of the order of the sums.
//
// One wave serves one instance (instance = wave / waves per instance), so the
// instance's couplings and table are read with scalar loads.
//
// Passes (all instances of one N at once):
//   BF_MIN      lowest energy per instance;
//   BF_COUNT    number of states with E <= T_b;
//   BF_COLLECT  every state with E <= T_b appended to the instance's buffer;
// then k_brute_sort puts each buffer in (E, psi) order in LDS and writes the
// K first.  The host picks T_b with K <= count <= BF_CAP.
#include "common.h"

namespace qi {

namespace {

__device__ inline unsigned long long ord_of(double v)
{
    const unsigned long long u = __double_as_longlong(v);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__device__ inline double val_of(unsigned long long o)
{
    const unsigned long long u = (o >> 63) ? (o & 0x7FFFFFFFFFFFFFFFull) : ~o;
    return __longlong_as_double((long long)u);
}

struct Visit {
    double emin;
    unsigned cnt;
    double T;
};

template <int MODE>
__device__ __forceinline__ void visit(Visit& v, double E, uint64_t psi)
{
    if constexpr (MODE == BF_MIN) {
        v.emin = fmin(v.emin, E);
    } else if constexpr (MODE == BF_COUNT) {
        v.cnt += (E <= v.T) ? 1u : 0u;
    }
}

// steps G .. END-1 of the Gray walk over the NL low sites
template <int NL, int MODE, int G, int END>
__device__ __forceinline__ void walk(Visit& v, double& E, const double (&C2)[NL > 0 ? NL : 1],
                                     const double* __restrict__ D, uint64_t prefix)
{
    if constexpr (G < END) {
        constexpr int i = __builtin_ctz(G);
        constexpr int yprev = (G - 1) ^ ((G - 1) >> 1);
        constexpr bool down = ((yprev >> i) & 1) != 0;   // s_i = -1 before the flip
        E += down ? C2[i] : -C2[i];
        E += D[G];
        visit<MODE>(v, E, prefix | (uint64_t)(G ^ (G >> 1)));
        walk<NL, MODE, G + 1, END>(v, E, C2, D, prefix);
    }
}

// Energy of the thread's first state (low spins all +1) and 2 C_i of its low sites.
template <int NL>
__device__ __forceinline__ double brute_start(const double* __restrict__ J, const double* __restrict__ h,
                                              const double* __restrict__ D, int N, uint64_t prefix, double* C2)
{
    double E = D[0];   // E_low(0)
    for (int i = 0; i < NL; ++i) {
        double c = h[i];
        for (int l = NL; l < N; ++l) c += J[i * N + l] * (((prefix >> l) & 1) ? -1.0 : 1.0);
        E += c;
        C2[i] = 2.0 * c;
    }
    for (int i = NL; i < N; ++i) {
        const double si = ((prefix >> i) & 1) ? -1.0 : 1.0;
        double r = h[i];
        for (int l = i + 1; l < N; ++l) r += J[i * N + l] * (((prefix >> l) & 1) ? -1.0 : 1.0);
        E += si * r;
    }
    return E;
}

// The minimum and count passes: the walk unrolled at compile time.
template <int NL, int MODE>
__global__ __launch_bounds__(256) void k_brute(BruteArgs a)
{
    const long long wave = (long long)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int N = a.N;
    const long long per_inst = 1ll << (N - NL);                     // threads per instance
    const long long wpi = (per_inst + 63) >> 6;                     // waves per instance
    const int k = (int)(wave / wpi);
    if (k >= a.n_list) return;
    const int b = a.list[k];
    const long long t = (wave - k * wpi) * 64 + lane;              // prefix of this thread
    const bool live = t < per_inst;
    const double* __restrict__ J = a.J + (size_t)b * N * N;
    const double* __restrict__ h = a.h + (size_t)b * N;
    const double* __restrict__ D = a.D + (size_t)b * BF_DSTRIDE;
    const uint64_t prefix = (uint64_t)(live ? t : 0) << NL;

    double C2[NL > 0 ? NL : 1];
    double E = brute_start<NL>(J, h, D, N, prefix, C2);

    Visit v;
    v.emin = __builtin_inf();
    v.cnt = 0;
    v.T = a.T ? a.T[b] : 0.0;
    if (!live) E = __builtin_nan("");   // a lane past the instance's states: no compare passes, fmin skips it
    visit<MODE>(v, E, prefix);
    walk<NL, MODE, 1, (1 << NL)>(v, E, C2, D, prefix);

    if constexpr (MODE == BF_MIN) {
        double m = v.emin;
        for (int off = 32; off > 0; off >>= 1) m = fmin(m, __shfl_xor(m, off, 64));
        if (lane == 0) atomicMin(a.emin + b, ord_of(m));
    } else if constexpr (MODE == BF_COUNT) {
        unsigned long long c = v.cnt;
        for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
        if (lane == 0 && c) atomicAdd(a.count + b, c);
    }
}

// The collect pass (one per call): the same walk as a loop, the 2 C_i in LDS;
// every state with E <= T_b takes a place in the instance's buffer.
template <int NL>
__global__ __launch_bounds__(256) void k_brute_collect(BruteArgs a)
{
    __shared__ double sC[NL > 0 ? NL : 1][256];
    const long long wave = (long long)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int N = a.N;
    const long long per_inst = 1ll << (N - NL);
    const long long wpi = (per_inst + 63) >> 6;
    const int k = (int)(wave / wpi);
    if (k >= a.n_list) return;
    const int b = a.list[k];
    const long long t = (wave - k * wpi) * 64 + lane;
    if (t >= per_inst) return;
    const double* __restrict__ J = a.J + (size_t)b * N * N;
    const double* __restrict__ h = a.h + (size_t)b * N;
    const double* __restrict__ D = a.D + (size_t)b * BF_DSTRIDE;
    const uint64_t prefix = (uint64_t)t << NL;
    double C2[NL > 0 ? NL : 1];
    double E = brute_start<NL>(J, h, D, N, prefix, C2);
    for (int i = 0; i < NL; ++i) sC[i][threadIdx.x] = C2[i];
    const double T = a.T[b];
    unsigned long long* ctr = a.count + b;
    BruteRec* rec = a.rec + (size_t)b * BF_CAP;
    uint32_t y = 0;
    for (int g = 0; g < (1 << NL); ++g) {
        if (g > 0) {
            const int i = __builtin_ctz(g);
            const double c2 = sC[i][threadIdx.x];
            E += ((y >> i) & 1) ? c2 : -c2;
            E += D[g];
            y ^= 1u << i;
        }
        if (E <= T) {
            const unsigned long long slot = atomicAdd(ctr, 1ull);
            if (slot < (unsigned long long)BF_CAP) rec[slot] = BruteRec{E, prefix | y};
        }
    }
}

// D_g for the Gray walk over the NL low sites of every listed instance, and
// D_0 = E_low(0) = sum_{i<j<NL} J_ij.  One thread per (instance, g).
__global__ __launch_bounds__(256) void k_brute_table(BruteArgs a, int NL)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (k >= a.n_list || g >= (1 << NL)) return;
    const int b = a.list[k];
    const int N = a.N;
    const double* __restrict__ J = a.J + (size_t)b * N * N;
    double* D = a.D + (size_t)b * BF_DSTRIDE;
    if (g == 0) {
        double e = 0.0;
        for (int i = 0; i < NL; ++i)
            for (int j = i + 1; j < NL; ++j) e += J[i * N + j];
        D[0] = e;
        return;
    }
    const int i = __builtin_ctz(g);
    const int y = (g - 1) ^ ((g - 1) >> 1);
    double f = 0.0;   // sum over the other low sites of J_ij s_j
    for (int j = 0; j < NL; ++j)
        if (j != i) f += J[i * N + j] * (((y >> j) & 1) ? -1.0 : 1.0);
    const double si = ((y >> i) & 1) ? -1.0 : 1.0;
    D[g] = -2.0 * si * f;
}

// One block per listed instance: sort its records by (E, psi) in LDS (bitonic)
// and write the first K.
__global__ __launch_bounds__(1024) void k_brute_sort(BruteArgs a, int K, uint64_t* __restrict__ out_bits,
                                                     double* __restrict__ out_E, int* __restrict__ out_n)
{
    extern __shared__ unsigned long long sk[];   // [2][n2]: ord(E), psi
    const int k = blockIdx.x;
    if (k >= a.n_list) return;
    const int b = a.list[k];
    const unsigned long long total = a.count[b];
    const int n = (int)(total < (unsigned long long)BF_CAP ? total : (unsigned long long)BF_CAP);
    int n2 = 1;
    while (n2 < n) n2 <<= 1;
    unsigned long long* ke = sk;
    unsigned long long* kp = sk + n2;
    const BruteRec* r = a.rec + (size_t)b * BF_CAP;
    for (int q = threadIdx.x; q < n2; q += blockDim.x) {
        if (q < n) {
            ke[q] = ord_of(r[q].E);
            kp[q] = r[q].psi;
        } else {
            ke[q] = ~0ull;
            kp[q] = ~0ull;
        }
    }
    __syncthreads();
    for (int size = 2; size <= n2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int q = threadIdx.x; q < n2; q += blockDim.x) {
                const int p = q ^ stride;
                if (p > q) {
                    const bool up = (q & size) == 0;
                    const bool gt = ke[q] > ke[p] || (ke[q] == ke[p] && kp[q] > kp[p]);
                    if (gt == up) {
                        const unsigned long long te = ke[q], tp = kp[q];
                        ke[q] = ke[p];
                        kp[q] = kp[p];
                        ke[p] = te;
                        kp[p] = tp;
                    }
                }
            }
            __syncthreads();
        }
    }
    const int m = n < K ? n : K;
    for (int q = threadIdx.x; q < m; q += blockDim.x) {
        out_bits[(size_t)b * K + q] = kp[q];
        out_E[(size_t)b * K + q] = val_of(ke[q]);
    }
    if (threadIdx.x == 0) out_n[b] = m;
}

hipError_t launch_collect(const BruteArgs& a, int NL, hipStream_t st)
{
    const long long per_inst = 1ll << (a.N - NL);
    const long long waves = ((per_inst + 63) >> 6) * a.n_list;
    const long long blocks = (waves + 3) / 4;
    if (blocks > 0x7FFFFFFFll) return hipErrorInvalidValue;
    switch (NL) {
#define BF_CASE(n)                                                                                  \
    case n:                                                                                         \
        hipLaunchKernelGGL(k_brute_collect<n>, dim3((unsigned)blocks), dim3(256), 0, st, a);      \
        break;
        BF_CASE(0) BF_CASE(1) BF_CASE(2) BF_CASE(3) BF_CASE(4) BF_CASE(5) BF_CASE(6) BF_CASE(7) BF_CASE(8)
#undef BF_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int MODE>
hipError_t launch_mode(const BruteArgs& a, int NL, hipStream_t st)
{
    const long long per_inst = 1ll << (a.N - NL);
    const long long wpi = (per_inst + 63) >> 6;
    const long long waves = wpi * a.n_list;
    const long long blocks = (waves + 3) / 4;
    if (blocks > 0x7FFFFFFFll) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks), block(256);
    switch (NL) {
#define BF_CASE(n)                                                           \
    case n:                                                                  \
        hipLaunchKernelGGL((k_brute<n, MODE>), grid, block, 0, st, a);      \
        break;
        BF_CASE(0) BF_CASE(1) BF_CASE(2) BF_CASE(3) BF_CASE(4) BF_CASE(5) BF_CASE(6) BF_CASE(7) BF_CASE(8)
#undef BF_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

int brute_low_sites(int N) { return N < BF_NL ? N : BF_NL; }

hipError_t launch_brute_table(const BruteArgs& a, hipStream_t st)
{
    const int NL = brute_low_sites(a.N);
    const dim3 grid((unsigned)(((1 << NL) + 255) / 256), (unsigned)a.n_list);
    hipLaunchKernelGGL(k_brute_table, grid, dim3(256), 0, st, a, NL);
    return hipGetLastError();
}

hipError_t launch_brute_pass(const BruteArgs& a, int mode, hipStream_t st)
{
    const int NL = brute_low_sites(a.N);
    if (mode == BF_MIN) return launch_mode<BF_MIN>(a, NL, st);
    if (mode == BF_COUNT) return launch_mode<BF_COUNT>(a, NL, st);
    return launch_collect(a, NL, st);
}

hipError_t brute_sort_set_lds()
{
    return hipFuncSetAttribute((const void*)k_brute_sort, hipFuncAttributeMaxDynamicSharedMemorySize,
                               2 * BF_CAP * (int)sizeof(unsigned long long));
}

hipError_t launch_brute_sort(const BruteArgs& a, int K, uint64_t* out_bits, double* out_E, int* out_n,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_brute_sort, dim3((unsigned)a.n_list), dim3(1024), 2 * BF_CAP * sizeof(unsigned long long),
                       st, a, K, out_bits, out_E, out_n);
    return hipGetLastError();
}

}  // namespace qi

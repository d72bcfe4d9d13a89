// Start of a search: local fields F = h + J s of the L initial states of every
// instance, their energies, and S_0 = {x0} (Sec. II; Alg. 4 draws the L
// initial states).  F is computed as one FP64 GEMM per instance on the matrix
// cores: (4J)[N x N] times S[N x L] with S the +-1 spins, using
// v_mfma_f64_16x16x4_f64.  With J and h on the 2^-24 grid every partial sum is
// exact, so the result does not depend on the accumulation order.
#include "common.h"

namespace qi {

// One wave computes a 16 (sites) x 16 (searches) tile of J4 * S.
// Operand layout of v_mfma_f64_16x16x4_f64 (per lane l):
//   A[i][k]: i = l % 16, k = l / 16        (J4 rows = sites, k = summed site)
//   B[k][j]: j = l % 16, k = l / 16        (spins of search j at site k)
//   D[i][j]: 4 values, i = l/16 + 4*r, j = l % 16   (register r of lane l)
__global__ __launch_bounds__(64) void k_init_fields(Layout lay, const double* __restrict__ J4,
                                                    const uint64_t* __restrict__ x0)
{
    const int b = blockIdx.x;
    const int N = lay.N[b], Np = lay.Npad[b];
    const int row0 = blockIdx.y * 16, col0 = blockIdx.z * 16;
    if (row0 >= Np || col0 >= lay.L) return;
    const int lane = threadIdx.x;
    const double* Jb = J4 + lay.joff[b];
    const int ai = row0 + (lane & 15);
    const int kq = lane >> 4;
    const int lj = col0 + (lane & 15);
    const bool colok = lj < lay.L;
    const uint64_t* xs = x0 + (size_t)(b * lay.L + (colok ? lj : 0)) * lay.Wmax;
    typedef double v4d __attribute__((ext_vector_type(4)));
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < Np; k0 += 4) {
        const int k = k0 + kq;
        const double a = Jb[(size_t)ai * Np + k];
        double sg = 0.0;
        if (colok && k < N) sg = ((xs[k >> 6] >> (k & 63)) & 1ull) ? -1.0 : 1.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, sg, acc, 0, 0, 0);
    }
    if (!colok) return;
    const int s = b * lay.L + lj;
    const size_t q = (size_t)s * 2 * lay.M;   // slot 0 of search s
    const double* h = lay.h + (size_t)b * lay.Npmax;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int site = row0 + (lane >> 4) + 4 * r;
        if (site < Np) field_store(lay, q, b, site, site < N ? h[site] + 0.25 * acc[r] : 0.0);
    }
}

__device__ inline double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One wave per search: E = (1/2) sum_i s_i (F_i + h_i), the Zobrist hash of x0,
// and the seed kept set {x0} marked for expansion.
__global__ __launch_bounds__(64) void k_seed(Layout lay, const uint64_t* __restrict__ x0)
{
    const int s = blockIdx.x;
    const int b = s / lay.L;
    const int N = lay.N[b];
    const int lane = threadIdx.x;
    const size_t q = (size_t)s * 2 * lay.M;   // slot 0
    const uint64_t* x = x0 + (size_t)s * lay.Wmax;
    const FieldRow F = field_row(lay, q, b);
    const double* h = lay.h + (size_t)b * lay.Npmax;
    double e = 0.0;
    uint64_t z = 0;
    for (int i = lane; i < N; i += 64) {
        const bool up = ((x[i >> 6] >> (i & 63)) & 1ull) != 0;
        const double si = up ? -1.0 : 1.0;
        e += si * (F[i] + h[i]);
        if (up) z ^= lay.zkey[i];
    }
    e = wave_sum(e);
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)z, off, 64);
        const uint32_t hi = __shfl_xor((uint32_t)(z >> 32), off, 64);
        z ^= ((uint64_t)hi << 32) | lo;
    }
    if (lane < lay.Wmax) lay.bits[q * lay.Wmax + lane] = x[lane];
    if (lane == 0) {
        lay.E[q] = 0.5 * e;
        lay.zob[q] = z;
        lay.fresh[q] = 1;
        lay.kept[(size_t)s * lay.M] = 0;
        lay.nkept[s] = 1;
        lay.active[s] = 1;
        lay.retry[s] = 0;
        if (lay.form == 2) {
            lay.xfull[q] = 0;
            lay.mode[s] = 0;
            lay.last_mode[s] = 0;
        }
        if (s == 0) lay.flags[FLAG_FIRST] = lay.form == 1 ? 1 : 0;
    }
}

hipError_t launch_init_fields(const Layout& lay, const uint64_t* d_x0, hipStream_t st)
{
    dim3 grid(lay.B, (lay.Npmax + 15) / 16, (lay.L + 15) / 16);
    hipLaunchKernelGGL(k_init_fields, grid, dim3(64), 0, st, lay, lay.J4, d_x0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_seed, dim3(lay.S), dim3(64), 0, st, lay, d_x0);
    return hipGetLastError();
}

// Local fields and energies of `count` given states of one search, by the
// direct sum (used when a caller installs a kept set).  The states sit in
// slots 0..count-1; one block per state, one thread per site.
__global__ __launch_bounds__(256) void k_fields_direct(Layout lay, int search)
{
    const int k = blockIdx.x;
    const int b = search / lay.L;
    const int N = lay.N[b], Np = lay.Npad[b];
    const size_t q = (size_t)search * 2 * lay.M + k;
    const uint64_t* x = lay.bits + q * lay.Wmax;
    const double* Jb = lay.J4 + lay.joff[b];
    const double* h = lay.h + (size_t)b * lay.Npmax;
    __shared__ double red[256];
    double e = 0.0;
    uint64_t z = 0;
    for (int i = threadIdx.x; i < Np; i += blockDim.x) {
        double f = 0.0;
        if (i < N) {
            double acc = 0.0;
            for (int j = 0; j < N; ++j)
                acc += ((x[j >> 6] >> (j & 63)) & 1ull) ? -Jb[(size_t)i * Np + j] : Jb[(size_t)i * Np + j];
            f = h[i] + 0.25 * acc;
            const bool up = ((x[i >> 6] >> (i & 63)) & 1ull) != 0;
            e += (up ? -1.0 : 1.0) * (f + h[i]);
            if (up) z ^= lay.zkey[i];
        }
        field_store(lay, q, b, i, f);
    }
    red[threadIdx.x] = e;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double etot = red[0];
    __syncthreads();
    // reuse the buffer for the hash (xor of per-thread parts)
    uint64_t* zr = reinterpret_cast<uint64_t*>(red);
    zr[threadIdx.x] = z;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) zr[threadIdx.x] ^= zr[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        lay.E[q] = 0.5 * etot;
        lay.zob[q] = zr[0];
    }
}

hipError_t launch_fields_for(const Layout& lay, int search, int count, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fields_direct, dim3(count), dim3(256), 0, st, lay, search);
    return hipGetLastError();
}

}  // namespace qi

// Training of the pair-scoring network of the learned-proposal form, in FP32:
// forward, backward (chain rule through the two relu layers), a deterministic
// reduction of per-block gradients, and Adam (Kingma and Ba).  The loss is the
// class-weighted binary cross-entropy with logits, averaged over the samples.
// Parameter layout: W1[64][4], b1[64], W2[64][64], b2[64], w3[64], b3.
//
// k_mlp_grad: one wave per block, one sample per lane, tiles of 64 samples.
// The weights sit in LDS (broadcast reads).  Per tile the lanes write their
// activations and back-propagated errors to LDS, and then lane l accumulates
// row l of every weight gradient over the tile (dW2[l][:] = sum_s d2[s][l] h1[s][:],
// dW1[l][:] = sum_s g1[s][l] x[s][:]), so no atomics are needed.
#include "common.h"

namespace qi {

constexpr int TS = 64;   // samples per tile
constexpr int HP = 65;   // padded row stride of the per-tile LDS arrays (no bank conflicts)
constexpr int MLP_GRID_MAX = 1024;

__device__ inline uint64_t mlp_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ inline float softplus_f(float v) { return v > 0.f ? v + log1pf(expf(-v)) : log1pf(expf(v)); }
__device__ inline float sigmoid_f(float v)
{
    if (v >= 0.f) return 1.f / (1.f + expf(-v));
    const float e = expf(v);
    return e / (1.f + e);
}

// count samples: sample k is X[k] (sampled = 0) or X[hash(seed, step, k) mod n].
__global__ __launch_bounds__(64) void k_mlp_grad(const float* __restrict__ P, const float* __restrict__ X,
                                                 const uint8_t* __restrict__ Y, long long n, long long count,
                                                 int sampled, uint64_t seed, int step, float pos_w, float inv_count,
                                                 float* __restrict__ partial)
{
    __shared__ float sW1[4 * MLP_H], sB1[MLP_H], sW2[MLP_H * MLP_H], sB2[MLP_H], sW3[MLP_H];
    __shared__ float sH1[TS * HP], sD2[TS * HP], sE2[TS * HP];
    __shared__ float sX[TS * 4], sdz[TS];
    const int l = threadIdx.x;
    for (int k = l; k < 4 * MLP_H; k += TS) sW1[k] = P[MLP_W1 + k];
    for (int k = l; k < MLP_H * MLP_H; k += TS) sW2[k] = P[MLP_W2 + k];
    sB1[l] = P[MLP_B1 + l];
    sB2[l] = P[MLP_B2 + l];
    sW3[l] = P[MLP_W3 + l];
    const float b3 = P[MLP_B3];
    __syncthreads();

    float gW2[MLP_H];
#pragma unroll
    for (int m = 0; m < MLP_H; ++m) gW2[m] = 0.f;
    float gW1[4] = {0.f, 0.f, 0.f, 0.f};
    float gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f, loss = 0.f;
    const long long ntiles = (count + TS - 1) / TS;
    for (long long t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const long long k = t * TS + l;
        const bool ok = k < count;
        long long idx = k;
        if (sampled) idx = (long long)(mlp_mix(seed ^ mlp_mix(((uint64_t)step << 40) ^ (uint64_t)k)) % (uint64_t)n);
        float x[4] = {0.f, 0.f, 0.f, 0.f};
        float y = 0.f;
        if (ok) {
#pragma unroll
            for (int c = 0; c < 4; ++c) x[c] = X[idx * 4 + c];
            y = Y[idx] ? 1.f : 0.f;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) sX[l * 4 + c] = x[c];
        // layer 1
        float h1[MLP_H];
#pragma unroll
        for (int m = 0; m < MLP_H; ++m) {
            const float a = sB1[m] + sW1[m * 4 + 0] * x[0] + sW1[m * 4 + 1] * x[1] + sW1[m * 4 + 2] * x[2] +
                            sW1[m * 4 + 3] * x[3];
            h1[m] = a > 0.f ? a : 0.f;
            sH1[l * HP + m] = h1[m];
        }
        // layer 2 and the output
        float z = b3;
        for (int o = 0; o < MLP_H; ++o) {
            float a = sB2[o];
#pragma unroll
            for (int m = 0; m < MLP_H; ++m) a += sW2[o * MLP_H + m] * h1[m];
            const float h2 = a > 0.f ? a : 0.f;
            z += sW3[o] * h2;
            sE2[l * HP + o] = h2;
        }
        float dz = 0.f;
        if (ok) {
            loss += pos_w * y * softplus_f(-z) + (1.f - y) * softplus_f(z);
            dz = (-pos_w * y * sigmoid_f(-z) + (1.f - y) * sigmoid_f(z)) * inv_count;
        }
        sdz[l] = dz;
        for (int o = 0; o < MLP_H; ++o) {
            const float h2 = sE2[l * HP + o];
            sD2[l * HP + o] = h2 > 0.f ? dz * sW3[o] : 0.f;
            sE2[l * HP + o] = dz * h2;
        }
        __syncthreads();
        // lane l: row l of dW2, b2[l], w3[l]
        for (int s = 0; s < TS; ++s) {
            const float d = sD2[s * HP + l];
            gb2 += d;
            gw3 += sE2[s * HP + l];
#pragma unroll
            for (int m = 0; m < MLP_H; ++m) gW2[m] += d * sH1[s * HP + m];
        }
        if (l == 0)
            for (int s = 0; s < TS; ++s) gb3 += sdz[s];
        __syncthreads();
        // lane = sample: g1[m] = [h1_m > 0] sum_o d2[o] W2[o][m], written over sE2
        float g1[MLP_H];
#pragma unroll
        for (int m = 0; m < MLP_H; ++m) g1[m] = 0.f;
        for (int o = 0; o < MLP_H; ++o) {
            const float d = sD2[l * HP + o];
#pragma unroll
            for (int m = 0; m < MLP_H; ++m) g1[m] += d * sW2[o * MLP_H + m];
        }
#pragma unroll
        for (int m = 0; m < MLP_H; ++m) sE2[l * HP + m] = sH1[l * HP + m] > 0.f ? g1[m] : 0.f;
        __syncthreads();
        // lane l: row l of dW1, b1[l]
        for (int s = 0; s < TS; ++s) {
            const float g = sE2[s * HP + l];
            gb1 += g;
#pragma unroll
            for (int c = 0; c < 4; ++c) gW1[c] += g * sX[s * 4 + c];
        }
        __syncthreads();
    }
    float* out = partial + (size_t)blockIdx.x * (MLP_NPARAM + 1);
#pragma unroll
    for (int c = 0; c < 4; ++c) out[MLP_W1 + l * 4 + c] = gW1[c];
    out[MLP_B1 + l] = gb1;
#pragma unroll
    for (int m = 0; m < MLP_H; ++m) out[MLP_W2 + l * MLP_H + m] = gW2[m];
    out[MLP_B2 + l] = gb2;
    out[MLP_W3 + l] = gw3;
    for (int off = 32; off > 0; off >>= 1) loss += __shfl_xor(loss, off, 64);
    if (l == 0) {
        out[MLP_B3] = gb3;
        out[MLP_NPARAM] = loss * inv_count;
    }
}

// grad[p] = sum over blocks in block order (deterministic); loss likewise.
__global__ __launch_bounds__(256) void k_mlp_reduce(const float* __restrict__ partial, int grid,
                                                    float* __restrict__ grad, float* __restrict__ loss)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > MLP_NPARAM) return;
    float acc = 0.f;
    for (int g = 0; g < grid; ++g) acc += partial[(size_t)g * (MLP_NPARAM + 1) + p];
    if (p < MLP_NPARAM) grad[p] = acc;
    else if (loss) *loss = acc;
}

// c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t) (bias corrections)
__global__ __launch_bounds__(256) void k_mlp_adam(float* __restrict__ P, float* __restrict__ m, float* __restrict__ v,
                                                  const float* __restrict__ g, float lr, float b1, float b2, float eps,
                                                  float c1, float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAM) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.f - b1) * gp;
    const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    P[p] -= lr * (mp * c1) / (sqrtf(vp * c2) + eps);
}

__global__ __launch_bounds__(64) void k_mlp_fwd(const float* __restrict__ P, const float* __restrict__ X, long long n,
                                                float* __restrict__ z)
{
    __shared__ float sW1[4 * MLP_H], sB1[MLP_H], sW2[MLP_H * MLP_H], sB2[MLP_H], sW3[MLP_H];
    const int l = threadIdx.x;
    for (int k = l; k < 4 * MLP_H; k += 64) sW1[k] = P[MLP_W1 + k];
    for (int k = l; k < MLP_H * MLP_H; k += 64) sW2[k] = P[MLP_W2 + k];
    sB1[l] = P[MLP_B1 + l];
    sB2[l] = P[MLP_B2 + l];
    sW3[l] = P[MLP_W3 + l];
    const float b3 = P[MLP_B3];
    __syncthreads();
    for (long long k = (long long)blockIdx.x * 64 + l; k < n; k += (long long)gridDim.x * 64) {
        float x[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) x[c] = X[k * 4 + c];
        float h1[MLP_H];
#pragma unroll
        for (int m = 0; m < MLP_H; ++m) {
            const float a = sB1[m] + sW1[m * 4 + 0] * x[0] + sW1[m * 4 + 1] * x[1] + sW1[m * 4 + 2] * x[2] +
                            sW1[m * 4 + 3] * x[3];
            h1[m] = a > 0.f ? a : 0.f;
        }
        float out = b3;
        for (int o = 0; o < MLP_H; ++o) {
            float a = sB2[o];
#pragma unroll
            for (int m = 0; m < MLP_H; ++m) a += sW2[o * MLP_H + m] * h1[m];
            out += sW3[o] * (a > 0.f ? a : 0.f);
        }
        z[k] = out;
    }
}

int mlp_grid_for(long long count)
{
    const long long tiles = (count + TS - 1) / TS;
    return (int)(tiles < 1 ? 1 : (tiles > MLP_GRID_MAX ? MLP_GRID_MAX : tiles));
}

hipError_t launch_mlp_grad(const float* P, const float* X, const uint8_t* y, long long n, long long count,
                           uint64_t seed, int step, float pos_w, float* partial, int grid, hipStream_t st)
{
    const int sampled = step >= 0 ? 1 : 0;
    hipLaunchKernelGGL(k_mlp_grad, dim3(grid), dim3(64), 0, st, P, X, y, n, count, sampled, seed, step, pos_w,
                       1.f / (float)count, partial);
    return hipGetLastError();
}

hipError_t launch_mlp_reduce(const float* partial, int grid, float* grad, float* loss, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_reduce, dim3((MLP_NPARAM + 1 + 255) / 256), dim3(256), 0, st, partial, grid, grad, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float* P, float* m, float* v, const float* g, float lr, float b1, float b2, float eps,
                           float c1, float c2, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, P, m, v, g, lr, b1, b2, eps, c1,
                       c2);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* P, const float* X, long long n, float* z, hipStream_t st)
{
    long long g = (n + 63) / 64;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)g), dim3(64), 0, st, P, X, n, z);
    return hipGetLastError();
}

}  // namespace qi

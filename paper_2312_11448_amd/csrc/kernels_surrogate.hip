// The mixing-correction surrogate: per-cell features, the 8-64-64-1 ReLU
// network on BF16 matrix cores (inference), and its FP32 training step
// (weighted-MSE gradient, Adam).
//
// The quantity approximated is y = ln M_c, M_c = A_c / A_c^fm, the ratio of a
// cell's Monte-Carlo absorption to its full-mixing share (Sec. IV.B,
// Eq. (dotne-mix); the mixing length of Sec. III.B decides how far M is from
// one).
//
// Parameters: one FP32 vector of 4801 numbers, W1 [64][8] at 0, b1 at 512,
// W2 [64][64] at 576, b2 at 4672, w3 at 4736, b3 at 4800 (row-major
// [out][in]).
#include "common.hpp"

namespace mclya {
namespace {

constexpr int kFeat = 8, kHid = 64;
constexpr int OFF_W1 = 0, OFF_B1 = 512, OFF_W2 = 576, OFF_B2 = 4672, OFF_W3 = 4736, OFF_B3 = 4800;

// max(z, 0) as one v_med3_f32 (median of z, 0 and the largest float); fmaxf
// would first canonicalise z with a second instruction
__device__ __forceinline__ float relu(float z) { return __builtin_amdgcn_fmed3f(z, 0.0f, 3.402823466e38f); }
__device__ __forceinline__ float relu_grad(float z) { return z > 0.0f ? 1.0f : 0.0f; }

// ---- features ---------------------------------------------------------------
// Per cell: ln Delta, mean and variance of Delta over the 27 cells around it
// (periodic), div U by central differences (thermal velocities per cell),
// ln(T / 3000 K), x_e, z / 1000 - 1.1, and the box's clumping
// ln(<Delta^2> / <Delta>^2) = ln(1 + b) (Sec. II.C, Eq. (clumpingfactor)): in
// the no-mixing limit M_c = S_c sum(n_1s) / (n_1s,c sum(S)), which carries
// that box-wide ratio.
__device__ __forceinline__ float vel_at(const FeatBox &fb, int comp, uint32_t i)
{
    const size_t k = (size_t)comp * fb.ncells + i;
    if (fb.vel_dtype == MC_LYA_VEL_F32) return static_cast<const float *>(fb.vel)[k];
    return (float)static_cast<const _Float16 *>(fb.vel)[k];
}

__global__ __launch_bounds__(256) void features_kernel(const FeatBox *__restrict__ fbs, float *__restrict__ out)
{
    const FeatBox fb = fbs[blockIdx.y];
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= fb.ncells) return;
    const int nx = fb.nx, ny = fb.ny, nz = fb.nz;
    const int ix = (int)(i % (uint32_t)nx), iy = (int)((i / (uint32_t)nx) % (uint32_t)ny),
              iz = (int)(i / ((uint32_t)nx * (uint32_t)ny));
    int xs[3], ys[3], zs[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        xs[d] = ix + d - 1 < 0 ? nx - 1 : (ix + d - 1 == nx ? 0 : ix + d - 1);
        ys[d] = iy + d - 1 < 0 ? ny - 1 : (iy + d - 1 == ny ? 0 : iy + d - 1);
        zs[d] = iz + d - 1 < 0 ? nz - 1 : (iz + d - 1 == nz ? 0 : iz + d - 1);
    }
    float v[27];
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 27; ++k) {
        const int dz = k / 9, dy = (k / 3) % 3, dx = k % 3;
        v[k] = fb.od[(size_t)xs[dx] + (size_t)nx * ((size_t)ys[dy] + (size_t)ny * (size_t)zs[dz])];
        s += v[k];
    }
    const float mean = s / 27.0f;
    float ss = 0.0f;
#pragma unroll
    for (int k = 0; k < 27; ++k) ss += (v[k] - mean) * (v[k] - mean);
    float div = 0.0f;
    if (fb.vel_dtype != MC_LYA_VEL_NONE) {
        const uint32_t sx = (uint32_t)nx, sxy = (uint32_t)nx * (uint32_t)ny;
        auto at = [&](int x, int y, int z) { return (uint32_t)x + sx * (uint32_t)y + sxy * (uint32_t)z; };
        div = 0.5f * (vel_at(fb, 0, at(xs[2], iy, iz)) - vel_at(fb, 0, at(xs[0], iy, iz))) +
              0.5f * (vel_at(fb, 1, at(ix, ys[2], iz)) - vel_at(fb, 1, at(ix, ys[0], iz))) +
              0.5f * (vel_at(fb, 2, at(ix, iy, zs[2])) - vel_at(fb, 2, at(ix, iy, zs[0])));
    }
    const float xe = fb.xe ? fb.xe[i] : fb.xe_uniform;
    float4 *o = reinterpret_cast<float4 *>(out + ((size_t)fb.cell_off + i) * kFeat);
    o[0] = make_float4(logf(v[13]), mean, ss / 27.0f, div);
    o[1] = make_float4(fb.ln_t, xe, fb.z_feat, fb.ln_clump);
}

// ---- inference on matrix cores ---------------------------------------------
// One wave evaluates 32 cells at a time with the activations held transposed
// (hidden units along the matrix rows, cells along the columns), so the
// layer-1 results a lane holds for its cell are the layer-2 operands it must
// supply, and no data moves between lanes until the final dot product.
//   Layer 1: v_mfma_f32_32x32x8_bf16 (K = the 8 features). Lane l holds
//   A[l%32][4(l/32)+e], B[4(l/32)+e][l%32] (e = 0..3) and
//   D[8q + 4(l/32) + t][l%32] in register 4q + t.
//   Layer 2: v_mfma_f32_32x32x16_bf16, K = 16 hidden units per step, lane
//   half l/32 and element e (0..7) of the A and B operands naming the same
//   K index. Step s takes its B elements straight from the layer-1 registers,
//   element e of lane half hb being hidden unit
//   16 s + 8 (e / 4) + 4 hb + e % 4 (a permutation of 0..63), and the A
//   operand (W2) is gathered in that same order.
// Biases enter as the accumulators' initial values.
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// binary32 -> bfloat16, round to nearest even (one v_cvt_pk_bf16_f32 per pair)
__device__ __forceinline__ short to_bf16(float f) { return __builtin_bit_cast(short, (__bf16)f); }

__device__ __forceinline__ int l2_unit(int s, int hb, int e) { return 16 * s + 8 * (e / 4) + 4 * hb + (e % 4); }

__global__ __launch_bounds__(256) void mlp_forward_kernel(const float *__restrict__ P, const float *__restrict__ X,
                                                          uint64_t n, float *__restrict__ y,
                                                          uint8_t *__restrict__ outside,
                                                          const float *__restrict__ lo,
                                                          const float *__restrict__ hi,
                                                          unsigned long long *__restrict__ n_out)
{
    __shared__ unsigned long long s_cnt;
    const int lane = threadIdx.x & 63, half = lane >> 5, col = lane & 31;
    if (threadIdx.x == 0) s_cnt = 0;
    bf16x4 a1[2];
    bf16x8 a2[2][4];
    f32x16 c1[2], c2[2];
    float w3r[2][16];
#pragma unroll
    for (int T = 0; T < 2; ++T) {
#pragma unroll
        for (int e = 0; e < 4; ++e) a1[T][e] = to_bf16(P[OFF_W1 + (32 * T + col) * kFeat + 4 * half + e]);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int e = 0; e < 8; ++e) a2[T][s][e] = (__bf16)P[OFF_W2 + (32 * T + col) * kHid + l2_unit(s, half, e)];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = 32 * T + 8 * (r / 4) + 4 * half + (r % 4);
            c1[T][r] = P[OFF_B1 + row];
            c2[T][r] = P[OFF_B2 + row];
            w3r[T][r] = P[OFF_W3 + row];
        }
    }
    const float b3 = P[OFF_B3];
    float flo[4], fhi[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        flo[e] = lo ? lo[4 * half + e] : -3.0e38f;
        fhi[e] = hi ? hi[4 * half + e] : 3.0e38f;
    }
    __syncthreads();
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / 64);
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const uint64_t tiles = (n + 31) / 32;
    uint32_t n_outside = 0;
    // the next tile's features are loaded while this one is computed
    auto load = [&](uint64_t tile) {
        const uint64_t cell = tile * 32 + (uint64_t)col;
        float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (cell < n) v = *reinterpret_cast<const float4 *>(X + cell * kFeat + 4 * half);
        return v;
    };
    float4 next = load(wave);
    for (uint64_t tile = wave; tile < tiles; tile += waves) {
        const uint64_t cell = tile * 32 + (uint64_t)col;
        const bool valid = cell < n;
        const float4 xv = next;
        next = load(tile + waves);
        const float xs[4] = {xv.x, xv.y, xv.z, xv.w};
        int out_env = 0;
        bf16x4 bx;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            out_env |= (xs[e] < flo[e]) | (xs[e] > fhi[e]);
            bx[e] = to_bf16(xs[e]);
        }
        out_env |= __shfl_xor(out_env, 32, 64);
        f32x16 d1[2];
#pragma unroll
        for (int T = 0; T < 2; ++T) d1[T] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a1[T], bx, c1[T], 0, 0, 0);
        bf16x8 b2[4];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int e = 0; e < 8; ++e) b2[s][e] = (__bf16)relu(d1[s / 2][4 * (2 * (s % 2) + e / 4) + e % 4]);
        f32x16 d2[2] = {c2[0], c2[1]};
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int T = 0; T < 2; ++T) d2[T] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2[T][s], b2[s], d2[T], 0, 0, 0);
        float part = 0.0f;
#pragma unroll
        for (int T = 0; T < 2; ++T)
#pragma unroll
            for (int r = 0; r < 16; ++r) part += w3r[T][r] * relu(d2[T][r]);
        part += __shfl_xor(part, 32, 64);
        if (half == 0 && valid) {
            y[cell] = part + b3;
            if (outside) outside[cell] = (uint8_t)out_env;
            n_outside += (uint32_t)out_env;
        }
    }
    if (n_out) {
        unsigned long long c = n_outside;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
        if (lane == 0 && c) atomicAdd(&s_cnt, c);
        __syncthreads();
        if (threadIdx.x == 0 && s_cnt) atomicAdd(n_out, s_cnt);
    }
}

// ---- training: weighted-MSE gradient in FP32 --------------------------------
// One wave per block; lane h is hidden unit h of both layers. Each block
// walks cells blockIdx.x, blockIdx.x + gridDim.x, ... and writes its partial
// sums (the unnormalised gradient sum_i 2 w_i r_i dy_i/dtheta, sum w r^2,
// sum w) to its own slot; a second kernel adds the slots in block order, so
// the result does not depend on timing.
__global__ __launch_bounds__(64) void mlp_grad_kernel(const float *__restrict__ P, const float *__restrict__ X,
                                                      const float *__restrict__ tgt, const float *__restrict__ wgt,
                                                      uint64_t n, float *__restrict__ partial)
{
    __shared__ float s_h1[kHid], s_gz2[kHid], s_x[kFeat];
    const int h = threadIdx.x;
    float w1[kFeat], w2r[kHid], w2c[kHid];
#pragma unroll
    for (int k = 0; k < kFeat; ++k) w1[k] = P[OFF_W1 + h * kFeat + k];
#pragma unroll
    for (int k = 0; k < kHid; ++k) {
        w2r[k] = P[OFF_W2 + h * kHid + k];
        w2c[k] = P[OFF_W2 + k * kHid + h];
    }
    const float b1 = P[OFF_B1 + h], b2 = P[OFF_B2 + h], w3 = P[OFF_W3 + h], b3 = P[OFF_B3];
    float gW1[kFeat], gW2[kHid];
#pragma unroll
    for (int k = 0; k < kFeat; ++k) gW1[k] = 0.0f;
#pragma unroll
    for (int k = 0; k < kHid; ++k) gW2[k] = 0.0f;
    float gb1 = 0.0f, gb2 = 0.0f, gw3 = 0.0f, gb3 = 0.0f, loss = 0.0f, wsum = 0.0f;
    for (uint64_t c = blockIdx.x; c < n; c += gridDim.x) {
        __syncthreads();
        if (h < kFeat) s_x[h] = X[c * kFeat + h];
        __syncthreads();
        float x[kFeat];
#pragma unroll
        for (int k = 0; k < kFeat; ++k) x[k] = s_x[k];
        float z1 = b1;
#pragma unroll
        for (int k = 0; k < kFeat; ++k) z1 += w1[k] * x[k];
        const float h1 = relu(z1);
        s_h1[h] = h1;
        __syncthreads();
        float z2 = b2;
#pragma unroll
        for (int k = 0; k < kHid; ++k) z2 += w2r[k] * s_h1[k];
        const float h2 = relu(z2);
        float yv = w3 * h2;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) yv += __shfl_xor(yv, off, 64);
        yv += b3;
        const float wc = wgt[c];
        const float r = yv - tgt[c];
        loss += wc * r * r;
        wsum += wc;
        const float gy = 2.0f * wc * r;
        gw3 += gy * h2;
        gb3 += gy;
        const float gz2 = gy * w3 * relu_grad(z2);
        gb2 += gz2;
#pragma unroll
        for (int k = 0; k < kHid; ++k) gW2[k] += gz2 * s_h1[k];
        s_gz2[h] = gz2;
        __syncthreads();
        float gh1 = 0.0f;
#pragma unroll
        for (int k = 0; k < kHid; ++k) gh1 += w2c[k] * s_gz2[k];
        const float gz1 = gh1 * relu_grad(z1);
        gb1 += gz1;
#pragma unroll
        for (int k = 0; k < kFeat; ++k) gW1[k] += gz1 * x[k];
    }
    float *p = partial + (size_t)blockIdx.x * kMlpPartStride;
#pragma unroll
    for (int k = 0; k < kFeat; ++k) p[OFF_W1 + h * kFeat + k] = gW1[k];
    p[OFF_B1 + h] = gb1;
#pragma unroll
    for (int k = 0; k < kHid; ++k) p[OFF_W2 + h * kHid + k] = gW2[k];
    p[OFF_B2 + h] = gb2;
    p[OFF_W3 + h] = gw3;
    if (h == 0) {
        p[OFF_B3] = gb3;
        p[kMlpParams] = loss;
        p[kMlpParams + 1] = wsum;
    }
}

// grad[j] = sum over blocks of partial[b][j], j < kMlpParams + 2 (the last
// two entries are sum w r^2 and sum w), in two fixed-order passes: groups of
// kMlpGroup consecutive blocks into tmp[g][j], then the groups in order.
constexpr int kMlpGroup = 32;

__global__ __launch_bounds__(256) void mlp_reduce_groups_kernel(const float *__restrict__ partial, int blocks,
                                                                float *__restrict__ tmp)
{
    const int j = blockIdx.x * 256 + threadIdx.x, g = blockIdx.y;
    if (j >= kMlpParams + 2) return;
    float s = 0.0f;
    const int b1 = min(blocks, (g + 1) * kMlpGroup);
    for (int b = g * kMlpGroup; b < b1; ++b) s += partial[(size_t)b * kMlpPartStride + j];
    tmp[(size_t)g * kMlpPartStride + j] = s;
}

__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float *__restrict__ tmp, int groups,
                                                         float *__restrict__ grad)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= kMlpParams + 2) return;
    float s = 0.0f;
    for (int g = 0; g < groups; ++g) s += tmp[(size_t)g * kMlpPartStride + j];
    grad[j] = s;
}

// Normalise by sum w and take one Adam step (Kingma & Ba 2015, Algorithm 1,
// with bias correction); step counts from 1.
__global__ __launch_bounds__(256) void mlp_adam_kernel(float *__restrict__ P, float *__restrict__ m,
                                                       float *__restrict__ v, float *__restrict__ grad,
                                                       MlpAdam a)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= kMlpParams) return;
    const float wsum = grad[kMlpParams + 1];
    const float g = wsum > 0.0f ? grad[j] / wsum : 0.0f;
    grad[j] = g;
    const float mj = a.beta1 * m[j] + (1.0f - a.beta1) * g;
    const float vj = a.beta2 * v[j] + (1.0f - a.beta2) * g * g;
    m[j] = mj;
    v[j] = vj;
    const float mhat = mj / a.bc1, vhat = vj / a.bc2;
    P[j] -= a.lr * mhat / (sqrtf(vhat) + a.eps);
}

__global__ __launch_bounds__(256) void mlp_normalise_kernel(float *__restrict__ grad)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= kMlpParams) return;
    const float wsum = grad[kMlpParams + 1];
    grad[j] = wsum > 0.0f ? grad[j] / wsum : 0.0f;
}

}  // namespace

hipError_t launch_features(const FeatBox *fb_dev, int n_boxes, int max_blk, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(features_kernel, dim3((unsigned)max_blk, (unsigned)n_boxes), dim3(256), 0, s, fb_dev, out);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float *params, const float *X, uint64_t n, float *y, uint8_t *outside,
                              const float *lo, const float *hi, unsigned long long *n_out, int grid,
                              hipStream_t s)
{
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)grid), dim3(256), 0, s, params, X, n, y, outside, lo, hi,
                       n_out);
    return hipGetLastError();
}

hipError_t launch_mlp_gradient(const float *params, const float *X, const float *t, const float *w, uint64_t n,
                               float *partial, int blocks, float *grad, hipStream_t s)
{
    const int groups = (blocks + kMlpGroup - 1) / kMlpGroup;
    float *tmp = partial + (size_t)blocks * kMlpPartStride;
    hipLaunchKernelGGL(mlp_grad_kernel, dim3((unsigned)blocks), dim3(64), 0, s, params, X, t, w, n, partial);
    hipLaunchKernelGGL(mlp_reduce_groups_kernel, dim3((unsigned)((kMlpParams + 2 + 255) / 256), (unsigned)groups),
                       dim3(256), 0, s, partial, blocks, tmp);
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((unsigned)((kMlpParams + 2 + 255) / 256)), dim3(256), 0, s, tmp,
                       groups, grad);
    return hipGetLastError();
}

hipError_t launch_mlp_normalise(float *grad, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_normalise_kernel, dim3((unsigned)((kMlpParams + 255) / 256)), dim3(256), 0, s, grad);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *params, float *m, float *v, float *grad, const MlpAdam &a, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((unsigned)((kMlpParams + 255) / 256)), dim3(256), 0, s, params, m, v,
                       grad, a);
    return hipGetLastError();
}

}  // namespace mclya

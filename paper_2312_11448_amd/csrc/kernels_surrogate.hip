// The mixing-correction surrogate: per-cell features, the 8-64-64-1 ReLU
// network on BF16 matrix cores (inference and the weighted-MSE gradient of
// training, FP32 accumulation), and Adam on the FP32 master parameters.
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
// ReLU's derivative (0 at z = 0)
__device__ __forceinline__ float step(float z) { return z > 0.0f ? 1.0f : 0.0f; }

// ---- features ---------------------------------------------------------------
// Per cell: ln Delta, mean and variance of Delta over the 27 cells around it
// (periodic), div U by central differences (thermal velocities per cell),
// ln(T / 3000 K), x_e, z / 1000 - 1.1, and the box's clumping
// ln(<Delta^2> / <Delta>^2) = ln(1 + b) (Sec. II.C, Eq. (clumpingfactor)): in
// the no-mixing limit M_c = S_c sum(n_1s) / (n_1s,c sum(S)), which carries
// that box-wide ratio.
// A load through the global (not flat) memory path at a byte offset from a
// base held in scalar registers. With 32-bit offsets (boxes of at most 2^30
// cells) each neighbour costs one add.
template <typename T, typename Off>
__device__ __forceinline__ T load_at(const void *base, Off byte_off)
{
    typedef const __attribute__((address_space(1))) char gchar;
    typedef const __attribute__((address_space(1))) T gT;
    return *(gT *)((gchar *)base + (uint64_t)byte_off);
}

// div U by central differences, from velocity components stored as V
// (component c starts c * ncells elements in; FP16 elements are half as far
// apart as the 4-byte offsets given)
template <typename V, typename Off>
__device__ __forceinline__ float divergence(const FeatBox &fb, const Off (&xo)[3], const Off (&yo)[3],
                                            const Off (&zo)[3])
{
    const char *vb = static_cast<const char *>(fb.vel);
    auto vel = [&](int comp, Off off) -> float {
        const void *base = vb + (uint64_t)comp * fb.ncells * sizeof(V);
        return (float)load_at<V>(base, (Off)(off / (4 / sizeof(V))));
    };
    return 0.5f * (vel(0, xo[2] + yo[1] + zo[1]) - vel(0, xo[0] + yo[1] + zo[1])) +
           0.5f * (vel(1, xo[1] + yo[2] + zo[1]) - vel(1, xo[1] + yo[0] + zo[1])) +
           0.5f * (vel(2, xo[1] + yo[1] + zo[2]) - vel(2, xo[1] + yo[1] + zo[0]));
}

// A store that streams past the caches: the 32 bytes a cell's features take
// are read back only by a later kernel, and keeping them out of L2 leaves it
// to the neighbour rows this kernel reads again and again.
__device__ __forceinline__ void store_stream(float4 *p, float4 v)
{
    typedef float f32x4 __attribute__((ext_vector_type(4)));
    __builtin_nontemporal_store(__builtin_bit_cast(f32x4, v), reinterpret_cast<f32x4 *>(p));
}

template <typename Off>
__device__ __forceinline__ void features_cell(const FeatBox &fb, uint32_t i, float *__restrict__ out)
{
    const uint32_t nx = (uint32_t)fb.nx, ny = (uint32_t)fb.ny, nz = (uint32_t)fb.nz;
    const uint32_t ix = i % nx, r = i / nx, iy = r % ny, iz = r / ny;
    const Off sx = (Off)nx * 4u, sxy = (Off)nx * ny * 4u;
    // byte offsets (4-byte elements) of the columns, rows and planes around
    // the cell, periodic: index 0 is the lower neighbour, 2 the upper
    Off xo[3], yo[3], zo[3];
    xo[0] = (Off)(ix == 0 ? nx - 1 : ix - 1) * 4u;
    xo[1] = (Off)ix * 4u;
    xo[2] = (Off)(ix + 1 == nx ? 0 : ix + 1) * 4u;
    yo[0] = (Off)(iy == 0 ? ny - 1 : iy - 1) * sx;
    yo[1] = (Off)iy * sx;
    yo[2] = (Off)(iy + 1 == ny ? 0 : iy + 1) * sx;
    zo[0] = (Off)(iz == 0 ? nz - 1 : iz - 1) * sxy;
    zo[1] = (Off)iz * sxy;
    zo[2] = (Off)(iz + 1 == nz ? 0 : iz + 1) * sxy;
    float v[27];
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 27; ++k) {
        const int dz = k / 9, dy = (k / 3) % 3, dx = k % 3;
        v[k] = load_at<float>(fb.od, xo[dx] + yo[dy] + zo[dz]);
        s += v[k];
    }
    const float mean = s / 27.0f;
    float ss = 0.0f;
#pragma unroll
    for (int k = 0; k < 27; ++k) ss += (v[k] - mean) * (v[k] - mean);
    float div = 0.0f;
    if (fb.vel_dtype == MC_LYA_VEL_F32)
        div = divergence<float>(fb, xo, yo, zo);
    else if (fb.vel_dtype == MC_LYA_VEL_F16)
        div = divergence<_Float16>(fb, xo, yo, zo);
    const float xe = fb.xe ? load_at<float>(fb.xe, xo[1] + yo[1] + zo[1]) : fb.xe_uniform;
    float4 *o = reinterpret_cast<float4 *>(out + ((size_t)fb.cell_off + i) * kFeat);
    store_stream(&o[0], make_float4(logf(v[13]), mean, ss / 27.0f, div));
    store_stream(&o[1], make_float4(fb.ln_t, xe, fb.z_feat, fb.ln_clump));
}

// 4 consecutive elements of type V at a byte offset, as float
template <typename V, typename Off>
__device__ __forceinline__ void load4(const void *base, Off byte_off, float *o)
{
    typedef V v4 __attribute__((ext_vector_type(4)));
    const v4 a = load_at<v4>(base, byte_off);
#pragma unroll
    for (int e = 0; e < 4; ++e) o[e] = (float)a[e];
}

// div U of four cells x..x+3 of one row (xm, x0, xp: byte offsets of x - 1,
// x and x + 4, periodic), with the same central differences as above
template <typename V, typename Off>
__device__ __forceinline__ void divergence4(const FeatBox &fb, Off xm, Off x0, Off xp, const Off (&yo)[3],
                                            const Off (&zo)[3], float (&dv)[4])
{
    const char *vb = static_cast<const char *>(fb.vel);
    const uint64_t comp = (uint64_t)fb.ncells * sizeof(V);
    constexpr Off div_off = 4 / sizeof(V);
    const Off row = yo[1] + zo[1];
    float vx[6], yp[4], ym[4], zp[4], zm[4];
    vx[0] = (float)load_at<V>(vb, (Off)((row + xm) / div_off));
    load4<V>(vb, (Off)((row + x0) / div_off), &vx[1]);
    vx[5] = (float)load_at<V>(vb, (Off)((row + xp) / div_off));
    load4<V>(vb + comp, (Off)((yo[2] + zo[1] + x0) / div_off), yp);
    load4<V>(vb + comp, (Off)((yo[0] + zo[1] + x0) / div_off), ym);
    load4<V>(vb + 2 * comp, (Off)((yo[1] + zo[2] + x0) / div_off), zp);
    load4<V>(vb + 2 * comp, (Off)((yo[1] + zo[0] + x0) / div_off), zm);
#pragma unroll
    for (int c = 0; c < 4; ++c)
        dv[c] = 0.5f * (vx[c + 2] - vx[c]) + 0.5f * (yp[c] - ym[c]) + 0.5f * (zp[c] - zm[c]);
}

// The same features for four cells along x (nx a multiple of 4): each of the
// 9 rows around them is read as one 16-byte load plus the cells beyond its
// two ends, 27 + 7 loads for four cells where one cell at a time takes 33
// each. The sums run in the same order as for one cell.
template <typename Off>
__device__ __forceinline__ void features_quad(const FeatBox &fb, uint32_t q, float4 *__restrict__ stage)
{
    const uint32_t nx = (uint32_t)fb.nx, ny = (uint32_t)fb.ny, nz = (uint32_t)fb.nz;
    const uint32_t i = 4u * q;
    const uint32_t ix = i % nx, r = i / nx, iy = r % ny, iz = r / ny;
    const Off sx = (Off)nx * 4u, sxy = (Off)nx * ny * 4u;
    const Off xm = (Off)(ix == 0 ? nx - 1 : ix - 1) * 4u, x0 = (Off)ix * 4u,
              xp = (Off)(ix + 4 == nx ? 0 : ix + 4) * 4u;
    Off yo[3], zo[3];
    yo[0] = (Off)(iy == 0 ? ny - 1 : iy - 1) * sx;
    yo[1] = (Off)iy * sx;
    yo[2] = (Off)(iy + 1 == ny ? 0 : iy + 1) * sx;
    zo[0] = (Off)(iz == 0 ? nz - 1 : iz - 1) * sxy;
    zo[1] = (Off)iz * sxy;
    zo[2] = (Off)(iz + 1 == nz ? 0 : iz + 1) * sxy;
    // w[3 dz + dy][j]: Delta at x - 1 + j of the row (dy, dz)
    float w[9][6];
#pragma unroll
    for (int rw = 0; rw < 9; ++rw) {
        const Off row = yo[rw % 3] + zo[rw / 3];
        w[rw][0] = load_at<float>(fb.od, row + xm);
        load4<float>(fb.od, row + x0, &w[rw][1]);
        w[rw][5] = load_at<float>(fb.od, row + xp);
    }
    float dv[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (fb.vel_dtype == MC_LYA_VEL_F32)
        divergence4<float>(fb, xm, x0, xp, yo, zo, dv);
    else if (fb.vel_dtype == MC_LYA_VEL_F16)
        divergence4<_Float16>(fb, xm, x0, xp, yo, zo, dv);
    float xe[4];
    if (fb.xe)
        load4<float>(fb.xe, yo[1] + zo[1] + x0, xe);
    else
#pragma unroll
        for (int c = 0; c < 4; ++c) xe[c] = fb.xe_uniform;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        float v[27];
        float s = 0.0f;
#pragma unroll
        for (int k = 0; k < 27; ++k) {
            const int dz = k / 9, dy = (k / 3) % 3, dx = k % 3;
            v[k] = w[3 * dz + dy][c + dx];
            s += v[k];
        }
        const float mean = s / 27.0f;
        float ss = 0.0f;
#pragma unroll
        for (int k = 0; k < 27; ++k) ss += (v[k] - mean) * (v[k] - mean);
        stage[2 * c] = make_float4(logf(v[13]), mean, ss / 27.0f, dv[c]);
        stage[2 * c + 1] = make_float4(fb.ln_t, xe[c], fb.z_feat, fb.ln_clump);
    }
}

// One thread per cell, or per four cells along x. Workgroups go round-robin
// to the chip's 8 XCDs; when a box's block count is a multiple of 8 its
// blocks are dealt so that each XCD takes a contiguous run of them (a slab of
// the box), whose neighbour rows and planes its own L2 then holds.
__global__ __launch_bounds__(256) void features_kernel(const FeatBox *__restrict__ fbs, float *__restrict__ out)
{
    // a wave's 256 cells of output (8 KB), written out contiguously (rows of
    // 9 for 8 values, so that the lanes' writes spread over the banks)
    __shared__ float4 s_out[4][64 * 9];
    const FeatBox fb = fbs[blockIdx.y];
    const uint32_t threads = fb.quad ? fb.ncells / 4u : fb.ncells;
    const uint32_t need = (threads + 255u) / 256u, bx = blockIdx.x;
    if (bx >= need) return;
    const uint32_t blk = need % 8u == 0 ? (bx % 8u) * (need / 8u) + bx / 8u : bx;
    const uint32_t t = blk * 256u + threadIdx.x;
    const bool narrow = fb.ncells <= (1u << 30);
    if (fb.quad) {
        const uint32_t wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const uint32_t t0 = t - lane;                  // the wave's first thread
        if (t0 >= threads) return;
        if (t < threads) {
            if (narrow)
                features_quad<uint32_t>(fb, t, &s_out[wv][9 * lane]);
            else
                features_quad<uint64_t>(fb, t, &s_out[wv][9 * lane]);
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t n16 = 8u * (threads - t0 < 64u ? threads - t0 : 64u);   // 16-byte chunks to write
        float4 *o = reinterpret_cast<float4 *>(out + ((size_t)fb.cell_off + 4u * (size_t)t0) * kFeat);
#pragma unroll
        for (uint32_t j = 0; j < 8; ++j) {
            const uint32_t k = 64u * j + lane;
            if (k < n16) store_stream(&o[k], s_out[wv][9 * (k / 8u) + k % 8u]);
        }
        return;
    }
    if (t >= threads) return;
    {
        if (narrow)
            features_cell<uint32_t>(fb, t, out);
        else
            features_cell<uint64_t>(fb, t, out);
    }
}

// ---- the network on the matrix cores ----------------------------------------
// Inference and training evaluate one function: W1, W2, the features and the
// layer-1 activations in BF16, products accumulated in FP32, each bias b1, b2
// entering as the two BF16 terms hi = bf16(b), lo = bf16(b - hi) (their sum
// is b to 2^-16 relative), w3 and b3 in FP32 (the last layer on the VALU).
//
// An MFMA D = A B reads A with its rows on the lanes (lane % 32) and B with
// its columns on the lanes, both with the K index in the registers: lane
// half hb = lane / 32 and element e (0..7) of v_mfma_f32_32x32x16_bf16 name
// K index 8 hb + e in both operands. D comes back with its columns on the
// lanes and row 8 (r / 4) + 4 hb + r % 4 in register r.
//   Layer 1, K = 16: the 8 features in lane half 0, and in half 1 the pair
//   (1, 1) against the pair (hi, lo) of b1, so the bias is part of the product.
//   Layer 2, K = 64 hidden units in four steps plus a fifth with the b2 pair.
//   Step s takes its B elements straight from the layer-1 registers: element
//   e of lane half hb is hidden unit l2_unit(s, hb, e) = 16 s + 8 (e / 4) +
//   4 hb + e % 4, a permutation of 0..63, and W2 is gathered in that order.
// Evaluated with the cells as the columns ("C": D1 = W1 X^T, D2 = W2 H1) a
// lane holds one cell and the hidden units in its registers, which is what
// the next layer's B operand needs, so no data moves between lanes until the
// final dot product. Swapping A and B transposes a product ("H": D1' = X W1^T,
// D2' = H1^T W2^T, hidden unit per lane, cells in the registers): the same
// operand registers serve both.
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ int l2_unit(int s, int hb, int e) { return 16 * s + 8 * (e / 4) + 4 * hb + (e % 4); }
// row of register r of a 32x32 result, in lane half `half`
__device__ __forceinline__ int d_row(int r, int half) { return 8 * (r >> 2) + 4 * half + (r & 3); }
// the layer-1 register of hidden unit l2_unit(s, hb, e) (in block s / 2)
__device__ __forceinline__ int l1_reg(int s, int e) { return 4 * (2 * (s % 2) + e / 4) + e % 4; }

__device__ __forceinline__ f32x16 mfma16(const bf16x8 &a, const bf16x8 &b, const f32x16 &c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x16 zero16()
{
    f32x16 z;
#pragma unroll
    for (int r = 0; r < 16; ++r) z[r] = 0.0f;
    return z;
}

// (hi, lo, 0, ...) in lane half 0 when `in_half0`, else in half 1; zeros in
// the other half
__device__ __forceinline__ bf16x8 bias_pair(float b, bool here)
{
    bf16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (__bf16)0.0f;
    if (here) {
        const __bf16 hi = (__bf16)b;
        v[0] = hi;
        v[1] = (__bf16)(b - (float)hi);
    }
    return v;
}

__device__ __forceinline__ bf16x8 ones_pair(bool here)
{
    bf16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (__bf16)(here && e < 2 ? 1.0f : 0.0f);
    return v;
}

// The weight operands of lane (half, col): a1[T] for unit u = 32 T + col
// (W1[u][0..7] in half 0, the b1 pair in half 1) and a2[T][s] (W2[u][unit
// l2_unit(s, half, e)] for s < 4, the b2 pair in half 0 for s = 4).
struct NetOps {
    bf16x8 a1[2];
    bf16x8 a2[2][5];
};

__device__ __forceinline__ void load_ops(const float *__restrict__ P, int half, int col, NetOps &o)
{
#pragma unroll
    for (int T = 0; T < 2; ++T) {
        const int u = 32 * T + col;
        if (half == 0) {
#pragma unroll
            for (int e = 0; e < 8; ++e) o.a1[T][e] = (__bf16)P[OFF_W1 + u * kFeat + e];
        } else {
            o.a1[T] = bias_pair(P[OFF_B1 + u], true);
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int e = 0; e < 8; ++e) o.a2[T][s][e] = (__bf16)P[OFF_W2 + u * kHid + l2_unit(s, half, e)];
        o.a2[T][4] = bias_pair(P[OFF_B2 + u], half == 0);
    }
}

// The K operand of a cell's features: the features in lane half 0, the pair
// (1, 1) that meets the b1 pair in half 1.
__device__ __forceinline__ bf16x8 feature_operand(const float (&x)[kFeat], int half)
{
    if (half == 0) {
        bf16x8 v;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (__bf16)x[e];
        return v;
    }
    return ones_pair(true);
}

// (bf16(a), bf16(b)) in one register, a in the low half
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
// cache-policy operand of a buffer load: non-temporal (streaming)
constexpr int kStreamingLoad = 2;

__device__ __forceinline__ uint32_t bf16_pair(float a, float b)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a, b}, bf16x2));
}

// h1 = relu(D1) as the four K steps of layer 2. Rounding to BF16 keeps the
// sign, so the ReLU is taken after it, on two BF16 values at once read as
// 16-bit integers (a set sign bit makes a negative integer, which becomes 0):
// the same values as rounding relu(D1), in half the instructions.
__device__ __forceinline__ void hidden_operand(const f32x16 (&d1)[2], bf16x8 (&h1)[4])
{
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        u32x4 u;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const uint32_t v = bf16_pair(d1[s / 2][l1_reg(s, 2 * p)], d1[s / 2][l1_reg(s, 2 * p + 1)]);
            u[p] = __builtin_bit_cast(uint32_t,
                                      __builtin_elementwise_max(__builtin_bit_cast(s16x2, v), (s16x2){0, 0}));
        }
        h1[s] = __builtin_bit_cast(bf16x8, u);
    }
}

__global__ __launch_bounds__(256) void mlp_forward_kernel(const float *__restrict__ P, const float *__restrict__ X,
                                                          uint64_t n, float *__restrict__ y,
                                                          uint8_t *__restrict__ outside,
                                                          const float *__restrict__ lo,
                                                          const float *__restrict__ hi,
                                                          unsigned long long *__restrict__ n_out)
{
    __shared__ unsigned long long s_cnt;
    // w3 in the order of the layer-2 result registers: [T][lane half][r]
    __shared__ float4 s_w3[2][2][4];
    const int lane = threadIdx.x & 63, half = lane >> 5, col = lane & 31;
    if (threadIdx.x == 0) s_cnt = 0;
    if (threadIdx.x < 64) {
        const int T = threadIdx.x >> 5, h = (threadIdx.x >> 4) & 1, r = threadIdx.x & 15;
        reinterpret_cast<float *>(&s_w3[T][h][0])[r] = P[OFF_W3 + 32 * T + d_row(r, h)];
    }
    NetOps o;
    load_ops(P, half, col, o);
    const bf16x8 ones = ones_pair(half == 0);
    const float b3 = P[OFF_B3];
    float flo[kFeat], fhi[kFeat];
#pragma unroll
    for (int e = 0; e < kFeat; ++e) {
        flo[e] = lo ? lo[e] : 0.0f;
        fhi[e] = lo ? hi[e] : 0.0f;
    }
    __syncthreads();
    // the wave's tiles are uniform: the loop and the tile's addresses stay
    // in scalar registers
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / 64);
    const uint64_t wave =
        (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6));
    const uint64_t tiles = (n + 31) / 32;
    uint32_t n_outside = 0;
    // Lane half 0 reads its cell's 8 features through a buffer view of the
    // tile's rows, which gives 0 for a row past the last cell; half 1 reads
    // past the view (zeros) and ORs in the pair (1, 1) that meets the b1 pair.
    // The next tile's features are loaded as soon as this tile's are rounded.
    const uint32_t voff = half == 0 ? 32u * (uint32_t)col : 1024u;
    const uint32_t ones_bits = half == 0 ? 0u : 0x3f803f80u;
    // rows of the tile starting at cell `first` (0 past the end)
    auto rows_at = [&](uint64_t first) -> uint32_t {
        return first < n ? (uint32_t)(n - first < 32 ? n - first : 32) : 0u;
    };
    auto load = [&](uint64_t tile, float (&x)[kFeat]) {
        const uint64_t first = tile * 32;
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(X + first * kFeat), (short)0, (int)(rows_at(first) * 32u), 0x00020000);
        // (streaming reads: the features are read once, and keeping them out
        // of the caches leaves those to the fields the features come from)
        const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, 0, kStreamingLoad);
        const u32x4 b = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff + 16, 0, kStreamingLoad);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            x[e] = __builtin_bit_cast(float, (uint32_t)a[e]);
            x[4 + e] = __builtin_bit_cast(float, (uint32_t)b[e]);
        }
    };
    // one tile from the features in x, loading those of tile + waves into
    // `next` (two register sets taken in turn, so nothing is copied)
    auto step = [&](uint64_t tile, const float (&x)[kFeat], float (&next)[kFeat]) {
        const uint64_t first = tile * 32;
        const uint32_t rows = rows_at(first);
        // the lanes whose features leave the envelope, as a wave mask taken
        // now, so that the features are not kept to the store (none without
        // an envelope)
        uint64_t env = 0;
        if (lo) {
            bool out_env = false;
#pragma unroll
            for (int e = 0; e < kFeat; ++e) out_env |= (x[e] < flo[e]) | (x[e] > fhi[e]);
            env = __ballot(out_env);
        }
        u32x4 bu;
#pragma unroll
        for (int p = 0; p < 4; ++p) bu[p] = bf16_pair(x[2 * p], x[2 * p + 1]);
        bu[0] |= ones_bits;
        const bf16x8 bx = __builtin_bit_cast(bf16x8, bu);
        load(tile + waves, next);
        f32x16 d1[2];
#pragma unroll
        for (int T = 0; T < 2; ++T) d1[T] = mfma16(o.a1[T], bx, zero16());
        bf16x8 h1[4];
        hidden_operand(d1, h1);
        f32x16 d2[2];
        // the wave issues its layer-2 products at raised priority, so that
        // the matrix cores start on them while the other waves' VALU work
        // (ReLU, conversions, the last layer) fills the SIMD around them
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int T = 0; T < 2; ++T) {
            d2[T] = mfma16(o.a2[T][4], ones, zero16());
#pragma unroll
            for (int s = 0; s < 4; ++s) d2[T] = mfma16(o.a2[T][s], h1[s], d2[T]);
        }
        __builtin_amdgcn_s_setprio(0);
        float part = 0.0f;
#pragma unroll
        for (int T = 0; T < 2; ++T)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float4 w = s_w3[T][half][q];
                part += w.x * relu(d2[T][4 * q]);
                part += w.y * relu(d2[T][4 * q + 1]);
                part += w.z * relu(d2[T][4 * q + 2]);
                part += w.w * relu(d2[T][4 * q + 3]);
            }
        part += __shfl_xor(part, 32, 64);
        if (half == 0 && (uint32_t)col < rows) {
            __builtin_nontemporal_store(part + b3, &y[first + (uint32_t)col]);
            if (outside) outside[first + (uint32_t)col] = (uint8_t)((env >> col) & 1u);
        }
        n_outside += (uint32_t)__popcll(env & (rows < 32 ? (1ull << rows) - 1ull : 0xffffffffull));
    };
    float xa[kFeat], xb[kFeat];
    load(wave, xa);
    for (uint64_t tile = wave; tile < tiles; tile += 2 * waves) {
        step(tile, xa, xb);
        if (tile + waves >= tiles) break;
        step(tile + waves, xb, xa);
    }
    if (n_out) {
        // n_outside is the wave's count
        const unsigned long long c = n_outside;
        if (lane == 0 && c) atomicAdd(&s_cnt, c);
        __syncthreads();
        if (threadIdx.x == 0 && s_cnt) atomicAdd(n_out, s_cnt);
    }
}

// ---- training: weighted-MSE gradient on the matrix cores --------------------
// The gradient of the function above with respect to the FP32 master
// parameters (every rounding passed through unchanged). Each tile of 32
// cells is evaluated in both orientations:
//   "C" gives y per lane and dL/dz2 with the output units in the registers,
//       the A operand of dL/dh1 = (dL/dz2)^T W2;
//   "H" gives h1 and dL/dz2 with the cells in the registers, the operands of
//       the weight gradients, which are sums over cells (K = cells):
//       dL/dW2 = (dL/dz2) H1^T and [dL/dW1 dL/db1] = (dL/dz1) [X 1].
// The error signals dL/dz2, dL/dz1 are rounded to BF16 for the matrix cores;
// the w3, b2 and b3 gradients are FP32 sums. X^T (feature per lane) and
// dL/dy per cell pass through a few hundred bytes of wave-private LDS, and
// the B operand of dL/dh1 (W2 with the output units in the registers) is
// read from the block's LDS.
//
// Each block of kGradWaves waves writes the sum of its waves' partial sums
// (in wave order) to its own slot; two more kernels add the slots in block
// order, so the result does not depend on timing.
constexpr int kGradWaves = 2;

struct GradLds {
    float w3[kHid];                              // by row, for "C"
    __bf16 w2[2][5][2][32][8];                   // a2[T][s] of lane (h, c) at [T][s][h][c]
    __bf16 w2t[2][4][2][32][8];                  // w3[o] W2[o][32 T + c], o = l2_unit(s, h, e), at [T][s][h][c][e]
    union {
        struct {
            __bf16 xs[kGradWaves][kFeat][32];    // the tile's features, [feature][cell]
            float gy[kGradWaves][32];            // dL/dy of the tile's cells
        } t;
        float part[kMlpPartStride];              // another wave's partial sums
    } u;
};

__global__ __launch_bounds__(64 * kGradWaves, 2) void mlp_grad_kernel(const float *__restrict__ P,
                                                                      const float *__restrict__ X,
                                                                      const float *__restrict__ tgt,
                                                                      const float *__restrict__ wgt, uint64_t n,
                                                                      float *__restrict__ partial)
{
    __shared__ GradLds L;
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63, half = lane >> 5, col = lane & 31;
    for (int j = threadIdx.x; j < kHid; j += blockDim.x) L.w3[j] = P[OFF_W3 + j];
    for (int j = threadIdx.x; j < kHid * kHid; j += blockDim.x) {
        const int e = j & 7, c = (j >> 3) & 31, h = (j >> 8) & 1, s = (j >> 9) & 3, T = j >> 11;
        const int o = l2_unit(s, h, e);
        L.w2t[T][s][h][c][e] = (__bf16)(P[OFF_W3 + o] * P[OFF_W2 + o * kHid + 32 * T + c]);
    }
    // the weight operands: layer 1 in registers, layer 2 in LDS (read as
    // needed; registers are short)
    NetOps o;
    load_ops(P, half, col, o);
#pragma unroll
    for (int T = 0; T < 2; ++T)
#pragma unroll
        for (int s = 0; s < 5; ++s)
            if (wid == 0) *reinterpret_cast<bf16x8 *>(&L.w2[T][s][half][col][0]) = o.a2[T][s];
    const bf16x8 ones = ones_pair(half == 0);
    auto a2 = [&](int T, int s) { return *reinterpret_cast<const bf16x8 *>(&L.w2[T][s][half][col][0]); };
    float w3h[2];                                // unit 32 T + col, for "H"
    w3h[0] = P[OFF_W3 + col];
    w3h[1] = P[OFF_W3 + 32 + col];
    const float b3 = P[OFF_B3];
    f32x16 gW2[2][2], gW1[2];
#pragma unroll
    for (int T = 0; T < 2; ++T) {
        gW1[T] = zero16();
        gW2[T][0] = zero16();
        gW2[T][1] = zero16();
    }
    float gw3[2] = {0.0f, 0.0f}, gb2[2] = {0.0f, 0.0f}, gb3 = 0.0f, loss = 0.0f, wsum = 0.0f;
    __syncthreads();

    __bf16(*xs)[32] = L.u.t.xs[wid];
    float *gys = L.u.t.gy[wid];
    const uint64_t waves = (uint64_t)gridDim.x * kGradWaves;
    const uint64_t tiles = (n + 31) / 32;
    for (uint64_t tile = (uint64_t)blockIdx.x * kGradWaves + wid; tile < tiles; tile += waves) {
        // the LDS tables are read in each tile, not held in registers across
        // tiles (the compiler may not hoist them past this)
        asm volatile("" ::: "memory");
        const uint64_t cell = tile * 32 + (uint64_t)col;
        const bool valid = cell < n;
        float x[kFeat];
        float tv = 0.0f, wv = 0.0f;                  // cells past n weigh nothing
        {
            float4 a = make_float4(0.0f, 0.0f, 0.0f, 0.0f), b = a;
            if (half == 0 && valid) {
                a = *reinterpret_cast<const float4 *>(X + cell * kFeat);
                b = *reinterpret_cast<const float4 *>(X + cell * kFeat + 4);
            }
            if (valid) {
                tv = tgt[cell];
                wv = wgt[cell];
            }
            x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
            x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
        }
        const bf16x8 bx = feature_operand(x, half);
        if (half == 0)
#pragma unroll
            for (int e = 0; e < kFeat; ++e) xs[e][col] = bx[e];

        // forward, "C"
        bf16x8 h1c[4];
        {
            f32x16 d1[2];
#pragma unroll
            for (int T = 0; T < 2; ++T) d1[T] = mfma16(o.a1[T], bx, zero16());
            hidden_operand(d1, h1c);
        }
        bf16x8 gzc[4];                 // dL/dz2 / w3, K operand of dL/dh1 (unit l2_unit(s, half, e))
        {
            f32x16 d2[2];
#pragma unroll
            for (int T = 0; T < 2; ++T) {
                d2[T] = mfma16(a2(T, 4), ones, zero16());
#pragma unroll
                for (int s = 0; s < 4; ++s) d2[T] = mfma16(a2(T, s), h1c[s], d2[T]);
            }
            float w3r[2][16];
#pragma unroll
            for (int T = 0; T < 2; ++T)
#pragma unroll
                for (int r = 0; r < 16; ++r) w3r[T][r] = L.w3[32 * T + d_row(r, half)];
            float part = 0.0f;
#pragma unroll
            for (int T = 0; T < 2; ++T)
#pragma unroll
                for (int r = 0; r < 16; ++r) part += w3r[T][r] * relu(d2[T][r]);
            part += __shfl_xor(part, 32, 64);
            const float res = part + b3 - tv;
            const float gy = 2.0f * wv * res;          // d(sum w r^2)/dy
            if (half == 0) {
                loss += wv * res * res;
                wsum += wv;
                gb3 += gy;
                gys[col] = gy;
            }
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int e = 0; e < 8; ++e) gzc[s][e] = (__bf16)(d2[s / 2][l1_reg(s, e)] > 0.0f ? gy : 0.0f);
        }

        // dL/dh1 = (dL/dz2)^T W2 ("H": cells in the registers), with w3
        // carried by the W2 operand
        f32x16 gh1[2];
#pragma unroll
        for (int T = 0; T < 2; ++T) {
            gh1[T] = zero16();
#pragma unroll
            for (int s = 0; s < 4; ++s)
                gh1[T] = mfma16(gzc[s], *reinterpret_cast<const bf16x8 *>(&L.w2t[T][s][half][col][0]), gh1[T]);
        }

        // X^T (feature per lane, element e of K step s' = cell
        // d_row(8 s' + e, half)) from the staged tile, with a column of ones
        bf16x8 xb[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if (col < kFeat) {
                // (read as the type it was written with: no type punning, so
                // the compiler keeps these loads after the stores above)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    xb[s][e] = xs[col][16 * s + 4 * half + e];
                    xb[s][4 + e] = xs[col][16 * s + 8 + 4 * half + e];
                }
            } else {
                const __bf16 v = (__bf16)(col == kFeat ? 1.0f : 0.0f);
#pragma unroll
                for (int e = 0; e < 8; ++e) xb[s][e] = v;
            }
        }

        // forward layer 1, "H": h1 with the cells in the registers (element e
        // of K step s' = register 8 s' + e); dL/dz1 through ReLU's derivative,
        // and [dL/dW1 dL/db1] += (dL/dz1) [X 1]
        bf16x8 h1h[2][2];
#pragma unroll
        for (int T = 0; T < 2; ++T) {
            const f32x16 d = mfma16(bx, o.a1[T], zero16());
            bf16x8 gz1[2];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                h1h[T][r / 8][r % 8] = (__bf16)relu(d[r]);
                gz1[r / 8][r % 8] = (__bf16)(d[r] > 0.0f ? gh1[T][r] : 0.0f);
            }
#pragma unroll
            for (int s = 0; s < 2; ++s) gW1[T] = mfma16(gz1[s], xb[s], gW1[T]);
        }

        // forward layer 2, "H": dL/dz2 / w3 with the cells in the registers
        // and the FP32 sums of the w3 and b2 gradients (w3, a factor of each
        // output unit's row, is applied to the dL/dW2 and dL/db2 sums at the
        // end)
        float gyr[16];                 // dL/dy of cell d_row(r, half)
#pragma unroll
        for (int r = 0; r < 16; ++r) gyr[r] = gys[d_row(r, half)];
#pragma unroll
        for (int To = 0; To < 2; ++To) {
            f32x16 d = mfma16(ones, a2(To, 4), zero16());
#pragma unroll
            for (int s = 0; s < 4; ++s) d = mfma16(h1c[s], a2(To, s), d);
            bf16x8 gzh[2];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float g = d[r] > 0.0f ? gyr[r] : 0.0f;
                gw3[To] += g * d[r];
                gb2[To] += g;
                gzh[r / 8][r % 8] = (__bf16)g;
            }
            // dL/dW2 += (dL/dz2) H1^T, K = the 32 cells in two steps
#pragma unroll
            for (int Ti = 0; Ti < 2; ++Ti)
#pragma unroll
                for (int s = 0; s < 2; ++s) gW2[To][Ti] = mfma16(gzh[s], h1h[Ti][s], gW2[To][Ti]);
        }
    }

    // this wave's sums: lanes col and col + 32 hold the two halves of the
    // cells of the unit sums; half 0 alone holds the per-cell sums
    gw3[0] += __shfl_xor(gw3[0], 32, 64);
    gw3[1] += __shfl_xor(gw3[1], 32, 64);
    gb2[0] = w3h[0] * (gb2[0] + __shfl_xor(gb2[0], 32, 64));
    gb2[1] = w3h[1] * (gb2[1] + __shfl_xor(gb2[1], 32, 64));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        gb3 += __shfl_down(gb3, off, 64);
        loss += __shfl_down(loss, off, 64);
        wsum += __shfl_down(wsum, off, 64);
    }
    // Every lane visits the entries it owns in the same order in every wave,
    // and the waves are added in index order through LDS.
    auto visit = [&](auto &&f) {
#pragma unroll
        for (int To = 0; To < 2; ++To)
#pragma unroll
            for (int Ti = 0; Ti < 2; ++Ti)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int o = 32 * To + d_row(r, half);
                    f(OFF_W2 + o * kHid + 32 * Ti + col, L.w3[o] * gW2[To][Ti][r]);
                }
        if (col <= kFeat)
#pragma unroll
            for (int T = 0; T < 2; ++T)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int u = 32 * T + d_row(r, half);
                    f(col < kFeat ? OFF_W1 + u * kFeat + col : OFF_B1 + u, gW1[T][r]);
                }
        if (half == 0)
#pragma unroll
            for (int T = 0; T < 2; ++T) {
                f(OFF_W3 + 32 * T + col, gw3[T]);
                f(OFF_B2 + 32 * T + col, gb2[T]);
            }
        if (lane == 0) {
            f(OFF_B3, gb3);
            f(kMlpParams, loss);
            f(kMlpParams + 1, wsum);
        }
    };
    __syncthreads();                                  // staging no longer in use
    for (int w = kGradWaves - 1; w > 0; --w) {
        if (wid == w) visit([&](int j, float v) { L.u.part[j] = (w == kGradWaves - 1 ? 0.0f : L.u.part[j]) + v; });
        __syncthreads();
    }
    if (wid == 0) {
        float *p = partial + (size_t)blockIdx.x * kMlpPartStride;
        visit([&](int j, float v) { p[j] = kGradWaves > 1 ? v + L.u.part[j] : v; });
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

// The correction with the Monte Carlo as fallback: a cell flagged outside the
// training envelope takes the Monte Carlo's M, every other exp(y).
__global__ __launch_bounds__(256) void mlp_correction_kernel(const float *__restrict__ y,
                                                             const uint8_t *__restrict__ outside,
                                                             const float *__restrict__ fallback, uint64_t n,
                                                             float *__restrict__ M)
{
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const bool mc = fallback && outside && outside[i];
    M[i] = mc ? fallback[i] : expf(y[i]);
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

int mlp_forward_blocks_per_cu()
{
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, mlp_forward_kernel, 256, 0) != hipSuccess || b < 1) b = 1;
    return b;
}

hipError_t launch_mlp_gradient(const float *params, const float *X, const float *t, const float *w, uint64_t n,
                               float *partial, int max_blocks, float *grad, hipStream_t s)
{
    // as many blocks as give every wave kGradMinTiles tiles, up to max_blocks:
    // fewer partial-sum slots to add for small batches (the count is a
    // function of n alone, so the summation order is too)
    constexpr uint64_t kGradMinTiles = 4;
    const uint64_t tiles = (n + 31) / 32;
    const int blocks = (int)std::max<uint64_t>(
        1, std::min<uint64_t>((uint64_t)max_blocks, tiles / (kGradWaves * kGradMinTiles)));
    const int groups = (blocks + kMlpGroup - 1) / kMlpGroup;
    float *tmp = partial + (size_t)blocks * kMlpPartStride;
    hipLaunchKernelGGL(mlp_grad_kernel, dim3((unsigned)blocks), dim3(64 * kGradWaves), 0, s, params, X, t, w, n,
                       partial);
    hipLaunchKernelGGL(mlp_reduce_groups_kernel, dim3((unsigned)((kMlpParams + 2 + 255) / 256), (unsigned)groups),
                       dim3(256), 0, s, partial, blocks, tmp);
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((unsigned)((kMlpParams + 2 + 255) / 256)), dim3(256), 0, s, tmp,
                       groups, grad);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void mlp_gather_kernel(const float *__restrict__ X, const float *__restrict__ t,
                                                         const float *__restrict__ w, uint64_t n_cells,
                                                         const int64_t *__restrict__ idx, uint64_t batch,
                                                         float *__restrict__ Xb, float *__restrict__ tb,
                                                         float *__restrict__ wb, unsigned int *__restrict__ bad)
{
    const uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    if (i >= batch) return;
    int64_t c = idx[i];
    if (c < 0 || (uint64_t)c >= n_cells) {
        atomicOr(bad, 1u);
        c = 0;
    }
#pragma unroll
    for (int e = 0; e < kFeat; ++e) Xb[i * kFeat + e] = X[(uint64_t)c * kFeat + e];
    tb[i] = t[c];
    wb[i] = w[c];
}

hipError_t launch_mlp_gather(const float *X, const float *t, const float *w, uint64_t n_cells, const int64_t *idx,
                             uint64_t batch, float *Xb, float *tb, float *wb, unsigned int *bad, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_gather_kernel, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, s, X, t, w, n_cells,
                       idx, batch, Xb, tb, wb, bad);
    return hipGetLastError();
}

hipError_t launch_mlp_correction(const float *y, const uint8_t *outside, const float *fallback, uint64_t n,
                                 float *M, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_correction_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, y, outside,
                       fallback, n, M);
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

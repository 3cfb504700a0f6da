// Per-cell setup kernels: pack the fields into walk records (kappa_c and the
// bulk velocity), reduce the per-box quantities the walk needs, quantise the
// emission weights and allocate packets to cells.
//
// Grids are two-dimensional: blockIdx.y is the box, blockIdx.x a block of
// cells inside it, so every per-box reduction sees the same partition whether
// the box runs alone or inside a batch (bitwise-identical results).
#include "common.hpp"

namespace mclya {
namespace {

constexpr int B = kSetupBlock;
constexpr int kWaves = B / 64;

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    return v;
}

__device__ __forceinline__ uint32_t wave_or(uint32_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v |= __shfl_down(v, off, 64);
    return v;
}

// Deterministic block sum: waves reduce by shuffles, wave totals are added in
// wave order by thread 0. Result valid in thread 0.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T *lds)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    T t = 0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < kWaves; ++w) t += lds[w];
    }
    return t;
}

// Block maximum (order independent). Result valid in thread 0.
__device__ __forceinline__ double block_max(double v, double *lds)
{
    v = wave_max(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < kWaves; ++w) t = fmax(t, lds[w]);
    }
    return t;
}

// Inclusive scan of a 64-bit value across the block; also returns the block
// total through *total (all threads).
__device__ __forceinline__ uint64_t block_inclusive_scan(uint64_t v, uint64_t *lds, uint64_t *total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint64_t o = __shfl_up(v, off, 64);
        if (lane >= off) v += o;
    }
    __syncthreads();
    if (lane == 63) lds[wid] = v;
    __syncthreads();
    uint64_t before = 0, all = 0;
    for (int w = 0; w < kWaves; ++w) {
        if (w < wid) before += lds[w];
        all += lds[w];
    }
    *total = all;
    return v + before;
}

__device__ __forceinline__ bool finite_f(float v) { return __builtin_isfinite(v); }

// -------------------------------------------------------------------------
// Pack: kappa_c = kappa_unit (1 - x_e) Delta (mean true-absorption depth of
// Eq. (<fnu>) with the cell's n_1s), the velocity, and the emission weight
// S_c (the given source, else (x_e Delta)^2, proportional to alpha_e n_e^2).
// -------------------------------------------------------------------------
template <bool VREC>
__global__ __launch_bounds__(B) void pack_kernel(const PackBox *__restrict__ pbs, void *__restrict__ rec,
                                                 double *__restrict__ wgt,
                                                 double *__restrict__ partials, BoxRed *red,
                                                 int max_blk)
{
    __shared__ double lds[kWaves];
    const int b = blockIdx.y;
    const PackBox pb = pbs[b];
    if ((int)blockIdx.x >= pb.nblk) return;
    const uint32_t i = blockIdx.x * B + threadIdx.x;
    double ux = 0.0, uy = 0.0, uz = 0.0, ks = 0.0, w = 0.0, d1 = 0.0, d2 = 0.0;
    uint32_t flags = 0;
    if (i < pb.ncells) {
        const float od = pb.od[i];
        const float xe = pb.xe ? pb.xe[i] : pb.xe_uniform;
        if (!(od >= 0.0f) || !finite_f(od)) flags |= FLAG_OD_BAD;
        if (!(xe >= 0.0f && xe <= 1.2f)) flags |= FLAG_XE_BAD;
        float vx = 0.0f, vy = 0.0f, vz = 0.0f;
        if (pb.vel_dtype == MC_LYA_VEL_F32) {
            const float *v = static_cast<const float *>(pb.vel);
            vx = v[i];
            vy = v[(size_t)pb.ncells + i];
            vz = v[2 * (size_t)pb.ncells + i];
        } else if (pb.vel_dtype == MC_LYA_VEL_F16) {
            const _Float16 *v = static_cast<const _Float16 *>(pb.vel);
            vx = (float)v[i];
            vy = (float)v[(size_t)pb.ncells + i];
            vz = (float)v[2 * (size_t)pb.ncells + i];
        }
        if (!finite_f(vx) || !finite_f(vy) || !finite_f(vz)) flags |= FLAG_VEL_BAD;
        const double kap = pb.kappa_unit * (1.0 - (double)xe) * (double)od;
        if (pb.src) {
            const float s = pb.src[i];
            if (!(s >= 0.0f) || !finite_f(s)) flags |= FLAG_SRC_BAD;
            w = (double)s;
        } else {
            const double m = (double)xe * (double)od;   // exact product of two binary32 values
            w = m * m;
        }
        const size_t g = (size_t)pb.cell_off + i;
        if (VREC)
            static_cast<float4 *>(rec)[g] = make_float4((float)kap, vx, vy, vz);
        else
            static_cast<float *>(rec)[g] = (float)kap;
        wgt[g] = w;
        ux = vx;
        uy = vy;
        uz = vz;
        ks = kap;
        d1 = (double)od;
        d2 = d1 * d1;
    }
    const double sx = block_sum(ux, lds);
    const double sy = block_sum(uy, lds);
    const double sz = block_sum(uz, lds);
    const double sk = block_sum(ks, lds);
    const double sd1 = block_sum(d1, lds);
    const double sd2 = block_sum(d2, lds);
    const double wm = block_max(w, lds);
    // validation failures are rare: an atomic only where one is found
    const uint32_t fl = wave_or(flags);
    if ((threadIdx.x & 63) == 0 && fl) atomicOr(&red[b].flags, fl);
    if (threadIdx.x == 0) {
        double *p = partials + ((size_t)b * max_blk + blockIdx.x) * kPartStride;
        p[0] = sx;
        p[1] = sy;
        p[2] = sz;
        p[3] = sk;
        p[4] = wm;
        p[7] = sd1;
        p[8] = sd2;
    }
}

// One block per box: add the block partials in a fixed order.
__global__ __launch_bounds__(B) void box_reduce_kernel(const PackBox *__restrict__ pbs,
                                                       const double *__restrict__ partials,
                                                       BoxRed *red, int max_blk)
{
    __shared__ double lds[kWaves];
    const int b = blockIdx.x;
    const int nblk = pbs[b].nblk;
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double wm = 0.0;
    for (int k = threadIdx.x; k < nblk; k += B) {
        const double *p = partials + ((size_t)b * max_blk + k) * kPartStride;
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] += p[j];
        acc[4] += p[7];
        acc[5] += p[8];
        wm = fmax(wm, p[4]);
    }
    double tot[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) tot[j] = block_sum(acc[j], lds);
    wm = block_max(wm, lds);
    if (threadIdx.x == 0) {
        red[b].usum[0] = tot[0];
        red[b].usum[1] = tot[1];
        red[b].usum[2] = tot[2];
        red[b].kappa_sum = tot[3];
        red[b].od_sum = tot[4];
        red[b].od2_sum = tot[5];
        red[b].wmax_bits = (unsigned long long)__double_as_longlong(wm);
    }
}

// max_c |U_c - <U>| per box (order independent): block maxima, then one
// block per box.
__global__ __launch_bounds__(B) void margin_kernel(const PackBox *__restrict__ pbs,
                                                   const float4 *__restrict__ rec, const BoxRed *red,
                                                   double *__restrict__ partials, int max_blk)
{
    __shared__ double lds[kWaves];
    const int b = blockIdx.y;
    const PackBox pb = pbs[b];
    if ((int)blockIdx.x >= pb.nblk) return;
    const uint32_t i = blockIdx.x * B + threadIdx.x;
    const double n = (double)pb.ncells;
    double dev = 0.0;
    if (i < pb.ncells) {
        const float4 r = rec[(size_t)pb.cell_off + i];
        // mean by division: exact for a uniform field
        const double mx = red[b].usum[0] / n, my = red[b].usum[1] / n, mz = red[b].usum[2] / n;
        const double dx = (double)r.y - mx, dy = (double)r.z - my, dz = (double)r.w - mz;
        dev = sqrt(dx * dx + dy * dy + dz * dz);
    }
    dev = block_max(dev, lds);
    if (threadIdx.x == 0) partials[((size_t)b * max_blk + blockIdx.x) * kPartStride + 5] = dev;
}

__global__ __launch_bounds__(B) void margin_reduce_kernel(const PackBox *__restrict__ pbs,
                                                          const double *__restrict__ partials, BoxRed *red,
                                                          int max_blk)
{
    __shared__ double lds[kWaves];
    const int b = blockIdx.x;
    const int nblk = pbs[b].nblk;
    double m = 0.0;
    for (int k = threadIdx.x; k < nblk; k += B) m = fmax(m, partials[((size_t)b * max_blk + k) * kPartStride + 5]);
    m = block_max(m, lds);
    if (threadIdx.x == 0) red[b].udev_bits = (unsigned long long)__double_as_longlong(m);
}

// -------------------------------------------------------------------------
// Quantise: q_c = floor(2^32 S_c / max S) in binary64 (one correctly rounded
// division, an exact power-of-two scaling, a floor), and the block sums.
// -------------------------------------------------------------------------
__global__ __launch_bounds__(B) void quantize_kernel(const PackBox *__restrict__ pbs,
                                                     const double *__restrict__ wgt,
                                                     const BoxRed *__restrict__ red,
                                                     uint64_t *__restrict__ q,
                                                     uint64_t *__restrict__ bsum, int max_blk)
{
    __shared__ uint64_t lds[kWaves];
    const int b = blockIdx.y;
    const PackBox pb = pbs[b];
    if ((int)blockIdx.x >= pb.nblk) return;
    const uint32_t i = blockIdx.x * B + threadIdx.x;
    const double wmax = __longlong_as_double((long long)red[b].wmax_bits);
    uint64_t v = 0;
    if (i < pb.ncells && wmax > 0.0) {
        const size_t g = (size_t)pb.cell_off + i;
        const double ratio = wgt[g] / wmax;   // IEEE division (no fast-math)
        v = (uint64_t)floor(ratio * 4294967296.0);
        q[g] = v;
    } else if (i < pb.ncells) {
        q[(size_t)pb.cell_off + i] = 0;
    }
    const uint64_t s = block_sum(v, lds);
    if (threadIdx.x == 0) bsum[(size_t)b * max_blk + blockIdx.x] = s;
}

// One block per box: exclusive scan of the block sums (in place) and the box
// total.
__global__ __launch_bounds__(B) void scan_blocks_kernel(const PackBox *__restrict__ pbs,
                                                        uint64_t *__restrict__ bsum, BoxRed *red,
                                                        int max_blk)
{
    __shared__ uint64_t lds[kWaves];
    const int b = blockIdx.x;
    const int nblk = pbs[b].nblk;
    uint64_t carry = 0;
    for (int base = 0; base < nblk; base += B) {
        const int k = base + threadIdx.x;
        uint64_t *p = bsum + (size_t)b * max_blk + k;
        const uint64_t v = k < nblk ? *p : 0;
        uint64_t tot;
        const uint64_t inc = block_inclusive_scan(v, lds, &tot);
        if (k < nblk) *p = carry + inc - v;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) red[b].qtot = carry;
}

// Packets p in [0, N) with systematic point floor((2p+1) Qtot / 2N) below Q:
// the odd integers o with o Qtot < 2 N Q, i.e. floor(ceil(2 N Q / Qtot) / 2).
// ceil(m / qtot) is below 2n < 2^41 (Q <= qtot): a binary64 quotient is
// within one of it, and exact 128-bit products settle it (no 128-bit
// division).
__device__ __forceinline__ uint64_t count_below(uint64_t Q, uint64_t qtot, uint64_t n)
{
    const unsigned __int128 m = (unsigned __int128)(2u * n) * Q;
    const double md = (double)(uint64_t)(m >> 64) * 18446744073709551616.0 + (double)(uint64_t)m;
    uint64_t c = (uint64_t)(md / (double)qtot);
    unsigned __int128 prod = (unsigned __int128)c * qtot;
    while (prod < m) {
        ++c;
        prod += qtot;
    }
    while (c > 0 && prod - qtot >= m) {
        --c;
        prod -= qtot;
    }
    return c >> 1;
}

// Allocation: each cell learns its first packet id and its count.
__global__ __launch_bounds__(B) void allocate_kernel(const PackBox *__restrict__ pbs,
                                                     const WalkBox *__restrict__ wbs,
                                                     const uint64_t *__restrict__ q,
                                                     const uint64_t *__restrict__ bsum,
                                                     const BoxRed *__restrict__ red,
                                                     uint32_t *__restrict__ npk,
                                                     uint64_t *__restrict__ pfirst, int max_blk)
{
    __shared__ uint64_t lds[kWaves];
    const int b = blockIdx.y;
    const PackBox pb = pbs[b];
    if ((int)blockIdx.x >= pb.nblk) return;
    const uint32_t i = blockIdx.x * B + threadIdx.x;
    const size_t g = (size_t)pb.cell_off + i;
    const uint64_t v = i < pb.ncells ? q[g] : 0;
    uint64_t tot;
    const uint64_t inc = block_inclusive_scan(v, lds, &tot);
    if (i >= pb.ncells) return;
    const uint64_t n = wbs[b].npkt;
    const uint64_t qtot = red[b].qtot;
    if (n == 0 || qtot == 0) {
        npk[g] = 0;
        pfirst[g] = wbs[b].pkt_off;
        return;
    }
    const uint64_t Q = bsum[(size_t)b * max_blk + blockIdx.x] + inc - v;
    const uint64_t first = count_below(Q, qtot, n);
    const uint64_t next = count_below(Q + v, qtot, n);
    const uint32_t cnt = (uint32_t)(next - first);
    npk[g] = cnt;
    pfirst[g] = wbs[b].pkt_off + first;
}

// The cell of every packet id (for the walks that take packets by id rather
// than by cell): cell g writes its index over its packet range.
__global__ __launch_bounds__(B) void cell_of_packet_kernel(const PackBox *__restrict__ pbs,
                                                           const uint32_t *__restrict__ npk,
                                                           const uint64_t *__restrict__ pfirst,
                                                           uint32_t *__restrict__ cop)
{
    const int b = blockIdx.y;
    const PackBox pb = pbs[b];
    if ((int)blockIdx.x >= pb.nblk) return;
    const uint32_t i = blockIdx.x * B + threadIdx.x;
    if (i >= pb.ncells) return;
    const size_t g = (size_t)pb.cell_off + i;
    const uint32_t cnt = npk[g];
    uint32_t *dst = cop + pfirst[g];
    for (uint32_t k = 0; k < cnt; ++k) dst[k] = (uint32_t)g;
}

inline dim3 grid2(int max_blk, int n_boxes) { return dim3((unsigned)max_blk, (unsigned)n_boxes, 1); }

}  // namespace

hipError_t launch_pack(const PackBox *pb_dev, int n_boxes, int max_blk, bool vel_rec, void *rec,
                       double *wgt, double *partials, BoxRed *red, hipStream_t s)
{
    if (vel_rec)
        hipLaunchKernelGGL(pack_kernel<true>, grid2(max_blk, n_boxes), dim3(B), 0, s, pb_dev, rec, wgt,
                           partials, red, max_blk);
    else
        hipLaunchKernelGGL(pack_kernel<false>, grid2(max_blk, n_boxes), dim3(B), 0, s, pb_dev, rec, wgt,
                           partials, red, max_blk);
    return hipGetLastError();
}

hipError_t launch_box_reduce(const PackBox *pb_dev, int n_boxes, int max_blk, const double *partials,
                             BoxRed *red, hipStream_t s)
{
    hipLaunchKernelGGL(box_reduce_kernel, dim3((unsigned)n_boxes), dim3(B), 0, s, pb_dev, partials, red,
                       max_blk);
    return hipGetLastError();
}

hipError_t launch_margin(const PackBox *pb_dev, int n_boxes, int max_blk, const float4 *rec, BoxRed *red,
                         double *partials, hipStream_t s)
{
    hipLaunchKernelGGL(margin_kernel, grid2(max_blk, n_boxes), dim3(B), 0, s, pb_dev, rec, red, partials,
                       max_blk);
    hipLaunchKernelGGL(margin_reduce_kernel, dim3((unsigned)n_boxes), dim3(B), 0, s, pb_dev, partials, red,
                       max_blk);
    return hipGetLastError();
}

hipError_t launch_quantize(const PackBox *pb_dev, int n_boxes, int max_blk, const double *wgt,
                           const BoxRed *red, uint64_t *q, uint64_t *bsum, hipStream_t s)
{
    hipLaunchKernelGGL(quantize_kernel, grid2(max_blk, n_boxes), dim3(B), 0, s, pb_dev, wgt, red, q, bsum,
                       max_blk);
    return hipGetLastError();
}

hipError_t launch_scan_blocks(const PackBox *pb_dev, int n_boxes, int max_blk, uint64_t *bsum, BoxRed *red,
                              hipStream_t s)
{
    hipLaunchKernelGGL(scan_blocks_kernel, dim3((unsigned)n_boxes), dim3(B), 0, s, pb_dev, bsum, red,
                       max_blk);
    return hipGetLastError();
}

hipError_t launch_allocate(const PackBox *pb_dev, const WalkBox *wb_dev, int n_boxes, int max_blk,
                           const uint64_t *q, const uint64_t *bsum, const BoxRed *red, uint32_t *npk,
                           uint64_t *pfirst, hipStream_t s)
{
    hipLaunchKernelGGL(allocate_kernel, grid2(max_blk, n_boxes), dim3(B), 0, s, pb_dev, wb_dev, q, bsum, red,
                       npk, pfirst, max_blk);
    return hipGetLastError();
}

hipError_t launch_cell_of_packet(const PackBox *pb_dev, int n_boxes, int max_blk, const uint32_t *npk,
                                 const uint64_t *pfirst, uint32_t *cell_of_packet, hipStream_t s)
{
    hipLaunchKernelGGL(cell_of_packet_kernel, grid2(max_blk, n_boxes), dim3(B), 0, s, pb_dev, npk, pfirst,
                       cell_of_packet);
    return hipGetLastError();
}

}  // namespace mclya

// Tally finalisation and the recombination feed.
//
// tally_kernel copies the int64 per-cell tallies out and sums them per box
// (integer sums, so the conservation identity is checked exactly).
// feed kernels turn the tallies into the per-cell recombination rate of
// Eq. (rec) / Eq. (dotne-mix) (Sec. III.A.1, IV.B) and the mixing correction.
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

__global__ __launch_bounds__(B) void tally_kernel(const WalkBox *__restrict__ wbs,
                                                  const unsigned long long *__restrict__ A,
                                                  const uint32_t *__restrict__ npk,
                                                  int64_t *__restrict__ absorbed_out,
                                                  int64_t *__restrict__ emitted_out,
                                                  double *__restrict__ partials, int max_blk)
{
    __shared__ unsigned long long lds[kWaves];
    const int b = blockIdx.y;
    const WalkBox wb = wbs[b];
    if (blockIdx.x * (uint32_t)B >= wb.cells()) return;
    const uint32_t i = blockIdx.x * B + threadIdx.x;
    unsigned long long a = 0;
    if (i < wb.cells()) {
        const size_t g = (size_t)wb.cell_off + i;
        a = A[g];
        if (absorbed_out) absorbed_out[g] = (int64_t)a;
        if (emitted_out) emitted_out[g] = (int64_t)((uint64_t)npk[g] * wb.w0);
    }
    const unsigned long long s = block_sum(a, lds);
    if (threadIdx.x == 0)
        reinterpret_cast<unsigned long long *>(partials)[((size_t)b * max_blk + blockIdx.x) * kPartStride + 6] = s;
}

// One block per box: the integer sum of the block sums (exact in any order).
__global__ __launch_bounds__(B) void tally_reduce_kernel(const WalkBox *__restrict__ wbs,
                                                         const double *__restrict__ partials,
                                                         unsigned long long *__restrict__ box_abs, int max_blk)
{
    __shared__ unsigned long long lds[kWaves];
    const int b = blockIdx.x;
    const uint32_t nblk = (wbs[b].cells() + B - 1) / B;
    const unsigned long long *p = reinterpret_cast<const unsigned long long *>(partials);
    unsigned long long a = 0;
    for (uint32_t k = threadIdx.x; k < nblk; k += B) a += p[((size_t)b * max_blk + k) * kPartStride + 6];
    a = block_sum(a, lds);
    if (threadIdx.x == 0) box_abs[b] = a;
}

// Per block: sum of weights, of (1 - x_e) Delta, of x_e Delta and of Delta.
__global__ __launch_bounds__(B) void feed_sums_kernel(const PackBox *__restrict__ pbs,
                                                      const double *__restrict__ wgt,
                                                      double *__restrict__ partials, int max_blk)
{
    __shared__ double lds[kWaves];
    const int b = blockIdx.y;
    const PackBox pb = pbs[b];
    if ((int)blockIdx.x >= pb.nblk) return;
    const uint32_t i = blockIdx.x * B + threadIdx.x;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (i < pb.ncells) {
        const double od = (double)pb.od[i];
        const double xe = (double)(pb.xe ? pb.xe[i] : pb.xe_uniform);
        s0 = wgt[(size_t)pb.cell_off + i];
        s1 = (1.0 - xe) * od;
        s2 = xe * od;
        s3 = od;
    }
    const double t0 = block_sum(s0, lds);
    const double t1 = block_sum(s1, lds);
    const double t2 = block_sum(s2, lds);
    const double t3 = block_sum(s3, lds);
    if (threadIdx.x == 0) {
        double *p = partials + ((size_t)b * max_blk + blockIdx.x) * kPartStride;
        p[0] = t0;
        p[1] = t1;
        p[2] = t2;
        p[3] = t3;
    }
}

// One block per box: fixed-order sum of the block partials.
__global__ __launch_bounds__(B) void reduce4_kernel(const PackBox *__restrict__ pbs,
                                                    const double *__restrict__ partials,
                                                    double *__restrict__ sums, int max_blk)
{
    __shared__ double lds[kWaves];
    const int b = blockIdx.x;
    const int nblk = pbs[b].nblk;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < nblk; k += B) {
        const double *p = partials + ((size_t)b * max_blk + k) * kPartStride;
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] += p[j];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const double t = block_sum(acc[j], lds);
        if (threadIdx.x == 0) sums[4 * b + j] = t;
    }
}

// ndot_e,c = -S_c + beta/(beta+Lambda) a_c + C_MC beta n_1s,c exp(-E_alpha/kT)
// M_c = A_c / (sum(A) n_1s,c / sum(n_1s))
__global__ __launch_bounds__(B) void feed_kernel(const PackBox *__restrict__ pbs,
                                                 const FeedBox *__restrict__ fbs,
                                                 const double *__restrict__ wgt,
                                                 const unsigned long long *__restrict__ A,
                                                 double *__restrict__ ndot, float *__restrict__ mix)
{
    const int b = blockIdx.y;
    const PackBox pb = pbs[b];
    if ((int)blockIdx.x >= pb.nblk) return;
    const uint32_t i = blockIdx.x * B + threadIdx.x;
    if (i >= pb.ncells) return;
    const FeedBox fb = fbs[b];
    const size_t g = (size_t)pb.cell_off + i;
    const double od = (double)pb.od[i];
    const double xe = (double)(pb.xe ? pb.xe[i] : pb.xe_uniform);
    const double n1s = fb.n_h * (1.0 - xe) * od;
    // the far damping wing's share is spread like n_1s (fully mixed)
    const double a = (double)A[g] + fb.wing_n1s * n1s;
    if (ndot) ndot[g] = -fb.S_scale * wgt[g] + fb.reion * (a * fb.a_norm) + fb.thermal * n1s;
    if (mix) {
        const double fm = fb.fm_norm * n1s;
        mix[g] = fm > 0.0 ? (float)(a / fm) : 0.0f;
    }
}

// The surrogate's regression data: the log of the mixing correction the
// feed forms (M_c = A_c / A_c^fm) and the weight of the cell in the loss, its
// share of the box's emission S_c / sum(S) (the cells that feed recombination
// most count most). A cell with M_c = 0 (nothing absorbed there) has no
// logarithm and gets weight 0.
__global__ __launch_bounds__(B) void targets_kernel(const PackBox *__restrict__ pbs,
                                                    const FeedBox *__restrict__ fbs,
                                                    const double *__restrict__ wgt,
                                                    const unsigned long long *__restrict__ A,
                                                    float *__restrict__ y, float *__restrict__ w)
{
    const int b = blockIdx.y;
    const PackBox pb = pbs[b];
    if ((int)blockIdx.x >= pb.nblk) return;
    const uint32_t i = blockIdx.x * B + threadIdx.x;
    if (i >= pb.ncells) return;
    const FeedBox fb = fbs[b];
    const size_t g = (size_t)pb.cell_off + i;
    const double od = (double)pb.od[i];
    const double xe = (double)(pb.xe ? pb.xe[i] : pb.xe_uniform);
    const double n1s = fb.n_h * (1.0 - xe) * od;
    const double a = (double)A[g] + fb.wing_n1s * n1s;
    const double fm = fb.fm_norm * n1s;
    const double m = fm > 0.0 ? a / fm : 0.0;
    const bool ok = m > 0.0;
    y[g] = ok ? (float)log(m) : 0.0f;
    w[g] = ok ? (float)(wgt[g] * fb.w_inv) : 0.0f;
}

inline dim3 grid2(int max_blk, int n_boxes) { return dim3((unsigned)max_blk, (unsigned)n_boxes, 1); }

}  // namespace

hipError_t launch_tally(const WalkBox *wb_dev, int n_boxes, int max_blk, const unsigned long long *A,
                        const uint32_t *npk, int64_t *absorbed_out, int64_t *emitted_out,
                        double *partials, unsigned long long *box_abs, hipStream_t s)
{
    hipLaunchKernelGGL(tally_kernel, grid2(max_blk, n_boxes), dim3(B), 0, s, wb_dev, A, npk, absorbed_out,
                       emitted_out, partials, max_blk);
    hipLaunchKernelGGL(tally_reduce_kernel, dim3((unsigned)n_boxes), dim3(B), 0, s, wb_dev, partials, box_abs,
                       max_blk);
    return hipGetLastError();
}

hipError_t launch_feed_sums(const PackBox *pb_dev, int n_boxes, int max_blk, const double *wgt,
                            double *partials, hipStream_t s)
{
    hipLaunchKernelGGL(feed_sums_kernel, grid2(max_blk, n_boxes), dim3(B), 0, s, pb_dev, wgt, partials,
                       max_blk);
    return hipGetLastError();
}

hipError_t launch_feed_reduce(int n_boxes, int max_blk, const PackBox *pb_dev, const double *partials,
                              double *sums, hipStream_t s)
{
    hipLaunchKernelGGL(reduce4_kernel, dim3((unsigned)n_boxes), dim3(B), 0, s, pb_dev, partials, sums,
                       max_blk);
    return hipGetLastError();
}

hipError_t launch_targets(const PackBox *pb_dev, const FeedBox *fb_dev, int n_boxes, int max_blk,
                          const double *wgt, const unsigned long long *A, float *y, float *w, hipStream_t s)
{
    hipLaunchKernelGGL(targets_kernel, grid2(max_blk, n_boxes), dim3(B), 0, s, pb_dev, fb_dev, wgt, A, y, w);
    return hipGetLastError();
}

hipError_t launch_feed(const PackBox *pb_dev, const FeedBox *fb_dev, int n_boxes, int max_blk,
                       const double *wgt, const unsigned long long *A, double *ndot, float *mix,
                       hipStream_t s)
{
    hipLaunchKernelGGL(feed_kernel, grid2(max_blk, n_boxes), dim3(B), 0, s, pb_dev, fb_dev, wgt, A, ndot,
                       mix);
    return hipGetLastError();
}

}  // namespace mclya

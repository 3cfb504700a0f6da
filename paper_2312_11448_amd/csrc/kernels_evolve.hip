// Recombination history driven by the Monte-Carlo feed (Sec. III.A.1,
// Sec. IV.B): per-cell free-electron fractions advanced in redshift by the
// classic fourth-order Runge-Kutta method. The library's driver runs each
// stage as a whole emit - transport - feed; these kernels turn the feed's
// net rate into dx_e/dz and combine the stages.
#include "common.hpp"

namespace mclya {
namespace {

constexpr int B = kSetupBlock;

// y[g] = x_e of every cell of every box (the caller's fields), in binary64.
__global__ __launch_bounds__(B) void xe_load_kernel(const PackBox *__restrict__ pbs, double *__restrict__ y)
{
    const int b = blockIdx.y;
    const PackBox pb = pbs[b];
    if ((int)blockIdx.x >= pb.nblk) return;
    const uint32_t i = blockIdx.x * B + threadIdx.x;
    if (i >= pb.ncells) return;
    y[(size_t)pb.cell_off + i] = (double)pb.xe[i];
}

// dx_e/dz = -ndot_e / (n_H Delta (1 + z) H) per cell: coef[b] holds
// -1 / (n_H (1 + z) H) of box b at the stage's redshift. Cells without
// hydrogen keep their x_e.
__global__ __launch_bounds__(B) void xe_rate_kernel(const PackBox *__restrict__ pbs, const double *__restrict__ coef,
                                                    const double *__restrict__ ndot, double *__restrict__ k)
{
    const int b = blockIdx.y;
    const PackBox pb = pbs[b];
    if ((int)blockIdx.x >= pb.nblk) return;
    const uint32_t i = blockIdx.x * B + threadIdx.x;
    if (i >= pb.ncells) return;
    const size_t g = (size_t)pb.cell_off + i;
    const double od = (double)pb.od[i];
    k[g] = od > 0.0 ? coef[b] * ndot[g] / od : 0.0;
}

// y_out = y0 + sum_j w_j k_j (j < nk) over every cell; with `field` the
// caller's x_e arrays receive the result in binary32, kept inside [0, 1]
// (an intermediate stage can overshoot by a rounding).
struct Combine {
    const double *k[4];
    double w[4];
    int nk;
};

__global__ __launch_bounds__(B) void xe_combine_kernel(const PackBox *__restrict__ pbs, const double *__restrict__ y0,
                                                       Combine cmb, double *__restrict__ y_out, int field)
{
    const int b = blockIdx.y;
    const PackBox pb = pbs[b];
    if ((int)blockIdx.x >= pb.nblk) return;
    const uint32_t i = blockIdx.x * B + threadIdx.x;
    if (i >= pb.ncells) return;
    const size_t g = (size_t)pb.cell_off + i;
    double y = y0[g];
    for (int j = 0; j < cmb.nk; ++j) y += cmb.w[j] * cmb.k[j][g];
    if (y_out) y_out[g] = y;
    if (field) const_cast<float *>(pb.xe)[i] = (float)fmin(fmax(y, 0.0), 1.0);
}

inline dim3 grid2(int max_blk, int n_boxes) { return dim3((unsigned)max_blk, (unsigned)n_boxes, 1); }

}  // namespace

hipError_t launch_xe_load(const PackBox *pb_dev, int n_boxes, int max_blk, double *y, hipStream_t s)
{
    hipLaunchKernelGGL(xe_load_kernel, grid2(max_blk, n_boxes), dim3(B), 0, s, pb_dev, y);
    return hipGetLastError();
}

hipError_t launch_xe_rate(const PackBox *pb_dev, int n_boxes, int max_blk, const double *coef, const double *ndot,
                          double *k, hipStream_t s)
{
    hipLaunchKernelGGL(xe_rate_kernel, grid2(max_blk, n_boxes), dim3(B), 0, s, pb_dev, coef, ndot, k);
    return hipGetLastError();
}

hipError_t launch_xe_combine(const PackBox *pb_dev, int n_boxes, int max_blk, const double *y0,
                             const double *const *k, const double *w, int nk, double *y_out, bool field,
                             hipStream_t s)
{
    Combine c{};
    c.nk = nk;
    for (int j = 0; j < nk && j < 4; ++j) {
        c.k[j] = k[j];
        c.w[j] = w[j];
    }
    hipLaunchKernelGGL(xe_combine_kernel, grid2(max_blk, n_boxes), dim3(B), 0, s, pb_dev, y0, c, y_out,
                       field ? 1 : 0);
    return hipGetLastError();
}

}  // namespace mclya

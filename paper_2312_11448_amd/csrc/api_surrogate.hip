// C ABI of the mixing-correction surrogate network (see mc_lya.h): a small
// object holding the FP32 parameters, the Adam moments, the feature envelope
// and the gradient workspace on one device and stream.
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"

using namespace mclya;

struct mc_lya_mlp {
    hipStream_t stream = nullptr;
    float *d_params = nullptr, *d_m = nullptr, *d_v = nullptr;
    float *d_grad = nullptr;                 // [kMlpParams + 2]: gradient, sum w r^2, sum w
    float *d_part = nullptr;                 // [kMlpGradBlocks + kMlpGradBlocks / 32][kMlpPartStride]
    float *d_env = nullptr;                  // [16]: lower then upper feature bounds
    unsigned long long *d_count = nullptr;
    bool envelope = false;
    int64_t step = 0;
    int forward_grid = 0;
    // mc_lya_mlp_train_steps: the gathered batch ([cap][8] + [cap] + [cap]),
    // the index-range flag, and two floats of loss tail per step
    float *d_batch = nullptr;
    uint64_t batch_cap = 0;
    unsigned int *d_bad = nullptr;
    float *d_tails = nullptr;
    int tails_cap = 0;
    std::string err;
};

namespace mclya {
// (kernels_surrogate.hip) rows idx[0..batch) of (X [.][8], t, w) into
// (Xb, tb, wb); an index outside [0, n_cells) reads row 0 and sets *bad
hipError_t launch_mlp_gather(const float *X, const float *t, const float *w, uint64_t n_cells, const int64_t *idx,
                             uint64_t batch, float *Xb, float *tb, float *wb, unsigned int *bad, hipStream_t s);
}  // namespace mclya

namespace {

thread_local std::string g_mlp_init_err;

mc_lya_status mlp_fail(mc_lya_mlp *m, mc_lya_status s, const std::string &what)
{
    m->err = what;
    return s;
}

mc_lya_status mlp_hip(mc_lya_mlp *m, hipError_t e, const char *what)
{
    m->err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? MC_LYA_ENOMEM : MC_LYA_EDEVICE;
}

#define MLP_TRY(m, expr)                                              \
    do {                                                              \
        hipError_t e_ = (expr);                                       \
        if (e_ != hipSuccess) return mlp_hip((m), e_, #expr);         \
    } while (0)

void mlp_free(mc_lya_mlp *m)
{
    void *ptrs[] = {m->d_params, m->d_m, m->d_v, m->d_grad, m->d_part, m->d_env, m->d_count, m->d_batch, m->d_bad,
                    m->d_tails};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
}

mc_lya_status check_batch(mc_lya_mlp *m, const float *features, uint64_t n)
{
    if (n > 0 && !features) return mlp_fail(m, MC_LYA_EINVAL, "features is NULL");
    if (n >= (1ull << 40)) return mlp_fail(m, MC_LYA_EINVAL, "too many cells");
    return MC_LYA_OK;
}

}  // namespace

extern "C" {

mc_lya_status mc_lya_mlp_create(mc_lya_mlp **out, const float *params, void *stream)
{
    g_mlp_init_err.clear();
    if (!out) return MC_LYA_EINVAL;
    *out = nullptr;
    if (!params) {
        g_mlp_init_err = "params is NULL";
        return MC_LYA_EINVAL;
    }
    for (int j = 0; j < kMlpParams; ++j)
        if (!std::isfinite(params[j])) {
            g_mlp_init_err = "params must be finite";
            return MC_LYA_EINVAL;
        }
    mc_lya_mlp *m = new (std::nothrow) mc_lya_mlp;
    if (!m) return MC_LYA_ENOMEM;
    m->stream = static_cast<hipStream_t>(stream);
    auto bail = [&](hipError_t e, const char *what) {
        g_mlp_init_err = std::string(what) + ": " + hipGetErrorString(e);
        mlp_free(m);
        delete m;
        return e == hipErrorOutOfMemory ? MC_LYA_ENOMEM : MC_LYA_EDEVICE;
    };
    hipError_t e;
    const size_t pb = sizeof(float) * kMlpParams;
    if ((e = hipMalloc(reinterpret_cast<void **>(&m->d_params), pb)) != hipSuccess) return bail(e, "allocation");
    if ((e = hipMalloc(reinterpret_cast<void **>(&m->d_m), pb)) != hipSuccess) return bail(e, "allocation");
    if ((e = hipMalloc(reinterpret_cast<void **>(&m->d_v), pb)) != hipSuccess) return bail(e, "allocation");
    if ((e = hipMalloc(reinterpret_cast<void **>(&m->d_grad), sizeof(float) * (kMlpParams + 2))) != hipSuccess)
        return bail(e, "allocation");
    if ((e = hipMalloc(reinterpret_cast<void **>(&m->d_part),
                       sizeof(float) * (size_t)(kMlpGradBlocks + (kMlpGradBlocks + 31) / 32) * kMlpPartStride)) !=
        hipSuccess)
        return bail(e, "allocation");
    if ((e = hipMalloc(reinterpret_cast<void **>(&m->d_env), sizeof(float) * 16)) != hipSuccess)
        return bail(e, "allocation");
    if ((e = hipMalloc(reinterpret_cast<void **>(&m->d_count), sizeof(unsigned long long))) != hipSuccess)
        return bail(e, "allocation");
    if ((e = hipMemcpyAsync(m->d_params, params, pb, hipMemcpyHostToDevice, m->stream)) != hipSuccess ||
        (e = hipMemsetAsync(m->d_m, 0, pb, m->stream)) != hipSuccess ||
        (e = hipMemsetAsync(m->d_v, 0, pb, m->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(m->stream)) != hipSuccess)
        return bail(e, "upload");
    int dev = 0, cu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
            cu = prop.multiProcessorCount;
    }
    // one wave per SIMD per resident workgroup, each wave looping over its
    // tiles: a grid the chip holds at once has no partly filled last round
    m->forward_grid = cu * mlp_forward_blocks_per_cu();
    *out = m;
    return MC_LYA_OK;
}

mc_lya_status mc_lya_mlp_get_params(mc_lya_mlp *m, float *params)
{
    if (!m) return MC_LYA_EINVAL;
    if (!params) return mlp_fail(m, MC_LYA_EINVAL, "params is NULL");
    MLP_TRY(m, hipMemcpyAsync(params, m->d_params, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, m->stream));
    MLP_TRY(m, hipStreamSynchronize(m->stream));
    return MC_LYA_OK;
}

mc_lya_status mc_lya_mlp_set_envelope(mc_lya_mlp *m, const float *lo, const float *hi)
{
    if (!m) return MC_LYA_EINVAL;
    if ((lo == nullptr) != (hi == nullptr)) return mlp_fail(m, MC_LYA_EINVAL, "give both bounds or neither");
    if (!lo) {
        m->envelope = false;
        return MC_LYA_OK;
    }
    float env[16];
    for (int k = 0; k < 8; ++k) {
        if (!(lo[k] <= hi[k])) return mlp_fail(m, MC_LYA_EINVAL, "every lower bound must be <= its upper bound");
        env[k] = lo[k];
        env[8 + k] = hi[k];
    }
    MLP_TRY(m, hipMemcpyAsync(m->d_env, env, sizeof env, hipMemcpyHostToDevice, m->stream));
    MLP_TRY(m, hipStreamSynchronize(m->stream));
    m->envelope = true;
    return MC_LYA_OK;
}

mc_lya_status mc_lya_mlp_forward(mc_lya_mlp *m, const float *features, uint64_t n, float *y, uint8_t *outside,
                                 uint64_t *n_outside)
{
    if (!m) return MC_LYA_EINVAL;
    mc_lya_status st = check_batch(m, features, n);
    if (st != MC_LYA_OK) return st;
    if (n > 0 && !y) return mlp_fail(m, MC_LYA_EINVAL, "y is NULL");
    if (n_outside) *n_outside = 0;
    if (n == 0) return MC_LYA_OK;
    if (n_outside) MLP_TRY(m, launch_zero_counters(m->d_count, 1, m->stream));
    const uint64_t tiles = (n + 31) / 32;
    const int grid = (int)std::min<uint64_t>((uint64_t)m->forward_grid, (tiles + 3) / 4);
    MLP_TRY(m, launch_mlp_forward(m->d_params, features, n, y, outside, m->envelope ? m->d_env : nullptr,
                                  m->envelope ? m->d_env + 8 : nullptr, n_outside ? m->d_count : nullptr, grid,
                                  m->stream));
    if (n_outside) {
        unsigned long long c = 0;
        MLP_TRY(m, hipMemcpyAsync(&c, m->d_count, sizeof c, hipMemcpyDeviceToHost, m->stream));
        MLP_TRY(m, hipStreamSynchronize(m->stream));
        *n_outside = c;
    }
    return MC_LYA_OK;
}

mc_lya_status mc_lya_mlp_correction(mc_lya_mlp *m, const float *features, uint64_t n, const float *fallback,
                                    float *y, float *M, uint8_t *outside, uint64_t *n_outside)
{
    if (!m) return MC_LYA_EINVAL;
    if (n > 0 && !M) return mlp_fail(m, MC_LYA_EINVAL, "M is NULL");
    if (n > 0 && (uint64_t)(n + 255) / 256 > 0x7fffffffull) return mlp_fail(m, MC_LYA_EINVAL, "too many cells");
    mc_lya_status st = mc_lya_mlp_forward(m, features, n, y, outside, n_outside);
    if (st != MC_LYA_OK || n == 0) return st;
    MLP_TRY(m, launch_mlp_correction(y, outside, fallback, n, M, m->stream));
    return MC_LYA_OK;
}

mc_lya_status mc_lya_mlp_gradient(mc_lya_mlp *m, const float *features, const float *targets, const float *weights,
                                  uint64_t n, float *grad, float *loss)
{
    if (!m) return MC_LYA_EINVAL;
    mc_lya_status st = check_batch(m, features, n);
    if (st != MC_LYA_OK) return st;
    if (n == 0 || !targets || !weights) return mlp_fail(m, MC_LYA_EINVAL, "need cells, targets and weights");
    MLP_TRY(m, launch_mlp_gradient(m->d_params, features, targets, weights, n, m->d_part, kMlpGradBlocks,
                                   m->d_grad, m->stream));
    MLP_TRY(m, launch_mlp_normalise(m->d_grad, m->stream));
    float tail[2];
    MLP_TRY(m, hipMemcpyAsync(tail, m->d_grad + kMlpParams, sizeof tail, hipMemcpyDeviceToHost, m->stream));
    if (grad) MLP_TRY(m, hipMemcpyAsync(grad, m->d_grad, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, m->stream));
    MLP_TRY(m, hipStreamSynchronize(m->stream));
    if (!(tail[1] > 0.0f)) return mlp_fail(m, MC_LYA_EINVAL, "the weights sum to zero");
    if (loss) *loss = tail[0] / tail[1];
    return MC_LYA_OK;
}

mc_lya_status mc_lya_mlp_train_step(mc_lya_mlp *m, const float *features, const float *targets, const float *weights,
                                    uint64_t n, const mc_lya_adam *hp, float *loss)
{
    if (!m) return MC_LYA_EINVAL;
    mc_lya_status st = check_batch(m, features, n);
    if (st != MC_LYA_OK) return st;
    if (n == 0 || !targets || !weights) return mlp_fail(m, MC_LYA_EINVAL, "need cells, targets and weights");
    if (!hp || !(hp->lr > 0.0f) || !(hp->beta1 >= 0.0f && hp->beta1 < 1.0f) ||
        !(hp->beta2 >= 0.0f && hp->beta2 < 1.0f) || !(hp->eps > 0.0f))
        return mlp_fail(m, MC_LYA_EINVAL, "Adam needs lr > 0, beta1 and beta2 in [0, 1), eps > 0");
    MLP_TRY(m, launch_mlp_gradient(m->d_params, features, targets, weights, n, m->d_part, kMlpGradBlocks,
                                   m->d_grad, m->stream));
    const int64_t t = m->step + 1;
    MlpAdam a;
    a.lr = hp->lr;
    a.beta1 = hp->beta1;
    a.beta2 = hp->beta2;
    a.eps = hp->eps;
    a.bc1 = (float)(1.0 - std::pow((double)hp->beta1, (double)t));
    a.bc2 = (float)(1.0 - std::pow((double)hp->beta2, (double)t));
    MLP_TRY(m, launch_mlp_adam(m->d_params, m->d_m, m->d_v, m->d_grad, a, m->stream));
    m->step = t;
    if (loss) {
        float tail[2];
        MLP_TRY(m, hipMemcpyAsync(tail, m->d_grad + kMlpParams, sizeof tail, hipMemcpyDeviceToHost, m->stream));
        MLP_TRY(m, hipStreamSynchronize(m->stream));
        *loss = tail[1] > 0.0f ? tail[0] / tail[1] : 0.0f;
    }
    return MC_LYA_OK;
}

mc_lya_status mc_lya_mlp_train_steps(mc_lya_mlp *m, const float *features, const float *targets,
                                     const float *weights, uint64_t n_cells, const int64_t *idx, uint64_t batch,
                                     int n_steps, const float *lr, float beta1, float beta2, float eps,
                                     float *losses)
{
    if (!m) return MC_LYA_EINVAL;
    mc_lya_status st = check_batch(m, features, n_cells);
    if (st != MC_LYA_OK) return st;
    if (n_cells == 0 || !targets || !weights) return mlp_fail(m, MC_LYA_EINVAL, "need cells, targets and weights");
    if (n_steps < 0 || (n_steps > 0 && (!idx || !lr || batch == 0)))
        return mlp_fail(m, MC_LYA_EINVAL, "need n_steps >= 0 and, for steps, idx, lr and batch > 0");
    if (batch > (1ull << 32)) return mlp_fail(m, MC_LYA_EINVAL, "batch must be at most 2^32");
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return mlp_fail(m, MC_LYA_EINVAL, "Adam needs beta1 and beta2 in [0, 1), eps > 0");
    for (int s = 0; s < n_steps; ++s)
        if (!(lr[s] > 0.0f)) return mlp_fail(m, MC_LYA_EINVAL, "every learning rate must be > 0");
    if (n_steps == 0) return MC_LYA_OK;
    if (batch > m->batch_cap) {
        if (m->d_batch) MLP_TRY(m, hipFree(m->d_batch));
        m->d_batch = nullptr;
        m->batch_cap = 0;
        if (hipMalloc(reinterpret_cast<void **>(&m->d_batch), sizeof(float) * batch * (8 + 2)) != hipSuccess)
            return mlp_fail(m, MC_LYA_ENOMEM, "device allocation of the gathered batch failed");
        m->batch_cap = batch;
    }
    if (!m->d_bad && hipMalloc(reinterpret_cast<void **>(&m->d_bad), sizeof(unsigned int)) != hipSuccess)
        return mlp_fail(m, MC_LYA_ENOMEM, "device allocation failed");
    if (losses && n_steps > m->tails_cap) {
        if (m->d_tails) MLP_TRY(m, hipFree(m->d_tails));
        m->d_tails = nullptr;
        m->tails_cap = 0;
        if (hipMalloc(reinterpret_cast<void **>(&m->d_tails), sizeof(float) * 2 * (size_t)n_steps) != hipSuccess)
            return mlp_fail(m, MC_LYA_ENOMEM, "device allocation of the losses failed");
        m->tails_cap = n_steps;
    }
    float *Xb = m->d_batch, *tb = Xb + batch * 8, *wb = tb + batch;    // [batch][8] features, then t, w
    MLP_TRY(m, hipMemsetAsync(m->d_bad, 0, sizeof(unsigned int), m->stream));
    for (int s = 0; s < n_steps; ++s) {
        MLP_TRY(m, launch_mlp_gather(features, targets, weights, n_cells, idx + (size_t)s * batch, batch, Xb, tb, wb,
                                     m->d_bad, m->stream));
        MLP_TRY(m, launch_mlp_gradient(m->d_params, Xb, tb, wb, batch, m->d_part, kMlpGradBlocks, m->d_grad,
                                       m->stream));
        const int64_t t = m->step + 1;
        MlpAdam a;
        a.lr = lr[s];
        a.beta1 = beta1;
        a.beta2 = beta2;
        a.eps = eps;
        a.bc1 = (float)(1.0 - std::pow((double)beta1, (double)t));
        a.bc2 = (float)(1.0 - std::pow((double)beta2, (double)t));
        MLP_TRY(m, launch_mlp_adam(m->d_params, m->d_m, m->d_v, m->d_grad, a, m->stream));
        m->step = t;
        if (losses)
            MLP_TRY(m, hipMemcpyAsync(m->d_tails + 2 * (size_t)s, m->d_grad + kMlpParams, 2 * sizeof(float),
                                      hipMemcpyDeviceToDevice, m->stream));
    }
    unsigned int bad = 0;
    std::vector<float> tails(losses ? 2 * (size_t)n_steps : 0);
    if (losses)
        MLP_TRY(m, hipMemcpyAsync(tails.data(), m->d_tails, sizeof(float) * tails.size(), hipMemcpyDeviceToHost,
                                  m->stream));
    MLP_TRY(m, hipMemcpyAsync(&bad, m->d_bad, sizeof bad, hipMemcpyDeviceToHost, m->stream));
    MLP_TRY(m, hipStreamSynchronize(m->stream));
    if (losses)
        for (int s = 0; s < n_steps; ++s)
            losses[s] = tails[2 * s + 1] > 0.0f ? tails[2 * s] / tails[2 * s + 1] : 0.0f;
    if (bad) return mlp_fail(m, MC_LYA_EINVAL, "an index is outside [0, n_cells)");
    return MC_LYA_OK;
}

}  // extern "C"

// ---- gradient without allocation ---------------------------------------------
// The workspace of mc_lya_mlp_gradient_static: the gradient kernel's per-block
// partial sums and the group sums of its fixed-order reduction, in one
// file-scope device array per GPU (held until the process ends). Host code
// never uses the array's name as an address: its device address is looked up
// once per device with hipGetSymbolAddress and kept below.
namespace {

constexpr size_t kStaticGradFloats =
    (size_t)(kMlpGradBlocks + (kMlpGradBlocks + 31) / 32) * kMlpPartStride;
static_assert(kStaticGradFloats * sizeof(float) == MC_LYA_STATIC_SCRATCH_BYTES, "static workspace size");
__device__ __align__(256) float scratch[kStaticGradFloats];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
thread_local std::string g_static_err;

mc_lya_status static_fail(mc_lya_status s, const std::string &what)
{
    g_static_err = what;
    return s;
}

// The device address of the current device's scratch array (looked up on the
// first call on that device, with that device current).
mc_lya_status scratch_address(float **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return static_fail(MC_LYA_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return static_fail(MC_LYA_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return static_fail(MC_LYA_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<float *>(g_scratch_ptr[dev]);
    return MC_LYA_OK;
}

}  // namespace

extern "C" {

mc_lya_status mc_lya_mlp_gradient_static(const float *params, const float *features, const float *targets,
                                         const float *weights, uint64_t n, float *grad_out, void *stream)
{
    g_static_err.clear();
    if (!params || !grad_out) return static_fail(MC_LYA_EINVAL, "params and grad_out must not be NULL");
    if (n == 0 || !features || !targets || !weights)
        return static_fail(MC_LYA_EINVAL, "need cells, features, targets and weights");
    if (n > MC_LYA_STATIC_MAX_CELLS)
        return static_fail(MC_LYA_EINVAL, "n exceeds MC_LYA_STATIC_MAX_CELLS (the static workspace's limit)");
    float *ws = nullptr;
    mc_lya_status st = scratch_address(&ws);
    if (st != MC_LYA_OK) return st;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = launch_mlp_gradient(params, features, targets, weights, n, ws, kMlpGradBlocks, grad_out, s);
    if (e == hipSuccess) e = launch_mlp_normalise(grad_out, s);
    if (e != hipSuccess) return static_fail(MC_LYA_EDEVICE, std::string("launch: ") + hipGetErrorString(e));
    return MC_LYA_OK;
}

const char *mc_lya_mlp_static_last_error(void) { return g_static_err.c_str(); }

void mc_lya_mlp_destroy(mc_lya_mlp *m)
{
    if (!m) return;
    (void)hipStreamSynchronize(m->stream);
    mlp_free(m);
    delete m;
}

const char *mc_lya_mlp_last_error(const mc_lya_mlp *m)
{
    if (!m) return g_mlp_init_err.c_str();
    return m->err.c_str();
}

}  // extern "C"

// Packet walk: emission (App. A step 1), straight-line cell walk with the
// Hubble drift (App. A step 4) and the bulk-velocity shift of Eq. (inout) at
// faces, expected-value deposits of the true absorption (kappa_c dPhi, the
// depth of Eq. (<fnu>) over the swept part of the profile) into 64-bit
// integer tallies, and escape by redshifting (end of App. A).
//
// Two drivers share one per-packet step:
//   walk_persistent  resident waves that pull blocks of packet ids from a
//                    queue and hand new packets to idle lanes (wave refill),
//                    so the 10-20% of packets emitted on the red side, which
//                    walk hundreds of cells, do not leave the rest of the wave
//                    idle;
//   walk_simple      one thread per packet (reference driver, same results).
// Both produce bit-identical integer tallies: each packet's arithmetic does
// not depend on the driver, and integer additions commute.
#include "common.hpp"

namespace mclya {
namespace {

constexpr double kFar = 1.0e300;   // face distance along an axis the ray does not move on

// Ray geometry (direction, position inside the cell, face distances) is kept
// in binary64: over paths of hundreds of cells binary32 directions drift by
// ~1e-5 cell, enough to clip a different cell corner than an exact ray. The
// line-profile arithmetic (drift, Phi, deposit) is binary32.
struct Lane {
    int32_t ix, iy, iz;
    uint32_t c;          // global cell
    double fx, fy, fz;   // position inside the cell, [0,1]
    double kx, ky, kz;   // direction
    double rx, ry, rz;   // 1/|k| per axis
    float x;             // gas-frame frequency, Doppler widths
    float kap;           // kappa of the current cell
    float ux, uy, uz;    // bulk velocity of the current cell (Doppler units)
    uint64_t w;          // remaining weight
    uint32_t ncross;
    int32_t nx, ny, nz;
    uint32_t coff;
    float delta, xeff;
};

template <bool VEL>
__device__ __forceinline__ void load_cell(Lane &L, const void *__restrict__ rec)
{
    if (VEL) {
        const float4 r = static_cast<const float4 *>(rec)[L.c];
        L.kap = r.x;
        L.ux = r.y;
        L.uy = r.z;
        L.uz = r.w;
    } else {
        L.kap = static_cast<const float *>(rec)[L.c];
    }
}

// Emission of packet p (box-local id) in global cell gcell: position uniform
// in the cell, isotropic direction, frequency from the Doppler profile
// exp(-x^2)/sqrt(pi) by the Box-Muller transform.
template <bool VEL>
__device__ __forceinline__ void init_packet(Lane &L, const WalkBox &B, uint64_t p, uint32_t gcell,
                                            const void *__restrict__ rec)
{
    const uint32_t k0 = (uint32_t)B.seed, k1 = (uint32_t)(B.seed >> 32);
    uint32_t a[4] = {(uint32_t)p, (uint32_t)(p >> 32), 0u, 0u};
    uint32_t b[4] = {(uint32_t)p, (uint32_t)(p >> 32), 1u, 0u};
    philox4x32_10(a, k0, k1);
    philox4x32_10(b, k0, k1);
    L.nx = B.nx;
    L.ny = B.ny;
    L.nz = B.nz;
    L.coff = B.cell_off;
    L.delta = B.delta;
    L.xeff = B.x_eff;
    const uint32_t local = gcell - B.cell_off;
    L.ix = (int32_t)(local % (uint32_t)B.nx);
    const uint32_t rest = local / (uint32_t)B.nx;
    L.iy = (int32_t)(rest % (uint32_t)B.ny);
    L.iz = (int32_t)(rest / (uint32_t)B.ny);
    L.c = gcell;
    L.fx = (double)u01(a[0]);
    L.fy = (double)u01(a[1]);
    L.fz = (double)u01(a[2]);
    const double mu = 2.0 * (double)u01(a[3]) - 1.0;   // exact
    double sp, cp;
    sincospi(2.0 * (double)u01(b[0]), &sp, &cp);         // azimuth 2 pi u
    const double st = sqrt((1.0 - mu) * (1.0 + mu));
    L.kx = st * cp;
    L.ky = st * sp;
    L.kz = mu;
    L.rx = L.kx != 0.0 ? 1.0 / fabs(L.kx) : kFar;
    L.ry = L.ky != 0.0 ? 1.0 / fabs(L.ky) : kFar;
    L.rz = L.kz != 0.0 ? 1.0 / fabs(L.kz) : kFar;
    L.x = (float)(sqrt(-log((double)u01(b[1]))) * cospi(2.0 * (double)u01(b[2])));
    L.w = B.w0;
    L.ncross = 0;
    load_cell<VEL>(L, rec);
}

// Phi(hi) - Phi(lo) for hi > lo, Phi(x) = erfc(-x)/2, written with the
// complementary function on the side where it is small so that the
// difference does not cancel.
// Clamped at 0: Phi is non-decreasing, but two rounded erfc values of nearly
// equal arguments (a sliver segment at a cell corner) can come out reversed.
__device__ __forceinline__ float delta_phi(float hi, float lo)
{
    const float d = lo >= 0.0f ? 0.5f * (erfcf(lo) - erfcf(hi)) : 0.5f * (erfcf(-hi) - erfcf(-lo));
    return fmaxf(d, 0.0f);
}

enum : int { kAlive = 0, kEscaped = 1, kAbsorbed = 2, kCapped = 3 };

// One (packet, cell) segment. Returns kAlive, or the packet's fate.
template <bool VEL, bool TALLY>
__device__ __forceinline__ int walk_step(Lane &L, const void *__restrict__ rec,
                                         unsigned long long *__restrict__ A, uint32_t max_cross,
                                         uint64_t &deposited)
{
    if (L.x <= -L.xeff) return kEscaped;            // redshifted out of the line
    if (L.ncross >= max_cross) return kCapped;
    ++L.ncross;

    // distance to the face the ray leaves through (ties: x, then y, then z)
    const double tx = (L.kx > 0.0 ? 1.0 - L.fx : L.fx) * L.rx;
    const double ty = (L.ky > 0.0 ? 1.0 - L.fy : L.fy) * L.ry;
    const double tz = (L.kz > 0.0 ? 1.0 - L.fz : L.fz) * L.rz;
    int axis = 0;
    double s = tx;
    if (ty < s) { axis = 1; s = ty; }
    if (tz < s) { axis = 2; s = tz; }

    // Hubble drift across the segment; the last one stops at -x_eff
    const float xo = fmaf(-L.delta, (float)s, L.x);
    const bool esc = xo <= -L.xeff;
    const float dphi = delta_phi(L.x, esc ? -L.xeff : xo);
    const float dtau = L.kap * dphi;
    const float pabs = -expm1f(-dtau);
    uint64_t d = (uint64_t)rintf((float)L.w * pabs);
    if (d > L.w) d = L.w;
    L.w -= d;
    deposited += d;
    if (TALLY && d) atomicAdd(&A[L.c], (unsigned long long)d);
    if (esc) return kEscaped;
    if (L.w == 0) return kAbsorbed;

    // move to the face and into the neighbour (periodic)
    L.fx = fmin(fmax(fma(L.kx, s, L.fx), 0.0), 1.0);
    L.fy = fmin(fmax(fma(L.ky, s, L.fy), 0.0), 1.0);
    L.fz = fmin(fmax(fma(L.kz, s, L.fz), 0.0), 1.0);
    if (axis == 0) {
        if (L.kx > 0.0) { L.fx = 0.0; L.ix = (L.ix + 1 == L.nx) ? 0 : L.ix + 1; }
        else { L.fx = 1.0; L.ix = (L.ix == 0) ? L.nx - 1 : L.ix - 1; }
    } else if (axis == 1) {
        if (L.ky > 0.0) { L.fy = 0.0; L.iy = (L.iy + 1 == L.ny) ? 0 : L.iy + 1; }
        else { L.fy = 1.0; L.iy = (L.iy == 0) ? L.ny - 1 : L.iy - 1; }
    } else {
        if (L.kz > 0.0) { L.fz = 0.0; L.iz = (L.iz + 1 == L.nz) ? 0 : L.iz + 1; }
        else { L.fz = 1.0; L.iz = (L.iz == 0) ? L.nz - 1 : L.iz - 1; }
    }
    L.c = L.coff + (uint32_t)L.ix + (uint32_t)L.nx * ((uint32_t)L.iy + (uint32_t)L.ny * (uint32_t)L.iz);
    L.x = xo;
    if (VEL) {
        const float ux = L.ux, uy = L.uy, uz = L.uz;
        load_cell<VEL>(L, rec);
        // Eq. (inout), bulk term: x_new = x_old - k.(U_new - U_old)
        const float du = (float)(L.kx * (double)(L.ux - ux) + L.ky * (double)(L.uy - uy) +
                                 L.kz * (double)(L.uz - uz));
        L.x = xo - du;
    } else {
        load_cell<VEL>(L, rec);
    }
    return kAlive;
}

// ---- wave helpers --------------------------------------------------------
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t rank_in(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ uint64_t bcast_u64(uint64_t v, int src)
{
    return __shfl(v, src, 64);
}

// Per-lane per-box totals, flushed with one atomic per box per wave.
struct Acc {
    int32_t box;
    uint64_t esc, cross, capn, capw;
};

// Convergent: every lane of the wave must call it. Lanes with `give` add
// their totals to their box; the wave issues one atomic per distinct box.
__device__ __forceinline__ void flush(Acc &a, bool give, BoxTot *__restrict__ tot)
{
    uint64_t pending = __ballot(give && a.box >= 0);
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int b = __shfl(a.box, leader, 64);
        const bool mine = give && a.box == b;
        const uint64_t e = wave_sum_u64(mine ? a.esc : 0);
        const uint64_t c = wave_sum_u64(mine ? a.cross : 0);
        const uint64_t n = wave_sum_u64(mine ? a.capn : 0);
        const uint64_t w = wave_sum_u64(mine ? a.capw : 0);
        if ((int)lane_id() == leader) {
            if (e) atomicAdd(&tot[b].escaped, (unsigned long long)e);
            if (c) atomicAdd(&tot[b].crossings, (unsigned long long)c);
            if (n) atomicAdd(&tot[b].capped_packets, (unsigned long long)n);
            if (w) atomicAdd(&tot[b].capped_weight, (unsigned long long)w);
        }
        pending &= ~__ballot(mine);
    }
    if (give) a.esc = a.cross = a.capn = a.capw = 0;
}

__device__ __forceinline__ void account(Acc &a, const Lane &L, int fate)
{
    a.cross += L.ncross;
    if (fate == kEscaped) a.esc += L.w;
    if (fate == kCapped) { a.capn += 1; a.capw += L.w; }
}

// Box of a global packet id (boxes sorted by packet offset).
__device__ __forceinline__ int box_of(const WalkBox *boxes, int n_boxes, uint64_t gp)
{
    int lo = 0, hi = n_boxes - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (boxes[mid].pkt_off <= gp) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---- persistent driver ---------------------------------------------------
template <bool VEL>
__global__ __launch_bounds__(256) void walk_persistent_kernel(WalkParams P)
{
    extern __shared__ WalkBox sbox[];
    for (int i = threadIdx.x; i < P.n_boxes; i += blockDim.x) sbox[i] = P.boxes[i];
    __syncthreads();

    const uint32_t lane = lane_id();
    const uint32_t max_cross = (uint32_t)P.max_cross;
    Lane L;
    Acc acc{-1, 0, 0, 0, 0};
    bool alive = false;
    bool more = true;                 // wave-uniform: queue not drained
    uint64_t cur = 0, end = 0;        // wave-uniform: current block of packet ids
    const uint32_t refill = (uint32_t)P.refill;
    const uint64_t chunk = (uint64_t)P.chunk;

    for (;;) {
        uint64_t idle = __ballot(!alive);
        if (more && (uint32_t)__popcll(idle) >= refill) {
            while (idle && more) {
                if (cur >= end) {
                    uint64_t base = 0;
                    if (lane == 0) base = atomicAdd(P.queue, (unsigned long long)chunk);
                    base = bcast_u64(base, 0);
                    if (base >= P.count) { more = false; break; }
                    cur = base;
                    end = base + chunk < P.count ? base + chunk : P.count;
                }
                const uint64_t n_idle = (uint64_t)__popcll(idle);
                const uint64_t take = n_idle < end - cur ? n_idle : end - cur;
                const uint32_t r = rank_in(idle);
                const bool fresh = !alive && (uint64_t)r < take;
                uint64_t gp = 0;
                int nb = acc.box;
                if (fresh) {
                    gp = P.first + cur + r;
                    nb = P.n_boxes == 1 ? 0 : box_of(sbox, P.n_boxes, gp);
                }
                const bool change = fresh && nb != acc.box;
                if (__ballot(change && acc.box >= 0)) flush(acc, change, P.tot);
                if (fresh) {
                    acc.box = nb;
                    const WalkBox &B = sbox[nb];
                    init_packet<VEL>(L, B, gp - B.pkt_off, P.cell_of_packet[gp], P.rec);
                    alive = true;
                }
                cur += take;
                idle = __ballot(!alive);
            }
        }
        if (!__ballot(alive)) {
            if (!more) break;
            continue;
        }
        if (alive) {
            uint64_t dep = 0;
            const int fate = walk_step<VEL, true>(L, P.rec, P.A, max_cross, dep);
            if (fate != kAlive) {
                account(acc, L, fate);
                alive = false;
            }
        }
    }
    flush(acc, true, P.tot);
}

// ---- one thread per packet -------------------------------------------------
template <bool VEL>
__global__ __launch_bounds__(256) void walk_simple_kernel(WalkParams P)
{
    extern __shared__ WalkBox sbox[];
    for (int i = threadIdx.x; i < P.n_boxes; i += blockDim.x) sbox[i] = P.boxes[i];
    __syncthreads();
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    Acc acc{-1, 0, 0, 0, 0};
    if (i < P.count) {
        const uint64_t gp = P.first + i;
        const int nb = P.n_boxes == 1 ? 0 : box_of(sbox, P.n_boxes, gp);
        const WalkBox &B = sbox[nb];
        Lane L;
        init_packet<VEL>(L, B, gp - B.pkt_off, P.cell_of_packet[gp], P.rec);
        acc.box = nb;
        uint64_t dep = 0;
        int fate;
        do {
            fate = walk_step<VEL, true>(L, P.rec, P.A, (uint32_t)P.max_cross, dep);
        } while (fate == kAlive);
        account(acc, L, fate);
    }
    flush(acc, true, P.tot);
}

// ---- packet histories (no tallies) -------------------------------------------
template <bool VEL>
__global__ __launch_bounds__(256) void trace_kernel(WalkParams P, mc_lya_packet_trace *out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.count) return;
    const uint64_t gp = P.first + i;
    const int nb = P.n_boxes == 1 ? 0 : box_of(P.boxes, P.n_boxes, gp);
    const WalkBox B = P.boxes[nb];
    Lane L;
    init_packet<VEL>(L, B, gp - B.pkt_off, P.cell_of_packet[gp], P.rec);
    mc_lya_packet_trace t;
    t.cell0 = L.c;
    t.fx = (float)L.fx;
    t.fy = (float)L.fy;
    t.fz = (float)L.fz;
    t.kx = (float)L.kx;
    t.ky = (float)L.ky;
    t.kz = (float)L.kz;
    t.x0 = L.x;
    uint64_t dep = 0;
    int fate;
    do {
        fate = walk_step<VEL, false>(L, P.rec, nullptr, (uint32_t)P.max_cross, dep);
    } while (fate == kAlive);
    t.escaped = fate == kAbsorbed ? 0 : (int64_t)L.w;
    t.absorbed = (int64_t)dep;
    t.crossings = L.ncross;
    t.fate = fate == kEscaped ? 1 : (fate == kCapped ? 2 : 0);
    out[i] = t;
}

__global__ void philox_kernel(const uint32_t *__restrict__ ctr, const uint32_t *__restrict__ key,
                              uint32_t *__restrict__ out, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t c[4] = {ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
    philox4x32_10(c, key[2 * i], key[2 * i + 1]);
    for (int j = 0; j < 4; ++j) out[4 * i + j] = c[j];
}

__global__ void reset_queue_kernel(unsigned long long *q) { *q = 0ull; }

}  // namespace

int persistent_blocks_per_cu(bool vel, int block)
{
    int n = 0;
    const size_t lds = sizeof(WalkBox);
    hipError_t e = vel ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, walk_persistent_kernel<true>, block, lds)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, walk_persistent_kernel<false>, block, lds);
    return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_walk_persistent(const WalkParams &p, int block, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(1), 0, s, p.queue);
    const size_t lds = sizeof(WalkBox) * (size_t)p.n_boxes;
    if (p.vel)
        hipLaunchKernelGGL(walk_persistent_kernel<true>, dim3((unsigned)grid), dim3((unsigned)block), lds, s, p);
    else
        hipLaunchKernelGGL(walk_persistent_kernel<false>, dim3((unsigned)grid), dim3((unsigned)block), lds, s, p);
    return hipGetLastError();
}

hipError_t launch_walk_simple(const WalkParams &p, int block, hipStream_t s)
{
    const uint64_t grid = (p.count + (uint64_t)block - 1) / (uint64_t)block;
    const size_t lds = sizeof(WalkBox) * (size_t)p.n_boxes;
    if (p.vel)
        hipLaunchKernelGGL(walk_simple_kernel<true>, dim3((unsigned)grid), dim3((unsigned)block), lds, s, p);
    else
        hipLaunchKernelGGL(walk_simple_kernel<false>, dim3((unsigned)grid), dim3((unsigned)block), lds, s, p);
    return hipGetLastError();
}

hipError_t launch_trace(const WalkParams &p, mc_lya_packet_trace *out, hipStream_t s)
{
    const uint64_t grid = (p.count + 255) / 256;
    if (p.vel)
        hipLaunchKernelGGL(trace_kernel<true>, dim3((unsigned)grid), dim3(256), 0, s, p, out);
    else
        hipLaunchKernelGGL(trace_kernel<false>, dim3((unsigned)grid), dim3(256), 0, s, p, out);
    return hipGetLastError();
}

hipError_t launch_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out, uint64_t n, hipStream_t s)
{
    const uint64_t grid = (n + 255) / 256;
    hipLaunchKernelGGL(philox_kernel, dim3((unsigned)grid), dim3(256), 0, s, ctr, key, out, n);
    return hipGetLastError();
}

}  // namespace mclya

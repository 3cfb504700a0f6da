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
#include "walk_core.hpp"

namespace mclya {
namespace {

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

// Tells the compiler a wave-uniform value is uniform (scalar registers).
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Per-lane per-box totals, flushed with one atomic per box per wave.
struct Acc {
    int32_t box;
    uint64_t esc, cross, capn, capw, wing;
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
        const uint64_t g = wave_sum_u64(mine ? a.wing : 0);
        if ((int)lane_id() == leader) {
            if (e) atomicAdd(&tot[b].escaped, (unsigned long long)e);
            if (c) atomicAdd(&tot[b].crossings, (unsigned long long)c);
            if (n) atomicAdd(&tot[b].capped_packets, (unsigned long long)n);
            if (w) atomicAdd(&tot[b].capped_weight, (unsigned long long)w);
            if (g) atomicAdd(&tot[b].wing, (unsigned long long)g);
        }
        pending &= ~__ballot(mine);
    }
    if (give) a.esc = a.cross = a.capn = a.capw = a.wing = 0;
}

__device__ __forceinline__ void account(Acc &a, const Lane &L, int fate, uint32_t wing)
{
    a.cross += L.ncross;
    a.esc += fate == kEscaped ? L.w : 0;
    a.capn += fate == kCapped ? 1 : 0;
    a.capw += fate == kCapped ? L.w : 0;
    a.wing += wing;
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

// Global packet id of index i of the walked range.
__device__ __forceinline__ uint64_t packet_id(const WalkParams &P, uint64_t i)
{
    if (P.n_seg == 0) return P.first + i;
    int lo = 0, hi = P.n_seg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (P.seg_start[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return P.seg_id[lo] + (i - P.seg_start[lo]);
}

// ---- persistent driver ---------------------------------------------------
template <bool VEL, bool VOIGT>
__global__ __launch_bounds__(256) void walk_persistent_kernel(WalkParams P)
{
    extern __shared__ WalkBox sbox[];
    for (int i = threadIdx.x; i < P.n_boxes; i += blockDim.x) sbox[i] = P.boxes[i];
    __syncthreads();

    const uint32_t lane = lane_id();
    const uint32_t max_cross = (uint32_t)P.max_cross;
    Lane L;
    idle_lane(L);
    Line ln{0.0f, 0.0f, 0.0f};
    Acc acc{-1, 0, 0, 0, 0, 0};
    bool alive = false;
    bool more = true;                 // wave-uniform: queue not drained
    uint64_t cur = 0, end = 0;        // wave-uniform: current block of packet ids
    const uint32_t refill = (uint32_t)P.refill;
    const uint64_t chunk = (uint64_t)P.chunk;
    // The packet range is split into nq contiguous parts (packet ids follow
    // the cell order, so each part is a slab of the grid). Workgroups are
    // dispatched round-robin over the chip's XCDs, so workgroup g starts on
    // part g % nq and moves on to the next part when its own is drained:
    // each XCD's L2 mostly sees one slab.
    const uint32_t nq = (uint32_t)P.nqueues;
    uint32_t part = blockIdx.x % nq, tried = 0;

    for (;;) {
        uint64_t idle = __ballot(!alive);
        if (more && (uint32_t)__popcll(idle) >= refill) {
            while (idle && more) {
                if (cur >= end) {
                    const uint64_t lo = P.count * part / nq, hi = P.count * (part + 1) / nq;
                    uint64_t base = 0;
                    if (lane == 0) base = atomicAdd(&P.queue[part], (unsigned long long)chunk);
                    base = lo + bcast_u64(base, 0);
                    base = uniform_u64(base);
                    if (base >= hi) {
                        if (++tried >= nq) { more = false; break; }
                        part = part + 1 == nq ? 0 : part + 1;
                        continue;
                    }
                    cur = base;
                    end = base + chunk < hi ? base + chunk : hi;
                }
        const uint64_t n_idle = (uint64_t)__popcll(idle);
                const uint64_t take = n_idle < end - cur ? n_idle : end - cur;
                const uint32_t r = rank_in(idle);
                const bool fresh = !alive && (uint64_t)r < take;
                uint64_t gp = 0;
                int nb = acc.box;
                if (fresh) {
                    gp = packet_id(P, cur + r);
                    nb = P.n_boxes == 1 ? 0 : box_of(sbox, P.n_boxes, gp);
                }
                const bool change = fresh && nb != acc.box;
                if (__ballot(change && acc.box >= 0)) flush(acc, change, P.tot);
                if (fresh) {
                    acc.box = nb;
                    const WalkBox &B = sbox[nb];
                    init_packet<VEL, VOIGT>(L, B, gp - B.pkt_off, P.cell_of_packet[gp], P.rec);
                    if (VOIGT) ln = line_of(B);
                    alive = true;
                }
                cur += take;
                idle = __ballot(!alive);
            }
        }
        // no live lane after a refill means the queue is drained
        if (!__ballot(alive) && !more) break;
        {
            // Every lane steps, by selects rather than branches (an idle lane
            // holds its last packet's state, or idle_lane's: its step deposits
            // nothing and reads a cell of its box), so that the lane state
            // stays in the same registers across the loop.
            uint64_t dep = 0;
            uint32_t wing = 0;
            Lane Ln = L;
            const int fate = walk_step<VEL, VOIGT>(Ln, P.rec, GlobalSink{P.A}, max_cross, dep, ln, wing, alive);
            keep_or_take(L, Ln, alive);
            const bool fin = alive && fate != kAlive;
            acc.cross += fin ? L.ncross : 0u;
            acc.esc += fin && fate == kEscaped ? L.w : 0u;
            acc.capn += fin && fate == kCapped ? 1u : 0u;
            acc.capw += fin && fate == kCapped ? L.w : 0u;
            acc.wing += fin ? wing : 0u;
            alive = alive && fate == kAlive;
        }
    }
    flush(acc, true, P.tot);
}

// ---- one thread per packet -------------------------------------------------
template <bool VEL, bool VOIGT>
__global__ __launch_bounds__(256) void walk_simple_kernel(WalkParams P)
{
    extern __shared__ WalkBox sbox[];
    for (int i = threadIdx.x; i < P.n_boxes; i += blockDim.x) sbox[i] = P.boxes[i];
    __syncthreads();
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    Acc acc{-1, 0, 0, 0, 0, 0};
    if (i < P.count) {
        const uint64_t gp = packet_id(P, i);
        const int nb = P.n_boxes == 1 ? 0 : box_of(sbox, P.n_boxes, gp);
        const WalkBox &B = sbox[nb];
        Lane L;
        init_packet<VEL, VOIGT>(L, B, gp - B.pkt_off, P.cell_of_packet[gp], P.rec);
        const Line ln = line_of(B);
        acc.box = nb;
        uint64_t dep = 0;
        uint32_t wing = 0;
        int fate;
        do {
            fate = walk_step<VEL, VOIGT>(L, P.rec, GlobalSink{P.A}, (uint32_t)P.max_cross, dep, ln, wing);
        } while (fate == kAlive);
        account(acc, L, fate, wing);
    }
    flush(acc, true, P.tot);
}

// ---- packet histories (no tallies) -------------------------------------------
template <bool VEL, bool VOIGT>
__global__ __launch_bounds__(256) void trace_kernel(WalkParams P, mc_lya_packet_trace *out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.count) return;
    const uint64_t gp = P.first + i;
    const int nb = P.n_boxes == 1 ? 0 : box_of(P.boxes, P.n_boxes, gp);
    const WalkBox B = P.boxes[nb];
    Lane L;
    float f0[3];
    init_packet<VEL, VOIGT>(L, B, gp - B.pkt_off, P.cell_of_packet[gp], P.rec, f0);
    const Line ln = line_of(B);
    mc_lya_packet_trace t;
    t.cell0 = L.c;
    t.fx = f0[0];
    t.fy = f0[1];
    t.fz = f0[2];
    t.kx = L.kx;
    t.ky = L.ky;
    t.kz = L.kz;
    t.x0 = L.x;
    uint64_t dep = 0;
    uint32_t wing = 0;
    int fate;
    do {
        fate = walk_step<VEL, VOIGT>(L, P.rec, NullSink{}, (uint32_t)P.max_cross, dep, ln, wing);
    } while (fate == kAlive);
    t.escaped = fate == kAbsorbed ? 0 : (int64_t)L.w;
    t.wing = (int64_t)wing;
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

__global__ void reset_queue_kernel(unsigned long long *q, int n)
{
    if ((int)threadIdx.x < n) q[threadIdx.x] = 0ull;
}

}  // namespace

int persistent_blocks_per_cu(bool vel, bool voigt, int block)
{
    int n = 0;
    const size_t lds = sizeof(WalkBox);
    hipError_t e;
    if (voigt)
        e = vel ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, walk_persistent_kernel<true, true>, block, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, walk_persistent_kernel<false, true>, block, lds);
    else
        e = vel ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, walk_persistent_kernel<true, false>, block, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, walk_persistent_kernel<false, false>, block, lds);
    return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_walk_persistent(const WalkParams &p, int block, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(64), 0, s, p.queue, (int)p.nqueues);
    const size_t lds = sizeof(WalkBox) * (size_t)p.n_boxes;
    const dim3 g((unsigned)grid), b((unsigned)block);
    if (p.voigt) {
        if (p.vel) hipLaunchKernelGGL((walk_persistent_kernel<true, true>), g, b, lds, s, p);
        else hipLaunchKernelGGL((walk_persistent_kernel<false, true>), g, b, lds, s, p);
    } else {
        if (p.vel) hipLaunchKernelGGL((walk_persistent_kernel<true, false>), g, b, lds, s, p);
        else hipLaunchKernelGGL((walk_persistent_kernel<false, false>), g, b, lds, s, p);
    }
    return hipGetLastError();
}

hipError_t launch_walk_simple(const WalkParams &p, int block, hipStream_t s)
{
    const uint64_t grid = (p.count + (uint64_t)block - 1) / (uint64_t)block;
    const size_t lds = sizeof(WalkBox) * (size_t)p.n_boxes;
    const dim3 g((unsigned)grid), b((unsigned)block);
    if (p.voigt) {
        if (p.vel) hipLaunchKernelGGL((walk_simple_kernel<true, true>), g, b, lds, s, p);
        else hipLaunchKernelGGL((walk_simple_kernel<false, true>), g, b, lds, s, p);
    } else {
        if (p.vel) hipLaunchKernelGGL((walk_simple_kernel<true, false>), g, b, lds, s, p);
        else hipLaunchKernelGGL((walk_simple_kernel<false, false>), g, b, lds, s, p);
    }
    return hipGetLastError();
}

hipError_t launch_trace(const WalkParams &p, mc_lya_packet_trace *out, hipStream_t s)
{
    const dim3 g((unsigned)((p.count + 255) / 256)), b(256);
    if (p.voigt) {
        if (p.vel) hipLaunchKernelGGL((trace_kernel<true, true>), g, b, 0, s, p, out);
        else hipLaunchKernelGGL((trace_kernel<false, true>), g, b, 0, s, p, out);
    } else {
        if (p.vel) hipLaunchKernelGGL((trace_kernel<true, false>), g, b, 0, s, p, out);
        else hipLaunchKernelGGL((trace_kernel<false, false>), g, b, 0, s, p, out);
    }
    return hipGetLastError();
}

hipError_t launch_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out, uint64_t n, hipStream_t s)
{
    const uint64_t grid = (n + 255) / 256;
    hipLaunchKernelGGL(philox_kernel, dim3((unsigned)grid), dim3(256), 0, s, ctr, key, out, n);
    return hipGetLastError();
}

}  // namespace mclya

// Tile-decomposed walk.
//
// Device-scope 64-bit atomics run at a fixed ~2.4e10 operations/s on this
// chip whatever the cache residency, while a packet deposits into one cell per
// crossing. So the grid is cut into tiles of kTileCells cells and the walk
// proceeds in generations: in each generation one workgroup owns one tile,
// walks every packet that is inside it, deposits into a tally in LDS (LDS
// atomics), and at the end adds that tally to the device tallies with plain
// read-modify-write (no other workgroup touches the tile's cells in that
// generation). A packet that leaves the tile is written, standing on the face
// with its pre-jump frequency, to the tile's exit region, and the region is
// indexed by face; in the next generation each tile pulls exactly the face
// lists that point at it and applies the face jump.
//
// Once a tile's input is used up, its waves thin out as packets finish; a
// wave left with only a few live lanes writes them to the tile's own
// deferred list instead, and the next generation takes them up again with
// full waves (a packet's walk does not depend on the generation that carries
// it, so the tallies are the same integers).
//
// The per-packet arithmetic is walk_core's, so the integer tallies are the
// same bits as those of the other drivers.
#include "walk_core.hpp"

namespace mclya {
namespace {

constexpr int TC = kTileCells;
constexpr int BLK = kTileBlock;
static_assert(TC % BLK == 0, "tile cells must be a multiple of the workgroup size");
constexpr int kWaves = BLK / 64;

// LDS slot of a tile cell: a 16 x 16 x kTileZ layout whatever the tile's
// extent (a tile at a box edge may be smaller), so that the slot is a shift
// and an or of the cell's offsets in the tile, not two multiplies.
static_assert(kTileX == 16 && kTileY == 16, "tile slots assume 16 x 16 cells across");
__device__ __forceinline__ int tile_slot(int32_t lx, int32_t ly, int32_t lz)
{
    return lx | (ly << 4) | (lz << 8);
}

// Deposits and opacity/velocity records of the cells of one tile, both in LDS.
// The packets' global cell index is not kept up to date inside the tile
// (kCell): the tiled walk sets it when a packet leaves.
template <bool VEL>
struct TileSink {
    static constexpr bool kCell = false;
    unsigned long long *tally;
    const float4 *rec4;          // VEL: (kappa, U) per cell
    const float *reck;           // !VEL: kappa per cell
    int32_t ox, oy, oz, sx, sy, sz;
    __device__ __forceinline__ int local(int32_t ix, int32_t iy, int32_t iz) const
    {
        return tile_slot(ix - ox, iy - oy, iz - oz);
    }
    __device__ __forceinline__ bool inside(int32_t jx, int32_t jy, int32_t jz) const
    {
        return ((uint32_t)(jx - ox) < (uint32_t)sx) & ((uint32_t)(jy - oy) < (uint32_t)sy) &
               ((uint32_t)(jz - oz) < (uint32_t)sz);
    }
    __device__ __forceinline__ void deposit(const Lane &L, uint32_t d) const
    {
        atomicAdd(&tally[local(L.ix, L.iy, L.iz)], (unsigned long long)d);
    }
    template <bool V>
    __device__ __forceinline__ Rec fetch(const void *, uint32_t, int32_t jx, int32_t jy, int32_t jz, bool stay) const
    {
        Rec r;
        const int lc = stay ? local(jx, jy, jz) : 0;    // leaving: the record is not used
        if (V) {
            const float4 v = rec4[lc];
            r.kap = v.x;
            r.ux = v.y;
            r.uy = v.z;
            r.uz = v.w;
        } else {
            r.kap = reck[lc];
            r.ux = r.uy = r.uz = 0.0f;
        }
        return r;
    }
};

__device__ __forceinline__ uint32_t rank_in(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ void save_state(PState &o, const Lane &L)
{
    o.tmx = L.tmx;
    o.tmy = L.tmy;
    o.tmz = L.tmz;
    o.tdx = L.tdx;
    o.tdy = L.tdy;
    o.tdz = L.tdz;
    o.t = L.t;
    o.w = L.w;
    o.x = L.x;
    o.kx = L.kx;
    o.ky = L.ky;
    o.kz = L.kz;
    o.ux = L.ux;
    o.uy = L.uy;
    o.uz = L.uz;
    o.cell = L.c;
    o.ncross = L.ncross;
    o.ix = L.ix;
    o.iy = L.iy;
    o.iz = L.iz;
}

__device__ __forceinline__ void load_state(Lane &L, const PState &o, const WalkBox &B)
{
    L.tmx = o.tmx;
    L.tmy = o.tmy;
    L.tmz = o.tmz;
    L.tdx = o.tdx;
    L.tdy = o.tdy;
    L.tdz = o.tdz;
    L.t = o.t;
    L.w = o.w;
    L.x = o.x;
    L.kx = o.kx;
    L.ky = o.ky;
    L.kz = o.kz;
    L.ux = o.ux;
    L.uy = o.uy;
    L.uz = o.uz;
    L.c = o.cell;
    L.ncross = o.ncross;
    L.ix = o.ix;
    L.iy = o.iy;
    L.iz = o.iz;
    L.nx = B.nx;
    L.ny = B.ny;
    L.nz = B.nz;
    L.coff = B.cell_off;
    L.delta = B.delta;
    L.xeff = B.x_eff;
}

// One generation. GEN0: the tile's input is the packets emitted in its cells
// (within the requested packet range); otherwise it is the face lists of the
// previous generation that point at this tile.
template <bool VEL, bool GEN0, bool VOIGT>
__global__ __launch_bounds__(BLK) void tile_walk_kernel(TileParams P)
{
    __shared__ unsigned long long tally[TC];
    __shared__ float4 srec4[VEL ? TC : 1];
    __shared__ float sreck[VEL ? 1 : TC];
    __shared__ uint32_t pre[GEN0 ? TC + 1 : 8];   // GEN0: cell prefix of packet counts; else list prefix
    __shared__ uint32_t lst[8];                    // pull: first index of each source list
    __shared__ uint32_t s_tsum[kWaves];
    __shared__ uint32_t s_next, s_exit, s_total, s_base;
    __shared__ uint32_t s_fcnt[8], s_fcur[8];
    __shared__ unsigned long long s_red[kWaves][5];

    const int T = blockIdx.x;
    const int tid = threadIdx.x;
    if (!GEN0) {
        const unsigned long long in_flight = *P.prev_exits;
        if (in_flight == 0) return;                 // the walk has drained (or went to the tail walk)
        if (in_flight < P.tail_min) {
            // few packets left: the tail walk takes them from the previous
            // generation's lists, and every later generation finds no exits
            if (blockIdx.x == 0 && threadIdx.x == 0) *P.tail_gen = (unsigned long long)P.gen;
            return;
        }
    }
    const TileInfo ti = P.tiles[T];
    const WalkBox B = P.boxes[ti.box];
    const Line ln = line_of(B);       // tile-uniform
    const int ncell = ti.sx * ti.sy * ti.sz;
    const uint32_t lane = __lane_id();
    const uint64_t r_lo = P.first, r_hi = P.first + P.count;

    // ---- input ----------------------------------------------------------
    uint32_t n_in = 0;
    if (GEN0) {
        // packet counts of the tile's cells, clipped to the range, scanned
        constexpr int PER = TC / BLK;
        uint32_t cnt[PER];
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int lc = tid * PER + k;
            uint32_t c = 0;
            if (lc < ncell) {
                const int lx = lc % ti.sx, ly = (lc / ti.sx) % ti.sy, lz = lc / (ti.sx * ti.sy);
                const uint32_t gc = B.cell_off + (uint32_t)(ti.ox + lx) +
                                    (uint32_t)B.nx * ((uint32_t)(ti.oy + ly) + (uint32_t)B.ny * (uint32_t)(ti.oz + lz));
                const uint64_t pf = P.pfirst[gc];
                const uint64_t lo = pf > r_lo ? pf : r_lo;
                const uint64_t pe = pf + P.npk[gc];
                const uint64_t hi = pe < r_hi ? pe : r_hi;
                c = hi > lo ? (uint32_t)(hi - lo) : 0u;
            }
            cnt[k] = c;
            sum += c;
        }
        // block exclusive scan of the per-thread sums
        uint32_t inc = sum;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(inc, off, 64);
            if ((int)lane >= off) inc += o;
        }
        if (lane == 63) s_tsum[tid >> 6] = inc;
        __syncthreads();
        if (tid == 0) {
            uint32_t run = 0;
            for (int w = 0; w < kWaves; ++w) {
                const uint32_t v = s_tsum[w];
                s_tsum[w] = run;
                run += v;
            }
            s_total = run;
        }
        __syncthreads();
        uint32_t run = s_tsum[tid >> 6] + inc - sum;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int lc = tid * PER + k;
            if (lc < ncell) pre[lc] = run;
            run += cnt[k];
        }
        if (tid == 0) pre[ncell] = s_total;
    } else {
        if (tid == 0) {
            uint32_t run = 0;
            const int32_t *src = P.tiles[T].src_tile;
            for (int k = 0; k <= ti.nsrc; ++k) {
                // the neighbours' face lists, then this tile's deferred list
                const int f = k < ti.nsrc ? (int)((ti.src_faces >> (4 * k)) & 15u) : kDeferred;
                const TileExits &e = P.in_exits[k < ti.nsrc ? src[k] : T];
                pre[k] = run;
                lst[k] = e.base + e.off[f];
                run += e.off[f + 1] - e.off[f];
            }
            pre[ti.nsrc + 1] = run;
            s_total = run;
        }
        __syncthreads();
    }
    n_in = s_total;
    if (n_in == 0) {
        if (tid == 0) {
            TileExits e;
            e.base = 0;
            for (int f = 0; f < 8; ++f) e.off[f] = 0;
            P.out_exits[T] = e;
        }
        return;
    }
    for (int q = tid; q < TC; q += BLK) {
        tally[q] = 0ull;
        const int lx = q & 15, ly = (q >> 4) & 15, lz = q >> 8;
        if (lx < ti.sx && ly < ti.sy && lz < ti.sz) {
            const uint32_t gc = B.cell_off + (uint32_t)(ti.ox + lx) +
                                (uint32_t)B.nx * ((uint32_t)(ti.oy + ly) + (uint32_t)B.ny * (uint32_t)(ti.oz + lz));
            if (VEL) srec4[q] = static_cast<const float4 *>(P.rec)[gc];
            else sreck[q] = static_cast<const float *>(P.rec)[gc];
        }
    }
    if (tid == 0) {
        s_next = 0;
        s_exit = 0;
        s_base = (uint32_t)atomicAdd(P.bump, (unsigned long long)n_in);
    }
    if (tid < 8) s_fcnt[tid] = 0;
    __syncthreads();

    // ---- walk -------------------------------------------------------------
    const TileSink<VEL> sink{tally, srec4, sreck, ti.ox, ti.oy, ti.oz, ti.sx, ti.sy, ti.sz};
    Lane L;
    idle_lane(L);               // every lane steps, so none starts undefined
    bool alive = false, more = true;
    bool fresh = false;          // wave-uniform: packets loaded since the wave's last step
    // A packet that leaves the tile parks in its lane (pending) and is written
    // out when the wave next refills or stops: one exit-writing pass for many
    // lanes instead of one per step for a few.
    bool pending = false;
    auto flush_exits = [&]() {
        if (pending) {
            const uint32_t g = s_base + atomicAdd(&s_exit, 1u);
            L.c = cell_of(L);
            save_state(P.out_state[g], L);
            // the face it left through: the one coordinate now outside the tile
            uint32_t f;
            if ((uint32_t)(L.ix - ti.ox) >= (uint32_t)ti.sx) f = L.kx > 0.0f ? 1u : 0u;
            else if ((uint32_t)(L.iy - ti.oy) >= (uint32_t)ti.sy) f = L.ky > 0.0f ? 3u : 2u;
            else f = L.kz > 0.0f ? 5u : 4u;
            P.out_face[g] = (uint8_t)f;
            atomicAdd(&s_fcnt[f], 1u);
            pending = false;
        }
    };
    uint32_t cur = 0, end = 0;
    uint64_t a_esc = 0, a_cross = 0, a_capn = 0, a_capw = 0, a_wing = 0;
    const uint32_t chunk = (uint32_t)P.chunk;
    const uint32_t refill = (uint32_t)P.refill;
    for (;;) {
        uint64_t idle = __ballot(!alive);
        // refilling stalls the whole wave on the new packets' loads: wait until
        // enough lanes are idle (or all are)
        if ((uint32_t)__popcll(idle) < refill && idle != ~0ull) idle = 0;
        if (idle && more) flush_exits();
        while (idle && more) {
            if (cur >= end) {
                uint32_t base = 0;
                if (lane == 0) base = atomicAdd(&s_next, chunk);
                base = uniform_u32(__shfl(base, 0, 64));
                if (base >= n_in) {
                    more = false;
                    break;
                }
                cur = base;
                end = base + chunk < n_in ? base + chunk : n_in;
            }
            const uint32_t take = min((uint32_t)__popcll(idle), end - cur);
            const uint32_t r = rank_in(idle);
            if (!alive && r < take) {
                const uint32_t j = cur + r;
                if (GEN0) {
                    int lo = 0, hi = ncell - 1;             // largest cell with pre <= j
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (pre[mid] <= j) lo = mid; else hi = mid - 1;
                    }
                    const int lx = lo % ti.sx, ly = (lo / ti.sx) % ti.sy, lz = lo / (ti.sx * ti.sy);
                    const uint32_t gc = B.cell_off + (uint32_t)(ti.ox + lx) +
                                        (uint32_t)B.nx * ((uint32_t)(ti.oy + ly) + (uint32_t)B.ny * (uint32_t)(ti.oz + lz));
                    const uint64_t pf = P.pfirst[gc];
                    const uint64_t gp = (pf > r_lo ? pf : r_lo) + (j - pre[lo]);
                    init_packet<VEL, VOIGT>(L, B, gp - B.pkt_off, gc, P.rec);
                } else {
                    int k = 0;
                    while (k + 1 <= ti.nsrc && pre[k + 1] <= j) ++k;
                    const uint32_t g = P.in_idx[lst[k] + (j - pre[k])];
                    load_state(L, P.in_state[g], B);
                    const Rec r = sink.template fetch<VEL>(P.rec, L.c, L.ix, L.iy, L.iz, true);
                    if (k < ti.nsrc) finish_entry<VEL>(L, r);   // entering through a face
                    else L.kap = r.kap;                         // deferred inside its cell
                }
                alive = true;
            }
            fresh = true;
            cur += take;
            idle = __ballot(!alive);
        }
        const uint64_t live = __ballot(alive);
        // no live lane after the refill means the input is used up (a wave
        // with idle lanes refills while there is input)
        if (!live && !more) {
            flush_exits();
            break;
        }
        // (only after a step, so every deferred packet has moved in this generation)
        if (!more && !fresh && n_in >= P.defer_min && (uint32_t)__popcll(live) <= (uint32_t)P.defer_lanes) {
            flush_exits();
            if (alive) {
                const uint32_t g = s_base + atomicAdd(&s_exit, 1u);
                L.c = cell_of(L);
                save_state(P.out_state[g], L);
                P.out_face[g] = (uint8_t)kDeferred;
                atomicAdd(&s_fcnt[kDeferred], 1u);
            }
            break;
        }
        fresh = false;
        {
            // Every lane steps, by selects rather than branches: an idle lane's
            // step deposits nothing and reads an in-tile record, and the idle
            // lane keeps its state. Branches here made the compiler copy the
            // lane state and the totals on every step.
            uint64_t dep = 0;
            uint32_t wing = 0;
            Lane Ln = L;
            const int fate = walk_step<VEL, VOIGT>(Ln, P.rec, sink, P.max_cross, dep, ln, wing, alive);
            keep_or_take(L, Ln, alive);
            const bool fin = alive && fate != kAlive && fate != kExit;
            a_cross += fin ? L.ncross : 0u;
            a_esc += alive && fate == kEscaped ? L.w : 0u;
            a_capn += alive && fate == kCapped ? 1u : 0u;
            a_capw += alive && fate == kCapped ? L.w : 0u;
            if (VOIGT) a_wing += fin ? wing : 0u;
            pending = pending || (alive && fate == kExit);
            alive = alive && fate == kAlive;
        }
    }

    // ---- finish: tally, totals, face lists of the exits ----------------------
    a_esc = wave_sum(a_esc);
    a_cross = wave_sum(a_cross);
    a_capn = wave_sum(a_capn);
    a_capw = wave_sum(a_capw);
    if (VOIGT) a_wing = wave_sum(a_wing);
    if (lane == 0) {
        s_red[tid >> 6][0] = a_esc;
        s_red[tid >> 6][1] = a_cross;
        s_red[tid >> 6][2] = a_capn;
        s_red[tid >> 6][3] = a_capw;
        s_red[tid >> 6][4] = a_wing;
    }
    __threadfence_block();
    __syncthreads();
    for (int q = tid; q < TC; q += BLK) {
        const unsigned long long v = tally[q];
        if (v) {
            const int lx = q & 15, ly = (q >> 4) & 15, lz = q >> 8;
            const uint32_t gc = B.cell_off + (uint32_t)(ti.ox + lx) +
                                (uint32_t)B.nx * ((uint32_t)(ti.oy + ly) + (uint32_t)B.ny * (uint32_t)(ti.oz + lz));
            P.A[gc] += v;    // this workgroup alone owns these cells in this generation
        }
    }
    if (tid < (VOIGT ? 5 : 4)) {
        unsigned long long t = 0;
        for (int w = 0; w < kWaves; ++w) t += s_red[w][tid];
        if (t) {
            unsigned long long *dst = tid == 0 ? &P.tot[ti.box].escaped
                                   : tid == 1 ? &P.tot[ti.box].crossings
                                   : tid == 2 ? &P.tot[ti.box].capped_packets
                                   : tid == 3 ? &P.tot[ti.box].capped_weight
                                              : &P.tot[ti.box].wing;
            atomicAdd(dst, t);
        }
    }
    const uint32_t n_exit = s_exit;
    if (tid == 0) {
        TileExits e;
        e.base = s_base;
        uint32_t run = 0;
        for (int f = 0; f <= kDeferred; ++f) {
            e.off[f] = run;
            s_fcur[f] = run;
            run += s_fcnt[f];
        }
        e.off[kDeferred + 1] = run;
        P.out_exits[T] = e;
        if (n_exit) atomicAdd(P.exits, (unsigned long long)n_exit);
    }
    __syncthreads();
    for (uint32_t k = tid; k < n_exit; k += BLK) {
        const uint32_t g = s_base + k;
        const uint32_t pos = atomicAdd(&s_fcur[P.out_face[g]], 1u);
        P.out_idx[s_base + pos] = g;
    }
}

// ---- tail walk -----------------------------------------------------------
// Exclusive prefix of the tail packets over tiles (one block).
__global__ __launch_bounds__(1024) void tail_prefix_kernel(TailParams P)
{
    __shared__ uint32_t s_wsum[16];
    __shared__ uint32_t s_carry;
    const unsigned long long g = P.counters[kTailGenSlot];
    if (g == 0) {
        if (threadIdx.x == 0) P.counters[kTailCountSlot] = 0;
        return;
    }
    const TileExits *ex = P.exits[(g - 1) & 1];
    const uint32_t lane = __lane_id(), wid = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int base = 0; base < P.ntiles; base += 1024) {
        const int t = base + (int)threadIdx.x;
        const uint32_t v = t < P.ntiles ? ex[t].off[kDeferred + 1] : 0u;
        uint32_t inc = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(inc, off, 64);
            if ((int)lane >= off) inc += o;
        }
        if (lane == 63) s_wsum[wid] = inc;
        __syncthreads();
        uint32_t before = s_carry;
        for (uint32_t w = 0; w < wid; ++w) before += s_wsum[w];
        if (t < P.ntiles) P.prefix[t] = before + inc - v;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t all = 0;
            for (int w = 0; w < 16; ++w) all += s_wsum[w];
            s_carry += all;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) P.counters[kTailCountSlot] = s_carry;
}

template <bool VEL, bool VOIGT>
__global__ __launch_bounds__(256) void tail_walk_kernel(TailParams P)
{
    const unsigned long long g = P.counters[kTailGenSlot];
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t esc = 0, cross = 0, capn = 0, capw = 0, gw = 0;
    int box = -1;
    if (g != 0 && i < P.counters[kTailCountSlot]) {
        const int q = (int)((g - 1) & 1);
        int lo = 0, hi = P.ntiles - 1;             // the tile whose list holds packet i
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (P.prefix[mid] <= (uint32_t)i) lo = mid; else hi = mid - 1;
        }
        const TileExits e = P.exits[q][lo];
        const uint32_t k = P.idx[q][e.base + ((uint32_t)i - P.prefix[lo])];
        box = P.tiles[lo].box;
        const WalkBox B = P.boxes[box];
        Lane L;
        load_state(L, P.state[q][k], B);
        const Rec r = load_rec<VEL>(P.rec, L.c);
        if (P.face[q][k] == kDeferred) L.kap = r.kap;   // deferred inside its cell
        else finish_entry<VEL>(L, r);                   // entering through a face
        const Line ln = line_of(B);
        uint64_t dep = 0;
        uint32_t wing = 0;
        int fate;
        do {
            fate = walk_step<VEL, VOIGT>(L, P.rec, GlobalSink{P.A}, P.max_cross, dep, ln, wing);
        } while (fate == kAlive);
        cross = L.ncross;
        esc = fate == kEscaped ? L.w : 0;
        capn = fate == kCapped ? 1 : 0;
        capw = fate == kCapped ? L.w : 0;
        gw = wing;
    }
    // per-box totals: one atomic per box present in the wave
    uint64_t pending = __ballot(box >= 0);
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int b = __shfl(box, leader, 64);
        const bool mine = box == b;
        const uint64_t se = wave_sum(mine ? esc : 0), sc = wave_sum(mine ? cross : 0),
                       sn = wave_sum(mine ? capn : 0), sw = wave_sum(mine ? capw : 0);
        const uint64_t sg = VOIGT ? wave_sum(mine ? gw : 0) : 0;
        if ((int)__lane_id() == leader) {
            if (sg) atomicAdd(&P.tot[b].wing, (unsigned long long)sg);
            if (se) atomicAdd(&P.tot[b].escaped, (unsigned long long)se);
            if (sc) atomicAdd(&P.tot[b].crossings, (unsigned long long)sc);
            if (sn) atomicAdd(&P.tot[b].capped_packets, (unsigned long long)sn);
            if (sw) atomicAdd(&P.tot[b].capped_weight, (unsigned long long)sw);
        }
        pending &= ~__ballot(mine);
    }
}

__global__ void zero_counters_kernel(unsigned long long *c, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] = 0ull;
}

}  // namespace

hipError_t launch_tile_generation(const TileParams &p, bool gen0, bool vel, bool voigt, hipStream_t s)
{
    const dim3 grid((unsigned)p.ntiles), block(BLK);
    if (voigt) {
        if (gen0) {
            if (vel) hipLaunchKernelGGL((tile_walk_kernel<true, true, true>), grid, block, 0, s, p);
            else hipLaunchKernelGGL((tile_walk_kernel<false, true, true>), grid, block, 0, s, p);
        } else {
            if (vel) hipLaunchKernelGGL((tile_walk_kernel<true, false, true>), grid, block, 0, s, p);
            else hipLaunchKernelGGL((tile_walk_kernel<false, false, true>), grid, block, 0, s, p);
        }
    } else {
        if (gen0) {
            if (vel) hipLaunchKernelGGL((tile_walk_kernel<true, true, false>), grid, block, 0, s, p);
            else hipLaunchKernelGGL((tile_walk_kernel<false, true, false>), grid, block, 0, s, p);
        } else {
            if (vel) hipLaunchKernelGGL((tile_walk_kernel<true, false, false>), grid, block, 0, s, p);
            else hipLaunchKernelGGL((tile_walk_kernel<false, false, false>), grid, block, 0, s, p);
        }
    }
    return hipGetLastError();
}

hipError_t launch_tail_walk(const TailParams &p, uint64_t capacity, bool vel, bool voigt, hipStream_t s)
{
    hipLaunchKernelGGL(tail_prefix_kernel, dim3(1), dim3(1024), 0, s, p);
    const dim3 grid((unsigned)std::max<uint64_t>(1, (capacity + 255) / 256));
    if (voigt) {
        if (vel) hipLaunchKernelGGL((tail_walk_kernel<true, true>), grid, dim3(256), 0, s, p);
        else hipLaunchKernelGGL((tail_walk_kernel<false, true>), grid, dim3(256), 0, s, p);
    } else {
        if (vel) hipLaunchKernelGGL((tail_walk_kernel<true, false>), grid, dim3(256), 0, s, p);
        else hipLaunchKernelGGL((tail_walk_kernel<false, false>), grid, dim3(256), 0, s, p);
    }
    return hipGetLastError();
}

hipError_t launch_zero_counters(unsigned long long *c, int n, hipStream_t s)
{
    hipLaunchKernelGGL(zero_counters_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, c, n);
    return hipGetLastError();
}

}  // namespace mclya

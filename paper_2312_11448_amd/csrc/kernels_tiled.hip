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
constexpr uint32_t kMinClaim = 8;   // smallest claim on a tile's input

// LDS slots: the tile's cells with a ring of one slot round them, in a
// (kTileX + 2) x (kTileY + 2) x (kTileZ + 2) layout whatever the tile's extent
// (a tile at a box edge may be smaller). Every slot that is not a cell of the
// tile (the ring, and the rest of the layout in a smaller tile) holds the
// record kOutside, so a packet about to step out of the tile finds out by
// reading the record of the slot it would enter: no per-packet count of the
// faces left before the tile's edge.
static_assert(kTileX == 16 && kTileY == 16, "the cell loops take rows and planes of 16 cells");
constexpr int kSX = kTileX + 2, kSY = kTileY + 2, kSZ = kTileZ + 2;
constexpr int kSlots = kSX * kSY * kSZ;
constexpr uint32_t kOutside = 0xFFFFFFFFu;   // kappa bits of a slot outside the tile (a NaN)
__device__ __forceinline__ int tile_slot(int32_t lx, int32_t ly, int32_t lz)
{
    return (lx + 1) + kSX * ((ly + 1) + kSY * (lz + 1));
}

// The cell offsets in the tile of slot s (-1 or the extent on the ring).
__device__ __forceinline__ void slot_cell(int32_t s, int32_t &lx, int32_t &ly, int32_t &lz)
{
    const int32_t r = s % (kSX * kSY);
    lz = s / (kSX * kSY) - 1;
    ly = r / kSX - 1;
    lx = r % kSX - 1;
}

// The tile a workgroup walks, uniform over it: the box's drift, escape
// threshold and line constants, the tile's origin and extent, and the axes
// along which it spans the whole box (the grid wraps round inside it).
struct TileCtx {
    float delta, xeff;
    uint32_t max_cross;
    Line ln;
    int32_t ox, oy, oz, sx, sy, sz;
    uint32_t span;
};

// A packet inside a tile. Ray geometry and line state are a Lane's; the cell
// is tracked by its record's byte offset q in the tile's LDS (RS bytes per
// record), with the change of q for a step along each axis. A step is then an
// add, where global cell coordinates would need the box's periodic wrap and
// the neighbour's index; they are formed only when the packet leaves the
// tile (found from the record of the slot it steps into, kOutside).
struct TLane {
    double tmx, tmy, tmz, tdx, tdy, tdz, t;
    float kx, ky, kz;
    float x, kap, ku;
    uint32_t w, ncross;
    int32_t q;
    int32_t dqx, dqy, dqz;
};

// The LDS tally of the cell whose record is at byte offset q (8-byte tallies).
template <int RS>
__device__ __forceinline__ unsigned long long *tally_of(unsigned long long *tally, int32_t q)
{
    const uint32_t b = RS >= 8 ? (uint32_t)q / (uint32_t)(RS / 8) : (uint32_t)q * (uint32_t)(8 / RS);
    return reinterpret_cast<unsigned long long *>(reinterpret_cast<char *>(tally) + b);
}

template <bool VEL>
__device__ __forceinline__ Rec rec_at(const char *recs, int32_t q)
{
    Rec r;
    if (VEL) {
        const float4 v = *reinterpret_cast<const float4 *>(recs + q);
        r.kap = v.x;
        r.ux = v.y;
        r.uy = v.z;
        r.uz = v.w;
    } else {
        r.kap = *reinterpret_cast<const float *>(recs + q);
        r.ux = r.uy = r.uz = 0.0f;
    }
    return r;
}

// A packet standing in cell (L.ix, L.iy, L.iz) of this tile, as a TLane.
template <int RS>
__device__ __forceinline__ void to_tile(TLane &T, const Lane &L, const TileCtx &C)
{
    T.tmx = L.tmx;
    T.tmy = L.tmy;
    T.tmz = L.tmz;
    T.tdx = L.tdx;
    T.tdy = L.tdy;
    T.tdz = L.tdz;
    T.t = L.t;
    T.kx = L.kx;
    T.ky = L.ky;
    T.kz = L.kz;
    T.x = L.x;
    T.kap = L.kap;
    T.ku = L.ku;
    T.w = L.w;
    T.ncross = L.ncross;
    T.q = tile_slot(L.ix - C.ox, L.iy - C.oy, L.iz - C.oz) * RS;
    // the walk steps +1 along an axis when the direction's component is > 0, else -1
    T.dqx = L.kx > 0.0f ? RS : -RS;
    T.dqy = L.ky > 0.0f ? kSX * RS : -kSX * RS;
    T.dqz = L.kz > 0.0f ? kSX * kSY * RS : -kSX * kSY * RS;
}

// Global coordinates of a TLane's cell.
template <int RS>
__device__ __forceinline__ void tile_cell(const TLane &T, const TileCtx &C, int32_t &ix, int32_t &iy, int32_t &iz)
{
    int32_t lx, ly, lz;
    slot_cell((int32_t)((uint32_t)T.q / (uint32_t)RS), lx, ly, lz);
    ix = C.ox + lx;
    iy = C.oy + ly;
    iz = C.oz + lz;
}

// Along an axis the tile spans, one cell past either end of the tile is its
// other end (the box is periodic and the tile is the whole box that way).
template <int RS>
__device__ __forceinline__ int32_t wrap_slot(const TLane &L, int32_t qn, const Face &f, const TileCtx &C)
{
    int32_t lx, ly, lz;
    slot_cell((int32_t)((uint32_t)L.q / (uint32_t)RS), lx, ly, lz);
    if (f.bx && (C.span & 1u)) {
        const int32_t m = L.kx > 0.0f ? (lx + 1 == C.sx ? 0 : lx + 1) : (lx == 0 ? C.sx - 1 : lx - 1);
        qn = L.q + (m - lx) * RS;
    } else if (f.by && (C.span & 2u)) {
        const int32_t m = L.ky > 0.0f ? (ly + 1 == C.sy ? 0 : ly + 1) : (ly == 0 ? C.sy - 1 : ly - 1);
        qn = L.q + (m - ly) * (kSX * RS);
    } else if (f.bz && (C.span & 4u)) {
        const int32_t m = L.kz > 0.0f ? (lz + 1 == C.sz ? 0 : lz + 1) : (lz == 0 ? C.sz - 1 : lz - 1);
        qn = L.q + (m - lz) * (kSX * kSY * RS);
    }
    return qn;
}

// Outcome of one step of a TLane.
struct TStep {
    bool walked;     // crossed a cell (deposited and counted)
    bool alive;      // walks on inside the tile
    bool exit;       // stands on the tile's edge, to be handed to the neighbour
    bool fin;        // finished: absorbed, escaped or capped
    bool escaped;    // finished by escape (its weight escapes)
    bool capped;     // finished at the crossing cap
    uint32_t wing;   // Voigt: the far wing's share of an escaping packet's weight
};

// One (packet, cell) segment inside a tile: the same face choice, line
// physics, deposit and face jump as walk_step, so that the integers are the
// same bits as those of every other driver. A packet whose next cell lies
// outside the tile stops on the face with its geometry not yet advanced, its
// drifted pre-jump frequency and its cell's velocity (save_exit completes the
// crossing). act = false leaves the lane's state as it is (an idle lane, or
// one waiting to be written out) and deposits nothing.
// The deposit of a step is issued in the next one, right after that step's
// record read (dep_q, dep_w: the cell's record offset and the weight; a lane
// that deposited nothing holds its spare slot spare_q and 0): the LDS atomic
// then runs while the step computes, and waiting for the record does not wait
// for it.
template <bool VEL, bool VOIGT, bool WRAP, int RS>
__device__ __forceinline__ TStep tile_step(TLane &L, bool act, const TileCtx &C, const char *recs,
                                           unsigned long long *tally, int32_t &dep_q, uint32_t &dep_w,
                                           int32_t spare_q)
{
    TStep o;
    const bool gone = VOIGT ? (L.x <= -C.xeff) | (L.x > C.ln.xblue) : L.x <= -C.xeff;
    const bool capped = !gone && L.ncross >= C.max_cross;
    const bool walk = act && !gone && !capped;
    const Face f = next_face(L.tmx, L.tmy, L.tmz);
    // sums of field-or-zero terms: a choice between fields would make the
    // compiler address the lane state in (scratch) memory
    int32_t qn = L.q + (f.bx ? L.dqx : 0) + (f.by ? L.dqy : 0) + (f.bz ? L.dqz : 0);
    // along an axis the tile spans, the step wraps round to the tile's other end
    if (WRAP) qn = wrap_slot<RS>(L, qn, f, C);
    // the next slot's record, in flight during the profile arithmetic; the
    // ring round the tile holds kOutside
    const Rec nr = rec_at<VEL>(recs, qn);
    // the last step's deposit, issued after the record read so that waiting
    // for the record does not wait for it; every lane issues it (a lane with
    // nothing to deposit adds 0 to a ring slot of its own), so the wait's
    // count is the same on every path
    atomicAdd(tally_of<RS>(tally, dep_q), (unsigned long long)dep_w);
    const Segment g = segment<VOIGT>(L.x, (float)(f.tn - L.t), C.delta, C.xeff, L.kap, L.w, walk, C.ln);
    dep_q = walk ? L.q : spare_q;   // the deposit goes into the cell being left
    dep_w = g.d;
    L.w -= g.d;
    L.ncross += walk ? 1u : 0u;
    o.walked = walk;
    const bool stay = __float_as_uint(nr.kap) != kOutside;
    const bool live = walk && !g.esc && L.w != 0u;
    o.alive = live && stay;
    o.exit = live && !stay;
    o.fin = act && !live;
    o.escaped = act && (gone || (walk && g.esc));
    o.capped = act && capped;
    o.wing = 0u;
    if (VOIGT && o.escaped) o.wing = wing_share(L.w, gone ? L.x : -C.xeff, C.ln);
    // cross the face (packets that walk on inside the tile). The path length
    // walked advances for every lane: a packet that stops here is written out
    // from its face distances (save_exit), not from t, and an idle lane's
    // next segment is then empty.
    const bool mv = o.alive;
    L.tmx = (mv && f.bx) ? L.tmx + L.tdx : L.tmx;
    L.tmy = (mv && f.by) ? L.tmy + L.tdy : L.tmy;
    L.tmz = (mv && f.bz) ? L.tmz + L.tdz : L.tmz;
    L.t = f.tn;
    L.q = mv ? qn : L.q;
    // the bulk term of Eq. (inout) on entering the new cell; a packet that
    // leaves keeps its pre-jump frequency
    if (VEL) {
        const float kn = ray_velocity(L.kx, L.ky, L.kz, nr);
        const float xj = g.xo - (kn - L.ku);
        L.x = act ? (mv ? xj : g.xo) : L.x;
        L.ku = mv ? kn : L.ku;
    } else {
        L.x = act ? g.xo : L.x;
    }
    L.kap = mv ? nr.kap : L.kap;
    return o;
}

// A lane that holds no packet: no weight, far below any escape threshold.
__device__ __forceinline__ void idle_tlane(TLane &T, int32_t rs)
{
    T.tmx = T.tmy = T.tmz = 1.0;
    T.tdx = T.tdy = T.tdz = 1.0;
    T.t = 0.0;
    T.kx = 1.0f;
    T.ky = T.kz = 0.0f;
    T.x = -3.0e38f;
    T.kap = 0.0f;
    T.ku = 0.0f;
    T.w = 0u;
    T.ncross = 0u;
    T.q = tile_slot(0, 0, 0) * rs;    // a cell of every tile
    T.dqx = rs;
    T.dqy = kSX * rs;
    T.dqz = kSX * kSY * rs;
}

// A packet standing on the tile's edge, written for the neighbouring tile:
// the face crossing that tile_step left undone (the same face choice and
// FP64 advance as walk_step, and the next cell with the box's periodic wrap),
// with the pre-jump frequency and the velocity of the cell it leaves.
template <int RS>
__device__ __forceinline__ uint32_t save_exit(PState &o, const TLane &L, const TileCtx &C, const WalkBox &B)
{
    const Face f = next_face(L.tmx, L.tmy, L.tmz);
    int32_t ix, iy, iz;
    tile_cell<RS>(L, C, ix, iy, iz);
    const int32_t ci = (f.bx ? ix : 0) + (f.by ? iy : 0) + (f.bz ? iz : 0);
    const int32_t ni = (f.bx ? B.nx : 0) + (f.by ? B.ny : 0) + (f.bz ? B.nz : 0);
    const bool up = (f.bx & (L.kx > 0.0f)) | (f.by & (L.ky > 0.0f)) | (f.bz & (L.kz > 0.0f));
    int32_t mi = ci + (up ? 1 : -1);
    mi = mi == ni ? 0 : mi;
    mi = mi < 0 ? ni - 1 : mi;
    const int32_t jx = f.bx ? mi : ix, jy = f.by ? mi : iy, jz = f.bz ? mi : iz;
    o.tmx = f.bx ? L.tmx + L.tdx : L.tmx;
    o.tmy = f.by ? L.tmy + L.tdy : L.tmy;
    o.tmz = f.bz ? L.tmz + L.tdz : L.tmz;
    o.tdx = L.tdx;
    o.tdy = L.tdy;
    o.tdz = L.tdz;
    o.t = f.tn;
    o.w = L.w;
    o.x = L.x;
    o.kx = L.kx;
    o.ky = L.ky;
    o.kz = L.kz;
    o.ku = L.ku;
    o.cell = B.cell_off + (uint32_t)jx + (uint32_t)B.nx * ((uint32_t)jy + (uint32_t)B.ny * (uint32_t)jz);
    o.ncross = L.ncross;
    o.ix = jx;
    o.iy = jy;
    o.iz = jz;
    return (f.bx ? 0u : (f.by ? 2u : 4u)) + (up ? 1u : 0u);   // the face it leaves through
}

// A packet deferred to the tile's next generation, standing inside its cell.
template <int RS>
__device__ __forceinline__ void save_here(PState &o, const TLane &L, const TileCtx &C, const WalkBox &B)
{
    int32_t ix, iy, iz;
    tile_cell<RS>(L, C, ix, iy, iz);
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
    o.ku = L.ku;
    o.cell = B.cell_off + (uint32_t)ix + (uint32_t)B.nx * ((uint32_t)iy + (uint32_t)B.ny * (uint32_t)iz);
    o.ncross = L.ncross;
    o.ix = ix;
    o.iy = iy;
    o.iz = iz;
}

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
    L.ku = o.ku;
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

// The tile's totals in LDS, in the order of the box totals they add to.
constexpr int kTotEscaped = 0, kTotCrossings = 1, kTotCapped = 2, kTotCappedWeight = 3, kTotWing = 4;

// Running total of a wave: crossings walked in this generation, counted from
// the wave's step masks (the same in every lane). Escaping and capped
// packets, one event per packet, go to the tile's LDS totals.
struct TileAcc {
    uint32_t cross;
};

// The walk of one tile's input by one workgroup (all its waves): refill
// idle lanes from the input list, step every lane, park packets that reach
// the tile's edge and write them out at the next refill, defer thin waves.
template <bool VEL, bool GEN0, bool VOIGT, bool WRAP>
__device__ __forceinline__ void walk_tile(const TileParams &P, const TileInfo &ti, const WalkBox &B,
                                          const TileCtx &C, uint32_t n_in, const uint32_t *pre, const uint32_t *lst,
                                          const char *recs, unsigned long long *tally, uint32_t *s_next,
                                          uint32_t *s_exit, uint32_t s_base, uint32_t *s_fcnt,
                                          unsigned long long *s_tot, TileAcc &acc)
{
    constexpr int RS = VEL ? 16 : 4;
    const int ncell = ti.sx * ti.sy * ti.sz;
    const uint32_t lane = __lane_id();
    const uint64_t r_lo = P.first;
    TLane L;
    idle_tlane(L, RS);          // every lane steps, so none starts undefined
    bool alive = false, more = true;
    bool fresh = false;          // wave-uniform: packets loaded since the wave's last step
    // A packet that reaches the tile's edge parks in its lane and is written
    // out when the wave next refills or stops: one exit-writing pass for many
    // lanes instead of one per step for a few. A lane is parked when it is not
    // live yet holds weight (a finished packet's lane holds none).
    auto flush_exits = [&]() {
        const bool parked = !alive && L.w != 0u;
        if (__ballot(parked)) {
            if (parked) {
                const uint32_t g = s_base + atomicAdd(s_exit, 1u);
                const uint32_t f = save_exit<RS>(P.out_state[g], L, C, B);
                P.out_face[g] = (uint8_t)f;
                atomicAdd(&s_fcnt[f], 1u);
                L.w = 0u;
            }
        }
    };
    uint32_t cur = 0, end = 0;
    const uint32_t chunk = (uint32_t)P.chunk;
    // refilling stalls the whole wave on the new packets' loads: wait until
    // this many lanes are idle (1..64; 64 waits for all)
    const uint32_t refill = (uint32_t)min(max(P.refill, 1), 64);
    // a ring slot of this lane's own (the ring's z = -1 plane has 324 slots),
    // whose tally is never read: where a lane with nothing to deposit adds 0
    const int32_t spare_q = tile_slot((int32_t)(lane % kSX) - 1, (int32_t)(lane / kSX) - 1, -1) * RS;
    int32_t dep_q = spare_q;     // the last step's deposit, not yet issued
    uint32_t dep_w = 0;
    for (;;) {
        uint64_t idle = __ballot(!alive);
        if (more && (uint32_t)__popcll(idle) >= refill) {
        flush_exits();
        while (idle && more) {
            if (cur >= end) {
                // near the end of the input the claims shrink, so that the
                // last packets spread over the waves instead of leaving one
                // wave with a whole chunk while the others are done
                uint32_t base = 0, want = 0;
                if (lane == 0) {
                    const uint32_t seen = __hip_atomic_load(s_next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    const uint32_t left = seen < n_in ? n_in - seen : 0u;
                    want = left < chunk * kWaves ? max(left / kWaves, min(chunk, kMinClaim)) : chunk;
                    base = atomicAdd(s_next, want);
                }
                base = uniform_u32(__shfl(base, 0, 64));
                want = uniform_u32(__shfl(want, 0, 64));
                if (base >= n_in) {
                    more = false;
                    break;
                }
                cur = base;
                end = base + want < n_in ? base + want : n_in;
            }
            const uint32_t take = min((uint32_t)__popcll(idle), end - cur);
            const uint32_t r = rank_in(idle);
            if (!alive && r < take) {
                const uint32_t j = cur + r;
                Lane N;
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
                    emit_packet<VOIGT>(N, B, gp - B.pkt_off, gc);
                    const Rec rc = rec_at<VEL>(recs, tile_slot(lx, ly, lz) * RS);   // the emission cell's record
                    N.kap = rc.kap;
                    N.ku = VEL ? ray_velocity(N.kx, N.ky, N.kz, rc) : 0.0f;
                } else {
                    // the list holding position j (independent reads of the
                    // list prefix, not a chain)
                    int k = 0;
#pragma unroll
                    for (int m = 1; m <= 6; ++m) k += (m <= ti.nsrc && pre[m] <= j) ? 1 : 0;
                    const uint32_t g = P.in_idx[lst[k] + (j - pre[k])];
                    load_state(N, P.in_state[g], B);
                    const Rec rc = rec_at<VEL>(recs, tile_slot(N.ix - ti.ox, N.iy - ti.oy, N.iz - ti.oz) * RS);
                    if (k < ti.nsrc) finish_entry<VEL>(N, rc);   // entering through a face
                    else N.kap = rc.kap;                         // deferred inside its cell
                }
                to_tile<RS>(L, N, C);
                alive = true;
            }
            fresh = true;
            cur += take;
            idle = __ballot(!alive);
        }
        }
        // The wave stops once the input is used up and no lane is live (while
        // there is input, a wave with every lane idle refills), or, once the
        // input is used up, when few lanes are live (deferred). One exit, on
        // a value the compiler sees as uniform, keeps the loop's state in
        // scalar registers where it is uniform.
        uint32_t stop = 0;
        if (!more) {
            const uint64_t live = __ballot(alive);
            if (!live) {
                flush_exits();
                stop = 1;
            } else if (!fresh && n_in >= P.defer_min && (uint32_t)__popcll(live) <= (uint32_t)P.defer_lanes) {
                // (only after a step, so every deferred packet has moved in this generation)
                flush_exits();
                if (alive) {
                    const uint32_t g = s_base + atomicAdd(s_exit, 1u);
                    save_here<RS>(P.out_state[g], L, C, B);
                    P.out_face[g] = (uint8_t)kDeferred;
                    atomicAdd(&s_fcnt[kDeferred], 1u);
                }
                stop = 1;
            }
        }
        if (uniform_u32(stop)) break;
        fresh = false;
        // Every lane steps: an idle or parked lane's step changes nothing and
        // deposits nothing (selects, not branches, keep the lane state in the
        // same registers round the loop).
        const TStep o = tile_step<VEL, VOIGT, WRAP, RS>(L, alive, C, recs, tally, dep_q, dep_w, spare_q);
        // (wave-uniform counts kept in scalar registers)
        acc.cross = uniform_u32(acc.cross + (uint32_t)__popcll(__ballot(o.walked)));
        if (o.escaped) {         // rare: the tile's LDS totals
            atomicAdd(&s_tot[kTotEscaped], (unsigned long long)L.w);
            if (VOIGT && o.wing) atomicAdd(&s_tot[kTotWing], (unsigned long long)o.wing);
        }
        if (o.capped) {
            atomicAdd(&s_tot[kTotCapped], 1ull);
            atomicAdd(&s_tot[kTotCappedWeight], (unsigned long long)L.w);
        }
        L.w = (o.escaped || o.capped) ? 0u : L.w;   // counted: the lane holds nothing
        alive = o.alive;
    }
    if (dep_w) atomicAdd(tally_of<RS>(tally, dep_q), (unsigned long long)dep_w);
}

// The tile's records into LDS (rows of 16 cells read together), with its
// tallies zeroed, and the record kOutside in every other slot.
template <bool VEL>
__device__ __forceinline__ void load_tile_records(const TileParams &P, const TileInfo &ti, const WalkBox &B,
                                                  float4 *srec4, float *sreck, unsigned long long *tally, int tid)
{
    for (int q = tid; q < TC; q += BLK) {
        const int lx = q & 15, ly = (q >> 4) & 15, lz = q >> 8;
        if (lx < ti.sx && ly < ti.sy && lz < ti.sz) {
            const int sl = tile_slot(lx, ly, lz);
            const uint32_t gc = B.cell_off + (uint32_t)(ti.ox + lx) +
                                (uint32_t)B.nx * ((uint32_t)(ti.oy + ly) + (uint32_t)B.ny * (uint32_t)(ti.oz + lz));
            tally[sl] = 0ull;
            if (VEL) srec4[sl] = static_cast<const float4 *>(P.rec)[gc];
            else sreck[sl] = static_cast<const float *>(P.rec)[gc];
        }
    }
    for (int sl = tid; sl < kSlots; sl += BLK) {
        int32_t lx, ly, lz;
        slot_cell(sl, lx, ly, lz);
        const bool in = (uint32_t)lx < (uint32_t)ti.sx && (uint32_t)ly < (uint32_t)ti.sy && (uint32_t)lz < (uint32_t)ti.sz;
        if (!in) {
            if (VEL) srec4[sl] = make_float4(__uint_as_float(kOutside), 0.0f, 0.0f, 0.0f);
            else sreck[sl] = __uint_as_float(kOutside);
        }
    }
}

// One generation. GEN0: the tile's input is the packets emitted in its cells
// (within the requested packet range); otherwise it is the face lists of the
// previous generation that point at this tile.
template <bool VEL, bool GEN0, bool VOIGT>
__global__ __launch_bounds__(BLK) void tile_walk_kernel(TileParams P)
{
    __shared__ unsigned long long tally[kSlots];   // slots of the tile's cells are used
    __shared__ float4 srec4[VEL ? kSlots : 1];
    __shared__ float sreck[VEL ? 1 : kSlots];
    __shared__ uint32_t pre[GEN0 ? TC + 1 : 8];   // GEN0: cell prefix of packet counts; else list prefix
    __shared__ uint32_t lst[8];                    // pull: first index of each source list
    __shared__ uint32_t s_tsum[kWaves];
    __shared__ uint32_t s_next, s_exit, s_total, s_base;
    __shared__ uint32_t s_fcnt[8], s_fcur[8];
    __shared__ unsigned long long s_red[kWaves];   // crossings of each wave
    __shared__ unsigned long long s_tot[5];        // escaped weight, -, capped packets and weight, wing

    const int T = blockIdx.x;
    const int tid = threadIdx.x;
    // (the tile's entry is read alongside the count of packets in flight)
    const TileInfo ti = P.tiles[T];
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
    const WalkBox B = P.boxes[ti.box];
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
        // the neighbours' face lists, then this tile's deferred list: one
        // thread per list reads its extent (independent reads), while every
        // thread loads the tile's records
        if (tid <= ti.nsrc) {
            const int k = tid;
            const int f = k < ti.nsrc ? (int)((ti.src_faces >> (4 * k)) & 15u) : kDeferred;
            const TileExits &e = P.in_exits[k < ti.nsrc ? P.tiles[T].src_tile[k] : T];
            lst[k] = e.base + e.off[f];
            s_tsum[k] = e.off[f + 1] - e.off[f];
        }
        load_tile_records<VEL>(P, ti, B, srec4, sreck, tally, tid);
        __syncthreads();
        if (tid == 0) {
            uint32_t run = 0;
            for (int k = 0; k <= ti.nsrc; ++k) {
                pre[k] = run;
                run += s_tsum[k];
            }
            pre[ti.nsrc + 1] = run;
            s_total = run;
        }
        __syncthreads();
    }
    n_in = uniform_u32(s_total);   // (uniform, so the walk loop's exits are too)
    if (n_in == 0) {
        if (tid == 0) {
            TileExits e;
            e.base = 0;
            for (int f = 0; f < 8; ++f) e.off[f] = 0;
            P.out_exits[T] = e;
        }
        return;
    }
    if (GEN0) load_tile_records<VEL>(P, ti, B, srec4, sreck, tally, tid);
    if (tid == 0) {
        s_next = 0;
        s_exit = 0;
        s_base = (uint32_t)atomicAdd(P.bump, (unsigned long long)n_in);
    }
    if (tid < 8) s_fcnt[tid] = 0;
    if (tid < 5) s_tot[tid] = 0;
    __syncthreads();

    // ---- walk -------------------------------------------------------------
    TileCtx C;
    C.delta = B.delta;
    C.xeff = B.x_eff;
    C.max_cross = P.max_cross;
    C.ln = line_of(B);
    C.ox = ti.ox;
    C.oy = ti.oy;
    C.oz = ti.oz;
    C.sx = ti.sx;
    C.sy = ti.sy;
    C.sz = ti.sz;
    C.span = ti.span;
    const char *recs = VEL ? reinterpret_cast<const char *>(srec4) : reinterpret_cast<const char *>(sreck);
    TileAcc acc{0};
    // a tile that spans the box along some axis wraps round inside itself
    if (ti.span)
        walk_tile<VEL, GEN0, VOIGT, true>(P, ti, B, C, n_in, pre, lst, recs, tally, &s_next, &s_exit, s_base, s_fcnt,
                                          s_tot, acc);
    else
        walk_tile<VEL, GEN0, VOIGT, false>(P, ti, B, C, n_in, pre, lst, recs, tally, &s_next, &s_exit, s_base, s_fcnt,
                                           s_tot, acc);

    // ---- finish: tally, totals, face lists of the exits ----------------------
    if (lane == 0) s_red[tid >> 6] = acc.cross;
    __threadfence_block();
    __syncthreads();
    {
        // this workgroup alone owns these cells in this generation: plain
        // read-modify-write, every read issued before the first is used
        constexpr int PER = TC / BLK;
        unsigned long long v[PER], old[PER];
        uint32_t gc[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int q = tid + k * BLK;
            const int lx = q & 15, ly = (q >> 4) & 15, lz = q >> 8;
            v[k] = (lx < ti.sx && ly < ti.sy && lz < ti.sz) ? tally[tile_slot(lx, ly, lz)] : 0ull;
            gc[k] = B.cell_off + (uint32_t)(ti.ox + lx) +
                    (uint32_t)B.nx * ((uint32_t)(ti.oy + ly) + (uint32_t)B.ny * (uint32_t)(ti.oz + lz));
            old[k] = 0ull;
        }
#pragma unroll
        for (int k = 0; k < PER; ++k)
            if (v[k]) old[k] = P.A[gc[k]];
#pragma unroll
        for (int k = 0; k < PER; ++k)
            if (v[k]) P.A[gc[k]] = old[k] + v[k];
    }
    if (tid < (VOIGT ? 5 : 4)) {
        // (after the barrier: every wave's walk has ended, so s_tot is final)
        unsigned long long t = s_tot[tid];
        if (tid == kTotCrossings)
            for (int w = 0; w < kWaves; ++w) t += s_red[w];
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
    // the face lists: four exits per thread at a time, their faces read first
    constexpr int kIdxBatch = 4;
    for (uint32_t k0 = tid; k0 < n_exit; k0 += kIdxBatch * BLK) {
        uint32_t f[kIdxBatch];
#pragma unroll
        for (int j = 0; j < kIdxBatch; ++j) {
            const uint32_t k = k0 + (uint32_t)(j * BLK);
            f[j] = k < n_exit ? (uint32_t)P.out_face[s_base + k] : 0u;
        }
#pragma unroll
        for (int j = 0; j < kIdxBatch; ++j) {
            const uint32_t k = k0 + (uint32_t)(j * BLK);
            if (k < n_exit) {
                const uint32_t pos = atomicAdd(&s_fcur[f[j]], 1u);
                P.out_idx[s_base + pos] = s_base + k;
            }
        }
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
        const uint32_t cross0 = L.ncross;          // crossings walked by the tile generations
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
        cross = L.ncross - cross0;                 // the generations counted theirs
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

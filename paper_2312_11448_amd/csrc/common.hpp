// Internal declarations of the MI355X Lyman-alpha transport library.
// Device-side data layout, the Philox generator and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "mc_lya.h"

namespace mclya {

// ---------------------------------------------------------------------------
// Device-side box descriptor used by every kernel (64 bytes, one cache line).
// ---------------------------------------------------------------------------
struct alignas(64) WalkBox {
    int32_t nx, ny, nz;
    float damp;           // Voigt profile: 2a/pi, the weight of Dawson's integral in the
                          // cumulative profile (0: Doppler profile)
    uint32_t cell_off;    // first global cell of the box
    float xblue;          // packets emitted above it are not walked (+inf: all are)
    uint64_t pkt_off;     // first global packet id of the box
    uint64_t npkt;        // packets emitted in the box
    uint64_t seed;        // Philox key
    uint32_t w0;          // weight of one packet
    float kfar;           // Voigt profile: mean kappa, for the far damping wing (0: none)
    float delta;          // red drift per cell width (Doppler units)
    float x_eff;          // escape once x <= -x_eff
    __host__ __device__ uint32_t cells() const { return (uint32_t)nx * (uint32_t)ny * (uint32_t)nz; }
};
static_assert(sizeof(WalkBox) == 64, "WalkBox layout");

// Inputs of the pack kernel for one box (device copy of the descriptor).
struct PackBox {
    const float *od;
    const void *vel;
    const float *xe;
    const float *src;
    double kappa_unit;    // kappa_c = kappa_unit * (1 - x_e) * Delta
    uint32_t cell_off, ncells;
    float xe_uniform;
    int32_t vel_dtype;
    int32_t nblk;         // blocks covering the box
    int32_t pad;
};

// Per-box reduction results (device).
struct BoxRed {
    double usum[3];       // sum of the velocity components
    double kappa_sum;     // sum of kappa_c
    double od_sum, od2_sum;   // sums of Delta and Delta^2
    unsigned long long wmax_bits;   // max emission weight (bit pattern of a double >= 0)
    unsigned long long udev_bits;   // max |U_c - <U>| (bit pattern of a double >= 0)
    uint32_t flags;       // validation failures (bit mask)
    uint32_t pad;
    uint64_t qtot;        // sum of the quantised weights
};

// Per-box running totals of the walk (device, int64).
struct BoxTot {
    unsigned long long escaped;
    unsigned long long crossings;
    unsigned long long capped_packets;
    unsigned long long capped_weight;
    unsigned long long wing;          // part of the escaped weight the far damping wing absorbs
    unsigned long long pad[3];
};

enum : uint32_t {
    FLAG_OD_BAD = 1u,     // non-finite or negative overdensity
    FLAG_XE_BAD = 2u,     // x_e outside [0, 1.2] or non-finite
    FLAG_VEL_BAD = 4u,    // non-finite velocity
    FLAG_SRC_BAD = 8u,    // negative or non-finite source
    FLAG_ZERO_SRC = 16u   // all emission weights zero
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    // each round's two 32 x 32 -> 64-bit products as whole 64-bit products:
    // one v_mad_u64_u32 apiece instead of separate high and low multiplies
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t m0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(m1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(m0 >> 32) ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = (uint32_t)m1;
        c[2] = n2;
        c[3] = (uint32_t)m0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// (w >> 9) + 1/2, scaled by 2^-23: exact in binary32, strictly inside (0,1).
__device__ __forceinline__ float u01(uint32_t w)
{
    return (float)(w >> 9) * 0x1p-23f + 0x1p-24f;
}

// ---------------------------------------------------------------------------
// Launchers (each defined next to its kernels).
// ---------------------------------------------------------------------------
constexpr int kSetupBlock = 256;
// Per-block partial results of the setup and tally kernels, kPartStride
// doubles per (box, block): [0..3] sums (pack, then feed), [4] the block's
// largest emission weight, [5] its largest |U - <U>|, [6] its absorbed-weight
// sum (uint64 bits), [7] sum of Delta and [8] of Delta^2 (pack). Reduced per
// box by one-block kernels; no same-address atomics, which serialise at the
// cache.
constexpr int kPartStride = 10;

hipError_t launch_pack(const PackBox *pb_dev, int n_boxes, int max_blk, bool vel_rec, void *rec,
                       double *wgt, double *partials, BoxRed *red, hipStream_t s);
hipError_t launch_box_reduce(const PackBox *pb_dev, int n_boxes, int max_blk, const double *partials,
                             BoxRed *red, hipStream_t s);
hipError_t launch_margin(const PackBox *pb_dev, int n_boxes, int max_blk, const float4 *rec, BoxRed *red,
                         double *partials, hipStream_t s);

hipError_t launch_quantize(const PackBox *pb_dev, int n_boxes, int max_blk, const double *wgt,
                           const BoxRed *red, uint64_t *q, uint64_t *bsum, hipStream_t s);
hipError_t launch_scan_blocks(const PackBox *pb_dev, int n_boxes, int max_blk, uint64_t *bsum,
                              BoxRed *red, hipStream_t s);
hipError_t launch_allocate(const PackBox *pb_dev, const WalkBox *wb_dev, int n_boxes, int max_blk,
                           const uint64_t *q, const uint64_t *bsum, const BoxRed *red,
                           uint32_t *npk, uint64_t *pfirst, hipStream_t s);
hipError_t launch_cell_of_packet(const PackBox *pb_dev, int n_boxes, int max_blk, const uint32_t *npk,
                                 const uint64_t *pfirst, uint32_t *cell_of_packet, hipStream_t s);

struct WalkParams {
    const WalkBox *boxes;
    int32_t n_boxes;
    int32_t vel;             // record layout: 0 = kappa only, 1 = float4 (kappa, U)
    const void *rec;
    int32_t voigt;           // some box has the Voigt profile (its own constants are in the box)
    int32_t pad0;
    const uint32_t *cell_of_packet;
    unsigned long long *A;   // per-cell absorbed weight
    BoxTot *tot;
    unsigned long long *queue;   // work counters, one per part of the range (persistent kernel)
    uint64_t first, count;   // global packet range
    int64_t max_cross;
    int32_t chunk, refill;
    int32_t nqueues;         // parts of the packet range (1..kMaxQueues)
    // optional: the range [0, count) is a concatenation of n_seg global packet
    // segments; segment k starts at index seg_start[k] (ascending, seg_start[0]
    // = 0) and global id seg_id[k]. n_seg = 0: packet i is global id first + i.
    int32_t n_seg;
    const uint64_t *seg_start;
    const uint64_t *seg_id;
};
constexpr int kMaxQueues = 64;

// ---- resonant scattering ----------------------------------------------------
// Per-box constants of the scattering Monte Carlo.
struct ScatBox {
    float inv_pab;           // 1/p_ab: the line opacity is kappa / p_ab per unit of swept profile
    float x_inert;           // lost to the line below -x_inert (and far above +x_inert)
    float a;                 // Voigt a (0: Doppler profile, resonant atoms)
    float damp;              // 2a/pi
    uint64_t destroy;        // destroyed iff a 64-bit event word is below this (floor(p 2^64))
    uint64_t pad;
};

struct ScatterParams {
    const WalkBox *boxes;
    const ScatBox *sbox;
    int32_t n_boxes;
    int32_t vel;
    const void *rec;
    const uint32_t *cell_of_packet;
    unsigned long long *A;
    BoxTot *tot;             // pad[0]: scatterings
    unsigned long long *queue;
    uint64_t first, count;
    uint64_t max_events;
    int32_t chunk, refill, nqueues;
    int32_t fixed_x0;        // test hook: inject every photon at x0
    float x0;
    float x_return;          // test hook: > 0 stops a photon scattered back inside |x| < x_return
    mc_lya_scatter_record *records;   // optional, one per photon of [first, first + count)
};
hipError_t launch_scatter(const ScatterParams &p, int block, int grid, hipStream_t s);

// ---- recombination history ---------------------------------------------------
hipError_t launch_xe_load(const PackBox *pb_dev, int n_boxes, int max_blk, double *y, hipStream_t s);
hipError_t launch_xe_rate(const PackBox *pb_dev, int n_boxes, int max_blk, const double *coef, const double *ndot,
                          double *k, hipStream_t s);
hipError_t launch_xe_combine(const PackBox *pb_dev, int n_boxes, int max_blk, const double *y0,
                             const double *const *k, const double *w, int nk, double *y_out, bool field,
                             hipStream_t s);

// ---- tile-decomposed walk -------------------------------------------------
// Tile extent in cells along x, y, z (the last tiles along an axis may be
// thinner) and the workgroup that walks one tile.
#ifndef MCLYA_TILE_Z
#define MCLYA_TILE_Z 16
#endif
#ifndef MCLYA_TILE_BLOCK
#define MCLYA_TILE_BLOCK 1024
#endif
constexpr int kTileX = 16, kTileY = 16, kTileZ = MCLYA_TILE_Z;
constexpr int kTileCells = kTileX * kTileY * kTileZ;
constexpr int kTileBlock = MCLYA_TILE_BLOCK;

struct TileInfo {
    int32_t box;
    int32_t ox, oy, oz;      // origin (cell coordinates in the box)
    int32_t sx, sy, sz;      // extent (cells)
    int32_t nsrc;            // exit lists this tile pulls from (0..6)
    int32_t src_tile[6];     // tile whose exits through face src_face[k] enter this tile
    uint32_t src_faces;      // 4 bits per source: the face (0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z)
    uint32_t span;           // bit a: the tile spans the box along axis a (a packet wraps
                             // round inside the tile instead of leaving it)
};
static_assert(sizeof(TileInfo) == 64, "TileInfo layout");

// A packet standing on the face between two tiles (112 bytes).
struct alignas(16) PState {
    double tmx, tmy, tmz, tdx, tdy, tdz, t;
    uint32_t w;
    uint32_t pad;
    float x, kx, ky, kz;     // pre-jump frequency and direction
    float ku;                // k . U of the cell it leaves (Doppler units)
    uint32_t pad2[2];
    uint32_t cell;           // cell it enters (global)
    uint32_t ncross;
    int32_t ix, iy, iz;      // coordinates of that cell
};
static_assert(sizeof(PState) == 112, "PState layout");

// Exit lists of one tile in one generation: states in [base, base + off[7]),
// and the states that left through face f are idx[base + off[f] .. base + off[f+1]).
// Faces 0..5 are -x, +x, -y, +y, -z, +z; list 6 holds packets the tile
// deferred to its own next generation (kDeferred).
constexpr int kDeferred = 6;
struct TileExits {
    uint32_t base;
    uint32_t off[8];
};

constexpr int kMaxGenerations = 4096;  // per transport batch (packets cross at most one tile per generation)
// Counters of a batch: per generation (bump allocator, exits), then the tail
// hand-off: the generation that found fewer than tail_min packets in flight
// (0 = none) and the number of packets handed to the tail walk.
constexpr int kGenCounters = 2 * kMaxGenerations + 2;
constexpr int kTailGenSlot = 2 * kMaxGenerations, kTailCountSlot = 2 * kMaxGenerations + 1;

struct TileParams {
    const WalkBox *boxes;
    const TileInfo *tiles;
    const void *rec;
    const uint32_t *npk;     // packets per cell
    const uint64_t *pfirst;  // global id of each cell's first packet
    unsigned long long *A;
    BoxTot *tot;
    const PState *in_state;
    const uint32_t *in_idx;
    const TileExits *in_exits;
    PState *out_state;
    uint8_t *out_face;
    uint32_t *out_idx;
    TileExits *out_exits;
    unsigned long long *bump;    // allocator of this generation's exit buffer
    unsigned long long *exits;   // packets written out this generation
    const unsigned long long *prev_exits;   // packets written out by the previous generation
    uint64_t first, count;   // packet range
    uint32_t max_cross;
    int32_t ntiles;
    int32_t chunk;
    int32_t refill;          // refill a wave once this many lanes are idle
    int32_t defer_lanes;     // once the tile's input is used up, a wave with at most this many live lanes
    uint32_t defer_min;      // ... defers them to the next generation, if the tile took >= defer_min packets
    int32_t gen;             // index of this generation in the batch
    uint64_t tail_min;       // fewer packets in flight than this: stop and leave them to the tail walk
    unsigned long long *tail_gen;   // where the first generation that stops records its index
};

// The tail walk: the packets the last full generation handed on, walked to
// the end one per thread with device-scope deposits.
struct TailParams {
    const WalkBox *boxes;
    const TileInfo *tiles;
    const void *rec;
    unsigned long long *A;
    BoxTot *tot;
    const PState *state[2];
    const uint8_t *face[2];
    const uint32_t *idx[2];
    const TileExits *exits[2];
    unsigned long long *counters;   // the batch counters (kTailGenSlot, kTailCountSlot)
    uint32_t *prefix;        // [ntiles] first tail packet of each tile
    int32_t ntiles;
    uint32_t max_cross;
};

hipError_t launch_tile_generation(const TileParams &p, bool gen0, bool vel, bool voigt, hipStream_t s);
// The tail walk of a batch (no-op when no generation stopped); `capacity`
// bounds the packets it can take (tail_min).
hipError_t launch_tail_walk(const TailParams &p, uint64_t capacity, bool vel, bool voigt, hipStream_t s);
hipError_t launch_zero_counters(unsigned long long *c, int n, hipStream_t s);

hipError_t launch_walk_simple(const WalkParams &p, int block, hipStream_t s);
hipError_t launch_walk_persistent(const WalkParams &p, int block, int grid, hipStream_t s);
int persistent_blocks_per_cu(bool vel, bool voigt, int block);   // resident workgroups per CU
hipError_t launch_trace(const WalkParams &p, mc_lya_packet_trace *out, hipStream_t s);
hipError_t launch_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out, uint64_t n,
                         hipStream_t s);

hipError_t launch_tally(const WalkBox *wb_dev, int n_boxes, int max_blk, const unsigned long long *A,
                        const uint32_t *npk, int64_t *absorbed_out, int64_t *emitted_out,
                        double *partials, unsigned long long *box_abs, hipStream_t s);

struct FeedBox {
    double S_scale;          // physical source = S_scale * weight
    double n_h;              // mean hydrogen density n_H0 (1+z)^3
    double a_norm;           // sum(S) / (w0 N)
    double reion;            // beta / (beta + Lambda)
    double thermal;          // C_MC beta exp(-E_alpha/kT)
    double fm_norm;          // (sum(A) + wing) / sum(n_1s)
    double wing_n1s;         // wing / sum(n_1s): the far damping wing's absorption per unit n_1s
    double w_inv;            // 1 / sum(weight): a cell's share of the box's emission is weight * w_inv
};
hipError_t launch_feed_sums(const PackBox *pb_dev, int n_boxes, int max_blk, const double *wgt,
                            double *partials, hipStream_t s);
hipError_t launch_feed_reduce(int n_boxes, int max_blk, const PackBox *pb_dev, const double *partials,
                              double *sums, hipStream_t s);
// The surrogate's regression data per cell: y = ln M_c and the cell's share
// of its box's emission (both 0 where M_c = 0).
hipError_t launch_targets(const PackBox *pb_dev, const FeedBox *fb_dev, int n_boxes, int max_blk,
                          const double *wgt, const unsigned long long *A, float *y, float *w, hipStream_t s);
hipError_t launch_feed(const PackBox *pb_dev, const FeedBox *fb_dev, int n_boxes, int max_blk,
                       const double *wgt, const unsigned long long *A, double *ndot,
                       float *mix, hipStream_t s);

// ---- mixing-correction surrogate ----------------------------------------------
// Per-box inputs of the feature kernel.
struct FeatBox {
    int32_t nx, ny, nz;
    uint32_t cell_off, ncells;
    int32_t vel_dtype;
    int32_t quad;            // 1: four cells along x per thread (nx % 4 == 0, fields 16-byte aligned)
    const float *od;
    const void *vel;
    const float *xe;
    float xe_uniform;
    float ln_t;              // ln(T / 3000 K)
    float z_feat;            // z / 1000 - 1.1
    float ln_clump;          // ln(<Delta^2> / <Delta>^2) from the pack's box sums
};

constexpr int kMlpParams = 4801;         // 8-64-64-1 network
constexpr int kMlpPartStride = 4808;     // floats per block of gradient partial sums (params, sum w r^2, sum w)
constexpr int kMlpGradBlocks = 1024;     // most blocks of the gradient kernel (partial-sum slots)

struct MlpAdam {
    float lr, beta1, beta2, eps;
    float bc1, bc2;          // 1 - beta1^t, 1 - beta2^t
};

hipError_t launch_features(const FeatBox *fb_dev, int n_boxes, int max_blk, float *out, hipStream_t s);
hipError_t launch_mlp_forward(const float *params, const float *X, uint64_t n, float *y, uint8_t *outside,
                              const float *lo, const float *hi, unsigned long long *n_out, int grid,
                              hipStream_t s);
// workgroups of the inference kernel that one compute unit holds at once
int mlp_forward_blocks_per_cu();
// partial: [max_blocks + ceil(max_blocks / 32)][kMlpPartStride] floats of workspace
hipError_t launch_mlp_gradient(const float *params, const float *X, const float *t, const float *w, uint64_t n,
                               float *partial, int max_blocks, float *grad, hipStream_t s);
hipError_t launch_mlp_normalise(float *grad, hipStream_t s);
hipError_t launch_mlp_correction(const float *y, const uint8_t *outside, const float *fallback, uint64_t n,
                                 float *M, hipStream_t s);
hipError_t launch_mlp_adam(float *params, float *m, float *v, float *grad, const MlpAdam &a, hipStream_t s);

}  // namespace mclya

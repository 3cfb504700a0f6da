// Host runtime behind the C ABI of mc_lya.h: argument validation, the FP64
// physics scalars of each box, device buffers, the state machine and the
// kernel launch sequence. All device work runs on the context's stream.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"

using namespace mclya;

static_assert(sizeof(mc_lya_box_desc) == 152, "mc_lya_box_desc layout");
static_assert(sizeof(mc_lya_box_stats) == 112, "mc_lya_box_stats layout");
static_assert(sizeof(mc_lya_scatter_record) == 72, "mc_lya_scatter_record layout");
static_assert(sizeof(mc_lya_scatter_opts) == 40, "mc_lya_scatter_opts layout");
static_assert(sizeof(mc_lya_feed_stats) == 56, "mc_lya_feed_stats layout");
static_assert(sizeof(mc_lya_packet_trace) == 64, "mc_lya_packet_trace layout");
static_assert(sizeof(mc_lya_tune_result) == 88, "mc_lya_tune_result layout");
static_assert(sizeof(mc_lya_limits) == 24, "mc_lya_limits layout");

namespace {

// ---------------------------------------------------------------------------
// Physics scalars (binary64, host). Paper: Sec. II.C (cosmology), Sec. III.A.1
// (three-level atom), Sec. IV.A (p_ab and the absorption depth), App. A
// (thermal velocity and the Hubble drift).
// ---------------------------------------------------------------------------
namespace phys {
constexpr double kC = 2.99792458e10;          // cm/s
constexpr double kBoltz = 1.380649e-16;       // erg/K
constexpr double kPlanck = 6.62607015e-27;    // erg s
constexpr double kMe = 9.1093837015e-28;      // g
constexpr double kMH = 1.6735328e-24;         // g, hydrogen atom
constexpr double kGrav = 6.67430e-8;          // cgs
constexpr double kMpc = 3.0856775814913673e24; // cm
constexpr double kEV = 1.602176634e-12;       // erg
constexpr double kArad = 7.565723e-15;        // erg cm^-3 K^-4
constexpr double kEion = 13.598434 * kEV;     // H ionisation energy
constexpr double kLya = 1215.67e-8;           // cm
constexpr double kA2p = 6.2649e8;             // s^-1
constexpr double kL2g = 8.22458;              // s^-1
constexpr double kPi = 3.14159265358979323846;

struct Box {
    double H, vth, delta, nH, kappa_unit, alpha, beta, pab, boltz, damping;
};

inline Box scalars(const mc_lya_box_desc &d)
{
    Box o;
    const double H0 = d.h * 1.0e7 / kMpc;                         // 100 h km/s/Mpc
    const double rhoc = 3.0 * H0 * H0 / (8.0 * kPi * kGrav);
    const double om = (d.omega_b_h2 + d.omega_c_h2) / (d.h * d.h);
    const double og = kArad * std::pow(d.t_cmb0, 4) / (rhoc * kC * kC);
    const double orad = og * (1.0 + 0.875 * std::pow(4.0 / 11.0, 4.0 / 3.0) * d.n_eff);
    const double ol = 1.0 - om - orad;
    const double a1 = 1.0 + d.z;
    o.H = d.zeta * H0 * std::sqrt(om * a1 * a1 * a1 + orad * a1 * a1 * a1 * a1 + ol);
    const double T = d.temp_K;
    o.vth = std::sqrt(2.0 * kBoltz * T / kMH);
    const double dl = d.cell_comoving_cm / a1;                    // physical cell width
    o.delta = o.H * dl / o.vth;                                   // App. A step 4 per cell
    o.nH = (1.0 - d.y_p) * (d.omega_b_h2 / (d.h * d.h)) * rhoc / kMH * a1 * a1 * a1;
    const double t4 = T / 1.0e4;                                  // alpha_e = 1.14 A_B
    o.alpha = 1.14e-13 * 4.309 * std::pow(t4, -0.6166) / (1.0 + 0.6703 * std::pow(t4, 0.5300));
    const double saha = std::pow(2.0 * kPi * kMe * kBoltz * T / (kPlanck * kPlanck), 1.5);
    o.beta = o.alpha * saha * std::exp(-0.25 * kEion / (kBoltz * T));   // per 2s atom
    o.pab = (o.beta + kL2g) / (3.0 * kA2p + o.beta + kL2g);
    // kappa_c = p_ab 3 lambda^3 A n_1s / (8 pi zeta H), n_1s = nH (1 - x_e) Delta
    o.kappa_unit = o.pab * 3.0 * kLya * kLya * kLya * kA2p / (8.0 * kPi * o.H) * o.nH;
    o.boltz = std::exp(-0.75 * kEion / (kBoltz * T));
    // Voigt parameter of Eq. (MC): half the natural width A over the Doppler
    // width nu_alpha v_th / c, in angular units, a = A lambda / (4 pi v_th)
    o.damping = kA2p * kLya / (4.0 * kPi * o.vth);
    return o;
}
}  // namespace phys

template <typename T>
hipError_t dalloc(T **p, size_t n)
{
    *p = nullptr;
    if (n == 0) n = 1;
    return hipMalloc(reinterpret_cast<void **>(p), n * sizeof(T));
}

}  // namespace

constexpr int kEagerGens = 16;
constexpr uint64_t kDefaultMaxPackets = 1ull << 20;   // limits == NULL

struct mc_lya_ctx {
    hipStream_t stream = nullptr;
    int n_boxes = 0;
    std::vector<mc_lya_box_desc> desc;
    std::vector<phys::Box> ph;
    std::vector<PackBox> pack;
    std::vector<WalkBox> walk;
    std::vector<BoxRed> red;
    std::vector<uint64_t> walked;     // packets walked per box since the last emit
    std::vector<uint8_t> walked_tiled;  // per box: the last walk of its packets was the tiled walk
    uint64_t total_cells = 0;
    uint64_t total_packets = 0;
    int max_blk = 1;
    bool vel = false;
    bool voigt = false;                      // some box has the Voigt profile
    int num_cu = 256;

    PackBox *d_pack = nullptr;
    WalkBox *d_walk = nullptr;
    BoxRed *d_red = nullptr;
    BoxTot *d_tot = nullptr;
    void *d_rec = nullptr;
    double *d_wgt = nullptr;
    double *d_part = nullptr;
    uint64_t *d_q = nullptr;
    uint64_t *d_bsum = nullptr;
    uint32_t *d_npk = nullptr;
    unsigned long long *d_A = nullptr;
    unsigned long long *d_queue = nullptr;
    ScatBox *d_sbox = nullptr;               // scattering constants per box
    double *d_ev = nullptr;                  // evolution: y0, k0..k3, ndot [6][total cells] (limits.evolve)
    double *d_ev_coef = nullptr;             // evolution: -1 / (n_H (1+z) H) per box
    uint64_t max_packets = 0;                // packet capacity reserved at init (limits.max_packets)
    unsigned long long *d_boxabs = nullptr;
    double *d_fsum = nullptr;
    FeedBox *d_feed = nullptr;
    uint32_t *d_cop = nullptr;               // [max_packets] cell of each packet
    bool cop_valid = false;      // d_cop holds the cells of the current emission
    uint64_t *d_pfirst = nullptr;

    // tile-decomposed walk
    std::vector<TileInfo> tiles;
    TileInfo *d_tiles = nullptr;
    TileExits *d_texits[2] = {nullptr, nullptr};
    PState *d_state[2] = {nullptr, nullptr};
    uint8_t *d_face[2] = {nullptr, nullptr};
    uint32_t *d_idx[2] = {nullptr, nullptr};
    unsigned long long *d_gen = nullptr;     // per generation: bump allocator, exits
    uint64_t state_cap = 0;
    int64_t generations = 0;                 // generations launched by the last tiled transport
    std::vector<uint8_t> tiled;              // per box: walked by tiles (1) or by the persistent walk (0)
    std::vector<double> cpp;                 // per box: estimated crossings per packet (set by refresh)
    std::vector<uint64_t> seg_host;          // packet segments of the persistent part: starts, then ids
    std::vector<FeatBox> featbox;            // surrogate features: per-box inputs
    FeatBox *d_featbox = nullptr;
    bool featbox_stale = true;               // rebuilt and uploaded after each refresh
    int feat_blocks = 1;                     // grid width of the features launch
    uint64_t *d_seg = nullptr;               // [2 (n_boxes + 1)]
    int tile_share = 100;
    int defer = 16;                          // MC_LYA_OPT_DEFER
    // captured transport (MC_LYA_OPT_GRAPH)
    bool graph = false;
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t cap_stream = nullptr;        // private stream the graph is captured on
    // the persistent part of a kernel-2 walk runs beside the tile generations
    // on its own stream (fork and join events), with at most this many waves
    // per compute unit (0: after them, on the context's stream)
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    int beside = 4;                          // MC_LYA_OPT_BESIDE
    std::vector<uint64_t> graph_key;
    int graph_gens = 64;                     // tile generations inside the graph
    int eager_gens = kEagerGens;             // tile generations in the first eager round
    int tail = 20000;                        // MC_LYA_OPT_TAIL (millionths of a batch)
    uint32_t *d_tail_prefix = nullptr;       // [tiles] first tail packet of each tile
    uint64_t epoch = 0;                      // bumped whenever a buffer a graph reads is reallocated

    int state = 0;                    // 0 packed, 1 emitted, 2 transported
    // options
    int kernel = 2, block = 256, waves_per_cu = 32, chunk = 256, refill = 16, nqueues = 8;
    int tile_chunk = 512, tile_refill = 40;  // the tiled walk's own chunk and refill
    int64_t max_cross = 1000000;
    int timing = 0;                          // 0 off, 1 per launch, 2 per transport
    int64_t coarse_launches = 0;
    int64_t graph_launches = 0;              // walk launches in the captured graph
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    size_t events_used = 0;
    std::string err;
};

namespace {

thread_local std::string g_init_err;   // last failure of mc_lya_init on this thread

mc_lya_status fail(mc_lya_ctx *c, mc_lya_status s, const std::string &msg)
{
    if (c) c->err = msg;
    else g_init_err = msg;
    return s;
}

mc_lya_status hip_fail(mc_lya_ctx *c, hipError_t e, const char *what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (c) c->err = m;
    return e == hipErrorOutOfMemory ? MC_LYA_ENOMEM : MC_LYA_EDEVICE;
}

#define HIP_TRY(ctx, expr)                                           \
    do {                                                             \
        hipError_t e_ = (expr);                                      \
        if (e_ != hipSuccess) return hip_fail((ctx), e_, #expr);     \
    } while (0)

void free_all(mc_lya_ctx *c)
{
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    c->graph_exec = nullptr;
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    c->cap_stream = nullptr;
    if (c->side) (void)hipStreamDestroy(c->side);
    if (c->fork) (void)hipEventDestroy(c->fork);
    if (c->join) (void)hipEventDestroy(c->join);
    c->side = nullptr;
    c->fork = c->join = nullptr;
    void *ptrs[] = {c->d_pack, c->d_walk, c->d_red, c->d_tot, c->d_rec, c->d_wgt, c->d_part, c->d_q,
                    c->d_bsum, c->d_npk, c->d_A, c->d_queue, c->d_boxabs, c->d_fsum, c->d_feed,
                    c->d_cop, c->d_pfirst, c->d_seg, c->d_featbox, c->d_tail_prefix, c->d_tiles, c->d_texits[0], c->d_texits[1], c->d_state[0], c->d_sbox, c->d_ev, c->d_ev_coef,
                    c->d_state[1], c->d_face[0], c->d_face[1], c->d_idx[0], c->d_idx[1], c->d_gen};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (auto &ev : c->events) {
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
    }
    c->events.clear();
}

std::string check_desc(const mc_lya_box_desc &d, int b)
{
    char buf[256];
    auto bad = [&](const char *what) {
        std::snprintf(buf, sizeof buf, "box %d: %s", b, what);
        return std::string(buf);
    };
    if (d.nx < 1 || d.ny < 1 || d.nz < 1) return bad("grid edges must be >= 1");
    if (!(d.cell_comoving_cm > 0.0) || !std::isfinite(d.cell_comoving_cm)) return bad("cell_comoving_cm must be > 0");
    if (!(d.z > 0.0) || !std::isfinite(d.z)) return bad("z must be > 0");
    if (!(d.zeta > 0.0) || !std::isfinite(d.zeta)) return bad("zeta must be > 0");
    if (!(d.x_esc > 0.0) || !std::isfinite(d.x_esc)) return bad("x_esc must be > 0");
    if (!(d.temp_K > 0.0) || !std::isfinite(d.temp_K)) return bad("temp_K must be > 0");
    if (!(d.h > 0.0) || !(d.omega_b_h2 > 0.0) || !(d.omega_c_h2 >= 0.0) || !(d.y_p >= 0.0 && d.y_p < 1.0) ||
        !(d.t_cmb0 > 0.0) || !(d.n_eff >= 0.0))
        return bad("cosmological parameters out of range");
    if (d.w0 == 0 || d.w0 >= (1ull << 32)) return bad("w0 must be in [1, 2^32)");
    if (!d.overdensity) return bad("overdensity is NULL");
    if (d.vel_dtype != MC_LYA_VEL_NONE && d.vel_dtype != MC_LYA_VEL_F32 && d.vel_dtype != MC_LYA_VEL_F16)
        return bad("unknown vel_dtype");
    if ((d.vel_dtype == MC_LYA_VEL_NONE) != (d.velocity == nullptr))
        return bad("velocity must be given exactly when vel_dtype is not NONE");
    if (!d.x_e && !(d.x_e_uniform >= 0.0f && d.x_e_uniform <= 1.2f)) return bad("x_e_uniform outside [0, 1.2]");
    if (d.profile != MC_LYA_PROFILE_DOPPLER && d.profile != MC_LYA_PROFILE_VOIGT)
        return bad("profile must be MC_LYA_PROFILE_DOPPLER or MC_LYA_PROFILE_VOIGT");
    return std::string();
}

// Expected crossings per packet in a homogeneous box with opacity kappa per
// unit Phi, drift delta per cell, escape at -x_eff and packet weight w0. A
// packet emitted at x0 walks until its weight rounds to zero, once
// kappa (Phi(x0) - Phi(x)) exceeds ln(2 w0), or until x = -x_eff; that is
// (x0 - x_end) / delta cells. Only used to balance work between the walks.
double crossings_per_packet(double kappa, double delta, double x_eff, double w0)
{
    if (!(delta > 0.0)) return 1.0;
    auto Phi = [](double x) { return 0.5 * std::erfc(-x); };
    const double need = kappa > 0.0 ? std::log(2.0 * w0) / kappa : 1e300;
    const double floor_phi = Phi(-x_eff);
    const int n = 64;
    const double lo = -x_eff, hi = 6.0;
    double sum = 0.0, norm = 0.0;
    for (int i = 0; i < n; ++i) {
        const double x0 = lo + (hi - lo) * (i + 0.5) / n;
        const double target = Phi(x0) - need;
        double xe = -x_eff;
        if (target > floor_phi) {
            double a = -x_eff, b = x0;
            for (int it = 0; it < 40; ++it) {
                const double m = 0.5 * (a + b);
                if (Phi(m) < target) a = m; else b = m;
            }
            xe = 0.5 * (a + b);
        }
        const double wgt = std::exp(-x0 * x0);
        sum += wgt * (x0 - xe) / delta;
        norm += wgt;
    }
    return 1.0 + sum / norm;
}

mc_lya_status do_refresh(mc_lya_ctx *c)
{
    const int nb = c->n_boxes;
    HIP_TRY(c, hipMemsetAsync(c->d_red, 0, sizeof(BoxRed) * nb, c->stream));
    HIP_TRY(c, launch_pack(c->d_pack, nb, c->max_blk, c->vel, c->d_rec, c->d_wgt, c->d_part, c->d_red,
                           c->stream));
    HIP_TRY(c, launch_box_reduce(c->d_pack, nb, c->max_blk, c->d_part, c->d_red, c->stream));
    if (c->vel)
        HIP_TRY(c, launch_margin(c->d_pack, nb, c->max_blk, static_cast<const float4 *>(c->d_rec), c->d_red,
                                 c->d_part, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->red.data(), c->d_red, sizeof(BoxRed) * nb, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->featbox_stale = true;                 // the box clumping comes from these sums
    for (int b = 0; b < nb; ++b) {
        const uint32_t f = c->red[b].flags;
        if (f) {
            std::string what;
            if (f & FLAG_OD_BAD) what += " overdensity negative or not finite;";
            if (f & FLAG_XE_BAD) what += " x_e outside [0, 1.2] or not finite;";
            if (f & FLAG_VEL_BAD) what += " velocity not finite;";
            if (f & FLAG_SRC_BAD) what += " source negative or not finite;";
            c->state = -1;
            return fail(c, MC_LYA_EINVAL, "box " + std::to_string(b) + ":" + what);
        }
        double udev = 0.0;
        std::memcpy(&udev, &c->red[b].udev_bits, sizeof udev);
        WalkBox &w = c->walk[b];
        w.x_eff = (float)(c->desc[b].x_esc + 2.0 * udev);
        w.delta = (float)c->ph[b].delta;
        if (c->desc[b].profile == MC_LYA_PROFILE_VOIGT) {
            // Voigt: the weight 2a/pi of Dawson's integral, the mean kappa seen
            // by the far damping wing, and the top of the walked window (a
            // walked packet never rises more than the velocity margin above
            // its emission frequency)
            w.damp = (float)(2.0 * c->ph[b].damping / phys::kPi);
            w.kfar = (float)(c->red[b].kappa_sum / (double)w.cells());
            w.xblue = (float)(c->desc[b].x_esc + 4.0 * udev);
        } else {
            w.damp = 0.0f;
            w.kfar = 0.0f;
            w.xblue = std::numeric_limits<float>::infinity();
        }
        c->cpp[b] = crossings_per_packet(c->red[b].kappa_sum / (double)w.cells(), w.delta, w.x_eff, (double)w.w0);
    }
    c->state = 0;
    return MC_LYA_OK;
}

// Tiles of kTileX x kTileY x kTileZ cells per box (the last ones along an axis may be
// thinner). For each tile, the exit lists it pulls: for each of its six faces
// whose neighbour is another tile, that neighbour's list through the
// opposite face (a tile that spans an axis wraps onto itself there).
void build_tiles(mc_lya_ctx *c)
{
    const int TE[3] = {kTileX, kTileY, kTileZ};
    c->tiles.clear();
    for (int b = 0; b < c->n_boxes; ++b) {
        if (!c->tiled[b]) continue;
        const mc_lya_box_desc &d = c->desc[b];
        const int nt[3] = {(d.nx + TE[0] - 1) / TE[0], (d.ny + TE[1] - 1) / TE[1], (d.nz + TE[2] - 1) / TE[2]};
        const int off = (int)c->tiles.size();
        const int n[3] = {d.nx, d.ny, d.nz};
        for (int tz = 0; tz < nt[2]; ++tz)
            for (int ty = 0; ty < nt[1]; ++ty)
                for (int tx = 0; tx < nt[0]; ++tx) {
                    TileInfo t;
                    std::memset(&t, 0, sizeof t);
                    t.box = b;
                    const int tc[3] = {tx, ty, tz};
                    int o[3], e[3];
                    for (int a = 0; a < 3; ++a) {
                        o[a] = tc[a] * TE[a];
                        e[a] = std::min(TE[a], n[a] - o[a]);
                    }
                    t.ox = o[0];
                    t.oy = o[1];
                    t.oz = o[2];
                    t.sx = e[0];
                    t.sy = e[1];
                    t.sz = e[2];
                    for (int a = 0; a < 3; ++a) {
                        if (nt[a] == 1) {
                            t.span |= 1u << a;
                            continue;
                        }
                        for (int dir = -1; dir <= 1; dir += 2) {
                            int q[3] = {tx, ty, tz};
                            q[a] = (q[a] + dir + nt[a]) % nt[a];
                            // the neighbour on side dir sends what leaves it through the opposite face
                            const int face = 2 * a + (dir < 0 ? 1 : 0);
                            t.src_tile[t.nsrc] = off + q[0] + nt[0] * (q[1] + nt[1] * q[2]);
                            t.src_faces |= (uint32_t)face << (4 * t.nsrc);
                            ++t.nsrc;
                        }
                    }
                    c->tiles.push_back(t);
                }
    }
}

int tiles_of_box(const mc_lya_box_desc &d)
{
    return ((d.nx + kTileX - 1) / kTileX) * ((d.ny + kTileY - 1) / kTileY) * ((d.nz + kTileZ - 1) / kTileZ);
}

constexpr int kMinTiles = 8;              // fewer tiles than this never pays
constexpr int kAllTiled = 1000000;        // tile_share at or above this: every box is tiled

// Which boxes the tiled walk takes: those whose estimated work per tile is at
// most tile_share % of one compute unit's fair share of the whole emission
// (a tile is walked by one workgroup, so a box with few tiles and many long
// walks would hold the whole launch); the rest go to the persistent walk.
// Rebuilds and uploads the tile table when the choice changes.
mc_lya_status classify_boxes(mc_lya_ctx *c)
{
    const int nb = c->n_boxes;
    std::vector<double> cost(nb, 0.0);
    double total = 0.0;
    for (int b = 0; b < nb; ++b) {
        cost[b] = (double)c->walk[b].npkt * c->cpp[b];
        total += cost[b];
    }
    const double fair = total / std::max(1, c->num_cu);
    std::vector<uint8_t> m(nb, 0);
    for (int b = 0; b < nb; ++b) {
        const int nt = tiles_of_box(c->desc[b]);
        if (c->tile_share >= kAllTiled) m[b] = 1;
        else if (c->tile_share > 0)
            m[b] = nt >= kMinTiles && cost[b] / nt <= 0.01 * c->tile_share * fair ? 1 : 0;
    }
    if (m == c->tiled) return MC_LYA_OK;
    HIP_TRY(c, hipStreamSynchronize(c->stream));      // the previous table may still be in flight
    c->tiled = m;
    build_tiles(c);
    if (!c->tiles.empty())
        HIP_TRY(c, hipMemcpyAsync(c->d_tiles, c->tiles.data(), sizeof(TileInfo) * c->tiles.size(),
                                  hipMemcpyHostToDevice, c->stream));
    return MC_LYA_OK;
}

// Packets per tiled batch: the packet-state buffers (two generations'
// states, faces and indices) are reserved at init for max_packets packets,
// or, if that much memory cannot be had, for as many as fit in halving steps
// down to 2^25; a larger emission then walks in batches. Every batch repeats
// the per-generation tile loads and flushes, so fewer batches are faster;
// the 2^28 packets of the 256^3 workload (63 GB of state) are one batch on a
// 288 GB device.
constexpr uint64_t kMinTiledBatch = 1ull << 25;
constexpr int kGenRound = 16;                  // generations queued between two checks
constexpr uint64_t kStateBytes = 2 * (sizeof(PState) + sizeof(uint8_t) + sizeof(uint32_t));

void free_tile_buffers(mc_lya_ctx *c)
{
    for (int i = 0; i < 2; ++i) {
        if (c->d_state[i]) (void)hipFree(c->d_state[i]);
        if (c->d_face[i]) (void)hipFree(c->d_face[i]);
        if (c->d_idx[i]) (void)hipFree(c->d_idx[i]);
        c->d_state[i] = nullptr;
        c->d_face[i] = nullptr;
        c->d_idx[i] = nullptr;
    }
    c->state_cap = 0;
}

// The packet-state buffers of the tiled walk (init only).
hipError_t alloc_tile_buffers(mc_lya_ctx *c, uint64_t packets)
{
    uint64_t cap = std::max<uint64_t>(1, packets);
    for (;;) {
        hipError_t e = hipSuccess;
        for (int i = 0; i < 2 && e == hipSuccess; ++i) {
            if ((e = dalloc(&c->d_state[i], cap)) == hipSuccess && (e = dalloc(&c->d_face[i], cap)) == hipSuccess)
                e = dalloc(&c->d_idx[i], cap);
        }
        if (e == hipSuccess) break;
        free_tile_buffers(c);
        (void)hipGetLastError();
        if (e != hipErrorOutOfMemory || cap <= kMinTiledBatch) return e;
        cap = std::max(kMinTiledBatch, cap / 2);               // smaller batches
    }
    c->state_cap = cap;
    return hipSuccess;
}

// Event pairs: one per walk launch (timing 1), or one per transport with the
// launches counted (timing 2).
mc_lya_status event_pair(mc_lya_ctx *c, hipEvent_t *e1)
{
    if (c->events_used == c->events.size()) {
        hipEvent_t a, b;
        HIP_TRY(c, hipEventCreate(&a));
        HIP_TRY(c, hipEventCreate(&b));
        c->events.emplace_back(a, b);
    }
    HIP_TRY(c, hipEventRecord(c->events[c->events_used].first, c->stream));
    *e1 = c->events[c->events_used].second;
    ++c->events_used;
    return MC_LYA_OK;
}

mc_lya_status timed_begin(mc_lya_ctx *c, hipEvent_t *e1)
{
    *e1 = nullptr;
    if (c->timing == 2) ++c->coarse_launches;
    if (c->timing != 1) return MC_LYA_OK;
    return event_pair(c, e1);
}

mc_lya_status timed_end(mc_lya_ctx *c, hipEvent_t e1)
{
    if (e1) HIP_TRY(c, hipEventRecord(e1, c->stream));
    return MC_LYA_OK;
}

// The tail walk takes over once fewer than this many of a batch's n packets
// are in flight (MC_LYA_OPT_TAIL, in millionths of the batch).
uint64_t tail_packets(const mc_lya_ctx *c, uint64_t n)
{
    return (uint64_t)((unsigned __int128)n * (uint64_t)c->tail / 1000000u);
}

TileParams tile_params(mc_lya_ctx *c, uint64_t first, uint64_t n)
{
    TileParams p;
    std::memset(&p, 0, sizeof p);
    p.boxes = c->d_walk;
    p.tiles = c->d_tiles;
    p.rec = c->d_rec;
    p.npk = c->d_npk;
    p.pfirst = c->d_pfirst;
    p.A = c->d_A;
    p.tot = c->d_tot;
    p.max_cross = (uint32_t)c->max_cross;
    p.ntiles = (int)c->tiles.size();
    p.chunk = c->tile_chunk;
    p.refill = c->tile_refill;
    p.defer_lanes = c->defer;
    p.defer_min = 2048;
    p.tail_min = tail_packets(c, n);
    p.tail_gen = c->d_gen + kTailGenSlot;
    p.first = first;
    p.count = n;
    return p;
}

// Enqueues tile generations [g0, g1) (buffers ping-pong by parity; the
// per-generation counters were zeroed at generation 0). timed: one event pair
// per launch (not while a graph is being captured).
mc_lya_status enqueue_generations(mc_lya_ctx *c, TileParams &p, int g0, int g1, bool timed)
{
    for (int gen = g0; gen < g1; ++gen) {
        const int cur = gen & 1, prev = cur ^ 1;
        p.in_state = c->d_state[prev];
        p.in_idx = c->d_idx[prev];
        p.in_exits = c->d_texits[prev];
        p.out_state = c->d_state[cur];
        p.out_face = c->d_face[cur];
        p.out_idx = c->d_idx[cur];
        p.out_exits = c->d_texits[cur];
        p.bump = c->d_gen + 2 * gen;
        p.exits = c->d_gen + 2 * gen + 1;
        p.prev_exits = gen > 0 ? c->d_gen + 2 * (gen - 1) + 1 : c->d_gen + 1;
        p.gen = gen;
        hipEvent_t e1 = nullptr;
        if (timed) {
            mc_lya_status st = timed_begin(c, &e1);
            if (st != MC_LYA_OK) return st;
        }
        HIP_TRY(c, launch_tile_generation(p, gen == 0, c->vel, c->voigt, c->stream));
        if (timed) {
            mc_lya_status st = timed_end(c, e1);
            if (st != MC_LYA_OK) return st;
        }
        ++c->generations;
    }
    return MC_LYA_OK;
}

// The tail walk of the current batch (a no-op unless a generation stopped).
mc_lya_status enqueue_tail(mc_lya_ctx *c, uint64_t n, bool timed)
{
    const uint64_t capacity = tail_packets(c, n);
    if (capacity == 0) return MC_LYA_OK;
    TailParams t;
    std::memset(&t, 0, sizeof t);
    t.boxes = c->d_walk;
    t.tiles = c->d_tiles;
    t.rec = c->d_rec;
    t.A = c->d_A;
    t.tot = c->d_tot;
    for (int i = 0; i < 2; ++i) {
        t.state[i] = c->d_state[i];
        t.face[i] = c->d_face[i];
        t.idx[i] = c->d_idx[i];
        t.exits[i] = c->d_texits[i];
    }
    t.counters = c->d_gen;
    t.prefix = c->d_tail_prefix;
    t.ntiles = (int)c->tiles.size();
    t.max_cross = (uint32_t)c->max_cross;
    hipEvent_t e1 = nullptr;
    if (timed) {
        mc_lya_status st = timed_begin(c, &e1);
        if (st != MC_LYA_OK) return st;
    }
    HIP_TRY(c, launch_tail_walk(t, capacity, c->vel, c->voigt, c->stream));
    if (timed) return timed_end(c, e1);
    return MC_LYA_OK;
}

// Packets still crossing tiles after generation gen - 1 (synchronises).
mc_lya_status exits_after(mc_lya_ctx *c, int gen, unsigned long long *exits)
{
    HIP_TRY(c, hipMemcpyAsync(exits, c->d_gen + 2 * (gen - 1) + 1, sizeof *exits, hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MC_LYA_OK;
}

// Continues a tiled batch from generation gen in rounds of kGenRound, reading
// the exit count after each round, until no packet is left crossing.
mc_lya_status drain_generations(mc_lya_ctx *c, TileParams &p, int gen, int *end = nullptr)
{
    for (;;) {
        unsigned long long exits = 0;
        mc_lya_status st = exits_after(c, gen, &exits);
        if (st != MC_LYA_OK) return st;
        if (exits == 0) {
            if (end) *end = gen;
            return MC_LYA_OK;
        }
        if (gen >= kMaxGenerations) return fail(c, MC_LYA_EDEVICE, "tiled walk did not drain");
        const int g1 = std::min(gen + kGenRound, kMaxGenerations);
        st = enqueue_generations(c, p, gen, g1, true);
        if (st != MC_LYA_OK) return st;
        gen = g1;
    }
}

// Generations are queued in rounds without waiting; a generation whose
// predecessor moved nothing returns at once. After each round the host reads
// the last generation's exit count: zero means every packet has finished.
// Emissions larger than the packet-state buffers walk in batches.
// The first round takes as many generations as the previous transport of the
// context needed (plus a few), so a repeated workload usually needs a single
// host read-back per batch.
mc_lya_status walk_tiled(mc_lya_ctx *c, uint64_t first, uint64_t count)
{
    int needed = 0;
    for (uint64_t done = 0; done < count;) {
        const uint64_t n = std::min(count - done, c->state_cap);
        TileParams p = tile_params(c, first + done, n);
        HIP_TRY(c, launch_zero_counters(c->d_gen, kGenCounters, c->stream));
        const int g1 = std::min(std::max(kGenRound, c->eager_gens), kMaxGenerations);
        int end = g1;
        // the tail walk goes in right after the first round (a no-op unless a
        // generation stopped in it), so it needs no host round trip
        mc_lya_status st = enqueue_generations(c, p, 0, g1, true);
        if (st == MC_LYA_OK) st = enqueue_tail(c, n, true);
        if (st == MC_LYA_OK) st = drain_generations(c, p, g1, &end);
        if (st == MC_LYA_OK && end > g1) st = enqueue_tail(c, n, true);
        if (st != MC_LYA_OK) return st;
        // the last generation that still handed packets on
        std::vector<unsigned long long> cnt(2 * (size_t)end);
        HIP_TRY(c, hipMemcpyAsync(cnt.data(), c->d_gen, sizeof(unsigned long long) * cnt.size(),
                                  hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        int last = 0;
        for (int g = 0; g < end; ++g)
            if (cnt[2 * g + 1]) last = g;
        needed = std::max(needed, last + 2);
        done += n;
    }
    c->eager_gens = needed + 4;
    return MC_LYA_OK;
}

// The per-packet cell list, built on first use after an emission (the
// persistent, per-packet and trace kernels take packets by id) in the buffer
// reserved at init.
mc_lya_status ensure_cell_of_packet(mc_lya_ctx *c)
{
    if (c->cop_valid) return MC_LYA_OK;
    const uint64_t ntot = c->total_packets;
    if (ntot) HIP_TRY(c, launch_cell_of_packet(c->d_pack, c->n_boxes, c->max_blk, c->d_npk, c->d_pfirst, c->d_cop,
                                               c->stream));
    c->cop_valid = true;
    return MC_LYA_OK;
}

mc_lya_status launch_global_walk(mc_lya_ctx *c, const WalkParams &p, bool timed, int waves_cap = 0);

// The persistent part of a kernel-2 walk on the side stream: fork_beside
// forks the side stream from the context's stream and enqueues `body` there
// (the context's stream is switched to the side stream meanwhile), and
// join_beside makes the context's stream wait for it, after the tile
// generations have been enqueued. Inside a stream capture the side stream
// joins the capture, and the graph holds the two as parallel branches.
template <typename F>
mc_lya_status fork_beside(mc_lya_ctx *c, F body)
{
    const hipStream_t main = c->stream;
    HIP_TRY(c, hipEventRecord(c->fork, main));
    HIP_TRY(c, hipStreamWaitEvent(c->side, c->fork, 0));
    c->stream = c->side;
    const mc_lya_status st = body();
    c->stream = main;
    // recorded even after a failed launch: the join then waits for whatever
    // reached the side stream
    HIP_TRY(c, hipEventRecord(c->join, c->side));
    return st;
}

mc_lya_status join_beside(mc_lya_ctx *c)
{
    HIP_TRY(c, hipStreamWaitEvent(c->stream, c->join, 0));
    return MC_LYA_OK;
}

// Everything a transport of [first, first + count) needs before its kernels
// are enqueued: the tiled / persistent split of the boxes, the packet-state
// buffers, the per-packet cell list and the packet segments of the
// persistent part (all in device memory, so a captured graph can replay the
// kernels alone).
struct WalkPlan {
    bool tiled = false;     // tiled generations over [first, first + count)
    bool global = false;    // persistent / per-packet walk over p
    WalkParams p{};
};

mc_lya_status plan_walk(mc_lya_ctx *c, uint64_t first, uint64_t count, WalkPlan *w)
{
    WalkParams &p = w->p;
    p.boxes = c->d_walk;
    p.n_boxes = c->n_boxes;
    p.vel = c->vel ? 1 : 0;
    p.voigt = c->voigt ? 1 : 0;
    p.rec = c->d_rec;
    p.A = c->d_A;
    p.tot = c->d_tot;
    p.queue = c->d_queue;
    p.first = first;
    p.count = count;
    p.max_cross = c->max_cross;
    p.chunk = c->chunk;
    p.refill = c->refill;
    p.nqueues = c->nqueues;
    p.n_seg = 0;
    w->global = true;
    if (c->kernel == 2) {
        // tiled boxes by tiles; the others, if any, by the persistent walk
        // over their packet segments inside [first, first + count)
        mc_lya_status st = classify_boxes(c);
        if (st != MC_LYA_OK) return st;
        w->tiled = !c->tiles.empty();
        std::vector<uint64_t> starts, ids;
        uint64_t n = 0;
        for (int b = 0; b < c->n_boxes; ++b) {
            if (c->tiled[b]) continue;
            const uint64_t lo = std::max(first, c->walk[b].pkt_off);
            const uint64_t hi = std::min(first + count, c->walk[b].pkt_off + c->walk[b].npkt);
            if (hi <= lo) continue;
            starts.push_back(n);
            ids.push_back(lo);
            n += hi - lo;
        }
        w->global = n > 0;
        if (w->global) {
            std::vector<uint64_t> segs = starts;
            segs.insert(segs.end(), ids.begin(), ids.end());
            if (segs != c->seg_host) {
                HIP_TRY(c, hipStreamSynchronize(c->stream));      // the previous segments may still be in flight
                c->seg_host = segs;
                HIP_TRY(c, hipMemcpyAsync(c->d_seg, c->seg_host.data(), sizeof(uint64_t) * segs.size(),
                                          hipMemcpyHostToDevice, c->stream));
            }
            const size_t k = starts.size();
            p.n_seg = (int32_t)k;
            p.seg_start = c->d_seg;
            p.seg_id = c->d_seg + k;
            p.count = n;
        }
    }
    if (w->global) {
        mc_lya_status st = ensure_cell_of_packet(c);
        if (st != MC_LYA_OK) return st;
        p.cell_of_packet = c->d_cop;
    }
    return MC_LYA_OK;
}

// tiled: the walk that took the range was kernel 2 (per box, the tile table's
// choice); false for the other walks and the scattering Monte Carlo
void account_walked(mc_lya_ctx *c, uint64_t first, uint64_t count, bool tiled)
{
    for (int b = 0; b < c->n_boxes; ++b) {
        const uint64_t lo = std::max(first, c->walk[b].pkt_off);
        const uint64_t hi = std::min(first + count, c->walk[b].pkt_off + c->walk[b].npkt);
        if (hi > lo) {
            c->walked[b] += hi - lo;
            c->walked_tiled[b] = tiled && c->tiled[b] ? 1 : 0;
        }
    }
    c->state = 2;
}

void drop_graph(mc_lya_ctx *c)
{
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    c->graph_exec = nullptr;
    c->graph_key.clear();
}

// What a captured transport depends on: any change means a new capture.
std::vector<uint64_t> graph_key(mc_lya_ctx *c, const WalkPlan &w, int budget)
{
    std::vector<uint64_t> k = {(uint64_t)c->kernel, (uint64_t)c->block, (uint64_t)c->waves_per_cu,
                               (uint64_t)c->chunk, (uint64_t)c->refill, (uint64_t)c->nqueues,
                               (uint64_t)c->tile_chunk, (uint64_t)c->tile_refill,
                               (uint64_t)c->max_cross, c->total_packets, c->state_cap, (uint64_t)budget,
                               (uint64_t)c->defer, (uint64_t)c->tail, (uint64_t)c->beside,
                               (uint64_t)w.tiled, (uint64_t)w.global, (uint64_t)c->tiles.size(),
                               (uint64_t)(uintptr_t)c->d_state[0], (uint64_t)(uintptr_t)c->d_cop,
                               (uint64_t)w.p.n_seg, w.p.count, c->epoch};
    k.insert(k.end(), c->tiled.begin(), c->tiled.end());
    return k;
}

// The whole transport as one captured HIP graph (zeroing the generation
// counters, `budget` tile generations, the persistent walk), replayed;
// generations beyond the budget, if any packet still crosses tiles, run
// eagerly after the replay, and the next capture takes a larger budget.
mc_lya_status transport_graph(mc_lya_ctx *c, WalkPlan &w)
{
    const int budget = w.tiled ? std::max(kGenRound, std::min(c->graph_gens, kMaxGenerations)) : 0;
    const std::vector<uint64_t> key = graph_key(c, w, budget);
    TileParams tp = tile_params(c, 0, c->total_packets);
    if (key != c->graph_key) {
        drop_graph(c);
        // capture on a private stream (the context's stream may be the null
        // stream, which cannot be captured); the graph is launched on the
        // context's stream
        if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        const hipStream_t user = c->stream;
        c->stream = c->cap_stream;
        hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            c->stream = user;
            return hip_fail(c, e, "hipStreamBeginCapture");
        }
        const int64_t gens = c->generations;
        const bool beside = w.tiled && w.global && c->beside > 0;
        bool forked = false;
        if (beside) {
            forked = true;
            if (fork_beside(c, [&] { return launch_global_walk(c, w.p, false, c->beside); }) != MC_LYA_OK)
                e = hipErrorUnknown;
        }
        if (e == hipSuccess && w.tiled) {
            e = launch_zero_counters(c->d_gen, kGenCounters, c->stream);
            if (e == hipSuccess && enqueue_generations(c, tp, 0, budget, false) != MC_LYA_OK) e = hipErrorUnknown;
            if (e == hipSuccess && enqueue_tail(c, c->total_packets, false) != MC_LYA_OK) e = hipErrorUnknown;
        }
        c->generations = gens;
        if (forked && join_beside(c) != MC_LYA_OK) e = hipErrorUnknown;
        if (e == hipSuccess && w.global && !beside && launch_global_walk(c, w.p, false) != MC_LYA_OK) e = hipErrorUnknown;
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(c->stream, &g);
        c->stream = user;
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            c->graph_exec = nullptr;
            return hip_fail(c, e, "capturing the transport graph");
        }
        c->graph_key = key;
        c->graph_launches = (w.tiled ? budget + (tail_packets(c, c->total_packets) ? 1 : 0) : 0) + (w.global ? 1 : 0);
    }
    hipEvent_t e1 = nullptr;
    mc_lya_status st = MC_LYA_OK;
    if (c->timing == 2) {
        c->coarse_launches += c->graph_launches;      // the transport's own event pair times them
    } else {
        st = timed_begin(c, &e1);
        if (st != MC_LYA_OK) return st;
    }
    HIP_TRY(c, hipGraphLaunch(c->graph_exec, c->stream));
    st = timed_end(c, e1);
    if (st != MC_LYA_OK) return st;
    c->generations = budget;
    if (w.tiled) {
        int end = budget;
        st = drain_generations(c, tp, budget, &end);
        // generations beyond the budget ran eagerly: their tail walk too
        if (st == MC_LYA_OK && end > budget) st = enqueue_tail(c, c->total_packets, true);
        if (st != MC_LYA_OK) return st;
        // ran out of captured generations: the next capture takes what this
        // emission needed plus one round of slack (empty generations return
        // at once)
        if (c->generations > budget) c->graph_gens = (int)std::min<int64_t>(c->generations + kGenRound, kMaxGenerations);
    }
    return MC_LYA_OK;
}

mc_lya_status launch_walk(mc_lya_ctx *c, uint64_t first, uint64_t count)
{
    if (count == 0) return MC_LYA_OK;
    WalkPlan w;
    mc_lya_status st = plan_walk(c, first, count, &w);
    if (st != MC_LYA_OK) return st;
    c->generations = 0;
    hipEvent_t coarse_end = nullptr;
    if (c->timing == 2) {
        st = event_pair(c, &coarse_end);
        if (st != MC_LYA_OK) return st;
    }
    const bool whole = first == 0 && count == c->total_packets;
    if (c->graph && whole && (!w.tiled || c->total_packets <= c->state_cap)) {
        st = transport_graph(c, w);
    } else if (w.tiled && w.global && c->beside > 0) {
        // the persistent part first, on the side stream, so that its
        // workgroups are resident before the tile generations fill the chip
        st = fork_beside(c, [&] { return launch_global_walk(c, w.p, true, c->beside); });
        if (st == MC_LYA_OK) st = walk_tiled(c, first, count);
        const mc_lya_status sj = join_beside(c);
        if (st == MC_LYA_OK) st = sj;
    } else {
        if (w.tiled) st = walk_tiled(c, first, count);
        if (st == MC_LYA_OK && w.global) st = launch_global_walk(c, w.p, true);
    }
    if (st == MC_LYA_OK && coarse_end) st = timed_end(c, coarse_end);
    if (st != MC_LYA_OK) return st;
    account_walked(c, first, count, c->kernel == 2);
    return MC_LYA_OK;
}

// The persistent (kernel 0 and the untiled part of kernel 2) or per-packet
// (kernel 1) walk over p.count packets.
mc_lya_status launch_global_walk(mc_lya_ctx *c, const WalkParams &p, bool timed, int waves_cap)
{
    const uint64_t count = p.count;
    hipEvent_t e1 = nullptr;
    if (timed) {
        mc_lya_status st = timed_begin(c, &e1);
        if (st != MC_LYA_OK) return st;
    }
    if (c->kernel == 1) {
        HIP_TRY(c, launch_walk_simple(p, c->block, c->stream));
    } else {
        const int waves_per_block = c->block / 64;
        // never more workgroups than can be resident at once
        const int resident = persistent_blocks_per_cu(c->vel, c->voigt, c->block);
        const int waves = waves_cap > 0 ? std::min(c->waves_per_cu, waves_cap) : c->waves_per_cu;
        const int per_cu = std::max(1, std::min(waves / waves_per_block, resident));
        int grid = c->num_cu * per_cu;
        const uint64_t need = (count + 63) / 64;     // no more waves than packets
        if ((uint64_t)grid * waves_per_block > need) grid = (int)std::max<uint64_t>(1, (need + waves_per_block - 1) / waves_per_block);
        HIP_TRY(c, launch_walk_persistent(p, c->block, grid, c->stream));
    }
    if (timed) return timed_end(c, e1);
    return MC_LYA_OK;
}

}  // namespace

extern "C" {

const char *mc_lya_strerror(mc_lya_status s)
{
    switch (s) {
    case MC_LYA_OK: return "ok";
    case MC_LYA_EINVAL: return "invalid argument or field value";
    case MC_LYA_ENOMEM: return "device allocation failed";
    case MC_LYA_EDEVICE: return "HIP runtime error";
    case MC_LYA_EOVERFLOW: return "integer range exceeded";
    case MC_LYA_ESTATE: return "call out of order";
    case MC_LYA_ECAP: return "a packet hit the crossing cap";
    case MC_LYA_ECONSERVE: return "conservation identity failed";
    }
    return "unknown status";
}

const char *mc_lya_last_error(const mc_lya_ctx *ctx) { return ctx ? ctx->err.c_str() : g_init_err.c_str(); }

mc_lya_status mc_lya_init(mc_lya_ctx **out, const mc_lya_box_desc *boxes, int32_t n_boxes,
                          const mc_lya_limits *limits, void *stream)
{
    g_init_err.clear();
    if (!out) return fail(nullptr, MC_LYA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!boxes || n_boxes < 1 || n_boxes > 1024)
        return fail(nullptr, MC_LYA_EINVAL, "need 1 to 1024 box descriptors");
    mc_lya_limits lim{};
    lim.max_packets = kDefaultMaxPackets;
    if (limits) lim = *limits;
    if (lim.max_packets == 0 || lim.max_packets >= (1ull << 40))
        return fail(nullptr, MC_LYA_EINVAL, "limits.max_packets must be in [1, 2^40)");
    if (lim.evolve != 0 && lim.evolve != 1) return fail(nullptr, MC_LYA_EINVAL, "limits.evolve must be 0 or 1");
    if (lim.reserved != 0) return fail(nullptr, MC_LYA_EINVAL, "limits.reserved must be 0");
    if (lim.batch_packets == 0 || lim.batch_packets > lim.max_packets) lim.batch_packets = lim.max_packets;
    uint64_t cells = 0;
    for (int b = 0; b < n_boxes; ++b) {
        const std::string why = check_desc(boxes[b], b);
        if (!why.empty()) return fail(nullptr, MC_LYA_EINVAL, why);
        cells += (uint64_t)boxes[b].nx * (uint64_t)boxes[b].ny * (uint64_t)boxes[b].nz;
        if (cells >= (1ull << 32)) return fail(nullptr, MC_LYA_EOVERFLOW, "more than 2^32 cells in total");
    }
    mc_lya_ctx *c = new (std::nothrow) mc_lya_ctx;
    if (!c) return fail(nullptr, MC_LYA_ENOMEM, "host allocation failed");
    c->stream = static_cast<hipStream_t>(stream);
    c->n_boxes = n_boxes;
    c->max_packets = lim.max_packets;
    c->desc.assign(boxes, boxes + n_boxes);
    c->total_cells = cells;
    c->pack.resize(n_boxes);
    c->walk.resize(n_boxes);
    c->red.resize(n_boxes);
    c->walked.assign(n_boxes, 0);
    c->walked_tiled.assign(n_boxes, 0);
    c->ph.resize(n_boxes);
    uint64_t off = 0;
    int max_blk = 1;
    for (int b = 0; b < n_boxes; ++b) {
        const mc_lya_box_desc &d = boxes[b];
        const uint64_t n = (uint64_t)d.nx * d.ny * d.nz;
        c->ph[b] = phys::scalars(d);
        PackBox &p = c->pack[b];
        std::memset(&p, 0, sizeof p);
        p.od = d.overdensity;
        p.vel = d.velocity;
        p.xe = d.x_e;
        p.src = d.source;
        p.kappa_unit = c->ph[b].kappa_unit;
        p.cell_off = (uint32_t)off;
        p.ncells = (uint32_t)n;
        p.xe_uniform = d.x_e_uniform;
        p.vel_dtype = d.vel_dtype;
        p.nblk = (int)((n + kSetupBlock - 1) / kSetupBlock);
        max_blk = std::max(max_blk, p.nblk);
        WalkBox &w = c->walk[b];
        std::memset(&w, 0, sizeof w);
        w.nx = d.nx;
        w.ny = d.ny;
        w.nz = d.nz;
        w.cell_off = (uint32_t)off;
        w.w0 = (uint32_t)d.w0;
        if (d.vel_dtype != MC_LYA_VEL_NONE) c->vel = true;
        if (d.profile == MC_LYA_PROFILE_VOIGT) c->voigt = true;
        off += n;
    }
    c->max_blk = max_blk;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cu > 0)
            c->num_cu = cu;
    }
    auto cleanup = [&](mc_lya_status s) {
        g_init_err = c->err.empty() ? std::string(mc_lya_strerror(s)) : c->err;
        free_all(c);
        delete c;
        return s;
    };
    const size_t nbk = (size_t)n_boxes * max_blk;
    hipError_t e = hipSuccess;
    if ((e = dalloc(&c->d_pack, n_boxes)) != hipSuccess || (e = dalloc(&c->d_walk, n_boxes)) != hipSuccess ||
        (e = dalloc(&c->d_red, n_boxes)) != hipSuccess || (e = dalloc(&c->d_tot, n_boxes)) != hipSuccess ||
        (e = hipMalloc(&c->d_rec, cells * (c->vel ? sizeof(float4) : sizeof(float)))) != hipSuccess ||
        (e = dalloc(&c->d_wgt, cells)) != hipSuccess || (e = dalloc(&c->d_part, nbk * kPartStride)) != hipSuccess ||
        (e = dalloc(&c->d_q, cells)) != hipSuccess || (e = dalloc(&c->d_bsum, nbk)) != hipSuccess ||
        (e = dalloc(&c->d_npk, cells)) != hipSuccess || (e = dalloc(&c->d_A, cells)) != hipSuccess ||
        (e = dalloc(&c->d_queue, kMaxQueues)) != hipSuccess || (e = dalloc(&c->d_boxabs, n_boxes)) != hipSuccess ||
        (e = dalloc(&c->d_fsum, (size_t)4 * n_boxes)) != hipSuccess ||
        (e = dalloc(&c->d_feed, n_boxes)) != hipSuccess || (e = dalloc(&c->d_pfirst, cells)) != hipSuccess ||
        (e = dalloc(&c->d_seg, 2 * ((size_t)n_boxes + 1))) != hipSuccess ||
        (e = dalloc(&c->d_featbox, n_boxes)) != hipSuccess || (e = dalloc(&c->d_sbox, n_boxes)) != hipSuccess ||
        (e = dalloc(&c->d_cop, lim.max_packets)) != hipSuccess ||
        (lim.evolve && ((e = dalloc(&c->d_ev, 6 * cells)) != hipSuccess ||
                        (e = dalloc(&c->d_ev_coef, (size_t)n_boxes)) != hipSuccess)) ||
        (e = alloc_tile_buffers(c, lim.batch_packets)) != hipSuccess)
        return cleanup(e == hipErrorOutOfMemory ? MC_LYA_ENOMEM : MC_LYA_EDEVICE);
    c->cpp.assign(n_boxes, 1.0);
    c->tiled.assign(n_boxes, 1);         // the tile table starts with every box; emit narrows it
    build_tiles(c);
    const size_t nt = c->tiles.size();
    if ((e = dalloc(&c->d_tiles, nt)) != hipSuccess || (e = dalloc(&c->d_texits[0], nt)) != hipSuccess ||
        (e = dalloc(&c->d_texits[1], nt)) != hipSuccess || (e = dalloc(&c->d_gen, kGenCounters)) != hipSuccess ||
        (e = dalloc(&c->d_tail_prefix, nt)) != hipSuccess)
        return cleanup(e == hipErrorOutOfMemory ? MC_LYA_ENOMEM : MC_LYA_EDEVICE);
    // (default stream priority)
    if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->join, hipEventDisableTiming) != hipSuccess)
        return cleanup(MC_LYA_EDEVICE);
    if (hipMemcpyAsync(c->d_tiles, c->tiles.data(), sizeof(TileInfo) * nt, hipMemcpyHostToDevice, c->stream) !=
            hipSuccess ||
        hipMemcpyAsync(c->d_pack, c->pack.data(), sizeof(PackBox) * n_boxes, hipMemcpyHostToDevice, c->stream) !=
            hipSuccess)
        return cleanup(MC_LYA_EDEVICE);
    mc_lya_status s = do_refresh(c);
    if (s != MC_LYA_OK) return cleanup(s);
    *out = c;
    return MC_LYA_OK;
}

mc_lya_status mc_lya_refresh(mc_lya_ctx *c)
{
    if (!c) return MC_LYA_EINVAL;
    return do_refresh(c);
}

mc_lya_status mc_lya_emit(mc_lya_ctx *c, const uint64_t *seeds, const uint64_t *n_packets)
{
    if (!c) return MC_LYA_EINVAL;
    if (c->state < 0) return fail(c, MC_LYA_ESTATE, "fields failed validation; call mc_lya_refresh");
    if (!seeds || !n_packets) return fail(c, MC_LYA_EINVAL, "seeds and n_packets must not be NULL");
    unsigned __int128 total = 0, weight = 0;
    for (int b = 0; b < c->n_boxes; ++b) {
        total += n_packets[b];
        weight += (unsigned __int128)n_packets[b] * c->desc[b].w0;
        double wmax = 0.0;
        std::memcpy(&wmax, &c->red[b].wmax_bits, sizeof wmax);
        if (n_packets[b] > 0 && !(wmax > 0.0))
            return fail(c, MC_LYA_EINVAL, "box " + std::to_string(b) + ": every emission weight is zero");
        if ((unsigned __int128)n_packets[b] * c->desc[b].w0 >= ((unsigned __int128)1 << 63))
            return fail(c, MC_LYA_EOVERFLOW, "w0 * packets of a box must stay below 2^63");
    }
    if (weight >= ((unsigned __int128)1 << 63) || total >= ((unsigned __int128)1 << 40))
        return fail(c, MC_LYA_EOVERFLOW, "total packets or total weight too large");
    if (total > c->max_packets)
        return fail(c, MC_LYA_EINVAL, "more packets than the max_packets reserved at mc_lya_init (" +
                                          std::to_string(c->max_packets) + ")");
    const uint64_t ntot = (uint64_t)total;
    uint64_t off = 0;
    for (int b = 0; b < c->n_boxes; ++b) {
        c->walk[b].pkt_off = off;
        c->walk[b].npkt = n_packets[b];
        c->walk[b].seed = seeds[b];
        off += n_packets[b];
        c->walked[b] = 0;
        c->walked_tiled[b] = 0;
    }
    c->total_packets = ntot;
    const int nb = c->n_boxes;
    HIP_TRY(c, hipMemcpyAsync(c->d_walk, c->walk.data(), sizeof(WalkBox) * nb, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, launch_quantize(c->d_pack, nb, c->max_blk, c->d_wgt, c->d_red, c->d_q, c->d_bsum, c->stream));
    HIP_TRY(c, launch_scan_blocks(c->d_pack, nb, c->max_blk, c->d_bsum, c->d_red, c->stream));
    HIP_TRY(c, launch_allocate(c->d_pack, c->d_walk, nb, c->max_blk, c->d_q, c->d_bsum, c->d_red, c->d_npk,
                               c->d_pfirst, c->stream));
    c->cop_valid = false;
    HIP_TRY(c, hipMemsetAsync(c->d_A, 0, sizeof(unsigned long long) * c->total_cells, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->d_tot, 0, sizeof(BoxTot) * nb, c->stream));
    c->state = 1;
    return MC_LYA_OK;
}

mc_lya_status mc_lya_transport(mc_lya_ctx *c)
{
    if (!c) return MC_LYA_EINVAL;
    if (c->state < 1) return fail(c, MC_LYA_ESTATE, "mc_lya_transport before mc_lya_emit");
    return launch_walk(c, 0, c->total_packets);
}

mc_lya_status mc_lya_transport_range(mc_lya_ctx *c, uint64_t first, uint64_t count)
{
    if (!c) return MC_LYA_EINVAL;
    if (c->state < 1) return fail(c, MC_LYA_ESTATE, "mc_lya_transport_range before mc_lya_emit");
    if (first > c->total_packets || count > c->total_packets - first)
        return fail(c, MC_LYA_EINVAL, "packet range outside the emitted packets");
    return launch_walk(c, first, count);
}

mc_lya_status mc_lya_tally(mc_lya_ctx *c, int64_t *absorbed, int64_t *emitted, mc_lya_box_stats *stats)
{
    if (!c) return MC_LYA_EINVAL;
    if (c->state < 1) return fail(c, MC_LYA_ESTATE, "mc_lya_tally before mc_lya_emit");
    const int nb = c->n_boxes;
    HIP_TRY(c, launch_tally(c->d_walk, nb, c->max_blk, c->d_A, c->d_npk, absorbed, emitted, c->d_part,
                            c->d_boxabs, c->stream));
    std::vector<BoxTot> tot(nb);
    std::vector<unsigned long long> abs(nb);
    HIP_TRY(c, hipMemcpyAsync(tot.data(), c->d_tot, sizeof(BoxTot) * nb, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(abs.data(), c->d_boxabs, sizeof(unsigned long long) * nb, hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    bool capped = false, broken = false;
    for (int b = 0; b < nb; ++b) {
        const uint64_t w0 = c->desc[b].w0;
        const uint64_t walked_w = c->walked[b] * w0;
        const uint64_t lhs = abs[b] + tot[b].escaped + tot[b].capped_weight;
        const bool ok = lhs == walked_w;
        if (!ok) broken = true;
        if (tot[b].capped_packets) capped = true;
        if (stats) {
            mc_lya_box_stats &s = stats[b];
            std::memset(&s, 0, sizeof s);
            s.emitted = (int64_t)walked_w;
            s.absorbed = (int64_t)abs[b];
            s.escaped = (int64_t)tot[b].escaped;
            s.capped_weight = (int64_t)tot[b].capped_weight;
            s.capped_packets = (int64_t)tot[b].capped_packets;
            s.crossings = (int64_t)tot[b].crossings;
            s.packets = (int64_t)c->walked[b];
            s.conserved = ok ? 1 : 0;
            s.tiled = c->walked_tiled[b];
            s.delta = c->walk[b].delta;
            s.x_eff = c->walk[b].x_eff;
            s.tau_ab_mean = c->red[b].kappa_sum / (double)c->walk[b].cells();
            s.damping = c->desc[b].profile == MC_LYA_PROFILE_VOIGT ? c->ph[b].damping : 0.0;
            s.wing = (int64_t)tot[b].wing;
            s.scatterings = (int64_t)tot[b].pad[0];
        }
    }
    if (broken) return fail(c, MC_LYA_ECONSERVE, "sum(absorbed) + escaped + capped != w0 * packets");
    if (capped) return fail(c, MC_LYA_ECAP, "some packets reached the crossing cap");
    return MC_LYA_OK;
}

// The per-box table of the features kernel, from the descriptors and the
// sums of the last refresh; uploaded once per refresh.
static hipError_t build_featbox(mc_lya_ctx *c)
{
    const int nb = c->n_boxes;
    hipError_t e = hipStreamSynchronize(c->stream);      // the previous table may still be in flight
    if (e != hipSuccess) return e;
    c->featbox.resize(nb);
    uint64_t blocks = 1;
    for (int b = 0; b < nb; ++b) {
        const mc_lya_box_desc &d = c->desc[b];
        FeatBox &f = c->featbox[b];
        std::memset(&f, 0, sizeof f);
        f.nx = d.nx;
        f.ny = d.ny;
        f.nz = d.nz;
        f.cell_off = c->pack[b].cell_off;
        f.ncells = c->pack[b].ncells;
        f.vel_dtype = d.vel_dtype;
        f.od = d.overdensity;
        f.vel = d.velocity;
        f.xe = d.x_e;
        f.xe_uniform = d.x_e_uniform;
        f.ln_t = (float)std::log(d.temp_K / 3000.0);
        f.z_feat = (float)(d.z / 1000.0 - 1.1);
        // the box clumping from the pack's FP64 sums (read back by refresh)
        const double n = (double)f.ncells, m1 = c->red[b].od_sum / n, m2 = c->red[b].od2_sum / n;
        f.ln_clump = m1 > 0.0 ? (float)std::log(m2 / (m1 * m1)) : 0.0f;
        // four cells per thread where rows hold whole groups of four and the
        // fields take 16-byte loads (8-byte for FP16 velocities)
        auto aligned = [](const void *p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; };
        f.quad = d.nx % 4 == 0 && aligned(d.overdensity, 16) && (!d.x_e || aligned(d.x_e, 16)) &&
                 (d.vel_dtype == MC_LYA_VEL_NONE || aligned(d.velocity, d.vel_dtype == MC_LYA_VEL_F16 ? 8 : 16));
        const uint64_t threads = f.quad ? f.ncells / 4u : f.ncells;
        blocks = std::max<uint64_t>(blocks, (threads + 255) / 256);
    }
    e = hipMemcpyAsync(c->d_featbox, c->featbox.data(), sizeof(FeatBox) * nb, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return e;
    c->feat_blocks = (int)blocks;
    c->featbox_stale = false;
    return hipSuccess;
}

mc_lya_status mc_lya_features(mc_lya_ctx *c, float *out)
{
    if (!c) return MC_LYA_EINVAL;
    if (!out) return fail(c, MC_LYA_EINVAL, "out is NULL");
    if (c->state < 0) return fail(c, MC_LYA_ESTATE, "fields failed validation; call mc_lya_refresh");
    const int nb = c->n_boxes;
    if (c->featbox_stale) HIP_TRY(c, build_featbox(c));
    HIP_TRY(c, launch_features(c->d_featbox, nb, c->feat_blocks, out, c->stream));
    return MC_LYA_OK;
}

// Per-box scalars of the feed from the last transport's tallies (uploaded to
// c->d_feed, queued on the stream) and, optionally, its statistics.
static mc_lya_status feed_prepare(mc_lya_ctx *c, mc_lya_feed_stats *stats)
{
    const int nb = c->n_boxes;
    HIP_TRY(c, launch_tally(c->d_walk, nb, c->max_blk, c->d_A, c->d_npk, nullptr, nullptr, c->d_part,
                            c->d_boxabs, c->stream));
    HIP_TRY(c, launch_feed_sums(c->d_pack, nb, c->max_blk, c->d_wgt, c->d_part, c->stream));
    HIP_TRY(c, launch_feed_reduce(nb, c->max_blk, c->d_pack, c->d_part, c->d_fsum, c->stream));
    std::vector<BoxTot> tot(nb);
    std::vector<unsigned long long> abs(nb);
    std::vector<double> sums((size_t)4 * nb);
    HIP_TRY(c, hipMemcpyAsync(tot.data(), c->d_tot, sizeof(BoxTot) * nb, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(abs.data(), c->d_boxabs, sizeof(unsigned long long) * nb, hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipMemcpyAsync(sums.data(), c->d_fsum, sizeof(double) * 4 * nb, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    std::vector<FeedBox> fb(nb);
    for (int b = 0; b < nb; ++b) {
        const phys::Box &ph = c->ph[b];
        const mc_lya_box_desc &d = c->desc[b];
        const double ncell = (double)c->walk[b].cells();
        const double wtot = (double)c->walked[b] * (double)d.w0;
        const double s_scale = d.source ? 1.0 : ph.alpha * ph.nH * ph.nH;
        const double sum_s = s_scale * sums[4 * b + 0];
        const double sum_n1s = ph.nH * sums[4 * b + 1];
        // the far damping wing's share of the escaped weight (Voigt profile)
        // is absorbed far away: it joins the absorption, spread like n_1s
        const double wing = (double)tot[b].wing;
        const double sum_A = (double)abs[b] + wing;
        const double reion = ph.beta / (ph.beta + phys::kL2g);
        const double e_true = (double)tot[b].escaped - wing;
        const double c_mc = wtot > 0.0 ? (e_true + sum_A * phys::kL2g / (ph.beta + phys::kL2g)) / wtot : 0.0;
        fb[b].S_scale = s_scale;
        fb[b].n_h = ph.nH;
        fb[b].a_norm = wtot > 0.0 ? sum_s / wtot : 0.0;
        fb[b].reion = reion;
        fb[b].thermal = c_mc * ph.beta * ph.boltz;
        fb[b].fm_norm = sum_n1s > 0.0 ? sum_A / sum_n1s : 0.0;
        fb[b].wing_n1s = sum_n1s > 0.0 ? wing / sum_n1s : 0.0;
        fb[b].w_inv = sums[4 * b + 0] > 0.0 ? 1.0 / sums[4 * b + 0] : 0.0;
        if (stats) {
            mc_lya_feed_stats &s = stats[b];
            const double n1s_mean = sum_n1s / ncell;
            const double r_mix = 8.0 * phys::kPi * ph.H /
                                 (phys::kLya * phys::kLya * phys::kLya * n1s_mean);
            s.c_mc = c_mc;
            s.c_mix = (phys::kL2g + r_mix) / (ph.beta + phys::kL2g + r_mix);
            s.f_escape = wtot > 0.0 ? e_true / wtot : 0.0;
            s.f_wing = wtot > 0.0 ? wing / wtot : 0.0;
            s.f_absorbed = wtot > 0.0 ? sum_A / wtot : 0.0;
            s.x_e_global = sums[4 * b + 3] > 0.0 ? sums[4 * b + 2] / sums[4 * b + 3] : 0.0;
            // volume mean of the rate: -<S> + reion <a> + thermal <n1s>
            s.ndot_e_mean = (-sum_s + reion * sum_A * fb[b].a_norm + fb[b].thermal * sum_n1s) / ncell;
        }
    }
    // (fb is host memory the copy reads: synchronise before it goes)
    HIP_TRY(c, hipMemcpyAsync(c->d_feed, fb.data(), sizeof(FeedBox) * nb, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MC_LYA_OK;
}

mc_lya_status mc_lya_feed(mc_lya_ctx *c, double *ndot_e, float *mix_corr, mc_lya_feed_stats *stats)
{
    if (!c) return MC_LYA_EINVAL;
    if (c->state < 2) return fail(c, MC_LYA_ESTATE, "mc_lya_feed before mc_lya_transport");
    mc_lya_status st = feed_prepare(c, stats);
    if (st != MC_LYA_OK) return st;
    if (ndot_e || mix_corr) {
        HIP_TRY(c, launch_feed(c->d_pack, c->d_feed, c->n_boxes, c->max_blk, c->d_wgt, c->d_A, ndot_e, mix_corr,
                               c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    return MC_LYA_OK;
}

mc_lya_status mc_lya_surrogate_targets(mc_lya_ctx *c, float *y, float *w)
{
    if (!c) return MC_LYA_EINVAL;
    if (c->state < 2) return fail(c, MC_LYA_ESTATE, "mc_lya_surrogate_targets before mc_lya_transport");
    if (!y || !w) return fail(c, MC_LYA_EINVAL, "y or w is NULL");
    mc_lya_status st = feed_prepare(c, nullptr);
    if (st != MC_LYA_OK) return st;
    HIP_TRY(c, launch_targets(c->d_pack, c->d_feed, c->n_boxes, c->max_blk, c->d_wgt, c->d_A, y, w, c->stream));
    return MC_LYA_OK;
}

mc_lya_status mc_lya_trace(mc_lya_ctx *c, uint64_t first, uint64_t count, mc_lya_packet_trace *out)
{
    if (!c) return MC_LYA_EINVAL;
    if (c->state < 1) return fail(c, MC_LYA_ESTATE, "mc_lya_trace before mc_lya_emit");
    if (!out && count) return fail(c, MC_LYA_EINVAL, "out is NULL");
    if (first > c->total_packets || count > c->total_packets - first)
        return fail(c, MC_LYA_EINVAL, "packet range outside the emitted packets");
    if (count == 0) return MC_LYA_OK;
    {
        mc_lya_status st = ensure_cell_of_packet(c);
        if (st != MC_LYA_OK) return st;
    }
    WalkParams p{};
    p.boxes = c->d_walk;
    p.n_boxes = c->n_boxes;
    p.vel = c->vel ? 1 : 0;
    p.voigt = c->voigt ? 1 : 0;
    p.rec = c->d_rec;
    p.cell_of_packet = c->d_cop;
    p.first = first;
    p.count = count;
    p.max_cross = c->max_cross;
    HIP_TRY(c, launch_trace(p, out, c->stream));
    return MC_LYA_OK;
}

mc_lya_status mc_lya_scatter(mc_lya_ctx *c, uint64_t first, uint64_t count, const mc_lya_scatter_opts *opts,
                             mc_lya_scatter_record *records)
{
    if (!c) return MC_LYA_EINVAL;
    if (c->state < 1) return fail(c, MC_LYA_ESTATE, "mc_lya_scatter before mc_lya_emit");
    if (first > c->total_packets || count > c->total_packets - first)
        return fail(c, MC_LYA_EINVAL, "packet range outside the emitted packets");
    mc_lya_scatter_opts o{};
    o.p_destroy = -1.0;                                   // NULL options: each box's p_ab
    if (opts) o = *opts;
    if (o.x_inert == 0.0) o.x_inert = 300.0;
    if (!(o.x_inert > 0.0) || !std::isfinite(o.x_inert)) return fail(c, MC_LYA_EINVAL, "x_inert must be > 0");
    if (!(o.p_destroy <= 1.0) || std::isnan(o.p_destroy)) return fail(c, MC_LYA_EINVAL, "p_destroy must be <= 1");
    if (o.max_events == 0) o.max_events = 0xffffffffull;
    if (o.max_events > 0xffffffffull) return fail(c, MC_LYA_EINVAL, "max_events must be < 2^32");
    if (!(o.x_return >= 0.0)) return fail(c, MC_LYA_EINVAL, "x_return must be >= 0");
    if (o.fixed_x0 != 0 && o.fixed_x0 != 1) return fail(c, MC_LYA_EINVAL, "fixed_x0 must be 0 or 1");
    if (o.fixed_x0 && !std::isfinite(o.x0)) return fail(c, MC_LYA_EINVAL, "x0 must be finite");
    if (count == 0) return MC_LYA_OK;
    mc_lya_status st = ensure_cell_of_packet(c);
    if (st != MC_LYA_OK) return st;
    const int nb = c->n_boxes;
    std::vector<ScatBox> sb(nb);
    for (int b = 0; b < nb; ++b) {
        const phys::Box &ph = c->ph[b];
        const bool voigt = c->desc[b].profile == MC_LYA_PROFILE_VOIGT;
        const double p = o.p_destroy < 0.0 ? ph.pab : o.p_destroy;
        sb[b].inv_pab = (float)(1.0 / ph.pab);
        sb[b].x_inert = (float)o.x_inert;
        sb[b].a = voigt ? (float)ph.damping : 0.0f;
        sb[b].damp = voigt ? (float)(2.0 * ph.damping / phys::kPi) : 0.0f;
        // destroyed iff the event's 64-bit word is below floor(p 2^64)
        sb[b].destroy = p <= 0.0 ? 0ull : (p >= 1.0 ? ~0ull : (uint64_t)std::ldexp(p, 64));
        sb[b].pad = 0;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));          // the previous table may still be in use
    HIP_TRY(c, hipMemcpyAsync(c->d_sbox, sb.data(), sizeof(ScatBox) * nb, hipMemcpyHostToDevice, c->stream));
    ScatterParams p{};
    p.boxes = c->d_walk;
    p.sbox = c->d_sbox;
    p.n_boxes = nb;
    p.vel = c->vel ? 1 : 0;
    p.rec = c->d_rec;
    p.cell_of_packet = c->d_cop;
    p.A = c->d_A;
    p.tot = c->d_tot;
    p.queue = c->d_queue;
    p.first = first;
    p.count = count;
    p.max_events = o.max_events;
    p.chunk = 64;
    p.refill = 16;
    p.nqueues = (int32_t)std::min<uint64_t>(8, std::max<uint64_t>(1, count / 64));
    p.fixed_x0 = o.fixed_x0;
    p.x0 = o.x0;
    p.x_return = (float)o.x_return;
    p.records = records;
    // resident waves: 8 workgroups of 256 per compute unit, capped by the work
    const uint64_t want = (count + 255) / 256;
    const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)c->num_cu * 8, want));
    hipEvent_t e1 = nullptr;
    st = timed_begin(c, &e1);
    if (st != MC_LYA_OK) return st;
    HIP_TRY(c, launch_scatter(p, 256, grid, c->stream));
    st = timed_end(c, e1);
    if (st != MC_LYA_OK) return st;
    account_walked(c, first, count, false);
    return MC_LYA_OK;
}

// Moves every box to redshift z with T = T_cmb0 (1 + z): the physical
// scalars, the packed opacity unit and the descriptors (the next refresh
// re-packs the fields with them).
mc_lya_status set_epoch(mc_lya_ctx *c, double z)
{
    for (int b = 0; b < c->n_boxes; ++b) {
        mc_lya_box_desc &d = c->desc[b];
        d.z = z;
        d.temp_K = d.t_cmb0 * (1.0 + z);
        c->ph[b] = phys::scalars(d);
        c->pack[b].kappa_unit = c->ph[b].kappa_unit;
    }
    HIP_TRY(c, hipMemcpyAsync(c->d_pack, c->pack.data(), sizeof(PackBox) * c->n_boxes, hipMemcpyHostToDevice,
                              c->stream));
    drop_graph(c);
    ++c->epoch;
    return MC_LYA_OK;
}

// Global X_e = sum(x_e Delta) / sum(Delta) of every box from the fields.
mc_lya_status global_xe(mc_lya_ctx *c, double *X)
{
    const int nb = c->n_boxes;
    HIP_TRY(c, launch_feed_sums(c->d_pack, nb, c->max_blk, c->d_wgt, c->d_part, c->stream));
    HIP_TRY(c, launch_feed_reduce(nb, c->max_blk, c->d_pack, c->d_part, c->d_fsum, c->stream));
    std::vector<double> sums((size_t)4 * nb);
    HIP_TRY(c, hipMemcpyAsync(sums.data(), c->d_fsum, sizeof(double) * 4 * nb, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int b = 0; b < nb; ++b) X[b] = sums[4 * b + 3] > 0.0 ? sums[4 * b + 2] / sums[4 * b + 3] : 0.0;
    return MC_LYA_OK;
}

mc_lya_status mc_lya_evolve(mc_lya_ctx *c, double z0, double z1, int32_t n_steps, const uint64_t *n_packets,
                            uint64_t seed, float *const *x_e, double *X_out)
{
    if (!c) return MC_LYA_EINVAL;
    if (c->state < 0) return fail(c, MC_LYA_ESTATE, "fields failed validation; call mc_lya_refresh");
    if (!(n_steps > 0)) return fail(c, MC_LYA_EINVAL, "n_steps must be > 0");
    if (!(std::isfinite(z0) && std::isfinite(z1) && z0 > z1 && z1 > 0.0))
        return fail(c, MC_LYA_EINVAL, "need finite z0 > z1 > 0");
    if (!n_packets || !x_e) return fail(c, MC_LYA_EINVAL, "n_packets and x_e must not be NULL");
    const int nb = c->n_boxes;
    for (int b = 0; b < nb; ++b)
        if (!x_e[b] || x_e[b] != c->desc[b].x_e)
            return fail(c, MC_LYA_EINVAL, "box " + std::to_string(b) + ": x_e must be its descriptor's x_e field");
    const size_t n = c->total_cells;
    if (!c->d_ev) return fail(c, MC_LYA_ESTATE, "mc_lya_evolve needs limits.evolve = 1 at mc_lya_init");
    double *y0 = c->d_ev, *ndot = c->d_ev + 5 * n;
    double *k[4] = {c->d_ev + n, c->d_ev + 2 * n, c->d_ev + 3 * n, c->d_ev + 4 * n};
    HIP_TRY(c, launch_xe_load(c->d_pack, nb, c->max_blk, y0, c->stream));
    if (X_out) {
        mc_lya_status st = global_xe(c, X_out);
        if (st != MC_LYA_OK) return st;
    }
    const double h = (z1 - z0) / n_steps;
    const double cz[4] = {0.0, 0.5, 0.5, 1.0};            // stage redshift offsets
    std::vector<uint64_t> seeds(nb);
    std::vector<double> coef(nb);
    for (int32_t i = 0; i < n_steps; ++i) {
        const double z = z0 + i * h;
        for (int s = 0; s < 4; ++s) {
            if (s > 0) {                                  // the stage's x_e: y0 + c_s h k_{s-1}
                const double w = cz[s] * h;
                const double *kk[1] = {k[s - 1]};
                HIP_TRY(c, launch_xe_combine(c->d_pack, nb, c->max_blk, y0, kk, &w, 1, nullptr, true, c->stream));
            }
            const double zs = z + cz[s] * h;
            mc_lya_status st = set_epoch(c, zs);
            if (st == MC_LYA_OK) st = do_refresh(c);
            for (int b = 0; b < nb; ++b) seeds[b] = seed + (((uint64_t)(4 * (uint64_t)i + s)) << 20) + (uint64_t)b;
            if (st == MC_LYA_OK) st = mc_lya_emit(c, seeds.data(), n_packets);
            if (st == MC_LYA_OK) st = launch_walk(c, 0, c->total_packets);
            if (st == MC_LYA_OK) st = mc_lya_feed(c, ndot, nullptr, nullptr);
            if (st != MC_LYA_OK) return st;
            for (int b = 0; b < nb; ++b) coef[b] = -1.0 / (c->ph[b].nH * (1.0 + zs) * c->ph[b].H);
            HIP_TRY(c, hipMemcpyAsync(c->d_ev_coef, coef.data(), sizeof(double) * nb, hipMemcpyHostToDevice,
                                      c->stream));
            HIP_TRY(c, launch_xe_rate(c->d_pack, nb, c->max_blk, c->d_ev_coef, ndot, k[s], c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));   // coef is reused by the next stage
        }
        const double w[4] = {h / 6.0, h / 3.0, h / 3.0, h / 6.0};
        const double *kk[4] = {k[0], k[1], k[2], k[3]};
        HIP_TRY(c, launch_xe_combine(c->d_pack, nb, c->max_blk, y0, kk, w, 4, y0, true, c->stream));
        if (X_out) {
            mc_lya_status st = global_xe(c, X_out + (size_t)(i + 1) * nb);
            if (st != MC_LYA_OK) return st;
        }
    }
    // leave the context at z1, re-packed from the final fields
    mc_lya_status st = set_epoch(c, z1);
    if (st == MC_LYA_OK) st = do_refresh(c);
    return st;
}

mc_lya_status mc_lya_set_option(mc_lya_ctx *c, int32_t option, int64_t v)
{
    if (!c) return MC_LYA_EINVAL;
    switch (option) {
    case MC_LYA_OPT_KERNEL:
        if (v < 0 || v > 2) return fail(c, MC_LYA_EINVAL, "kernel must be 0, 1 or 2");
        c->kernel = (int)v;
        return MC_LYA_OK;
    case MC_LYA_OPT_BLOCK:
        if (v != 64 && v != 128 && v != 256) return fail(c, MC_LYA_EINVAL, "block must be 64, 128 or 256");
        c->block = (int)v;
        return MC_LYA_OK;
    case MC_LYA_OPT_WAVES_PER_CU:
        if (v < 1 || v > 64) return fail(c, MC_LYA_EINVAL, "waves per CU must be in [1, 64]");
        c->waves_per_cu = (int)v;
        return MC_LYA_OK;
    case MC_LYA_OPT_CHUNK:
        if (v < 1 || v > (1 << 20)) return fail(c, MC_LYA_EINVAL, "chunk must be in [1, 2^20]");
        c->chunk = (int)v;
        return MC_LYA_OK;
    case MC_LYA_OPT_REFILL:
        if (v < 1 || v > 64) return fail(c, MC_LYA_EINVAL, "refill must be in [1, 64]");
        c->refill = (int)v;
        return MC_LYA_OK;
    case MC_LYA_OPT_MAX_CROSSINGS:
        if (v < 1 || v > 0x7fffffff) return fail(c, MC_LYA_EINVAL, "crossing cap must be in [1, 2^31)");
        c->max_cross = v;
        return MC_LYA_OK;
    case MC_LYA_OPT_QUEUES:
        if (v < 1 || v > kMaxQueues) return fail(c, MC_LYA_EINVAL, "queues must be in [1, 64]");
        c->nqueues = (int)v;
        return MC_LYA_OK;
    case MC_LYA_OPT_TIMING:
        if (v < 0 || v > 2) return fail(c, MC_LYA_EINVAL, "timing must be 0, 1 or 2");
        if (v != c->timing) {
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            c->events_used = 0;        // pairs of the other mode are dropped
            c->coarse_launches = 0;
        }
        c->timing = (int)v;
        return MC_LYA_OK;
    case MC_LYA_OPT_TILE_SHARE:
        if (v < 0 || v > kAllTiled) return fail(c, MC_LYA_EINVAL, "tile share must be in [0, 1000000]");
        c->tile_share = (int)v;
        return MC_LYA_OK;
    case MC_LYA_OPT_TILE_CHUNK:
        if (v < 1 || v > 1024) return fail(c, MC_LYA_EINVAL, "tile chunk must be in [1, 1024]");
        c->tile_chunk = (int)v;
        return MC_LYA_OK;
    case MC_LYA_OPT_TILE_REFILL:
        if (v < 1 || v > 64) return fail(c, MC_LYA_EINVAL, "tile refill must be in [1, 64]");
        c->tile_refill = (int)v;
        return MC_LYA_OK;
    case MC_LYA_OPT_BESIDE:
        if (v < 0 || v > 32) return fail(c, MC_LYA_EINVAL, "beside must be in [0, 32]");
        c->beside = (int)v;
        return MC_LYA_OK;
    case MC_LYA_OPT_TAIL:
        if (v < 0 || v > 1000000) return fail(c, MC_LYA_EINVAL, "tail must be in [0, 1000000] (ppm)");
        c->tail = (int)v;
        return MC_LYA_OK;
    case MC_LYA_OPT_DEFER:
        if (v < 0 || v > 64) return fail(c, MC_LYA_EINVAL, "defer must be in [0, 64]");
        c->defer = (int)v;
        return MC_LYA_OK;
    case MC_LYA_OPT_GRAPH_GENS:
        if (v < kGenRound || v > kMaxGenerations)
            return fail(c, MC_LYA_EINVAL, "graph generations must be in [16, 4096]");
        c->graph_gens = (int)v;
        return MC_LYA_OK;
    case MC_LYA_OPT_GRAPH:
        if (v != 0 && v != 1) return fail(c, MC_LYA_EINVAL, "graph must be 0 or 1");
        c->graph = v == 1;
        return MC_LYA_OK;
    }
    return fail(c, MC_LYA_EINVAL, "unknown option");
}

mc_lya_status mc_lya_autotune(mc_lya_ctx *c, int32_t reps, mc_lya_tune_result *result)
{
    if (!c) return MC_LYA_EINVAL;
    if (c->state < 1) return fail(c, MC_LYA_ESTATE, "mc_lya_autotune before mc_lya_emit");
    if (reps < 1 || reps > 100) return fail(c, MC_LYA_EINVAL, "reps must be in [1, 100]");
    struct Opts {
        int kernel, share, block, waves, chunk, refill, tchunk, trefill;
        bool operator==(const Opts &o) const
        {
            return kernel == o.kernel && share == o.share && block == o.block && waves == o.waves &&
                   chunk == o.chunk && refill == o.refill && tchunk == o.tchunk && trefill == o.trefill;
        }
    };
    const Opts start{c->kernel, c->tile_share, c->block, c->waves_per_cu, c->chunk, c->refill, c->tile_chunk,
                     c->tile_refill};
    std::vector<Opts> cand = {start};
    // tiled walk (with the persistent walk for crowded boxes) at several tile
    // shares, tile chunks and refill thresholds; the persistent walk alone
    const Opts fixed[] = {
        {2, 100, 256, 32, 256, 16, 512, 40}, {2, 50, 256, 32, 256, 16, 512, 40}, {2, 25, 256, 32, 256, 16, 512, 40},
        {2, 100, 256, 32, 256, 16, 128, 40}, {2, 100, 256, 32, 256, 16, 1024, 40}, {2, 100, 256, 32, 256, 16, 512, 48},
        {2, 100, 256, 32, 256, 16, 512, 32},
        {0, 100, 256, 32, 256, 16, 512, 40}, {0, 100, 256, 16, 256, 16, 512, 40}, {0, 100, 256, 32, 64, 16, 512, 40},
        {0, 100, 256, 32, 256, 32, 512, 40}, {0, 100, 128, 32, 256, 16, 512, 40},
    };
    for (const Opts &o : fixed)
        if (std::find(cand.begin(), cand.end(), o) == cand.end()) cand.push_back(o);
    const int timing = c->timing;
    c->timing = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto finish = [&](mc_lya_status st) {
        c->timing = timing;
        if (st != MC_LYA_OK) {
            // a failed tuning leaves the options it started with
            c->kernel = start.kernel;
            c->tile_share = start.share;
            c->block = start.block;
            c->waves_per_cu = start.waves;
            c->chunk = start.chunk;
            c->refill = start.refill;
            c->tile_chunk = start.tchunk;
            c->tile_refill = start.trefill;
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        return st;
    };
    auto reset = [&]() -> mc_lya_status {
        HIP_TRY(c, hipMemsetAsync(c->d_A, 0, sizeof(unsigned long long) * c->total_cells, c->stream));
        HIP_TRY(c, hipMemsetAsync(c->d_tot, 0, sizeof(BoxTot) * c->n_boxes, c->stream));
        std::fill(c->walked.begin(), c->walked.end(), 0);
        std::fill(c->walked_tiled.begin(), c->walked_tiled.end(), 0);
        c->state = 1;
        return MC_LYA_OK;
    };
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return finish(fail(c, MC_LYA_EDEVICE, "event creation"));
    double best = 1e300, first_ms = 0.0;
    Opts pick = start;
    for (size_t i = 0; i < cand.size(); ++i) {
        const Opts &o = cand[i];
        c->kernel = o.kernel;
        c->tile_share = o.share;
        c->block = o.block;
        c->waves_per_cu = o.waves;
        c->chunk = o.chunk;
        c->refill = o.refill;
        c->tile_chunk = o.tchunk;
        c->tile_refill = o.trefill;
        double t_min = 1e300;
        for (int r = 0; r <= reps; ++r) {      // the first run warms up (captures, allocations)
            mc_lya_status st = reset();
            if (st != MC_LYA_OK) return finish(st);
            if (hipEventRecord(e0, c->stream) != hipSuccess) return finish(fail(c, MC_LYA_EDEVICE, "event"));
            st = launch_walk(c, 0, c->total_packets);
            if (st != MC_LYA_OK) return finish(st);
            if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
                return finish(fail(c, MC_LYA_EDEVICE, "event"));
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return finish(fail(c, MC_LYA_EDEVICE, "event"));
            if (r > 0) t_min = std::min(t_min, (double)ms);
        }
        if (i == 0) first_ms = t_min;
        if (t_min < best) {
            best = t_min;
            pick = o;
        }
    }
    c->kernel = pick.kernel;
    c->tile_share = pick.share;
    c->block = pick.block;
    c->waves_per_cu = pick.waves;
    c->chunk = pick.chunk;
    c->refill = pick.refill;
    c->tile_chunk = pick.tchunk;
    c->tile_refill = pick.trefill;
    mc_lya_status st = reset();
    if (st != MC_LYA_OK) return finish(st);
    if (result) {
        result->kernel = pick.kernel;
        result->tile_share = pick.share;
        result->block = pick.block;
        result->waves_per_cu = pick.waves;
        result->chunk = pick.chunk;
        result->refill = pick.refill;
        result->tile_chunk = pick.tchunk;
        result->tile_refill = pick.trefill;
        result->best_ms = best;
        result->start_ms = first_ms;
        result->trials = (int32_t)cand.size();
        result->reserved = 0;
    }
    return finish(MC_LYA_OK);
}

mc_lya_status mc_lya_kernel_time(mc_lya_ctx *c, double *ms, int64_t *launches)
{
    if (!c || !ms) return MC_LYA_EINVAL;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    double tot = 0.0;
    for (size_t i = 0; i < c->events_used; ++i) {
        float t = 0.0f;
        HIP_TRY(c, hipEventElapsedTime(&t, c->events[i].first, c->events[i].second));
        tot += t;
    }
    *ms = tot;
    if (launches) *launches = c->timing == 2 ? c->coarse_launches : (int64_t)c->events_used;
    c->events_used = 0;
    c->coarse_launches = 0;
    return MC_LYA_OK;
}

}  // extern "C"

namespace mclya {
// the read probe (kernels_probe.hip), a measurement utility
hipError_t launch_probe_read(const void *buf, uint64_t bytes, int passes, int grid, float *sink, hipStream_t s);
}  // namespace mclya

extern "C" {

mc_lya_status mc_lya_probe_read(const void *buf, uint64_t bytes, int32_t passes, int32_t grid, float *sink,
                                void *stream)
{
    if (!buf || !sink || bytes < 16 || bytes % 16 != 0 || passes < 1 || grid < 1) return MC_LYA_EINVAL;
    if (launch_probe_read(buf, bytes, passes, grid, sink, static_cast<hipStream_t>(stream)) != hipSuccess)
        return MC_LYA_EDEVICE;
    return MC_LYA_OK;
}

mc_lya_status mc_lya_philox4x32_10(const uint32_t *ctr, const uint32_t *key, uint32_t *out, uint64_t n,
                                   void *stream)
{
    if (n == 0) return MC_LYA_OK;
    if (!ctr || !key || !out) return MC_LYA_EINVAL;
    if (launch_philox(ctr, key, out, n, static_cast<hipStream_t>(stream)) != hipSuccess) return MC_LYA_EDEVICE;
    return MC_LYA_OK;
}

void mc_lya_destroy(mc_lya_ctx *c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
}

}  // extern "C"

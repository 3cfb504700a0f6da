/*
 * mc_lya.h -- C ABI of the MI355X (gfx950) Monte-Carlo Lyman-alpha packet
 * transport library (libmclya.so).
 *
 * The library computes, for one or many periodic boxes of baryons, where the
 * Lyman-alpha photons emitted by recombination are destroyed, and turns the
 * result into the local recombination rate. It follows Jedamzik, Abel &
 * Ali-Haimoud, "Cosmic recombination in the presence of primordial magnetic
 * fields" (arXiv:2312.11448):
 *   - emission in proportion to the recombination source alpha_e n_e^2
 *     (Eq. rec0; the Monte-Carlo integral of the footnote in Sec. III.B);
 *   - frequency drift by the Hubble flow along the path (App. A, step 4) and
 *     the bulk-velocity shift of Eq. (inout) between cells;
 *   - destruction by the true-absorption opacity p_ab n_1s sigma(x), whose
 *     integral over the line is the mean optical depth of Eq. (<fnu>);
 *   - escape by redshifting out of the line (end of App. A);
 *   - the per-cell feed of Eq. (rec) / Eq. (dotne-mix) (Sec. III.A.1, IV.B).
 * Packets stream in straight lines (no resonant scattering); their weight is
 * deposited as an expected value into 64-bit integer per-cell tallies, so
 * the tallies do not depend on the order of the atomic updates and
 *   sum(absorbed) + escaped + capped == w0 * packets   holds exactly.
 *
 * Conventions
 *   - Grids are C-ordered [nz][ny][nx] (x fastest), periodic in all three
 *     directions. With several boxes, cells and packets are concatenated box
 *     by box ("box-major") in the order the boxes were given.
 *   - "dev" pointers are HIP device memory; "host" pointers are host memory.
 *     All device work is queued on the HIP stream given to mc_lya_init. The
 *     one exception is the persistent walk of a kernel-2 transport's untiled
 *     boxes (MC_LYA_OPT_BESIDE), which runs on a stream the context creates at
 *     init, forked from that stream and joined back into it before the call
 *     returns its work to it: work queued afterwards on the context's stream
 *     waits for both.
 *   - Every call returns a status and never aborts. On failure the context is
 *     left as it was and mc_lya_last_error() describes the failure.
 *   - Call order: init -> [refresh] -> emit -> transport (or transport_range,
 *     any number of times) -> tally / feed / trace -> emit ... ; calling out
 *     of this order returns MC_LYA_ESTATE.
 *   - A context is not thread-safe; use one context per host thread.
 */
#ifndef MC_LYA_H
#define MC_LYA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MC_LYA_ABI_VERSION 4

typedef struct mc_lya_ctx mc_lya_ctx;

typedef enum mc_lya_status {
    MC_LYA_OK = 0,
    MC_LYA_EINVAL = 1,      /* bad argument or field value (NaN, negative density, ...) */
    MC_LYA_ENOMEM = 2,      /* a device allocation failed */
    MC_LYA_EDEVICE = 3,     /* the HIP runtime reported an error */
    MC_LYA_EOVERFLOW = 4,   /* w0 * packets >= 2^63, or more than 2^32 cells */
    MC_LYA_ESTATE = 5,      /* call out of order */
    MC_LYA_ECAP = 6,        /* some packet hit the crossing cap (weights still conserved) */
    MC_LYA_ECONSERVE = 7    /* the integer conservation identity failed (internal error) */
} mc_lya_status;

/* velocity field element type */
enum { MC_LYA_VEL_NONE = 0, MC_LYA_VEL_F32 = 1, MC_LYA_VEL_F16 = 2 };

/* Line profile of a box.
 *   DOPPLER: the thermal profile exp(-x^2)/sqrt(pi).
 *   VOIGT:   the profile of Eq. (MC), the thermal one convolved with the
 *            natural (Lorentz) width of the 2p level, half width
 *            a = A_2p lambda_alpha / (4 pi v_th) in Doppler units (8.6e-4 at
 *            3000 K). Emission adds a Cauchy deviate of half width a to the
 *            thermal frequency. The walk uses the cumulative profile to first
 *            order in a, erfc(-x)/2 - (2a/pi) F(x) with F Dawson's integral
 *            (error O(a^2)). The damping wing keeps absorbing past -x_eff:
 *            an escaping packet leaves the expected share
 *            1 - exp(-<kappa> Phi(x_stop)) of its weight to it (<kappa> the
 *            box's mean kappa; x_stop = -x_eff, or the emission frequency of
 *            a packet emitted outside the walked window). That share is
 *            counted in `escaped` and reported as `wing`; the feed treats it
 *            as absorbed and spread like n_1s (fully mixed). Packets emitted
 *            above x_blue = x_eff + (x_eff - x_esc), blue of every frequency
 *            a walked packet can reach, are not walked (App. A's photons far
 *            in the blue wing meet the line hundreds of cells away). */
enum { MC_LYA_PROFILE_DOPPLER = 0, MC_LYA_PROFILE_VOIGT = 1 };

/* One periodic box: its grid, its physics and its (caller-owned) fields.
 * Physics parameters are those of the paper's runs (Sec. II.C): cosmology
 * (h, Omega_b h^2, Omega_c h^2, Y_p), the redshift z, and zeta, the factor
 * multiplying the expansion rate in the paper's Monte-Carlo test problem
 * (App. A, H -> zeta H; 1 for physical runs). */
typedef struct mc_lya_box_desc {
    int32_t nx, ny, nz;           /* grid edge in cells, each >= 1 */
    int32_t vel_dtype;            /* MC_LYA_VEL_NONE / _F32 / _F16 */
    double cell_comoving_cm;      /* comoving cell edge, cm (> 0) */
    double z;                     /* redshift (> 0) */
    double zeta;                  /* expansion-rate factor (> 0), 1 = physical */
    double x_esc;                 /* red-wing escape threshold in Doppler widths (> 0) */
    double temp_K;                /* gas and radiation temperature, uniform in the box (> 0) */
    double h, omega_b_h2, omega_c_h2, y_p, t_cmb0, n_eff;   /* cosmology */
    uint64_t w0;                  /* integer weight of one packet, 1 <= w0 < 2^32 (e.g. 2^31) */
    const float *overdensity;     /* dev [ncells]: Delta = rho_b / <rho_b>, finite, >= 0 */
    const void *velocity;         /* dev [3][ncells] (x, y, z components) in units of the
                                     thermal velocity sqrt(2kT/m_H), or NULL */
    const float *x_e;             /* dev [ncells] free-electron fraction in [0, 1.2], or NULL */
    float x_e_uniform;            /* used when x_e == NULL */
    int32_t profile;              /* MC_LYA_PROFILE_DOPPLER (0) or MC_LYA_PROFILE_VOIGT */
    const float *source;          /* dev [ncells] emission rate density (cm^-3 s^-1, finite,
                                     >= 0), or NULL for alpha_e(T) n_e^2 */
} mc_lya_box_desc;

/* Per-box integer totals from mc_lya_tally. */
typedef struct mc_lya_box_stats {
    int64_t emitted;              /* w0 * packets emitted in the box */
    int64_t absorbed;             /* sum of the box's per-cell tallies */
    int64_t escaped;              /* weight redshifted out of the line */
    int64_t capped_weight;        /* weight of packets stopped by the crossing cap */
    int64_t capped_packets;
    int64_t crossings;            /* (packet, cell) segments walked */
    int64_t packets;              /* packets emitted in the box */
    int32_t conserved;            /* 1 iff absorbed + escaped + capped_weight == emitted */
    int32_t tiled;                /* 1 if the last walk of the box's packets was the tile-decomposed
                                     walk, 0 if the persistent or one-thread-per-packet walk (or the
                                     scattering Monte Carlo) took them */
    double delta;                 /* red drift per cell width, Doppler units (App. A step 4) */
    double x_eff;                 /* escape threshold used (x_esc + velocity margin) */
    double tau_ab_mean;           /* <kappa_c>: mean optical depth to true absorption */
    double damping;               /* Voigt a (0 for the Doppler profile) */
    int64_t wing;                 /* part of `escaped` that the far damping wing absorbs
                                     (Voigt; 0 for the Doppler profile) */
    int64_t scatterings;          /* resonant scatterings (mc_lya_scatter; 0 for the walk) */
} mc_lya_box_stats;

/* Per-box scalars from mc_lya_feed. */
typedef struct mc_lya_feed_stats {
    double c_mc;                  /* Monte-Carlo Peebles factor [E + sum(A) L/(b+L)] / (w0 N),
                                     E = escaped - wing and sum(A) including wing */
    double c_mix;                 /* Eq. (Cfactor) with R_alpha -> R_alpha^mix (Sec. IV.A.2) */
    double f_escape;              /* (escaped - wing) / emitted: the weight that truly escapes */
    double f_absorbed;            /* absorbed / emitted */
    double x_e_global;            /* X_e = <n_e> / <n_H> (Sec. II.A) */
    double ndot_e_mean;           /* volume mean of the per-cell rate, cm^-3 s^-1 */
    double f_wing;                /* wing / emitted (Voigt: absorbed by the far damping wing) */
} mc_lya_feed_stats;

/* One packet's history from mc_lya_trace (64 bytes). */
typedef struct mc_lya_packet_trace {
    uint32_t cell0;               /* global emission cell */
    float fx, fy, fz;             /* emission position inside the cell, [0,1) */
    float kx, ky, kz;             /* direction */
    float x0;                     /* emission frequency, gas frame, Doppler widths */
    int64_t escaped;              /* weight that escaped (0 if absorbed) */
    int64_t absorbed;             /* weight deposited into the grid */
    uint32_t crossings;
    int32_t fate;                 /* 0 absorbed, 1 escaped, 2 capped */
    int64_t wing;                 /* part of `escaped` the far damping wing absorbs (Voigt) */
} mc_lya_packet_trace;

/* Tunables for mc_lya_set_option (all results are independent of them, bit
 * for bit, except MC_LYA_OPT_MAX_CROSSINGS). */
enum {
    MC_LYA_OPT_KERNEL = 1,        /* 0 = persistent walk with wave refill and device
                                     atomics, 1 = one thread per packet,
                                     2 = tile-decomposed walk (default): 16^3-cell
                                     tiles, tallies in LDS, packets handed between
                                     tiles once per generation */
    MC_LYA_OPT_BLOCK = 2,         /* threads per workgroup: 64, 128 or 256 */
    MC_LYA_OPT_WAVES_PER_CU = 3,  /* resident waves per compute unit for the persistent grid */
    MC_LYA_OPT_CHUNK = 4,         /* persistent walk: packets a wave takes from the queue at
                                     once (>= 1) */
    MC_LYA_OPT_REFILL = 5,        /* persistent walk: refill a wave once this many lanes are
                                     idle (1..64) */
    MC_LYA_OPT_MAX_CROSSINGS = 6, /* crossing cap per packet (>= 1, default 1e6) */
    MC_LYA_OPT_TIMING = 7,        /* 0 = off (default); 1 = a HIP event pair around every walk
                                     launch; 2 = one pair around each transport's walk, with
                                     its launches counted (no events between launches, so the
                                     launches run back to back) */
    MC_LYA_OPT_GRAPH = 8,         /* 1 = a whole-emission mc_lya_transport replays a captured
                                     HIP graph of its kernels (recaptured when options, packet
                                     count or buffers change; tiled emissions larger than the
                                     packet-state buffers, 2^25 packets, and
                                     mc_lya_transport_range stay eager) */
    MC_LYA_OPT_QUEUES = 9,        /* parts the packet range is split into for the persistent
                                     walk (1..64, default 8: one grid slab per XCD) */
    MC_LYA_OPT_TILE_SHARE = 10,   /* kernel 2: a box is walked by tiles when it has at least 8
                                     tiles and its estimated crossings per tile are at most
                                     this percentage of the emission's crossings per compute
                                     unit (default 100); other boxes take the persistent walk.
                                     0 = no box tiled, 1000000 = every box tiled */
    MC_LYA_OPT_GRAPH_GENS = 11,   /* tile generations inside a captured transport graph
                                     (16..4096, default 64); a replay that needs more
                                     continues eagerly and the next capture takes enough */
    MC_LYA_OPT_DEFER = 12,        /* tiled walk: once a tile's input is used up, a wave with
                                     at most this many live packets (0..64, default 16) hands
                                     them to the tile's next generation instead of walking on
                                     with idle lanes (tiles that took >= 2048 packets) */
    MC_LYA_OPT_TILE_CHUNK = 13,   /* tiled walk: packets a wave takes from its tile's input at
                                     once (1..1024, default 512; smaller claims near the end
                                     of the input) */
    MC_LYA_OPT_TILE_REFILL = 14,  /* tiled walk: refill a wave once this many lanes are idle
                                     (1..64, default 40) */
    MC_LYA_OPT_TAIL = 15,         /* tiled walk: once fewer packets than this many millionths
                                     of a batch are in flight (0..1000000, default 20000 =
                                     2 %; 0 = never), one kernel walks them to the end with
                                     device-wide deposits instead of further, thinning tile
                                     generations */
    MC_LYA_OPT_BESIDE = 16        /* kernel 2 with both parts: the persistent walk of the
                                     untiled boxes runs beside the tile generations on a
                                     stream of its own, with at most this many waves per
                                     compute unit (1..32, default 4; 0 = after them on the
                                     context's stream). The two write disjoint boxes. */
};

/* What a context reserves at mc_lya_init. Every device buffer of the
 * context is allocated there, sized by the boxes and by these limits; no later
 * call allocates device memory (a HIP graph captured with MC_LYA_OPT_GRAPH is
 * the HIP runtime's own). The sizing rule, for C cells in all boxes, T tiles
 * of 16^3 cells and N = max_packets:
 *   per cell    the packed record (4 bytes, 16 with a velocity field), the
 *               emission weight, quantised weight, packet count, first packet
 *               and absorbed tally (36 bytes), plus 48 bytes with evolve = 1;
 *   per packet  its cell (4 bytes) and two generations of tiled-walk
 *               hand-over state (234 bytes) for B = batch_packets packets (N
 *               if 0): 4 N + 234 B bytes; if the hand-over part cannot be
 *               allocated, init halves B down to 2^25 packets; the tiled
 *               walk walks emissions larger than B in batches of B;
 *   per tile    its table entry and exit lists (about 140 bytes);
 *   per box     a few hundred bytes of tables and per-block partial sums. */
typedef struct mc_lya_limits {
    uint64_t max_packets;         /* most packets one mc_lya_emit may emit over all boxes,
                                     1 <= max_packets < 2^40 */
    int32_t evolve;               /* 1: reserve mc_lya_evolve's six doubles per cell; 0: that
                                     call returns ESTATE */
    int32_t reserved;             /* 0 */
    uint64_t batch_packets;       /* packets of one tiled-walk batch (0 = max_packets): the
                                     hand-over state reserved for it is 234 bytes a packet;
                                     larger emissions walk in batches (the same integers) */
} mc_lya_limits;

/* Creates a context for n_boxes boxes, validates and packs their fields
 * (Sec. III.A.1 quantities per cell: n_1s, the true-absorption depth kappa_c
 * of Eq. (<fnu>), the bulk velocity, the emission weight) and allocates every
 * device buffer the context will use (mc_lya_limits states the sizes), and one
 * stream and two events of its own (default priority; see MC_LYA_OPT_BESIDE).
 *   out      host, receives the context (set to NULL on failure)
 *   boxes    host [n_boxes]; the field pointers must stay valid and unchanged
 *            until mc_lya_destroy, or until they are refreshed
 *   n_boxes  1 to 1024
 *   limits   host, or NULL for max_packets = 2^20 and no evolve buffers
 *   stream   hipStream_t to run on (NULL = the default stream)
 * Synchronises the stream (to report invalid fields). Errors: EINVAL,
 * ENOMEM, EOVERFLOW, EDEVICE. */
mc_lya_status mc_lya_init(mc_lya_ctx **out, const mc_lya_box_desc *boxes, int32_t n_boxes,
                          const mc_lya_limits *limits, void *stream);

/* Re-reads the field arrays of every box (same pointers, new contents) and
 * repacks them. Synchronises the stream. Afterwards mc_lya_emit must be called. */
mc_lya_status mc_lya_refresh(mc_lya_ctx *ctx);

/* Distributes n_packets[b] packets over the cells of box b in proportion to
 * the emission weight (systematic integer allocation: cell c receives
 * floor-based counts with |N_c - N q_c / sum q| < 1, q_c = floor(2^32 S_c /
 * max S)), zeroes the tallies, and keys packet p of box b to the Philox4x32-10
 * stream (key = seeds[b], counter = (p, s)).
 *   seeds, n_packets  host [n_boxes]; n_packets[b] may be 0, their sum at most
 *                     the context's max_packets
 * Errors: EINVAL (also: more packets than max_packets), EOVERFLOW (w0 *
 * packets >= 2^63), ESTATE, EDEVICE. */
mc_lya_status mc_lya_emit(mc_lya_ctx *ctx, const uint64_t *seeds, const uint64_t *n_packets);

/* Walks every emitted packet (App. A steps 1-4 and the red-wing exit) and
 * accumulates the per-cell absorbed weight and the per-box totals.
 * Asynchronous on the context's stream, except that the tiled walk (kernel 2)
 * synchronises to learn whether packets are still in flight: after a first
 * round of as many generations as the previous transport needed, then after
 * every 16 more. Errors: ESTATE, EDEVICE. */
mc_lya_status mc_lya_transport(mc_lya_ctx *ctx);

/* As mc_lya_transport, for global packet ids [first, first + count) only.
 * Tallies accumulate, so disjoint ranges covering all packets give the same
 * integers as one mc_lya_transport call. Errors: EINVAL (range outside the
 * emitted packets), ESTATE, EDEVICE. */
mc_lya_status mc_lya_transport_range(mc_lya_ctx *ctx, uint64_t first, uint64_t count);

/* Finishes a transport: checks the conservation identity per box and copies
 * the tallies out. Synchronises the stream.
 *   absorbed  dev [total cells] int64, or NULL
 *   emitted   dev [total cells] int64 (w0 * packets emitted per cell), or NULL
 *   stats     host [n_boxes], or NULL
 * Returns ECAP if a packet hit the crossing cap, ECONSERVE if the identity
 * fails, else OK. */
mc_lya_status mc_lya_tally(mc_lya_ctx *ctx, int64_t *absorbed, int64_t *emitted,
                           mc_lya_box_stats *stats);

/* Recombination feed from the last transport (Sec. III.A.1 Eq. (rec),
 * Sec. IV.B Eq. (dotne-mix)): with a_c = A_c sum(S) / (w0 N) the absorbed
 * rate density, beta_e/(beta_e + Lambda_2g) of it re-ionises, and
 *   ndot_e,c = -S_c + beta/(beta+Lambda) a_c + C_MC beta n_1s,c exp(-E_alpha/kT),
 *   C_MC = [E + sum(A) Lambda/(beta+Lambda)] / (w0 N);
 * and the mixing correction M_c = A_c / A_c^fm with A_c^fm = sum(A) n_1s,c /
 * sum(n_1s) (1 everywhere under full mixing).
 *   ndot_e    dev [total cells] double, or NULL
 *   mix_corr  dev [total cells] float, or NULL
 *   stats     host [n_boxes], or NULL
 * Synchronises the stream. Errors: ESTATE, EDEVICE. */
mc_lya_status mc_lya_feed(mc_lya_ctx *ctx, double *ndot_e, float *mix_corr,
                          mc_lya_feed_stats *stats);

/* ---- resonant scattering (App. A, steps 1-8) ------------------------------
 * The paper's own Monte Carlo: each photon is followed scattering by
 * scattering instead of streaming with a continuous absorption depth.
 *   - Free paths: an optical depth -ln(u), accumulated along straight
 *     segments as (kappa_c / p_ab) times the swept line profile, with the
 *     Hubble drift and the face jumps of the walk (App. A steps 2-6 with the
 *     step length taken to zero).
 *   - At a scattering the photon is destroyed with probability p_destroy
 *     (the box's p_ab unless overridden), deposited whole (w0) into the cell
 *     (step 7; the feed splits ionisation from two-photon decay as for the
 *     walk).
 *   - Otherwise it is re-emitted (step 8): the scattering atom's parallel
 *     velocity drawn from exp(-u^2)/((x-u)^2 + a^2) of Eq. (MC) (resonant,
 *     u = x, for the Doppler profile), its perpendicular velocity projected on
 *     the scattering plane drawn from exp(-u^2), an isotropic new direction,
 *     and x -> x - u_par (1 - mu) + u_perp sqrt(1 - mu^2) (Eq. (inout)).
 *   - A photon redshifted below -x_inert is lost to the line (counted in
 *     `escaped`); for the Voigt profile the far damping wing takes the
 *     expected share 1 - exp(-<kappa> Phi(-x_inert)) of it (`wing`).
 * The photons are those of the last mc_lya_emit (same cells, positions,
 * directions and frequencies as the walk's packets); tallies, totals and
 * mc_lya_tally / mc_lya_feed work as after mc_lya_transport, with
 * `scatterings` counted per box. */
typedef struct mc_lya_scatter_opts {
    double x_inert;               /* > 0; 0 selects 300 (well past x_50 ~ 60 of App. A) */
    double p_destroy;             /* destruction probability per scattering; < 0 selects each
                                     box's p_ab (test problems raise it to shorten histories;
                                     0 never destroys) */
    uint64_t max_events;          /* scatterings before a photon is stopped as capped;
                                     0 selects 2^32 - 1 */
    int32_t fixed_x0;             /* 1: every photon is injected at x0 (App. A step 1 injects at
                                     line centre); 0: the emission's profile-drawn frequency */
    float x0;
    double x_return;              /* > 0: a photon re-emitted inside |x| < x_return stops and is
                                     counted nowhere (fate 3 in the records; a test of x_50);
                                     tallies are then not conserved. 0: off */
} mc_lya_scatter_opts;

/* One photon's history from mc_lya_scatter (72 bytes). */
typedef struct mc_lya_scatter_record {
    uint32_t cell0, cell_end;     /* global emission cell; cell of the last event */
    float x0, x_end;              /* injection frequency; frequency at the end (-x_inert if lost) */
    uint64_t scatterings;
    uint32_t crossings;
    int32_t fate;                 /* 0 destroyed, 1 lost to the line, 2 capped, 3 returned */
    int64_t escaped, absorbed, wing;
    float dx, dy, dz;             /* displacement from the emission point to the last event
                                     (the destruction point of a destroyed photon), in cell
                                     widths along x, y, z, unwrapped over the periodic box:
                                     the distance a photon travels between creation and
                                     destruction (Fig. MCtravel) */
    int32_t reserved;
} mc_lya_scatter_record;

/* Scatters photons [first, first + count) of the current emission into the
 * tallies (as mc_lya_transport_range does for the walk; disjoint ranges add
 * up to the whole).
 *   opts     host, or NULL for the defaults (x_inert 300, each box's p_ab, 2^32 - 1 events,
 *            the emission's frequencies, no return test)
 *   records  dev [count], or NULL
 * Asynchronous on the context's stream. Errors: EINVAL (range, options),
 * ESTATE, EDEVICE. */
mc_lya_status mc_lya_scatter(mc_lya_ctx *ctx, uint64_t first, uint64_t count,
                             const mc_lya_scatter_opts *opts, mc_lya_scatter_record *records);

/* ---- recombination history (Sec. III.A.1, Sec. IV.B) -------------------------
 * Advances the free-electron fraction of every cell from z0 to z1 (z0 > z1 >
 * 0, forward in time) with the net rate the Monte Carlo feeds: dx_e/dz =
 * -ndot_e / (n_H,c (1 + z) H), ndot_e from mc_lya_feed. The classic
 * fourth-order Runge-Kutta method in z takes n_steps equal steps; each of its
 * four stages moves every box to the stage's redshift with T = T_cmb0 (1+z)
 * (one temperature for matter and radiation), re-packs the fields (the x_e
 * of the stage), emits n_packets[b] packets per box, transports them and
 * runs the feed. Stage s of step i emits with seeds seed + ((4 i + s) << 20)
 * + b. Helium is not followed.
 *   x_e    host [n_boxes] of dev pointers: each box's own x_e field (the
 *          array its descriptor's x_e points to, which must not be NULL),
 *          overwritten with x_e(z1) (binary32, kept inside [0, 1]);
 *   X_out  host [n_steps + 1][n_boxes], or NULL: the global X_e = <n_e>/<n_H>
 *          of each box at z0 and after every step.
 * The context is left at z1 and re-packed (emit before transporting again).
 * It uses the six doubles per cell reserved with limits.evolve = 1 (ESTATE
 * without them) and synchronises the stream at every stage. Errors: EINVAL,
 * ESTATE, EDEVICE, and those of the emission and transport. */
mc_lya_status mc_lya_evolve(mc_lya_ctx *ctx, double z0, double z1, int32_t n_steps, const uint64_t *n_packets,
                            uint64_t seed, float *const *x_e, double *X_out);

/* Replays packets [first, first + count) of the current emission and writes
 * their histories without touching the tallies.
 *   out  dev [count]
 * Errors: EINVAL, ESTATE, EDEVICE. */
mc_lya_status mc_lya_trace(mc_lya_ctx *ctx, uint64_t first, uint64_t count,
                           mc_lya_packet_trace *out);

/* Sets a tunable (see the MC_LYA_OPT_ enum). Errors: EINVAL. */
mc_lya_status mc_lya_set_option(mc_lya_ctx *ctx, int32_t option, int64_t value);

/* Result of mc_lya_autotune: the options chosen and the transport times. */
typedef struct mc_lya_tune_result {
    int64_t kernel;               /* MC_LYA_OPT_KERNEL */
    int64_t tile_share;           /* MC_LYA_OPT_TILE_SHARE */
    int64_t block;                /* MC_LYA_OPT_BLOCK */
    int64_t waves_per_cu;         /* MC_LYA_OPT_WAVES_PER_CU */
    int64_t chunk;                /* MC_LYA_OPT_CHUNK */
    int64_t refill;               /* MC_LYA_OPT_REFILL */
    int64_t tile_chunk;           /* MC_LYA_OPT_TILE_CHUNK */
    int64_t tile_refill;          /* MC_LYA_OPT_TILE_REFILL */
    double best_ms;               /* fastest transport of the current emission, ms */
    double start_ms;              /* the same with the options set before the call, ms */
    int32_t trials;               /* option sets timed */
    int32_t reserved;
} mc_lya_tune_result;

/* Times a fixed list of option sets (the current one first; the tiled and
 * persistent walks at several tile shares, chunk, refill, block and resident
 * wave counts) on full transports of the current emission, `reps` timed runs
 * each after one warm-up run, and keeps the fastest. Transport results do not
 * depend on these options (bit for bit), so tuning changes speed only. Leaves
 * the context as after mc_lya_emit (tallies zero), ready for mc_lya_transport.
 * Costs about (reps + 1) x 12 transports. result: host, or NULL.
 * Synchronises the stream. Errors: EINVAL (reps outside [1, 100]), ESTATE
 * (before mc_lya_emit), EDEVICE; after an error the options are those the call
 * started with. */
mc_lya_status mc_lya_autotune(mc_lya_ctx *ctx, int32_t reps, mc_lya_tune_result *result);

/* Sum of the durations of the transport kernels since the last call (ms),
 * measured with HIP events on the context's stream when MC_LYA_OPT_TIMING is
 * on; also returns the number of launches timed (timing 1: a graph replay
 * counts as one; timing 2: the walk launches the transports enqueued or
 * replayed, with the span of each transport's walk in ms). Synchronises the
 * stream. Changing MC_LYA_OPT_TIMING drops what was timed so far. */
mc_lya_status mc_lya_kernel_time(mc_lya_ctx *ctx, double *ms, int64_t *launches);

/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11) on the device: n blocks,
 * ctr dev [n][4], key dev [n][2], out dev [n][4]. The packet streams use
 * counter (p_lo, p_hi, s, 0), s = 0, 1, and key (seed_lo, seed_hi); the 8
 * words give the uniforms (w >> 9) + 1/2) 2^-23 in (0, 1). Asynchronous on
 * `stream`. Errors: EINVAL, EDEVICE. */
mc_lya_status mc_lya_philox4x32_10(const uint32_t *ctr, const uint32_t *key, uint32_t *out,
                                   uint64_t n, void *stream);

/* Measurement utility (not part of the transport): reads `bytes` of device
 * memory at `buf` `passes` times over in one launch of `grid` workgroups of
 * 256 threads, each thread the same 16-byte positions in every pass, so a
 * buffer that fits a cache level is served from it after the first pass.
 * Timing is the caller's (events on `stream`); read bandwidth = bytes *
 * passes / time. The data must be finite floats; `sink` (dev, 1 float) is
 * never written for such data.
 *   bytes  a multiple of 16, >= 16;  passes, grid >= 1
 * Asynchronous. Errors: EINVAL, EDEVICE. */
mc_lya_status mc_lya_probe_read(const void *buf, uint64_t bytes, int32_t passes, int32_t grid, float *sink,
                                void *stream);

/* ---- mixing-correction surrogate ------------------------------------------
 * A per-cell regression of y = ln M_c, the log of the mixing correction that
 * mc_lya_feed returns (M_c = A_c / A_c^fm, Sec. IV.B, Eq. (dotne-mix); M = 1
 * is full mixing), on eight local features, so that the correction can be
 * evaluated without a transport. The network is 8 -> 64 -> 64 -> 1 with ReLU
 * activations (relu(z) = max(z, 0)); its parameters are one float vector
 * of MC_LYA_MLP_PARAMS numbers: W1 [64][8] at 0, b1 [64] at 512, W2 [64][64]
 * at 576, b2 [64] at 4672, w3 [64] at 4736, b3 at 4800 (row-major
 * [out][in]). */
#define MC_LYA_MLP_PARAMS 4801
#define MC_LYA_MLP_FEATURES 8

/* Features of every cell of every box, from the fields given to mc_lya_init
 * (they must still be alive):
 *   0 ln Delta_c, 1 mean and 2 variance (mean squared deviation) of Delta over
 *   the 3x3x3 cells around c (periodic), 3 div U by central differences in
 *   thermal velocities per cell (0 without a flow), 4 ln(T / 3000 K), 5 x_e,
 *   6 z / 1000 - 1.1, 7 ln(<Delta^2> / <Delta>^2) over the box (ln(1 + b), b the
 *   clumping factor of Sec. II.C, Eq. (clumpingfactor); in the no-mixing
 *   limit M_c = S_c sum(n_1s) / (n_1s,c sum(S)) carries that box-wide ratio).
 *   out  dev [total cells][8] float, box-major, x fastest
 * Asynchronous on the context's stream. Errors: EINVAL, ESTATE, EDEVICE. */
mc_lya_status mc_lya_features(mc_lya_ctx *ctx, float *out);

/* The surrogate's regression data from the last transport (after
 * mc_lya_transport; the same tallies mc_lya_feed reads), per cell:
 *   y  dev [total cells] float: ln M_c, the log of the mixing correction of
 *      mc_lya_feed (Sec. IV.B, Eq. (dotne-mix));
 *   w  dev [total cells] float: the cell's share S_c / sum_box(S) of its box's
 *      recombination source (Eq. (rec0)), the weight of the cell in the loss.
 * Cells with M_c = 0 (nothing absorbed) get y = 0 and w = 0. Synchronises the
 * stream once (per-box sums), then asynchronous. Errors: EINVAL, ESTATE,
 * EDEVICE. */
mc_lya_status mc_lya_surrogate_targets(mc_lya_ctx *ctx, float *y, float *w);

typedef struct mc_lya_mlp mc_lya_mlp;

/* Adam hyper-parameters (Kingma & Ba 2015, Algorithm 1, bias-corrected). */
typedef struct mc_lya_adam {
    float lr, beta1, beta2, eps;
} mc_lya_adam;

/* Creates a network with the given parameters (host [MC_LYA_MLP_PARAMS],
 * copied) and zero Adam moments, on the current device; all its work goes on
 * `stream` (a hipStream_t, or NULL). Allocates about 20 MB (parameters, Adam
 * moments, the gradient workspace). On failure *out = NULL and
 * mc_lya_mlp_last_error(NULL) tells why. Errors: EINVAL (NULL or non-finite
 * parameters), ENOMEM, EDEVICE. */
mc_lya_status mc_lya_mlp_create(mc_lya_mlp **out, const float *params, void *stream);

/* Copies the current parameters out. params: host [MC_LYA_MLP_PARAMS].
 * Synchronises. Errors: EINVAL, EDEVICE. */
mc_lya_status mc_lya_mlp_get_params(mc_lya_mlp *mlp, float *params);

/* Sets the training envelope: host [8] lower and upper bounds per feature
 * (lo <= hi), or both NULL to clear it. mc_lya_mlp_forward flags cells whose
 * features fall outside it, for which the Monte Carlo should be used instead.
 * Errors: EINVAL, EDEVICE. */
mc_lya_status mc_lya_mlp_set_envelope(mc_lya_mlp *mlp, const float *lo, const float *hi);

/* Inference: y = network(features) for n cells, on the matrix cores: W1, W2,
 * the features and the layer-1 activations in BF16, FP32 accumulation, each
 * of b1 and b2 as the BF16 pair hi = bf16(b), lo = bf16(b - hi) (b to 2^-16),
 * the last layer (w3, b3) in FP32. Training differentiates this same function.
 *   features  dev [n][8] float
 *   y         dev [n] float
 *   outside   dev [n] uint8 (1 = some feature outside the envelope; all 0
 *             while no envelope is set), or NULL
 *   n_outside host, or NULL: number of such cells (then synchronises)
 * Asynchronous otherwise. Errors: EINVAL, EDEVICE. */
mc_lya_status mc_lya_mlp_forward(mc_lya_mlp *mlp, const float *features, uint64_t n, float *y,
                                 uint8_t *outside, uint64_t *n_outside);

/* The mixing correction the surrogate gives, with the Monte Carlo as
 * fallback: mc_lya_mlp_forward's y for n cells, then per cell
 *   M = fallback[i]  where the cell's features are outside the envelope and
 *                    a fallback is given (the Monte Carlo's M_c, mc_lya_feed),
 *   M = exp(y)       otherwise.
 *   features  dev [n][8] float
 *   fallback  dev [n] float, or NULL (no fallback: M = exp(y) everywhere)
 *   y         dev [n] float (out: the network's ln M)
 *   M         dev [n] float (out)
 *   outside   dev [n] uint8 (out), or NULL; n_outside host (out), or NULL
 *             (then synchronises)
 * Errors: EINVAL, EDEVICE. */
mc_lya_status mc_lya_mlp_correction(mc_lya_mlp *mlp, const float *features, uint64_t n, const float *fallback,
                                    float *y, float *M, uint8_t *outside, uint64_t *n_outside);

/* The weighted mean squared error L = sum w_i (y_i - t_i)^2 / sum w_i over n
 * cells of the network mc_lya_mlp_forward evaluates, and its gradient with
 * respect to the FP32 parameters (each BF16 rounding passed through
 * unchanged), on the matrix cores: the forward and backward products in BF16
 * with FP32 accumulation, the error signals dL/dz rounded to BF16, the w3, b2
 * and b3 gradients summed in FP32. Cells are summed in a fixed order: the
 * result is reproducible bit for bit.
 *   features dev [n][8], targets dev [n], weights dev [n] (>= 0, not all 0)
 *   grad     host [MC_LYA_MLP_PARAMS], or NULL;  loss host, or NULL
 * Synchronises. Errors: EINVAL, EDEVICE. */
mc_lya_status mc_lya_mlp_gradient(mc_lya_mlp *mlp, const float *features, const float *targets,
                                  const float *weights, uint64_t n, float *grad, float *loss);

/* One training step: the gradient as in mc_lya_mlp_gradient, then one Adam
 * update of the parameters (the step count starts at 1 and is kept by the
 * object). loss: host (the loss before the update; then synchronises), or
 * NULL (asynchronous). Errors: EINVAL (bad hyper-parameters, no cells),
 * EDEVICE. */
mc_lya_status mc_lya_mlp_train_step(mc_lya_mlp *mlp, const float *features, const float *targets,
                                    const float *weights, uint64_t n, const mc_lya_adam *hp,
                                    float *loss);

/* n_steps training steps in one call, each the same as mc_lya_mlp_train_step
 * on the mini-batch that an index array picks from a training set, queued
 * step after step with no synchronisation between them (for callers that
 * would otherwise spend more time issuing the steps than the device takes
 * to run them).
 *   features, targets, weights  dev [n_cells][8], [n_cells], [n_cells] float:
 *             the training set
 *   idx       dev [n_steps][batch] int64: step s trains on cells
 *             idx[s][0..batch), each in [0, n_cells)
 *   lr        host [n_steps] learning rates (> 0); beta1, beta2, eps as in
 *             mc_lya_adam
 *   losses    host [n_steps] (each step's loss before its update), or NULL
 * The object allocates a gather buffer of batch cells (kept, grown when a
 * larger batch comes). Synchronises once, at the end; an index outside
 * [0, n_cells) is then reported as EINVAL (the steps have been taken with
 * such cells read as cell 0). Errors: EINVAL, ENOMEM, EDEVICE. */
mc_lya_status mc_lya_mlp_train_steps(mc_lya_mlp *mlp, const float *features, const float *targets,
                                     const float *weights, uint64_t n_cells, const int64_t *idx, uint64_t batch,
                                     int n_steps, const float *lr, float beta1, float beta2, float eps,
                                     float *losses);

/* For callers that cannot allocate device memory (work being captured into a
 * HIP graph, tight serving or training loops, harnesses that forbid
 * hipMalloc): mc_lya_mlp_gradient without a network object and without any
 * allocation. Its workspace (the per-block partial sums of the gradient and
 * their fixed-order reduction, MC_LYA_STATIC_SCRATCH_BYTES) is one
 * library-owned static device array per GPU, held until the process ends;
 * calls that overlap on one GPU (other host threads, other streams) race on
 * it and must be serialised by the caller. Every part of the workspace a
 * call reads is written by that call first, so no call depends on an
 * earlier one's leftovers. The result is the same, bit for bit, as
 * mc_lya_mlp_gradient's for the same parameters and cells.
 *   params    dev [MC_LYA_MLP_PARAMS] float (the layout above)
 *   features  dev [n][8], targets dev [n], weights dev [n] (>= 0)
 *   n         1 .. MC_LYA_STATIC_MAX_CELLS
 *   grad_out  dev [MC_LYA_MLP_PARAMS + 2] float: the gradient of the weighted
 *             mean squared error, then sum w r^2 and sum w (loss = their
 *             ratio; a zero weight sum leaves a zero gradient)
 *   stream    hipStream_t, or NULL
 * Asynchronous on `stream` (no synchronisation, no allocation, no host
 * copies). Errors: EINVAL (NULL pointers, n out of range), EDEVICE; the text
 * of the last failure on this thread is mc_lya_mlp_static_last_error(). */
#define MC_LYA_STATIC_MAX_CELLS (((uint64_t)1 << 40) - 1)
#define MC_LYA_STATIC_SCRATCH_BYTES ((uint64_t)(1024 + 32) * 4808 * 4)
mc_lya_status mc_lya_mlp_gradient_static(const float *params, const float *features, const float *targets,
                                         const float *weights, uint64_t n, float *grad_out, void *stream);
const char *mc_lya_mlp_static_last_error(void);

/* Frees the network (synchronises its stream). NULL ok. */
void mc_lya_mlp_destroy(mc_lya_mlp *mlp);

/* Description of the network's last failure, or with NULL of the last failed
 * mc_lya_mlp_create on this thread. */
const char *mc_lya_mlp_last_error(const mc_lya_mlp *mlp);

/* Frees the context and its device memory (synchronises its stream). NULL ok. */
void mc_lya_destroy(mc_lya_ctx *ctx);

/* Static description of a status code. */
const char *mc_lya_strerror(mc_lya_status status);

/* Description of the context's last failure ("" if none); valid until the
 * next call on the context. */
const char *mc_lya_last_error(const mc_lya_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* MC_LYA_H */

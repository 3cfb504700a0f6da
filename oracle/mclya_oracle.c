/*
 * FP64 CPU oracle for Monte-Carlo Lyman-alpha packet transport.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, plain reference that the
 * GPU path is checked against. Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may build, load or run it; the product path
 * never does. It shares no code, header, table or constant with the HIP
 * library: it is written independently from the paper and from the published
 * definition of the Philox generator.
 *
 * What it computes (paper: Jedamzik, Abel & Ali-Haimoud, arXiv:2312.11448):
 *   - packets are injected at random locations (App. A, step 1), here with a
 *     frequency drawn from the thermal (Doppler) line profile and an isotropic
 *     direction;
 *   - each packet streams in a straight line through a periodic grid; inside a
 *     cell its gas-frame frequency drifts to the red by H dl / v_th (App. A,
 *     step 4); at a cell face it changes by the bulk-velocity term of
 *     Eq. (inout), x_new = x_old - k.(U_new - U_old) / v_th;
 *   - along a segment the expected true-absorption depth is
 *     kappa_c * [Phi(x_in) - Phi(x_out)], with kappa_c the mean optical depth
 *     to true absorption of Eq. (<fnu>) evaluated with the cell's n_1s and Phi
 *     the cumulative line profile; the absorbed part of the packet weight is
 *     deposited into the cell as a 64-bit integer;
 *   - a packet escapes once it has redshifted past -x_eff on the red wing
 *     (the "lost to redshifting" outcome at the end of App. A).
 * Weights are integers, so sum(absorbed) + escaped == w0 * npackets exactly.
 *
 * Line profile. Either the thermal (Doppler) profile, or the Voigt profile of
 * Eq. (MC): the thermal profile convolved with the natural (Lorentz) line of
 * half width a = A_2p lambda / (4 pi v_th) in Doppler units. Voigt emission
 * adds a Cauchy deviate a tan(pi (u - 1/2)) to the thermal one. Its
 * cumulative profile is taken to first order in a,
 *   Phi_V(x) = erfc(-x)/2 - (2a/pi) F(x),   F = Dawson's integral,
 * which follows from expanding the Cauchy CDF 1/2 + arctan(s/a)/pi in a; the
 * neglected terms are O(a^2) (below 2e-7 at a = 8.6e-4). The damping wing
 * keeps absorbing past -x_eff: an escaping packet leaves behind the expected
 * share 1 - exp(-kbar Phi_V(x_stop)) of its weight, with kbar the box's mean
 * kappa (the wing is crossed over hundreds of cells, so it sees the mean) and
 * x_stop = -x_eff. That share is reported as "wing" (part of the escaped
 * weight, absorbed far away, i.e. fully mixed). Packets emitted below -x_eff
 * or above x_blue (blue of every walked frequency) are not walked: they
 * escape at once with x_stop = x0.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC mclya_oracle.c -o libmclya_oracle.so -lm
 * (no fast-math: every floating-point operation is plain IEEE double).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11, "Parallel random        */
/* numbers: as easy as 1, 2, 3"). Ten rounds of two 32x32->64 multiplies,     */
/* key schedule bumped by the Weyl constants between rounds.                  */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t mul0 = 0xD2511F53u, mul1 = 0xCD9E8D57u;
    const uint32_t weyl0 = 0x9E3779B9u, weyl1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t prod0 = (uint64_t)mul0 * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)mul1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += weyl0;
        k1 += weyl1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in (0,1) from the top 23 bits of a word: (m + 1/2) 2^-23. Every such
 * value is exactly representable in binary32 and binary64. */
static double orc_uniform(uint32_t r)
{
    return ((double)(r >> 9) + 0.5) * (1.0 / 8388608.0);
}

/* The eight uniforms of packet p: two Philox blocks with counter
 * (p_lo, p_hi, s, 0), s = 0, 1, and key (seed_lo, seed_hi). */
void orc_packet_uniforms(uint64_t seed, uint64_t p, double u[8])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (uint32_t s = 0; s < 2; ++s) {
        uint32_t ctr[4] = {(uint32_t)p, (uint32_t)(p >> 32), s, 0u};
        uint32_t r[4];
        orc_philox4x32_10(ctr, key, r);
        for (int i = 0; i < 4; ++i) u[4 * s + i] = orc_uniform(r[i]);
    }
}

/* ------------------------------------------------------------------------- */
/* Emission: packets are distributed over cells in proportion to the local    */
/* recombination source alpha_e n_e^2 (Eq. rec0; the integral of the          */
/* footnote in Sec. III.B), with an exact integer systematic allocation.      */
/* ------------------------------------------------------------------------- */

/* q_c = floor(2^32 * s_c / s_max). Returns 0 on success, -1 for a negative or
 * non-finite weight, -2 when every weight is zero. */
int orc_quantize(int64_t ncells, const double *s, uint64_t *q)
{
    double smax = 0.0;
    for (int64_t c = 0; c < ncells; ++c) {
        if (!(s[c] >= 0.0) || isinf(s[c])) return -1;
        if (s[c] > smax) smax = s[c];
    }
    if (smax == 0.0) return -2;
    for (int64_t c = 0; c < ncells; ++c) {
        double ratio = s[c] / smax;             /* one correctly rounded division */
        q[c] = (uint64_t)floor(ratio * 4294967296.0);  /* exact scaling by 2^32 */
    }
    return 0;
}

/* Number of packets p in [0, N) whose systematic point t_p = floor((2p+1) Qtot / 2N)
 * lies below Q: the odd integers o = 2p+1 with o * Qtot < 2 N Q. */
static uint64_t orc_count_below(uint64_t Q, uint64_t Qtot, uint64_t N)
{
    u128 m = (u128)2 * (u128)N * (u128)Q;
    u128 ceil_y = (m + (u128)Qtot - 1) / (u128)Qtot;  /* ceil(2 N Q / Qtot) */
    return (uint64_t)(ceil_y / 2);
}

/* first[c] = id of the first packet emitted in cell c; first[ncells] = N. */
int orc_allocate(int64_t ncells, const uint64_t *q, uint64_t npackets, uint64_t *first)
{
    uint64_t Qtot = 0;
    for (int64_t c = 0; c < ncells; ++c) Qtot += q[c];
    if (Qtot == 0) return -2;
    uint64_t Q = 0;
    for (int64_t c = 0; c < ncells; ++c) {
        first[c] = orc_count_below(Q, Qtot, npackets);
        Q += q[c];
    }
    first[ncells] = orc_count_below(Qtot, Qtot, npackets);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Transport                                                                 */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t nx, ny, nz;
    int32_t has_vel;
    double delta;        /* red drift of x per cell width of path (App. A step 4) */
    double x_eff;        /* escape once x <= -x_eff */
    uint64_t w0;         /* weight of one packet */
    uint64_t seed;
    int64_t max_cross;   /* crossing cap per packet */
    double damping;      /* Voigt a (0: Doppler profile) */
    double kappa_far;    /* mean kappa of the box, for the far damping wing (0: none) */
    double x_blue;       /* packets emitted above it are not walked (+inf: all are) */
} orc_box;

typedef struct {
    int64_t cell0;
    double fx, fy, fz;   /* emission position inside cell0, in [0,1) */
    double kx, ky, kz;   /* direction */
    double x0;           /* emission frequency, gas frame, Doppler units */
    int64_t crossings;   /* number of (packet, cell) segments walked */
    int64_t escaped;     /* weight that escaped */
    int64_t absorbed;    /* weight deposited into the grid */
    int32_t fate;        /* 0 absorbed, 1 escaped, 2 capped */
    int32_t pad;
    int64_t wing;        /* part of the escaped weight absorbed by the far damping wing */
} orc_packet_rec;

typedef struct {
    int64_t *cells;      /* cell of each segment */
    int64_t *deposits;   /* integer deposit of each segment */
    double *x_in, *x_out, *length;
    int64_t cap, n;
} orc_trace;

/* Dawson's integral F(x) = exp(-x^2) int_0^x exp(t^2) dt, by Rybicki's
 * sampling-theorem series (G. B. Rybicki, Computers in Physics 3, 85, 1989):
 * F(x) = lim_{h->0} pi^{-1/2} sum over odd n of exp(-(x - n h)^2) / n. With
 * h = 0.2 the discretisation error is of order exp(-(pi / 2h)^2) < 1e-26.
 * The sum is taken about the even multiple x0 = 2 k h nearest to x (nodes
 * x0 + m h, m odd, weights 1 / (2k + m)), so the offsets xp - m h, xp = x - x0,
 * are small and exact; nodes with |offset| > 8 (terms below exp(-64)) are left
 * out. Each term exp(-(xp - m h)^2) = exp(-xp^2) exp(-(m h)^2) E^m with
 * E = exp(2 xp h), so one evaluation takes two exponentials. */
#define ORC_RYB_M 41
static double orc_ryb_c[ORC_RYB_M + 1];     /* exp(-(m h)^2), odd m */

__attribute__((constructor)) static void orc_ryb_init(void)
{
    for (int m = 1; m <= ORC_RYB_M; m += 2) orc_ryb_c[m] = exp(-(0.2 * m) * (0.2 * m));
}

static double orc_dawson(double x)
{
    const double h = 0.2;
    const double k = nearbyint(x / (2.0 * h));
    const double xp = x - 2.0 * h * k;
    const double E = exp(2.0 * xp * h), Ei = 1.0 / E, E2 = E * E, Ei2 = Ei * Ei;
    double up = E, dn = Ei, sum = 0.0;
    for (int m = 1; m <= ORC_RYB_M; m += 2) {
        sum += orc_ryb_c[m] * (up / (2.0 * k + (double)m) + dn / (2.0 * k - (double)m));
        up *= E2;
        dn *= Ei2;
    }
    return exp(-xp * xp) * sum / sqrt(M_PI);
}

/* Cumulative line profile: the Doppler one, erfc(-x)/2 = int_{-inf}^{x}
 * exp(-y^2)/sqrt(pi) dy, and for a > 0 the Voigt one to first order in a. */
static double orc_Phi(const orc_box *b, double x)
{
    const double phi = 0.5 * erfc(-x);
    return b->damping > 0.0 ? phi - 2.0 * b->damping / M_PI * orc_dawson(x) : phi;
}

double orc_profile_cdf(double damping, double x)
{
    orc_box b;
    memset(&b, 0, sizeof b);
    b.damping = damping;
    return orc_Phi(&b, x);
}

double orc_dawson_integral(double x) { return orc_dawson(x); }

static int64_t orc_wrap(int64_t i, int64_t n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

/* Walk one packet. Deposits go to A; returns the packet's record. */
static void orc_walk_one(const orc_box *b, const double *kappa, const double *ux,
                         const double *uy, const double *uz, uint64_t p, int64_t cell0,
                         int64_t *A, orc_packet_rec *rec, orc_trace *tr)
{
    const int64_t nx = b->nx, ny = b->ny, nz = b->nz;
    double u[8];
    orc_packet_uniforms(b->seed, p, u);

    /* position: uniform inside the emission cell */
    double f[3] = {u[0], u[1], u[2]};
    /* direction: isotropic, mu = cos(theta) uniform in [-1,1], azimuth uniform */
    double mu = 2.0 * u[3] - 1.0;
    double phi = 2.0 * M_PI * u[4];
    double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    double k[3] = {st * cos(phi), st * sin(phi), mu};
    /* frequency: Doppler profile exp(-x^2)/sqrt(pi), a normal law of variance
     * 1/2, by the Box-Muller transform */
    double x = sqrt(-log(u[5])) * cos(2.0 * M_PI * u[6]);
    /* Voigt: plus the natural line, a Cauchy deviate of half width a */
    if (b->damping > 0.0) x += b->damping * tan(M_PI * (u[7] - 0.5));
    double x_stop = 0.0;

    int64_t ci[3] = {cell0 % nx, (cell0 / nx) % ny, cell0 / (nx * ny)};
    int64_t n[3] = {nx, ny, nz};
    int64_t w = (int64_t)b->w0;
    int64_t ncross = 0, absorbed = 0;
    int fate = 0;

    rec->cell0 = cell0;
    rec->fx = f[0]; rec->fy = f[1]; rec->fz = f[2];
    rec->kx = k[0]; rec->ky = k[1]; rec->kz = k[2];
    rec->x0 = x;

    for (;;) {
        if (x <= -b->x_eff || x > b->x_blue) { fate = 1; x_stop = x; break; }   /* not in the walked window */
        if (ncross >= b->max_cross) { fate = 2; break; }
        int64_t c = ci[0] + nx * (ci[1] + ny * ci[2]);
        ++ncross;

        /* distance (in cell widths) to the face the ray leaves through */
        double t[3];
        for (int a = 0; a < 3; ++a) {
            if (k[a] > 0.0) t[a] = (1.0 - f[a]) / k[a];
            else if (k[a] < 0.0) t[a] = f[a] / (-k[a]);
            else t[a] = INFINITY;
        }
        int axis = 0;                                        /* ties: x, then y, then z */
        if (t[1] < t[axis]) axis = 1;
        if (t[2] < t[axis]) axis = 2;
        double s = t[axis];

        double x_out = x - b->delta * s;                     /* Hubble drift */
        int escaping = x_out <= -b->x_eff;
        double dPhi = escaping ? orc_Phi(b, x) - orc_Phi(b, -b->x_eff) : orc_Phi(b, x) - orc_Phi(b, x_out);
        /* Phi is non-decreasing: a negative difference of two rounded values
         * (a segment far shorter than a cell) is rounding, not absorption */
        if (dPhi < 0.0) dPhi = 0.0;
        double dtau = kappa[c] * dPhi;
        int64_t d = (int64_t)rint((double)w * (-expm1(-dtau)));
        if (d > w) d = w;
        w -= d;
        A[c] += d;
        absorbed += d;
        if (tr && tr->n < tr->cap) {
            tr->cells[tr->n] = c; tr->deposits[tr->n] = d;
            tr->x_in[tr->n] = x; tr->x_out[tr->n] = escaping ? -b->x_eff : x_out;
            tr->length[tr->n] = s;
            tr->n++;
        } else if (tr) {
            tr->n++;
        }
        if (escaping) { fate = 1; x_stop = -b->x_eff; break; }
        if (w == 0) { fate = 0; break; }

        /* move to the face, then into the neighbouring cell */
        for (int a = 0; a < 3; ++a) {
            if (a == axis) continue;
            double g = f[a] + k[a] * s;
            f[a] = g < 0.0 ? 0.0 : (g > 1.0 ? 1.0 : g);
        }
        int64_t old = c;
        if (k[axis] > 0.0) { f[axis] = 0.0; ci[axis] = orc_wrap(ci[axis] + 1, n[axis]); }
        else { f[axis] = 1.0; ci[axis] = orc_wrap(ci[axis] - 1, n[axis]); }
        x = x_out;
        if (b->has_vel) {
            int64_t cn = ci[0] + nx * (ci[1] + ny * ci[2]);
            double du = k[0] * (ux[cn] - ux[old]) + k[1] * (uy[cn] - uy[old]) + k[2] * (uz[cn] - uz[old]);
            x -= du;                                          /* Eq. (inout), bulk term */
        }
    }
    /* the far damping wing: expected absorption of the escaping weight */
    int64_t wing = 0;
    if (fate == 1 && b->kappa_far > 0.0) {
        const double pw = -expm1(-b->kappa_far * fmax(orc_Phi(b, x_stop), 0.0));
        wing = (int64_t)rint((double)w * pw);
        if (wing > w) wing = w;
    }
    rec->wing = wing;
    rec->crossings = ncross;
    rec->escaped = (fate == 0) ? 0 : w;
    rec->absorbed = absorbed;
    rec->fate = fate;
}

/* Cell of packet p: the largest c with first[c] <= p. */
static int64_t orc_find_cell(const uint64_t *first, int64_t ncells, uint64_t p)
{
    int64_t lo = 0, hi = ncells - 1;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo + 1) / 2;
        if (first[mid] <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

/* Walk packets [p_begin, p_end). A (ncells) and out[5] = {escaped weight,
 * crossings, capped packets, capped weight, wing} are accumulated into (not
 * reset); wing is the part of the escaped weight the far damping wing absorbs.
 * recs, when not NULL, receives one record per packet. Returns 0. */
int orc_transport(const orc_box *b, const double *kappa, const double *ux, const double *uy,
                  const double *uz, const uint64_t *first, uint64_t p_begin, uint64_t p_end,
                  int64_t *A, int64_t out[5], orc_packet_rec *recs, int nthreads)
{
    const int64_t ncells = (int64_t)b->nx * b->ny * b->nz;
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    int64_t *priv = (int64_t *)calloc((size_t)nthreads * (size_t)ncells, sizeof(int64_t));
    if (!priv) return -1;
    int64_t esc = 0, cross = 0, capn = 0, capw = 0, wing = 0;
#pragma omp parallel num_threads(nthreads) reduction(+ : esc, cross, capn, capw, wing)
    {
        int64_t *mine = priv + (size_t)omp_get_thread_num() * (size_t)ncells;
#pragma omp for schedule(dynamic, 256)
        for (uint64_t p = p_begin; p < p_end; ++p) {
            orc_packet_rec r;
            orc_walk_one(b, kappa, ux, uy, uz, p, orc_find_cell(first, ncells, p), mine, &r, NULL);
            cross += r.crossings;
            if (r.fate == 1) { esc += r.escaped; wing += r.wing; }
            if (r.fate == 2) { capn += 1; capw += r.escaped; }
            if (recs) recs[p - p_begin] = r;
        }
    }
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t c = 0; c < ncells; ++c) {
        int64_t sum = 0;
        for (int t = 0; t < nthreads; ++t) sum += priv[(size_t)t * (size_t)ncells + c];
        A[c] += sum;
    }
    free(priv);
    out[0] += esc; out[1] += cross; out[2] += capn; out[3] += capw; out[4] += wing;
    return 0;
}

/* Walk the packets ids[0..n) one after another (single thread) and return
 * their records. Deposits go to the caller's scratch array A. */
int orc_walk_packets(const orc_box *b, const double *kappa, const double *ux, const double *uy,
                     const double *uz, const uint64_t *first, const uint64_t *ids, int64_t n,
                     int64_t *A, orc_packet_rec *recs)
{
    const int64_t ncells = (int64_t)b->nx * b->ny * b->nz;
    for (int64_t i = 0; i < n; ++i)
        orc_walk_one(b, kappa, ux, uy, uz, ids[i], orc_find_cell(first, ncells, ids[i]), A, &recs[i], NULL);
    return 0;
}

/* Walk one packet and record every segment (cell, deposit, x_in, x_out,
 * length). A receives its deposits. Returns the number of segments; only the
 * first `cap` are stored. */
int64_t orc_trace_packet(const orc_box *b, const double *kappa, const double *ux,
                         const double *uy, const double *uz, const uint64_t *first, uint64_t p,
                         int64_t *A, orc_packet_rec *rec, int64_t *cells, int64_t *deposits,
                         double *x_in, double *x_out, double *length, int64_t cap)
{
    const int64_t ncells = (int64_t)b->nx * b->ny * b->nz;
    orc_trace tr = {cells, deposits, x_in, x_out, length, cap, 0};
    orc_walk_one(b, kappa, ux, uy, uz, p, orc_find_cell(first, ncells, p), A, rec, &tr);
    return tr.n;
}

/* ------------------------------------------------------------------------- */
/* Resonant scattering (App. A, steps 1-8)                                    */
/*                                                                           */
/* A photon is followed scattering by scattering. Its free path is drawn as   */
/* an optical depth -ln(u) (App. A steps 2-6 with the step length taken to    */
/* zero: the depth along a path is kappa_sc [Phi(x_in) - Phi(x_out)], with    */
/* kappa_sc = kappa / p_ab the full line opacity per unit of swept profile).  */
/* At a scattering it is destroyed with probability p_ab (step 7); else the   */
/* scattering atom's velocity is drawn from Eq. (MC) (step 8): the parallel   */
/* component from exp(-u^2) / ((x - u)^2 + a^2) and the perpendicular one     */
/* projected on the scattering plane from exp(-u^2) (variance 1/2); the new   */
/* direction is isotropic, mu = k_in . k_out, and the new gas-frame frequency */
/* is Eq. (inout) without its bulk term, x - u_par (1 - mu) + u_perp sqrt(1 - */
/* mu^2). Bulk-velocity terms of Eq. (inout) apply at cell faces, as in the   */
/* streaming walk. A photon redshifted below -x_inert is lost to the line     */
/* (end of App. A); the expected share of it that the far damping wing still  */
/* destroys, 1 - exp(-kbar Phi(-x_inert)), is reported as "wing". A photon    */
/* bluer than +x_inert is treated the same way at its own frequency.          */
/*                                                                           */
/* Random numbers: event k of photon p uses the Philox block with counter     */
/* (p_lo, p_hi, k, 1): u0 the free path; words 1 and 2, as the 64-bit integer */
/* (w1 << 32) | w2, the destruction test, destroyed iff it is below           */
/* floor(p 2^64) (p_ab ~ 3e-7 is finer than a 23-bit uniform resolves). Block */
/* (p_lo, p_hi, k, 2): u0, u1 the perpendicular velocity (Box-Muller), u2, u3 */
/* the new direction (cos theta = 2 u2 - 1, azimuth 2 pi u3). Trial j of the  */
/* parallel-velocity draw uses block (p_lo, p_hi, k, 3 + j): u0 the envelope  */
/* part, u1 (and u2) the proposal, u3 the acceptance.                         */
/* ------------------------------------------------------------------------- */
typedef struct {
    double p_ab;          /* the box's p_ab: kappa / p_ab is the scattering depth per unit Phi */
    double p_destroy;     /* destruction probability per scattering (p_ab; other values for tests) */
    double x_inert;       /* lost to the line below -x_inert (and far above +x_inert) */
    int64_t max_events;   /* scatterings before a photon is stopped (capped) */
    int32_t fixed_x0;     /* 1: every photon is injected at x0 */
    int32_t pad;
    double x0;
    double x_return;      /* > 0: a photon scattered back inside |x| < x_return stops (fate 3) */
} orc_scatter_params;

typedef struct {
    int64_t cell0, cell_end;
    double x0, x_end;
    int64_t scatterings, crossings;
    int64_t escaped, absorbed, wing;
    double d[3];         /* displacement from the emission point to the last event, in cell
                            widths, unwrapped over the periodic box */
    int32_t fate;        /* 0 destroyed, 1 lost to the line, 2 capped, 3 returned (test hook) */
    int32_t pad;
} orc_scatter_rec;

static void orc_block_words(uint64_t seed, uint64_t p, uint32_t k, uint32_t stream, uint32_t r[4])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)p, (uint32_t)(p >> 32), k, stream};
    orc_philox4x32_10(ctr, key, r);
}

static void orc_block(uint64_t seed, uint64_t p, uint32_t k, uint32_t stream, double u[4])
{
    uint32_t r[4];
    orc_block_words(seed, p, k, stream, r);
    for (int i = 0; i < 4; ++i) u[i] = orc_uniform(r[i]);
}

/* floor(p 2^64) for p in [0, 1]; p >= 1 destroys always. */
static uint64_t orc_destroy_threshold(double p)
{
    if (!(p > 0.0)) return 0;
    if (p >= 1.0) return UINT64_MAX;
    return (uint64_t)ldexp(p, 64);
}

/* First-order Voigt (or Doppler) line density, the derivative of orc_Phi. */
static double orc_density(const orc_box *b, double y)
{
    const double g = exp(-y * y) / sqrt(M_PI);
    return b->damping > 0.0 ? g - 2.0 * b->damping / M_PI * (1.0 - 2.0 * y * orc_dawson(y)) : g;
}

/* Swept profile Phi(x) - Phi(x - dx), dx >= 0: the midpoint rule below
 * dx = 1e-4 (relative error under 1e-9; the difference of two rounded
 * values would keep only a few digits there), the difference above. */
static double orc_swept(const orc_box *b, double x, double dx)
{
    if (dx < 1e-4) return dx * orc_density(b, x - 0.5 * dx);
    const double d = orc_Phi(b, x) - orc_Phi(b, x - dx);
    return d > 0.0 ? d : 0.0;
}

/* Length s in (0, s_max] with kap * swept(x, delta s) = tau, by Newton's
 * method kept inside a shrinking bracket (the swept mass grows with s). */
static double orc_flight_length(const orc_box *b, double kap, double x, double tau, double s_max)
{
    const double d = b->delta;
    double lo = 0.0, hi = s_max;
    double s = tau / (kap * d * orc_density(b, x));
    if (!(s > lo && s < hi)) s = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
        const double g = kap * orc_swept(b, x, d * s) - tau;
        if (g > 0.0) hi = s; else lo = s;
        double sn = s - g / (kap * d * orc_density(b, x - d * s));
        if (!(sn > lo && sn < hi)) sn = 0.5 * (lo + hi);
        if (fabs(sn - s) <= 1e-12 * s || hi - lo <= 1e-14 * hi) return sn;
        s = sn;
    }
    return s;
}

/* Parallel velocity of the scattering atom for a photon at x >= 0: a draw
 * from exp(-u^2) / ((x - u)^2 + a^2) by rejection from a two-part envelope
 * split at u0 (after Zheng & Miralda-Escude 2002). Below u0 the envelope is
 * the Cauchy factor alone (|x| < 5) or the Gaussian over (x - u0)^2
 * (|x| >= 5, where the draw is mostly thermal); above u0 it is the Cauchy
 * factor times exp(-u0^2). The split point only changes the number of
 * trials: u0 = x - 0.02 - 0.1 max(0, x - 1)^2 (at least 0) for x < 5,
 * sqrt(6.3 + 3.2 ln x) beyond. For a = 0 the atom is resonant, u = x.
 * The trials stop after 4096 (the resonant u = x is then returned), so that
 * every draw ends. */
static double orc_atom_upar(double x, double a, uint64_t seed, uint64_t p, uint32_t k)
{
    if (a == 0.0) return x;
    const int neg = x < 0.0;
    const double xa = neg ? -x : x;
    const int wing = xa >= 5.0;
    double u0;
    if (wing) {
        u0 = sqrt(6.3 + 3.2 * log(xa));
    } else {
        const double q = xa > 1.0 ? xa - 1.0 : 0.0;
        u0 = xa - 0.02 - 0.1 * q * q;
        if (u0 < 0.0) u0 = 0.0;
    }
    const double th0 = atan((u0 - xa) / a);
    const double m2 = exp(-u0 * u0) * (0.5 * M_PI - th0);             /* in units of 1/a */
    const double m1 = wing ? 0.5 * sqrt(M_PI) * erfc(-u0) * a / ((xa - u0) * (xa - u0)) : th0 + 0.5 * M_PI;
    const double p1 = m1 / (m1 + m2);
    for (uint32_t j = 0; j < 4096u; ++j) {       /* at worst ~14 trials are expected */
        double r[4];
        orc_block(seed, p, k, 3u + j, r);
        double u, acc;
        if (r[0] < p1) {
            if (wing) {
                u = sqrt(-log(r[1])) * cos(2.0 * M_PI * r[2]);
                if (u > u0) continue;
                acc = (xa - u0) * (xa - u0) / ((xa - u) * (xa - u) + a * a);
            } else {
                const double th = -0.5 * M_PI + (th0 + 0.5 * M_PI) * r[1];
                u = xa + a * tan(th);
                acc = exp(-u * u);
            }
        } else {
            const double th = th0 + (0.5 * M_PI - th0) * r[1];
            u = xa + a * tan(th);
            acc = exp(u0 * u0 - u * u);
        }
        if (r[3] <= acc) return neg ? -u : u;
    }
    return x;                                       /* unreachable in practice (probability < 1e-100) */
}

/* One re-emission: atom velocity, isotropic new direction, new frequency. */
static void orc_redistribute(double a, uint64_t seed, uint64_t p, uint32_t k, double kdir[3], double *x)
{
    double t[4];
    orc_block(seed, p, k, 2u, t);
    const double uperp = sqrt(-log(t[0])) * cos(2.0 * M_PI * t[1]);
    const double upar = orc_atom_upar(*x, a, seed, p, k);
    const double ct = 2.0 * t[2] - 1.0, st = sqrt(fmax(0.0, 1.0 - ct * ct));
    const double ph = 2.0 * M_PI * t[3];
    const double kn[3] = {st * cos(ph), st * sin(ph), ct};
    double mu = kdir[0] * kn[0] + kdir[1] * kn[1] + kdir[2] * kn[2];
    if (mu > 1.0) mu = 1.0;
    if (mu < -1.0) mu = -1.0;
    *x = *x - upar * (1.0 - mu) + uperp * sqrt(1.0 - mu * mu);
    for (int i = 0; i < 3; ++i) kdir[i] = kn[i];
}

static void orc_scatter_one(const orc_box *b, const orc_scatter_params *sp, const double *kappa, const double *ux,
                            const double *uy, const double *uz, uint64_t p, int64_t cell0, int64_t *A,
                            orc_scatter_rec *rec)
{
    const int64_t nx = b->nx, ny = b->ny, nz = b->nz;
    double u[8];
    orc_packet_uniforms(b->seed, p, u);
    double f[3] = {u[0], u[1], u[2]};
    double mu0 = 2.0 * u[3] - 1.0, ph0 = 2.0 * M_PI * u[4];
    double st0 = sqrt(fmax(0.0, 1.0 - mu0 * mu0));
    double k[3] = {st0 * cos(ph0), st0 * sin(ph0), mu0};
    double x = sqrt(-log(u[5])) * cos(2.0 * M_PI * u[6]);
    if (b->damping > 0.0) x += b->damping * tan(M_PI * (u[7] - 0.5));
    if (sp->fixed_x0) x = sp->x0;
    int64_t ci[3] = {cell0 % nx, (cell0 / nx) % ny, cell0 / (nx * ny)};
    const int64_t n[3] = {nx, ny, nz};
    const int64_t w = (int64_t)b->w0;
    int64_t nscat = 0, ncross = 0;
    int fate = 2;
    double x_stop = 0.0;
    int64_t c = cell0;
    int64_t moved[3] = {0, 0, 0};                             /* net face crossings per axis */
    rec->cell0 = cell0;
    rec->x0 = x;
    for (;;) {
        if (x <= -sp->x_inert || x > sp->x_inert) { fate = 1; x_stop = x; break; }
        if (nscat >= sp->max_events) { fate = 2; break; }
        uint32_t ew[4];
        orc_block_words(b->seed, p, (uint32_t)nscat, 1u, ew);
        double tau = -log(orc_uniform(ew[0]));
        int lost = 0;
        for (;;) {                                            /* free flight */
            c = ci[0] + nx * (ci[1] + ny * ci[2]);
            const double kap = kappa[c] / sp->p_ab;
            double t[3];
            for (int a = 0; a < 3; ++a) {
                if (k[a] > 0.0) t[a] = (1.0 - f[a]) / k[a];
                else if (k[a] < 0.0) t[a] = f[a] / (-k[a]);
                else t[a] = INFINITY;
            }
            int axis = 0;
            if (t[1] < t[axis]) axis = 1;
            if (t[2] < t[axis]) axis = 2;
            const double sf = t[axis];
            const double xf = x - b->delta * sf;
            const int inert = xf <= -sp->x_inert;
            const double slim = inert ? (x + sp->x_inert) / b->delta : sf;
            const double dtau = kap * orc_swept(b, x, inert ? x + sp->x_inert : b->delta * sf);
            if (dtau < tau) {
                if (inert) {                                  /* lost where x reaches -x_inert */
                    for (int a = 0; a < 3; ++a) {
                        const double g = f[a] + k[a] * slim;
                        f[a] = g < 0.0 ? 0.0 : (g > 1.0 ? 1.0 : g);
                    }
                    lost = 1;
                    break;
                }
                tau -= dtau;
                for (int a = 0; a < 3; ++a) {
                    if (a == axis) continue;
                    const double g = f[a] + k[a] * sf;
                    f[a] = g < 0.0 ? 0.0 : (g > 1.0 ? 1.0 : g);
                }
                const int64_t old = c;
                if (k[axis] > 0.0) { f[axis] = 0.0; ci[axis] = orc_wrap(ci[axis] + 1, n[axis]); ++moved[axis]; }
                else { f[axis] = 1.0; ci[axis] = orc_wrap(ci[axis] - 1, n[axis]); --moved[axis]; }
                x = xf;
                ++ncross;
                if (b->has_vel) {
                    const int64_t cn = ci[0] + nx * (ci[1] + ny * ci[2]);
                    x -= k[0] * (ux[cn] - ux[old]) + k[1] * (uy[cn] - uy[old]) + k[2] * (uz[cn] - uz[old]);
                }
                continue;
            }
            const double s = orc_flight_length(b, kap, x, tau, slim);
            for (int a = 0; a < 3; ++a) {
                const double g = f[a] + k[a] * s;
                f[a] = g < 0.0 ? 0.0 : (g > 1.0 ? 1.0 : g);
            }
            x -= b->delta * s;
            break;
        }
        if (lost) { fate = 1; x_stop = -sp->x_inert; break; }
        ++nscat;                                              /* a scattering in cell c */
        if ((((uint64_t)ew[1] << 32) | ew[2]) < orc_destroy_threshold(sp->p_destroy)) { fate = 0; break; }
        orc_redistribute(b->damping, b->seed, p, (uint32_t)(nscat - 1), k, &x);
        if (sp->x_return > 0.0 && fabs(x) < sp->x_return) { fate = 3; break; }
    }
    int64_t wing = 0;
    if (fate == 1 && b->kappa_far > 0.0) {
        const double pw = -expm1(-b->kappa_far * fmax(orc_Phi(b, x_stop), 0.0));
        wing = (int64_t)rint((double)w * pw);
        if (wing > w) wing = w;
    }
    if (fate == 0) A[c] += w;
    rec->cell_end = c;
    rec->x_end = fate == 1 ? x_stop : x;
    rec->scatterings = nscat;
    rec->crossings = ncross;
    rec->escaped = (fate == 1 || fate == 2) ? w : 0;
    rec->absorbed = fate == 0 ? w : 0;
    rec->wing = wing;
    for (int a = 0; a < 3; ++a) rec->d[a] = (double)moved[a] + f[a] - u[a];
    rec->fate = fate;
    rec->pad = 0;
}

/* Photons [p_begin, p_end) with resonant scattering. A (ncells) and out[6] =
 * {escaped weight, crossings, capped photons, capped weight, wing,
 * scatterings} are accumulated into. recs, when not NULL, gets one record per
 * photon. */
int orc_scatter(const orc_box *b, const orc_scatter_params *sp, const double *kappa, const double *ux,
                const double *uy, const double *uz, const uint64_t *first, uint64_t p_begin, uint64_t p_end,
                int64_t *A, int64_t out[6], orc_scatter_rec *recs, int nthreads)
{
    const int64_t ncells = (int64_t)b->nx * b->ny * b->nz;
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    int64_t *priv = (int64_t *)calloc((size_t)nthreads * (size_t)ncells, sizeof(int64_t));
    if (!priv) return -1;
    int64_t esc = 0, cross = 0, capn = 0, capw = 0, wing = 0, nscat = 0;
#pragma omp parallel num_threads(nthreads) reduction(+ : esc, cross, capn, capw, wing, nscat)
    {
        int64_t *mine = priv + (size_t)omp_get_thread_num() * (size_t)ncells;
#pragma omp for schedule(dynamic, 16)
        for (uint64_t p = p_begin; p < p_end; ++p) {
            orc_scatter_rec r;
            orc_scatter_one(b, sp, kappa, ux, uy, uz, p, orc_find_cell(first, ncells, p), mine, &r);
            cross += r.crossings;
            nscat += r.scatterings;
            if (r.fate == 1) { esc += r.escaped; wing += r.wing; }
            if (r.fate == 2) { capn += 1; capw += r.escaped; }
            if (recs) recs[p - p_begin] = r;
        }
    }
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t c = 0; c < ncells; ++c) {
        int64_t sum = 0;
        for (int t = 0; t < nthreads; ++t) sum += priv[(size_t)t * (size_t)ncells + c];
        A[c] += sum;
    }
    free(priv);
    out[0] += esc; out[1] += cross; out[2] += capn; out[3] += capw; out[4] += wing; out[5] += nscat;
    return 0;
}

/* Test hooks: n draws of the atom's parallel velocity at frequency x (photon
 * ids 0..n-1, event 0), and n successive re-emissions of one photon starting
 * at x0 with direction (0, 0, 1), with no flight between them. */
void orc_atom_upar_draws(double x, double a, uint64_t seed, int64_t n, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = orc_atom_upar(x, a, seed, (uint64_t)i, 0u);
}

void orc_redistribution_chain(double x0, double a, uint64_t seed, uint64_t p, int64_t n, double *xs)
{
    double k[3] = {0.0, 0.0, 1.0}, x = x0;
    for (int64_t i = 0; i < n; ++i) {
        orc_redistribute(a, seed, p, (uint32_t)i, k, &x);
        xs[i] = x;
    }
}

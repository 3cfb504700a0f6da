// Resonant-scattering Monte Carlo (App. A, steps 1-8): photons followed
// scattering by scattering through the same grid, records and tallies as the
// streaming walk.
//
// A photon's free path is an optical depth -ln(u); along a straight segment
// the depth is kappa_sc times the swept profile, kappa_sc = kappa / p_ab the
// full line opacity per unit of the cumulative profile (the streaming walk's
// kappa is the true-absorption part). Where the drawn depth runs out inside a
// cell, the scattering point follows by Newton's method on the swept profile.
// At a scattering the photon is destroyed when a 64-bit integer from its
// event block is below floor(p_destroy 2^64) (step 7); otherwise the atom's
// parallel velocity is drawn from exp(-u^2) / ((x - u)^2 + a^2) (Eq. (MC),
// split rejection after Zheng & Miralda-Escude 2002), its perpendicular one
// projected on the scattering plane from exp(-u^2), the new direction is
// isotropic, and the frequency becomes x - u_par (1 - mu) + u_perp
// sqrt(1 - mu^2) (Eq. (inout); its bulk term applies at cell faces). A photon
// redshifted below -x_inert is lost to the line; the far damping wing takes
// the expected share 1 - exp(-kbar Phi(-x_inert)) of it (reported as wing).
//
// Random numbers (the same counters as the oracle): event k of photon p uses
// Philox blocks (p_lo, p_hi, k, 1) [free path; destruction word pair],
// (p_lo, p_hi, k, 2) [perpendicular velocity; new direction] and
// (p_lo, p_hi, k, 3 + j) for trial j of the parallel velocity.
//
// Driver: resident waves pull blocks of photon ids from a queue and refill
// idle lanes (a photon's life ranges from one scattering to millions). Each
// loop iteration advances a lane by one event: a face crossing, or a
// scattering.
#include "walk_core.hpp"

namespace mclya {
namespace {

__device__ __forceinline__ void event_block(uint64_t seed, uint64_t p, uint32_t k, uint32_t stream, uint32_t w[4])
{
    w[0] = (uint32_t)p;
    w[1] = (uint32_t)(p >> 32);
    w[2] = k;
    w[3] = stream;
    philox4x32_10(w, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// Line density: the derivative of the cumulative profile the walk uses
// (Doppler, or Voigt to first order in a with damp = 2a/pi).
__device__ __forceinline__ float line_density(float y, float damp)
{
    const float g = 0.5641895835477563f * __expf(-y * y);     // exp(-y^2)/sqrt(pi)
    return damp != 0.0f ? fmaf(-damp, dawson_deriv_f32(y), g) : g;
}

__device__ __forceinline__ float swept(float x, float dx, float damp)
{
    return damp != 0.0f ? swept_profile_voigt(x, dx, damp) : swept_profile(x, dx);
}

// Length s in (0, s_max] with kap * swept(x, delta s) = tau: Newton's method
// inside a shrinking bracket (the swept mass grows with s), from the linear
// estimate s_lin = tau / (kap delta phi(x)). A Newton step that leaves the closed
// bracket is replaced by its midpoint; one that lands on an end of it (a
// step below binary32 resolution) ends the search, as does a residual of
// exactly zero. Over a short segment (delta s <= 0.05) a step below 3e-4 of
// s also ends it: the error after a Newton step is about |y| delta s times
// the square of the step's relative size (y the frequency, for the Gaussian
// core), below 1e-8 |y| there, so the search usually ends after one step.
// A flight from the wing across the core (high zeta) takes up to about
// twenty, as the swept mass turns from flat to steep there. `found` is false
// when the depth over the whole of (0, s_max] stays below tau (no root was
// bracketed).
__device__ __forceinline__ float flight_length(float kap, float delta, float damp, float x, float tau, float s_lin,
                                               float s_max, bool &found)
{
    float lo = 0.0f, hi = s_max;
    float s = s_lin;
    if (!(s > lo && s < hi)) s = 0.5f * (lo + hi);
    bool root = false;
#pragma unroll 1
    for (int it = 0; it < 32; ++it) {
        const float g = kap * swept(x, delta * s, damp) - tau;
        if (g == 0.0f) {
            root = true;
            break;
        }
        if (g > 0.0f) hi = s; else lo = s;
        float sn = s - g * __builtin_amdgcn_rcpf(kap * delta * line_density(x - delta * s, damp));
        if (!(sn >= lo && sn <= hi)) sn = 0.5f * (lo + hi);
        const float step = fabsf(sn - s);
        const bool done = step <= 1e-6f * s || (step <= 3e-4f * s && delta * sn <= 0.05f);
        s = sn;
        if (done) break;
    }
    found = root || hi < s_max;
    return s;
}

// Parallel velocity of the scattering atom (step 8): a draw from
// exp(-u^2) / ((x - u)^2 + a^2) for x >= 0 (mirrored for x < 0) by rejection
// from an envelope split at u0. Below u0: the Cauchy factor alone (|x| < 5),
// or the Gaussian over (x - u0)^2 (|x| >= 5, where the draw is mostly
// thermal); above u0: the Cauchy factor times exp(-u0^2). The split point
// changes only the number of trials: u0 = x - 0.02 - 0.1 max(0, x - 1)^2 (at
// least 0) for x < 5, sqrt(6.3 + 3.2 ln x) beyond. a = 0: resonant, u = x.
// The trials stop after 4096 (returning the resonant u = x) so that every
// draw ends.
__device__ __forceinline__ float atom_upar(float x, float a, uint64_t seed, uint64_t p, uint32_t k)
{
    if (a == 0.0f) return x;
    constexpr float kHalfPi = 1.5707963267948966f;
    const bool neg = x < 0.0f;
    const float xa = fabsf(x);
    const bool wing = xa >= 5.0f;
    float u0;
    if (wing) {
        u0 = sqrtf(fmaf(3.2f, logf(xa), 6.3f));
    } else {
        const float q = fmaxf(xa - 1.0f, 0.0f);
        u0 = fmaxf(xa - 0.02f - 0.1f * q * q, 0.0f);
    }
    // phi0: the Cauchy angle of the split measured from -pi/2, atan(a / (x - u0))
    // (taken directly, not as atan((u0 - x) / a) + pi/2, which cancels in
    // binary32 where the split sits far below resonance)
    const float phi0 = atanf(a / (xa - u0));
    const float m2 = expf(-u0 * u0) * (2.0f * kHalfPi - phi0);
    const float m1 = wing ? 0.886226925452758f * erfcf(-u0) * a / ((xa - u0) * (xa - u0)) : phi0;
    const float p1 = m1 / (m1 + m2);
#pragma unroll 1
    for (uint32_t j = 0; j < 4096u; ++j) {       // at worst ~14 trials are expected
        uint32_t w[4];
        event_block(seed, p, k, 3u + j, w);
        const float r0 = u01(w[0]), r1 = u01(w[1]), r3 = u01(w[3]);
        float u, acc;
        if (r0 < p1) {
            if (wing) {
                u = sqrtf(-logf(r1)) * cospif(2.0f * u01(w[2]));
                if (u > u0) continue;
                acc = (xa - u0) * (xa - u0) / fmaf(xa - u, xa - u, a * a);
            } else {
                // angle psi = phi0 r1 above -pi/2: tan(psi - pi/2) = -1 / tan(psi)
                u = xa - a / tanf(phi0 * r1);
                acc = expf(-u * u);
            }
        } else {
            const float th = fmaf(2.0f * kHalfPi - phi0, r1, phi0 - kHalfPi);
            u = fmaf(a, tanf(th), xa);
            acc = expf(u0 * u0 - u * u);
        }
        if (r3 <= acc) return neg ? -u : u;
    }
    return x;                                       // unreachable in practice (probability < 1e-100)
}

struct Photon {
    int32_t ix, iy, iz;
    uint32_t c;
    double fx, fy, fz;        // position inside the cell
    double kx, ky, kz;        // direction
    float x;                  // gas-frame frequency (Doppler widths)
    float tau;                // optical depth left to the next scattering
    Rec r;                    // the cell's record
    uint32_t nscat, ncross;
    int32_t mx, my, mz;       // net face crossings per axis (the unwrapped cell offset)
    uint64_t p;               // box-local photon id
    uint32_t cell0;
    float x0;
    bool need_event;
    uint32_t dw1, dw2;        // destruction word pair of the current event
};

// Emission: position uniform in the cell, isotropic direction, frequency
// from the line profile: the same formulas and Philox words as the
// streaming walk's emission.
template <bool VEL>
__device__ __forceinline__ void init_photon(Photon &P, const WalkBox &B, float a, uint64_t p, uint32_t gcell,
                                            const void *__restrict__ rec, bool fixed_x0, float x0)
{
    const uint32_t k0 = (uint32_t)B.seed, k1 = (uint32_t)(B.seed >> 32);
    uint32_t wa[4] = {(uint32_t)p, (uint32_t)(p >> 32), 0u, 0u};
    uint32_t wb[4] = {(uint32_t)p, (uint32_t)(p >> 32), 1u, 0u};
    philox4x32_10(wa, k0, k1);
    philox4x32_10(wb, k0, k1);
    const uint32_t local = gcell - B.cell_off;
    P.ix = (int32_t)(local % (uint32_t)B.nx);
    const uint32_t rest = local / (uint32_t)B.nx;
    P.iy = (int32_t)(rest % (uint32_t)B.ny);
    P.iz = (int32_t)(rest / (uint32_t)B.ny);
    P.c = gcell;
    P.fx = (double)u01(wa[0]);
    P.fy = (double)u01(wa[1]);
    P.fz = (double)u01(wa[2]);
    const double mu = 2.0 * (double)u01(wa[3]) - 1.0;
    double sp, cp;
    sincospi(2.0 * (double)u01(wb[0]), &sp, &cp);
    const double st = sqrt((1.0 - mu) * (1.0 + mu));
    P.kx = st * cp;
    P.ky = st * sp;
    P.kz = mu;
    float x = sqrtf(-logf(u01(wb[1]))) * cospif(2.0f * u01(wb[2]));
    if (a != 0.0f) {
        const float v = u01(wb[3]) - 0.5f;
        x += a * (sinpif(v) / cospif(v));
    }
    P.x = fixed_x0 ? x0 : x;
    P.x0 = P.x;
    P.cell0 = gcell;
    P.r = load_rec<VEL>(rec, gcell);
    P.nscat = 0;
    P.ncross = 0;
    P.mx = P.my = P.mz = 0;
    P.p = p;
    P.need_event = true;
}

__device__ __forceinline__ int box_index(const WalkBox *boxes, int n_boxes, uint64_t gp)
{
    int lo = 0, hi = n_boxes - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (boxes[mid].pkt_off <= gp) lo = mid; else hi = mid - 1;
    }
    return lo;
}

enum : int { kSAlive = 0, kSDestroyed = 1, kSLost = 2, kSCapped = 3, kSReturned = 4 };
constexpr int kBurst = 64;

template <bool VEL>
__device__ __forceinline__ int scatter_at(Photon &P, const WalkBox &B, const ScatBox &S, unsigned long long *A,
                                          const ScatterParams &SP, float s);

// One event of a photon: a face crossing, or a scattering (free-path end,
// destruction test, re-emission). Returns the photon's state afterwards.
template <bool VEL>
__device__ __forceinline__ int scatter_event(Photon &P, const WalkBox &B, const ScatBox &S, const void *rec,
                                             unsigned long long *A, const ScatterParams &SP, float &x_stop)
{
    if (P.need_event) {
        // a new free flight: first the line window and the event cap
        if (P.x <= -S.x_inert || P.x > S.x_inert) {
            x_stop = P.x;
            return kSLost;
        }
        if ((uint64_t)P.nscat >= SP.max_events) return kSCapped;
        uint32_t w[4];
        event_block(B.seed, P.p, P.nscat, 1u, w);
        P.tau = -logf(u01(w[0]));
        P.dw1 = w[1];
        P.dw2 = w[2];
        P.need_event = false;
    }
    const float kap = P.r.kap * S.inv_pab;
    // Most flights (in the line core) are far shorter than the distance to
    // the nearest face in any direction, r_safe: the linear estimate of the
    // flight and the cell-independent bound on how much it can grow over
    // delta s <= 1e-3 (phi changes by under 1 %) decide it without the face
    // search, and the root is then sought in (0, r_safe].
    const float s_lin = P.tau * __builtin_amdgcn_rcpf(kap * B.delta * line_density(P.x, S.damp));
    {
        const double rsafe = fmin(fmin(fmin(P.fx, 1.0 - P.fx), fmin(P.fy, 1.0 - P.fy)), fmin(P.fz, 1.0 - P.fz));
        if (B.delta * s_lin <= 1e-3f && 1.02f * s_lin < (float)rsafe && P.x - 2e-3f > -S.x_inert) {
            // over delta s < 1e-6 the density changes by about 1e-5 of itself
            // at most (|phi'/phi| = 2|x| in the thermal core, 2/|x| in the
            // damping wing): the linear estimate is the flight
            if (B.delta * s_lin < 1e-6f) return scatter_at<VEL>(P, B, S, A, SP, s_lin);
            bool found = false;
            const float s = flight_length(kap, B.delta, S.damp, P.x, P.tau, s_lin, (float)rsafe, found);
            if (found) return scatter_at<VEL>(P, B, S, A, SP, s);
        }
    }
    // next face (ties: x, then y, then z)
    const double tx = P.kx > 0.0 ? (1.0 - P.fx) / P.kx : (P.kx < 0.0 ? P.fx / -P.kx : 1.0e300);
    const double ty = P.ky > 0.0 ? (1.0 - P.fy) / P.ky : (P.ky < 0.0 ? P.fy / -P.ky : 1.0e300);
    const double tz = P.kz > 0.0 ? (1.0 - P.fz) / P.kz : (P.kz < 0.0 ? P.fz / -P.kz : 1.0e300);
    const bool bx = tx <= ty && tx <= tz;
    const bool by = !bx && ty <= tz;
    const double sf = bx ? tx : (by ? ty : tz);
    const float xf = fmaf(-B.delta, (float)sf, P.x);
    const bool inert = xf <= -S.x_inert;
    const float dx = inert ? P.x + S.x_inert : B.delta * (float)sf;
    const float dtau = kap * swept(P.x, dx, S.damp);
    if (dtau < P.tau) {
        if (inert) {
            // lost where the frequency reaches -x_inert, inside this cell
            const double sl = (double)((P.x + S.x_inert) / B.delta);
            P.fx = fmin(fmax(P.fx + P.kx * sl, 0.0), 1.0);
            P.fy = fmin(fmax(P.fy + P.ky * sl, 0.0), 1.0);
            P.fz = fmin(fmax(P.fz + P.kz * sl, 0.0), 1.0);
            x_stop = -S.x_inert;
            return kSLost;
        }
        P.tau -= dtau;
        // cross the face into the neighbour (periodic)
        const double nfx = fmin(fmax(P.fx + P.kx * sf, 0.0), 1.0);
        const double nfy = fmin(fmax(P.fy + P.ky * sf, 0.0), 1.0);
        const double nfz = fmin(fmax(P.fz + P.kz * sf, 0.0), 1.0);
        P.fx = nfx;
        P.fy = nfy;
        P.fz = nfz;
        if (bx) {
            if (P.kx > 0.0) { P.fx = 0.0; P.ix = P.ix + 1 == B.nx ? 0 : P.ix + 1; ++P.mx; }
            else { P.fx = 1.0; P.ix = P.ix == 0 ? B.nx - 1 : P.ix - 1; --P.mx; }
        } else if (by) {
            if (P.ky > 0.0) { P.fy = 0.0; P.iy = P.iy + 1 == B.ny ? 0 : P.iy + 1; ++P.my; }
            else { P.fy = 1.0; P.iy = P.iy == 0 ? B.ny - 1 : P.iy - 1; --P.my; }
        } else {
            if (P.kz > 0.0) { P.fz = 0.0; P.iz = P.iz + 1 == B.nz ? 0 : P.iz + 1; ++P.mz; }
            else { P.fz = 1.0; P.iz = P.iz == 0 ? B.nz - 1 : P.iz - 1; --P.mz; }
        }
        P.c = B.cell_off + (uint32_t)P.ix + (uint32_t)B.nx * ((uint32_t)P.iy + (uint32_t)B.ny * (uint32_t)P.iz);
        const Rec nr = load_rec<VEL>(rec, P.c);
        if (VEL)
            P.x = xf - ((float)P.kx * (nr.ux - P.r.ux) + (float)P.ky * (nr.uy - P.r.uy) +
                        (float)P.kz * (nr.uz - P.r.uz));
        else
            P.x = xf;
        P.r = nr;
        ++P.ncross;
        return kSAlive;
    }
    // the scattering point inside this cell
    const float slim = inert ? (P.x + S.x_inert) / B.delta : (float)sf;
    bool found = false;
    const float s = flight_length(kap, B.delta, S.damp, P.x, P.tau, s_lin, slim, found);
    return scatter_at<VEL>(P, B, S, A, SP, s);
}

// Moves the photon s along its path and scatters it there (steps 7-8).
template <bool VEL>
__device__ __forceinline__ int scatter_at(Photon &P, const WalkBox &B, const ScatBox &S, unsigned long long *A,
                                          const ScatterParams &SP, float s)
{
    const double sd = (double)s;
    P.fx = fmin(fmax(P.fx + P.kx * sd, 0.0), 1.0);
    P.fy = fmin(fmax(P.fy + P.ky * sd, 0.0), 1.0);
    P.fz = fmin(fmax(P.fz + P.kz * sd, 0.0), 1.0);
    P.x = fmaf(-B.delta, s, P.x);
    const uint32_t k = P.nscat;
    ++P.nscat;
    P.need_event = true;
    if ((((uint64_t)P.dw1 << 32) | P.dw2) < S.destroy) {
        atomicAdd(&A[P.c], (unsigned long long)B.w0);
        return kSDestroyed;
    }
    // re-emission (step 8)
    uint32_t t[4];
    event_block(B.seed, P.p, k, 2u, t);
    const float uperp = sqrtf(-logf(u01(t[0]))) * cospif(2.0f * u01(t[1]));
    const float upar = atom_upar(P.x, S.a, B.seed, P.p, k);
    // new direction: cos theta exact, the azimuth in binary32
    const double ct = 2.0 * (double)u01(t[2]) - 1.0;
    const double st = sqrt(fmax(0.0, (1.0 - ct) * (1.0 + ct)));
    float spf, cpf;
    sincospif(2.0f * u01(t[3]), &spf, &cpf);
    const double nkx = st * (double)cpf, nky = st * (double)spf, nkz = ct;
    const float mu = fminf(fmaxf((float)(P.kx * nkx + P.ky * nky + P.kz * nkz), -1.0f), 1.0f);
    P.x = P.x - upar * (1.0f - mu) + uperp * sqrtf((1.0f - mu) * (1.0f + mu));
    P.kx = nkx;
    P.ky = nky;
    P.kz = nkz;
    if (SP.x_return > 0.0f && fabsf(P.x) < SP.x_return) return kSReturned;
    return kSAlive;
}

// The end of a photon: its totals (one set of atomics per photon: a photon
// lives for thousands to millions of events) and its record.
__device__ __forceinline__ void finish_photon(const Photon &P, const WalkBox &B, int box, int st, float x_stop,
                                              const ScatterParams &SP)
{
    uint32_t wing = 0;
    if (st == kSLost && B.kfar > 0.0f) {
        wing = absorbed_share(B.w0, B.kfar * cumulative_voigt(x_stop, B.damp));
    }
    BoxTot &t = SP.tot[box];
    const bool out = st == kSLost || st == kSCapped;
    if (out) atomicAdd(&t.escaped, (unsigned long long)B.w0);
    if (P.ncross) atomicAdd(&t.crossings, (unsigned long long)P.ncross);
    if (st == kSCapped) {
        atomicAdd(&t.capped_packets, 1ull);
        atomicAdd(&t.capped_weight, (unsigned long long)B.w0);
    }
    if (wing) atomicAdd(&t.wing, (unsigned long long)wing);
    if (P.nscat) atomicAdd(&t.pad[0], (unsigned long long)P.nscat);
    if (SP.records) {
        mc_lya_scatter_record &o = SP.records[P.p + B.pkt_off - SP.first];
        o.cell0 = P.cell0;
        o.cell_end = P.c;
        o.x0 = P.x0;
        o.x_end = st == kSLost ? x_stop : P.x;
        o.scatterings = P.nscat;
        o.crossings = P.ncross;
        o.fate = st == kSDestroyed ? 0 : st == kSLost ? 1 : st == kSCapped ? 2 : 3;
        o.escaped = out ? (int64_t)B.w0 : 0;
        o.absorbed = st == kSDestroyed ? (int64_t)B.w0 : 0;
        o.wing = (int64_t)wing;
        // the emission point's place in its cell: the emission's own Philox words
        uint32_t wa[4] = {(uint32_t)P.p, (uint32_t)(P.p >> 32), 0u, 0u};
        philox4x32_10(wa, (uint32_t)B.seed, (uint32_t)(B.seed >> 32));
        o.dx = (float)((double)P.mx + P.fx - (double)u01(wa[0]));
        o.dy = (float)((double)P.my + P.fy - (double)u01(wa[1]));
        o.dz = (float)((double)P.mz + P.fz - (double)u01(wa[2]));
        o.reserved = 0;
    }
}

// Waves per SIMD the register allocation aims at (0: the compiler's choice).
#ifndef MCLYA_SCATTER_WAVES
#define MCLYA_SCATTER_WAVES 0
#endif
#if MCLYA_SCATTER_WAVES > 0
#define MCLYA_SCATTER_OCCUPANCY __attribute__((amdgpu_waves_per_eu(MCLYA_SCATTER_WAVES)))
#else
#define MCLYA_SCATTER_OCCUPANCY
#endif

// SINGLE: one box, whose constants are wave-uniform (scalar registers).
template <bool VEL, bool SINGLE>
__global__ __launch_bounds__(256) MCLYA_SCATTER_OCCUPANCY void scatter_kernel(ScatterParams SP)
{
    const uint32_t lane = __lane_id();
    Photon P;
    int box = 0;
    bool alive = false;
    bool more = true;
    uint64_t cur = 0, end = 0;
    const uint32_t nq = (uint32_t)SP.nqueues;
    uint32_t part = blockIdx.x % nq, tried = 0;
    const uint64_t chunk = (uint64_t)SP.chunk;
    WalkBox B1;
    ScatBox S1;
    if (SINGLE) {
        B1 = SP.boxes[0];
        S1 = SP.sbox[0];
    }
    for (;;) {
        uint64_t idle = __ballot(!alive);
        if (more && (uint32_t)__popcll(idle) >= (uint32_t)SP.refill) {
            while (idle && more) {
                if (cur >= end) {
                    const uint64_t lo = SP.count * part / nq, hi = SP.count * (part + 1) / nq;
                    uint64_t base = 0;
                    if (lane == 0) base = atomicAdd(&SP.queue[part], (unsigned long long)chunk);
                    base = lo + __shfl(base, 0, 64);
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
                const uint32_t r = __builtin_amdgcn_mbcnt_hi((uint32_t)(idle >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
                if (!alive && (uint64_t)r < take) {
                    const uint64_t gp = SP.first + cur + r;
                    if (SINGLE) {
                        init_photon<VEL>(P, B1, S1.a, gp - B1.pkt_off, SP.cell_of_packet[gp], SP.rec,
                                         SP.fixed_x0 != 0, SP.x0);
                    } else {
                        box = box_index(SP.boxes, SP.n_boxes, gp);
                        const WalkBox B = SP.boxes[box];
                        init_photon<VEL>(P, B, SP.sbox[box].a, gp - B.pkt_off, SP.cell_of_packet[gp], SP.rec,
                                         SP.fixed_x0 != 0, SP.x0);
                    }
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
            // up to kBurst events per lane before the wave looks at refills
            // again (photons live for up to millions of events)
            const WalkBox B = SINGLE ? B1 : SP.boxes[box];
            const ScatBox S = SINGLE ? S1 : SP.sbox[box];
#pragma unroll 1
            for (int ev = 0; ev < kBurst; ++ev) {
                float x_stop = 0.0f;
                const int st = scatter_event<VEL>(P, B, S, SP.rec, SP.A, SP, x_stop);
                if (st != kSAlive) {
                    finish_photon(P, B, box, st, x_stop, SP);
                    alive = false;
                    break;
                }
            }
        }
    }
}

__global__ void reset_scatter_queue_kernel(unsigned long long *q, int n)
{
    if ((int)threadIdx.x < n) q[threadIdx.x] = 0ull;
}

}  // namespace

hipError_t launch_scatter(const ScatterParams &p, int block, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(reset_scatter_queue_kernel, dim3(1), dim3(64), 0, s, p.queue, (int)p.nqueues);
    const dim3 g((unsigned)grid), b((unsigned)block);
    if (p.n_boxes == 1) {
        if (p.vel) hipLaunchKernelGGL((scatter_kernel<true, true>), g, b, 0, s, p);
        else hipLaunchKernelGGL((scatter_kernel<false, true>), g, b, 0, s, p);
    } else {
        if (p.vel) hipLaunchKernelGGL((scatter_kernel<true, false>), g, b, 0, s, p);
        else hipLaunchKernelGGL((scatter_kernel<false, false>), g, b, 0, s, p);
    }
    return hipGetLastError();
}

}  // namespace mclya

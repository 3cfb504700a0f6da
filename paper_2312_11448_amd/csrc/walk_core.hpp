// Per-packet arithmetic of the Lyman-alpha walk, shared by every driver:
// emission (App. A step 1), the straight-line cell walk with the Hubble drift
// (App. A step 4), the bulk-velocity shift of Eq. (inout) at faces, the
// expected-value deposit of the true absorption (kappa_c times the swept part
// of the profile, the depth of Eq. (<fnu>)) and escape by redshifting (end of
// App. A). Drivers differ only in where deposits go and which cells they own,
// so every driver produces the same integers.
//
// Two line profiles: the thermal (Doppler) one, and the Voigt profile of
// Eq. (MC) (the thermal profile convolved with the natural width of the 2p
// level, half width a in Doppler units). For the Voigt profile the emission
// adds a Cauchy deviate a tan(pi (u - 1/2)) to the thermal one, the cumulative
// profile is taken to first order in a, Phi_V = erfc(-x)/2 - (2a/pi) F(x)
// with F Dawson's integral (the neglected terms are O(a^2), below 2e-7 at
// a = 8.6e-4), and an escaping packet leaves the expected share
// 1 - exp(-kbar Phi_V(x_stop)) of its weight to the far damping wing (kbar the
// box's mean kappa: beyond -x_eff the wing is crossed over hundreds of cells).
// Packets emitted above x_blue, blue of every walked frequency, are not
// walked: they escape at once and the wing takes its share at x0.
#pragma once

#include "common.hpp"
#include "dawson.hpp"

namespace mclya {

constexpr double kFar = 1.0e300;   // face distance along an axis the ray does not move on

// Ray geometry is kept in binary64: over paths of hundreds of cells binary32
// directions drift by ~1e-5 cell, enough to clip a different cell corner than
// an exact ray. The walk is incremental (Amanatides & Woo): tm[a] is the path
// length from the emission point to the next face on axis a, td[a] = 1/|k_a|
// the length between two faces, t the length walked so far. The line-profile
// arithmetic (drift, swept profile, deposit) is binary32.
struct Lane {
    int32_t ix, iy, iz;
    uint32_t c;          // global cell
    double tmx, tmy, tmz;
    double tdx, tdy, tdz;
    double t;
    float kx, ky, kz;    // direction (binary32: velocity terms only)
    float x;             // gas-frame frequency, Doppler widths
    float kap;           // kappa of the current cell
    float ku;            // k . U of the current cell (bulk velocity along the ray, Doppler units)
    uint32_t w;          // remaining weight (w0 < 2^32)
    uint32_t ncross;
    int32_t nx, ny, nz;
    uint32_t coff;
    float delta, xeff;
};

struct Rec {
    float kap, ux, uy, uz;
};

template <bool VEL>
__device__ __forceinline__ Rec load_rec(const void *__restrict__ rec, uint32_t c)
{
    Rec r;
    if (VEL) {
        const float4 v = static_cast<const float4 *>(rec)[c];
        r.kap = v.x;
        r.ux = v.y;
        r.uy = v.z;
        r.uz = v.w;
    } else {
        r.kap = static_cast<const float *>(rec)[c];
        r.ux = r.uy = r.uz = 0.0f;
    }
    return r;
}

// k . U of a cell for a ray of direction k (Doppler units). The frequency
// shift of Eq. (inout) at a face is the change of this projection,
// x_new = x_old - (k.U_new - k.U_old). One expression, shared by every place
// that forms it, so that the rounding is the same wherever a face is crossed
// (a uniform flow gives exactly equal projections and no shift).
__device__ __forceinline__ float ray_velocity(float kx, float ky, float kz, const Rec &r)
{
    return fmaf(kz, r.uz, fmaf(ky, r.uy, kx * r.ux));
}

// Line constants of a box (uniform over a tile): the Voigt walk's, and
// whether every segment is short. A segment is at most a cell's diagonal
// long (sqrt 3 cells; its binary32 length rounds below 1.75), so its swept
// frequency dx = delta * length (or less, when it stops at -x_eff) stays
// below 0.05 Doppler widths in every box with delta <= 0.05 / 1.75; there the
// short-segment form of the swept profile is taken without a per-segment
// test (the same form the test would choose, so the same bits).
struct Line {
    float damp;     // 2a/pi
    float kfar;     // mean kappa of the box
    float xblue;    // packets above it are not walked
    bool short_seg; // delta * 1.75 <= 0.05
};

__device__ __forceinline__ Line line_of(const WalkBox &B)
{
    return Line{B.damp, B.kfar, B.xblue, B.delta * 1.75f <= 0.05f};
}

// Emission of packet p (box-local id) in global cell gcell: position uniform
// in the cell, isotropic direction, frequency from the Doppler profile
// exp(-x^2)/sqrt(pi) by the Box-Muller transform, plus for the Voigt profile
// the Cauchy deviate of the natural line from the eighth uniform. Optionally
// returns the initial state (position inside the cell and direction) for
// traces.
template <bool VOIGT>
__device__ __forceinline__ void emit_packet(Lane &L, const WalkBox &B, uint64_t p, uint32_t gcell,
                                            float *state = nullptr)
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
    const double fx = (double)u01(a[0]), fy = (double)u01(a[1]), fz = (double)u01(a[2]);
    const double mu = 2.0 * (double)u01(a[3]) - 1.0;   // exact
    double sp, cp;
    sincospi(2.0 * (double)u01(b[0]), &sp, &cp);         // azimuth 2 pi u
    const double st = sqrt((1.0 - mu) * (1.0 + mu));
    const double kx = st * cp, ky = st * sp, kz = mu;
    L.tdx = kx != 0.0 ? 1.0 / fabs(kx) : kFar;
    L.tdy = ky != 0.0 ? 1.0 / fabs(ky) : kFar;
    L.tdz = kz != 0.0 ? 1.0 / fabs(kz) : kFar;
    L.tmx = kx != 0.0 ? (kx > 0.0 ? 1.0 - fx : fx) * L.tdx : kFar;
    L.tmy = ky != 0.0 ? (ky > 0.0 ? 1.0 - fy : fy) * L.tdy : kFar;
    L.tmz = kz != 0.0 ? (kz > 0.0 ? 1.0 - fz : fz) * L.tdz : kFar;
    L.t = 0.0;
    L.kx = (float)kx;
    L.ky = (float)ky;
    L.kz = (float)kz;
    L.x = sqrtf(-logf(u01(b[1]))) * cospif(2.0f * u01(b[2]));
    if (VOIGT) {
        // a tan(pi v), v = u - 1/2 in (-1/2, 1/2), a = (pi/2) (2a/pi)
        const float v = u01(b[3]) - 0.5f;
        L.x += 1.5707963267948966f * B.damp * (sinpif(v) / cospif(v));
    }
    L.w = (uint32_t)B.w0;
    L.ncross = 0;
    if (state) {
        state[0] = (float)fx;
        state[1] = (float)fy;
        state[2] = (float)fz;
    }
}

// Emission (emit_packet) with the emission cell's opacity and velocity read
// from the packed records.
template <bool VEL, bool VOIGT = false>
__device__ __forceinline__ void init_packet(Lane &L, const WalkBox &B, uint64_t p, uint32_t gcell,
                                            const void *__restrict__ rec, float *state = nullptr)
{
    emit_packet<VOIGT>(L, B, p, gcell, state);
    const Rec r = load_rec<VEL>(rec, gcell);
    L.kap = r.kap;
    L.ku = VEL ? ray_velocity(L.kx, L.ky, L.kz, r) : 0.0f;
}

// Swept profile mass Phi(x) - Phi(x - dx) for dx > 0, Phi the cumulative
// Doppler profile. Segments are short (dx = delta * length, at most 0.033
// Doppler widths for the paper's cells), so the integral of
// f(y) = exp(-y^2)/sqrt(pi) over the segment is taken from the Taylor series
// of f about the midpoint m = x - h, h = dx/2:
//   integral = 2h f(m) [1 + (h^2/6) f2(m) + (h^4/120) f4(m)],
//   f2 = f''/f = 4m^2 - 2,   f4 = f''''/f = 16m^4 - 48m^2 + 12,
// with one exponential per segment. The next term of the series is below
// 3e-7 of the result for dx <= 0.05 and |x| <= 7, so the error is that of the
// binary32 exponential of -m^2 (about 6e-8 m^2 relative, as for any
// single-precision evaluation of the profile). Longer segments use the
// difference of complementary error functions, each taken where it is small.
// Never negative.
__device__ __forceinline__ float swept_short(float x, float dx)
{
    const float h = 0.5f * dx;
    const float m = x - h;
    const float m2 = m * m;
    const float h2 = h * h;
    const float c2 = fmaf(m2, 2.0f / 3.0f, -1.0f / 3.0f);                 // f2 / 6
    const float c4 = fmaf(m2, fmaf(m2, 2.0f / 15.0f, -0.4f), 0.1f);       // f4 / 120
    const float br = fmaf(h2, fmaf(h2, c4, c2), 1.0f);
    // 2h / sqrt(pi) = dx / sqrt(pi)
    return (dx * 0.5641895835477563f) * __expf(-m2) * br;
}

__device__ __forceinline__ float swept_profile(float x, float dx, bool short_seg = false)
{
    if (short_seg) return swept_short(x, dx);   // (uniform over a tile: no per-lane branch)
    if (dx <= 0.05f) return swept_short(x, dx);
    const float lo = x - dx;
    const float d = lo >= 0.0f ? 0.5f * (erfcf(lo) - erfcf(x)) : 0.5f * (erfcf(-x) - erfcf(-lo));
    return fmaxf(d, 0.0f);
}

// The same swept mass for the Voigt profile to first order in a:
// Phi_V(x) - Phi_V(x - dx) = (thermal part) - (2a/pi) int_{x-dx}^{x} F'(y) dy,
// F' = 1 - 2yF. Short segments take the integral by the midpoint rule (one
// Dawson evaluation). Its relative error is dx^2 / 24 times the ratio of the
// third derivative of F to F', about 6 / y^2 in the wing: below 3e-4 for
// dx <= 0.1 at |y| >= 3 and 3e-5 for the paper's cells (dx <= 0.033); in the
// core the thermal part dominates. Longer segments use the difference
// F(x - dx) - F(x). Never negative.
__device__ __forceinline__ float swept_profile_voigt(float x, float dx, float damp, bool short_seg = false)
{
    const float corr = (short_seg || dx <= 0.1f) ? -dx * dawson_deriv_f32(x - 0.5f * dx)
                                                 : dawson_f32(x - dx) - dawson_f32(x);
    return fmaxf(fmaf(damp, corr, swept_profile(x, dx, short_seg)), 0.0f);
}

// Cumulative Voigt profile to first order in a (the far-wing share).
__device__ __forceinline__ float cumulative_voigt(float x, float damp)
{
    return fmaxf(0.5f * erfcf(-x) - damp * dawson_f32(x), 0.0f);
}

// The integer weight that a packet of weight w < 2^32 leaves in a segment of
// true-absorption depth tau >= 0: rint(w (1 - e^-tau)), never more than w.
// A thin segment (tau < 0.1) takes the absorbed fraction from its Taylor
// series (no cancellation). A thicker one rounds the weight that passes,
// rint(w e^-tau), and deposits the rest: past tau ~ 17 the passing fraction
// is below binary32's resolution of 1 - e^-tau, yet w e^-tau can still be
// some units of weight that the packet carries into the next cell. The
// products are at most 0.1 w and 0.905 w, so both conversions stay inside
// the unsigned range and the result inside [0, w].
__device__ __forceinline__ uint32_t absorbed_share(uint32_t w, float tau)
{
    const bool thin = tau < 0.1f;
    const float series = tau * (1.0f - tau * (0.5f - tau * (1.0f / 6.0f - tau * (1.0f / 24.0f -
                                          tau * (1.0f / 120.0f - tau * (1.0f / 720.0f))))));
    const float pass = __expf(-tau);
    const uint32_t k = (uint32_t)rintf((float)w * (thin ? series : pass));
    return thin ? k : w - k;
}

// Entering a cell: the bulk term of Eq. (inout), x_new = x_old - (k.U_new -
// k.U_old), then the new cell's opacity and velocity projection.
template <bool VEL>
__device__ __forceinline__ void finish_entry(Lane &L, const Rec &nr)
{
    if (VEL) {
        const float kn = ray_velocity(L.kx, L.ky, L.kz, nr);
        L.x = L.x - (kn - L.ku);
        L.ku = kn;
    }
    L.kap = nr.kap;
}

// Global cell index of a lane's cell.
__device__ __forceinline__ uint32_t cell_of(const Lane &L)
{
    return L.coff + (uint32_t)L.ix + (uint32_t)L.nx * ((uint32_t)L.iy + (uint32_t)L.ny * (uint32_t)L.iz);
}

// Deposits go straight to the per-cell int64 tallies in device memory.
struct GlobalSink {
    static constexpr bool kCell = true;   // keeps each lane's global cell index
    unsigned long long *A;
    __device__ __forceinline__ void deposit(const Lane &L, uint32_t d) const
    {
        atomicAdd(&A[L.c], (unsigned long long)d);
    }
    __device__ __forceinline__ bool inside(int32_t, int32_t, int32_t) const { return true; }
    template <bool VEL>
    __device__ __forceinline__ Rec fetch(const void *__restrict__ rec, uint32_t cn, int32_t, int32_t, int32_t,
                                         bool) const
    {
        return load_rec<VEL>(rec, cn);
    }
};

// Histories only: nothing is tallied.
struct NullSink {
    static constexpr bool kCell = true;
    __device__ __forceinline__ void deposit(const Lane &, uint32_t) const {}
    __device__ __forceinline__ bool inside(int32_t, int32_t, int32_t) const { return true; }
    template <bool VEL>
    __device__ __forceinline__ Rec fetch(const void *__restrict__ rec, uint32_t cn, int32_t, int32_t, int32_t,
                                         bool) const
    {
        return load_rec<VEL>(rec, cn);
    }
};

// L = take ? N : L, field by field (selects, not a branch).
__device__ __forceinline__ void keep_or_take(Lane &L, const Lane &N, bool take)
{
    L.ix = take ? N.ix : L.ix;
    L.iy = take ? N.iy : L.iy;
    L.iz = take ? N.iz : L.iz;
    L.c = take ? N.c : L.c;
    L.tmx = take ? N.tmx : L.tmx;
    L.tmy = take ? N.tmy : L.tmy;
    L.tmz = take ? N.tmz : L.tmz;
    L.t = take ? N.t : L.t;
    L.x = take ? N.x : L.x;
    L.kap = take ? N.kap : L.kap;
    L.ku = take ? N.ku : L.ku;
    L.w = take ? N.w : L.w;
    L.ncross = take ? N.ncross : L.ncross;
}

// A lane state on which a step is harmless: cell 0 of a 1-cell grid (the
// first cell of the first box), no weight, far below any escape threshold.
__device__ __forceinline__ void idle_lane(Lane &L)
{
    L.ix = L.iy = L.iz = 0;
    L.nx = L.ny = L.nz = 1;
    L.coff = 0u;
    L.c = 0u;
    L.tmx = L.tmy = L.tmz = 1.0;
    L.tdx = L.tdy = L.tdz = 1.0;
    L.t = 0.0;
    L.kx = 1.0f;
    L.ky = L.kz = 0.0f;
    L.x = -3.0e38f;
    L.kap = 0.0f;
    L.ku = 0.0f;
    L.w = 0u;
    L.ncross = 0u;
    L.delta = 1.0f;
    L.xeff = 0.0f;
}

enum : int { kAlive = 0, kEscaped = 1, kAbsorbed = 2, kCapped = 3, kExit = 4 };

// The next face a ray crosses (Amanatides & Woo): the axis with the smallest
// face distance (ties: x, then y, then z) and that distance. Shared by every
// driver, so that each packet takes the same faces whichever driver walks it.
struct Face {
    bool bx, by, bz;
    double tn;
};

__device__ __forceinline__ Face next_face(double tmx, double tmy, double tmz)
{
    Face f;
    f.bx = tmx <= tmy && tmx <= tmz;
    f.by = !f.bx && tmy <= tmz;
    f.bz = !f.bx && !f.by;
    // the chosen distance, selected on the bit patterns (fmin would
    // canonicalise its operands with three extra FP64 instructions)
    const long long ux = __double_as_longlong(tmx), uy = __double_as_longlong(tmy), uz = __double_as_longlong(tmz);
    f.tn = __longlong_as_double(f.bx ? ux : (f.by ? uy : uz));
    return f;
}

// The line physics of one segment of length s (cells) through a cell of
// true-absorption depth kap per unit swept profile: the Hubble drift to
// xo = x - delta s (App. A step 4), the stop at -x_eff on the last segment
// (esc), and the expected-value deposit d of the absorbed weight (zero unless
// walk). One function for every driver: the same bits wherever a packet
// crosses a cell.
struct Segment {
    float xo;
    bool esc;
    uint32_t d;
};

template <bool VOIGT>
__device__ __forceinline__ Segment segment(float x, float s, float delta, float xeff, float kap, uint32_t w,
                                           bool walk, const Line &ln)
{
    Segment g;
    g.xo = fmaf(-delta, s, x);
    g.esc = g.xo <= -xeff;
    const float dx = g.esc ? x + xeff : delta * s;
    const float dphi = VOIGT ? swept_profile_voigt(x, dx, ln.damp, ln.short_seg) : swept_profile(x, dx, ln.short_seg);
    g.d = walk ? absorbed_share(w, kap * dphi) : 0u;
    return g;
}

// The far damping wing's share of an escaping packet's weight (Voigt): the
// wing beyond the stopping frequency xs, crossed at the box's mean kappa.
__device__ __forceinline__ uint32_t wing_share(uint32_t w, float xs, const Line &ln)
{
    return absorbed_share(w, ln.kfar * cumulative_voigt(xs, ln.damp));
}

// One (packet, cell) segment. Returns kAlive, or the packet's fate, or kExit
// when the next cell is outside the sink's region: the packet then stands on
// the face with its pre-jump frequency and the old cell's velocity, and the
// region that owns the new cell applies the jump (finish_entry).
//
// Written as straight-line code with one exit: the fate is a value, the
// deposit is predicated, and the state always advances to the next cell
// (harmless for a packet that has finished, whose weight and crossing count
// are left as they were). Early returns would make the compiler copy the
// whole lane state on every path.
//
// VOIGT: the Voigt profile of the box's Line; `wing` receives the far-wing
// share of an escaping packet's weight (0 otherwise). The packet's own weight
// L.w is left whole: the share is part of the escaped weight.
//
// act = false steps a lane that holds no packet (its state a finished
// packet's, or idle_lane's): it deposits and counts nothing, and the caller
// discards the state it leaves and the fate it returns.
template <bool VEL, bool VOIGT, class Sink>
__device__ __forceinline__ int walk_step(Lane &L, const void *__restrict__ rec, const Sink &sink,
                                         uint32_t max_cross, uint64_t &deposited, const Line &ln,
                                         uint32_t &wing, bool act = true)
{
    // redshifted out of the line (or, Voigt, emitted blue of the walked window)
    const bool gone = VOIGT ? (L.x <= -L.xeff) | (L.x > ln.xblue) : L.x <= -L.xeff;
    const bool capped = !gone && L.ncross >= max_cross;
    const bool walk = act && !gone && !capped;

    // next face and the neighbour behind it
    const Face f = next_face(L.tmx, L.tmy, L.tmz);
    const bool bx = f.bx, by = f.by, bz = f.bz;
    const double tn = f.tn;
    // only the coordinate on the chosen axis moves, by one cell (periodic);
    // sums of field-or-zero terms: a choice between fields would make the
    // compiler address the lane state in memory
    const int32_t ci = (bx ? L.ix : 0) + (by ? L.iy : 0) + (bz ? L.iz : 0);
    const int32_t ni = (bx ? L.nx : 0) + (by ? L.ny : 0) + (bz ? L.nz : 0);
    const bool up = (bx & (L.kx > 0.0f)) | (by & (L.ky > 0.0f)) | (bz & (L.kz > 0.0f));
    int32_t mi = ci + (up ? 1 : -1);
    mi = mi == ni ? 0 : mi;
    mi = mi < 0 ? ni - 1 : mi;
    const int32_t jx = bx ? mi : L.ix, jy = by ? mi : L.iy, jz = bz ? mi : L.iz;
    // the neighbour's global index, for sinks that address global memory by it
    const uint32_t cn = Sink::kCell
                            ? L.coff + (uint32_t)jx + (uint32_t)L.nx * ((uint32_t)jy + (uint32_t)L.ny * (uint32_t)jz)
                            : 0u;
    const bool stay = sink.inside(jx, jy, jz);
    const Rec nr = sink.template fetch<VEL>(rec, cn, jx, jy, jz, stay);   // in flight during the profile arithmetic

    // Hubble drift across the segment (the last one stops at -x_eff) and the deposit
    const Segment g = segment<VOIGT>(L.x, (float)(tn - L.t), L.delta, L.xeff, L.kap, L.w, walk, ln);
    const float xo = g.xo;
    const bool esc = g.esc;
    const uint32_t d = g.d;
    if (d) sink.deposit(L, d);
    L.w -= d;
    deposited += d;
    L.ncross += walk ? 1u : 0u;
    const int fate = gone ? kEscaped
                   : capped ? kCapped
                   : esc ? kEscaped
                   : L.w == 0 ? kAbsorbed
                   : stay ? kAlive : kExit;
    wing = 0u;
    if (VOIGT && fate == kEscaped) {
        // the far damping wing beyond the stopping frequency
        wing = wing_share(L.w, gone ? L.x : -L.xeff, ln);
    }

    // cross the face
    L.t = tn;
    L.tmx = bx ? L.tmx + L.tdx : L.tmx;
    L.tmy = by ? L.tmy + L.tdy : L.tmy;
    L.tmz = bz ? L.tmz + L.tdz : L.tmz;
    L.ix = jx;
    L.iy = jy;
    L.iz = jz;
    if (Sink::kCell) L.c = cn;
    // entering a cell owned by the same region: the bulk term of Eq. (inout)
    // and the new cell's opacity; leaving it: keep the pre-jump frequency
    if (VEL) {
        const float kn = ray_velocity(L.kx, L.ky, L.kz, nr);
        L.x = stay ? xo - (kn - L.ku) : xo;
        L.ku = stay ? kn : L.ku;
    } else {
        L.x = xo;
    }
    L.kap = stay ? nr.kap : L.kap;
    return fate;
}

}  // namespace mclya

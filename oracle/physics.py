"""FP64 physics of the oracle: scalars, closed forms and the recombination feed.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the benchmark's
CPU-baseline leg use this module. It is written independently of the HIP
library (which derives its own scalars in its own host code).

Paper: Jedamzik, Abel & Ali-Haimoud, "Cosmic recombination in the presence of
primordial magnetic fields", arXiv:2312.11448. Section, equation and appendix
names below refer to it.

Readings where the paper is silent or rounded (each also listed in the design
notes): constants not printed in the paper take standard values; the case-B fit
the paper cites (Pequignot et al. 1991, as in RecFast) uses the coefficients
a=4.309, b=-0.6166, c=0.6703, d=0.5300; beta_e follows from detailed balance
with the n=2 binding energy E_I/4 per 2s atom (footnote of Sec. III.A.1); one
temperature serves as both T_b and T_gamma; p_ab is the effective three-level
branching (beta_e + Lambda_2g) / (3 A + beta_e + Lambda_2g) of an excited atom.
"""
import math
import numpy as np
from scipy import integrate
from scipy.special import erfc, dawsn, voigt_profile

# --- constants (CGS) ---------------------------------------------------------
C_LIGHT = 2.99792458e10          # cm/s
K_B = 1.380649e-16               # erg/K
H_PLANCK = 6.62607015e-27        # erg s
M_E = 9.1093837015e-28           # g
M_H = 1.6735328e-24              # g, hydrogen atom (1.007825 u)
G_NEWTON = 6.67430e-8            # cm^3 g^-1 s^-2
MPC_CM = 3.0856775814913673e24
EV = 1.602176634e-12             # erg
A_RAD = 7.565723e-15             # erg cm^-3 K^-4 (radiation constant)
E_ION = 13.598434 * EV           # hydrogen ionisation energy
E_ALPHA = 0.75 * E_ION           # 1s-2p energy, "10.2 eV" (Sec. III.A.1)
E_2 = 0.25 * E_ION               # n=2 binding energy
LAMBDA_ALPHA = 1215.67e-8        # cm, Lyman-alpha wavelength
A_2P1S = 6.2649e8                # s^-1, "~6.3e8" (Sec. III.A.1)
LAMBDA_2G = 8.22458              # s^-1, "~8.22" (Sec. III.A.1)


# --- cosmology (Sec. II.C parameters) ----------------------------------------
def hubble0(h):
    """H0 = 100 h km/s/Mpc in s^-1."""
    return 100.0 * h * 1.0e5 / MPC_CM


def rho_crit0(h):
    return 3.0 * hubble0(h) ** 2 / (8.0 * math.pi * G_NEWTON)


def omega_m(cosmo):
    return (cosmo.omega_b_h2 + cosmo.omega_c_h2) / cosmo.h ** 2


def omega_r(cosmo):
    """Photons plus massless neutrinos: Omega_gamma (1 + 7/8 (4/11)^(4/3) N_eff)."""
    omega_g = A_RAD * cosmo.t_cmb0 ** 4 / (rho_crit0(cosmo.h) * C_LIGHT ** 2)
    return omega_g * (1.0 + 0.875 * (4.0 / 11.0) ** (4.0 / 3.0) * cosmo.n_eff)


def hubble(z, cosmo, zeta=1.0):
    """zeta * H(z) for a flat universe of matter, radiation and Lambda."""
    om, orad = omega_m(cosmo), omega_r(cosmo)
    ol = 1.0 - om - orad
    a1 = 1.0 + z
    return zeta * hubble0(cosmo.h) * math.sqrt(om * a1 ** 3 + orad * a1 ** 4 + ol)


def n_h0(cosmo):
    """Comoving hydrogen density (1 - Y_p) Omega_b rho_c / m_H at z=0, cm^-3."""
    omega_b = cosmo.omega_b_h2 / cosmo.h ** 2
    return (1.0 - cosmo.y_p) * omega_b * rho_crit0(cosmo.h) / M_H


# --- atomic rates (Sec. III.A.1) ---------------------------------------------
# Case-B fit A_B(T) = 1e-13 a t^b / (1 + c t^d) cm^3/s, t = T / 1e4 K
# (Pequignot, Petitjean & Boisson 1991, the fit RecFast uses; the paper cites
# it without printing the coefficients). Module-level so that the pins can
# plant a perturbed coefficient and see it caught.
CASE_B_FIT = (4.309, -0.6166, 0.6703, 0.5300)


def case_b(T):
    """Case-B recombination coefficient of hydrogen from the fit, cm^3/s."""
    a, b, c, d = CASE_B_FIT
    t = T / 1.0e4
    return 1.0e-13 * a * t ** b / (1.0 + c * t ** d)


def alpha_e(T):
    """alpha_e = 1.14 x case-B coefficient (Sec. III.A.1), cm^3/s."""
    return 1.14 * case_b(T)


def beta_e(T):
    """Photo-ionisation rate per 2s atom by detailed balance with alpha_e."""
    return alpha_e(T) * (2.0 * math.pi * M_E * K_B * T / H_PLANCK ** 2) ** 1.5 \
        * math.exp(-E_2 / (K_B * T))


def p_ab(T):
    """Probability that an excited atom is destroyed (ionised or 2-photon decay)
    rather than re-emitting Lyman-alpha: p_ab = 1 - p_sc (Sec. IV.A.1)."""
    b = beta_e(T)
    return (b + LAMBDA_2G) / (3.0 * A_2P1S + b + LAMBDA_2G)


def thermal_velocity(T):
    """v_th = sqrt(2 k T / m_H) (App. A), cm/s."""
    return math.sqrt(2.0 * K_B * T / M_H)


def damping(T):
    """Voigt parameter of Eq. (MC): the natural half width Gamma / 2 of the 2p
    level over the Doppler width omega_alpha v_th, a = A lambda / (4 pi v_th)."""
    return A_2P1S * LAMBDA_ALPHA / (4.0 * math.pi * thermal_velocity(T))


def tau_ab_per_n1s(T, H):
    """Mean optical depth to true absorption per unit n_1s, Eq. (<fnu>):
    3 A p_ab lambda^3 / (8 pi H)."""
    return p_ab(T) * 3.0 * LAMBDA_ALPHA ** 3 * A_2P1S / (8.0 * math.pi * H)


# --- closed forms ------------------------------------------------------------
def Phi(x):
    """Cumulative Doppler profile, int_{-inf}^x exp(-y^2)/sqrt(pi) dy."""
    return 0.5 * erfc(-np.asarray(x, dtype=np.float64))


def Phi_voigt(x, a):
    """Cumulative Voigt profile to first order in a: erfc(-x)/2 - (2a/pi) F(x),
    F Dawson's integral (the Cauchy CDF 1/2 + arctan(s/a)/pi expanded in a;
    the principal-value integral of the Gaussian against 1/s is the Dawson
    function)."""
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * erfc(-x) - 2.0 * a / math.pi * dawsn(x)


def voigt_cdf_exact(x, a):
    """Cumulative Voigt profile by quadrature of its definition: the thermal
    density exp(-y^2)/sqrt(pi) times the Cauchy CDF 1/2 + arctan((x-y)/a)/pi,
    integrated over y (the quadrature is split where the Cauchy factor turns)."""
    f = lambda y: math.exp(-y * y) / math.sqrt(math.pi) * (0.5 + math.atan((x - y) / a) / math.pi)
    lo, hi = min(-12.0, x - 1.0), max(12.0, x + 1.0)
    cuts = sorted({lo, hi, *[c for c in (x - 50 * a, x - a, x, x + a, x + 50 * a) if lo < c < hi]})
    return sum(integrate.quad(f, c0, c1, epsabs=1e-16, epsrel=1e-13, limit=400)[0]
               for c0, c1 in zip(cuts[:-1], cuts[1:]))


def voigt_density(x, a):
    """Normalised Voigt density in Doppler units (Gaussian of variance 1/2
    convolved with a Cauchy law of half width a)."""
    return voigt_profile(np.asarray(x, dtype=np.float64), 1.0 / math.sqrt(2.0), a)


def wing_homogeneous(tau, X, X_blue, a, kbar=None):
    """Expected fractions of the emitted weight in a homogeneous, static box
    with the Voigt profile and escape at -X: (walked absorption, far-wing
    absorption, true escape). A packet emitted at x0 in (-X, X_blue] keeps
    exp(-tau (Phi(x0) - Phi(-X))) when it reaches -X, and the wing then takes
    1 - exp(-kbar Phi(-X)) of it; a packet emitted outside that window is not
    walked and the wing takes 1 - exp(-kbar Phi(x0)). Integrated over the
    Voigt emission density by quadrature."""
    kbar = tau if kbar is None else kbar
    P = lambda x: float(Phi_voigt(x, a))
    px = P(-X)
    def keep(x0):
        return math.exp(-tau * max(P(x0) - px, 0.0)) if -X < x0 <= X_blue else 1.0
    def stop(x0):
        return px if -X < x0 <= X_blue else P(x0)
    dens = lambda x0: float(voigt_density(x0, a))
    def integ(fn):
        pts = [-1e6, -1e3, -50.0, -X, -3.0, 0.0, 3.0, X_blue, 50.0, 1e3, 1e6]
        return sum(integrate.quad(lambda y: dens(y) * fn(y), p0, p1, limit=400, epsabs=1e-14,
                                  epsrel=1e-11)[0] for p0, p1 in zip(pts[:-1], pts[1:]))
    walked = integ(lambda y: 1.0 - keep(y))
    wing = integ(lambda y: keep(y) * -math.expm1(-kbar * stop(y)))
    # the mass beyond +-1e6 (Cauchy tails, 2 a / (pi 1e6)) is escaped-and-absorbed
    # by the wing in full on the blue side and negligible on the red side
    wing += a / (math.pi * 1e6)
    return walked, wing, 1.0 - walked - wing


def escape_homogeneous(tau, X):
    """Escaped fraction in a homogeneous, static medium with profile-sampled
    emission and escape at x = -X: Phi(-X) + (1 - exp(-tau (1 - Phi(-X)))) / tau.
    The Sobolev escape probability (Sec. III.A.1) with the exact profile
    integral of the full-mixing solution (Sec. IV.A.2)."""
    px = float(Phi(-X))
    return px + (-math.expm1(-tau * (1.0 - px))) / tau


def escape_uniform_gradient(tau, g, X):
    """Escaped fraction in a homogeneous medium whose bulk flow along one axis
    has the uniform gradient dv_x/dx = g H (g > -1): along a direction at
    cosine mu to that axis a packet's gas-frame frequency drifts (1 + g mu^2)
    times as fast as by the expansion alone, so its depth per unit of swept
    profile is tau / (1 + g mu^2). The static closed form averaged over the
    isotropic directions; g = 0 is that closed form, and for tau >> 1 the
    result is (1 + g/3) / tau: H -> H + div v / 3 (Fig. MCescape caption)."""
    if not g > -1.0:
        raise ValueError("a converging flow with g <= -1 traps packets along the flow axis")
    from scipy import integrate
    f = lambda mu: escape_homogeneous(tau / (1.0 + g * mu * mu), X)
    val, _ = integrate.quad(f, 0.0, 1.0, epsabs=0.0, epsrel=1e-13, limit=200)
    return val


def sobolev_p_esc(H, n1s):
    """P_esc = 8 pi H / (3 lambda^3 n_1s A) (Sec. III.A.1)."""
    return 8.0 * math.pi * H / (3.0 * LAMBDA_ALPHA ** 3 * n1s * A_2P1S)


def r_alpha(H, n1s):
    """R_alpha = 8 pi H / (lambda^3 n_1s), Eq. (R-alpha)."""
    return 8.0 * math.pi * H / (LAMBDA_ALPHA ** 3 * n1s)


def peebles_c(T, H, n1s, lambda_2g=LAMBDA_2G):
    """Peebles C of Eq. (Cfactor)."""
    r = r_alpha(H, n1s)
    return (lambda_2g + r) / (beta_e(T) + lambda_2g + r)


# --- per-box derived quantities ----------------------------------------------
def box_scalars(spec):
    """FP64 scalars of one box (see BoxSpec in the workload presets)."""
    c = spec.cosmo
    H = hubble(spec.z, c, spec.zeta)
    T = spec.temp_K
    vth = thermal_velocity(T)
    dl = spec.cell_cm / (1.0 + spec.z)
    nH = n_h0(c) * (1.0 + spec.z) ** 3
    return dict(H=H, T=T, v_th=vth, dl_phys=dl, delta=H * dl / vth, n_H=nH,
                kappa_per_n1s=tau_ab_per_n1s(T, H), alpha=alpha_e(T), beta=beta_e(T),
                p_ab=p_ab(T), damping=damping(T))


def profile_of(spec):
    """"doppler" (default) or "voigt"."""
    return getattr(spec, "profile", "doppler")


def _f64(a):
    return None if a is None else np.asarray(a, dtype=np.float64)


def x_e_field(spec):
    if spec.x_e is not None:
        return _f64(spec.x_e).reshape(-1)
    return np.full(spec.ncells, float(np.float32(spec.x_e_uniform)))


def n1s_field(spec):
    sc = box_scalars(spec)
    return (1.0 - x_e_field(spec)) * sc["n_H"] * _f64(spec.overdensity).reshape(-1)


def kappa_field(spec):
    """kappa_c = tau_ab per unit Phi in cell c (Eq. (<fnu>) with the local n_1s)."""
    return box_scalars(spec)["kappa_per_n1s"] * n1s_field(spec)


def emission_weights(spec):
    """Relative emission per cell: the given source, else (x_e Delta)^2, which is
    alpha_e n_e^2 up to a per-box constant (Eq. rec0)."""
    if spec.source is not None:
        return _f64(spec.source).reshape(-1)
    m = x_e_field(spec) * _f64(spec.overdensity).reshape(-1)
    return m * m


def source_scale(spec):
    """Physical source S_c = scale * weight_c in cm^-3 s^-1."""
    if spec.source is not None:
        return 1.0
    sc = box_scalars(spec)
    return sc["alpha"] * sc["n_H"] ** 2


def velocity_field(spec):
    if spec.velocity is None:
        return None
    v = _f64(spec.velocity).reshape(3, -1)
    return v


def x_eff(spec):
    """Escape threshold X_esc + 2 max_c |U_c - <U>| (Doppler units). Past it a
    packet can never come back above -X_esc in any cell's gas frame."""
    v = velocity_field(spec)
    if v is None:
        return float(spec.x_esc)
    mean = v.mean(axis=1, keepdims=True)
    return float(spec.x_esc) + 2.0 * float(np.sqrt(((v - mean) ** 2).sum(axis=0)).max())


def x_blue(spec):
    """Voigt only: packets emitted above x_eff + (x_eff - x_esc) are not walked.
    A walked packet's gas-frame frequency never exceeds its emission frequency
    plus the velocity margin x_eff - x_esc, so every walked frequency stays
    below this bound; beyond it the Lorentz tail holds a fraction a / (pi x)
    of the emission, which meets the line core hundreds of cells away."""
    xe = x_eff(spec)
    return 2.0 * xe - float(spec.x_esc)


# --- recombination feed (Sec. III.A.1 Eq. rec, Sec. IV.B Eq. dotne-mix) -------
def feed(spec, A, E, n_packets, wing=0):
    """Per-cell net recombination rate from the absorption tallies.

    A_c is the integer weight absorbed in cell c, E the escaped weight and
    wing the part of E that the far damping wing absorbs (Voigt profile; it is
    spread like n_1s, i.e. fully mixed). The absorbed weight is a rate density
    a_c = A_c * sum(S) / (w0 N); a fraction beta/(beta+Lambda) of it
    re-ionises. The thermal term uses the Monte-Carlo Peebles factor
    C_MC = [E_true + sum(A) Lambda/(beta+Lambda)] / (w0 N), E_true = E - wing.
    In a homogeneous box this is Eq. (rec); with absorptions distributed like
    n_1s it is Eq. (dotne-mix).
    """
    sc = box_scalars(spec)
    beta, lam = sc["beta"], LAMBDA_2G
    w = emission_weights(spec)
    S = source_scale(spec) * w
    wtot = float(spec.w0) * float(n_packets)
    n1s = n1s_field(spec)
    A = np.asarray(A, dtype=np.float64).reshape(-1) + float(wing) * n1s / n1s.sum()
    a = A * S.sum() / wtot
    boltz = math.exp(-E_ALPHA / (K_B * sc["T"]))
    c_mc = (float(E) - float(wing) + A.sum() * lam / (beta + lam)) / wtot
    ndot = -S + beta / (beta + lam) * a + c_mc * beta * n1s * boltz
    a_fm = A.sum() * n1s / n1s.sum()
    with np.errstate(divide="ignore", invalid="ignore"):
        mix = np.where(a_fm > 0, A / a_fm, 0.0)
    n1s_mean = n1s.mean()
    c_mix = peebles_c(sc["T"], sc["H"], n1s_mean)
    ne = x_e_field(spec) * sc["n_H"] * _f64(spec.overdensity).reshape(-1)
    x_global = ne.sum() / (sc["n_H"] * _f64(spec.overdensity).sum())
    return dict(ndot_e=ndot, absorbed_rate=a, c_mc=c_mc, c_mix=c_mix, mix_corr=mix,
                x_e_global=x_global, boltzmann=boltz)

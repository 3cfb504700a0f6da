"""ctypes glue to the oracle's C walker (test infrastructure only).

Everything here is bookkeeping: promote inputs to FP64, call the C functions,
return numpy arrays. The arithmetic lives in mclya_oracle.c and physics.py.
"""
import ctypes as C
import math
import os
import numpy as np

from . import build as _build
from . import physics as P

_lib = None


class OrcBox(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("has_vel", C.c_int32),
                ("delta", C.c_double), ("x_eff", C.c_double), ("w0", C.c_uint64),
                ("seed", C.c_uint64), ("max_cross", C.c_int64), ("damping", C.c_double),
                ("kappa_far", C.c_double), ("x_blue", C.c_double)]


class OrcScatterParams(C.Structure):
    _fields_ = [("p_ab", C.c_double), ("p_destroy", C.c_double), ("x_inert", C.c_double),
                ("max_events", C.c_int64),
                ("fixed_x0", C.c_int32), ("pad", C.c_int32), ("x0", C.c_double),
                ("x_return", C.c_double)]


SCATTER_REC_DTYPE = np.dtype([("cell0", np.int64), ("cell_end", np.int64), ("x0", np.float64),
                              ("x_end", np.float64), ("scatterings", np.int64),
                              ("crossings", np.int64), ("escaped", np.int64), ("absorbed", np.int64),
                              ("wing", np.int64), ("dx", np.float64), ("dy", np.float64),
                              ("dz", np.float64), ("fate", np.int32), ("pad", np.int32)])


REC_DTYPE = np.dtype([("cell0", np.int64), ("fx", np.float64), ("fy", np.float64),
                      ("fz", np.float64), ("kx", np.float64), ("ky", np.float64),
                      ("kz", np.float64), ("x0", np.float64), ("crossings", np.int64),
                      ("escaped", np.int64), ("absorbed", np.int64), ("fate", np.int32),
                      ("pad", np.int32), ("wing", np.int64)])


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = C.CDLL(path)
        P_ = C.POINTER
        L.orc_philox4x32_10.argtypes = [P_(C.c_uint32), P_(C.c_uint32), P_(C.c_uint32)]
        L.orc_packet_uniforms.argtypes = [C.c_uint64, C.c_uint64, P_(C.c_double)]
        L.orc_quantize.argtypes = [C.c_int64, P_(C.c_double), P_(C.c_uint64)]
        L.orc_quantize.restype = C.c_int
        L.orc_allocate.argtypes = [C.c_int64, P_(C.c_uint64), C.c_uint64, P_(C.c_uint64)]
        L.orc_allocate.restype = C.c_int
        L.orc_transport.argtypes = [P_(OrcBox), P_(C.c_double), P_(C.c_double), P_(C.c_double),
                                    P_(C.c_double), P_(C.c_uint64), C.c_uint64, C.c_uint64,
                                    P_(C.c_int64), P_(C.c_int64), C.c_void_p, C.c_int]
        L.orc_transport.restype = C.c_int
        L.orc_trace_packet.argtypes = [P_(OrcBox), P_(C.c_double), P_(C.c_double), P_(C.c_double),
                                       P_(C.c_double), P_(C.c_uint64), C.c_uint64, P_(C.c_int64),
                                       C.c_void_p, P_(C.c_int64), P_(C.c_int64), P_(C.c_double),
                                       P_(C.c_double), P_(C.c_double), C.c_int64]
        L.orc_trace_packet.restype = C.c_int64
        L.orc_walk_packets.argtypes = [P_(OrcBox), P_(C.c_double), P_(C.c_double), P_(C.c_double),
                                       P_(C.c_double), P_(C.c_uint64), P_(C.c_uint64), C.c_int64,
                                       P_(C.c_int64), C.c_void_p]
        L.orc_walk_packets.restype = C.c_int
        L.orc_scatter.argtypes = [P_(OrcBox), P_(OrcScatterParams), P_(C.c_double), P_(C.c_double),
                                  P_(C.c_double), P_(C.c_double), P_(C.c_uint64), C.c_uint64,
                                  C.c_uint64, P_(C.c_int64), P_(C.c_int64), C.c_void_p, C.c_int]
        L.orc_scatter.restype = C.c_int
        L.orc_atom_upar_draws.argtypes = [C.c_double, C.c_double, C.c_uint64, C.c_int64, P_(C.c_double)]
        L.orc_redistribution_chain.argtypes = [C.c_double, C.c_double, C.c_uint64, C.c_uint64, C.c_int64,
                                               P_(C.c_double)]
        L.orc_profile_cdf.argtypes = [C.c_double, C.c_double]
        L.orc_profile_cdf.restype = C.c_double
        L.orc_dawson_integral.argtypes = [C.c_double]
        L.orc_dawson_integral.restype = C.c_double
        _lib = L
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype)) if a is not None else None


def philox4x32_10(ctr, key):
    """Philox4x32-10 block: 4 words of counter, 2 words of key -> 4 words."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def packet_uniforms(seed, p):
    u = np.zeros(8, dtype=np.float64)
    lib().orc_packet_uniforms(int(seed), int(p), _ptr(u, C.c_double))
    return u


def profile_cdf(x, damping=0.0):
    """The oracle's cumulative line profile at x (Doppler for damping 0, else
    Voigt to first order in the damping)."""
    return lib().orc_profile_cdf(float(damping), float(x))


def dawson(x):
    """The oracle's Dawson integral (Rybicki's series)."""
    return lib().orc_dawson_integral(float(x))


def atom_upar_draws(x, a, n, seed=1):
    """n draws of the scattering atom's parallel velocity for a photon at x."""
    out = np.zeros(int(n))
    lib().orc_atom_upar_draws(float(x), float(a), int(seed), int(n), _ptr(out, C.c_double))
    return out


def redistribution_chain(x0, a, n, seed=1, p=0):
    """Frequencies after each of n successive re-emissions of one photon."""
    out = np.zeros(int(n))
    lib().orc_redistribution_chain(float(x0), float(a), int(seed), int(p), int(n), _ptr(out, C.c_double))
    return out


def quantize(weights):
    s = np.ascontiguousarray(weights, dtype=np.float64).reshape(-1)
    q = np.zeros(s.size, dtype=np.uint64)
    rc = lib().orc_quantize(s.size, _ptr(s, C.c_double), _ptr(q, C.c_uint64))
    if rc != 0:
        raise ValueError(f"invalid emission weights (code {rc})")
    return q


def allocate(q, n_packets):
    """first[c] = first packet id of cell c, first[ncells] = N."""
    q = np.ascontiguousarray(q, dtype=np.uint64)
    first = np.zeros(q.size + 1, dtype=np.uint64)
    rc = lib().orc_allocate(q.size, _ptr(q, C.c_uint64), int(n_packets), _ptr(first, C.c_uint64))
    if rc != 0:
        raise ValueError("all emission weights are zero")
    return first


class Prepared:
    """Oracle inputs of one box: FP64 fields, scalars, allocation."""

    @classmethod
    def custom(cls, shape, kappa, weights, n_packets, seed, delta, x_eff, vel=None,
               w0=1 << 32, max_cross=1_000_000, damping=0.0, kappa_far=None, x_blue=None):
        """Walk parameters given directly (no physics): for tests of the walk."""
        self = cls.__new__(cls)
        self.spec = None
        self.w0 = int(w0)
        self.n_packets = int(n_packets)
        self.seed = int(seed)
        self.scal = None
        self.kappa = np.ascontiguousarray(kappa, dtype=np.float64).reshape(-1)
        self.vel = None if vel is None else [np.ascontiguousarray(np.asarray(vel, dtype=np.float64).reshape(3, -1)[i]) for i in range(3)]
        self.x_eff = float(x_eff)
        self.q = quantize(weights)
        self.first = allocate(self.q, self.n_packets)
        nx, ny, nz = (int(t) for t in shape)
        if kappa_far is None:
            kappa_far = float(self.kappa.mean()) if damping > 0 else 0.0
        if x_blue is None:
            x_blue = 2.0 * self.x_eff - float(x_eff) if damping > 0 else math.inf
        self.box = OrcBox(nx, ny, nz, 0 if self.vel is None else 1, float(delta), self.x_eff,
                          self.w0, self.seed, int(max_cross), float(damping), float(kappa_far),
                          float(x_blue))
        return self

    def __init__(self, spec, n_packets=None, seed=None, max_cross=1_000_000):
        self.spec = spec
        self.w0 = int(spec.w0)
        self.n_packets = int(spec.n_packets if n_packets is None else n_packets)
        self.seed = int(spec.seed if seed is None else seed)
        self.scal = P.box_scalars(spec)
        self.kappa = np.ascontiguousarray(P.kappa_field(spec))
        v = P.velocity_field(spec)
        self.vel = None if v is None else [np.ascontiguousarray(v[i]) for i in range(3)]
        self.x_eff = P.x_eff(spec)
        self.q = quantize(P.emission_weights(spec))
        self.first = allocate(self.q, self.n_packets)
        nx, ny, nz = (int(t) for t in spec.n)
        voigt = P.profile_of(spec) == "voigt"
        self.box = OrcBox(nx, ny, nz, 0 if self.vel is None else 1, self.scal["delta"],
                          self.x_eff, int(spec.w0), self.seed, int(max_cross),
                          self.scal["damping"] if voigt else 0.0,
                          float(self.kappa.mean()) if voigt else 0.0,
                          P.x_blue(spec) if voigt else math.inf)

    @property
    def emitted_per_cell(self):
        return np.diff(self.first.astype(np.int64)) * self.w0

    def _vp(self, i):
        return None if self.vel is None else _ptr(self.vel[i], C.c_double)

    def transport(self, p_begin=0, p_end=None, records=False, nthreads=None):
        """Walk packets [p_begin, p_end). Returns dict(A, escaped, crossings,
        capped, capped_weight, wing[, records]); wing is the part of the
        escaped weight that the far damping wing absorbs (Voigt only)."""
        p_end = self.n_packets if p_end is None else int(p_end)
        ncells = self.kappa.size
        A = np.zeros(ncells, dtype=np.int64)
        out = np.zeros(5, dtype=np.int64)
        recs = np.zeros(p_end - p_begin, dtype=REC_DTYPE) if records else None
        nt = int(nthreads or os.environ.get("ORACLE_THREADS", 0) or 0)
        lib().orc_transport(C.byref(self.box), _ptr(self.kappa, C.c_double), self._vp(0),
                            self._vp(1), self._vp(2), _ptr(self.first, C.c_uint64), int(p_begin),
                            int(p_end), _ptr(A, C.c_int64), _ptr(out, C.c_int64),
                            None if recs is None else recs.ctypes.data, nt)
        res = dict(A=A, escaped=int(out[0]), crossings=int(out[1]), capped=int(out[2]),
                   capped_weight=int(out[3]), wing=int(out[4]))
        if records:
            res["records"] = recs
        return res

    def scatter(self, p_ab, x_inert=300.0, max_events=1 << 31, x0=None, p_begin=0, p_end=None,
                records=False, nthreads=None, x_return=0.0, p_destroy=None):
        """Photons [p_begin, p_end) with resonant scattering (App. A): the line
        opacity is kappa / p_ab per unit of swept profile; a photon is destroyed
        with probability p_destroy (default p_ab) per scattering and lost to the
        line below -x_inert.
        Returns dict(A, escaped, crossings, capped, capped_weight, wing,
        scatterings[, records]); x0 fixes the injection frequency; x_return > 0
        stops a photon once it is scattered back inside |x| < x_return (its
        weight is then in no total: a test hook)."""
        p_end = self.n_packets if p_end is None else int(p_end)
        A = np.zeros(self.kappa.size, dtype=np.int64)
        out = np.zeros(6, dtype=np.int64)
        sp = OrcScatterParams(float(p_ab), float(p_ab if p_destroy is None else p_destroy), float(x_inert),
                              int(max_events), 0 if x0 is None else 1, 0,
                              0.0 if x0 is None else float(x0), float(x_return))
        recs = np.zeros(p_end - p_begin, dtype=SCATTER_REC_DTYPE) if records else None
        nt = int(nthreads or os.environ.get("ORACLE_THREADS", 0) or 0)
        lib().orc_scatter(C.byref(self.box), C.byref(sp), _ptr(self.kappa, C.c_double), self._vp(0),
                          self._vp(1), self._vp(2), _ptr(self.first, C.c_uint64), int(p_begin), int(p_end),
                          _ptr(A, C.c_int64), _ptr(out, C.c_int64),
                          None if recs is None else recs.ctypes.data, nt)
        res = dict(A=A, escaped=int(out[0]), crossings=int(out[1]), capped=int(out[2]),
                   capped_weight=int(out[3]), wing=int(out[4]), scatterings=int(out[5]))
        if records:
            res["records"] = recs
        return res

    def records(self, ids):
        """Per-packet records of the given packet ids (single thread)."""
        ids = np.ascontiguousarray(ids, dtype=np.uint64)
        recs = np.zeros(ids.size, dtype=REC_DTYPE)
        scratch = np.zeros(self.kappa.size, dtype=np.int64)
        lib().orc_walk_packets(C.byref(self.box), _ptr(self.kappa, C.c_double), self._vp(0),
                               self._vp(1), self._vp(2), _ptr(self.first, C.c_uint64),
                               _ptr(ids, C.c_uint64), ids.size, _ptr(scratch, C.c_int64),
                               recs.ctypes.data)
        return recs

    def trace(self, p, cap=100_000):
        """Every segment of packet p: dict(cells, deposits, x_in, x_out, length, record)."""
        cells = np.zeros(cap, dtype=np.int64)
        dep = np.zeros(cap, dtype=np.int64)
        xi = np.zeros(cap)
        xo = np.zeros(cap)
        ln = np.zeros(cap)
        A = np.zeros(self.kappa.size, dtype=np.int64)
        rec = np.zeros(1, dtype=REC_DTYPE)
        n = lib().orc_trace_packet(C.byref(self.box), _ptr(self.kappa, C.c_double), self._vp(0),
                                   self._vp(1), self._vp(2), _ptr(self.first, C.c_uint64), int(p),
                                   _ptr(A, C.c_int64), rec.ctypes.data, _ptr(cells, C.c_int64),
                                   _ptr(dep, C.c_int64), _ptr(xi, C.c_double),
                                   _ptr(xo, C.c_double), _ptr(ln, C.c_double), cap)
        if n > cap:
            raise ValueError("trace longer than cap")
        return dict(cells=cells[:n], deposits=dep[:n], x_in=xi[:n], x_out=xo[:n], length=ln[:n],
                    record=rec[0])


def run_box(spec, n_packets=None, seed=None, p_begin=0, p_end=None, records=False,
            nthreads=None, max_cross=1_000_000):
    """Full oracle run of one box: allocation, transport, conservation check."""
    prep = Prepared(spec, n_packets, seed, max_cross)
    res = prep.transport(p_begin, p_end, records, nthreads)
    res["emitted"] = prep.emitted_per_cell
    res["prepared"] = prep
    return res

"""Simulation: device-memory holder around one library context.

Uploads the fields of one or more boxes to HIP device memory (torch tensors,
kept alive as long as the context), fills the box descriptors and forwards
every operation to the C ABI. Marshalling only.
"""
import ctypes as C

import numpy as np
import torch

from . import _abi as A

TRACE_DTYPE = np.dtype([("cell0", np.uint32), ("fx", np.float32), ("fy", np.float32),
                        ("fz", np.float32), ("kx", np.float32), ("ky", np.float32),
                        ("kz", np.float32), ("x0", np.float32), ("escaped", np.int64),
                        ("absorbed", np.int64), ("crossings", np.uint32), ("fate", np.int32),
                        ("wing", np.int64)])
assert TRACE_DTYPE.itemsize == C.sizeof(A.mc_lya_packet_trace)

SCATTER_DTYPE = np.dtype([("cell0", np.uint32), ("cell_end", np.uint32), ("x0", np.float32),
                          ("x_end", np.float32), ("scatterings", np.uint64), ("crossings", np.uint32),
                          ("fate", np.int32), ("escaped", np.int64), ("absorbed", np.int64),
                          ("wing", np.int64), ("dx", np.float32), ("dy", np.float32), ("dz", np.float32),
                          ("reserved", np.int32)])
assert SCATTER_DTYPE.itemsize == C.sizeof(A.mc_lya_scatter_record)


def _dev(a, dtype, device):
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=dtype).contiguous()
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dtype).contiguous()


def desc_from_spec(spec, tensors, device="cuda"):
    """mc_lya_box_desc for a box spec (geometry, physics, fields); the device
    tensors it points to are appended to ``tensors`` to keep them alive."""
    od = _dev(spec.overdensity, torch.float32, device)
    vel = None
    vdt = A.MC_LYA_VEL_NONE
    if spec.velocity is not None:
        half = (getattr(spec.velocity, "dtype", None) in (np.float16, torch.float16))
        vel = _dev(spec.velocity, torch.float16 if half else torch.float32, device)
        vdt = A.MC_LYA_VEL_F16 if half else A.MC_LYA_VEL_F32
    xe = _dev(spec.x_e, torch.float32, device)
    src = _dev(spec.source, torch.float32, device)
    tensors.extend(t for t in (od, vel, xe, src) if t is not None)
    c = spec.cosmo
    nx, ny, nz = (int(v) for v in spec.n)
    return A.mc_lya_box_desc(
        nx=nx, ny=ny, nz=nz, vel_dtype=vdt, cell_comoving_cm=float(spec.cell_cm), z=float(spec.z),
        zeta=float(spec.zeta), x_esc=float(spec.x_esc), temp_K=float(spec.temp_K), h=c.h,
        omega_b_h2=c.omega_b_h2, omega_c_h2=c.omega_c_h2, y_p=c.y_p, t_cmb0=c.t_cmb0,
        n_eff=c.n_eff, w0=int(spec.w0), overdensity=od.data_ptr(),
        velocity=None if vel is None else vel.data_ptr(),
        x_e=None if xe is None else xe.data_ptr(), x_e_uniform=float(spec.x_e_uniform),
        profile=_PROFILES[getattr(spec, "profile", "doppler")],
        source=None if src is None else src.data_ptr())


_PROFILES = {"doppler": A.MC_LYA_PROFILE_DOPPLER, "voigt": A.MC_LYA_PROFILE_VOIGT}


class Simulation:
    """One context over ``specs`` (a box spec or a list of them). The context
    reserves its device memory here: room for ``max_packets`` packets per
    emission (default: the specs' packet counts summed) and, with
    ``evolve=True``, the buffers of the recombination history."""

    def __init__(self, specs, device="cuda", stream=None, max_packets=None, evolve=False, batch_packets=0):
        if not isinstance(specs, (list, tuple)):
            specs = [specs]
        self.specs = list(specs)
        self.device = torch.device(device)
        self._keep = []
        self._fields = []        # per box: its device field tensors (overdensity, flow, x_e, source: those given)
        descs = []
        for s in self.specs:
            keep = []
            descs.append(desc_from_spec(s, keep, self.device))
            self._fields.append(keep)
            self._keep.extend(keep)
        self._descs = descs
        self.ncells = [s.ncells for s in self.specs]
        self.total_cells = int(sum(self.ncells))
        self.cell_off = np.concatenate([[0], np.cumsum(self.ncells)]).astype(np.int64)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        if max_packets is None:
            max_packets = max(1, sum(int(s.n_packets) for s in self.specs))
        self.max_packets = int(max_packets)
        self.ctx = A.mc_lya_init(descs, self.stream, max_packets=self.max_packets, evolve=evolve,
                                 batch_packets=batch_packets)
        self.n_packets = [0] * len(self.specs)

    # -- C calls --------------------------------------------------------------
    def refresh(self):
        A.mc_lya_refresh(self.ctx)

    def load_fields(self, specs):
        """New field contents for every box (the same shapes and the same
        fields given as at init; the boxes' physics stay those of init), copied
        into the context's device arrays, then mc_lya_refresh. The packet
        seeds and counts become those of `specs`."""
        specs = list(specs) if isinstance(specs, (list, tuple)) else [specs]
        if len(specs) != len(self.specs):
            raise ValueError("load_fields needs one spec per box")
        for b, s in enumerate(specs):
            new = [a for a in (s.overdensity, s.velocity, s.x_e, s.source) if a is not None]
            if len(new) != len(self._fields[b]):
                raise ValueError("load_fields: box %d gives other fields than at init" % b)
            for t, a in zip(self._fields[b], new):
                src = a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(a))
                if tuple(src.shape) != tuple(t.shape):
                    raise ValueError("load_fields: box %d field shape %s, expected %s" % (b, tuple(src.shape),
                                                                                       tuple(t.shape)))
                t.copy_(src.to(dtype=t.dtype))
        torch.cuda.synchronize(self.device)
        self.specs = specs
        self.refresh()

    def emit(self, seeds=None, n_packets=None):
        seeds = [s.seed for s in self.specs] if seeds is None else list(seeds)
        n_packets = [s.n_packets for s in self.specs] if n_packets is None else list(n_packets)
        A.mc_lya_emit(self.ctx, seeds, n_packets)
        self.n_packets = [int(n) for n in n_packets]

    def transport(self, first=None, count=None):
        if first is None:
            A.mc_lya_transport(self.ctx)
        else:
            A.mc_lya_transport_range(self.ctx, first, count)

    def tally(self, check=True, want_emitted=True):
        """Returns dict(absorbed: int64 tensor [cells], emitted, stats, status)."""
        absorbed = torch.empty(self.total_cells, dtype=torch.int64, device=self.device)
        emitted = torch.empty_like(absorbed) if want_emitted else None
        status, stats = A.mc_lya_tally(self.ctx, absorbed.data_ptr(),
                                       None if emitted is None else emitted.data_ptr(),
                                       len(self.specs), check=check)
        return dict(absorbed=absorbed, emitted=emitted, stats=stats, status=status)

    def feed(self):
        ndot = torch.empty(self.total_cells, dtype=torch.float64, device=self.device)
        mix = torch.empty(self.total_cells, dtype=torch.float32, device=self.device)
        stats = A.mc_lya_feed(self.ctx, ndot.data_ptr(), mix.data_ptr(), len(self.specs))
        return dict(ndot_e=ndot, mix_corr=mix, stats=stats)

    def features(self):
        """Surrogate features of every cell: float32 tensor [cells, 8]."""
        out = torch.empty((self.total_cells, A.MC_LYA_MLP_FEATURES), dtype=torch.float32, device=self.device)
        A.mc_lya_features(self.ctx, out.data_ptr())
        return out

    def targets(self):
        """The surrogate's regression data from the last transport: ln M_c and
        each cell's share of its box's emission (float32 tensors [cells])."""
        y = torch.empty(self.total_cells, dtype=torch.float32, device=self.device)
        w = torch.empty_like(y)
        A.mc_lya_surrogate_targets(self.ctx, y.data_ptr(), w.data_ptr())
        return y, w

    def trace(self, first, count):
        buf = torch.empty(int(count) * TRACE_DTYPE.itemsize, dtype=torch.uint8, device=self.device)
        A.mc_lya_trace(self.ctx, first, count, buf.data_ptr())
        torch.cuda.synchronize(self.device)
        return np.frombuffer(buf.cpu().numpy().tobytes(), dtype=TRACE_DTYPE)

    def scatter(self, first=0, count=None, x_inert=0.0, p_destroy=-1.0, max_events=0, x0=None,
                x_return=0.0, records=False):
        """Resonant-scattering Monte Carlo (App. A) of photons [first,
        first + count) into the tallies; with records=True also returns one
        history per photon (numpy structured array)."""
        count = sum(self.n_packets) - first if count is None else int(count)
        o = A.mc_lya_scatter_opts(x_inert=float(x_inert), p_destroy=float(p_destroy),
                                  max_events=int(max_events), fixed_x0=0 if x0 is None else 1,
                                  x0=0.0 if x0 is None else float(x0), x_return=float(x_return))
        buf = None
        if records:
            buf = torch.empty(max(1, count) * SCATTER_DTYPE.itemsize, dtype=torch.uint8, device=self.device)
        A.mc_lya_scatter(self.ctx, first, count, o, None if buf is None else buf.data_ptr())
        if records:
            torch.cuda.synchronize(self.device)
            return np.frombuffer(buf.cpu().numpy().tobytes(), dtype=SCATTER_DTYPE)[:count]
        return None

    def x_e_field(self, b=0):
        """The device x_e array of box b (the one its descriptor points to)."""
        ptr = self._descs[b].x_e
        for t in self._keep:
            if t.data_ptr() == ptr:
                return t
        raise ValueError(f"box {b} has no x_e field")

    def evolve(self, z0, z1, n_steps, n_packets=None, seed=1):
        """Recombination history driven by the Monte Carlo: every cell's x_e
        from z0 to z1 by fourth-order Runge-Kutta in z, each stage a whole
        emit - transport - feed. Every box needs an x_e field; the fields are
        updated in place. Returns the global X_e of each box after each step,
        numpy [n_steps + 1, n_boxes]."""
        n_packets = [s.n_packets for s in self.specs] if n_packets is None else list(n_packets)
        ptrs = [self._descs[b].x_e for b in range(len(self.specs))]
        for b, p in enumerate(ptrs):
            if not p:
                raise ValueError(f"box {b} has no x_e field (give the spec an x_e array)")
        X = np.zeros((int(n_steps) + 1, len(self.specs)))
        A.mc_lya_evolve(self.ctx, z0, z1, n_steps, n_packets, seed, ptrs, X)
        self.n_packets = [0] * len(self.specs)
        return X

    def set_option(self, option, value):
        A.mc_lya_set_option(self.ctx, option, value)

    def autotune(self, reps=1):
        """Times the built-in option sets on the current emission, keeps the
        fastest; the context is left as after emit. Returns the result struct."""
        return A.mc_lya_autotune(self.ctx, reps)

    def kernel_time(self):
        return A.mc_lya_kernel_time(self.ctx)

    def close(self):
        if self.ctx:
            A.mc_lya_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

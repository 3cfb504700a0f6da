"""ctypes binding of libmclya.so: the C ABI of include/mc_lya.h, same names.

Argument marshalling only. Every step of the transport runs in the HIP
kernels of the library; nothing here computes. torch is imported first so that
the library binds to the HIP runtime torch already loaded (one runtime, shared
streams and device pointers).
"""
import ctypes as C
import os

import torch  # noqa: F401  (loads the HIP runtime the library must share)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmclya.so")

MC_LYA_OK, MC_LYA_EINVAL, MC_LYA_ENOMEM, MC_LYA_EDEVICE = 0, 1, 2, 3
MC_LYA_EOVERFLOW, MC_LYA_ESTATE, MC_LYA_ECAP, MC_LYA_ECONSERVE = 4, 5, 6, 7
MC_LYA_VEL_NONE, MC_LYA_VEL_F32, MC_LYA_VEL_F16 = 0, 1, 2
MC_LYA_PROFILE_DOPPLER, MC_LYA_PROFILE_VOIGT = 0, 1
MC_LYA_OPT_KERNEL, MC_LYA_OPT_BLOCK, MC_LYA_OPT_WAVES_PER_CU, MC_LYA_OPT_CHUNK = 1, 2, 3, 4
MC_LYA_OPT_REFILL, MC_LYA_OPT_MAX_CROSSINGS, MC_LYA_OPT_TIMING, MC_LYA_OPT_GRAPH = 5, 6, 7, 8
MC_LYA_OPT_QUEUES = 9
MC_LYA_OPT_TILE_SHARE = 10
MC_LYA_OPT_GRAPH_GENS = 11
MC_LYA_OPT_DEFER = 12
MC_LYA_OPT_TILE_CHUNK = 13
MC_LYA_OPT_TILE_REFILL = 14
MC_LYA_OPT_TAIL = 15
MC_LYA_OPT_BESIDE = 16


class mc_lya_box_desc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("vel_dtype", C.c_int32),
                ("cell_comoving_cm", C.c_double), ("z", C.c_double), ("zeta", C.c_double),
                ("x_esc", C.c_double), ("temp_K", C.c_double), ("h", C.c_double),
                ("omega_b_h2", C.c_double), ("omega_c_h2", C.c_double), ("y_p", C.c_double),
                ("t_cmb0", C.c_double), ("n_eff", C.c_double), ("w0", C.c_uint64),
                ("overdensity", C.c_void_p), ("velocity", C.c_void_p), ("x_e", C.c_void_p),
                ("x_e_uniform", C.c_float), ("profile", C.c_int32), ("source", C.c_void_p)]


class mc_lya_limits(C.Structure):
    _fields_ = [("max_packets", C.c_uint64), ("evolve", C.c_int32), ("reserved", C.c_int32),
                ("batch_packets", C.c_uint64)]


class mc_lya_box_stats(C.Structure):
    _fields_ = [("emitted", C.c_int64), ("absorbed", C.c_int64), ("escaped", C.c_int64),
                ("capped_weight", C.c_int64), ("capped_packets", C.c_int64),
                ("crossings", C.c_int64), ("packets", C.c_int64), ("conserved", C.c_int32),
                ("tiled", C.c_int32), ("delta", C.c_double), ("x_eff", C.c_double),
                ("tau_ab_mean", C.c_double), ("damping", C.c_double), ("wing", C.c_int64),
                ("scatterings", C.c_int64)]


class mc_lya_scatter_opts(C.Structure):
    _fields_ = [("x_inert", C.c_double), ("p_destroy", C.c_double), ("max_events", C.c_uint64),
                ("fixed_x0", C.c_int32), ("x0", C.c_float), ("x_return", C.c_double)]


class mc_lya_scatter_record(C.Structure):
    _fields_ = [("cell0", C.c_uint32), ("cell_end", C.c_uint32), ("x0", C.c_float), ("x_end", C.c_float),
                ("scatterings", C.c_uint64), ("crossings", C.c_uint32), ("fate", C.c_int32),
                ("escaped", C.c_int64), ("absorbed", C.c_int64), ("wing", C.c_int64),
                ("dx", C.c_float), ("dy", C.c_float), ("dz", C.c_float), ("reserved", C.c_int32)]


class mc_lya_feed_stats(C.Structure):
    _fields_ = [("c_mc", C.c_double), ("c_mix", C.c_double), ("f_escape", C.c_double),
                ("f_absorbed", C.c_double), ("x_e_global", C.c_double),
                ("ndot_e_mean", C.c_double), ("f_wing", C.c_double)]


class mc_lya_packet_trace(C.Structure):
    _fields_ = [("cell0", C.c_uint32), ("fx", C.c_float), ("fy", C.c_float), ("fz", C.c_float),
                ("kx", C.c_float), ("ky", C.c_float), ("kz", C.c_float), ("x0", C.c_float),
                ("escaped", C.c_int64), ("absorbed", C.c_int64), ("crossings", C.c_uint32),
                ("fate", C.c_int32), ("wing", C.c_int64)]


class mc_lya_tune_result(C.Structure):
    _fields_ = [("kernel", C.c_int64), ("tile_share", C.c_int64), ("block", C.c_int64),
                ("waves_per_cu", C.c_int64), ("chunk", C.c_int64), ("refill", C.c_int64),
                ("tile_chunk", C.c_int64), ("tile_refill", C.c_int64),
                ("best_ms", C.c_double), ("start_ms", C.c_double), ("trials", C.c_int32),
                ("reserved", C.c_int32)]


EXPORTS = ["mc_lya_init", "mc_lya_refresh", "mc_lya_emit", "mc_lya_transport",
           "mc_lya_transport_range", "mc_lya_tally", "mc_lya_feed", "mc_lya_trace", "mc_lya_scatter",
           "mc_lya_evolve",
           "mc_lya_set_option", "mc_lya_autotune", "mc_lya_kernel_time", "mc_lya_philox4x32_10",
           "mc_lya_probe_read",
           "mc_lya_destroy", "mc_lya_strerror", "mc_lya_last_error",
           "mc_lya_features", "mc_lya_surrogate_targets", "mc_lya_mlp_create", "mc_lya_mlp_get_params",
           "mc_lya_mlp_set_envelope", "mc_lya_mlp_forward", "mc_lya_mlp_correction", "mc_lya_mlp_gradient", "mc_lya_mlp_train_step", "mc_lya_mlp_train_steps", "mc_lya_mlp_destroy",
           "mc_lya_mlp_last_error", "mc_lya_mlp_gradient_static", "mc_lya_mlp_static_last_error"]
# the static workspace of mc_lya_mlp_gradient_static (mc_lya.h)
MC_LYA_STATIC_MAX_CELLS = (1 << 40) - 1
MC_LYA_STATIC_SCRATCH_BYTES = (1024 + 32) * 4808 * 4
MC_LYA_MLP_PARAMS = 4801
MC_LYA_MLP_FEATURES = 8


class mc_lya_adam(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float)]


class MCLyaError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{message} (status {status})")
        self.status = status


_lib = None


def load():
    """Loads libmclya.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(hipcc for gfx950); there is no fallback")
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    vp, u64, i32, i64 = C.c_void_p, C.c_uint64, C.c_int32, C.c_int64
    L.mc_lya_init.argtypes = [P(vp), P(mc_lya_box_desc), i32, P(mc_lya_limits), vp]
    L.mc_lya_refresh.argtypes = [vp]
    L.mc_lya_emit.argtypes = [vp, P(u64), P(u64)]
    L.mc_lya_transport.argtypes = [vp]
    L.mc_lya_transport_range.argtypes = [vp, u64, u64]
    L.mc_lya_tally.argtypes = [vp, vp, vp, P(mc_lya_box_stats)]
    L.mc_lya_feed.argtypes = [vp, vp, vp, P(mc_lya_feed_stats)]
    L.mc_lya_trace.argtypes = [vp, u64, u64, vp]
    L.mc_lya_scatter.argtypes = [vp, u64, u64, P(mc_lya_scatter_opts), vp]
    L.mc_lya_evolve.argtypes = [vp, C.c_double, C.c_double, i32, P(u64), u64, P(vp), P(C.c_double)]
    L.mc_lya_set_option.argtypes = [vp, i32, i64]
    L.mc_lya_autotune.argtypes = [vp, i32, P(mc_lya_tune_result)]
    L.mc_lya_kernel_time.argtypes = [vp, P(C.c_double), P(i64)]
    L.mc_lya_philox4x32_10.argtypes = [vp, vp, vp, u64, vp]
    for name in EXPORTS:
        if name in ("mc_lya_destroy", "mc_lya_strerror", "mc_lya_last_error", "mc_lya_mlp_destroy",
                    "mc_lya_mlp_last_error", "mc_lya_mlp_static_last_error"):
            continue
        getattr(L, name).restype = C.c_int
    L.mc_lya_destroy.argtypes = [vp]
    L.mc_lya_destroy.restype = None
    L.mc_lya_strerror.argtypes = [C.c_int]
    L.mc_lya_strerror.restype = C.c_char_p
    L.mc_lya_last_error.argtypes = [vp]
    L.mc_lya_last_error.restype = C.c_char_p
    fp = P(C.c_float)
    L.mc_lya_features.argtypes = [vp, vp]
    L.mc_lya_probe_read.argtypes = [vp, u64, i32, i32, vp, vp]
    L.mc_lya_surrogate_targets.argtypes = [vp, vp, vp]
    L.mc_lya_mlp_correction.argtypes = [vp, vp, u64, vp, vp, vp, vp, P(u64)]
    L.mc_lya_mlp_create.argtypes = [P(vp), fp, vp]
    L.mc_lya_mlp_get_params.argtypes = [vp, fp]
    L.mc_lya_mlp_set_envelope.argtypes = [vp, fp, fp]
    L.mc_lya_mlp_forward.argtypes = [vp, vp, u64, vp, vp, P(u64)]
    L.mc_lya_mlp_gradient.argtypes = [vp, vp, vp, vp, u64, fp, fp]
    L.mc_lya_mlp_train_step.argtypes = [vp, vp, vp, vp, u64, P(mc_lya_adam), fp]
    L.mc_lya_mlp_train_steps.argtypes = [vp, vp, vp, vp, u64, vp, u64, C.c_int, fp, C.c_float, C.c_float, C.c_float,
                                         fp]
    L.mc_lya_mlp_destroy.argtypes = [vp]
    L.mc_lya_mlp_destroy.restype = None
    L.mc_lya_mlp_last_error.argtypes = [vp]
    L.mc_lya_mlp_last_error.restype = C.c_char_p
    L.mc_lya_mlp_gradient_static.argtypes = [vp, vp, vp, vp, u64, vp, vp]
    L.mc_lya_mlp_static_last_error.argtypes = []
    L.mc_lya_mlp_static_last_error.restype = C.c_char_p
    _lib = L
    return L


def _check(status, ctx=None):
    if status != MC_LYA_OK:
        L = load()
        msg = L.mc_lya_last_error(ctx).decode() or L.mc_lya_strerror(status).decode()
        raise MCLyaError(status, msg)
    return status


def _arr(ctype, values):
    values = list(values)
    return (ctype * len(values))(*values)


def mc_lya_init(boxes, stream=None, max_packets=None, evolve=False, batch_packets=0):
    """boxes: sequence of mc_lya_box_desc; stream: hipStream_t as int (None =
    torch's current stream); max_packets / evolve / batch_packets: the
    mc_lya_limits (None: the library's defaults). Returns the context handle."""
    L = load()
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    arr = (mc_lya_box_desc * len(boxes))(*boxes)
    ctx = C.c_void_p()
    lim = None
    if max_packets is not None or evolve or batch_packets:
        lim = mc_lya_limits(max_packets=int(max_packets if max_packets is not None else 1 << 20),
                            evolve=1 if evolve else 0, reserved=0, batch_packets=int(batch_packets))
    _check(L.mc_lya_init(C.byref(ctx), arr, len(boxes), None if lim is None else C.byref(lim),
                         C.c_void_p(stream)))
    return ctx


def mc_lya_refresh(ctx):
    return _check(load().mc_lya_refresh(ctx), ctx)


def mc_lya_emit(ctx, seeds, n_packets):
    return _check(load().mc_lya_emit(ctx, _arr(C.c_uint64, seeds), _arr(C.c_uint64, n_packets)), ctx)


def mc_lya_transport(ctx):
    return _check(load().mc_lya_transport(ctx), ctx)


def mc_lya_transport_range(ctx, first, count):
    return _check(load().mc_lya_transport_range(ctx, int(first), int(count)), ctx)


def mc_lya_tally(ctx, absorbed_ptr, emitted_ptr, n_boxes, check=True):
    """Returns (status, [mc_lya_box_stats]); raises unless check is False."""
    stats = (mc_lya_box_stats * n_boxes)()
    s = load().mc_lya_tally(ctx, absorbed_ptr, emitted_ptr, stats)
    if check:
        _check(s, ctx)
    return s, list(stats)


def mc_lya_feed(ctx, ndot_ptr, mix_ptr, n_boxes):
    stats = (mc_lya_feed_stats * n_boxes)()
    _check(load().mc_lya_feed(ctx, ndot_ptr, mix_ptr, stats), ctx)
    return list(stats)


def mc_lya_trace(ctx, first, count, out_ptr):
    return _check(load().mc_lya_trace(ctx, int(first), int(count), out_ptr), ctx)


def mc_lya_scatter(ctx, first, count, opts=None, records_ptr=None):
    return _check(load().mc_lya_scatter(ctx, int(first), int(count),
                                        None if opts is None else C.byref(opts), records_ptr), ctx)


def mc_lya_evolve(ctx, z0, z1, n_steps, n_packets, seed, xe_ptrs, X_out=None):
    nb = len(n_packets)
    npk = _arr(C.c_uint64, n_packets)
    ptrs = (C.c_void_p * nb)(*[int(v) for v in xe_ptrs])
    out = None
    if X_out is not None:
        out = X_out.ctypes.data_as(C.POINTER(C.c_double))
    return _check(load().mc_lya_evolve(ctx, float(z0), float(z1), int(n_steps), npk, int(seed), ptrs, out), ctx)


def mc_lya_set_option(ctx, option, value):
    return _check(load().mc_lya_set_option(ctx, int(option), int(value)), ctx)


def mc_lya_autotune(ctx, reps=1):
    r = mc_lya_tune_result()
    _check(load().mc_lya_autotune(ctx, int(reps), C.byref(r)), ctx)
    return r


def mc_lya_kernel_time(ctx):
    ms = C.c_double()
    n = C.c_int64()
    _check(load().mc_lya_kernel_time(ctx, C.byref(ms), C.byref(n)), ctx)
    return ms.value, n.value


def mc_lya_philox4x32_10(ctr_ptr, key_ptr, out_ptr, n, stream=None):
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    return _check(load().mc_lya_philox4x32_10(ctr_ptr, key_ptr, out_ptr, int(n), C.c_void_p(stream)))


def mc_lya_destroy(ctx):
    if ctx:
        load().mc_lya_destroy(ctx)


def mc_lya_strerror(status):
    return load().mc_lya_strerror(int(status)).decode()


def mc_lya_last_error(ctx=None):
    return load().mc_lya_last_error(ctx).decode()


# ---- mixing-correction surrogate --------------------------------------------
def mc_lya_features(ctx, out_ptr):
    return _check(load().mc_lya_features(ctx, out_ptr), ctx)


def mc_lya_probe_read(buf_ptr, nbytes, passes, grid, sink_ptr, stream=None):
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    st = load().mc_lya_probe_read(buf_ptr, int(nbytes), int(passes), int(grid), sink_ptr, C.c_void_p(stream))
    if st != MC_LYA_OK:
        raise MCLyaError(st, load().mc_lya_strerror(st).decode())


def mc_lya_surrogate_targets(ctx, y_ptr, w_ptr):
    return _check(load().mc_lya_surrogate_targets(ctx, y_ptr, w_ptr), ctx)


def _check_mlp(status, mlp=None):
    if status != MC_LYA_OK:
        L = load()
        msg = L.mc_lya_mlp_last_error(mlp).decode() or L.mc_lya_strerror(status).decode()
        raise MCLyaError(status, msg)
    return status


def mc_lya_mlp_create(params, stream=None):
    """params: sequence of MC_LYA_MLP_PARAMS floats; returns the handle."""
    L = load()
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    arr = (C.c_float * MC_LYA_MLP_PARAMS)(*[float(x) for x in params])
    h = C.c_void_p()
    _check_mlp(L.mc_lya_mlp_create(C.byref(h), arr, C.c_void_p(stream)))
    return h


def mc_lya_mlp_get_params(mlp):
    arr = (C.c_float * MC_LYA_MLP_PARAMS)()
    _check_mlp(load().mc_lya_mlp_get_params(mlp, arr), mlp)
    return list(arr)


def mc_lya_mlp_set_envelope(mlp, lo, hi):
    if lo is None:
        return _check_mlp(load().mc_lya_mlp_set_envelope(mlp, None, None), mlp)
    return _check_mlp(load().mc_lya_mlp_set_envelope(mlp, _arr(C.c_float, lo), _arr(C.c_float, hi)), mlp)


def mc_lya_mlp_forward(mlp, feat_ptr, n, y_ptr, outside_ptr=None, count=False):
    c = C.c_uint64()
    _check_mlp(load().mc_lya_mlp_forward(mlp, feat_ptr, int(n), y_ptr, outside_ptr,
                                         C.byref(c) if count else None), mlp)
    return c.value if count else None


def mc_lya_mlp_correction(mlp, feat_ptr, n, fallback_ptr, y_ptr, m_ptr, outside_ptr=None, count=False):
    c = C.c_uint64()
    _check_mlp(load().mc_lya_mlp_correction(mlp, feat_ptr, int(n), fallback_ptr, y_ptr, m_ptr, outside_ptr,
                                            C.byref(c) if count else None), mlp)
    return c.value if count else None


def mc_lya_mlp_gradient(mlp, feat_ptr, t_ptr, w_ptr, n):
    g = (C.c_float * MC_LYA_MLP_PARAMS)()
    loss = C.c_float()
    _check_mlp(load().mc_lya_mlp_gradient(mlp, feat_ptr, t_ptr, w_ptr, int(n), g, C.byref(loss)), mlp)
    return list(g), loss.value


def mc_lya_mlp_train_step(mlp, feat_ptr, t_ptr, w_ptr, n, lr, beta1=0.9, beta2=0.999, eps=1e-8, want_loss=False):
    hp = mc_lya_adam(lr, beta1, beta2, eps)
    loss = C.c_float()
    _check_mlp(load().mc_lya_mlp_train_step(mlp, feat_ptr, t_ptr, w_ptr, int(n), C.byref(hp),
                                            C.byref(loss) if want_loss else None), mlp)
    return loss.value if want_loss else None


def mc_lya_mlp_train_steps(mlp, feat_ptr, t_ptr, w_ptr, n_cells, idx_ptr, batch, lrs, beta1=0.9, beta2=0.999,
                           eps=1e-8, want_losses=False):
    k = len(lrs)
    lr = (C.c_float * max(1, k))(*[float(x) for x in lrs])
    out = (C.c_float * max(1, k))() if want_losses else None
    _check_mlp(load().mc_lya_mlp_train_steps(mlp, feat_ptr, t_ptr, w_ptr, int(n_cells), idx_ptr, int(batch), k, lr,
                                             beta1, beta2, eps, out), mlp)
    return [float(out[i]) for i in range(k)] if want_losses else None


def mc_lya_mlp_destroy(mlp):
    if mlp:
        load().mc_lya_mlp_destroy(mlp)


def mc_lya_mlp_gradient_static(params_ptr, feat_ptr, t_ptr, w_ptr, n, grad_out_ptr, stream=None):
    """The allocation-free gradient: every pointer is device memory; grad_out
    receives MC_LYA_MLP_PARAMS + 2 floats. Asynchronous on `stream`."""
    L = load()
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    status = L.mc_lya_mlp_gradient_static(params_ptr, feat_ptr, t_ptr, w_ptr, int(n), grad_out_ptr,
                                          C.c_void_p(stream))
    if status != MC_LYA_OK:
        msg = L.mc_lya_mlp_static_last_error().decode() or L.mc_lya_strerror(status).decode()
        raise MCLyaError(status, msg)

"""The C-ABI library loads and exports every declared symbol; host-side
argument checks work without a GPU (no compute calls)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mc_lya.h")


def _lib():
    import paper_2312_11448_amd as M
    if not os.path.exists(M.LIB_PATH):
        from paper_2312_11448_amd import build
        build.build()
    return M


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(mc_lya_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    M = _lib()
    L = M.load()
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(M._abi.EXPORTS)


def test_struct_sizes_match_header_layout():
    M = _lib()
    assert C.sizeof(M.mc_lya_packet_trace) == 64
    assert C.sizeof(M.mc_lya_box_stats) == 112
    assert C.sizeof(M.mc_lya_scatter_record) == 72
    assert C.sizeof(M.mc_lya_scatter_opts) == 40
    assert C.sizeof(M.mc_lya_feed_stats) == 56
    assert C.sizeof(M.mc_lya_tune_result) == 88
    assert C.sizeof(M.mc_lya_limits) == 24
    # 4 int32, 11 doubles, w0, 3 pointers, float + int32, 1 pointer
    assert C.sizeof(M.mc_lya_box_desc) == 16 + 88 + 8 + 24 + 8 + 8


def test_status_strings():
    M = _lib()
    assert M.mc_lya_strerror(0) == "ok"
    assert "cap" in M.mc_lya_strerror(M.MC_LYA_ECAP)
    assert M.mc_lya_strerror(99) == "unknown status"


def _desc(M, **kw):
    d = dict(nx=4, ny=4, nz=4, vel_dtype=0, cell_comoving_cm=2.9e20, z=1100.0, zeta=1.0,
             x_esc=6.0, temp_K=3000.0, h=0.67, omega_b_h2=0.0224, omega_c_h2=0.12, y_p=0.24,
             t_cmb0=2.7255, n_eff=3.046, w0=1 << 31, overdensity=0x1000, velocity=None,
             x_e=None, x_e_uniform=0.1, profile=0, source=None)
    d.update(kw)
    return M.mc_lya_box_desc(**d)


@pytest.mark.parametrize("bad,msg", [(dict(nx=0), "grid"), (dict(z=-1.0), "z must"),
                                     (dict(zeta=0.0), "zeta"), (dict(w0=0), "w0"), (dict(w0=1 << 32), "w0"),
                                     (dict(overdensity=None), "overdensity"),
                                     (dict(vel_dtype=1), "velocity"),
                                     (dict(x_e_uniform=1.5), "x_e_uniform"),
                                     (dict(temp_K=float("nan")), "temp_K"),
                                     (dict(profile=3), "profile")])
def test_init_rejects_bad_descriptors_before_any_device_call(bad, msg):
    M = _lib()
    with pytest.raises(M.MCLyaError) as e:
        M.mc_lya_init([_desc(M, **bad)], stream=0)
    assert e.value.status == M.MC_LYA_EINVAL
    assert msg in str(e.value)


@pytest.mark.parametrize("limits,msg", [(dict(max_packets=0), "max_packets"),
                                        (dict(max_packets=1 << 40), "max_packets"),
                                        (dict(max_packets=10, evolve=2), "evolve"),
                                        (dict(max_packets=10, reserved=1), "reserved")])
def test_init_rejects_bad_limits_before_any_device_call(limits, msg):
    M = _lib()
    L = M.load()
    lim = M.mc_lya_limits(**limits)
    arr = (M.mc_lya_box_desc * 1)(_desc(M))
    ctx = C.c_void_p()
    assert L.mc_lya_init(C.byref(ctx), arr, 1, C.byref(lim), None) == M.MC_LYA_EINVAL
    assert not ctx.value
    assert msg in L.mc_lya_last_error(None).decode()


def test_null_context_calls():
    M = _lib()
    L = M.load()
    assert L.mc_lya_transport(None) == M.MC_LYA_EINVAL
    assert L.mc_lya_set_option(None, 1, 0) == M.MC_LYA_EINVAL
    assert L.mc_lya_emit(None, None, None) == M.MC_LYA_EINVAL
    L.mc_lya_destroy(None)


def test_null_network_calls():
    """The network's entry points refuse a null handle before any device
    work (the training entry points included)."""
    M = _lib()
    L = M.load()
    lr = (C.c_float * 1)(1e-3)
    assert L.mc_lya_mlp_train_steps(None, None, None, None, 0, None, 0, 1, lr, 0.9, 0.999, 1e-8, None) \
        == M.MC_LYA_EINVAL
    hp = M.mc_lya_adam(1e-3, 0.9, 0.999, 1e-8)
    assert L.mc_lya_mlp_train_step(None, None, None, None, 0, C.byref(hp), None) == M.MC_LYA_EINVAL
    assert L.mc_lya_mlp_forward(None, None, 0, None, None, None) == M.MC_LYA_EINVAL
    L.mc_lya_mlp_destroy(None)

"""Python binding of the C ABI in include/lbm.h (argument marshalling only).

Every function here has the name of the C entry point it calls and does no
arithmetic of the method: all of it runs in the HIP library.  PyTorch provides
device memory (tensors whose data pointers are handed over) and the stream.
The library must have been built (``paper_2005_08674_amd.build.build()``);
loading fails loudly if it is missing -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "_lib", "liblbm.so")

LBM_OK = 0
LBM_ERR_ARG = -1
LBM_ERR_HIP = -2
LBM_ERR_STATE = -3
LBM_ERR_NONFINITE = -4
LBM_ERR_UNSUPPORTED = -5

LBM_BC_PERIODIC = 0
LBM_BC_NSBC = 1
LBM_BC_VELOCITY = 2

LBM_STORE_F64 = 0
LBM_STORE_F32 = 1
LBM_STORE_F16DEV = 2
LBM_STORE_BF16DEV = 3
LBM_F16_EXP_AUTO = -1000
LBM_COLL_BGK = 0
LBM_COLL_MRT = 1

STORE_NAMES = {"f64": LBM_STORE_F64, "f32": LBM_STORE_F32, "f16": LBM_STORE_F16DEV, "bf16": LBM_STORE_BF16DEV}


class LbmError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where} failed ({code}): {msg}")
        self.code = code


class lbm_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("tau", ctypes.c_double), ("rho0", ctypes.c_double),
                ("bc", ctypes.c_int32 * 4),
                ("gamma", ctypes.c_double),
                ("store", ctypes.c_int32), ("corr_mode", ctypes.c_int32),
                ("grad_order", ctypes.c_int32), ("corner_mode", ctypes.c_int32),
                ("f16_exp", ctypes.c_int32), ("collision", ctypes.c_int32),
                ("ubase", ctypes.c_double * 2),
                ("omega_e", ctypes.c_double), ("omega_eps", ctypes.c_double), ("omega_q", ctypes.c_double)]


_lib = None

_P = ctypes.c_void_p
_SIGS = {
    "lbm_params_default": [_P],
    "lbm_workspace_bytes": [_P, _P],
    "lbm_init": [_P, _P, _P, ctypes.c_size_t, _P, _P, _P, _P],
    "lbm_set_farfield": [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double],
    "lbm_set_velocity_edge": [_P, ctypes.c_double, ctypes.c_double],
    "lbm_step": [_P, ctypes.c_int32],
    "lbm_moments": [_P, _P, _P, _P, ctypes.c_int, ctypes.c_int],
    "lbm_time": [_P, _P],
    "lbm_get_populations": [_P, _P],
    "lbm_set_populations": [_P, _P],
    "lbm_check_finite": [_P, _P],
    "lbm_f16_exp": [_P, _P],
    "lbm_energy": [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double, _P],
    "lbm_energy_noalloc": [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double, _P],
    "lbm_tile_count": [],
    "lbm_tile_describe": [ctypes.c_int32, _P, ctypes.c_size_t],
    "lbm_set_tile": [_P, ctypes.c_int32],
    "lbm_get_tile": [_P, _P],
    "lbm_autotune": [_P, ctypes.c_int32, _P, _P],
    "lbm_enable_timing": [_P, ctypes.c_int],
    "lbm_kernel_times": [_P, _P, _P, _P, _P],
    "lbm_bulk_traffic": [_P, _P, _P],
    "lbm_set_overlap": [_P, ctypes.c_int],
    "lbm_set_fused": [_P, ctypes.c_int],
    "lbm_stream_copy": [_P, _P, ctypes.c_size_t, _P],
    "lbm_two_step_count": [],
    "lbm_two_step_describe": [ctypes.c_int32, _P, ctypes.c_size_t],
    "lbm_two_step_steps": [ctypes.c_int32, _P],
    "lbm_set_two_step": [_P, ctypes.c_int32],
    "lbm_get_two_step": [_P, _P],
    "lbm_autotune_two_step": [_P, ctypes.c_int32, _P, _P],
    "lbm_two_step_times": [_P, _P, _P],
    "lbm_save_bytes": [_P, _P],
    "lbm_save": [_P, _P, ctypes.c_size_t],
    "lbm_load": [_P, _P, ctypes.c_size_t],
    "lbm_set_debug": [ctypes.c_int32],
    "lbm_debug_level": [_P],
    # ensemble (include/lbm_ensemble.h)
    "lbm_ens_workspace_bytes": [_P, ctypes.c_int32, _P],
    "lbm_ens_init": [_P, _P, ctypes.c_int32, _P, ctypes.c_size_t, _P, _P, _P, _P],
    "lbm_ens_set_farfield": [_P, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                             ctypes.c_double],
    "lbm_ens_set_velocity_edge": [_P, ctypes.c_int32, ctypes.c_double, ctypes.c_double],
    "lbm_ens_step": [_P, ctypes.c_int32],
    "lbm_ens_step_graph": [_P, ctypes.c_int32, _P, ctypes.c_size_t, ctypes.c_int32],
    "lbm_ens_set_log_sites": [_P, _P, _P, ctypes.c_int32],
    "lbm_ens_log_bytes": [_P, ctypes.c_int32, ctypes.c_int32, _P],
    "lbm_ens_set_fused": [_P, ctypes.c_int],
    "lbm_ens_moments": [_P, ctypes.c_int32, _P, _P, _P, ctypes.c_int, ctypes.c_int],
    "lbm_ens_get_populations": [_P, ctypes.c_int32, _P],
    "lbm_ens_time": [_P, _P],
    "lbm_ens_info": [_P, _P, _P, _P],
    "lbm_ens_shape_count": [],
    "lbm_ens_shape_describe": [ctypes.c_int32, _P, ctypes.c_size_t],
    "lbm_ens_set_shape": [_P, ctypes.c_int32],
    "lbm_ens_autotune": [_P, ctypes.c_int32, _P, _P],
    "lbm_ens_set_two_step": [_P, ctypes.c_int32],
    "lbm_ens_get_two_step": [_P, _P],
    "lbm_ens_autotune_two_step": [_P, ctypes.c_int32, _P, _P],
    "lbm3d_params_default": [_P],
    "lbm3d_workspace_bytes": [_P, _P],
    "lbm3d_init": [_P, _P, _P, ctypes.c_size_t, _P, _P, _P, _P, _P],
    "lbm3d_set_farfield": [_P] + [ctypes.c_double] * 5,
    "lbm3d_step": [_P, ctypes.c_int32],
    "lbm3d_moments": [_P, _P],
    "lbm3d_time": [_P, _P],
    "lbm3d_get_populations": [_P, _P],
    "lbm3d_set_populations": [_P, _P],
    "lbm3d_check_finite": [_P, _P],
    "lbm3d_f16_exp": [_P, _P],
    "lbm3d_shape_count": [],
    "lbm3d_shape_describe": [ctypes.c_int32, _P, ctypes.c_size_t],
    "lbm3d_set_shape": [_P, ctypes.c_int32],
    "lbm3d_autotune": [_P, ctypes.c_int32, _P, _P],
    # learned closure (include/lbm_closure.h)
    "lbm_closure_net_bytes": [_P],
    "lbm_set_closure": [_P, _P, ctypes.c_int],
    "lbm_closure_features": [_P, _P, ctypes.c_int32, _P, _P],
    "lbm_closure_moments": [_P, _P, ctypes.c_int32, _P, _P],
    "lbm_ens_set_closure": [_P, ctypes.c_int32, _P, ctypes.c_int],
    "lbm_ens_closure_features": [_P, _P, ctypes.c_int32, _P, _P],
    "lbm_ens_closure_moments": [_P, _P, ctypes.c_int32, _P, _P],
    "lbm_mlp_workspace_bytes": [ctypes.c_int32, _P],
    "lbm_mlp_init": [_P, ctypes.c_int32, _P, ctypes.c_size_t, _P, _P],
    "lbm_mlp_fit_normalization": [_P, _P, _P, ctypes.c_int64],
    "lbm_mlp_pack": [_P, _P, _P, ctypes.c_int64, _P, _P],
    "lbm_mlp_train_step": [_P, _P, _P, ctypes.c_int64, _P, ctypes.c_int32, ctypes.c_float, _P],
    "lbm_mlp_grads": [_P, _P, _P, ctypes.c_int64, _P, ctypes.c_int32, _P, _P],
    "lbm_mlp_forward": [_P, _P, ctypes.c_int64, _P],
    "lbm_mlp_params": [_P, _P],
    "lbm_mlp_normalization": [_P, _P, _P, _P],
    "lbm_mlp_export": [_P, ctypes.c_float, ctypes.c_float, ctypes.c_float, _P],
    "lbm_mlp_set_normalization": [_P, _P, _P, _P],
}


def load():
    """Load liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run paper_2005_08674_amd.build.build())")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.lbm_last_error.argtypes = []
    lib.lbm_last_error.restype = ctypes.c_char_p
    lib.lbm_destroy.argtypes = [_P]
    lib.lbm_destroy.restype = None
    lib.lbm_ens_destroy.argtypes = [_P]
    lib.lbm_ens_destroy.restype = None
    lib.lbm_mlp_destroy.argtypes = [_P]
    lib.lbm_mlp_destroy.restype = None
    lib.lbm3d_destroy.argtypes = [_P]
    lib.lbm3d_destroy.restype = None
    _lib = lib
    return lib


def exported_symbols():
    return list(_SIGS) + ["lbm_last_error", "lbm_destroy", "lbm_ens_destroy", "lbm_mlp_destroy", "lbm3d_destroy"]


def _check(rc: int, where: str):
    if rc != LBM_OK:
        raise LbmError(rc, where, lbm_last_error())
    return rc


def lbm_last_error() -> str:
    return load().lbm_last_error().decode()


def lbm_params_default() -> lbm_params:
    p = lbm_params()
    _check(load().lbm_params_default(ctypes.byref(p)), "lbm_params_default")
    return p


def lbm_workspace_bytes(p: lbm_params) -> int:
    n = ctypes.c_size_t()
    _check(load().lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(n)), "lbm_workspace_bytes")
    return n.value


def lbm_init(p: lbm_params, workspace_ptr: int, nbytes: int, drho_ptr: int, ux_ptr: int, uy_ptr: int,
             stream_ptr: int):
    ctx = ctypes.c_void_p()
    _check(load().lbm_init(ctypes.byref(ctx), ctypes.byref(p), workspace_ptr, nbytes, drho_ptr, ux_ptr, uy_ptr,
                           stream_ptr), "lbm_init")
    return ctx


def lbm_set_farfield(ctx, beta, rho_ref, ux_ref, uy_ref):
    _check(load().lbm_set_farfield(ctx, beta, rho_ref, ux_ref, uy_ref), "lbm_set_farfield")


def lbm_set_velocity_edge(ctx, ux, uy):
    _check(load().lbm_set_velocity_edge(ctx, float(ux), float(uy)), "lbm_set_velocity_edge")


def lbm_step(ctx, n: int):
    _check(load().lbm_step(ctx, int(n)), "lbm_step")


def lbm_moments(ctx, drho_ptr, ux_ptr, uy_ptr, out_f64: bool = True, deviation: bool = True):
    _check(load().lbm_moments(ctx, drho_ptr, ux_ptr, uy_ptr, int(out_f64), int(deviation)), "lbm_moments")


def lbm_time(ctx) -> int:
    t = ctypes.c_int64()
    _check(load().lbm_time(ctx, ctypes.byref(t)), "lbm_time")
    return t.value


def lbm_destroy(ctx):
    load().lbm_destroy(ctx)


def lbm_get_populations(ctx, g_ptr):
    _check(load().lbm_get_populations(ctx, g_ptr), "lbm_get_populations")


def lbm_set_populations(ctx, g_ptr):
    _check(load().lbm_set_populations(ctx, g_ptr), "lbm_set_populations")


def lbm_save_bytes(ctx) -> int:
    n = ctypes.c_size_t()
    _check(load().lbm_save_bytes(ctx, ctypes.byref(n)), "lbm_save_bytes")
    return n.value


def lbm_save(ctx) -> bytes:
    """The context's checkpoint (header + populations as stored) as host bytes."""
    n = lbm_save_bytes(ctx)
    buf = ctypes.create_string_buffer(n)
    _check(load().lbm_save(ctx, buf, n), "lbm_save")
    return buf.raw


def lbm_load(ctx, data: bytes):
    buf = ctypes.create_string_buffer(bytes(data), len(data))
    _check(load().lbm_load(ctx, buf, len(data)), "lbm_load")


def lbm_set_debug(level: int):
    _check(load().lbm_set_debug(int(level)), "lbm_set_debug")


def lbm_debug_level() -> int:
    k = ctypes.c_int32()
    _check(load().lbm_debug_level(ctypes.byref(k)), "lbm_debug_level")
    return k.value


def lbm_check_finite(ctx) -> bool:
    ok = ctypes.c_int()
    rc = load().lbm_check_finite(ctx, ctypes.byref(ok))
    if rc not in (LBM_OK, LBM_ERR_NONFINITE):
        _check(rc, "lbm_check_finite")
    return bool(ok.value)


def lbm_f16_exp(ctx) -> int:
    k = ctypes.c_int32()
    _check(load().lbm_f16_exp(ctx, ctypes.byref(k)), "lbm_f16_exp")
    return k.value


def lbm_energy(test_ctx, ref_ctx, x_off, y_off, ux_ref, uy_ref, out_ptr):
    _check(load().lbm_energy(test_ctx, ref_ctx, int(x_off), int(y_off), float(ux_ref), float(uy_ref), out_ptr),
           "lbm_energy")


def lbm_energy_noalloc(test_ctx, ref_ctx, x_off, y_off, ux_ref, uy_ref, out_ptr):
    _check(load().lbm_energy_noalloc(test_ctx, ref_ctx, int(x_off), int(y_off), float(ux_ref), float(uy_ref),
                                     out_ptr), "lbm_energy_noalloc")


def lbm_tile_count() -> int:
    return int(load().lbm_tile_count())


def lbm_tile_describe(tile_id: int) -> str:
    buf = ctypes.create_string_buffer(64)
    _check(load().lbm_tile_describe(int(tile_id), buf, 64), "lbm_tile_describe")
    return buf.value.decode()


def lbm_set_tile(ctx, tile_id: int):
    _check(load().lbm_set_tile(ctx, int(tile_id)), "lbm_set_tile")


def lbm_get_tile(ctx) -> int:
    t = ctypes.c_int32()
    _check(load().lbm_get_tile(ctx, ctypes.byref(t)), "lbm_get_tile")
    return t.value


def lbm_autotune(ctx, reps: int = 5):
    best = ctypes.c_int32()
    n = lbm_tile_count()
    times = (ctypes.c_float * n)()
    _check(load().lbm_autotune(ctx, int(reps), ctypes.byref(best), times), "lbm_autotune")
    return best.value, list(times)


def lbm_enable_timing(ctx, on: bool):
    _check(load().lbm_enable_timing(ctx, int(on)), "lbm_enable_timing")


def lbm_kernel_times(ctx):
    bm, em = ctypes.c_double(), ctypes.c_double()
    bn, en = ctypes.c_int64(), ctypes.c_int64()
    _check(load().lbm_kernel_times(ctx, ctypes.byref(bm), ctypes.byref(bn), ctypes.byref(em), ctypes.byref(en)),
           "lbm_kernel_times")
    return bm.value, bn.value, em.value, en.value


def lbm_two_step_count() -> int:
    return int(load().lbm_two_step_count())


def lbm_two_step_describe(shape_id: int) -> str:
    buf = ctypes.create_string_buffer(64)
    _check(load().lbm_two_step_describe(int(shape_id), buf, 64), "lbm_two_step_describe")
    return buf.value.decode()


def lbm_two_step_steps(shape_id: int) -> int:
    """Steps one launch of multi-step shape `shape_id` advances (2 or 3)."""
    k = ctypes.c_int32()
    _check(load().lbm_two_step_steps(int(shape_id), ctypes.byref(k)), "lbm_two_step_steps")
    return k.value


def lbm_set_two_step(ctx, shape_id: int):
    _check(load().lbm_set_two_step(ctx, int(shape_id)), "lbm_set_two_step")


def lbm_get_two_step(ctx) -> int:
    t = ctypes.c_int32()
    _check(load().lbm_get_two_step(ctx, ctypes.byref(t)), "lbm_get_two_step")
    return t.value


def lbm_autotune_two_step(ctx, reps: int = 5):
    best = ctypes.c_int32()
    n = lbm_two_step_count()
    times = (ctypes.c_float * n)()
    _check(load().lbm_autotune_two_step(ctx, int(reps), ctypes.byref(best), times), "lbm_autotune_two_step")
    return best.value, list(times)


def lbm_two_step_times(ctx):
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(load().lbm_two_step_times(ctx, ctypes.byref(ms), ctypes.byref(n)), "lbm_two_step_times")
    return ms.value, n.value


def lbm_set_fused(ctx, on: bool):
    _check(load().lbm_set_fused(ctx, int(on)), "lbm_set_fused")


def lbm_set_overlap(ctx, on: bool):
    _check(load().lbm_set_overlap(ctx, int(on)), "lbm_set_overlap")


def lbm_stream_copy(src_ptr, dst_ptr, nbytes, stream_ptr):
    _check(load().lbm_stream_copy(src_ptr, dst_ptr, int(nbytes), stream_ptr), "lbm_stream_copy")


def lbm_bulk_traffic(ctx):
    b, n = ctypes.c_int64(), ctypes.c_int64()
    _check(load().lbm_bulk_traffic(ctx, ctypes.byref(b), ctypes.byref(n)), "lbm_bulk_traffic")
    return b.value, n.value


# ------------------------------------------------------------------ ensemble

def lbm_ens_workspace_bytes(members) -> int:
    arr = (lbm_params * len(members))(*members)
    n = ctypes.c_size_t()
    _check(load().lbm_ens_workspace_bytes(arr, len(members), ctypes.byref(n)), "lbm_ens_workspace_bytes")
    return n.value


def lbm_ens_init(members, workspace_ptr, nbytes, drho_ptr, ux_ptr, uy_ptr, stream_ptr):
    arr = (lbm_params * len(members))(*members)
    ens = ctypes.c_void_p()
    _check(load().lbm_ens_init(ctypes.byref(ens), arr, len(members), workspace_ptr, nbytes, drho_ptr, ux_ptr,
                               uy_ptr, stream_ptr), "lbm_ens_init")
    return ens


def lbm_ens_set_farfield(ens, member, beta, rho_ref, ux_ref, uy_ref):
    _check(load().lbm_ens_set_farfield(ens, int(member), beta, rho_ref, ux_ref, uy_ref), "lbm_ens_set_farfield")


def lbm_ens_set_velocity_edge(ens, member, ux, uy):
    _check(load().lbm_ens_set_velocity_edge(ens, int(member), float(ux), float(uy)), "lbm_ens_set_velocity_edge")


def lbm_ens_step(ens, n: int):
    _check(load().lbm_ens_step(ens, int(n)), "lbm_ens_step")


LBM_ENS_LOG_FLOATS = 103


def lbm_ens_step_graph(ens, n: int, log_ptr=None, log_bytes: int = 0, log_every: int = 0):
    _check(load().lbm_ens_step_graph(ens, int(n), log_ptr, int(log_bytes), int(log_every)), "lbm_ens_step_graph")


def lbm_ens_set_log_sites(ens, member_sites_ptr, twin_sites_ptr, n: int):
    _check(load().lbm_ens_set_log_sites(ens, member_sites_ptr, twin_sites_ptr, int(n)), "lbm_ens_set_log_sites")


def lbm_ens_log_bytes(ens, n: int, log_every: int) -> int:
    b = ctypes.c_size_t()
    _check(load().lbm_ens_log_bytes(ens, int(n), int(log_every), ctypes.byref(b)), "lbm_ens_log_bytes")
    return b.value


def lbm_ens_set_fused(ens, on: bool):
    _check(load().lbm_ens_set_fused(ens, int(on)), "lbm_ens_set_fused")


def lbm_ens_moments(ens, member, drho_ptr, ux_ptr, uy_ptr, out_f64=True, deviation=True):
    _check(load().lbm_ens_moments(ens, int(member), drho_ptr, ux_ptr, uy_ptr, int(out_f64), int(deviation)),
           "lbm_ens_moments")


def lbm_ens_get_populations(ens, member, g_ptr):
    _check(load().lbm_ens_get_populations(ens, int(member), g_ptr), "lbm_ens_get_populations")


def lbm_ens_time(ens) -> int:
    t = ctypes.c_int64()
    _check(load().lbm_ens_time(ens, ctypes.byref(t)), "lbm_ens_time")
    return t.value


def lbm_ens_info(ens):
    n, b, e = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
    _check(load().lbm_ens_info(ens, ctypes.byref(n), ctypes.byref(b), ctypes.byref(e)), "lbm_ens_info")
    return n.value, b.value, e.value


def lbm_ens_shape_count() -> int:
    return int(load().lbm_ens_shape_count())


def lbm_ens_shape_describe(shape_id: int) -> str:
    buf = ctypes.create_string_buffer(64)
    _check(load().lbm_ens_shape_describe(int(shape_id), buf, 64), "lbm_ens_shape_describe")
    return buf.value.decode()


def lbm_ens_set_shape(ens, shape_id: int):
    _check(load().lbm_ens_set_shape(ens, int(shape_id)), "lbm_ens_set_shape")


def lbm_ens_autotune(ens, reps: int = 5):
    best = ctypes.c_int32()
    times = (ctypes.c_float * lbm_ens_shape_count())()
    _check(load().lbm_ens_autotune(ens, int(reps), ctypes.byref(best), times), "lbm_ens_autotune")
    return best.value, list(times)


def lbm_ens_set_two_step(ens, shape_id: int):
    _check(load().lbm_ens_set_two_step(ens, int(shape_id)), "lbm_ens_set_two_step")


def lbm_ens_get_two_step(ens) -> int:
    v = ctypes.c_int32()
    _check(load().lbm_ens_get_two_step(ens, ctypes.byref(v)), "lbm_ens_get_two_step")
    return v.value


def lbm_ens_autotune_two_step(ens, reps: int = 5):
    best = ctypes.c_int32()
    times = (ctypes.c_float * lbm_two_step_count())()
    _check(load().lbm_ens_autotune_two_step(ens, int(reps), ctypes.byref(best), times), "lbm_ens_autotune_two_step")
    return best.value, list(times)


def lbm_ens_destroy(ens):
    load().lbm_ens_destroy(ens)


# ------------------------------------------------------------------ closure

LBM_MLP_INPUTS = 96
LBM_MLP_FEATURES = 87
LBM_MLP_NPARAM = 10563


def lbm_closure_net_bytes() -> int:
    n = ctypes.c_size_t()
    _check(load().lbm_closure_net_bytes(ctypes.byref(n)), "lbm_closure_net_bytes")
    return n.value


def lbm_set_closure(ctx, net_ptr, mode: int):
    _check(load().lbm_set_closure(ctx, net_ptr, int(mode)), "lbm_set_closure")


def lbm_closure_features(ctx, sites_ptr, n, feat_ptr, mc_ptr):
    _check(load().lbm_closure_features(ctx, sites_ptr, int(n), feat_ptr, mc_ptr), "lbm_closure_features")


def lbm_closure_moments(ctx, sites_ptr, n, sub_ptr, m_ptr):
    _check(load().lbm_closure_moments(ctx, sites_ptr, int(n), sub_ptr, m_ptr), "lbm_closure_moments")


def lbm_ens_set_closure(ens, member, net_ptr, mode: int):
    _check(load().lbm_ens_set_closure(ens, int(member), net_ptr, int(mode)), "lbm_ens_set_closure")


def lbm_ens_closure_features(ens, sites_ptr, n, feat_ptr, mc_ptr):
    _check(load().lbm_ens_closure_features(ens, sites_ptr, int(n), feat_ptr, mc_ptr), "lbm_ens_closure_features")


def lbm_ens_closure_moments(ens, sites_ptr, n, sub_ptr, m_ptr):
    _check(load().lbm_ens_closure_moments(ens, sites_ptr, int(n), sub_ptr, m_ptr), "lbm_ens_closure_moments")


def lbm_mlp_workspace_bytes(max_batch: int) -> int:
    n = ctypes.c_size_t()
    _check(load().lbm_mlp_workspace_bytes(int(max_batch), ctypes.byref(n)), "lbm_mlp_workspace_bytes")
    return n.value


def lbm_mlp_init(max_batch, workspace_ptr, nbytes, params_ptr, stream_ptr):
    m = ctypes.c_void_p()
    _check(load().lbm_mlp_init(ctypes.byref(m), int(max_batch), workspace_ptr, nbytes, params_ptr, stream_ptr),
           "lbm_mlp_init")
    return m


def lbm_mlp_fit_normalization(m, feat_ptr, resid_ptr, n):
    _check(load().lbm_mlp_fit_normalization(m, feat_ptr, resid_ptr, int(n)), "lbm_mlp_fit_normalization")


def lbm_mlp_pack(m, feat_ptr, resid_ptr, n, x_ptr, t_ptr):
    _check(load().lbm_mlp_pack(m, feat_ptr, resid_ptr, int(n), x_ptr, t_ptr), "lbm_mlp_pack")


def lbm_mlp_train_step(m, x_ptr, t_ptr, nsamples, rows_ptr, batch, lr, loss_ptr):
    _check(load().lbm_mlp_train_step(m, x_ptr, t_ptr, int(nsamples), rows_ptr, int(batch), float(lr), loss_ptr),
           "lbm_mlp_train_step")


def lbm_mlp_grads(m, x_ptr, t_ptr, nsamples, rows_ptr, batch, grads_ptr, loss_ptr):
    _check(load().lbm_mlp_grads(m, x_ptr, t_ptr, int(nsamples), rows_ptr, int(batch), grads_ptr, loss_ptr),
           "lbm_mlp_grads")


def lbm_mlp_forward(m, x_ptr, n, y_ptr):
    _check(load().lbm_mlp_forward(m, x_ptr, int(n), y_ptr), "lbm_mlp_forward")


def lbm_mlp_params(m, out_ptr):
    _check(load().lbm_mlp_params(m, out_ptr), "lbm_mlp_params")


def lbm_mlp_normalization(m, mean_ptr, inv_std_ptr, scale_ptr):
    _check(load().lbm_mlp_normalization(m, mean_ptr, inv_std_ptr, scale_ptr), "lbm_mlp_normalization")


def lbm_mlp_set_normalization(m, mean_ptr, inv_std_ptr, scale_ptr):
    _check(load().lbm_mlp_set_normalization(m, mean_ptr, inv_std_ptr, scale_ptr), "lbm_mlp_set_normalization")


def lbm_mlp_export(m, trust, gain, kmin, net_ptr):
    _check(load().lbm_mlp_export(m, float(trust), float(gain), float(kmin), net_ptr), "lbm_mlp_export")


def lbm_mlp_destroy(m):
    load().lbm_mlp_destroy(m)


# ------------------------------------------------------------------ D3Q19 / D3Q27 (include/lbm3d.h)

LBM3D_D3Q19 = 0
LBM3D_D3Q27 = 1
VELOCITY_SETS = {19: LBM3D_D3Q19, 27: LBM3D_D3Q27}


class lbm3d_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("tau", ctypes.c_double), ("rho0", ctypes.c_double),
                ("bc", ctypes.c_int32 * 6),
                ("gamma", ctypes.c_double),
                ("store", ctypes.c_int32), ("velocity_set", ctypes.c_int32)]


def lbm3d_params_default() -> lbm3d_params:
    p = lbm3d_params()
    _check(load().lbm3d_params_default(ctypes.byref(p)), "lbm3d_params_default")
    return p


def lbm3d_workspace_bytes(p: lbm3d_params) -> int:
    n = ctypes.c_size_t()
    _check(load().lbm3d_workspace_bytes(ctypes.byref(p), ctypes.byref(n)), "lbm3d_workspace_bytes")
    return n.value


def lbm3d_init(p: lbm3d_params, ws_ptr, nbytes, drho_ptr, ux_ptr, uy_ptr, uz_ptr, stream_ptr):
    ctx = ctypes.c_void_p()
    _check(load().lbm3d_init(ctypes.byref(ctx), ctypes.byref(p), ws_ptr, nbytes, drho_ptr, ux_ptr, uy_ptr, uz_ptr,
                             stream_ptr), "lbm3d_init")
    return ctx


def lbm3d_set_farfield(ctx, beta, rho, ux, uy, uz):
    _check(load().lbm3d_set_farfield(ctx, beta, rho, ux, uy, uz), "lbm3d_set_farfield")


def lbm3d_step(ctx, n: int):
    _check(load().lbm3d_step(ctx, int(n)), "lbm3d_step")


def lbm3d_moments(ctx, out_ptr):
    _check(load().lbm3d_moments(ctx, out_ptr), "lbm3d_moments")


def lbm3d_get_populations(ctx, out_ptr):
    _check(load().lbm3d_get_populations(ctx, out_ptr), "lbm3d_get_populations")


def lbm3d_set_populations(ctx, in_ptr):
    _check(load().lbm3d_set_populations(ctx, in_ptr), "lbm3d_set_populations")


def lbm3d_check_finite(ctx) -> bool:
    """True if every stored population is finite (synchronizes the stream)."""
    ok = ctypes.c_int()
    rc = load().lbm3d_check_finite(ctx, ctypes.byref(ok))
    if rc not in (LBM_OK, LBM_ERR_NONFINITE):
        _check(rc, "lbm3d_check_finite")
    return bool(ok.value)


def lbm3d_f16_exp(ctx) -> int:
    k = ctypes.c_int32()
    _check(load().lbm3d_f16_exp(ctx, ctypes.byref(k)), "lbm3d_f16_exp")
    return k.value


def lbm3d_time(ctx) -> int:
    t = ctypes.c_int64()
    _check(load().lbm3d_time(ctx, ctypes.byref(t)), "lbm3d_time")
    return t.value


def lbm3d_shape_count() -> int:
    return int(load().lbm3d_shape_count())


def lbm3d_shape_describe(shape_id: int) -> str:
    buf = ctypes.create_string_buffer(64)
    _check(load().lbm3d_shape_describe(int(shape_id), buf, 64), "lbm3d_shape_describe")
    return buf.value.decode()


def lbm3d_set_shape(ctx, shape_id: int):
    _check(load().lbm3d_set_shape(ctx, int(shape_id)), "lbm3d_set_shape")


def lbm3d_autotune(ctx, reps: int = 5):
    best = ctypes.c_int32()
    times = (ctypes.c_float * lbm3d_shape_count())()
    _check(load().lbm3d_autotune(ctx, int(reps), ctypes.byref(best), times), "lbm3d_autotune")
    return best.value, list(times)


def lbm3d_destroy(ctx):
    load().lbm3d_destroy(ctx)

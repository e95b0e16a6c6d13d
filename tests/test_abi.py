"""Host-side checks of the C-ABI library (no GPU needed): the built
liblbm.so loads, exports every entry point include/lbm.h declares, and its
argument validation and workspace arithmetic behave as documented."""
import ctypes
import os
import re

import pytest

from paper_2005_08674_amd import lbm as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def _declared():
    names = set()
    for h in HEADERS:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(lbm_\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_2005_08674_amd import build
        build.build()
    return L.load()


def test_header_declares_the_core_calls():
    names = _declared()
    for n in ["lbm_init", "lbm_step", "lbm_set_farfield", "lbm_moments"]:
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    cdll = ctypes.CDLL(L.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(cdll, n)]
    assert not missing, missing
    for n in _declared():
        assert n in L.exported_symbols(), f"binding lacks {n}"


def test_defaults_and_workspace(lib):
    p = L.lbm_params_default()
    assert (p.nx, p.ny, p.tau, p.rho0, p.gamma) == (3, 3, 0.6, 1.0, 0.6)
    assert list(p.bc) == [1, 1, 1, 1] and p.store == L.LBM_STORE_F32
    p.nx, p.ny = 4096, 4096
    n32 = L.lbm_workspace_bytes(p)
    assert n32 >= 2 * 9 * 4096 * 4096 * 4
    p.store = L.LBM_STORE_F16DEV
    n16 = L.lbm_workspace_bytes(p)
    assert 2 * 9 * 4096 * 4096 * 2 <= n16 < n32
    p.store = L.LBM_STORE_F64
    assert L.lbm_workspace_bytes(p) >= 2 * 9 * 4096 * 4096 * 8


@pytest.mark.parametrize("field,value,msg", [
    ("nx", 2, "each side"), ("tau", 0.5, "tau"), ("store", 7, "store"), ("grad_order", 3, "grad_order"),
    ("corr_mode", 2, "corr_mode"), ("corner_mode", -1, "corner_mode"), ("rho0", 0.0, "rho0"),
])
def test_invalid_params_rejected(lib, field, value, msg):
    p = L.lbm_params_default()
    p.nx = p.ny = 16
    setattr(p, field, value)
    with pytest.raises(L.LbmError) as e:
        L.lbm_workspace_bytes(p)
    assert e.value.code == L.LBM_ERR_ARG and msg in str(e.value)


@pytest.mark.parametrize("store,esize", [("LBM_STORE_F32", 4), ("LBM_STORE_F64", 8), ("LBM_STORE_BF16DEV", 2)])
def test_plane_beyond_32bit_offsets_rejected(lib, store, esize):
    """The sweeps address a plane with 32-bit byte offsets: a thin lattice under the 2^28-node cap whose
    256-byte-padded rows make a plane of 4 GiB or more is refused, and one just below is accepted."""
    p = L.lbm_params_default()
    p.store = getattr(L, store)
    p.nx = 9                                   # one 256-byte row per lattice row in every format
    p.ny = (1 << 32) // 256                    # 2^24 rows: a 4 GiB plane, 1.5e8 nodes < 2^28
    with pytest.raises(L.LbmError) as e:
        L.lbm_workspace_bytes(p)
    assert e.value.code == L.LBM_ERR_ARG and "4 GiB" in str(e.value)
    p.ny = (1 << 32) // 256 - 1024             # 256 KiB below the bound
    assert L.lbm_workspace_bytes(p) >= 2 * 9 * p.ny * 256


def test_collision_model_parameters(lib):
    """BGK needs tau > 1/2; MRT (Sec. 4) takes tau >= 1/2 and rates in (0, 2]."""
    p = L.lbm_params_default()
    assert p.collision == L.LBM_COLL_BGK and (p.omega_e, p.omega_eps, p.omega_q) == (1.9, 1.9, 1.9)
    p.nx = p.ny = 16
    p.collision = 7
    with pytest.raises(L.LbmError, match="collision"):
        L.lbm_workspace_bytes(p)
    p.collision = L.LBM_COLL_MRT
    p.tau = 0.5
    assert L.lbm_workspace_bytes(p) > 0
    p.tau = 0.49
    with pytest.raises(L.LbmError, match="tau"):
        L.lbm_workspace_bytes(p)
    p.tau = 0.6
    for bad in (0.0, 2.01, float("nan")):
        p.omega_q = bad
        with pytest.raises(L.LbmError, match="MRT rates"):
            L.lbm_workspace_bytes(p)
    p.omega_q = 2.0
    assert L.lbm_workspace_bytes(p) > 0


@pytest.mark.parametrize("bc,ok", [((2, 1, 0, 0), True), ((1, 2, 0, 0), True), ((2, 2, 0, 0), True),
                                   ((2, 1, 1, 1), False), ((1, 1, 2, 0), False), ((0, 0, 2, 2), False)])
def test_velocity_edges_left_right_with_periodic_bottom_top(lib, bc, ok):
    p = L.lbm_params_default()
    p.nx = p.ny = 16
    for e in range(4):
        p.bc[e] = bc[e]
    if ok:
        assert L.lbm_workspace_bytes(p) > 0
    else:
        with pytest.raises(L.LbmError, match="velocity edge"):
            L.lbm_workspace_bytes(p)


def test_3d_parameters(lib):
    p = L.lbm3d_params_default()
    assert (p.nx, p.ny, p.nz, p.tau, p.gamma, p.store) == (3, 3, 3, 0.6, 0.6, L.LBM_STORE_F32)
    assert p.velocity_set == L.LBM3D_D3Q19
    p.nx = p.ny = p.nz = 64
    n32 = L.lbm3d_workspace_bytes(p)
    assert n32 >= 2 * 19 * 64 ** 3 * 4
    p.store = L.LBM_STORE_F64
    assert L.lbm3d_workspace_bytes(p) >= 2 * 19 * 64 ** 3 * 8
    p.velocity_set = L.LBM3D_D3Q27
    assert L.lbm3d_workspace_bytes(p) >= 2 * 27 * 64 ** 3 * 8
    for field, value, msg in [("nz", 2, "each side"), ("tau", 0.5, "tau"), ("store", 7, "store"),
                              ("velocity_set", 2, "velocity_set"), ("nx", 1 << 27, "2\\^28"),
                              ("ny", 1 << 13, "4 GiB")]:
        q = L.lbm3d_params_default()
        setattr(q, field, value)
        if field == "ny":
            q.nz = 1 << 13      # 3 x 8192 x 8192 nodes (< 2^28), but rows padded to 256 B make 16 GiB planes
        with pytest.raises(L.LbmError, match=msg):
            L.lbm3d_workspace_bytes(q)
    q = L.lbm3d_params_default()
    q.bc[4] = L.LBM_BC_PERIODIC
    with pytest.raises(L.LbmError, match="pairs"):
        L.lbm3d_workspace_bytes(q)


def test_unpaired_periodic_edges_rejected(lib):
    p = L.lbm_params_default()
    p.nx = p.ny = 16
    p.bc[0] = L.LBM_BC_PERIODIC
    with pytest.raises(L.LbmError, match="pairs"):
        L.lbm_workspace_bytes(p)


def test_init_rejects_bad_workspace_before_any_gpu_work(lib):
    p = L.lbm_params_default()
    p.nx = p.ny = 16
    with pytest.raises(L.LbmError, match="aligned"):
        L.lbm_init(p, 0, 1 << 20, 8, 8, 8, 0)
    with pytest.raises(L.LbmError, match="required"):
        L.lbm_init(p, 1 << 12, 16, 8, 8, 8, 0)


def test_tile_table(lib):
    n = L.lbm_tile_count()
    assert n >= 8
    names = [L.lbm_tile_describe(i) for i in range(n)]
    assert len(set(names)) == n
    with pytest.raises(L.LbmError):
        L.lbm_tile_describe(n)


def test_multi_step_shape_table(lib):
    """Two-step shapes first, then three-step shapes; each name's prefix agrees with its steps per
    launch, names are unique, and ids outside the table are refused (host-only calls)."""
    n = L.lbm_two_step_count()
    names = [L.lbm_two_step_describe(i) for i in range(n)]
    steps = [L.lbm_two_step_steps(i) for i in range(n)]
    assert len(set(names)) == n
    assert all(name.startswith(f"{k}step:64x") for name, k in zip(names, steps))
    assert 2 in steps and 3 in steps and steps == sorted(steps)
    for bad in (-1, n):
        with pytest.raises(L.LbmError):
            L.lbm_two_step_steps(bad)
        with pytest.raises(L.LbmError):
            L.lbm_two_step_describe(bad)


def test_debug_level_from_environment_and_setter(lib):
    """LBM_DEBUG is read once from the environment; lbm_set_debug accepts 0..2 only."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r); from paper_2005_08674_amd import lbm; "
            "print(lbm.lbm_debug_level())" % ROOT)
    for env_val, want in (("2", 2), ("1", 1), ("0", 0), ("7", 2)):
        out = subprocess.run([sys.executable, "-c", code], env={**os.environ, "LBM_DEBUG": env_val},
                             capture_output=True, text=True, check=True).stdout.strip()
        assert out == str(want), (env_val, out)
    env = {k: v for k, v in os.environ.items() if k != "LBM_DEBUG"}
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, check=True)
    assert out.stdout.strip() == "0"
    old = L.lbm_debug_level()
    try:
        L.lbm_set_debug(1)
        assert L.lbm_debug_level() == 1
        for bad in (-1, 3):
            with pytest.raises(L.LbmError) as e:
                L.lbm_set_debug(bad)
            assert e.value.code == L.LBM_ERR_ARG
    finally:
        L.lbm_set_debug(old)


def test_checkpoint_calls_reject_null_context(lib):
    import ctypes as C
    n = C.c_size_t()
    assert lib.lbm_save_bytes(None, C.byref(n)) == L.LBM_ERR_ARG
    buf = C.create_string_buffer(16)
    assert lib.lbm_save(None, buf, 16) == L.LBM_ERR_ARG
    assert lib.lbm_load(None, buf, 16) == L.LBM_ERR_ARG

"""CPU oracle for D2Q9 BGK/MRT + NSBC (Euser & Vuik, arXiv 2005.08674).

TEST INFRASTRUCTURE ONLY: the test-suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only users.  The product path
(the HIP library and its Python binding) never imports anything from here, and
this package imports nothing from the product package.

``lbm_oracle.c`` holds the lattice arithmetic (plain C, fp64, or x87 extended
precision when built with ``-DORC_LONG_DOUBLE``) and ``lbm_oracle3d.c`` the
same for D3Q19; this module builds both with gcc and wraps them with ctypes.  ``mlp.py`` is the numpy fp64 oracle of the
boundary-closure network and ``reflection.py`` the fp64 reflection-energy norm.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_BUILD_DIR selects another build of the same sources (the sanitizer build of
# oracle/sanitize.py); the default is the plain build below
BUILD_DIR = os.environ.get("ORACLE_BUILD_DIR") or os.path.join(HERE, "_build")
SRC = os.path.join(HERE, "lbm_oracle.c")
SRC3 = os.path.join(HERE, "lbm_oracle3d.c")
LIBS = {"double": os.path.join(BUILD_DIR, "liblbm_oracle.so"),
        "longdouble": os.path.join(BUILD_DIR, "liblbm_oracle_ld.so"),
        "3d": os.path.join(BUILD_DIR, "liblbm_oracle3d.so"),
        "3d_longdouble": os.path.join(BUILD_DIR, "liblbm_oracle3d_ld.so")}

BC_PERIODIC = 0
BC_NSBC = 1
BC_VELOCITY = 2


def build(verbose: bool = False, extra_flags=(), build_dir: str | None = None) -> None:
    """Compile both precisions of the oracle with gcc (always recompiles), into `build_dir`
    (default BUILD_DIR) with `extra_flags` added."""
    bdir = build_dir or BUILD_DIR
    os.makedirs(bdir, exist_ok=True)
    for kind, out in LIBS.items():
        out = os.path.join(bdir, os.path.basename(out))
        src = SRC3 if kind.startswith("3d") else SRC
        cmd = ["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off",
               "-fopenmp", "-shared", "-fPIC", *extra_flags, src, "-lm", "-o", out + ".tmp"]
        if kind.endswith("longdouble"):
            cmd.insert(1, "-DORC_LONG_DOUBLE")
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


class OrcParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("tau", ctypes.c_double), ("rho0", ctypes.c_double),
                ("bc", ctypes.c_int * 4),
                ("gamma", ctypes.c_double), ("beta", ctypes.c_double),
                ("m0_rho", ctypes.c_double), ("m0_ux", ctypes.c_double), ("m0_uy", ctypes.c_double),
                ("corr_mode", ctypes.c_int), ("grad_order", ctypes.c_int),
                ("corner_mode", ctypes.c_int),
                ("coll", ctypes.c_int),
                ("omega_e", ctypes.c_double), ("omega_eps", ctypes.c_double), ("omega_q", ctypes.c_double),
                ("uw_x", ctypes.c_double), ("uw_y", ctypes.c_double)]


_handles: dict = {}


def _lib(kind: str = "double"):
    if kind in _handles:
        return _handles[kind]
    path = LIBS[kind]
    if not os.path.exists(path):
        build()
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    for name, args in [("orc_feq", [ctypes.c_double] * 4 + [P]),
                       ("orc_collide_node", [ctypes.c_double, ctypes.c_double, P, P]),
                       ("orc_collide_node_mrt", [ctypes.c_double] * 5 + [P, P]),
                       ("orc_mrt_matrix", [P]),
                       ("orc_moments_node", [ctypes.c_double, P, P]),
                       ("orc_lattice_c", [P, P, P, P]),
                       ("orc_init", [P, P, P, P, P]),
                       ("orc_moments", [P, P, P, P, P]),
                       ("orc_step", [P, P, ctypes.c_int]),
                       ("orc_post_collision", [P, P, P]),
                       ("orc_num_threads", []),
                       ("orc_real_bytes", [])]:
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    _handles[kind] = lib
    return lib


def _dtype(kind: str):
    return np.float64 if kind == "double" else np.longdouble


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def lattice_constants(kind: str = "double"):
    """(cx, cy, w, opp) as the oracle defines them."""
    lib = _lib(kind)
    cx = np.zeros(9, np.int32)
    cy = np.zeros(9, np.int32)
    w = np.zeros(9, _dtype(kind))
    opp = np.zeros(9, np.int32)
    lib.orc_lattice_c(_ptr(cx), _ptr(cy), _ptr(w), _ptr(opp))
    return cx, cy, w, opp


def feq(rho0, drho, ux, uy, kind: str = "double") -> np.ndarray:
    out = np.zeros(9, _dtype(kind))
    _lib(kind).orc_feq(float(rho0), float(drho), float(ux), float(uy), _ptr(out))
    return out


def collide_node(tau, rho0, g9, kind: str = "double") -> np.ndarray:
    g9 = np.ascontiguousarray(g9, dtype=_dtype(kind))
    out = np.zeros(9, _dtype(kind))
    _lib(kind).orc_collide_node(float(tau), float(rho0), _ptr(g9), _ptr(out))
    return out


def collide_node_mrt(tau, rates, rho0, g9, kind: str = "double") -> np.ndarray:
    """One MRT collision (Sec. 4, eq. mrt_lbe); rates = (omega_e, omega_eps, omega_q), omega_nu = 1/tau."""
    g9 = np.ascontiguousarray(g9, dtype=_dtype(kind))
    out = np.zeros(9, _dtype(kind))
    we, weps, wq = (float(r) for r in rates)
    if _lib(kind).orc_collide_node_mrt(float(tau), we, weps, wq, float(rho0), _ptr(g9), _ptr(out)) != 0:
        raise ValueError("oracle rejected the MRT parameters")
    return out


def mrt_matrix(kind: str = "double") -> np.ndarray:
    """The oracle's transformation matrix M (eq. mrt_vm), [moment][direction]."""
    out = np.zeros(81, _dtype(kind))
    _lib(kind).orc_mrt_matrix(_ptr(out))
    return out.reshape(9, 9)


def moments_node(rho0, g9, kind: str = "double") -> np.ndarray:
    g9 = np.ascontiguousarray(g9, dtype=_dtype(kind))
    out = np.zeros(3, _dtype(kind))
    _lib(kind).orc_moments_node(float(rho0), _ptr(g9), _ptr(out))
    return out


class Lattice:
    """One D2Q9 lattice advanced by the oracle.

    ``bc`` is (left, right, bottom, top), each BC_PERIODIC, BC_NSBC or (left/right, with periodic
    bottom and top) BC_VELOCITY, a Dirichlet velocity edge at velocity ``uw``.
    Fields are [ny][nx] arrays; ``drho`` is rho - rho0.  ``mrt`` = (omega_e,
    omega_eps, omega_q) selects the MRT collision of Sec. 4 with omega_nu =
    1/tau; None keeps BGK.
    """

    def __init__(self, nx, ny, tau, drho, ux, uy, rho0=1.0, bc=(1, 1, 1, 1),
                 gamma=0.6, beta=0.0, m0=(1.0, 0.0, 0.0), corr_mode=0,
                 grad_order=1, corner_mode=0, mrt=None, uw=(0.0, 0.0), kind: str = "double"):
        self.kind = kind
        self.lib = _lib(kind)
        p = OrcParams()
        p.nx, p.ny, p.tau, p.rho0 = int(nx), int(ny), float(tau), float(rho0)
        for e in range(4):
            p.bc[e] = int(bc[e])
        p.gamma, p.beta = float(gamma), float(beta)
        p.m0_rho, p.m0_ux, p.m0_uy = (float(v) for v in m0)
        p.corr_mode, p.grad_order, p.corner_mode = int(corr_mode), int(grad_order), int(corner_mode)
        p.uw_x, p.uw_y = float(uw[0]), float(uw[1])
        if mrt is not None:
            p.coll = 1
            p.omega_e, p.omega_eps, p.omega_q = (float(r) for r in mrt)
        self.p = p
        self.nx, self.ny, self.rho0 = int(nx), int(ny), float(rho0)
        self.t = 0
        self.g = np.zeros((9, ny, nx), _dtype(kind))
        f = [np.ascontiguousarray(a, dtype=np.float64).reshape(ny, nx) for a in (drho, ux, uy)]
        rc = self.lib.orc_init(ctypes.byref(p), _ptr(f[0]), _ptr(f[1]), _ptr(f[2]), _ptr(self.g))
        if rc != 0:
            raise ValueError("oracle rejected the lattice parameters")

    def set_farfield(self, beta, rho, ux, uy):
        self.p.beta = float(beta)
        self.p.m0_rho, self.p.m0_ux, self.p.m0_uy = float(rho), float(ux), float(uy)

    def step(self, n: int = 1):
        rc = self.lib.orc_step(ctypes.byref(self.p), _ptr(self.g), int(n))
        if rc != 0:
            raise RuntimeError(f"orc_step failed ({rc})")
        self.t += int(n)
        return self

    def post_collision(self):
        """Post-collision populations g* = f* - w rho0 of every node, [9][ny][nx]."""
        out = np.zeros_like(self.g)
        self.lib.orc_post_collision(ctypes.byref(self.p), _ptr(self.g), _ptr(out))
        return out

    def moments(self):
        """(rho - rho0, ux, uy), each [ny][nx] float64."""
        out = [np.zeros((self.ny, self.nx), np.float64) for _ in range(3)]
        self.lib.orc_moments(ctypes.byref(self.p), _ptr(self.g), _ptr(out[0]), _ptr(out[1]), _ptr(out[2]))
        return tuple(out)


class Orc3Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("tau", ctypes.c_double), ("rho0", ctypes.c_double),
                ("bc", ctypes.c_int * 6),
                ("gamma", ctypes.c_double), ("beta", ctypes.c_double),
                ("m0", ctypes.c_double * 4), ("q", ctypes.c_int)]


_handles3: dict = {}


def _lib3(kind: str = "double"):
    key = "3d" if kind == "double" else "3d_longdouble"
    if key in _handles3:
        return _handles3[key]
    if not os.path.exists(LIBS[key]):
        build()
    lib = ctypes.CDLL(LIBS[key])
    P = ctypes.c_void_p
    I = ctypes.c_int
    for name, args in [("orc3_lattice", [I, P, P, P]), ("orc3_feq", [I, ctypes.c_double, P, P]),
                       ("orc3_collide_node", [I, ctypes.c_double, ctypes.c_double, P, P]),
                       ("orc3_moments_node", [I, ctypes.c_double, P, P]),
                       ("orc3_init", [P, P, P, P, P, P]), ("orc3_moments", [P, P, P]),
                       ("orc3_step", [P, P, ctypes.c_int])]:
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    _handles3[key] = lib
    return lib


def lattice_constants_3d(kind: str = "double", q: int = 19):
    """(c [q][3], w [q], opp [q]) of the oracle's D3Q19 (q = 19) or D3Q27 (q = 27) lattice."""
    c = np.zeros((q, 3), np.int32)
    w = np.zeros(q, _dtype(kind))
    opp = np.zeros(q, np.int32)
    if _lib3(kind).orc3_lattice(int(q), _ptr(c), _ptr(w), _ptr(opp)) != 0:
        raise ValueError(f"no {q}-velocity set")
    return c, w, opp


def feq_3d(rho0, m4, kind: str = "double", q: int = 19) -> np.ndarray:
    m = np.ascontiguousarray(m4, dtype=np.float64)
    out = np.zeros(q, _dtype(kind))
    if _lib3(kind).orc3_feq(int(q), float(rho0), _ptr(m), _ptr(out)) != 0:
        raise ValueError(f"no {q}-velocity set")
    return out


def collide_node_3d(tau, rho0, g, kind: str = "double") -> np.ndarray:
    """BGK of one node; the velocity set is len(g) (19 or 27)."""
    g = np.ascontiguousarray(g, dtype=_dtype(kind))
    out = np.zeros(len(g), _dtype(kind))
    if _lib3(kind).orc3_collide_node(len(g), float(tau), float(rho0), _ptr(g), _ptr(out)) != 0:
        raise ValueError(f"no {len(g)}-velocity set")
    return out


def moments_node_3d(rho0, g, kind: str = "double") -> np.ndarray:
    """(rho - rho0, ux, uy, uz) of one node; the velocity set is len(g)."""
    g = np.ascontiguousarray(g, dtype=_dtype(kind))
    out = np.zeros(4, _dtype(kind))
    if _lib3(kind).orc3_moments_node(len(g), float(rho0), _ptr(g), _ptr(out)) != 0:
        raise ValueError(f"no {len(g)}-velocity set")
    return out


class Lattice3D:
    """One D3Q19 (q = 19) or D3Q27 (q = 27) lattice advanced by the oracle.  ``bc`` = (x low, x high,
    y low, y high, z low, z high), each BC_PERIODIC or BC_NSBC.  Fields are [nz][ny][nx] arrays;
    ``drho`` is rho - rho0."""

    def __init__(self, nx, ny, nz, tau, drho, ux, uy, uz, rho0=1.0, bc=(1, 1, 1, 1, 1, 1), gamma=0.6, beta=0.0,
                 m0=(1.0, 0.0, 0.0, 0.0), kind: str = "double", q: int = 19):
        self.kind = kind
        self.lib = _lib3(kind)
        p = Orc3Params()
        p.nx, p.ny, p.nz, p.tau, p.rho0 = int(nx), int(ny), int(nz), float(tau), float(rho0)
        for f in range(6):
            p.bc[f] = int(bc[f])
        p.gamma, p.beta = float(gamma), float(beta)
        for a in range(4):
            p.m0[a] = float(m0[a])
        p.q = int(q)
        self.q = int(q)
        self.p = p
        self.shape = (int(nz), int(ny), int(nx))
        self.rho0 = float(rho0)
        self.t = 0
        self.g = np.zeros((self.q,) + self.shape, _dtype(kind))
        f = [np.ascontiguousarray(a, dtype=np.float64).reshape(self.shape) for a in (drho, ux, uy, uz)]
        if self.lib.orc3_init(ctypes.byref(p), _ptr(f[0]), _ptr(f[1]), _ptr(f[2]), _ptr(f[3]), _ptr(self.g)) != 0:
            raise ValueError("oracle rejected the lattice parameters")

    def set_farfield(self, beta, rho, ux, uy, uz):
        self.p.beta = float(beta)
        for a, v in enumerate((rho, ux, uy, uz)):
            self.p.m0[a] = float(v)

    def step(self, n: int = 1):
        if self.lib.orc3_step(ctypes.byref(self.p), _ptr(self.g), int(n)) != 0:
            raise RuntimeError("orc3_step failed")
        self.t += int(n)
        return self

    def moments(self):
        """(rho - rho0, ux, uy, uz), each [nz][ny][nx] float64."""
        out = np.zeros((4,) + self.shape, np.float64)
        self.lib.orc3_moments(ctypes.byref(self.p), _ptr(self.g), _ptr(out))
        return tuple(out)


def num_threads() -> int:
    return int(_lib("double").orc_num_threads())

"""ctypes wrapper of the plain FP64 CPU oracle (``fslbm_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of ``bench.py``.  The GPU library never imports,
links or calls anything here, and this package never touches the GPU
library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fslbm_oracle.c")
# FSLBM_ORACLE_LIB points the tests at another build of the same source
# (used to check that the pins catch planted mistakes).
LIB = os.environ.get("FSLBM_ORACLE_LIB", os.path.join(HERE, "liboracle.so"))

# Built without fast-math and without FMA contraction so that every
# operation rounds once, in the order the source states.
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-Wall", "-Wno-unused-function"]


def build(force: bool = True) -> str:
    if "FSLBM_ORACLE_LIB" in os.environ:
        return LIB
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("periodic", C.c_int32 * 3), ("collision", C.c_int32), ("freeze_conversions", C.c_int32),
                ("tau", C.c_double), ("trt_lambda", C.c_double), ("sigma", C.c_double),
                ("g", C.c_double * 3), ("p0", C.c_double), ("eps", C.c_double),
                ("inject_rate", C.c_double), ("contact_angle", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if "FSLBM_ORACLE_LIB" not in os.environ and (
                not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC)):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.orc_create.restype = P
        L.orc_create.argtypes = [C.POINTER(_Params), P, P, P, P, P, P, P, P, P, C.c_int32, P, P,
                                 C.c_int64, C.c_int32, C.c_double, C.c_char_p, C.c_int32]
        L.orc_destroy.argtypes = [P]
        L.orc_step.argtypes = [P, C.c_int32]
        L.orc_step.restype = C.c_int32
        L.orc_error.argtypes = [P]
        L.orc_error.restype = C.c_char_p
        L.orc_read.argtypes = [P] + [P] * 7
        L.orc_nbubbles.argtypes = [P]
        L.orc_nbubbles.restype = C.c_int32
        L.orc_bubbles.argtypes = [P] + [P] * 6
        L.orc_scalars.argtypes = [P] + [P] * 5
        L.orc_lattice.argtypes = [P, P, P]
        L.orc_feq.argtypes = [C.c_double, P, P]
        L.orc_collide.argtypes = [C.POINTER(_Params), P, P, P, P]
        L.orc_boundary_velocity.argtypes = [C.POINTER(_Params), P, P]
        L.orc_geometry.argtypes = [P, P, P]
        L.orc_label.argtypes = [C.c_int32, C.c_int32, C.c_int32, P, P, P]
        L.orc_fsum.restype = C.c_double
        L.orc_fsum.argtypes = [P, C.c_int64]
        L.orc_set_threads.argtypes = [C.c_int32]
        L.orc_threads.restype = C.c_int32
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def make_params(d: dict) -> _Params:
    p = _Params()
    p.nx, p.ny, p.nz = d["nx"], d["ny"], d["nz"]
    for k in range(3):
        p.periodic[k] = int(d["periodic"][k])
        p.g[k] = float(d["g"][k])
    p.collision = int(d.get("collision", 0))
    p.freeze_conversions = int(d.get("freeze_conversions", 0))
    p.tau = float(d["tau"])
    p.trt_lambda = float(d.get("trt_lambda", 3.0 / 16.0))
    p.sigma = float(d["sigma"])
    p.p0 = float(d.get("p0", 1.0 / 3.0))
    p.eps = float(d.get("eps_convert", d.get("eps", 1e-2)))
    p.inject_rate = float(d.get("inject_rate", 0.0))
    p.contact_angle = float(d.get("contact_angle", 0.0))
    return p


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def lattice():
    c = np.zeros((19, 3), np.int32)
    w = np.zeros(19, np.float64)
    o = np.zeros(19, np.int32)
    lib().orc_lattice(_ptr(c), _ptr(w), _ptr(o))
    return c, w, o


def feq(rho: float, u) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(19, np.float64)
    lib().orc_feq(C.c_double(rho), _ptr(u), _ptr(out))
    return out


def collide(params: dict, fin):
    p = make_params(params)
    fin = np.ascontiguousarray(fin, dtype=np.float64)
    fout = np.zeros(19, np.float64)
    rho = np.zeros(1, np.float64)
    u = np.zeros(3, np.float64)
    lib().orc_collide(C.byref(p), _ptr(fin), _ptr(fout), _ptr(rho), _ptr(u))
    return fout, float(rho[0]), u


def boundary_velocity(params: dict, fs) -> np.ndarray:
    """Velocity the interface reconstruction uses for a cell with
    post-collision PDFs fs."""
    p = make_params(params)
    fs = np.ascontiguousarray(fs, dtype=np.float64)
    u = np.zeros(3, np.float64)
    lib().orc_boundary_velocity(C.byref(p), _ptr(fs), _ptr(u))
    return u


def fsum(values) -> float:
    v = np.ascontiguousarray(values, dtype=np.float64)
    return float(lib().orc_fsum(_ptr(v), len(v)))


def label(inset: np.ndarray, shape, periodic) -> np.ndarray:
    nx, ny, nz = shape
    m = np.ascontiguousarray(inset.reshape(-1), dtype=np.uint8)
    per = np.asarray(periodic, dtype=np.int32)
    out = np.zeros(nx * ny * nz, np.int32)
    lib().orc_label(nx, ny, nz, _ptr(per), _ptr(m), _ptr(out))
    return out


class Oracle:
    """One oracle simulation built from a scene (``scenes.Scene``) or from
    explicit arrays."""

    def __init__(self, params: dict, cell_type, phi, rho, u, bubble_id, bubbles,
                 f_init=None, step0=0, next_id0=0, bucket0=0.0, mass_init=None):
        self.params = dict(params)
        self.nx, self.ny, self.nz = params["nx"], params["ny"], params["nz"]
        self.N = self.nx * self.ny * self.nz
        p = make_params(params)
        t = np.ascontiguousarray(cell_type, np.uint8)
        ph = np.ascontiguousarray(phi, np.float64)
        r = np.ascontiguousarray(rho, np.float64)
        uu = np.ascontiguousarray(u, np.float64)
        bid = np.ascontiguousarray(bubble_id, np.int32)
        b_id = np.asarray([b[0] for b in bubbles], np.int32)
        b_fl = np.asarray([b[1] for b in bubbles], np.int32)
        b_vs = np.asarray([b[2] for b in bubbles], np.float64)
        b_pi = np.asarray([b[3] for b in bubbles], np.float64)
        fi = None if f_init is None else np.ascontiguousarray(f_init, np.float64)
        mi = None if mass_init is None else np.ascontiguousarray(mass_init, np.float64)
        err = C.create_string_buffer(256)
        h = lib().orc_create(C.byref(p), _ptr(t), _ptr(ph), _ptr(r), _ptr(uu), _ptr(bid),
                             _ptr(b_id), _ptr(b_fl), _ptr(b_vs), _ptr(b_pi), len(bubbles),
                             _ptr(fi), _ptr(mi), int(step0), int(next_id0), float(bucket0),
                             err, 256)
        if not h:
            raise ValueError("oracle rejected input: " + err.value.decode())
        self._h = C.c_void_p(h)

    @classmethod
    def from_scene(cls, sc, **over):
        return cls(sc.params(**over), sc.cell_type, sc.phi, sc.rho, sc.u, sc.bubble_id,
                   sc.bubbles)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def step(self, n: int = 1) -> None:
        if lib().orc_step(self._h, int(n)) != 0:
            raise RuntimeError(lib().orc_error(self._h).decode())

    def read(self) -> dict:
        N = self.N
        out = dict(cell_type=np.zeros(N, np.uint8), phi=np.zeros(N), mass=np.zeros(N),
                   f=np.zeros(19 * N), bubble_id=np.zeros(N, np.int32), rho=np.zeros(N),
                   u=np.zeros(3 * N))
        lib().orc_read(self._h, _ptr(out["cell_type"]), _ptr(out["phi"]), _ptr(out["mass"]),
                       _ptr(out["f"]), _ptr(out["bubble_id"]), _ptr(out["rho"]), _ptr(out["u"]))
        return out

    def bubbles(self) -> dict:
        n = lib().orc_nbubbles(self._h)
        out = dict(id=np.zeros(n, np.int32), flags=np.zeros(n, np.int32), volume=np.zeros(n),
                   v_star=np.zeros(n), pressure=np.zeros(n), n_cells=np.zeros(n, np.int64))
        lib().orc_bubbles(self._h, _ptr(out["id"]), _ptr(out["flags"]), _ptr(out["volume"]),
                          _ptr(out["v_star"]), _ptr(out["pressure"]), _ptr(out["n_cells"]))
        return out

    def scalars(self) -> dict:
        st = np.zeros(1, np.int64)
        ni = np.zeros(1, np.int32)
        b = np.zeros(1)
        m = np.zeros(1)
        nt = np.zeros(1, np.int64)
        lib().orc_scalars(self._h, _ptr(st), _ptr(ni), _ptr(b), _ptr(m), _ptr(nt))
        return dict(step=int(st[0]), next_id=int(ni[0]), bucket=float(b[0]), total_mass=float(m[0]),
                    n_topology=int(nt[0]))

    def geometry(self):
        k = np.zeros(self.N)
        n = np.zeros(3 * self.N)
        lib().orc_geometry(self._h, _ptr(k), _ptr(n))
        return k, n.reshape(3, self.N)

"""Python binding of libfslbm (the MI355X FSLBM library with the enhanced
bubble model, arXiv:1604.01632).

Argument marshalling only: every step runs in the library's HIP kernels.
PyTorch supplies the device workspace (one uint8 tensor) and the stream.
The functions carry the names of the C ABI in ``include/fslbm.h``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfslbm.so")

FSLBM_OK, FSLBM_EINVAL, FSLBM_ENOMEM, FSLBM_EDEVICE, FSLBM_ENUMERIC, FSLBM_ECAPACITY = 0, -1, -2, -3, -4, -5
FP64, FP32, FP16DEV = 0, 1, 2
DEBUG_NO_LAYER_CHECK = 1
TRIGGER_EXACT, TRIGGER_NORMALS = 0, 1
PHASES = ("iface", "bulk", "convert", "excess", "gather", "label", "bubbles")
PHASE_BITS = {name: 1 << k for k, name in enumerate(PHASES)}
BGK, TRT = 0, 1
PRECISIONS = {"fp64": FP64, "fp32": FP32, "fp16dev": FP16DEV}


class FslbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fslbm error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("periodic", C.c_int32 * 3), ("precision", C.c_int32), ("collision", C.c_int32),
                ("tau", C.c_double), ("trt_lambda", C.c_double), ("sigma", C.c_double),
                ("g", C.c_double * 3), ("p0", C.c_double), ("eps_convert", C.c_double),
                ("inject_rate", C.c_double), ("max_bubbles", C.c_int32),
                ("force_topology", C.c_int32), ("freeze_conversions", C.c_int32),
                ("watchdog_every", C.c_int32), ("watchdog_drift", C.c_double),
                ("debug_flags", C.c_int32), ("split_trigger", C.c_int32),
                ("trigger_cos", C.c_double), ("iface_capacity", C.c_int32), ("pad_", C.c_int32),
                ("contact_angle", C.c_double)]


class BubbleInit(C.Structure):
    _fields_ = [("id", C.c_int32), ("flags", C.c_int32), ("v_star", C.c_double),
                ("p_init", C.c_double)]


class Bubble(C.Structure):
    _fields_ = [("id", C.c_int32), ("flags", C.c_int32), ("volume", C.c_double),
                ("v_star", C.c_double), ("pressure", C.c_double), ("n_cells", C.c_int64)]


class Scalars(C.Structure):
    _fields_ = [("step", C.c_int64), ("next_id", C.c_int32), ("n_bubbles", C.c_int32),
                ("bucket", C.c_double), ("total_mass", C.c_double), ("n_topology", C.c_int64),
                ("n_label_runs", C.c_int64)]


class BatchInfo(C.Structure):
    _fields_ = [("bulk_threads", C.c_int32), ("order", C.c_int32), ("from_cache", C.c_int32),
                ("list_cells", C.c_int32), ("cells", C.c_int64), ("probe_ms", C.c_float * 9),
                ("pad", C.c_int32)]


class Timing(C.Structure):
    _fields_ = [("bulk_ms", C.c_double), ("iface_ms", C.c_double), ("convert_ms", C.c_double),
                ("excess_ms", C.c_double), ("gather_ms", C.c_double), ("label_ms", C.c_double),
                ("bubbles_ms", C.c_double), ("step_ms", C.c_double), ("steps", C.c_int64)]


_lib = None


def lib() -> C.CDLL:
    """Load libfslbm.so; raises if it has not been built (there is no
    fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1604_01632_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.fslbm_workspace_bytes.restype = C.c_size_t
        L.fslbm_workspace_bytes.argtypes = [C.POINTER(Params)]
        L.fslbm_create.restype = C.c_int
        L.fslbm_create.argtypes = [C.POINTER(Params), P, P, P, P, P, C.POINTER(BubbleInit),
                                   C.c_int32, P, P, C.POINTER(Scalars), P, C.c_size_t, P,
                                   C.POINTER(C.c_void_p)]
        L.fslbm_step.restype = C.c_int
        L.fslbm_step.argtypes = [P, C.c_int32]
        L.fslbm_read_fields.restype = C.c_int
        L.fslbm_read_fields.argtypes = [P, P, P, P, P, P, P, P, C.POINTER(Scalars)]
        L.fslbm_bubbles.restype = C.c_int
        L.fslbm_bubbles.argtypes = [P, C.POINTER(Bubble), C.c_int32, C.POINTER(C.c_int32)]
        L.fslbm_sync.restype = C.c_int
        L.fslbm_sync.argtypes = [P]
        L.fslbm_destroy.restype = C.c_int
        L.fslbm_destroy.argtypes = [P]
        L.fslbm_set_timing.restype = C.c_int
        L.fslbm_set_timing.argtypes = [P, C.c_int32, C.c_uint32]
        L.fslbm_copy_bandwidth.restype = C.c_int
        L.fslbm_copy_bandwidth.argtypes = [P, P, C.c_size_t, C.c_int32, P, C.POINTER(C.c_double)]
        L.fslbm_get_timing.restype = C.c_int
        L.fslbm_get_timing.argtypes = [P, C.POINTER(Timing)]
        L.fslbm_last_error.restype = C.c_char_p
        L.fslbm_last_error.argtypes = []
        L.fslbm_batch_workspace_bytes.restype = C.c_size_t
        L.fslbm_batch_workspace_bytes.argtypes = [C.c_int32]
        L.fslbm_batch_create.restype = C.c_int
        L.fslbm_batch_create.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.c_char_p, P,
                                         C.c_size_t, P, C.POINTER(C.c_void_p)]
        L.fslbm_batch_create_noalloc.restype = C.c_int
        L.fslbm_batch_create_noalloc.argtypes = [C.POINTER(C.c_void_p), C.c_int32, P,
                                                 C.POINTER(C.c_void_p)]
        L.fslbm_batch_reset.restype = C.c_int
        L.fslbm_batch_reset.argtypes = [P, C.POINTER(C.c_void_p), C.c_int32]
        L.fslbm_batch_step.restype = C.c_int
        L.fslbm_batch_step.argtypes = [P, C.c_int32]
        L.fslbm_batch_info_get.restype = C.c_int
        L.fslbm_batch_info_get.argtypes = [P, C.POINTER(BatchInfo)]
        L.fslbm_batch_destroy.restype = C.c_int
        L.fslbm_batch_destroy.argtypes = [P]
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != FSLBM_OK:
        raise FslbmError(rc, lib().fslbm_last_error().decode())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def make_params(d: dict) -> Params:
    p = Params()
    p.nx, p.ny, p.nz = int(d["nx"]), int(d["ny"]), int(d["nz"])
    for k in range(3):
        p.periodic[k] = int(d["periodic"][k])
        p.g[k] = float(d["g"][k])
    prec = d.get("precision", FP64)
    p.precision = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
    p.collision = int(d.get("collision", BGK))
    p.tau = float(d["tau"])
    p.trt_lambda = float(d.get("trt_lambda", 3.0 / 16.0))
    p.sigma = float(d["sigma"])
    p.p0 = float(d.get("p0", 1.0 / 3.0))
    p.eps_convert = float(d.get("eps_convert", 1e-2))
    p.inject_rate = float(d.get("inject_rate", 0.0))
    p.max_bubbles = int(d.get("max_bubbles", 1024))
    p.force_topology = int(d.get("force_topology", 0))
    p.freeze_conversions = int(d.get("freeze_conversions", 0))
    p.watchdog_every = int(d.get("watchdog_every", 0))
    p.watchdog_drift = float(d.get("watchdog_drift", 0.0))
    p.debug_flags = int(d.get("debug_flags", 0))
    p.split_trigger = int(d.get("split_trigger", TRIGGER_EXACT))
    p.trigger_cos = float(d.get("trigger_cos", -0.5))
    p.iface_capacity = int(d.get("iface_capacity", 0))
    p.contact_angle = float(d.get("contact_angle", 0.0))
    return p


def fslbm_workspace_bytes(params: dict) -> int:
    return int(lib().fslbm_workspace_bytes(C.byref(make_params(params))))


def fslbm_create(params: dict, cell_type, phi, rho, u, bubble_id, bubbles, workspace,
                 stream=None, f_init=None, restore=None, mass_init=None):
    """Create a handle.  workspace: a CUDA uint8 torch tensor of at least
    fslbm_workspace_bytes(params) bytes; stream: a torch.cuda.Stream (default:
    the current stream).  bubbles: [(id, flags, v_star, p_init)]."""
    import torch

    p = make_params(params)
    t = np.ascontiguousarray(cell_type, np.uint8)
    ph = np.ascontiguousarray(phi, np.float64)
    r = np.ascontiguousarray(rho, np.float64)
    uu = np.ascontiguousarray(u, np.float64)
    bid = np.ascontiguousarray(bubble_id, np.int32)
    arr = (BubbleInit * max(1, len(bubbles)))()
    for k, b in enumerate(bubbles):
        arr[k].id, arr[k].flags, arr[k].v_star, arr[k].p_init = int(b[0]), int(b[1]), float(b[2]), float(b[3])
    fi = None if f_init is None else np.ascontiguousarray(f_init, np.float64)
    mi = None if mass_init is None else np.ascontiguousarray(mass_init, np.float64)
    rs = None
    if restore is not None:
        rs = Scalars()
        rs.step, rs.next_id, rs.bucket = int(restore["step"]), int(restore["next_id"]), float(restore["bucket"])
    if not (isinstance(workspace, torch.Tensor) and workspace.is_cuda and workspace.dtype == torch.uint8):
        raise TypeError("workspace must be a CUDA uint8 tensor")
    st = stream if stream is not None else torch.cuda.current_stream(workspace.device)
    h = C.c_void_p()
    rc = lib().fslbm_create(C.byref(p), _ptr(t), _ptr(ph), _ptr(r), _ptr(uu), _ptr(bid), arr,
                            len(bubbles), _ptr(fi), _ptr(mi), None if rs is None else C.byref(rs),
                            C.c_void_p(workspace.data_ptr()), workspace.numel(),
                            C.c_void_p(st.cuda_stream), C.byref(h))
    _check(rc)
    return h


def fslbm_step(handle, n_steps: int) -> None:
    _check(lib().fslbm_step(handle, int(n_steps)))


def fslbm_sync(handle) -> None:
    _check(lib().fslbm_sync(handle))


def fslbm_read_fields(handle, N: int, what=("cell_type", "phi", "mass", "f", "bubble_id", "rho", "u")) -> dict:
    out = {}
    shapes = dict(cell_type=(N, np.uint8), phi=(N, np.float64), mass=(N, np.float64),
                  f=(19 * N, np.float64), bubble_id=(N, np.int32), rho=(N, np.float64),
                  u=(3 * N, np.float64))
    for k in what:
        out[k] = np.zeros(shapes[k][0], shapes[k][1])
    sc = Scalars()
    rc = lib().fslbm_read_fields(handle, *[_ptr(out.get(k)) for k in
                                           ("cell_type", "phi", "mass", "f", "bubble_id", "rho", "u")],
                                 C.byref(sc))
    _check(rc)
    out["scalars"] = dict(step=sc.step, next_id=sc.next_id, n_bubbles=sc.n_bubbles,
                          bucket=sc.bucket, total_mass=sc.total_mass, n_topology=sc.n_topology,
                          n_label_runs=sc.n_label_runs)
    return out


def fslbm_bubbles(handle, capacity: int = 4096) -> dict:
    arr = (Bubble * capacity)()
    n = C.c_int32()
    _check(lib().fslbm_bubbles(handle, arr, capacity, C.byref(n)))
    m = n.value
    return dict(id=np.array([arr[k].id for k in range(m)], np.int32),
                flags=np.array([arr[k].flags for k in range(m)], np.int32),
                volume=np.array([arr[k].volume for k in range(m)]),
                v_star=np.array([arr[k].v_star for k in range(m)]),
                pressure=np.array([arr[k].pressure for k in range(m)]),
                n_cells=np.array([arr[k].n_cells for k in range(m)], np.int64))


def fslbm_destroy(handle) -> None:
    _check(lib().fslbm_destroy(handle))


def fslbm_set_timing(handle, period: int, phases=None) -> None:
    """Event timing of every `period`-th step (1: every step, 0: off) for
    the named phases (default: all)."""
    mask = 0 if phases is None else sum(PHASE_BITS[p] for p in phases)
    _check(lib().fslbm_set_timing(handle, int(period), mask))


def fslbm_copy_bandwidth(dst, src, reps: int = 10, stream=None) -> float:
    """GB/s (read + written) of the library's streaming copy kernel between
    two CUDA tensors of equal byte size."""
    import torch

    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    st = stream if stream is not None else torch.cuda.current_stream(src.device)
    out = C.c_double()
    _check(lib().fslbm_copy_bandwidth(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()),
                                      nbytes, int(reps), C.c_void_p(st.cuda_stream), C.byref(out)))
    return out.value


def fslbm_get_timing(handle) -> dict:
    t = Timing()
    _check(lib().fslbm_get_timing(handle, C.byref(t)))
    return {k: getattr(t, k) for k, _ in Timing._fields_}


def fslbm_last_error() -> str:
    return lib().fslbm_last_error().decode()


class Domain:
    """One simulation domain: owns its torch workspace and its handle."""

    def __init__(self, params: dict, cell_type, phi, rho, u, bubble_id, bubbles, device="cuda",
                 stream=None, f_init=None, restore=None, mass_init=None):
        import torch

        self.params = dict(params)
        self.N = int(params["nx"]) * int(params["ny"]) * int(params["nz"])
        nbytes = fslbm_workspace_bytes(params)
        if nbytes == 0:
            raise FslbmError(FSLBM_EINVAL, "invalid parameters")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = stream
        self.handle = fslbm_create(params, cell_type, phi, rho, u, bubble_id, bubbles,
                                   self.workspace, stream, f_init, restore, mass_init)

    @classmethod
    def from_scene(cls, sc, precision="fp64", stream=None, **over):
        return cls(sc.params(precision=PRECISIONS[precision] if isinstance(precision, str) else precision, **over),
                   sc.cell_type, sc.phi, sc.rho, sc.u, sc.bubble_id, sc.bubbles, stream=stream)

    def step(self, n: int = 1) -> None:
        fslbm_step(self.handle, n)

    def sync(self) -> None:
        fslbm_sync(self.handle)

    def read(self, what=("cell_type", "phi", "mass", "f", "bubble_id", "rho", "u")) -> dict:
        return fslbm_read_fields(self.handle, self.N, what)

    def bubbles(self) -> dict:
        return fslbm_bubbles(self.handle, max(16, int(self.params.get("max_bubbles", 1024))))

    def close(self) -> None:
        if getattr(self, "handle", None):
            fslbm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fslbm_batch_workspace_bytes(n_domains: int) -> int:
    return int(lib().fslbm_batch_workspace_bytes(int(n_domains)))


def fslbm_batch_create(handles, tuning_cache_path, workspace, stream=None):
    """Batch over the given handles.  workspace: a CUDA uint8 tensor of at
    least fslbm_batch_workspace_bytes(len(handles)) bytes."""
    import torch

    arr = (C.c_void_p * len(handles))(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
    st = stream if stream is not None else torch.cuda.current_stream(workspace.device)
    b = C.c_void_p()
    path = None if tuning_cache_path is None else str(tuning_cache_path).encode()
    _check(lib().fslbm_batch_create(arr, len(handles), path, C.c_void_p(workspace.data_ptr()),
                                    workspace.numel(), C.c_void_p(st.cuda_stream), C.byref(b)))
    return b


def fslbm_batch_create_noalloc(handles, stream=None):
    """Batch over the given handles with its tables in the library's static
    device array (no workspace); every domain must have been created on
    `stream` (default: the current stream)."""
    import torch

    arr = (C.c_void_p * len(handles))(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
    st = stream if stream is not None else torch.cuda.current_stream()
    b = C.c_void_p()
    _check(lib().fslbm_batch_create_noalloc(arr, len(handles), C.c_void_p(st.cuda_stream),
                                            C.byref(b)))
    return b


def fslbm_batch_step(batch, n_steps: int) -> None:
    _check(lib().fslbm_batch_step(batch, int(n_steps)))


def fslbm_batch_reset(batch, handles) -> None:
    arr = (C.c_void_p * len(handles))(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
    _check(lib().fslbm_batch_reset(batch, arr, len(handles)))


def fslbm_batch_info_get(batch) -> dict:
    info = BatchInfo()
    _check(lib().fslbm_batch_info_get(batch, C.byref(info)))
    return dict(bulk_threads=info.bulk_threads, order=info.order, from_cache=info.from_cache,
                list_cells=info.list_cells, cells=info.cells, probe_ms=list(info.probe_ms))


def fslbm_batch_destroy(batch) -> None:
    _check(lib().fslbm_batch_destroy(batch))


class Batch:
    """Many domains advanced together (one graph launch per step).
    capacity: domains the batch may hold after a reset (default: the given
    ones)."""

    def __init__(self, domains, tuning_cache_path=None, stream=None, capacity=None):
        import torch

        self.domains = list(domains)
        nbytes = fslbm_batch_workspace_bytes(max(len(self.domains), capacity or 0))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.domains[0].workspace.device)
        self.handle = fslbm_batch_create([d.handle for d in self.domains], tuning_cache_path,
                                         self.workspace, stream)

    def step(self, n: int = 1) -> None:
        fslbm_batch_step(self.handle, n)

    def reset(self, domains) -> None:
        """Replace the members (the batch then steps with plain launches)."""
        fslbm_batch_reset(self.handle, [d.handle for d in domains])
        self.domains = list(domains)

    def info(self) -> dict:
        return fslbm_batch_info_get(self.handle)

    def close(self) -> None:
        if getattr(self, "handle", None):
            fslbm_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

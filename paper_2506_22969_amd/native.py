"""ctypes binding of libsparstencil.so (argument marshalling only).

Every function here forwards to the C entry point of the same name in
include/sparstencil.h; all stencil work runs in the library's HIP kernels.
Device buffers are passed as integer addresses or as objects with a
``data_ptr()`` method (torch tensors); streams as integer hipStream_t handles
(``torch.cuda.current_stream().cuda_stream``) or None for the null stream.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsparstencil.so")

SS_OK, SS_PENDING = 0, 1
SS_E_INVALID, SS_E_UNSUPPORTED, SS_E_NOMEM, SS_E_DEVICE, SS_E_NOT_FOUND, SS_E_BUSY = -1, -2, -3, -4, -5, -6
SHAPES = {"box": 0, "star": 1, "custom": 2}
DTYPES = {"f64": 0, "f32": 1, "f16": 2, "f32_split_f16": 3, "f32_split_bf16": 4, "split_bf16": 5,
          "split3_bf16": 6}
BOUNDARIES = {"zero": 0, "periodic": 1}
ENGINES = {"auto": 0, "smfmac": 1, "mfma": 2, "direct": 3}
ENGINE_NAMES = {v: k for k, v in ENGINES.items()}
(Q_INFO, Q_COEFFS, Q_PERM, Q_VALUES, Q_META, Q_HI, Q_LO, Q_LUT, Q_MODEL, Q_KERNEL_LUT, Q_KERNEL_PERM,
 Q_MID, Q_KERNEL_FRAGS) = range(13)

EXPORTS = ["sparstencil_plan", "sparstencil_plan_points", "sparstencil_plan_query", "sparstencil_plan_destroy", "sparstencil_run",
           "sparstencil_sweep", "sparstencil_sweep_batch", "sparstencil_launch_count", "sparstencil_grid_bytes",
           "sparstencil_status_string", "sparstencil_server_create", "sparstencil_submit",
           "sparstencil_poll", "sparstencil_job_release", "sparstencil_server_drain",
           "sparstencil_server_clock", "sparstencil_server_destroy", "sparstencil_probe_mma_peak"]


class SparStencilError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_string(status)} ({status})")
        self.status = status


class PlanOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("boundary", ctypes.c_int32),
                ("fuse_steps", ctypes.c_int32), ("r1", ctypes.c_int32), ("r2", ctypes.c_int32),
                ("engine", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class JobInfo(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("state", ctypes.c_int32), ("status", ctypes.c_int32),
                ("steps_total", ctypes.c_int64), ("steps_done", ctypes.c_int64),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class PlanInfo(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("radius", ctypes.c_int32), ("k", ctypes.c_int32),
                ("fuse_steps", ctypes.c_int32), ("r1", ctypes.c_int32), ("r2", ctypes.c_int32),
                ("m_b", ctypes.c_int32), ("g", ctypes.c_int32), ("planes", ctypes.c_int32),
                ("m_prime", ctypes.c_int32), ("k_prime", ctypes.c_int32), ("k_pad", ctypes.c_int32),
                ("zeros", ctypes.c_int32), ("engine", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("boundary", ctypes.c_int32), ("passes", ctypes.c_int32),
                ("launches_per_sweep", ctypes.c_int32), ("sigma", ctypes.c_double),
                ("plan_seconds", ctypes.c_double), ("dims", ctypes.c_int64 * 3)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "dims"}
        d["dims"] = tuple(self.dims)
        d["engine_name"] = ENGINE_NAMES.get(self.engine, "?")
        return d


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "or python paper_2506_22969_amd/build.py")
        # torch ships its own HIP and HSA runtime libraries.  Loaded after
        # this library, torch's HIP runtime binds to the HSA runtime this
        # library already brought in and finds no GPU; loaded first, both
        # work.  So torch, when installed, is loaded before this library.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        L.sparstencil_plan.restype = i32
        L.sparstencil_plan.argtypes = [ctypes.POINTER(vp), i32, i32, ctypes.POINTER(ctypes.c_double), i32,
                                       ctypes.POINTER(i64), i32, ctypes.POINTER(PlanOpts)]
        L.sparstencil_plan_points.restype = i32
        L.sparstencil_plan_points.argtypes = [ctypes.POINTER(vp), i32, i32, ctypes.POINTER(i32),
                                              ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64), i32,
                                              ctypes.POINTER(PlanOpts)]
        L.sparstencil_plan_query.restype = i32
        L.sparstencil_plan_query.argtypes = [vp, i32, vp, ctypes.POINTER(sz)]
        L.sparstencil_plan_destroy.restype = i32
        L.sparstencil_plan_destroy.argtypes = [vp]
        L.sparstencil_run.restype = i32
        L.sparstencil_run.argtypes = [vp, vp, vp, i64, vp]
        L.sparstencil_sweep.restype = i32
        L.sparstencil_sweep.argtypes = [vp, vp, vp, vp]
        L.sparstencil_sweep_batch.restype = i32
        L.sparstencil_sweep_batch.argtypes = [vp, i32, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
        L.sparstencil_launch_count.restype = i64
        L.sparstencil_launch_count.argtypes = [vp, i64]
        L.sparstencil_grid_bytes.restype = sz
        L.sparstencil_grid_bytes.argtypes = [vp]
        L.sparstencil_status_string.restype = ctypes.c_char_p
        L.sparstencil_status_string.argtypes = [i32]
        u64 = ctypes.c_uint64
        L.sparstencil_server_create.restype = i32
        L.sparstencil_server_create.argtypes = [ctypes.POINTER(vp), vp, sz, i32, i32]
        L.sparstencil_submit.restype = i32
        L.sparstencil_submit.argtypes = [vp, vp, vp, vp, i64, ctypes.POINTER(u64)]
        L.sparstencil_poll.restype = i32
        L.sparstencil_poll.argtypes = [vp, u64, ctypes.POINTER(JobInfo)]
        L.sparstencil_job_release.restype = i32
        L.sparstencil_job_release.argtypes = [vp, u64]
        L.sparstencil_server_drain.restype = i32
        L.sparstencil_server_drain.argtypes = [vp]
        L.sparstencil_server_clock.restype = ctypes.c_double
        L.sparstencil_server_clock.argtypes = [vp]
        L.sparstencil_server_destroy.restype = i32
        L.sparstencil_server_destroy.argtypes = [vp]
        L.sparstencil_probe_mma_peak.restype = i32
        L.sparstencil_probe_mma_peak.argtypes = [i32, i64, i32, vp, ctypes.POINTER(ctypes.c_double), vp]
        _lib = L
    return _lib


def _ptr(x) -> int:
    if x is None:
        return 0
    if hasattr(x, "data_ptr"):
        return int(x.data_ptr())
    return int(x)


def _check(status: int, what: str) -> int:
    if status < 0:
        raise SparStencilError(status, what)
    return status


def status_string(status: int) -> str:
    return lib().sparstencil_status_string(int(status)).decode()


# ----------------------------------------------------------------------------
# the C entry points

def sparstencil_plan(shape, radius, coeffs, ndim, grid_dims, dtype, opts=None) -> int:
    """Returns the plan handle (int).  shape/dtype may be names or ints."""
    shape = SHAPES.get(shape, shape)
    dtype = DTYPES.get(dtype, dtype)
    w = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64).reshape(-1))
    dims = (ctypes.c_int64 * int(ndim))(*[int(d) for d in grid_dims])
    h = ctypes.c_void_p()
    popts = ctypes.byref(opts) if opts is not None else None
    st = lib().sparstencil_plan(ctypes.byref(h), int(shape), int(radius),
                                w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(ndim), dims,
                                int(dtype), popts)
    _check(st, "sparstencil_plan")
    return int(h.value)


def sparstencil_plan_points(offsets, coeffs, grid_dims, dtype, opts=None) -> int:
    """Plan from a list of points: offsets (npoints, ndim) ints, coeffs
    (npoints,) values.  Returns the plan handle (int)."""
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32))
    if off.ndim != 2:
        raise ValueError("offsets must be (npoints, ndim)")
    dtype = DTYPES.get(dtype, dtype)
    w = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64).reshape(-1))
    if w.size != off.shape[0]:
        raise ValueError("one coefficient per offset")
    dims = (ctypes.c_int64 * len(grid_dims))(*[int(d) for d in grid_dims])
    h = ctypes.c_void_p()
    popts = ctypes.byref(opts) if opts is not None else None
    st = lib().sparstencil_plan_points(ctypes.byref(h), int(off.shape[1]), int(off.shape[0]),
                                       off.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                       w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), dims, int(dtype), popts)
    _check(st, "sparstencil_plan_points")
    return int(h.value)


def sparstencil_plan_query(plan: int, what: int) -> bytes:
    n = ctypes.c_size_t(0)
    _check(lib().sparstencil_plan_query(plan, what, None, ctypes.byref(n)), "sparstencil_plan_query")
    buf = ctypes.create_string_buffer(max(1, n.value))
    _check(lib().sparstencil_plan_query(plan, what, buf, ctypes.byref(n)), "sparstencil_plan_query")
    return buf.raw[: n.value]


def sparstencil_plan_destroy(plan: int) -> None:
    _check(lib().sparstencil_plan_destroy(plan), "sparstencil_plan_destroy")


def sparstencil_run(plan: int, inp, out, steps: int, stream=None) -> None:
    _check(lib().sparstencil_run(plan, _ptr(inp), _ptr(out), int(steps), _ptr(stream)), "sparstencil_run")


def sparstencil_sweep(plan: int, inp, out, stream=None) -> None:
    _check(lib().sparstencil_sweep(plan, _ptr(inp), _ptr(out), _ptr(stream)), "sparstencil_sweep")


def sparstencil_sweep_batch(plan: int, inputs, outputs, stream=None) -> None:
    n = len(inputs)
    if len(outputs) != n:
        raise ValueError("inputs and outputs differ in length")
    ins = (ctypes.c_void_p * max(1, n))(*[_ptr(x) for x in inputs])
    outs = (ctypes.c_void_p * max(1, n))(*[_ptr(x) for x in outputs])
    _check(lib().sparstencil_sweep_batch(plan, n, ins, outs, _ptr(stream)), "sparstencil_sweep_batch")


def sparstencil_launch_count(plan: int, steps: int) -> int:
    return int(lib().sparstencil_launch_count(plan, int(steps)))


def sparstencil_grid_bytes(plan: int) -> int:
    return int(lib().sparstencil_grid_bytes(plan))


def sparstencil_status_string(status: int) -> str:
    return status_string(status)


def sparstencil_server_create(arena, arena_bytes: int, max_jobs: int, num_streams: int = 4) -> int:
    h = ctypes.c_void_p()
    _check(lib().sparstencil_server_create(ctypes.byref(h), _ptr(arena), int(arena_bytes), int(max_jobs),
                                           int(num_streams)), "sparstencil_server_create")
    return int(h.value)


def sparstencil_submit(server: int, plan: int, inp, out, steps: int) -> int:
    jid = ctypes.c_uint64(0)
    _check(lib().sparstencil_submit(server, plan, _ptr(inp), _ptr(out), int(steps), ctypes.byref(jid)),
           "sparstencil_submit")
    return int(jid.value)


def sparstencil_poll(server: int, job_id: int):
    """(status, info dict); status is SS_PENDING, SS_OK or the job's error."""
    info = JobInfo()
    st = lib().sparstencil_poll(server, int(job_id), ctypes.byref(info))
    if st == SS_E_NOT_FOUND or st == SS_E_INVALID:
        raise SparStencilError(st, "sparstencil_poll")
    return st, info.as_dict()


def sparstencil_job_release(server: int, job_id: int) -> None:
    _check(lib().sparstencil_job_release(server, int(job_id)), "sparstencil_job_release")


def sparstencil_server_drain(server: int) -> None:
    _check(lib().sparstencil_server_drain(server), "sparstencil_server_drain")


def sparstencil_server_clock(server: int) -> float:
    return float(lib().sparstencil_server_clock(server))


def sparstencil_server_destroy(server: int) -> None:
    _check(lib().sparstencil_server_destroy(server), "sparstencil_server_destroy")


def sparstencil_probe_mma_peak(engine, iters: int, workgroups: int, out, stream=None) -> float:
    """Enqueue the matrix-core throughput probe; returns the dense-equivalent
    flops it issues (time it with events around the call)."""
    flops = ctypes.c_double(0.0)
    _check(lib().sparstencil_probe_mma_peak(ENGINES.get(engine, engine), int(iters), int(workgroups), _ptr(out),
                                            ctypes.byref(flops), stream or 0), "sparstencil_probe_mma_peak")
    return float(flops.value)


# ----------------------------------------------------------------------------
# convenience wrapper

FLAG_HOST_ONLY = 1


def make_opts(boundary="zero", fuse_steps=1, r1=0, r2=0, engine="auto", flags=0) -> PlanOpts:
    return PlanOpts(ctypes.sizeof(PlanOpts), BOUNDARIES.get(boundary, boundary), int(fuse_steps),
                    int(r1), int(r2), ENGINES.get(engine, engine), int(flags))


class Plan:
    """Owns one plan handle; see sparstencil_plan for the arguments (shape
    "custom" with offsets=(npoints, ndim) and one coefficient per point:
    sparstencil_plan_points; radius is then unused)."""

    def __init__(self, shape, radius, coeffs, grid_dims, dtype, boundary="zero", fuse_steps=1,
                 r1=0, r2=0, engine="auto", host_only=False, offsets=None):
        grid_dims = tuple(int(d) for d in grid_dims)
        self.grid_dims = grid_dims
        self.dtype = dtype
        self.handle = 0
        opts = make_opts(boundary, fuse_steps, r1, r2, engine, FLAG_HOST_ONLY if host_only else 0)
        if offsets is not None:
            self.handle = sparstencil_plan_points(offsets, coeffs, grid_dims, dtype, opts)
        else:
            self.handle = sparstencil_plan(shape, radius, coeffs, len(grid_dims), grid_dims, dtype, opts)

    def close(self):
        if getattr(self, "handle", 0):
            sparstencil_plan_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def info(self) -> dict:
        raw = sparstencil_plan_query(self.handle, Q_INFO)
        return PlanInfo.from_buffer_copy(raw).as_dict()

    def table(self, what: int) -> np.ndarray:
        raw = sparstencil_plan_query(self.handle, what)
        dt = {Q_COEFFS: np.float64, Q_PERM: np.int32, Q_VALUES: np.float64, Q_META: np.uint8,
              Q_HI: np.uint16, Q_LO: np.uint16, Q_LUT: np.int32, Q_MODEL: np.float64,
              Q_KERNEL_LUT: np.int32, Q_KERNEL_PERM: np.int32, Q_MID: np.uint16}[what]
        return np.frombuffer(raw, dtype=dt).copy()

    def kernel_fragments(self) -> dict:
        """The matrix-core kernel's A operand registers (SS_Q_KERNEL_FRAGS):
        hi, lo (and mid) as uint16 [MB][KC][64][8], idx as uint32
        [MB][KC][64] (sparse), with mode and parts."""
        raw = sparstencil_plan_query(self.handle, Q_KERNEL_FRAGS)
        if not raw:
            return {}
        mb, kc, mode, parts = np.frombuffer(raw[:16], dtype=np.int32)
        n = int(mb) * int(kc) * 64 * 8
        at = 16
        out = {"mode": "sparse" if mode == 0 else "dense", "parts": int(parts)}
        for name in ("hi", "lo", "mid")[:int(parts)]:
            out[name] = np.frombuffer(raw[at:at + 2 * n], dtype=np.uint16).reshape(mb, kc, 64, 8).copy()
            at += 2 * n
        if mode == 0:
            out["idx"] = np.frombuffer(raw[at:at + 4 * n // 8], dtype=np.uint32).reshape(mb, kc, 64).copy()
        return out

    def run(self, inp, out, steps, stream=None):
        sparstencil_run(self.handle, inp, out, steps, stream)

    def sweep(self, inp, out, stream=None):
        sparstencil_sweep(self.handle, inp, out, stream)

    def sweep_batch(self, inputs, outputs, stream=None):
        sparstencil_sweep_batch(self.handle, inputs, outputs, stream)

    def launch_count(self, steps):
        return sparstencil_launch_count(self.handle, steps)

    @property
    def grid_bytes(self) -> int:
        return sparstencil_grid_bytes(self.handle)


class Server:
    """Owns one server handle over a caller-provided device arena."""

    def __init__(self, arena, arena_bytes, max_jobs=4096, num_streams=4):
        self.handle = 0
        self.arena = arena  # keeps the arena alive while the server runs
        self.handle = sparstencil_server_create(arena, arena_bytes, max_jobs, num_streams)

    def submit(self, plan, inp, out, steps) -> int:
        h = plan.handle if isinstance(plan, Plan) else int(plan)
        return sparstencil_submit(self.handle, h, inp, out, steps)

    def poll(self, job_id):
        return sparstencil_poll(self.handle, job_id)

    def release(self, job_id):
        sparstencil_job_release(self.handle, job_id)

    def drain(self):
        sparstencil_server_drain(self.handle)

    def clock(self) -> float:
        return sparstencil_server_clock(self.handle)

    def close(self):
        if getattr(self, "handle", 0):
            sparstencil_server_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

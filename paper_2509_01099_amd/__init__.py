"""Python binding of the MI355X ISLBM library (libislbm.so, C-ABI in include/islbm.h).

Argument marshalling only: every step of the solver runs in the HIP kernels of
libislbm.so.  The functions keep the C names; ``Cavity`` is a small
convenience wrapper that lets PyTorch provide the device buffers and the
stream.  Importing this package without the built library raises
ImportError: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libislbm.so")

ISLBM_OK, ISLBM_EINVAL, ISLBM_EMESH, ISLBM_EPARAM = 0, -1, -2, -3
ISLBM_ENOMEM, ISLBM_EDEVICE, ISLBM_ENONFINITE = -4, -5, -6
ISLBM_D2Q9_D2Q5, ISLBM_D3Q19_D3Q7 = 2, 3
ISLBM_FP32, ISLBM_FP64, ISLBM_FP16DEV, ISLBM_BF16DEV, ISLBM_FP32SR = 0, 1, 2, 3, 4
MESH_KINDS = {"uniform": 0, "erf": 1, "cosine": 2, "tanh": 3}
STORAGE = {"fp32": ISLBM_FP32, "fp64": ISLBM_FP64, "fp16": ISLBM_FP16DEV, "bf16": ISLBM_BF16DEV,
           "fp32sr": ISLBM_FP32SR}

EXPORTS = ("islbm_default_options", "islbm_query_bytes", "islbm_mesh_spacing", "islbm_create",
           "islbm_step", "islbm_fields", "islbm_fields_device", "islbm_nu_re",
           "islbm_get_populations", "islbm_set_populations", "islbm_init_fields",
           "islbm_init_fields_device", "islbm_info", "islbm_time", "islbm_set_time",
           "islbm_sync", "islbm_destroy", "islbm_strerror", "islbm_last_error",
           "islbm_time_steps", "islbm_state_bytes", "islbm_save_state", "islbm_load_state",
           "islbm_steady_change", "islbm_time_steps_split", "islbm_copy_bytes",
           "islbm_plan_steps")


class islbm_options(C.Structure):
    _fields_ = [("u_f", C.c_double), ("T_hot", C.c_double), ("T_cold", C.c_double),
                ("s_e", C.c_double), ("s_eps", C.c_double), ("s_q", C.c_double),
                ("s_pi", C.c_double), ("s_m", C.c_double), ("q_j", C.c_double),
                ("q_e", C.c_double), ("q_nu", C.c_double), ("storage", C.c_int),
                ("stream", C.c_void_p), ("buffers", C.c_void_p * 4),
                ("allow_unstable", C.c_int), ("stream_only", C.c_int), ("no_graph", C.c_int),
                ("force_interp", C.c_int)]


class islbm_stats(C.Structure):
    _fields_ = [("nu_vol", C.c_double), ("nu_hot", C.c_double), ("nu_cold", C.c_double),
                ("nu_mid", C.c_double), ("re_vol", C.c_double), ("re_uv", C.c_double),
                ("mass", C.c_double), ("rho_sum", C.c_double), ("umax", C.c_double),
                ("vmax", C.c_double), ("wmax", C.c_double), ("nonfinite", C.c_longlong),
                ("step", C.c_longlong), ("re_rms", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_D = C.POINTER(C.c_double)
_lib = None


def load() -> C.CDLL:
    """Loads libislbm.so; raises ImportError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    # PyTorch bundles its own HIP runtime under the same soname as the system
    # one.  Importing torch first makes libislbm.so bind to that runtime, so
    # the process holds a single HIP runtime whose device pointers and
    # streams both sides share.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    lib.islbm_default_options.argtypes = [C.POINTER(islbm_options)]
    lib.islbm_default_options.restype = None
    lib.islbm_query_bytes.argtypes = [C.c_int, C.POINTER(C.c_int), C.c_int,
                                      C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
    lib.islbm_mesh_spacing.argtypes = [C.c_int, C.c_int, C.c_double, _D]
    lib.islbm_create.argtypes = [C.POINTER(P), C.c_int, C.POINTER(C.c_int), C.POINTER(_D),
                                 C.c_double, C.c_double, C.POINTER(islbm_options)]
    lib.islbm_step.argtypes = [P, C.c_longlong]
    lib.islbm_plan_steps.argtypes = [P, C.c_longlong]
    lib.islbm_fields.argtypes = [P, _D, _D, _D, _D, _D]
    lib.islbm_fields_device.argtypes = [P, P, P, P, P, P]
    lib.islbm_nu_re.argtypes = [P, C.POINTER(islbm_stats)]
    lib.islbm_get_populations.argtypes = [P, _D, _D]
    lib.islbm_set_populations.argtypes = [P, _D, _D, C.c_int]
    lib.islbm_init_fields.argtypes = [P, _D, _D, _D, _D]
    lib.islbm_init_fields_device.argtypes = [P, P, P, P, P]
    lib.islbm_info.argtypes = [P, _D, _D, _D, _D, _D, _D]
    lib.islbm_time.argtypes = [P]
    lib.islbm_time.restype = C.c_longlong
    lib.islbm_set_time.argtypes = [P, C.c_longlong]
    lib.islbm_sync.argtypes = [P]
    lib.islbm_destroy.argtypes = [P]
    lib.islbm_destroy.restype = None
    lib.islbm_strerror.argtypes = [C.c_int]
    lib.islbm_strerror.restype = C.c_char_p
    lib.islbm_last_error.argtypes = [P]
    lib.islbm_last_error.restype = C.c_char_p
    lib.islbm_time_steps.argtypes = [P, C.c_longlong, _D]
    lib.islbm_time_steps_split.argtypes = [P, C.c_longlong, _D, _D, _D]
    lib.islbm_copy_bytes.argtypes = [P, P, C.c_size_t, P]
    lib.islbm_state_bytes.argtypes = [P, C.POINTER(C.c_size_t)]
    lib.islbm_save_state.argtypes = [P, C.c_void_p, C.c_size_t]
    lib.islbm_load_state.argtypes = [P, C.c_void_p, C.c_size_t]
    lib.islbm_steady_change.argtypes = [P, _D, _D, C.POINTER(C.c_longlong)]
    special = {"islbm_default_options", "islbm_destroy", "islbm_strerror", "islbm_last_error",
               "islbm_time"}
    for name in EXPORTS:
        if name not in special:
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


class IslbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


def _check(code: int, ctx=None) -> int:
    if code != ISLBM_OK:
        lib = load()
        detail = lib.islbm_last_error(ctx).decode() if ctx is not None else \
            lib.islbm_last_error(None).decode()
        raise IslbmError(code, f"{lib.islbm_strerror(code).decode()}: {detail}")
    return code


def _dp(a):
    return None if a is None else a.ctypes.data_as(_D)


# ------------------------------------------------------------ C-name wrappers

def islbm_default_options() -> islbm_options:
    o = islbm_options()
    load().islbm_default_options(C.byref(o))
    return o


def islbm_mesh_spacing(kind, n: int, a: float = 1.5) -> np.ndarray:
    k = MESH_KINDS[kind] if isinstance(kind, str) else int(kind)
    out = np.zeros(n + 1)
    _check(load().islbm_mesh_spacing(k, n, a, _dp(out)))
    return out


def islbm_query_bytes(lattice: int, n, storage: int):
    fb, gb = C.c_size_t(), C.c_size_t()
    nn = (C.c_int * 3)(*(list(n) + [1] * (3 - len(n))))
    _check(load().islbm_query_bytes(lattice, nn, storage, C.byref(fb), C.byref(gb)))
    return fb.value, gb.value


def islbm_create(lattice: int, n, spacings, Ra: float, Pr: float, options=None):
    """Returns an opaque context handle (c_void_p)."""
    lib = load()
    ctx = C.c_void_p()
    nn = (C.c_int * 3)(*(list(n) + [1] * (3 - len(n))))
    sp = [np.ascontiguousarray(s, dtype=np.float64) for s in spacings]
    arr = (_D * 3)(*([_dp(s) for s in sp] + [None] * (3 - len(sp))))
    rc = lib.islbm_create(C.byref(ctx), lattice, nn, arr, Ra, Pr,
                          C.byref(options) if options is not None else None)
    _check(rc)
    return ctx


def islbm_step(ctx, nsteps: int) -> None:
    _check(load().islbm_step(ctx, int(nsteps)), ctx)


def islbm_time_steps(ctx, nsteps: int) -> float:
    ms = C.c_double()
    _check(load().islbm_time_steps(ctx, int(nsteps), C.byref(ms)), ctx)
    return ms.value


def islbm_time_steps_split(ctx, nsteps: int) -> tuple:
    """(ms of all nsteps launches, ms of the nsteps - 1 plain ones, ms of the
    final reducing launch), from HIP events on the context's stream."""
    tot, plain, red = C.c_double(), C.c_double(), C.c_double()
    _check(load().islbm_time_steps_split(ctx, int(nsteps), C.byref(tot), C.byref(plain),
                                         C.byref(red)), ctx)
    return tot.value, plain.value, red.value


def islbm_plan_steps(ctx, nsteps: int) -> None:
    """Captures the launch graphs a following islbm_step(ctx, nsteps) from the
    current state replays; advances nothing."""
    _check(load().islbm_plan_steps(ctx, int(nsteps)), ctx)


def islbm_copy_bytes(dst_ptr: int, src_ptr: int, nbytes: int, stream=None) -> None:
    """Device copy with 16-byte vectors (bandwidth ceiling measurement)."""
    rc = load().islbm_copy_bytes(C.c_void_p(dst_ptr), C.c_void_p(src_ptr), int(nbytes),
                                 C.c_void_p(stream) if stream else None)
    if rc != 0:
        raise RuntimeError(f"islbm_copy_bytes failed with status {rc}")


def islbm_nu_re(ctx, allow_nonfinite: bool = False) -> dict:
    st = islbm_stats()
    rc = load().islbm_nu_re(ctx, C.byref(st))
    if not (allow_nonfinite and rc == ISLBM_ENONFINITE):
        _check(rc, ctx)
    return st.as_dict()


def islbm_steady_change(ctx) -> tuple:
    """(du, dT, steps) since the previous call; (inf, inf, 0) on the first."""
    du, dT, k = C.c_double(), C.c_double(), C.c_longlong()
    _check(load().islbm_steady_change(ctx, C.byref(du), C.byref(dT), C.byref(k)), ctx)
    return du.value, dT.value, k.value


def islbm_fields(ctx, shape) -> dict:
    arrs = {k: np.zeros(shape) for k in ("rho", "ux", "uy", "uz", "T")}
    _check(load().islbm_fields(ctx, *[_dp(arrs[k]) for k in ("rho", "ux", "uy", "uz", "T")]), ctx)
    return arrs


def islbm_fields_device(ctx, rho, ux, uy, uz, T) -> None:
    ptr = (lambda t: None if t is None else C.c_void_p(t.data_ptr()))
    _check(load().islbm_fields_device(ctx, ptr(rho), ptr(ux), ptr(uy), ptr(uz), ptr(T)), ctx)


def islbm_get_populations(ctx, qf: int, qg: int, shape):
    f = np.zeros((qf,) + tuple(shape))
    g = np.zeros((qg,) + tuple(shape))
    _check(load().islbm_get_populations(ctx, _dp(f), _dp(g)), ctx)
    return f, g


def islbm_set_populations(ctx, f, g, post_collision: bool) -> None:
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    _check(load().islbm_set_populations(ctx, _dp(f), _dp(g), 1 if post_collision else 0), ctx)


def islbm_init_fields(ctx, ux, uy, uz, T) -> None:
    cv = (lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64))
    ux, uy, uz, T = cv(ux), cv(uy), cv(uz), cv(T)
    _check(load().islbm_init_fields(ctx, _dp(ux), _dp(uy), _dp(uz), _dp(T)), ctx)


def islbm_init_fields_device(ctx, ux, uy, uz, T) -> None:
    ptr = (lambda t: None if t is None else C.c_void_p(t.data_ptr()))
    _check(load().islbm_init_fields_device(ctx, ptr(ux), ptr(uy), ptr(uz), ptr(T)), ctx)


def islbm_state_bytes(ctx) -> int:
    b = C.c_size_t()
    _check(load().islbm_state_bytes(ctx, C.byref(b)), ctx)
    return b.value


def islbm_save_state(ctx) -> bytes:
    buf = C.create_string_buffer(islbm_state_bytes(ctx))
    _check(load().islbm_save_state(ctx, buf, len(buf)), ctx)
    return buf.raw


def islbm_load_state(ctx, blob: bytes) -> None:
    _check(load().islbm_load_state(ctx, blob, len(blob)), ctx)


def islbm_info(ctx) -> dict:
    vals = [C.c_double() for _ in range(6)]
    _check(load().islbm_info(ctx, *[C.byref(v) for v in vals]), ctx)
    return dict(zip(("delta", "H_lu", "nu", "alpha", "aT", "gbeta"), [v.value for v in vals]))


def islbm_time(ctx) -> int:
    return load().islbm_time(ctx)


def islbm_set_time(ctx, t: int) -> None:
    _check(load().islbm_set_time(ctx, int(t)), ctx)


def islbm_sync(ctx) -> None:
    _check(load().islbm_sync(ctx), ctx)


def islbm_destroy(ctx) -> None:
    load().islbm_destroy(ctx)


def islbm_strerror(code: int) -> str:
    return load().islbm_strerror(code).decode()


# ----------------------------------------------------------------- wrapper

class Cavity:
    """Side-heated cavity on one GPU.  PyTorch provides the four population
    buffers (uint8 tensors on ``device``) and the stream; the library does the
    rest.  ``spacings`` is one array of n[a]+1 spacings per axis."""

    def __init__(self, spacings, Ra: float, Pr: float, storage="fp32", device="cuda:0",
                 use_torch_buffers: bool = True, own_stream: bool = False, **opts):
        import torch

        self.dim = len(spacings)
        self.n = [len(s) - 1 for s in spacings]
        self.shape = tuple(reversed(self.n))
        self.qf, self.qg = (9, 5) if self.dim == 2 else (19, 7)
        self.lattice = ISLBM_D2Q9_D2Q5 if self.dim == 2 else ISLBM_D3Q19_D3Q7
        o = islbm_default_options()
        o.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        for k, v in opts.items():
            setattr(o, k, v)
        self.device = torch.device(device)
        self._torch = torch
        with torch.cuda.device(self.device):
            # torch's current stream, or (own_stream) a stream of the library's
            # own, so that several cavities advance concurrently
            self.stream = None if own_stream else torch.cuda.current_stream(self.device)
            o.stream = None if own_stream else self.stream.cuda_stream
            self._bufs = []
            if use_torch_buffers:
                fb, gb = islbm_query_bytes(self.lattice, self.n, o.storage)
                self._bufs = [torch.empty(b, dtype=torch.uint8, device=self.device)
                              for b in (fb, fb, gb, gb)]
                for i, t in enumerate(self._bufs):
                    o.buffers[i] = t.data_ptr()
            self.options = o
            self.ctx = islbm_create(self.lattice, self.n, spacings, Ra, Pr, o)

    def close(self) -> None:
        if getattr(self, "ctx", None) is not None:
            islbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: the library may be gone already
            pass

    def step(self, n: int) -> None:
        islbm_step(self.ctx, n)

    def plan(self, n: int) -> None:
        islbm_plan_steps(self.ctx, n)

    def time_steps(self, n: int) -> float:
        return islbm_time_steps(self.ctx, n)

    def time_steps_split(self, n: int) -> tuple:
        return islbm_time_steps_split(self.ctx, n)

    def stats(self, allow_nonfinite: bool = False) -> dict:
        return islbm_nu_re(self.ctx, allow_nonfinite)

    def fields(self) -> dict:
        return islbm_fields(self.ctx, self.shape)

    def steady_change(self) -> tuple:
        return islbm_steady_change(self.ctx)

    def populations(self):
        return islbm_get_populations(self.ctx, self.qf, self.qg, self.shape)

    def set_populations(self, f, g, post_collision: bool) -> None:
        islbm_set_populations(self.ctx, f, g, post_collision)

    def save_state(self) -> bytes:
        return islbm_save_state(self.ctx)

    def load_state(self, blob: bytes) -> None:
        islbm_load_state(self.ctx, blob)

    def init_fields(self, ux, uy, uz, T) -> None:
        islbm_init_fields(self.ctx, ux, uy, uz, T)

    @property
    def info(self) -> dict:
        return islbm_info(self.ctx)

    @property
    def t(self) -> int:
        return islbm_time(self.ctx)

    def sync(self) -> None:
        islbm_sync(self.ctx)

"""ctypes wrapper of the FP64 ISLBM oracle (``islbm_oracle.c``).

Test infrastructure only: the test-suite, the smoke check and the CPU-baseline
leg of ``bench.py`` use it.  The product package never imports it.

Population arrays are ``[q][nz][ny][nx]`` (x fastest), float64, in the
interface ordering of the velocity sets (see ``lattice``).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "islbm_oracle.c")
# ISLBM_ORACLE_LIB selects another build of the same source (the sanitizer
# test runs the oracle pins against an AddressSanitizer build this way)
_LIB = os.environ.get("ISLBM_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

STATS = ("nu_vol", "nu_hot", "nu_cold", "nu_mid", "re_vol", "re_uv", "mass",
         "rho_sum", "umax", "vmax", "wmax", "nonfinite", "re_rms")

MESH_KINDS = {"uniform": 0, "erf": 1, "cosine": 2, "tanh": 3}


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C99, IEEE FP64, optional OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-std=gnu99", "-O2", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None
_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int)
_L = C.POINTER(C.c_long)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.environ.get("ISLBM_ORACLE_LIB") and (
            not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
        build()
    lib = C.CDLL(_LIB)
    lib.oracle_create.restype = C.c_void_p
    lib.oracle_create.argtypes = [C.c_int, _I, _D, _D, _D, C.c_double, C.c_double,
                                  C.c_double, C.c_double, C.c_double]
    lib.oracle_destroy.argtypes = [C.c_void_p]
    for name in ("oracle_set_state", "oracle_get_state", "oracle_set_post", "oracle_get_post"):
        getattr(lib, name).argtypes = [C.c_void_p, _D, _D]
    lib.oracle_params.argtypes = [C.c_void_p, _D]
    lib.oracle_override.argtypes = [C.c_void_p, _D, _D, _D, C.c_int]
    lib.oracle_get_rates.argtypes = [C.c_void_p, _D, _D]
    lib.oracle_collide.argtypes = [C.c_void_p]
    lib.oracle_stream.argtypes = [C.c_void_p]
    lib.oracle_run.argtypes = [C.c_void_p, C.c_long]
    lib.oracle_stats.argtypes = [C.c_void_p, _D]
    lib.oracle_fields.argtypes = [C.c_void_p, _D, _D, _D, _D, _D]
    lib.oracle_collide_node.argtypes = [C.c_void_p, _D, _D, _D, _D]
    lib.oracle_stream_node.argtypes = [C.c_void_p, _D, _D, C.c_long, _D, _D]
    lib.oracle_sample_step.argtypes = [C.c_void_p, _D, _D, _L, C.c_long, _D, _D]
    lib.oracle_lattice.restype = C.c_int
    lib.oracle_lattice.argtypes = [C.c_int, C.c_int, _I, _D, _D]
    lib.oracle_mesh.restype = C.c_int
    lib.oracle_mesh.argtypes = [C.c_int, C.c_int, C.c_double, _D]
    lib.oracle_meq.argtypes = [C.c_int, C.c_double, _D, _D]
    lib.oracle_mforce.argtypes = [C.c_int, _D, _D, _D]
    lib.oracle_neq.argtypes = [C.c_int, C.c_double, C.c_double, _D, _D]
    lib.oracle_lagrange3.argtypes = [_D, C.c_double, C.c_double, _D]
    lib.oracle_wall_derivative.restype = C.c_double
    lib.oracle_wall_derivative.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double,
                                           C.c_double]
    lib.oracle_set_threads.argtypes = [C.c_int]
    lib.oracle_get_threads.restype = C.c_int
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def mesh(kind: str, n: int, a: float = 1.5) -> np.ndarray:
    """Node coordinates x_0..x_{N+1} (N fluid nodes, ghost mirrors at both ends)."""
    x = np.zeros(n + 2)
    if _load().oracle_mesh(MESH_KINDS[kind], n, a, _dp(x)) != 0:
        raise ValueError("bad mesh request")
    return x


def lattice(dim: int, which: int):
    """(e [q,3] int, w [q] (flow set only, else zeros), M [q,q]) of a lattice."""
    q = {(2, 0): 9, (2, 1): 5, (3, 0): 19, (3, 1): 7}[(dim, which)]
    e = np.zeros((q, 3), dtype=np.int32)
    w = np.zeros(q)
    m = np.zeros((q, q))
    _load().oracle_lattice(dim, which, e.ctypes.data_as(_I), _dp(w), _dp(m))
    return e, w, m


def meq(dim: int, rho: float, u) -> np.ndarray:
    out = np.zeros(9 if dim == 2 else 19)
    uu = _f64(list(u) + [0.0] * (3 - len(u)))
    _load().oracle_meq(dim, rho, _dp(uu), _dp(out))
    return out


def mforce(dim: int, u, F) -> np.ndarray:
    out = np.zeros(9 if dim == 2 else 19)
    uu = _f64(list(u) + [0.0] * (3 - len(u)))
    FF = _f64(list(F) + [0.0] * (3 - len(F)))
    _load().oracle_mforce(dim, _dp(uu), _dp(FF), _dp(out))
    return out


def neq(dim: int, aT: float, T: float, u) -> np.ndarray:
    out = np.zeros(5 if dim == 2 else 7)
    uu = _f64(list(u) + [0.0] * (3 - len(u)))
    _load().oracle_neq(dim, aT, T, _dp(uu), _dp(out))
    return out


def lagrange3(xs, xd: float, delta: float) -> np.ndarray:
    w = np.zeros(3)
    xs = _f64(xs)
    _load().oracle_lagrange3(_dp(xs), xd, delta, _dp(w))
    return w


def wall_derivative(top: int, q: float, phiw: float, phi1: float, phi2: float) -> float:
    return _load().oracle_wall_derivative(top, q, phiw, phi1, phi2)


def steady_change(before: dict, after: dict) -> tuple:
    """Steady-state measure of Sec. 3 (its convergence criterion, applied in
    the paper to fields 2000 steps apart): the summed 2-norm of the velocity
    change over the summed 2-norm of the earlier velocity, and the summed
    absolute temperature change over the summed absolute earlier
    temperature.  ``before`` / ``after`` are field dicts as from
    ``Oracle.fields`` (uz may be absent or zero in 2-D)."""
    def vel(f):
        uz = f.get("uz")
        return f["ux"], f["uy"], (np.zeros_like(f["ux"]) if uz is None else uz)

    bx, by, bz = vel(before)
    ax, ay, az = vel(after)
    num_u = np.sum(np.sqrt((ax - bx) ** 2 + (ay - by) ** 2 + (az - bz) ** 2))
    den_u = np.sum(np.sqrt(bx ** 2 + by ** 2 + bz ** 2))
    num_T = np.sum(np.abs(after["T"] - before["T"]))
    den_T = np.sum(np.abs(before["T"]))
    return float(num_u / den_u), float(num_T / den_T)


def set_threads(n: int) -> None:
    _load().oracle_set_threads(n)


def get_threads() -> int:
    return _load().oracle_get_threads()


class Oracle:
    """One cavity: ``dim`` 2 or 3, node coordinates per axis (each N+2 long)."""

    def __init__(self, coords, Ra: float, Pr: float, uf: float = 0.0,
                 Thot: float = 0.5, Tcold: float = -0.5):
        lib = _load()
        self.dim = len(coords)
        self.Ra, self.Pr = Ra, Pr
        self.coords = [_f64(c) for c in coords]
        self.n = [len(c) - 2 for c in self.coords]
        n3 = (C.c_int * 3)(*(self.n + [1] * (3 - self.dim)))
        xs = [_dp(c) for c in self.coords] + [None] * (3 - self.dim)
        self._h = lib.oracle_create(self.dim, n3, xs[0], xs[1], xs[2], Ra, Pr, uf, Thot, Tcold)
        if not self._h:
            raise ValueError("oracle_create failed")
        self.qf = 9 if self.dim == 2 else 19
        self.qg = 5 if self.dim == 2 else 7
        self.shape = tuple(reversed(self.n))  # (ny, nx) or (nz, ny, nx)
        self.lib = lib

    def __del__(self):
        if getattr(self, "_h", None):
            self.lib.oracle_destroy(self._h)
            self._h = None

    @property
    def params(self) -> dict:
        out = np.zeros(10)
        self.lib.oracle_params(self._h, _dp(out))
        keys = ("delta", "H_lu", "nu", "alpha", "gbeta", "aT", "omega", "uf", "T0", "s_nu")
        return dict(zip(keys, out.tolist()))

    def rates(self):
        S = np.zeros(self.qf)
        Q = np.zeros(self.qg)
        self.lib.oracle_get_rates(self._h, _dp(S), _dp(Q))
        return S, Q

    def override(self, S=None, Q=None, gbeta=None, collide: bool = True) -> None:
        s = _f64(S) if S is not None else None
        q = _f64(Q) if Q is not None else None
        gb = _f64([gbeta]) if gbeta is not None else None
        self.lib.oracle_override(self._h, _dp(s) if s is not None else None,
                                 _dp(q) if q is not None else None,
                                 _dp(gb) if gb is not None else None, 1 if collide else 0)

    def _pair(self):
        f = np.zeros((self.qf,) + self.shape)
        g = np.zeros((self.qg,) + self.shape)
        return f, g

    def set_state(self, f, g) -> None:
        f, g = _f64(f), _f64(g)
        self.lib.oracle_set_state(self._h, _dp(f), _dp(g))

    def state(self):
        f, g = self._pair()
        self.lib.oracle_get_state(self._h, _dp(f), _dp(g))
        return f, g

    def set_post(self, fp, gp) -> None:
        fp, gp = _f64(fp), _f64(gp)
        self.lib.oracle_set_post(self._h, _dp(fp), _dp(gp))

    def post(self):
        f, g = self._pair()
        self.lib.oracle_get_post(self._h, _dp(f), _dp(g))
        return f, g

    def collide(self) -> None:
        self.lib.oracle_collide(self._h)

    def stream(self) -> None:
        self.lib.oracle_stream(self._h)

    def run(self, nsteps: int) -> None:
        self.lib.oracle_run(self._h, int(nsteps))

    def stats(self) -> dict:
        out = np.zeros(len(STATS))
        self.lib.oracle_stats(self._h, _dp(out))
        return dict(zip(STATS, out.tolist()))

    def fields(self):
        arrs = [np.zeros(self.shape) for _ in range(5)]
        self.lib.oracle_fields(self._h, *[_dp(a) for a in arrs])
        return dict(zip(("rho", "ux", "uy", "uz", "T"), arrs))

    def collide_node(self, f, g):
        f, g = _f64(f), _f64(g)
        fo = np.zeros(self.qf)
        go = np.zeros(self.qg)
        self.lib.oracle_collide_node(self._h, _dp(f), _dp(g), _dp(fo), _dp(go))
        return fo, go

    def sample_step(self, fp, gp, nodes):
        """One step (stream, collide) at the flat node indices ``nodes`` from
        post-collision arrays; returns post-collision values [count, q]."""
        fp, gp = _f64(fp), _f64(gp)
        nodes = np.ascontiguousarray(nodes, dtype=np.int64)
        fo = np.zeros((len(nodes), self.qf))
        go = np.zeros((len(nodes), self.qg))
        self.lib.oracle_sample_step(self._h, _dp(fp), _dp(gp), nodes.ctypes.data_as(_L),
                                    len(nodes), _dp(fo), _dp(go))
        return fo, go

"""Shared helpers of the GPU tests (no method arithmetic here)."""
from __future__ import annotations

import numpy as np

import oracle
import paper_2509_01099_amd as pkg


def lu_spacings(kind: str, n: int, a: float = 1.5) -> np.ndarray:
    """Library mesh spacings rescaled to lattice units (first spacing 1), so
    axes of different node counts share one lattice unit."""
    sp = pkg.islbm_mesh_spacing(kind, n, a)
    return sp / sp[0]


def coords(sp: np.ndarray) -> np.ndarray:
    return np.concatenate([[0.0], np.cumsum(sp)])


def rel_f(a: np.ndarray, b: np.ndarray) -> float:
    """max |a - b| / |b| (flow populations are bounded away from 0)."""
    return float(np.max(np.abs(a - b) / np.abs(b)))


def rel_g(a: np.ndarray, b: np.ndarray) -> float:
    """max |a - b| / max |b| (thermal populations vanish in places)."""
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def rel(a: float, b: float) -> float:
    return abs(a - b) / abs(b)


def make_pair(meshes, Ra, Pr, storage="fp32", **opts):
    """(GPU cavity, oracle) on the same lattice-unit mesh."""
    sp = [lu_spacings(k, n, a) for (k, n, a) in meshes]
    cav = pkg.Cavity(sp, Ra, Pr, storage=storage, **opts)
    okw = {}
    for key, name in (("u_f", "uf"), ("T_hot", "Thot"), ("T_cold", "Tcold")):
        if key in opts:
            okw[name] = opts[key]
    orc = oracle.Oracle([coords(s) for s in sp], Ra, Pr, **okw)
    return cav, orc

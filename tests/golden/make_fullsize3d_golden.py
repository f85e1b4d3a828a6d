"""Writes fullsize3d_tanh256_100steps.json: the FP64 oracle's populations at
sampled nodes (and its statistics) after 100 steps of the 256^3 tanh-mesh
cavity at Ra = 1e7 (the 3-D FP32 benchmark size), started from a seeded
random post-collision state.

Calls only ``oracle`` and the seeded input generators.  The case is the cubic
side-heated cavity of Sec. 4 (hot wall x = 0, cold wall x = 1, the other
walls adiabatic and no-slip), D3Q19 + D3Q7 MRT.  The free-fall velocity is
the largest one with a non-negative rest weight of the thermal equilibrium
(a_T = 1), capped at the Ma = 0.1 value.

The GPU keeps FP32 deviations f_i - w_i, so the oracle starts from the input
rounded that way: f = w + fl32(f_random - w), g = fl32(g_random).  The test
checks that the library holds exactly these values before it steps.

Usage: python tests/golden/make_fullsize3d_golden.py [--threads N]
(about 15 minutes on 8 cores, 16 GB of memory).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from tests.seeded import random_populations, random_scalar_populations  # noqa: E402

N = 256
RA, PR = 1e7, 0.71
STEPS = 100
SEED_F, SEED_G, SEED_NODES = 21, 22, 23
AMP_F, AMP_G = 0.05, 0.5
SAMPLES = 1200


def lattice_spacings(n: int) -> np.ndarray:
    """tanh-mesh spacings (a = 1.5) in lattice units (first spacing 1)."""
    x = oracle.mesh("tanh", n, 1.5)
    sp = np.diff(x)
    return sp / sp[0]


def free_fall_velocity(coords: np.ndarray) -> float:
    """u_f with a_T = 1 (D3Q7: a_T = 42 sqrt(3) alpha - 6, alpha = u_f H / sqrt(Ra Pr)),
    capped at the Ma = 0.1 value."""
    H = 0.5 * (coords[-1] + coords[-2]) - 0.5 * (coords[0] + coords[1])
    return min(0.1 / 3 ** 0.5, 7.0 / (42.0 * 3 ** 0.5) * (RA * PR) ** 0.5 / H)


def fp32_deviation_input(shape, w):
    """The seeded random post-collision state as the FP32-deviation store holds it."""
    f = random_populations(shape, w, AMP_F, seed=SEED_F)
    for i, wi in enumerate(w):
        f[i] = (f[i] - wi).astype(np.float32).astype(np.float64) + wi
    g = random_scalar_populations(shape, 7, AMP_G, seed=SEED_G)
    g = g.astype(np.float32).astype(np.float64)
    return f, g


def sample_nodes(n: int, rng: np.random.Generator, count: int) -> np.ndarray:
    """Flat indices (x fastest) of corners, wall and tile-seam nodes and
    random interior nodes of an n^3 mesh."""
    special = [0, 1, 2, 3, 4, 5, 7, 8, 31, 32, 33, 63, 64, n // 2, n - 6, n - 5, n - 4, n - 3, n - 2, n - 1]
    picks = [[int(rng.choice(special)) for _ in range(3)] for _ in range(count // 2)]
    picks += [[int(rng.integers(0, n)) for _ in range(3)] for _ in range(count - count // 2)]
    flat = [x + n * (y + n * z) for x, y, z in picks]
    return np.unique(np.array(flat, dtype=np.int64))


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--out", default=os.path.join(HERE, "fullsize3d_tanh256_100steps.json"))
    args = ap.parse_args()
    oracle.set_threads(args.threads)
    sp = lattice_spacings(N)
    coords = np.concatenate([[0.0], np.cumsum(sp)])
    uf = free_fall_velocity(coords)
    orc = oracle.Oracle([coords, coords, coords], RA, PR, uf=uf)
    _, w, _ = oracle.lattice(3, 0)
    t0 = time.time()
    f, g = fp32_deviation_input(orc.shape, w)
    in_sums = [float(np.sum(f)), float(np.sum(g))]
    g_absmax = float(np.abs(g).max())
    orc.set_post(f, g)
    del f, g
    orc.stream()
    orc.run(STEPS - 1)
    orc.collide()
    print(f"oracle: {STEPS} steps in {time.time() - t0:.0f} s", flush=True)
    fo, go = orc.post()
    # size of the volume-averaged convective term of <Nu> (random states make
    # it cancel, so the relative bar of <Nu> is taken against it)
    p, fl = orc.params, orc.fields()
    nu_conv = float(np.sqrt(RA * PR) * np.mean(np.abs(fl["ux"] / p["uf"] * (fl["T"] - p["T0"]))))
    del fl
    nodes = sample_nodes(N, np.random.default_rng(SEED_NODES), SAMPLES)
    out = {
        "source": "FP64 oracle (oracle/islbm_oracle.c), written by tests/golden/make_fullsize3d_golden.py",
        "case": "3-D side-heated cubic cavity (Sec. 4), 256^3 tanh mesh (a = 1.5), Ra 1e7, Pr 0.71, "
                "walls +-0.5, D3Q19 + D3Q7 MRT, 100 steps from a seeded random post-collision state",
        "n": N, "Ra": RA, "Pr": PR, "u_f": uf, "steps": STEPS,
        "seeds": {"f": SEED_F, "g": SEED_G, "nodes": SEED_NODES}, "amplitudes": {"f": AMP_F, "g": AMP_G},
        "spacings": sp.tolist(),
        "input_sums": in_sums,
        "stats": orc.stats(),
        "nu_vol_convective_scale": nu_conv,
        "nodes": nodes.tolist(),
        "f": fo.reshape(19, -1)[:, nodes].T.tolist(),
        "g": go.reshape(7, -1)[:, nodes].T.tolist(),
        "g_in_absmax": g_absmax,
    }
    with open(args.out, "w") as fh:
        json.dump(out, fh)
    print(f"wrote {args.out}: {len(nodes)} nodes", flush=True)


if __name__ == "__main__":
    main()

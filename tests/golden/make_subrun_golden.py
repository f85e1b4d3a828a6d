"""Writes subrun_cosine256_ra1e8.json: the FP64 oracle's statistics of the
256^2 cosine-mesh cavity at Ra = 1e8 (the 256^2 subrun of the 1024^2
benchmark workload) over 200 000 steps from rest.

Calls only ``oracle``.  The run is the side-heated cavity of Sec. 3 (hot wall
x = 0, cold wall x = 1, adiabatic top and bottom, start at rest with T = 0
inside), D2Q9 + D2Q5 MRT.  The free-fall velocity is the largest one with a
non-negative rest weight of the thermal equilibrium (a_T = 1), as in the
benchmark; the stated Ma = 0.1 velocity gives a_T = 2.35 on this mesh.

Usage: python tests/golden/make_subrun_golden.py [--threads N]
(about 10 minutes on 8 cores).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

N = 256
RA, PR = 1e8, 0.71
CHECKPOINTS = (100, 2000, 20000, 50000, 100000, 150000, 200000)
STRIDE = 16  # field samples on every 16th node per axis


def lattice_coords(n: int) -> np.ndarray:
    """Cosine-mesh coordinates x_0..x_{N+1} in lattice units (first spacing 1)."""
    x = oracle.mesh("cosine", n, 0.0)
    return (x - x[0]) / (x[1] - x[0])


def subrun_uf(x: np.ndarray) -> float:
    """u_f with a_T = 1 (D2Q5: a_T = 20 sqrt(3) alpha - 4, alpha = u_f H / sqrt(Ra Pr)),
    capped at the Ma = 0.1 value."""
    H = 0.5 * (x[-1] + x[-2]) - 0.5 * (x[0] + x[1])
    return min(0.1 / 3 ** 0.5, 5.0 / (20.0 * 3 ** 0.5) * (RA * PR) ** 0.5 / H)


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--out", default=os.path.join(HERE, "subrun_cosine256_ra1e8.json"))
    args = ap.parse_args()
    oracle.set_threads(args.threads)
    x = lattice_coords(N)
    uf = subrun_uf(x)
    orc = oracle.Oracle([x, x], RA, PR, uf=uf)
    out = {
        "source": "FP64 oracle (oracle/islbm_oracle.c), written by tests/golden/make_subrun_golden.py",
        "case": "2-D side-heated cavity (Sec. 3), 256^2 cosine mesh x_j = (1 - cos(pi j/257))/2, "
                "Ra 1e8, Pr 0.71, walls +-0.5, start at rest, D2Q9 + D2Q5 MRT",
        "n": N, "Ra": RA, "Pr": PR, "u_f": uf, "params": orc.params,
        "sample_stride": STRIDE, "checkpoints": {},
    }
    done, t0 = 0, time.time()
    for c in CHECKPOINTS:
        orc.run(c - done)
        done = c
        st = orc.stats()
        fl = orc.fields()
        sl = (slice(STRIDE // 2, None, STRIDE), slice(STRIDE // 2, None, STRIDE))
        out["checkpoints"][str(c)] = {
            "stats": st,
            "ux": fl["ux"][sl].round(17).tolist(),
            "uy": fl["uy"][sl].round(17).tolist(),
            "T": fl["T"][sl].round(17).tolist(),
        }
        print(f"step {c}: nu_vol {st['nu_vol']:.10g} nu_hot {st['nu_hot']:.10g} "
              f"re_vol {st['re_vol']:.10g} ({time.time() - t0:.0f} s)", flush=True)
    with open(args.out, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()

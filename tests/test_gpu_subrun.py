"""The 256^2 subrun of the 1024^2 benchmark workload, run to its full length
(2-D side-heated cavity, cosine mesh, Ra = 1e8, Pr = 0.71, from rest,
200 000 steps), against the FP64 oracle's statistics written by
tests/golden/make_subrun_golden.py (oracle only).

Bar: 1e-4 relative at the end of the run on the volume, hot- and cold-wall
Nusselt numbers, the two Reynolds numbers and the peak velocities (Sec. 3
definitions).  The mid-plane Nusselt number is zero up to round-off here
(the from-rest start is centro-symmetric), so it is held to 1e-4 of the
conduction value 1 instead.  The intermediate checkpoints are printed, not
asserted.

FP32 storage with FP32 arithmetic does not meet the end-of-run bar: on this
mesh the centre cells are ~160 lattice units wide, so a step moves a
population by ~1/160 of its difference to the neighbour, and the thermal
populations (stored as values of order 0.1, not as deviations) lose part of
that increment to round-to-nearest at every step, in the same direction
step after step.  The hot-wall Nusselt number drifts from the FP64 run
roughly linearly in time (4e-5 at 2 000 steps, 1.2e-3 at 50 000, 3.2e-3 at
200 000, measured on MI355X).  FP32 storage with FP64 arithmetic and
stochastic rounding on store (fp32sr) meets the bar; the FP32 case is kept
as a regression check of its measured drift (bar 5e-3)."""
import json
import os

import numpy as np
import pytest

import paper_2509_01099_amd as pkg
from tests.helpers import lu_spacings

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "subrun_cosine256_ra1e8.json")
KEYS = ("nu_vol", "nu_hot", "nu_cold", "re_vol", "re_rms", "umax", "vmax")


@pytest.mark.parametrize("storage", ["fp32", "fp32sr"])
def test_subrun_cosine256_ra1e8_200k_steps(storage):
    with open(GOLDEN) as f:
        gold = json.load(f)
    sp = lu_spacings("cosine", gold["n"], 0)
    cav = pkg.Cavity([sp, sp], gold["Ra"], gold["Pr"], storage=storage, u_f=gold["u_f"])
    done, errs = 0, {}
    stride = gold["sample_stride"]
    sl = (slice(stride // 2, None, stride), slice(stride // 2, None, stride))
    for c in sorted(int(k) for k in gold["checkpoints"]):
        cav.step(c - done)
        done = c
        st = cav.stats()
        ref = gold["checkpoints"][str(c)]
        errs = {k: abs(st[k] - ref["stats"][k]) / abs(ref["stats"][k]) for k in KEYS}
        errs["nu_mid(abs)"] = abs(st["nu_mid"] - ref["stats"]["nu_mid"])
        fl = cav.fields()
        eT = float(np.max(np.abs(fl["T"][sl] - np.array(ref["T"]))))
        umax = max(np.abs(np.array(ref["ux"])).max(), np.abs(np.array(ref["uy"])).max(), 1e-30)
        eu = float(max(np.max(np.abs(fl["ux"][sl] - np.array(ref["ux"]))),
                       np.max(np.abs(fl["uy"][sl] - np.array(ref["uy"]))))) / umax
        print(f"{storage} step {c}: " + " ".join(f"{k} {v:.1e}" for k, v in errs.items())
              + f" | sampled T abs {eT:.1e}, u rel {eu:.1e}", flush=True)
    cav.close()
    bar = 1e-4 if storage == "fp32sr" else 5e-3
    for k in KEYS:
        assert errs[k] <= bar, (storage, k, errs[k])
    assert errs["nu_mid(abs)"] <= 1e-4, errs["nu_mid(abs)"]

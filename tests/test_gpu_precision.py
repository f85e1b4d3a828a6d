"""Reduced-precision storage (FP16 / BF16 deviations, FP32 arithmetic) against
the FP64 oracle.  The bars are set by the storage precision: one rounding of
each deviation per step (2^-11 relative for FP16, 2^-8 for BF16), growing like
a random walk over the run; they are stated, not fitted."""
import numpy as np
import pytest

import oracle
from tests.helpers import make_pair, rel_f, rel_g
from tests.seeded import random_populations, random_scalar_populations

pytestmark = pytest.mark.gpu

STEPS = 100
# unit roundoff of the stored deviations (FP16 11 significant bits, BF16 8)
UNIT = {"fp16": 2.0 ** -11, "bf16": 2.0 ** -8}


def bars(storage):
    """Rounding of every stored value once per step, accumulated like a
    random walk over the run, with a factor 3 of headroom: e = 3 sqrt(K) u.
    g and the statistics are measured against their maximum; f against
    itself, where the deviations are at most ~10 % of f for these states."""
    e = 3.0 * np.sqrt(STEPS) * UNIT[storage]
    return 0.1 * e, e, e


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
@pytest.mark.parametrize("dim,kind,nz", [(2, "tanh", 0), (3, "tanh", 18), (3, "uniform", 18), (3, "uniform", 40)])
def test_reduced_storage_vs_oracle(storage, dim, kind, nz):
    """nz = 40 takes the 3-D march across a z-segment boundary (32 planes),
    with columns cut short in x (70) and y (37)."""
    oracle.set_threads(16)
    a = 0 if kind == "uniform" else 1.5
    meshes = [(kind, 70, a), (kind, 37, a), (kind, nz, a)][:dim]
    cav, orc = make_pair(meshes, 1e6 if dim == 2 else 1e7, 0.71, storage=storage)
    _, w, _ = oracle.lattice(dim, 0)
    f = random_populations(orc.shape, w, 0.05, seed=21)
    g = random_scalar_populations(orc.shape, orc.qg, 0.5, seed=22)
    cav.set_populations(f, g, post_collision=False)
    orc.set_state(f, g)
    cav.step(STEPS)
    orc.run(STEPS)
    fp, gp = cav.populations()
    orc.collide()
    ofp, ogp = orc.post()
    st, ost = cav.stats(), orc.stats()
    ef, eg = rel_f(fp, ofp), rel_g(gp, ogp)
    fb, gb, sb = bars(storage)
    errs = {k: abs(st[k] - ost[k]) / max(abs(ost[k]), 1.0) for k in ("nu_hot", "nu_cold")}
    errs["re_vol"] = abs(st["re_vol"] - ost["re_vol"]) / abs(ost["re_vol"])
    print(f"{storage} {dim}d {kind} nz {nz}: f {ef:.2e} g {eg:.2e} " +
          " ".join(f"{k} {v:.1e}" for k, v in errs.items()), flush=True)
    assert ef < fb and eg < gb
    assert all(v < sb for v in errs.values())
    cav.close()


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_reduced_storage_rest_state_exact(storage):
    """Deviation storage keeps the rest state exactly (all deviations zero)."""
    cav, orc = make_pair([("cosine", 40, 0), ("cosine", 30, 0)], 1e6, 0.71, storage=storage,
                         T_hot=0.0, T_cold=0.0, allow_unstable=1)
    cav.step(50)
    f, g = cav.populations()
    _, w, _ = oracle.lattice(2, 0)
    assert np.array_equal(f, np.broadcast_to(w[:, None, None], f.shape))
    assert not np.any(g)
    cav.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_fp32_storage_fp64_arithmetic_vs_oracle(dim):
    """FP32 storage with FP64 arithmetic and stochastic rounding on store:
    within the FP32 bars of the parity tests after 100 steps."""
    oracle.set_threads(16)
    meshes = [("tanh", 70, 1.5), ("tanh", 37, 1.5), ("tanh", 18, 1.5)][:dim]
    cav, orc = make_pair(meshes, 1e6 if dim == 2 else 1e7, 0.71, storage="fp32sr")
    _, w, _ = oracle.lattice(dim, 0)
    f = random_populations(orc.shape, w, 0.05, seed=31)
    g = random_scalar_populations(orc.shape, orc.qg, 0.5, seed=32)
    cav.set_populations(f, g, post_collision=False)
    orc.set_state(f, g)
    cav.step(100)
    orc.run(100)
    fp, gp = cav.populations()
    orc.collide()
    ofp, ogp = orc.post()
    ef, eg = rel_f(fp, ofp), rel_g(gp, ogp)
    st, ost = cav.stats(), orc.stats()
    enu = abs(st["nu_hot"] - ost["nu_hot"]) / max(abs(ost["nu_hot"]), 1.0)
    print(f"fp32sr {dim}d: f {ef:.2e} g {eg:.2e} nu_hot {enu:.1e}", flush=True)
    assert ef <= 1e-5 and eg <= 1e-5 and enu <= 1e-4
    cav.close()

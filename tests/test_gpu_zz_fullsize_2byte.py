"""Parity of the 2-byte storage types at the 3-D 2-byte workload size (384^3
tanh mesh, Ra 1e7), in the launch configuration the benchmark times: one
fused step from a seeded post-collision state, compared with the oracle on
sampled nodes (corners, faces, tile seams and random interior nodes), each
recomputed by the oracle from the same stored input.  The inputs are
separable seeded fields, cheap at 5.7e7 nodes.  Bars: one rounding of each
stored deviation, at most one unit in the last place with stochastic
rounding (FP16 2^-10, BF16 2^-7 of the value), with headroom; f relative to
itself (deviations are at most ~6 % of f), g relative to its maximum."""
import numpy as np
import pytest

import oracle
import paper_2509_01099_amd as pkg
from tests.helpers import coords, lu_spacings, rel_f
from tests.seeded import separable_populations, separable_scalar_populations
from tests.test_gpu_fullsize import sample_nodes

pytestmark = pytest.mark.gpu

TOL = {"fp16": (1e-4, 2e-3), "bf16": (1.2e-3, 1.2e-2)}


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_one_step_384_cubed_sampled(storage):
    oracle.set_threads(16)
    n, Ra = (384, 384, 384), 1e7
    sp = [lu_spacings("tanh", k, 1.5) for k in n]
    H = coords(sp[1])
    H = 0.5 * (H[-1] + H[-2]) - 0.5 * (H[0] + H[1])
    alpha_max = 7.0 / (42.0 * 3 ** 0.5)
    uf = min(0.1 / 3 ** 0.5, alpha_max * (Ra * 0.71) ** 0.5 / H)
    print(f"384^3 tanh {storage}: u_f {uf:.3e}", flush=True)
    cav = pkg.Cavity(sp, Ra, 0.71, u_f=uf, storage=storage)
    orc = oracle.Oracle([coords(s) for s in sp], Ra, 0.71, uf=uf)
    shape = orc.shape
    _, w, _ = oracle.lattice(3, 0)
    fp = separable_populations(shape, w, 0.05, seed=41)
    gp = separable_scalar_populations(shape, orc.qg, 0.5, seed=42)
    cav.set_populations(fp, gp, post_collision=True)
    del fp, gp
    f_in, g_in = cav.populations()       # the stored (rounded) deviations
    cav.step(1)
    f_out, g_out = cav.populations()
    cav.close()
    nodes = sample_nodes(shape, np.random.default_rng(43))
    ofo, ogo = orc.sample_step(f_in, g_in, nodes)
    gf = f_out.reshape(orc.qf, -1)[:, nodes].T
    gg = g_out.reshape(orc.qg, -1)[:, nodes].T
    ef = rel_f(gf, ofo)
    eg = float(np.abs(gg - ogo).max() / np.abs(g_in).max())
    print(f"384^3 tanh {storage}: {len(nodes)} nodes, f {ef:.2e} g {eg:.2e}", flush=True)
    tf, tg = TOL[storage]
    assert ef < tf and eg < tg

"""Parity at the benchmark sizes, in the launch configuration the benchmark
times: one fused step from a seeded random post-collision state, compared
with the oracle on sampled nodes (corners, edges, walls, tile seams and
random interior nodes), each recomputed by the oracle from the same input."""
import numpy as np
import pytest

import oracle
import paper_2509_01099_amd as pkg
from tests.helpers import coords, lu_spacings, rel_f
from tests.seeded import random_populations, random_scalar_populations

pytestmark = pytest.mark.gpu


def sample_nodes(shape, rng, count=4000):
    """Flat indices: all 2^d corners, points on every face and tile seams,
    plus random interior nodes (shape is (nz, ny, nx) or (ny, nx))."""
    dims = shape[::-1]                      # x, y, (z)
    picks = []
    special = [[0, 1, 2, 31, 32, 63, 64, 65, n // 2, n - 3, n - 2, n - 1] for n in dims]
    for _ in range(count // 2):
        idx = [int(rng.choice(s)) % n for s, n in zip(special, dims)]
        picks.append(idx)
    for _ in range(count // 2):
        picks.append([int(rng.integers(0, n)) for n in dims])
    flat = []
    for idx in picks:
        f, stride = 0, 1
        for i, n in zip(idx, dims):
            f += i * stride
            stride *= n
        flat.append(f)
    return np.unique(np.array(flat, dtype=np.int64))


# one step of 2-byte storage: the stored deviation of a value is off by at most
# one unit in the last place after stochastic rounding (2^-10 of |g| in FP16)
TOL = {"fp32": (1e-5, 1e-5), "fp16": (1e-4, 2e-3), "fp32sr": (1e-5, 1e-5), "fp64": (1e-10, 1e-10)}


@pytest.mark.parametrize("dim,kind,n,Ra,storage", [
    (2, "cosine", (1024, 1024), 1e8, "fp32"),      # the benchmark workload
    (2, "erf", (2050, 1100), 1e8, "fp32"),         # beyond the last-level cache: large tiles
    (2, "erf", (4096, 2048), 1e8, "fp16"),         # 2-byte storage, large class
    (2, "cosine", (1024, 1024), 1e8, "fp32sr"),    # FP32 storage, FP64 arithmetic
    (2, "erf", (4096, 2048), 1e8, "fp64"),         # FP64 beyond 1 GB: streaming stores
    (3, "tanh", (256, 256, 256), 1e7, "fp32sr"),   # the same for FP64 arithmetic in 3-D
    (3, "tanh", (256, 256, 256), 1e7, "fp32"),     # the 3-D workload
    (3, "uniform", (256, 256, 256), 1e7, "fp32"),  # uniform 3-D: z-marching kernel
])
def test_one_step_full_size_sampled(dim, kind, n, Ra, storage):
    oracle.set_threads(16)
    sp = [lu_spacings(kind, k, 1.5) for k in n]
    H = coords(sp[1])
    H = 0.5 * (H[-1] + H[-2]) - 0.5 * (H[0] + H[1])
    alpha_max = 5.0 / (20.0 * 3 ** 0.5) if dim == 2 else 7.0 / (42.0 * 3 ** 0.5)
    uf = min(0.1 / 3 ** 0.5, alpha_max * (Ra * 0.71) ** 0.5 / H)
    cav = pkg.Cavity(sp, Ra, 0.71, u_f=uf, storage=storage)
    orc = oracle.Oracle([coords(s) for s in sp], Ra, 0.71, uf=uf)
    shape = orc.shape
    _, w, _ = oracle.lattice(dim, 0)
    fp = random_populations(shape, w, 0.05, seed=11)
    gp = random_scalar_populations(shape, orc.qg, 0.5, seed=12)
    cav.set_populations(fp, gp, post_collision=True)
    # the GPU keeps rounded deviations f - w: give the oracle the same stored values
    f_in, g_in = cav.populations()
    cav.step(1)
    f_out, g_out = cav.populations()
    cav.close()
    nodes = sample_nodes(shape, np.random.default_rng(13))
    ofo, ogo = orc.sample_step(f_in, g_in, nodes)
    gf = f_out.reshape(orc.qf, -1)[:, nodes].T
    gg = g_out.reshape(orc.qg, -1)[:, nodes].T
    ef = rel_f(gf, ofo)
    eg = float(np.abs(gg - ogo).max() / np.abs(g_in).max())
    print(f"{dim}d {kind} {n} {storage}: {len(nodes)} nodes, f {ef:.2e} g {eg:.2e}", flush=True)
    tf, tg = TOL[storage]
    assert ef < tf and eg < tg

"""GPU (HIP, through the C-ABI) vs the FP64 oracle, element by element.

Bars: FP32 storage/arithmetic within 1e-5 relative on populations after 100
steps and 1e-4 relative on the Nusselt / Reynolds numbers; FP64 within
1e-10 (round-off of a different summation order, grown over the run).
Meshes are chosen so that tiles are ragged in every direction.
"""
import numpy as np
import pytest

import oracle
import paper_2509_01099_amd as pkg
from tests.helpers import coords, lu_spacings, make_pair, rel, rel_f, rel_g
from tests.seeded import random_populations, random_scalar_populations

pytestmark = pytest.mark.gpu

STAT_KEYS = ("nu_vol", "nu_hot", "nu_cold", "nu_mid", "re_vol", "re_rms")


def _random_state(orc, seed):
    _, w, _ = oracle.lattice(orc.dim, 0)
    f = random_populations(orc.shape, w, 0.05, seed=seed)
    g = random_scalar_populations(orc.shape, orc.qg, 0.5, seed=seed + 100)
    return f, g


def _nu_scale(orc, key, ref):
    """Scale of a Nusselt number for its relative bar: the value itself,
    floored at 1 (the conduction value), and for the volume average also
    the size of the averaged convective term (random states make it cancel)."""
    scale = max(abs(ref), 1.0)
    if key == "nu_vol":
        p, fl = orc.params, orc.fields()
        conv = np.mean(np.abs(fl["ux"] / p["uf"] * (fl["T"] - p["T0"])))
        scale = max(scale, np.sqrt(orc.Ra * orc.Pr) * conv)
    return scale


def _compare(cav, orc, ftol, stol, what):
    fp, gp = cav.populations()
    orc.collide()
    ofp, ogp = orc.post()
    ef, eg = rel_f(fp, ofp), rel_g(gp, ogp)
    st, ost = cav.stats(), orc.stats()
    errs = {}
    for k in STAT_KEYS:
        scale = abs(ost[k]) if k.startswith("re_") else _nu_scale(orc, k, ost[k])
        errs[k] = abs(st[k] - ost[k]) / scale
    print(f"{what}: f {ef:.2e} g {eg:.2e} " + " ".join(f"{k} {v:.1e}" for k, v in errs.items()),
          flush=True)
    assert ef <= ftol and eg <= ftol, (ef, eg)
    for k in STAT_KEYS:
        assert errs[k] <= stol, (k, st[k], ost[k])
    return st, ost


@pytest.mark.parametrize("kind,seed", [("tanh", 0), ("erf", 1), ("cosine", 2)])
def test_parity_2d_fp32_random(kind, seed):
    """Seeded random pre-collision state, 100 steps, 150 x 70 (ragged tiles)."""
    cav, orc = make_pair([(kind, 150, 1.5), (kind, 70, 1.5)], 1e6, 0.71, allow_unstable=1)
    f, g = _random_state(orc, seed)
    cav.set_populations(f, g, post_collision=False)
    orc.set_state(f, g)
    cav.step(100)
    orc.run(100)
    _compare(cav, orc, 1e-5, 1e-4, f"2d fp32 {kind}")
    cav.close()


def test_parity_2d_fp32_from_rest_cosine64():
    """Start at rest (T = 0 inside, walls +-0.5) on the 64^2 cosine mesh with
    u_f = 0.1, Ra = 1e6 (the small 2-D workload), FP32, 100 steps."""
    cav, orc = make_pair([("cosine", 64, 0), ("cosine", 64, 0)], 1e6, 0.71, u_f=0.1,
                         allow_unstable=1)
    cav.step(100)
    orc.run(100)
    _compare(cav, orc, 1e-5, 1e-4, "2d fp32 rest")
    cav.close()


def test_parity_2d_cosine256_ra1e8_subrun():
    """The 256^2 subrun of the benchmark workload (cosine mesh, Ra = 1e8,
    Pr = 0.71, FP32, u_f at the a_T <= 1 limit as in the benchmark) against
    the FP64 oracle: 2000 steps from rest."""
    oracle.set_threads(16)
    sp = lu_spacings("cosine", 256, 0)
    H = coords(sp)
    H = 0.5 * (H[-1] + H[-2]) - 0.5 * (H[0] + H[1])
    uf = min(0.1 / 3 ** 0.5, 5.0 / (20.0 * 3 ** 0.5) * (1e8 * 0.71) ** 0.5 / H)
    cav, orc = make_pair([("cosine", 256, 0), ("cosine", 256, 0)], 1e8, 0.71, u_f=uf)
    cav.step(100)
    orc.run(100)
    _compare(cav, orc, 1e-5, 1e-4, "2d fp32 cosine 256 Ra 1e8, 100 steps")
    cav.step(1900)
    orc.run(1900)
    # FP32 rounding accumulates like a random walk: the 100-step population
    # bar grows by sqrt(2000 / 100)
    _compare(cav, orc, 1e-5 * 20 ** 0.5, 1e-4, "2d fp32 cosine 256 Ra 1e8, 2000 steps")
    cav.close()


def test_parity_2d_fp64_cosine64_full_run():
    """The small 2-D workload in full: 64^2 cosine, Ra = 1e6, Pr = 0.71,
    u_f = 0.1, FP64, 20000 steps from rest."""
    oracle.set_threads(16)
    cav, orc = make_pair([("cosine", 64, 0), ("cosine", 64, 0)], 1e6, 0.71, storage="fp64",
                         u_f=0.1, allow_unstable=1)
    cav.step(20000)
    orc.run(20000)
    _compare(cav, orc, 1e-10, 1e-10, "2d fp64 cosine 64 20k")
    cav.close()


@pytest.mark.parametrize("kind,seed", [("erf", 3), ("tanh", 4)])
def test_parity_3d_fp32_random(kind, seed):
    """Seeded random state, 100 steps, 40 x 22 x 18 (ragged in x, y and z)."""
    oracle.set_threads(16)
    cav, orc = make_pair([(kind, 40, 1.5), (kind, 22, 1.5), (kind, 18, 1.5)], 1e7, 0.71)
    f, g = _random_state(orc, seed)
    cav.set_populations(f, g, post_collision=False)
    orc.set_state(f, g)
    cav.step(100)
    orc.run(100)
    _compare(cav, orc, 1e-5, 1e-4, f"3d fp32 {kind}")
    cav.close()


@pytest.mark.parametrize("nx,nz,seed", [(36, 65, 7), (36, 67, 8), (100, 67, 9)])
def test_parity_3d_fp32_uniform_random(nx, nz, seed):
    """Uniform 3-D mesh (plain-shift streaming, z-marching kernel): nx x 20 x nz
    is ragged in x and y, and nz = 65 / 67 leaves a last z segment of one /
    three planes (32-plane segments of 64 x 8 columns for nx = 36; nx = 100
    takes the 128 x 4 columns of 64 planes, one column cut short in x)."""
    oracle.set_threads(16)
    cav, orc = make_pair([("uniform", nx, 0), ("uniform", 20, 0), ("uniform", nz, 0)], 1e7, 0.71)
    f, g = _random_state(orc, seed)
    cav.set_populations(f, g, post_collision=False)
    orc.set_state(f, g)
    cav.step(100)
    orc.run(100)
    _compare(cav, orc, 1e-5, 1e-4, f"3d fp32 uniform nx={nx} nz={nz}")
    cav.close()


@pytest.mark.parametrize("meshes", [
    [("tanh", 3, 1.5), ("tanh", 3, 1.5)],                          # smallest 2-D mesh
    [("erf", 5, 1.5), ("erf", 3, 1.5)],
    [("tanh", 3, 1.5), ("tanh", 3, 1.5), ("tanh", 3, 1.5)],        # smallest 3-D mesh
    [("uniform", 4, 0), ("uniform", 3, 0), ("uniform", 5, 0)],     # 3-D marching kernel
])
def test_parity_smallest_meshes(meshes):
    """Three fluid nodes per axis (every node a wall node, every stencil
    clamped), 100 steps from a seeded random state."""
    oracle.set_threads(16)
    cav, orc = make_pair(meshes, 1e6, 0.71, allow_unstable=1)
    f, g = _random_state(orc, 12)
    cav.set_populations(f, g, post_collision=False)
    orc.set_state(f, g)
    cav.step(100)
    orc.run(100)
    fp, gp = cav.populations()
    orc.collide()
    ofp, ogp = orc.post()
    ef, eg = rel_f(fp, ofp), rel_g(gp, ogp)
    print(f"{[m[1] for m in meshes]}: f {ef:.2e} g {eg:.2e}", flush=True)
    assert ef <= 1e-5 and eg <= 1e-5
    cav.close()


def test_zero_steps_is_a_no_op():
    """islbm_step(0) changes neither the state nor the time level."""
    cav, orc = make_pair([("tanh", 40, 1.5), ("tanh", 30, 1.5)], 1e6, 0.71)
    cav.step(7)
    f0, g0 = cav.populations()
    t0 = cav.t
    cav.step(0)
    f1, g1 = cav.populations()
    assert cav.t == t0 and np.array_equal(f0, f1) and np.array_equal(g0, g1)
    cav.close()


def test_parity_3d_fp64_random():
    oracle.set_threads(16)
    cav, orc = make_pair([("tanh", 21, 1.5), ("tanh", 19, 1.5), ("tanh", 9, 1.5)], 1e7, 0.71,
                         storage="fp64")
    f, g = _random_state(orc, 5)
    cav.set_populations(f, g, post_collision=False)
    orc.set_state(f, g)
    cav.step(60)
    orc.run(60)
    _compare(cav, orc, 1e-12, 1e-11, "3d fp64")
    cav.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_uniform_shift_kernel_is_bitwise_the_interpolating_kernel(dim):
    """Property (a) on the GPU: on a uniform mesh the interpolating kernel and
    the plain-shift kernel give bitwise equal states."""
    meshes = [("uniform", 67, 0), ("uniform", 35, 0), ("uniform", 10, 0)][:dim]
    a, orc = make_pair(meshes, 1e6, 0.71)
    b, _ = make_pair(meshes, 1e6, 0.71, force_interp=1)
    f, g = _random_state(orc, 6)
    for c in (a, b):
        c.set_populations(f, g, post_collision=False)
        c.step(50)
    fa, ga = a.populations()
    fb, gb = b.populations()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    a.close()
    b.close()


@pytest.mark.parametrize("dim,kind", [(2, "cosine"), (3, "erf")])
def test_stream_only_reproduces_quadratics(dim, kind):
    """Property (b) on the GPU: with collision off, per-axis quadratic
    post-collision fields stream to their values at the departure points."""
    n = [37, 20, 9][:dim]
    sp = [lu_spacings(kind, k, 1.5) for k in n]
    cav = pkg.Cavity(sp, 1e6, 0.71, stream_only=1, allow_unstable=1)
    X = np.meshgrid(*[coords(s)[1:-1] for s in sp[::-1]], indexing="ij")[::-1]
    rng = np.random.default_rng(7)
    e, _, _ = oracle.lattice(dim, 0)
    eg, _, _ = oracle.lattice(dim, 1)

    def fields(ev, polys, shift):
        out = []
        for p in range(len(ev)):
            v = np.ones(X[0].shape)
            for ax in range(dim):
                v = v * np.polyval(polys[p, ax], (X[ax] - shift * ev[p, ax]) / X[ax].max())
            out.append(0.05 * v + (0.2 if p == 0 else 0.05))
        return np.stack(out)

    pf = rng.normal(size=(len(e), dim, 3))
    pg = rng.normal(size=(len(eg), dim, 3))
    cav.set_populations(fields(e, pf, 0), fields(eg, pg, 0), post_collision=True)
    cav.step(1)
    f, g = cav.populations()
    for arr, ev, polys in ((f, e, pf), (g, eg, pg)):
        expect = fields(ev, polys, 1.0)
        for p in range(len(ev)):
            mask = np.ones(X[0].shape, bool)
            for ax in range(dim):
                sl = [slice(None)] * dim
                if ev[p, ax] != 0:
                    sl[dim - 1 - ax] = 0 if ev[p, ax] == 1 else -1
                    mask[tuple(sl)] = False
            err = np.abs(arr[p][mask] - expect[p][mask]).max() / np.abs(expect[p]).max()
            assert err < 2e-6, (p, err)
    cav.close()


@pytest.mark.parametrize("dim,storage,tol", [(2, "fp32", 1e-5), (2, "fp64", 1e-11),
                                             (3, "fp32", 1e-5)])
def test_steady_change_matches_oracle(dim, storage, tol):
    """Sec. 3 steady-state measure between two times 50 steps apart from a
    seeded random state, against the oracle's fields at the same times."""
    oracle.set_threads(16)
    meshes = [("erf", 46, 1.5), ("erf", 30, 1.5), ("erf", 12, 1.5)][:dim]
    cav, orc = make_pair(meshes, 1e6, 0.71, storage=storage)
    f, g = _random_state(orc, 9)
    cav.set_populations(f, g, post_collision=False)
    orc.set_state(f, g)
    first = cav.steady_change()
    assert first[0] == np.inf and first[1] == np.inf and first[2] == 0
    before = orc.fields()
    cav.step(50)
    orc.run(50)
    du, dT, k = cav.steady_change()
    odu, odT = oracle.steady_change(before, orc.fields())
    print(f"{dim}d {storage}: du {du:.6e} ({odu:.6e}) dT {dT:.6e} ({odT:.6e})", flush=True)
    assert k == 50
    assert abs(du - odu) <= tol * odu and abs(dT - odT) <= tol * odT
    # a replaced state restarts the measure
    cav.set_populations(f, g, post_collision=False)
    assert cav.steady_change()[0] == np.inf
    cav.close()


@pytest.mark.parametrize("storage", ["fp32", "fp16", "bf16"])
def test_checkpoint_restore_is_bitwise(storage):
    """run(2n) equals run(n) -> save -> new context -> restore -> run(n)
    (for 2-byte storage the saved step counter keeps the rounding bits)."""
    meshes = [("tanh", 90, 1.5), ("tanh", 50, 1.5)]
    a, _ = make_pair(meshes, 1e6, 0.71, storage=storage)
    a.step(300)
    ref_f, ref_g = a.populations()
    b, _ = make_pair(meshes, 1e6, 0.71, storage=storage)
    b.step(150)
    blob = b.save_state()
    b.close()
    c, _ = make_pair(meshes, 1e6, 0.71, storage=storage)
    c.load_state(blob)
    c.step(150)
    cf, cg = c.populations()
    assert np.array_equal(cf, ref_f) and np.array_equal(cg, ref_g)
    a.close()
    c.close()


def test_mass_conserved_uniform_gpu():
    cav, orc = make_pair([("uniform", 80, 0), ("uniform", 48, 0)], 1e6, 0.71)
    f, g = _random_state(orc, 8)
    cav.set_populations(f, g, post_collision=False)
    m0 = cav.stats()["rho_sum"]
    cav.step(1000)
    m1 = cav.stats()["rho_sum"]
    assert abs(m1 / m0 - 1) < 1e-6


def test_fields_and_init_fields_match_oracle():
    """islbm_fields against the oracle's fields after a run; islbm_init_fields
    against the oracle collision of textbook equilibria."""
    cav, orc = make_pair([("erf", 45, 1.5), ("erf", 33, 1.5)], 1e6, 0.71)
    cav.step(80)
    orc.run(80)
    fl, ofl = cav.fields(), orc.fields()
    for k in ("rho", "ux", "uy", "T"):
        scale = np.abs(ofl[k]).max() if k != "rho" else 1.0
        assert np.abs(fl[k] - ofl[k]).max() <= 1e-5 * scale, k
    # equilibrium initialisation
    e, w, _ = oracle.lattice(2, 0)
    eg, _, _ = oracle.lattice(2, 1)
    rng = np.random.default_rng(9)
    ux = 0.02 * rng.normal(size=orc.shape)
    uy = 0.02 * rng.normal(size=orc.shape)
    T = 0.4 * rng.uniform(-1, 1, size=orc.shape)
    aT = orc.params["aT"]
    eu = e[:, 0, None, None] * ux + e[:, 1, None, None] * uy
    feq = w[:, None, None] * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * (ux ** 2 + uy ** 2))
    wm = (4 + aT) / 20
    geq = np.stack([T * (1 - 4 * wm)] + [T * (wm + 0.5 * (eg[p, 0] * ux + eg[p, 1] * uy))
                                         for p in range(1, 5)])
    cav.init_fields(ux, uy, None, T)
    orc.set_state(feq, geq)
    orc.collide()
    ofp, ogp = orc.post()
    fp, gp = cav.populations()
    assert rel_f(fp, ofp) < 1e-6 and rel_g(gp, ogp) < 1e-6
    cav.close()


def test_validation_errors_on_gpu():
    sp = lu_spacings("tanh", 40)
    # a_T > 1 refused unless allowed
    with pytest.raises(pkg.IslbmError) as ei:
        pkg.Cavity([sp, sp], 1e2, 0.71)
    assert ei.value.code == pkg.ISLBM_EPARAM
    cav = pkg.Cavity([sp, sp], 1e6, 0.71)
    with pytest.raises(pkg.IslbmError):
        pkg.islbm_step(cav.ctx, -1)
    cav.close()


def test_nonfinite_flag():
    cav, orc = make_pair([("tanh", 40, 1.5), ("tanh", 30, 1.5)], 1e6, 0.71)
    f, g = _random_state(orc, 10)
    f[3, 5, 7] = np.nan
    cav.set_populations(f, g, post_collision=True)
    st = cav.stats(allow_nonfinite=True)
    assert st["nonfinite"] >= 1
    with pytest.raises(pkg.IslbmError) as ei:
        cav.stats()
    assert ei.value.code == pkg.ISLBM_ENONFINITE
    cav.close()

"""Host logic of the studies in bench.py, run without a GPU: a stand-in
cavity whose integrals follow a known power law in the mesh spacing checks
that the 3-D convergence study interpolates each mesh's fields onto the next
one, stops on its integral criterion and returns the Richardson order of the
law."""
import numpy as np

import bench
import paper_2509_01099_amd as pkg


class _Cavity:
    P = 2.5

    def __init__(self, sp, Ra, Pr, storage):
        self.n = len(sp[0]) - 1
        self.steps = 0
        self.inits = None

    def init_fields(self, ux, uy, uz, T):
        self.inits = (ux, uy, uz, T)

    def step(self, k):
        self.steps += k

    def steady_change(self):
        return 1e-9, 1e-9, self.steps

    def stats(self):
        h = 1.0 / self.n
        decay = np.exp(-self.steps / 20000.0)          # reaches a steady value
        v = {"nu_vol": 4.3 + 2.0 * h ** self.P, "nu_hot": 4.3 + 3.0 * h ** self.P,
             "nu_cold": 4.3 + 3.0 * h ** self.P, "re_rms": 39.0 - 50.0 * h ** self.P}
        return {k: x * (1 + 1e-3 * decay) for k, x in v.items()}

    def fields(self):
        c = np.linspace(0.0, 1.0, self.n)
        T = np.broadcast_to(0.5 - c[None, None, :], (self.n,) * 3).copy()
        return {"ux": 0 * T, "uy": 0 * T, "uz": 0 * T, "T": T}

    def close(self):
        pass


def test_convergence_3d_host_logic(monkeypatch):
    made = []

    def factory(*a, **k):
        made.append(_Cavity(*a, **k))
        return made[-1]

    monkeypatch.setattr(pkg, "Cavity", factory)
    sizes = (9, 13, 19)
    out = bench.convergence_3d(1e5, sizes, max_steps=(10 ** 6,) * 3)
    assert made[0].inits is None
    for cav, n in zip(made[1:], sizes[1:]):
        assert all(a.shape == (n, n, n) for a in cav.inits)
        # T is linear in x: the interpolated field is the same linear profile
        assert abs(cav.inits[3][0, 0, 0] - cav.inits[3][0, 0, -1] - 1.0) < 0.2
    for run in out["runs"]:
        assert run["integral_change"] < 1e-8
    assert set(out["richardson"]) == {"nu_vol", "nu_hot", "nu_cold", "re_rms"}
    # a power law sampled at ratios 13/9 and 19/13 (not exactly 1.41) gives
    # an order near the law's when read with r = 1.41
    p = out["richardson"]["nu_vol"]["p"]
    assert abs(p - _Cavity.P) < 0.3, p


def test_convergence_3d_split_over_processes(monkeypatch, tmp_path):
    """The same study run as two parts (the coarse meshes saving their last
    steady fields, the finest mesh starting from them with the earlier runs
    as prior) gives the same runs and Richardson values as one run."""
    import json

    monkeypatch.setattr(pkg, "Cavity", lambda *a, **k: _Cavity(*a, **k))
    sizes = (9, 13, 19)
    whole = bench.convergence_3d(1e5, sizes, max_steps=(10 ** 6,) * 3)
    npz = str(tmp_path / "f.npz")
    first = bench.convergence_3d(1e5, sizes[:2], max_steps=(10 ** 6,) * 2, save_file=npz)
    assert "richardson" not in first
    prior = json.loads(json.dumps(first))
    made = []

    def factory(*a, **k):
        made.append(_Cavity(*a, **k))
        return made[-1]

    monkeypatch.setattr(pkg, "Cavity", factory)
    second = bench.convergence_3d(1e5, sizes[2:], max_steps=(10 ** 6,), init_file=npz, prior=prior)
    # the finest mesh starts from the saved (FP16) coarse fields
    assert made[0].inits is not None and made[0].inits[3].shape == (19, 19, 19)
    assert abs(made[0].inits[3][0, 0, 0] - made[0].inits[3][0, 0, -1] - 1.0) < 0.2
    assert [r["n"] for r in second["runs"]] == list(sizes)
    assert second["richardson_meshes"] == list(sizes)
    for k in ("nu_vol", "re_rms"):
        assert abs(second["richardson"][k]["p"] - whole["richardson"][k]["p"]) < 1e-12


def test_wctpdt_rows_scale_with_free_fall_time(monkeypatch):
    """WCTpDT = time per step x H_lu / u_f; the erf row carries the paper's
    figure and the ratios to the uniform mesh of the same node count."""

    class Cav:
        def __init__(self, sp, Ra, Pr, storage, u_f):
            self.H = float(np.sum(sp[0]) - 0.5 * sp[0][0] - 0.5 * sp[0][-1])
            self.uf = u_f

        @property
        def info(self):
            return {"H_lu": self.H}

        def stats(self, allow_nonfinite=False):
            return {"nonfinite": 0}

        def close(self):
            pass

    monkeypatch.setattr(pkg, "Cavity", Cav)
    monkeypatch.setattr(bench, "PAPER_WCTPDT", ((2, 65, 1e8, 100.0, 10),))
    monkeypatch.setattr(bench, "time_run", lambda cav, steps, warm: (0.0, steps * 1e-3))
    out = bench.wctpdt_study(storages=("fp64",))
    erf, uni = out["rows"]
    uf = 0.1 / 3 ** 0.5
    for r in (erf, uni):
        assert abs(r["wctpdt_s"] - 1e-3 * r["H_lu"] / uf) < 0.01
        assert abs(r["mlups"] - 65 * 65 / 1e-3 / 1e6) < 0.1
    assert abs(uni["H_lu"] - 65) < 1e-9 and erf["H_lu"] > 65
    assert abs(erf["paper_over_ours"] - 100.0 / erf["wctpdt_s"]) < 0.01
    assert abs(erf["wctpdt_over_uniform"] / (erf["H_lu"] / 65) - 1) < 1e-2   # rounded rows

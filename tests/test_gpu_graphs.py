"""Graph-replayed steps against directly launched ones.

islbm_step replays 64-step batches and the remaining plain launches from HIP
graphs (the latter once a count recurs or after islbm_plan_steps); a context
created with options.no_graph launches every step directly.  Both must give
bitwise the same populations and statistics after every call, for every
mix of batch, remainder and odd counts, with eager work (statistics, field
reads) and synchronisations between the replays, and with stochastic
rounding, whose random words depend on a device-side step counter."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _pair(dim, storage):
    import paper_2509_01099_amd as pkg

    n = (70, 36) if dim == 2 else (20, 18, 16)
    sp = [pkg.islbm_mesh_spacing("tanh", k, 1.5) for k in n]
    sp = [s / s[0] for s in sp]
    Ra = 1e5 if dim == 2 else 1e4
    g = pkg.Cavity(sp, Ra, 0.71, storage=storage)
    e = pkg.Cavity(sp, Ra, 0.71, storage=storage, no_graph=1)
    return g, e


# step counts per call: repeated small counts (the remainder graph is built on
# the second call), a planned count, batches with a remainder, odd counts that
# flip the buffer parity, and a fifth remainder count that evicts a graph
SCHEDULE = [20, 20, 20, ("plan", 7), 7, 300, 300, 1001, 1001, 9, 9, 12, 12, 33, 33, 20, 2, 1]


@pytest.mark.parametrize("dim,storage", [(2, "fp32"), (2, "fp16"), (2, "fp64"), (3, "fp32"),
                                         (3, "bf16"), (3, "fp32sr")])
def test_graph_replays_match_direct_launches(dim, storage):
    g, e = _pair(dim, storage)
    try:
        for k, item in enumerate(SCHEDULE):
            if isinstance(item, tuple):
                g.plan(item[1])
                continue
            g.step(item)
            e.step(item)
            sg, se = g.stats(allow_nonfinite=True), e.stats(allow_nonfinite=True)
            assert sg == se, (k, item, sg, se)
            fg, gg = g.populations()
            fe, ge = e.populations()
            assert np.array_equal(fg, fe) and np.array_equal(gg, ge), (k, item)
            if k % 3 == 0:
                torch.cuda.synchronize()
                _ = g.fields()
        assert sg["step"] == sum(i for i in SCHEDULE if not isinstance(i, tuple))
        assert sg["nonfinite"] == 0
    finally:
        g.close()
        e.close()


def test_plan_runs_no_step():
    g, e = _pair(2, "fp32")
    try:
        g.step(5)
        e.step(5)
        before = g.populations()
        g.plan(20)
        g.plan(300)
        g.plan(0)
        after = g.populations()
        assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
        assert g.stats()["step"] == 5
        g.step(300)
        e.step(300)
        assert np.array_equal(g.populations()[0], e.populations()[0])
    finally:
        g.close()
        e.close()

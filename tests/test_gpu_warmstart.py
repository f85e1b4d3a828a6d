"""The learned warm start, end to end at a small size: the solver produces
steady fields at a set of training Rayleigh numbers, the network (trained by
the BF16 matrix-core kernels) predicts the fields at unseen Ra, and the
solver started from that prediction reaches the steady Nusselt number
(within 1e-3) in fewer steps than the cold start from rest, at the same
steady value.

The solver runs with FP64 storage here: with FP32 storage the slowest
thermal modes stall once their per-step change falls below half a unit in
the last place, so the state it settles in depends on where it started (on
this mesh by up to ~2e-3 in Nu), and the two runs could not be compared."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _progress(tag):
    def log(done, hist):
        if done % 50_000 == 0:
            print(f"{tag}: {done} steps, Nu_hot {hist[-1][-1][1]:.5f}", flush=True)
    return log


def test_warm_start_saves_steps():
    """2-D, 129^2 erf mesh: ten training (stratified) and three held-out
    Rayleigh numbers drawn log-uniform in [1e6, 1e7]; the network's prediction must at least
    halve the total steps to a steady Nu_hot (within 1e-3) over the three
    held-out cases, and each warm run must end within 1e-3 of the cold one."""
    from paper_2509_01099_amd import warmstart as W

    res = W.quick_study(n=129, n_train=10, n_held=3, steps=600_000,
                        log=lambda m: print(m, flush=True))
    for r in res["held_out"]:
        print(f"Ra {r['Ra']:.3e}: cold {r['cold_steps']} warm {r['warm_steps']} steps, "
              f"Nu_hot {r['nu_hot_cold_end']:.5f} / {r['nu_hot_warm_end']:.5f}, "
              f"prediction error {r['prediction_rel_err']:.2e}", flush=True)
    print(f"loss {res['train']['loss_first']:.3e} -> {res['train']['loss_last']:.3e}; total cold "
          f"{res['cold_steps_total']} warm {res['warm_steps_total']}", flush=True)
    assert res["cold_steps_total"] is not None and res["warm_steps_total"] is not None
    assert res["warm_steps_total"] <= 0.5 * res["cold_steps_total"]
    assert res["max_rel_diff_end"] <= 1e-3


def test_warm_start_saves_steps_3d():
    """The same in 3-D: (x, y, z, log10 Ra) -> (u, v, w, T) on a 33^3 erf mesh,
    five training Rayleigh numbers in [1.2e5, 2e6], held-out Ra = 7e5; the
    training loss must fall at least 20-fold before the comparison."""
    import paper_2509_01099_amd as pkg
    from paper_2509_01099_amd import warmstart as W

    sp = W.mesh_spacing("erf", 33, 1.5)
    train_ra = [1.2e5, 2.5e5, 5e5, 1e6, 2e6]
    test_ra = 7e5
    steps, chunk = 300_000, 5_000
    uf = 0.1 / 3 ** 0.5
    cavs = [pkg.Cavity([sp, sp, sp], ra, 0.71, storage="fp64", use_torch_buffers=False,
                       own_stream=True) for ra in train_ra + [test_ra]]
    hist = W.run_concurrent(cavs, steps, chunk, log=_progress("cold 3d"))
    inputs = np.concatenate([W.node_inputs(sp, ra, dim=3) for ra in train_ra])
    targets = np.concatenate([W.fields_star(c, uf) for c in cavs[:-1]])
    assert inputs.shape[1] == 4 and targets.shape[1] == 4
    cold = [(h[0], h[1]) for h in hist[-1]]
    ref = cold[-1][1]
    for c in cavs:
        c.close()
    net = W.WarmStartMLP(W.MLPConfig(dim=3))
    losses = net.train(torch.tensor(inputs, device="cuda"), torch.tensor(targets, device="cuda"),
                       steps=8000, batch=4096, log_every=1000)
    # the network must have learned the fields before the comparison means anything
    assert losses[-1][1] <= losses[0][1] / 20.0, losses
    warm_cav = pkg.Cavity([sp, sp, sp], test_ra, 0.71, storage="fp64", use_torch_buffers=False,
                          own_stream=True)
    W.predict_init(net, warm_cav, sp, test_ra, uf)
    warm = [(h[0], h[1]) for h in W.run_concurrent([warm_cav], steps, chunk,
                                                   log=_progress("warm 3d"))[0]]
    warm_cav.close()
    cs, ws = W.steps_within(cold, ref), W.steps_within(warm, ref)
    print(f"3d: loss {losses[0][1]:.3e} -> {losses[-1][1]:.3e}; cold {cs} steps, warm {ws} steps, "
          f"Nu_hot steady {ref:.5f}, warm end {warm[-1][1]:.5f}", flush=True)
    assert cs is not None and ws is not None
    assert ws < cs
    assert abs(warm[-1][1] - ref) <= 1e-3 * ref

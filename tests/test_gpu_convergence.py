"""Grid convergence of the steady 2-D cavity (Sec. 3): three erf meshes
(a = 1.5) refined by 2, each started from the previous mesh's steady fields
and run in FP64 to the paper's steady criterion (relative change of u and T
below 1e-9 over 2000 steps).  The observed order of the domain-integrated
quantities must be near third order, as the paper reports (p = 2.5-3.1 for
<Nu> and <Re> in Table 2).  Ra = 1e5 on 65/129/257 keeps the run short; the
full Table 2 case (Ra = 1e6 on 257/513/1025) is `bench.py --convergence 1e6`."""
import math

import numpy as np
import pytest

import paper_2509_01099_amd as pkg

pytestmark = pytest.mark.gpu


def _coords(sp):
    X = np.concatenate([[0.0], np.cumsum(sp)])
    w0 = 0.5 * (X[0] + X[1])
    return (X[1:-1] - w0) / (0.5 * (X[-1] + X[-2]) - w0)


def _spacing(n):
    sp = pkg.islbm_mesh_spacing("erf", n, 1.5)
    return sp / sp[0]


def test_near_third_order_global_convergence():
    from scipy.interpolate import RegularGridInterpolator

    vals, prev = [], None
    for n in (65, 129, 257):
        sp = _spacing(n)
        c = _coords(sp)
        cav = pkg.Cavity([sp, sp], 1e5, 0.71, storage="fp64", use_torch_buffers=False)
        if prev is not None:
            pc, pf = prev
            yy, xx = np.meshgrid(c, c, indexing="ij")
            pts = np.column_stack([yy.ravel(), xx.ravel()])
            init = [RegularGridInterpolator((pc, pc), pf[k], bounds_error=False,
                                            fill_value=None)(pts).reshape(n, n)
                    for k in ("ux", "uy", "T")]
            cav.init_fields(init[0], init[1], None, init[2])
        steps, du, dT = 0, np.inf, np.inf
        while steps < 3_000_000 and not (du < 1e-9 and dT < 1e-9):
            cav.step(18000)
            cav.steady_change()
            cav.step(2000)
            du, dT, _ = cav.steady_change()
            steps += 20000
        st = cav.stats()
        f = cav.fields()
        prev = (c, f)
        cav.close()
        print(f"{n}^2: {steps} steps du {du:.1e} dT {dT:.1e} nu_vol {st['nu_vol']:.8f} "
              f"nu_mid {st['nu_mid']:.8f} re_rms {st['re_rms']:.6f}", flush=True)
        assert du < 1e-9 and dT < 1e-9
        vals.append(st)
    for k in ("nu_vol", "nu_mid", "re_rms"):
        fc, fm, ff = (v[k] for v in vals)
        p = math.log(abs((fc - fm) / (fm - ff))) / math.log(2.0)
        print(f"{k}: p = {p:.2f}", flush=True)
        assert 2.2 < p < 3.6, (k, p)

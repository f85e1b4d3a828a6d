"""Learned warm start for the cavity solver.

A coordinate network maps Fourier features of (x, y[, z], log10 Ra) to the
steady (u*, v*[, w*], T*) of the side-heated cavity (2-D or 3-D).  It is trained on steady fields that
the solver itself produced at a set of Rayleigh numbers; at an unseen Ra its
prediction sets equilibrium initial populations (islbm_init_fields_device) in
place of the cold start from rest, and the solver then runs unchanged.

Every arithmetic step of training and inference runs in the HIP kernels of
libislbm.so (include/islbm_mlp.h): Fourier features, BF16 matrix-core GEMMs
with FP32 accumulation and fused bias/SiLU epilogues, the loss gradient,
column sums and Adam.  PyTorch provides device memory and the stream only.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass

import numpy as np

from . import load

_VP = C.c_void_p


def _lib():
    lib = load()
    if not getattr(lib, "_mlp_ready", False):
        P, I, F, S = C.c_void_p, C.c_int, C.c_float, C.c_size_t
        lib.islbm_mlp_features.argtypes = [P, I, P, I, P, I, P]
        lib.islbm_mlp_features_d.argtypes = [P, I, I, P, I, P, I, P]
        lib.islbm_gemm_bf16.argtypes = [I, I, I, I, P, I, P, I, P, I, P, I, P, P, I, I, P, S, P]
        lib.islbm_mlp_mse_grad.argtypes = [P, I, P, I, P, I, I, P, P, I, P, P]
        lib.islbm_mlp_colsum.argtypes = [P, I, I, I, P, P]
        lib.islbm_mlp_gather.argtypes = [P, I, P, I, I, P, I, P]
        lib.islbm_f32_to_bf16.argtypes = [P, P, S, P]
        lib.islbm_mlp_adam.argtypes = [P, P, P, P, P, S, F, F, F, F, F, I, P]
        lib.islbm_gemm_bf16_tn_noalloc.argtypes = [I, I, I, P, I, P, I, P, I, P]
        for n in ("islbm_mlp_features", "islbm_mlp_features_d", "islbm_gemm_bf16", "islbm_mlp_mse_grad", "islbm_mlp_colsum",
                  "islbm_mlp_gather", "islbm_f32_to_bf16", "islbm_mlp_adam",
                  "islbm_gemm_bf16_tn_noalloc"):
            getattr(lib, n).restype = C.c_int
        lib._mlp_ready = True
    return lib


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _ok(rc: int, what: str) -> None:
    if rc != 0:
        raise RuntimeError(f"{what} failed with status {rc}")


# --------------------------------------------------------------- C-name wrappers

def islbm_mlp_features(p, B, out, stream=None):
    n, F = p.shape[0], B.shape[0]
    _ok(_lib().islbm_mlp_features(_p(p), n, _p(B), F, _p(out), out.shape[1], stream), "features")


def islbm_mlp_features_d(p, B, out, stream=None):
    n, d = p.shape
    _ok(_lib().islbm_mlp_features_d(_p(p), n, d, _p(B), B.shape[0], _p(out), out.shape[1], stream),
        "features_d")


def islbm_gemm_bf16(mode, M, N, K, A, lda, Bm, ldb, Cf=None, ldc=0, Cb=None, ldcb=0, bias=None,
                    aux=None, ldaux=0, epilogue=0, ws=None, stream=None):
    wsb = ws.numel() * ws.element_size() if ws is not None else 0
    _ok(_lib().islbm_gemm_bf16(mode, M, N, K, _p(A), lda, _p(Bm), ldb, _p(Cf), ldc, _p(Cb), ldcb,
                               _p(bias), _p(aux), ldaux, epilogue, _p(ws), wsb, stream), "gemm")


def islbm_gemm_bf16_tn_noalloc(M, N, K, A, lda, Bm, ldb, Cf, ldc, stream=None) -> int:
    """C = A^T B with split-K partials in the library's fixed device array;
    returns the status (0, -1 beyond the array or bad arguments, -5)."""
    return _lib().islbm_gemm_bf16_tn_noalloc(M, N, K, _p(A), lda, _p(Bm), ldb, _p(Cf), ldc, stream)


def islbm_mlp_mse_grad(y, t, w, gf=None, gb=None, loss=None, stream=None):
    n, m = y.shape
    ldg = (gf if gf is not None else gb).shape[1] if (gf is not None or gb is not None) else m
    _ok(_lib().islbm_mlp_mse_grad(_p(y), y.shape[1], _p(t), t.shape[1], _p(w), n, m, _p(gf),
                                  _p(gb), ldg, _p(loss), stream), "mse_grad")


def islbm_mlp_colsum(a, out, n=None, m=None, stream=None):
    n = a.shape[0] if n is None else n
    m = a.shape[1] if m is None else m
    _ok(_lib().islbm_mlp_colsum(_p(a), n, m, a.shape[1], _p(out), stream), "colsum")


def islbm_mlp_gather(src, idx, dst, stream=None):
    _ok(_lib().islbm_mlp_gather(_p(src), src.shape[1], _p(idx), idx.shape[0], dst.shape[1],
                                _p(dst), dst.shape[1], stream), "gather")


def islbm_f32_to_bf16(src, dst, stream=None):
    _ok(_lib().islbm_f32_to_bf16(_p(src), _p(dst), src.numel(), stream), "to_bf16")


def islbm_mlp_adam(w, g, m, v, wb, lr, t, b1=0.9, b2=0.999, eps=1e-8, wd=0.0, stream=None):
    _ok(_lib().islbm_mlp_adam(_p(w), _p(g), _p(m), _p(v), _p(wb), w.numel(), lr, b1, b2, eps, wd,
                              t, stream), "adam")


# ----------------------------------------------------------------------- model

# fixed output scales: u*, v* (, w*) are O(0.3) in the cavity, T* lies in [-1/2, 1/2]
def out_scale(dim: int) -> np.ndarray:
    return np.array([1.0 / 0.3] * dim + [2.0])


@dataclass
class MLPConfig:
    n_freq: int = 32              # 2 * n_freq Fourier features
    hidden: int = 256
    depth: int = 4                # hidden layers
    sigma: tuple = None           # frequency scale per input; None => 6 per axis, 1 for s
    seed: int = 0
    dim: int = 2                  # cavity dimension: inputs (x, y[, z], s), outputs (u, v[, w], T)


def ra_coord(Ra: float) -> float:
    """Third network input: s = log10(Ra) - 7 (s in [-1, 1] over 1e6..1e8)."""
    return math.log10(Ra) - 7.0


class WarmStartMLP:
    """Parameters live in FP32 (master) with BF16 copies for the GEMMs."""

    def __init__(self, cfg: MLPConfig = MLPConfig(), device="cuda:0"):
        import torch

        self.torch = torch
        self.cfg = cfg
        self.device = torch.device(device)
        rng = np.random.default_rng(cfg.seed)
        self.n_in = self.n_out = cfg.dim + 1
        sigma = cfg.sigma if cfg.sigma is not None else (6.0,) * cfg.dim + (1.0,)
        B = rng.normal(size=(cfg.n_freq, self.n_in)) * np.asarray(sigma)[None, :]
        self.B = torch.tensor(B, dtype=torch.float32, device=self.device)
        dims = [2 * cfg.n_freq] + [cfg.hidden] * cfg.depth + [self.n_out]
        self.dims = dims
        self.W, self.b = [], []
        for i in range(len(dims) - 1):
            fan_in, fan_out = dims[i], dims[i + 1]
            lim = math.sqrt(6.0 / fan_in) if i < len(dims) - 2 else math.sqrt(1.0 / fan_in)
            W = rng.uniform(-lim, lim, size=(fan_out, fan_in))
            self.W.append(torch.tensor(W, dtype=torch.float32, device=self.device))
            self.b.append(torch.zeros(fan_out, dtype=torch.float32, device=self.device))
        self.Wb = [torch.empty(w.shape, dtype=torch.bfloat16, device=self.device) for w in self.W]
        self.sync_bf16()
        self.adam_state = None
        self.t = 0
        self.scale = out_scale(cfg.dim)

    # -- parameters
    def sync_bf16(self):
        for w, wb in zip(self.W, self.Wb):
            islbm_f32_to_bf16(w, wb)

    def state_dict(self) -> dict:
        return {"B": self.B.cpu().numpy(), "W": [w.cpu().numpy() for w in self.W],
                "b": [b.cpu().numpy() for b in self.b]}

    def load_state(self, sd: dict) -> None:
        torch = self.torch
        self.B = torch.tensor(sd["B"], dtype=torch.float32, device=self.device)
        self.W = [torch.tensor(w, dtype=torch.float32, device=self.device) for w in sd["W"]]
        self.b = [torch.tensor(b, dtype=torch.float32, device=self.device) for b in sd["b"]]
        self.Wb = [torch.empty(w.shape, dtype=torch.bfloat16, device=self.device) for w in self.W]
        self.sync_bf16()

    # -- passes
    def _buffers(self, n: int):
        torch = self.torch
        key = n
        if getattr(self, "_buf_n", None) != key:
            d = self.dims
            self._x0 = torch.empty((n, d[0]), dtype=torch.bfloat16, device=self.device)
            self._Z = [torch.empty((n, d[i + 1]), dtype=torch.float32, device=self.device)
                       for i in range(len(d) - 1)]
            self._H = [torch.empty((n, d[i + 1]), dtype=torch.bfloat16, device=self.device)
                       for i in range(len(d) - 2)]
            self._dZf = [torch.empty((n, d[i + 1]), dtype=torch.float32, device=self.device)
                         for i in range(len(d) - 1)]
            self._dZb = [torch.empty((n, d[i + 1]), dtype=torch.bfloat16, device=self.device)
                         for i in range(len(d) - 1)]
            self._buf_n = key
        return self

    def forward(self, p):
        """p: (n, dim + 1) float32 device tensor of (x, y[, z], s); returns
        (n, dim + 1) float32 outputs (u*, v*[, w*], T*)."""
        n = p.shape[0]
        self._buffers(n)
        islbm_mlp_features_d(p, self.B, self._x0)
        h, k = self._x0, self.dims[0]
        L = len(self.W)
        for i in range(L):
            m = self.dims[i + 1]
            if i < L - 1:
                islbm_gemm_bf16(0, n, m, k, h, k, self.Wb[i], k, Cf=self._Z[i], ldc=m, Cb=self._H[i],
                                ldcb=m, bias=self.b[i], epilogue=1)
                h, k = self._H[i], m
            else:
                islbm_gemm_bf16(0, n, m, k, h, k, self.Wb[i], k, Cf=self._Z[i], ldc=m,
                                bias=self.b[i], epilogue=2)
        return self._Z[L - 1]

    def backward(self, dout_b, dout_f, gW, gb, ws):
        """Backpropagates dL/d(out) (bf16 and f32 copies, n x outputs) into gW / gb."""
        n = dout_b.shape[0]
        L = len(self.W)
        dzb, dzf = dout_b, dout_f
        for i in range(L - 1, -1, -1):
            m, k = self.dims[i + 1], self.dims[i]
            x = self._x0 if i == 0 else self._H[i - 1]
            islbm_gemm_bf16(2, m, k, n, dzb, m, x, k, Cf=gW[i], ldc=k, epilogue=0, ws=ws)
            islbm_mlp_colsum(dzf, gb[i])
            if i > 0:
                # dZ_{i-1} = (dZ_i W_i) * silu'(Z_{i-1})
                islbm_gemm_bf16(1, n, k, m, dzb, m, self.Wb[i], k, Cf=self._dZf[i - 1], ldc=k,
                                Cb=self._dZb[i - 1], ldcb=k, aux=self._Z[i - 1], ldaux=k, epilogue=3)
                dzb, dzf = self._dZb[i - 1], self._dZf[i - 1]

    # -- training
    def train(self, inputs, targets, steps: int = 3000, batch: int = 8192, lr: float = 2e-3,
              seed: int = 1, weights=None, log_every: int = 0):
        """inputs (N, dim + 1) float32, targets (N, dim + 1) float32
        (u*, v*[, w*], T*), on the device.  Returns the loss history (every
        log_every steps)."""
        torch = self.torch
        N = inputs.shape[0]
        ni, no = self.n_in, self.n_out
        weights = np.ones(no) if weights is None else np.asarray(weights)
        # the network outputs (u*, v*[, w*], T*) directly; the loss weights
        # w_j = weights_j * scale_j^2 make it the MSE of O(1)-scaled outputs
        w = torch.tensor(weights * self.scale ** 2, dtype=torch.float32, device=self.device)
        if self.adam_state is None:
            self.adam_state = [(torch.zeros_like(W), torch.zeros_like(W), torch.zeros_like(b),
                                torch.zeros_like(b)) for W, b in zip(self.W, self.b)]
        gW = [torch.empty_like(W) for W in self.W]
        gb = [torch.empty_like(b) for b in self.b]
        ws = torch.empty(4 * 256 * 256 * ((batch + 1023) // 1024) + 1024, dtype=torch.float32,
                         device=self.device)
        pb = torch.empty((batch, ni), dtype=torch.float32, device=self.device)
        tb = torch.empty((batch, no), dtype=torch.float32, device=self.device)
        dof = torch.empty((batch, no), dtype=torch.float32, device=self.device)
        dob = torch.empty((batch, no), dtype=torch.bfloat16, device=self.device)
        loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        rng = np.random.default_rng(seed)
        hist = []
        for s in range(steps):
            idx = torch.from_numpy(rng.integers(0, N, size=batch, dtype=np.int32)).to(self.device)
            islbm_mlp_gather(inputs, idx, pb)
            islbm_mlp_gather(targets, idx, tb)
            out = self.forward(pb)
            islbm_mlp_mse_grad(out, tb, w, gf=dof, gb=dob, loss=loss)
            self.backward(dob, dof, gW, gb, ws)
            self.t += 1
            lr_t = lr * 0.5 * (1.0 + math.cos(math.pi * s / steps))
            for i in range(len(self.W)):
                mW, vW, mb, vb = self.adam_state[i]
                islbm_mlp_adam(self.W[i], gW[i], mW, vW, self.Wb[i], lr_t, self.t)
                islbm_mlp_adam(self.b[i], gb[i], mb, vb, None, lr_t, self.t)
            if log_every and (s % log_every == 0 or s == steps - 1):
                hist.append((s, float(loss.item())))
        return hist

    def predict(self, p):
        """(n, dim + 1) inputs -> (n, dim + 1) float32 (u*, v*[, w*], T*) on the device."""
        return self.forward(p)


# ------------------------------------------------------------- study driver

def draw_ra(count: int = 40, seed: int = 2025, lo: float = 6.0, hi: float = 8.0,
            stratified: bool = False) -> np.ndarray:
    """Rayleigh numbers log-uniform in [10^lo, 10^hi] from a seed.  With
    stratified=True the k-th draw is uniform in the k-th of `count` equal
    sub-intervals of [lo, hi] (each draw is still log-uniform over the whole
    range when k is picked at random; the set covers the range evenly)."""
    u = np.random.default_rng(seed).uniform(0.0, 1.0, count)
    if stratified:
        u = (np.arange(count) + u) / count
    return 10.0 ** (lo + (hi - lo) * u)


def mesh_spacing(kind: str = "erf", n: int = 513, a: float = 1.5) -> np.ndarray:
    from . import islbm_mesh_spacing

    sp = islbm_mesh_spacing(kind, n, a)
    return sp / sp[0]


def node_inputs(sp: np.ndarray, Ra: float, sub: int = 1, dim: int = 2) -> np.ndarray:
    """Network inputs (x*, y*[, z*], s) of the mesh nodes (square / cubic
    mesh with spacings sp on every axis), coordinates measured from the walls
    in units of the wall-to-wall extent; every sub-th node per axis; rows in
    x-fastest order."""
    X = np.concatenate([[0.0], np.cumsum(sp)])
    wall0 = 0.5 * (X[0] + X[1])
    H = 0.5 * (X[-1] + X[-2]) - wall0
    c = (X[1:-1] - wall0) / H
    c = c[::sub]
    grids = np.meshgrid(*([c] * dim), indexing="ij")      # slowest axis first
    cols = [g.ravel() for g in reversed(grids)]           # x, y[, z]
    s = np.full(cols[0].size, ra_coord(Ra))
    return np.column_stack(cols + [s]).astype(np.float32)


def steps_within(history, ref: float, tol: float = 1e-3) -> int | None:
    """First recorded step from which every later record stays within tol
    (relative) of ref; None if the last record is outside."""
    ok_from = None
    for step, val in history:
        if abs(val - ref) <= tol * abs(ref):
            if ok_from is None:
                ok_from = step
        else:
            ok_from = None
    return ok_from


def run_concurrent(cavs, steps: int, chunk: int, keys=("nu_hot", "nu_vol", "re_rms"), log=None,
                   steady_interval: int = 0):
    """Advances every cavity by `steps` in chunks (each cavity on its own
    stream, so the launches overlap); records statistics after each chunk.
    With steady_interval > 0 each record also carries the Sec. 3 steady-state
    measure (du, dT) over the last steady_interval steps of the chunk."""
    hist = [[] for _ in cavs]
    done = 0
    while done < steps:
        n = min(chunk, steps - done)
        lead = n - steady_interval if 0 < steady_interval < n else n
        for c in cavs:
            c.step(lead)
        if lead < n:
            for c in cavs:
                c.steady_change()
            for c in cavs:
                c.step(n - lead)
        done += n
        for h, c in zip(hist, cavs):
            st = c.stats(allow_nonfinite=True)
            rec = (done, *[st[k] for k in keys])
            if lead < n:
                rec = rec + c.steady_change()[:2]
            h.append(rec)
        if log:
            log(done, hist)
    return hist


def steps_to_steady(history, tol: float = 1e-9):
    """First recorded step at which both steady-state measures (the last two
    entries of a record) are below tol (Sec. 3 uses 1e-9); None if never."""
    for rec in history:
        if rec[-2] < tol and rec[-1] < tol:
            return rec[0]
    return None


def fields_star(cav, uf: float) -> np.ndarray:
    """(n, dim + 1) float32 (u*, v*[, w*], T*) of a cavity (x-fastest node order)."""
    f = cav.fields()
    vel = [f[k].ravel() / uf for k in ("ux", "uy", "uz")[:cav.dim]]
    return np.column_stack(vel + [f["T"].ravel()]).astype(np.float32)


def predict_init(net: "WarmStartMLP", cav, sp: np.ndarray, Ra: float, uf: float) -> None:
    """Sets the cavity's state to equilibrium populations of the predicted
    steady fields at Ra (rho = 1; u = u* u_f; T = T*)."""
    import torch

    from . import islbm_init_fields_device

    p = torch.tensor(node_inputs(sp, Ra, dim=cav.dim), device=net.device)
    out = net.predict(p)
    u = (out[:, 0] * uf).double().contiguous()
    v = (out[:, 1] * uf).double().contiguous()
    w = (out[:, 2] * uf).double().contiguous() if cav.dim == 3 else None
    T = out[:, cav.dim].double().contiguous()
    torch.cuda.synchronize()
    islbm_init_fields_device(cav.ctx, u, v, w, T)
    cav.sync()  # u, v, w, T are released when this returns


def quick_study(n: int = 129, n_train: int = 10, n_held: int = 3, steps: int = 600_000,
                chunk: int = 10_000, train_steps: int = 8000, lo: float = 6.0, hi: float = 7.0,
                seed: int = 11, storage: str = "fp64", log=None) -> dict:
    """Learned warm start end to end on a small 2-D cavity (n^2 erf mesh,
    a = 1.5, Pr 0.71, Ma 0.1): cold solves from rest at n_train training and
    n_held held-out Rayleigh numbers (log-uniform in [10^lo, 10^hi], drawn
    from two seeds), all run concurrently; the network is trained on the
    training fields; the held-out cavities are then run again from the
    network's prediction.  The training Ra are stratified draws (one per
    equal sub-interval of log10 Ra), the held-out Ra plain draws from the
    next seed.  For each held-out Ra: steps until Nu_hot stays
    within 1e-3 of the cold run's final value (recorded every `chunk` steps),
    cold and warm, and the relative Nu_hot difference of the two final states."""
    import time

    import torch

    from . import Cavity

    t0 = time.perf_counter()
    sp = mesh_spacing("erf", n, 1.5)
    train_ra = [float(r) for r in draw_ra(n_train, seed=seed, lo=lo, hi=hi, stratified=True)]
    held_ra = [float(r) for r in draw_ra(n_held, seed=seed + 1, lo=lo, hi=hi)]
    uf = 0.1 / 3 ** 0.5

    def cavity(ra):
        return Cavity([sp, sp], ra, 0.71, storage=storage, use_torch_buffers=False, own_stream=True)

    cavs = [cavity(ra) for ra in train_ra + held_ra]
    hist = run_concurrent(cavs, steps, chunk)
    inputs = np.concatenate([node_inputs(sp, ra) for ra in train_ra])
    targets = np.concatenate([fields_star(c, uf) for c in cavs[:n_train]])
    cold = [[(h[0], h[1]) for h in hh] for hh in hist[n_train:]]
    for c in cavs:
        c.close()
    t_cold = time.perf_counter() - t0
    if log:
        log(f"warm-start study: cold solves done in {t_cold:.1f} s")
    net = WarmStartMLP(MLPConfig(seed=seed))
    losses = net.train(torch.tensor(inputs, device=net.device), torch.tensor(targets, device=net.device),
                       steps=train_steps, batch=4096, log_every=max(1, train_steps // 4))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0 - t_cold
    wcavs = [cavity(ra) for ra in held_ra]
    for c, ra in zip(wcavs, held_ra):
        predict_init(net, c, sp, ra, uf)
    warm_hist = run_concurrent(wcavs, steps, chunk)
    for c in wcavs:
        c.close()
    rows = []
    for ra, ch, wh in zip(held_ra, cold, warm_hist):
        wl = [(h[0], h[1]) for h in wh]
        ref = ch[-1][1]
        rows.append({"Ra": ra, "nu_hot_cold_end": ref, "nu_hot_warm_end": wl[-1][1],
                     "rel_diff_end": abs(wl[-1][1] - ref) / abs(ref),
                     "prediction_rel_err": abs(wl[0][1] - ref) / abs(ref),
                     "cold_steps": steps_within(ch, ref), "warm_steps": steps_within(wl, ref)})
    cs = [r["cold_steps"] for r in rows]
    ws = [r["warm_steps"] for r in rows]
    total_c = sum(cs) if None not in cs else None
    total_w = sum(ws) if None not in ws else None
    return {"workload": f"2-D cavity {n}^2 erf mesh (a=1.5), Pr 0.71, Ma 0.1, {storage} storage; "
                        f"{n_train} training / {n_held} held-out Ra log-uniform in "
                        f"[1e{lo:g}, 1e{hi:g}]",
            "criterion": "steps until Nu_hot stays within 1e-3 of the cold run's final value "
                         f"(records every {chunk} steps; {steps} steps per run)",
            "train": {"samples": int(inputs.shape[0]), "steps": train_steps, "batch": 4096,
                      "loss_first": losses[0][1], "loss_last": losses[-1][1]},
            "held_out": rows, "cold_steps_total": total_c, "warm_steps_total": total_w,
            "steps_ratio_warm_over_cold": (total_w / total_c) if total_c and total_w is not None
            else None,
            "max_rel_diff_end": max(r["rel_diff_end"] for r in rows),
            "seconds": {"cold": round(t_cold, 1), "train": round(t_train, 1),
                        "total": round(time.perf_counter() - t0, 1)}}

"""Warm-start network kernels (BF16 matrix cores, FP32 accumulation) against the
FP64 reference in oracle/mlp.py.  Operands are rounded to bfloat16 on both
sides at the points where the kernels hold them in bfloat16, so the remaining
differences are FP32 accumulation order and the FP32 exponential of SiLU."""
import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a, dtype):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


@pytest.mark.parametrize("M,N,K", [(200, 70, 50), (64, 64, 32), (1000, 256, 256), (33, 3, 256)])
@pytest.mark.parametrize("epi", [0, 1, 2])
def test_gemm_nt_forward(M, N, K, epi):
    from paper_2509_01099_amd import warmstart as ws

    rng = np.random.default_rng(M + N + K + epi)
    A = mlp.bf16(rng.normal(size=(M, K)))
    B = mlp.bf16(rng.normal(size=(N, K)) / np.sqrt(K))
    bias = rng.normal(size=N).astype(np.float32).astype(np.float64)
    ref = A @ B.T
    C = torch.zeros((M, N), dtype=torch.float32, device="cuda")
    Cb = torch.zeros((M, N), dtype=torch.bfloat16, device="cuda")
    ws.islbm_gemm_bf16(0, M, N, K, _dev(A, torch.bfloat16), K, _dev(B, torch.bfloat16), K, Cf=C,
                       ldc=N, Cb=Cb if epi == 1 else None, ldcb=N,
                       bias=_dev(bias, torch.float32) if epi else None, epilogue=epi)
    got = C.cpu().double().numpy()
    if epi:
        ref = ref + bias
    assert np.abs(got - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max())
    if epi == 1:
        act = Cb.float().cpu().double().numpy()
        assert np.abs(act - mlp.bf16(mlp.silu(ref))).max() <= 2 ** -7 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("M,N,K", [(300, 64, 256), (77, 256, 3), (128, 256, 256)])
def test_gemm_nn_backward_through_silu(M, N, K):
    from paper_2509_01099_amd import warmstart as ws

    rng = np.random.default_rng(M * 3 + N + K)
    A = mlp.bf16(rng.normal(size=(M, K)))
    B = mlp.bf16(rng.normal(size=(K, N)))
    aux = rng.normal(size=(M, N)).astype(np.float32).astype(np.float64)
    ref0 = A @ B
    C = torch.zeros((M, N), dtype=torch.float32, device="cuda")
    ws.islbm_gemm_bf16(1, M, N, K, _dev(A, torch.bfloat16), K, _dev(B, torch.bfloat16), N, Cf=C,
                       ldc=N, epilogue=0)
    assert np.abs(C.cpu().double().numpy() - ref0).max() <= 1e-5 * max(1.0, np.abs(ref0).max())
    Cb = torch.zeros((M, N), dtype=torch.bfloat16, device="cuda")
    ws.islbm_gemm_bf16(1, M, N, K, _dev(A, torch.bfloat16), K, _dev(B, torch.bfloat16), N, Cf=C,
                       ldc=N, Cb=Cb, ldcb=N, aux=_dev(aux, torch.float32), ldaux=N, epilogue=3)
    ref3 = ref0 * mlp.dsilu(aux)
    assert np.abs(C.cpu().double().numpy() - ref3).max() <= 1e-5 * max(1.0, np.abs(ref3).max())


@pytest.mark.parametrize("M,N,K,use_ws", [(256, 64, 3000, True), (3, 256, 2500, True),
                                          (70, 50, 200, False)])
def test_gemm_tn_weight_gradient(M, N, K, use_ws):
    from paper_2509_01099_amd import warmstart as ws

    rng = np.random.default_rng(M + 7 * N + K)
    A = mlp.bf16(rng.normal(size=(K, M)))
    B = mlp.bf16(rng.normal(size=(K, N)))
    ref = A.T @ B
    C = torch.zeros((M, N), dtype=torch.float32, device="cuda")
    wsb = torch.empty(4 * M * N * ((K + 1023) // 1024), dtype=torch.float32, device="cuda") \
        if use_ws else None
    ws.islbm_gemm_bf16(2, M, N, K, _dev(A, torch.bfloat16), M, _dev(B, torch.bfloat16), N, Cf=C,
                       ldc=N, epilogue=0, ws=wsb)
    assert np.abs(C.cpu().double().numpy() - ref).max() <= 2e-5 * max(1.0, np.abs(ref).max())


def test_network_gradients_match_reference():
    """Forward and backward of the full network (64 -> 4 x 256 -> 3) against
    the FP64 reference with the same bfloat16 rounding points."""
    from paper_2509_01099_amd.warmstart import MLPConfig, WarmStartMLP, islbm_mlp_mse_grad

    net = WarmStartMLP(MLPConfig(seed=3))
    rng = np.random.default_rng(4)
    n = 300
    p = np.column_stack([rng.random(n), rng.random(n), rng.uniform(-1, 1, n)])
    t = rng.normal(size=(n, 3)) * 0.1
    w = np.array([2.0, 3.0, 1.0])
    pd = _dev(p, torch.float32)
    out = net.forward(pd).clone()
    dof = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    dob = torch.empty((n, 3), dtype=torch.bfloat16, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    islbm_mlp_mse_grad(out, _dev(t, torch.float32), _dev(w, torch.float32), gf=dof, gb=dob, loss=loss)
    gW = [torch.empty_like(W) for W in net.W]
    gb = [torch.empty_like(b) for b in net.b]
    wsb = torch.empty(4 * 256 * 256 + 16, dtype=torch.float32, device="cuda")
    net.backward(dob, dof, gW, gb, wsb)
    torch.cuda.synchronize()
    # reference: same parameters, features from float32 inputs
    W = [x.cpu().double().numpy() for x in net.W]
    b = [x.cpu().double().numpy() for x in net.b]
    Bf = net.B.cpu().double().numpy()
    x0 = mlp.features(p.astype(np.float32).astype(np.float64), Bf)
    y, cache = mlp.forward(W, b, x0, quant=True)
    L, dout = mlp.mse(y, t, w)
    gW_ref, gb_ref = mlp.backward(W, cache, dout, quant=True)
    got = out.cpu().double().numpy()
    assert np.abs(got - y).max() <= 2e-2 * np.abs(y).max()
    assert abs(loss.item() - L) <= 2e-2 * L
    for i in range(len(W)):
        g, r = gW[i].cpu().double().numpy(), gW_ref[i]
        cos = float(np.sum(g * r) / np.sqrt(np.sum(g * g) * np.sum(r * r)))
        rel = float(np.linalg.norm(g - r) / np.linalg.norm(r))
        print(f"layer {i}: dW rel {rel:.2e} cos {cos:.6f}", flush=True)
        assert rel < 3e-2 and cos > 0.999
        gbr = gb[i].cpu().double().numpy()
        assert np.linalg.norm(gbr - gb_ref[i]) <= 3e-2 * np.linalg.norm(gb_ref[i])


def test_training_fits_a_smooth_field():
    """A few hundred Adam steps fit a smooth synthetic (u, v, T) field."""
    from paper_2509_01099_amd.warmstart import MLPConfig, WarmStartMLP

    net = WarmStartMLP(MLPConfig(seed=5))
    rng = np.random.default_rng(6)
    n = 20000
    p = np.column_stack([rng.random(n), rng.random(n), rng.uniform(-1, 1, n)])
    t = np.column_stack([0.1 * np.sin(np.pi * p[:, 0]) * np.cos(np.pi * p[:, 1]) * (1 + 0.2 * p[:, 2]),
                         -0.1 * np.cos(np.pi * p[:, 0]) * np.sin(np.pi * p[:, 1]),
                         0.5 - p[:, 0] + 0.1 * p[:, 2] * np.sin(2 * np.pi * p[:, 1])])
    hist = net.train(_dev(p, torch.float32), _dev(t, torch.float32), steps=400, batch=4096,
                     log_every=50)
    print(hist, flush=True)
    assert hist[-1][1] < 0.05 * hist[0][1]


@pytest.mark.parametrize("d", [3, 4])
def test_features_any_input_dimension(d):
    """Fourier features of d inputs (the 3-D warm start uses d = 4) against
    the FP64 reference, to bfloat16 resolution."""
    from paper_2509_01099_amd.warmstart import islbm_mlp_features_d

    rng = np.random.default_rng(d)
    n, F = 777, 32
    p = rng.random((n, d)).astype(np.float32)
    B = (rng.normal(size=(F, d)) * 3).astype(np.float32)
    out = torch.empty((n, 2 * F), dtype=torch.bfloat16, device="cuda")
    islbm_mlp_features_d(_dev(p, torch.float32), _dev(B, torch.float32), out)
    ref = mlp.features(p.astype(np.float64), B.astype(np.float64))
    assert np.abs(out.float().cpu().double().numpy() - ref).max() <= 2 ** -8 + 1e-5

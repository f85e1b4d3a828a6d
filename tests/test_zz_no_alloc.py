"""The allocation-free TN product (islbm_gemm_bf16_tn_noalloc, split-K
partials in the library's fixed device array) against islbm_gemm_bf16 in
mode 2 with a workspace: bitwise equal results on two calls in a row, the
second with a smaller input (the array keeps the first call's contents),
and sizes beyond the array rejected with nothing launched."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _pair(M, N, K, seed):
    from paper_2509_01099_amd import warmstart as ws

    g = torch.Generator(device="cpu").manual_seed(seed)
    A = torch.randn(K, M, generator=g).to(torch.bfloat16).cuda()
    B = torch.randn(K, N, generator=g).to(torch.bfloat16).cuda()
    ref = torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda")
    wsb = torch.empty(M * N * ((K + 1023) // 1024), dtype=torch.float32, device="cuda")
    ws.islbm_gemm_bf16(2, M, N, K, A, M, B, N, Cf=ref, ldc=N, epilogue=0, ws=wsb)
    out = torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda")
    rc = ws.islbm_gemm_bf16_tn_noalloc(M, N, K, A, M, B, N, out, N)
    torch.cuda.synchronize()
    return rc, ref.cpu().numpy(), out.cpu().numpy(), A, B


def test_noalloc_tn_matches_workspace_version_twice():
    rc1, ref1, out1, _, _ = _pair(256, 192, 5000, 1)
    assert rc1 == 0
    assert np.array_equal(ref1.view(np.uint32), out1.view(np.uint32))
    # second, smaller call: the array still holds the first call's partials
    rc2, ref2, out2, _, _ = _pair(64, 40, 1500, 2)
    assert rc2 == 0
    assert np.array_equal(ref2.view(np.uint32), out2.view(np.uint32))
    # and the exact product of the bfloat16 operands, to FP32 accumulation
    _, _, _, A, B = _pair(64, 40, 1500, 2)
    exact = A.double().cpu().numpy().T @ B.double().cpu().numpy()
    assert np.abs(out2 - exact).max() <= 2e-5 * max(1.0, np.abs(exact).max())


def test_noalloc_tn_rejects_beyond_scratch():
    from paper_2509_01099_amd import warmstart as ws

    M, N, K = 512, 512, 9 * 1024   # 4 * M * N * 9 bytes > 8 MiB
    A = torch.zeros(K, M, dtype=torch.bfloat16, device="cuda")
    B = torch.zeros(K, N, dtype=torch.bfloat16, device="cuda")
    C = torch.full((M, N), 7.0, dtype=torch.float32, device="cuda")
    assert ws.islbm_gemm_bf16_tn_noalloc(M, N, K, A, M, B, N, C, N) == -1
    torch.cuda.synchronize()
    assert bool(torch.all(C == 7.0))   # nothing launched

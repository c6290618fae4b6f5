"""The build's batched FP64 matrix-core product (sfm_dgemm_batched) against numpy in FP64.

Shapes are those of the Stage 1 build (M = 6m rows of a Lanczos block; K the nodes of a
subdomain for the projections and Gram matrices, split over work-groups; K = 6m or a multiple
for the updates; square p x p for the S-fraction), plus ragged sizes that cut every tile.  Bar:
|C - C_ref| <= 4 K u (|op(A)| |op(B)| + |beta C0|) elementwise, u = 2^-53 (the FP64 dot-product
error bound with margin)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

U64 = 2.0 ** -53


def _colmajor(rng, rows, cols, ld, batch):
    """Random column-major batch: array [batch][cols][ld] whose [:, :, :rows] is the matrix^T."""
    return rng.standard_normal((batch, cols, ld))


@pytest.mark.parametrize("ta, tb, M, N, K, batch", [
    (False, True, 96, 96, 35937, 3),      # C2_j / Gram: reduction over the nodes (split)
    (False, True, 96, 480, 4913, 2),      # full re-orthogonalisation projections
    (False, False, 96, 1000, 96, 2),      # block updates W -= C Z
    (False, False, 96, 777, 480, 2),      # long updates
    (True, False, 96, 500, 96, 2),        # W -= B^T Z
    (True, False, 72, 72, 72, 5),         # S-fraction products
    (False, True, 24, 24, 24, 4),
    (True, True, 18, 37, 45, 3),          # ragged everything
    (False, False, 100, 33, 17, 2),
])
def test_dgemm_matches_numpy(ta, tb, M, N, K, batch):
    from paper_1406_6923_amd import sfm
    rng = np.random.default_rng(M * 7 + N + K)
    ar, ac = (K, M) if ta else (M, K)          # stored A is ar x ac (column-major)
    br, bc = (N, K) if tb else (K, N)
    lda, ldb, ldc = ar + 3, br + 1, M + 5
    A = rng.standard_normal((batch, ac, lda))
    B = rng.standard_normal((batch, bc, ldb))
    C0 = rng.standard_normal((batch, N, ldc))
    alpha, beta = -0.75, 0.5
    opA = [(A[b, :, :ar].T).T if ta else A[b, :, :ar].T for b in range(batch)]
    opB = [(B[b, :, :br].T).T if tb else B[b, :, :br].T for b in range(batch)]
    ref = np.stack([alpha * opA[b] @ opB[b] + beta * C0[b, :, :M].T for b in range(batch)])
    bound = np.stack([4 * K * U64 * (np.abs(opA[b]) @ np.abs(opB[b]) + np.abs(beta * C0[b, :, :M].T)) + 1e-300
                      for b in range(batch)])
    dA = torch.tensor(A, device="cuda")
    dB = torch.tensor(B, device="cuda")
    dC = torch.tensor(C0, device="cuda")
    work = torch.empty(64 << 20, dtype=torch.float64, device="cuda")
    print(f"[case] dgemm ta={ta} tb={tb} M={M} N={N} K={K} batch={batch}", flush=True)
    sfm.sfm_dgemm_batched(ta, tb, M, N, K, alpha, dA, lda, ac * lda, dB, ldb, bc * ldb, beta, dC, ldc, N * ldc, batch,
                          work)
    torch.cuda.synchronize()
    got = dC.cpu().numpy()
    gotC = np.stack([got[b, :, :M].T for b in range(batch)])
    ratio = np.max(np.abs(gotC - ref) / bound)
    print(f"dgemm ta={ta} tb={tb} {M}x{N}x{K} x{batch}: max error / bound {ratio:.3f}")
    assert ratio < 1.0
    assert np.array_equal(got[:, :, M:], C0[:, :, M:])       # padding rows untouched


def test_fp64_matrix_rate_probe():
    """The sustained-rate probe returns a rate between 1 TFLOP/s and the published 78.6 TFLOP/s."""
    from paper_1406_6923_amd import sfm
    out = torch.empty(1024 * 256, dtype=torch.float64, device="cuda")
    print("[case] FP64 matrix-rate probe, 1024 work-groups", flush=True)
    rate = sfm.sfm_probe_fp64_matrix_rate(out, 1024, 500)
    print(f"FP64 matrix cores: {rate:.1f} TFLOP/s")
    assert 1.0 < rate < 78.6 * 1.05
    assert torch.isfinite(out).all()
    with pytest.raises(ValueError):
        sfm.sfm_probe_fp64_matrix_rate(out, 2048, 10)

"""GPU checks of the library's building blocks against plain references.

GEMM (every layout, batches, outer reduction, split-K, ragged edges) against a
float64 numpy product; the one-workgroup eigensolver and Cholesky against
LAPACK.  All calls go through the C ABI test hooks.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2512_09811_amd import binding
    binding.lib()
    assert torch.cuda.is_available()
    return binding


def _ref_gemm(A, Bm, M, N, K, KB, nb, tA, lda, sA, sAk, tB, ldb, sB, sBk):
    out = np.zeros((nb, M, N))
    for b in range(nb):
        for kb in range(KB):
            a0 = b * sA + kb * sAk
            b0 = b * sB + kb * sBk
            if tA:
                Am = np.array([[A[a0 + k * lda + m] for k in range(K)] for m in range(M)])
            else:
                Am = np.array([[A[a0 + m * lda + k] for k in range(K)] for m in range(M)])
            if tB:
                Bk = np.array([[Bm[b0 + n * ldb + k] for n in range(N)] for k in range(K)])
            else:
                Bk = np.array([[Bm[b0 + k * ldb + n] for n in range(N)] for k in range(K)])
            out[b] += Am @ Bk
    return out


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("pads", ["odd", "even"])
@pytest.mark.parametrize("M,N,K,KB,nb,tA,tB", [
    (1, 1, 1, 1, 1, 0, 0), (37, 53, 29, 1, 1, 0, 0), (37, 53, 29, 1, 1, 1, 0), (37, 53, 29, 1, 1, 0, 1),
    (37, 53, 29, 1, 1, 1, 1), (130, 150, 70, 1, 2, 0, 1), (20, 30, 17, 3, 2, 1, 0), (3, 5, 2000, 1, 1, 0, 1),
    (200, 7, 3000, 2, 1, 1, 1), (260, 300, 100, 2, 2, 0, 0), (260, 300, 100, 2, 2, 1, 0),
    (260, 300, 100, 2, 2, 0, 1), (260, 300, 100, 2, 2, 1, 1), (96, 80, 64, 1, 1, 0, 1)])
def test_gemm_layouts(B, fp32, pads, M, N, K, KB, nb, tA, tB):
    """'odd' pads give strides that are mostly not 2-element aligned (element-wise guarded
    loads); 'even' pads keep every stride and batch offset 2-element aligned, so interior
    tiles take the whole-pair load path and the ragged edges the guarded one."""
    rng = np.random.default_rng(M * 7 + N * 13 + K + KB + nb + tA * 3 + tB * 5)
    pa, pb, pak, pbk, psa, psb = (3, 2, 5, 4, 7, 3) if pads == "odd" else (2, 4, 6, 2, 4, 8)
    lda = (M if tA else K) + pa
    ldb = (K if tB else N) + pb
    rowsA = K if tA else M
    rowsB = N if tB else K
    sAk = rowsA * lda + pak
    sBk = rowsB * ldb + pbk
    sA = KB * sAk + psa
    sB = KB * sBk + psb
    ldc = N + 1
    sC = M * ldc + 2
    A = rng.standard_normal(nb * sA + 8)
    Bm = rng.standard_normal(nb * sB + 8)
    C0 = rng.standard_normal(nb * sC + 8)
    ref = _ref_gemm(A, Bm, M, N, K, KB, nb, tA, lda, sA, sAk, tB, ldb, sB, sBk)
    dt = torch.float32 if fp32 else torch.float64
    dA = torch.tensor(A, dtype=dt, device="cuda")
    dB = torch.tensor(Bm, dtype=dt, device="cuda")
    for beta, ws in ((0.0, 0), (0.5, 1 << 24)):
        dC = torch.tensor(C0, dtype=dt, device="cuda")
        B.gemm(dA, dB, dC, M=M, N=N, K=K, KB=KB, nbatch=nb, transA=tA, lda=lda, sA=sA, sAk=sAk, transB=tB, ldb=ldb,
               sB=sB, sBk=sBk, ldc=ldc, sC=sC, alpha=1.5, beta=beta, ws_bytes=ws, fp32=fp32)
        got = dC.double().cpu().numpy()
        exp = C0.copy()
        for b in range(nb):
            for m in range(M):
                exp[b * sC + m * ldc: b * sC + m * ldc + N] = 1.5 * ref[b, m] + beta * C0[b * sC + m * ldc:
                                                                                       b * sC + m * ldc + N]
        scale = np.sqrt(K * KB) * 3
        tol = (2e-6 if fp32 else 1e-14) * scale
        np.testing.assert_allclose(got, exp, rtol=(2e-5 if fp32 else 0), atol=tol)


@pytest.mark.parametrize("fp32", [False, True])
def test_gemm_peeled_tail(B, fp32):
    """A GEMM of 32 x 34 tiles (1088 workgroups: two full waves of 512 and 64 left over):
    the two trailing tile columns are peeled into a launch of 64 x 64 tiles; the result
    must equal the plain product (k-contiguous operands, the amplitude-contraction layout)
    and, with or without a workspace, be bit-identical to the unpeeled GEMM."""
    rng = np.random.default_rng(8)
    M, N, K = 4096, 128 * 33 + 40, 40
    A = rng.standard_normal((M, K))
    Bt = rng.standard_normal((N, K))
    C0 = rng.standard_normal((M, N))
    ref = 1.25 * (A @ Bt.T) + 0.5 * C0
    dt = torch.float32 if fp32 else torch.float64
    dA = torch.tensor(A, dtype=dt, device="cuda")
    dB = torch.tensor(Bt, dtype=dt, device="cuda")
    dC = torch.tensor(C0, dtype=dt, device="cuda")
    B.gemm(dA, dB, dC, M=M, N=N, K=K, KB=1, nbatch=1, transA=0, lda=K, sA=0, sAk=0, transB=1, ldb=K, sB=0, sBk=0,
           ldc=N, sC=0, alpha=1.25, beta=0.5, ws_bytes=64 << 20, fp32=fp32)
    got = dC.double().cpu().numpy()
    tol = (2e-5 if fp32 else 1e-13) * np.sqrt(K) * 3
    np.testing.assert_allclose(got, ref, rtol=(2e-5 if fp32 else 0), atol=tol)
    # bit-identical to the same product with no peeling (a batch of one GEMM per launch
    # is never peeled: the same operands as two stacked copies, batch stride 0 on A)
    dC2 = torch.tensor(np.stack([C0, C0]), dtype=dt, device="cuda")
    dB2 = torch.stack([dB, dB]).contiguous()
    B.gemm(dA, dB2, dC2, M=M, N=N, K=K, KB=1, nbatch=2, transA=0, lda=K, sA=0, sAk=0, transB=1, ldb=K,
           sB=N * K, sBk=0, ldc=N, sC=M * N, alpha=1.25, beta=0.5, ws_bytes=64 << 20, fp32=fp32)
    assert torch.equal(dC2[0], dC) and torch.equal(dC2[1], dC)


def _cmap_offsets(M, N, ldc, cRm, cSm, cRn, cSn):
    m, n = np.arange(M)[:, None], np.arange(N)[None, :]
    ro = (m // cRm) * cSm + (m % cRm) * ldc if cRm else m * ldc
    co = (n // cRn) * cSn + n % cRn if cRn else n
    return ro + co


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("case", ["g1_small", "g1_tiles", "rows_only", "cols_only", "splitk"])
def test_gemm_cmap(B, fp32, case):
    """C rows and columns split into index pairs: every mapped element equals the plain
    product (alpha, beta applied), every other element of the output array is left as it
    was.  g1_* write rows (q, j) and columns (P, d) of V B^vv into a [q][P][j][d] array,
    across several 128 x 128 tiles with the direct-to-LDS loads (g1_tiles) and in one
    ragged 64 x 64 tile (g1_small); splitk maps through the split-K reduction."""
    rng = np.random.default_rng({"g1_small": 1, "g1_tiles": 2, "rows_only": 3, "cols_only": 4, "splitk": 5}[case])
    beta = 0.0
    if case in ("g1_small", "g1_tiles"):
        o, v, X, k = (6, 10, 5, 3) if case == "g1_small" else (40, 160, 20, 4)
        M, N, K = k * o, X * v, v
        ldc, cRm, cSm, cRn, cSn = v, o, X * o * v, v, o * v
        size = k * X * o * v
    elif case == "rows_only":
        M, N, K = 200, 96, 48
        ldc, cRm, cSm, cRn, cSn = 100, 50, 50 * 100 + 7, 0, 0
        size = 4 * (50 * 100 + 7)
        beta = 0.5
    elif case == "cols_only":
        M, N, K = 130, 300, 36
        ldc, cRm, cSm, cRn, cSn = 4 * 80, 0, 0, 75, 80
        size = M * ldc
        beta = -1.0
    else:
        M, N, K = 40, 96, 6000
        ldc, cRm, cSm, cRn, cSn = 32, 8, 40 * 32, 32, 8 * 32
        size = 5 * 40 * 32
        beta = 0.25
    A = rng.standard_normal((M, K))
    Bt = rng.standard_normal((N, K))
    C0 = rng.standard_normal(size)
    off = _cmap_offsets(M, N, ldc, cRm, cSm, cRn, cSn)
    assert off.max() < size and len(np.unique(off)) == M * N
    exp = C0.copy()
    exp[off] = 1.5 * (A @ Bt.T) + beta * C0[off]
    dt = torch.float32 if fp32 else torch.float64
    dA, dB, dC = (torch.tensor(x, dtype=dt, device="cuda") for x in (A, Bt, C0))
    B.gemm_cmap(dA, dB, dC, M=M, N=N, K=K, transA=0, lda=K, transB=1, ldb=K, ldc=ldc, cRm=cRm, cSm=cSm, cRn=cRn,
                cSn=cSn, alpha=1.5, beta=beta, ws_bytes=64 << 20, fp32=fp32)
    got = dC.double().cpu().numpy()
    tol = (2e-5 if fp32 else 1e-13) * np.sqrt(K) * 3
    np.testing.assert_allclose(got, exp if not fp32 else exp, rtol=(2e-5 if fp32 else 0), atol=tol)
    untouched = np.ones(size, bool)
    untouched[off] = False
    assert np.array_equal(got[untouched], C0.astype(np.float32 if fp32 else np.float64)[untouched].astype(np.float64))


@pytest.mark.parametrize("fp32", [False, True])
def test_gemm_cmap_peeled(B, fp32):
    """Column-split output on a GEMM large enough for the peeled 64 x 64 tail (32 x 34
    tiles of 128): the product lands at the mapped places, and equals bit for bit the
    same GEMM written plainly (both tiles shapes accumulate every element over the same
    k sequence), the amplitude contraction's layout [q][(i,c)][P]."""
    rng = np.random.default_rng(9)
    M, N, K, R = 4096, 128 * 33 + 40, 40, 600
    nblk = (N + R - 1) // R
    A = rng.standard_normal((M, K))
    Bt = rng.standard_normal((N, K))
    dt = torch.float32 if fp32 else torch.float64
    dA, dB = (torch.tensor(x, dtype=dt, device="cuda") for x in (A, Bt))
    dC = torch.full((nblk * M * R,), 7.0, dtype=dt, device="cuda")
    B.gemm_cmap(dA, dB, dC, M=M, N=N, K=K, transA=0, lda=K, transB=1, ldb=K, ldc=R, cRn=R, cSn=M * R, fp32=fp32)
    dP = torch.empty((M, N), dtype=dt, device="cuda")
    B.gemm(dA, dB, dP, M=M, N=N, K=K, transA=0, lda=K, transB=1, ldb=K, ldc=N, fp32=fp32)
    off = torch.tensor(_cmap_offsets(M, N, R, 0, 0, R, M * R), device="cuda")
    assert torch.equal(dC[off], dP)
    ref = A @ Bt.T
    tol = (2e-5 if fp32 else 1e-13) * np.sqrt(K) * 3
    np.testing.assert_allclose(dP.double().cpu().numpy(), ref, rtol=(2e-5 if fp32 else 0), atol=tol)
    untouched = torch.ones(nblk * M * R, dtype=torch.bool, device="cuda")
    untouched[off.reshape(-1)] = False
    assert bool((dC[untouched] == 7.0).all())


@pytest.mark.parametrize("shape", [(300, 260, 100), (256, 384, 6400), (130, 4200, 64)])
def test_gemm_split_bf16(B, shape):
    """Split-BF16 GEMM (k-contiguous operands, the amplitude contraction's layout) against
    the float64 product of the same FP32 inputs: the split leaves about 2^-17 of |a||b| per
    product, so the error stays below 1e-5 sqrt(K) max|a| max|b|; ragged tiles in m, n and
    k, alpha and beta applied; and with a column index split on the output."""
    M, N, K = shape
    rng = np.random.default_rng(M + N + K)
    A = rng.standard_normal((M, K)).astype(np.float32)
    Bt = rng.standard_normal((N, K)).astype(np.float32)
    C0 = rng.standard_normal((M, N)).astype(np.float32)
    ref = 1.5 * (A.astype(np.float64) @ Bt.astype(np.float64).T) + 0.5 * C0
    dA, dB, dC = (torch.tensor(x, device="cuda") for x in (A, Bt, C0))
    B.gemm(dA, dB, dC, M=M, N=N, K=K, transA=0, lda=K, transB=1, ldb=K, ldc=N, alpha=1.5, beta=0.5, fp32=2)
    tol = 1e-5 * np.sqrt(K) * np.abs(A).max() * np.abs(Bt).max()
    err = np.abs(dC.double().cpu().numpy() - ref).max()
    assert err <= tol, (err, tol)
    # the same product through the split-BF16 kernel's mapped epilogue: blocks of 64 columns
    R = 64
    nblk = (N + R - 1) // R
    dM = torch.zeros(nblk * M * R, dtype=torch.float32, device="cuda")
    B.gemm_cmap(dA, dB, dM, M=M, N=N, K=K, transA=0, lda=K, transB=1, ldb=K, ldc=R, cRn=R, cSn=M * R, fp32=2)
    dP = torch.zeros((M, N), dtype=torch.float32, device="cuda")
    B.gemm(dA, dB, dP, M=M, N=N, K=K, transA=0, lda=K, transB=1, ldb=K, ldc=N, fp32=2)
    off = torch.tensor(_cmap_offsets(M, N, R, 0, 0, R, M * R), device="cuda")
    assert torch.equal(dM[off], dP)
    with pytest.raises(B.PPError):
        B.gemm(dA, dB, dP, M=M, N=N, K=K, transA=1, lda=M, transB=1, ldb=K, ldc=N, fp32=2)


@pytest.mark.parametrize("fp32", [False, True])
def test_gemm_long_rows(B, fp32):
    """A k-contiguous left operand with few rows and a row stride of 2^28 + 64 elements
    (the layout of the amplitude strip against the B^vv factors at large sizes): a 128-row
    tile would span more than 2^31 elements, but only the 5 existing rows are addressed, so
    the product runs and matches; 16 such rows exceed 32-bit in-tile offsets and are
    rejected before any launch."""
    rng = np.random.default_rng(11)
    M, N, K, lda = 5, 200, 40, (1 << 28) + 64
    dt = torch.float32 if fp32 else torch.float64
    A = rng.standard_normal((M, K))
    Bt = rng.standard_normal((N, K))
    dA = torch.zeros((M - 1) * lda + K, dtype=dt, device="cuda")
    for m in range(M):
        dA[m * lda:m * lda + K] = torch.tensor(A[m], dtype=dt)
    dB = torch.tensor(Bt, dtype=dt, device="cuda")
    dC = torch.zeros((M, N), dtype=dt, device="cuda")
    B.gemm(dA, dB, dC, M=M, N=N, K=K, transA=0, lda=lda, transB=1, ldb=K, ldc=N, fp32=fp32)
    tol = (2e-5 if fp32 else 1e-13) * np.sqrt(K) * 3
    np.testing.assert_allclose(dC.double().cpu().numpy(), A @ Bt.T, rtol=(2e-5 if fp32 else 0), atol=tol)
    del dA
    small = torch.zeros(64, dtype=dt, device="cuda")
    with pytest.raises(B.PPError, match="32-bit tile offsets"):
        B.gemm(small, dB, dC, M=16, N=N, K=K, transA=0, lda=lda, transB=1, ldb=K, ldc=N, fp32=fp32)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 24, 34, 37, 64, 65, 130, 400])
def test_small_syev(B, n):
    rng = np.random.default_rng(n)
    X = rng.standard_normal((n, n))
    A = X + X.T
    if n >= 5:
        A[0, :] = A[:, 0] = 0.0          # a decoupled block
        A[0, 0] = 0.5
    w_ref = np.linalg.eigvalsh(A)
    dA = torch.tensor(A, dtype=torch.float64, device="cuda")
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    Z = torch.empty((n, n), dtype=torch.float64, device="cuda")
    B.syev(dA, w, Z)
    w, Z = w.cpu().numpy(), Z.cpu().numpy()
    np.testing.assert_allclose(w, w_ref, rtol=0, atol=1e-12 * max(1.0, np.abs(w_ref).max()))
    assert np.abs(A @ Z - Z * w).max() < 1e-11 * max(1.0, np.abs(w_ref).max())
    assert np.abs(Z.T @ Z - np.eye(n)).max() < 1e-12


@pytest.mark.parametrize("n,kind", [(6, "identity"), (30, "repeated"), (48, "clustered"), (64, "diagonal")])
def test_small_syev_degenerate(B, n, kind):
    """Small eigenproblems with repeated, clustered or already diagonal spectra (the Gram
    matrices of nearly dependent vectors the solver orthonormalises)."""
    rng = np.random.default_rng(n)
    if kind == "identity":
        lam = np.ones(n)
    elif kind == "repeated":
        lam = np.repeat([0.5, 1.0, 2.0], n // 3)
    elif kind == "clustered":
        lam = np.concatenate([1.0 + 1e-13 * rng.standard_normal(n // 2), rng.uniform(1e-14, 3.0, n - n // 2)])
    else:
        lam = rng.uniform(-1.0, 1.0, n)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = np.diag(lam) if kind == "diagonal" else (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    dA = torch.tensor(A, dtype=torch.float64, device="cuda")
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    Z = torch.empty((n, n), dtype=torch.float64, device="cuda")
    B.syev(dA, w, Z)
    w, Z = w.cpu().numpy(), Z.cpu().numpy()
    np.testing.assert_allclose(w, np.sort(lam), rtol=0, atol=1e-13 * max(1.0, np.abs(lam).max()))
    assert np.abs(A @ Z - Z * w).max() < 1e-12 * max(1.0, np.abs(lam).max())
    assert np.abs(Z.T @ Z - np.eye(n)).max() < 1e-12


@pytest.mark.parametrize("n", [1, 4, 33, 64, 65, 130, 257, 480, 512])
def test_small_cholesky(B, n):
    rng = np.random.default_rng(n + 100)
    X = rng.standard_normal((n, n))
    A = X @ X.T + n * np.eye(n)
    dA = torch.tensor(A, dtype=torch.float64, device="cuda")
    L = torch.empty((n, n), dtype=torch.float64, device="cuda")
    B.cholesky(dA, L)
    np.testing.assert_allclose(L.cpu().numpy(), np.linalg.cholesky(A), rtol=0, atol=1e-12 * np.sqrt(n))


@pytest.mark.parametrize("fp32", [False, True])
def test_gemm_group(B, fp32):
    """Independent GEMMs issued together (grouped launches across members of one tile
    shape, single launches for the rest) equal their plain products."""
    rng = np.random.default_rng(77)
    dt = torch.float32 if fp32 else torch.float64
    # (M, N, K, transA, transB): the first five share a shape class and fill the chip
    # together (grouped); the 64-tile pair is too small and runs one by one
    shapes = [(1500, 1400, 96, 0, 1), (1300, 1100, 61, 0, 1), (997, 1603, 130, 0, 1), (1200, 1200, 16, 0, 1),
              (1100, 1300, 77, 0, 1), (1400, 1500, 40, 1, 0), (1024, 1301, 33, 1, 0), (1600, 1700, 30, 1, 0), (1400, 1300, 20, 1, 0),
              (60, 70, 50, 0, 0), (33, 90, 21, 0, 0)]
    members, refs = [], []
    for M, N, K, tA, tB in shapes:
        A = rng.standard_normal((K, M) if tA else (M, K))
        Bm = rng.standard_normal((N, K) if tB else (K, N))
        C0 = rng.standard_normal((M, N))
        a = A.T if tA else A
        b = Bm.T if tB else Bm
        refs.append(0.75 * (a @ b) + 0.5 * C0)
        members.append(dict(M=M, N=N, K=K, transA=tA, transB=tB, lda=A.shape[1], ldb=Bm.shape[1], ldc=N,
                            A=torch.tensor(A, dtype=dt, device="cuda"), B=torch.tensor(Bm, dtype=dt, device="cuda"),
                            C=torch.tensor(C0, dtype=dt, device="cuda"), alpha=0.75, beta=0.5))
    g = B.gemm_group(members, fp32=fp32)
    assert g >= 2  # both 128-tile shape classes went out as grouped launches
    for m, ref, (M, N, K, tA, tB) in zip(members, refs, shapes):
        got = m["C"].double().cpu().numpy()
        tol = (2e-6 if fp32 else 1e-13) * np.sqrt(K) * 3
        np.testing.assert_allclose(got, ref, rtol=0, atol=tol)


def _spectrum_matrix(lam, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((len(lam), len(lam))))
    return (Q * lam) @ Q.T


@pytest.mark.parametrize("case", ["uniform", "dense_near_target", "near_degenerate", "edge_target", "small",
                                  "diagonal", "block_diagonal"])
def test_partial_syev(B, case):
    """The p eigenpairs nearest a target (projected problem of the window solver)."""
    rng = np.random.default_rng(5)
    n, p, target = 400, 34, 0.9025
    if case == "uniform":
        lam = rng.uniform(0.1, 3.0, n)
    elif case == "dense_near_target":
        lam = np.concatenate([target + 5e-4 * np.arange(-60, 60) + 1e-5 * rng.standard_normal(120),
                              rng.uniform(0.14, 9.0, n - 120)])
    elif case == "near_degenerate":
        base = target + 4e-4 * np.arange(-20, 20)
        lam = np.concatenate([base, base[::3] + 1e-5, base[1::5] + 1e-8, base[2::7] + 1e-12,
                              rng.uniform(0.14, 9.0, n - 40 - len(base[::3]) - len(base[1::5]) - len(base[2::7]))])
    elif case == "edge_target":
        target = 0.05
        lam = rng.uniform(0.1, 3.0, n)
    elif case in ("diagonal", "block_diagonal"):
        lam = rng.uniform(0.1, 3.0, n)
    else:
        n, p = 30, 12
        lam = rng.uniform(0.5, 1.5, n)
    A = _spectrum_matrix(lam, 11)
    if case == "diagonal":
        # every Householder column is already zero below the subdiagonal
        A = np.diag(lam)
    elif case == "block_diagonal":
        # zero columns (first 150 rows/columns diagonal) then a dense block
        A = np.zeros((n, n))
        A[:150, :150] = np.diag(lam[:150])
        A[150:, 150:] = _spectrum_matrix(lam[150:], 12)
    dA = torch.tensor(A, device="cuda")
    lam_d = torch.zeros(p, dtype=torch.float64, device="cuda")
    Z = torch.zeros(n * p, dtype=torch.float64, device="cuda")
    q = B.partial_syev(dA, target, p, lam_d, Z)
    w = lam_d.cpu().numpy()[:q]
    Zh = Z.cpu().numpy().reshape(n, p)[:, :q]
    exact = np.sort(lam)
    nearest = np.sort(exact[np.argsort(np.abs(exact - target), kind="stable")[:p]])
    assert q == p, (q, p)
    np.testing.assert_allclose(np.sort(w), nearest, rtol=0, atol=1e-12 * np.abs(lam).max())
    res = np.linalg.norm(A @ Zh - Zh * w, axis=0)
    assert res.max() < 1e-10 * np.abs(lam).max(), res.max()
    np.testing.assert_allclose(Zh.T @ Zh, np.eye(q), atol=1e-10)


def _bf16_rne(x32):
    """float32 -> bf16 bit patterns, round to nearest even (finite inputs)."""
    b = x32.view(np.uint32).astype(np.uint64)
    return (((b + 0x7FFF + ((b >> 16) & 1)) >> 16) & 0xFFFF).astype(np.uint16)


def _bf16_value(h):
    return (h.astype(np.uint32) << 16).view(np.float32)


def test_split_sbf16_layout(B):
    """The split layout of the split-BF16 products, in place: every chunk of 8 float32
    values becomes their 8 bf16 hi parts (round to nearest even) followed by the 8 bf16
    lo parts of x - hi, and hi + lo reproduces x to 2^-16 relative; a length that is not
    a whole number of chunks is refused."""
    rng = np.random.default_rng(5)
    x = (rng.standard_normal(8 * 1001) * np.exp(rng.uniform(-20, 20, 8 * 1001))).astype(np.float32)
    x[:8] = [0.0, -0.0, 1.0, -1.0, 3.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, -(1.0 + 2.0 ** -8)]
    d = torch.tensor(x, device="cuda")
    B.split_sbf16(d)
    got = d.cpu().numpy().view(np.uint16).reshape(-1, 16)
    hi = _bf16_rne(x)
    lo = _bf16_rne((x - _bf16_value(hi)).astype(np.float32))
    np.testing.assert_array_equal(got[:, :8].ravel(), hi)
    np.testing.assert_array_equal(got[:, 8:].ravel(), lo)
    back = _bf16_value(hi).astype(np.float64) + _bf16_value(lo).astype(np.float64)
    assert np.all(np.abs(back - x) <= 2.0 ** -16 * np.abs(x))
    # ties go to even: 1 + 2^-8 rounds down to 1, 1 + 3 * 2^-9 up to 1 + 2^-7
    assert _bf16_value(hi[5:7]).tolist() == [1.0, 1.0 + 2.0 ** -7]
    with pytest.raises(B.PPError):
        B.split_sbf16(torch.zeros(12, dtype=torch.float32, device="cuda"))


@pytest.mark.parametrize("shape", [(256, 256, 4096), (200, 300, 1000)])
def test_gemm_split_bf16_presplit(B, shape):
    """The split-BF16 kernel on operands split in place (rows padded to 8 values with
    zeros): the same result as the path that splits copies, bit for bit, and within the
    split's error of the float64 product; leading dimensions that are not whole chunks
    are refused."""
    M, N, K = shape
    ld = (K + 7) // 8 * 8
    rng = np.random.default_rng(M * 3 + K)
    A = np.zeros((M, ld), np.float32)
    Bt = np.zeros((N, ld), np.float32)
    A[:, :K] = rng.standard_normal((M, K))
    Bt[:, :K] = rng.standard_normal((N, K))
    dA, dB = torch.tensor(A, device="cuda"), torch.tensor(Bt, device="cuda")
    ref_c = torch.empty((M, N), dtype=torch.float32, device="cuda")
    B.gemm(dA, dB, ref_c, M=M, N=N, K=K, transA=0, lda=ld, transB=1, ldb=ld, ldc=N, fp32=2)
    B.split_sbf16(dA)
    B.split_sbf16(dB)
    dC = torch.empty((M, N), dtype=torch.float32, device="cuda")
    B.gemm(dA, dB, dC, M=M, N=N, K=K, transA=0, lda=ld, transB=1, ldb=ld, ldc=N, fp32=3)
    assert torch.equal(dC, ref_c)
    ref = A[:, :K].astype(np.float64) @ Bt[:, :K].astype(np.float64).T
    err = np.abs(dC.double().cpu().numpy() - ref).max()
    assert err <= 1e-5 * np.sqrt(K) * np.abs(A).max() * np.abs(Bt).max(), err
    if K % 8:
        with pytest.raises(B.PPError):
            B.gemm(dA, dB, dC, M=M, N=N, K=K, transA=0, lda=K, transB=1, ldb=K, ldc=N, fp32=3)


@pytest.mark.parametrize("shape", [(4000, 8000, 333), (512, 768, 2048)])
def test_gemm_split_bf16_tiles(B, shape):
    """The split-BF16 kernel's 128 x 128 and 256 x 256 tiles (and the shape-chosen one)
    give bit-identical products: every element sums the same 16-value steps in the same
    order, hi-lo, lo-hi, hi-hi; ragged edges in m, n and k; within the split's error of
    the float64 product."""
    M, N, K = shape
    ld = (K + 7) // 8 * 8
    g = torch.Generator(device="cuda").manual_seed(K)
    dA = torch.zeros((M, ld), dtype=torch.float32, device="cuda")
    dB = torch.zeros((N, ld), dtype=torch.float32, device="cuda")
    dA[:, :K] = torch.randn((M, K), generator=g, device="cuda")
    dB[:, :K] = torch.randn((N, K), generator=g, device="cuda")
    ref = (dA[:, :K].double() @ dB[:, :K].double().T).cpu().numpy()
    B.split_sbf16(dA)
    B.split_sbf16(dB)
    outs = []
    for code in (3, 4, 5):
        dC = torch.full((M, N), 3.0, dtype=torch.float32, device="cuda")
        B.gemm(dA, dB, dC, M=M, N=N, K=K, transA=0, lda=ld, transB=1, ldb=ld, ldc=N, alpha=0.5, beta=2.0, fp32=code)
        outs.append(dC)
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])
    err = np.abs(outs[0].double().cpu().numpy() - (0.5 * ref + 6.0)).max()
    assert err <= 1e-5 * np.sqrt(K) * 0.5 * 25.0, err

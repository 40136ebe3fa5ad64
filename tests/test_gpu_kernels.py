"""Kernel-level parity on the GPU: MFMA contractions, collocation, shift-sums, point sampling and
the Jacobi SVD, each against the CPU oracle or exact arithmetic."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import dev, empty, host, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    # Jacobi on blocks of 8 columns here; the 16-column blocks have a test of their own
    require_gpu()
    import paper_1411_1994_amd as L
    c = L.Context(0)
    c.set_option(L.OPT_JACOBI_BLOCK, 8)
    yield c
    c.close()


# ------------------------------------------------------------------------------------------
# MFMA contraction (projections and mode products)
# ------------------------------------------------------------------------------------------

@pytest.fixture(params=[0, 1], ids=["own-kernel", "blas-library"])
def gemm_lib(request):
    # FP64 products on the library's own MFMA kernel, or (large unit-stride ones) on the ROCm
    # BLAS DGEMM; the switch is process-wide, so it is restored afterwards
    import paper_1411_1994_amd as L
    with L.Context(0) as c:
        c.set_option(L.OPT_GEMM_LIBRARY, request.param)
    yield request.param
    with L.Context(0) as c:
        c.set_option(L.OPT_GEMM_LIBRARY, 1)


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (16, 16, 4), (64, 64, 16), (70, 33, 129), (200, 150, 517),
                                   (300, 400, 301)])
@pytest.mark.parametrize("layout", ["nn", "tn", "nt", "tt"])
def test_contract_fp64(ctx, gemm_lib, m, n, k, layout):
    import torch
    import paper_1411_1994_amd as L
    rng = np.random.default_rng(m * 1000 + n + k)
    A = rng.standard_normal((m, k))
    B = rng.standard_normal((k, n))
    Cin = rng.standard_normal((m, n))
    As = A if layout[0] == "n" else np.ascontiguousarray(A.T)
    Bs = B if layout[1] == "n" else np.ascontiguousarray(B.T)
    sam, sak = (k, 1) if layout[0] == "n" else (1, m)
    sbk, sbn = (n, 1) if layout[1] == "n" else (1, k)
    dA, dB, dC = dev(As), dev(Bs), dev(Cin)
    ctx.contract(L.FP64, m, n, k, dA, sam, sak, dB, sbk, sbn, dC, n, 1, alpha=0.5, beta=2.0)
    got = host(dC)
    ref = 0.5 * (A @ B) + 2.0 * Cin
    # FP64 with k-term sums: |err| <= k u sum |a||b| (deterministic bound, u = 2^-53)
    bound = k * 2.0 ** -53 * (0.5 * np.abs(A) @ np.abs(B) + 2 * np.abs(Cin)) * 4 + 1e-300
    assert np.all(np.abs(got - ref) <= bound)


@pytest.mark.parametrize("m,n,k", [(33, 33, 34305), (50, 50, 4099), (7, 200, 5000), (128, 64, 2048),
                                   (1, 1, 100003)])
@pytest.mark.parametrize("layout", ["nn", "tn", "nt", "tt"])
def test_contract_fp64_split_reduction(ctx, gemm_lib, m, n, k, layout):
    # few output tiles and a long reduction: the reduction is split over workgroups and the slices'
    # products summed in order; C has a row stride wider than n (only its m x n part is written)
    import paper_1411_1994_amd as L
    rng = np.random.default_rng(m * 7 + n * 3 + k)
    A = rng.standard_normal((m, k))
    B = rng.standard_normal((k, n))
    ldc = n + 5
    Cin = rng.standard_normal((m, ldc))
    As = A if layout[0] == "n" else np.ascontiguousarray(A.T)
    Bs = B if layout[1] == "n" else np.ascontiguousarray(B.T)
    sam, sak = (k, 1) if layout[0] == "n" else (1, m)
    sbk, sbn = (n, 1) if layout[1] == "n" else (1, k)
    dA, dB, dC = dev(As), dev(Bs), dev(Cin)
    ctx.contract(L.FP64, m, n, k, dA, sam, sak, dB, sbk, sbn, dC, ldc, 1, alpha=0.5, beta=2.0)
    got = host(dC)
    ref = Cin.copy()
    ref[:, :n] = 0.5 * (A @ B) + 2.0 * Cin[:, :n]
    bound = k * 2.0 ** -53 * (0.5 * np.abs(A) @ np.abs(B) + 2 * np.abs(Cin[:, :n])) * 4 + 1e-300
    assert np.all(np.abs(got[:, :n] - ref[:, :n]) <= bound)
    assert np.array_equal(got[:, n:], Cin[:, n:])


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("m,n,k", [(16, 16, 32), (70, 33, 129), (130, 257, 700), (300, 400, 301)])
@pytest.mark.parametrize("layout", ["nn", "tn", "nt", "tt"])
def test_contract_fp32_and_split_bf16(ctx, prec, m, n, k, layout):
    import paper_1411_1994_amd as L
    rng = np.random.default_rng(7 + m + n + k)
    A = rng.standard_normal((m, k)).astype(np.float32)
    B = rng.standard_normal((k, n)).astype(np.float32)
    As = A if layout[0] == "n" else np.ascontiguousarray(A.T)
    Bs = B if layout[1] == "n" else np.ascontiguousarray(B.T)
    sam, sak = (k, 1) if layout[0] == "n" else (1, m)
    sbk, sbn = (n, 1) if layout[1] == "n" else (1, k)
    dA, dB, dC = dev(As), dev(Bs), dev(np.zeros((m, n), np.float32))
    P = L.FP32 if prec == "fp32" else L.BF16X3
    ctx.contract(P, m, n, k, dA, sam, sak, dB, sbk, sbn, dC, n, 1)
    got = host(dC).astype(np.float64)
    ref = A.astype(np.float64) @ B.astype(np.float64)
    scale = np.abs(A).astype(np.float64) @ np.abs(B).astype(np.float64)
    # FP32 accumulation: k 2^-24 relative to sum|a||b|; split-BF16x3 drops lo*lo (2^-16 each)
    # and rounds the split (2^-17): about 2^-15 relative per product
    unit = 2.0 ** -24 * k if prec == "fp32" else 2.0 ** -15 + 2.0 ** -24 * k
    assert np.all(np.abs(got - ref) <= 2 * unit * scale + 1e-30)
    if prec == "bf16x3":
        # and clearly better than plain bfloat16 (2^-8)
        assert np.max(np.abs(got - ref) / scale) < 2.0 ** -12


# ------------------------------------------------------------------------------------------
# collocation and shift-sums
# ------------------------------------------------------------------------------------------

def colloc_tol(N, ldg, R):
    # per entry: erf differences lose log10((|d|+h)/h) digits; device and numpy erfc differ by
    # a few ulp (scipy is good to ~2e-14 in the deep tail)
    m = np.arange(2 * N - 1)
    return 1e-13 + 1e-15 * np.abs(m - (N - 1))


@pytest.mark.parametrize("kind,param,N,h,M", [(W.NEWTON, 0.0, 129, 3 / 32, 32),
                                             (W.YUKAWA, 0.5, 513, 0.07, 40),
                                             (W.SLATER, 1.0, 257, 0.11, 40),
                                             (W.NEWTON, 0.0, 4097, 5 / 256, 40)])
def test_collocation_matches_oracle(ctx, kind, param, N, h, M):
    import torch
    import paper_1411_1994_amd as L
    t, w = L.lsum_nodes(kind, param, M, (N, N, N), h)
    ldg = (2 * N - 1 + 7) // 8 * 8
    G = empty(len(t) * ldg, torch.float64)
    ctx.collocate(t, w, N, h, G, ldg)
    got = host(G).reshape(len(t), ldg)
    ref = O.reference_vectors(t, w, N, h)        # oracle's own collocation of the same nodes
    assert np.all(got[:, 2 * N - 1:] == 0.0)
    g = got[:, :2 * N - 1]
    rel = np.abs(g - ref) / np.maximum(np.abs(ref), 1e-300)
    tol = colloc_tol(N, ldg, len(t))[None, :]
    small = ref < 1e-280
    assert np.all((rel <= tol) | small)


COMB_51_2 = [int(np.sign(x) * np.floor(abs(x) + 0.5)) + 1024 for x in (np.arange(40) - 19.5) * 51.2 / 2]


@pytest.mark.parametrize("N_axis,N_ref,sites,M", [(129, 129, [48, 59, 69, 80], 30),
                                                  (33, 41, [0, 5, 32, 17, 17], 30),
                                                  (777, 777, list(range(3, 770, 11)), 30),   # one comb
                                                  (2049, 2049, COMB_51_2, 30),               # five combs
                                                  (2049, 2049, COMB_51_2[:38], 60),          # 8 and 7 sites
                                                  (300, 311, [7, 30, 53, 76, 99], 80),       # two node blocks
                                                  (1000, 1001, [], 30),
                                                  (1, 1, [0], 30),                           # one cell
                                                  (2, 3, [1, 0], 12)])
def test_shift_sum_matches_oracle(ctx, N_axis, N_ref, sites, M):
    import torch
    import paper_1411_1994_amd as L
    h = 0.05
    # a one-cell grid has no default quadrature scale: give (h_u, s) explicitly there
    t, w = L.lsum_nodes(W.NEWTON, 0.0, M, (N_ref, N_ref, N_ref), h, *((0.35, 1.0) if N_ref == 1 else ()))
    R = len(t)
    ldg = 2 * N_ref - 1 + 5
    G = empty(R * ldg, torch.float64)
    ctx.collocate(t, w, N_ref, h, G, ldg)
    U = empty(R * (N_axis + 3), torch.float64)
    ctx.shift_sum(R, G, ldg, N_ref, N_axis, np.array(sites, np.int32), U, N_axis + 3)
    Gh = host(G).reshape(R, ldg)[:, :2 * N_ref - 1]
    got = host(U).reshape(R, N_axis + 3)[:, :N_axis]
    # same reference rows on both sides: every term is positive, so any summation order (site
    # by site, or comb by comb) agrees to (n - 1) unit roundoffs relative
    ref = O.shift_sum(Gh, np.array(sites), N_axis, N_ref)
    assert np.all(np.abs(got - ref) <= 1.2e-16 * max(1, len(sites)) * np.abs(ref))
    # and against the oracle's own reference rows (deep-tail entries of the collocation agree to
    # an absolute floor, far below the row's total)
    ref2 = O.shift_sum(O.reference_vectors(t, w, N_ref, h), np.array(sites), N_axis, N_ref)
    floor = 1e-14 * np.sum(np.abs(Gh), axis=1, keepdims=True)
    assert np.all(np.abs(got - ref2) <= 1e-12 * np.abs(ref2) + floor)


def _snapped(L, beta, N):
    # L sites at spacing beta cells, centred on an N-cell axis and snapped to the nearest cell
    x = (np.arange(L) - (L - 1) / 2) * beta
    return [int(np.sign(v) * np.floor(abs(v) + 0.5)) + (N - 1) // 2 for v in x]


# sites whose spacing in cells has no short period (the served mix's b/h = (N - 1) / (L + 16)
# with L + 16 odd): they split into a few runs of one stride, each read as the difference of two
# strided prefix or suffix sums of the rows
STRIDED = [(4097, 4097, _snapped(87, 4096 / 103, 4097)),     # 9 runs of stride 159 (period 43)
           (4097, 4097, _snapped(82, 4096 / 98, 4097)),      # 6 runs of stride 209
           (809, 809, _snapped(36, 1024 / 66, 809)),         # 4 runs of stride 31
           (2969, 4097, _snapped(55, 4096 / 98, 2969)),      # N_axis < N_ref: 7 runs
           (4097, 4097, _snapped(87, 4096 / 103, 4097) + [2048, 30, 4000]),   # 12 runs, lone sites among them
           (3915, 4097, _snapped(91, 4096 / 112, 3915))]     # period 7: the comb form stays


@pytest.mark.parametrize("N_axis,N_ref,sites", STRIDED)
def test_shift_sum_on_strided_runs_matches_oracle(ctx, N_axis, N_ref, sites):
    import torch
    import paper_1411_1994_amd as L
    h = 0.03
    t, w = L.lsum_nodes(W.NEWTON, 0.0, 40, (N_ref, N_ref, N_ref), h)
    R = len(t)
    ldg = 2 * N_ref - 1 + 1
    G = empty(R * ldg, torch.float64)
    ctx.collocate(t, w, N_ref, h, G, ldg)
    U = empty(R * N_axis, torch.float64)
    ctx.shift_sum(R, G, ldg, N_ref, N_axis, np.array(sites, np.int32), U, N_axis)
    Gh = host(G).reshape(R, ldg)[:, :2 * N_ref - 1]
    got = host(U).reshape(R, N_axis)
    ref = O.shift_sum(Gh, np.array(sites), N_axis, N_ref)
    # a run read as a difference of two strided sums: each table entry is a compensated sum
    # (within two unit roundoffs of its chain's sum, and a chain is a subset of the row), and the
    # at most n terms are added in order, so the error is below 3.5 n u times the row's sum
    # besides the (n - 1) u relative of the positive site terms themselves
    n = len(sites)
    u = 2.0 ** -53
    rowsum = np.sum(np.abs(Gh), axis=1, keepdims=True)
    assert np.all(np.abs(got - ref) <= 1.2e-16 * n * np.abs(ref) + 3.5 * n * u * rowsum)
    # where the lattice sits (every cell between its first and last site) the sum is of the
    # row's order, and the comparison is relative to it
    lo, hi = min(sites), max(sites)
    inner = slice(lo, hi + 1)
    assert np.all(np.abs(got[:, inner] - ref[:, inner]) <= 1e-13 * np.abs(ref[:, inner]) + 1e-15 * rowsum)


def test_shift_sum_rejects_bad_sites(ctx):
    import torch
    import paper_1411_1994_amd as L
    G = empty(100, torch.float64)
    U = empty(100, torch.float64)
    with pytest.raises(L.LsumError) as e:
        ctx.shift_sum(1, G, 100, 40, 40, np.array([3, 40], np.int32), U, 50)
    assert e.value.code == -2


def test_sample_canonical_snaps_like_oracle(ctx):
    import torch
    import paper_1411_1994_amd as L
    rng = np.random.default_rng(3)
    N = (41, 37, 53)
    h = 0.3
    R = 5
    U = [rng.standard_normal((R, n)) for n in N]
    ldu = max(N)
    packed = np.zeros((3, R, ldu))
    for l in range(3):
        packed[l, :, :N[l]] = U[l]
    B = np.array([(n - 1) * h / 2 for n in N])
    xyz = rng.uniform(-B - 0.49 * h, B + 0.49 * h, size=(500, 3))
    xyz[:5] = np.array([[0.15, 0.45, -0.15], [0.75, -0.75, 1.05], [-6.0, 5.4, 7.8],
                        [6.0, -5.4, -7.8], [0.0, 0.0, 0.0]])
    dU, dx, dout = dev(packed), dev(xyz), empty(500, torch.float64)
    ctx.sample_canonical(1, R, dU, ldu, np.array([2.0]), N, h, 500, dx, dout)
    got = host(dout)
    pts = O.points_to_cells(xyz, h, N)
    ref = 2.0 * O.canonical_eval(U, pts)
    assert np.allclose(got, ref, rtol=1e-14, atol=1e-14)


# ------------------------------------------------------------------------------------------
# Jacobi SVD
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("D,N,decay", [(16, 40, 1.0), (40, 100, 1e-12), (100, 64, 1e-6), (257, 300, 1e-14)])
def test_jacobi_svd_known_spectrum(ctx, D, N, decay):
    _check_known_spectrum(ctx, D, N, decay)


@pytest.mark.parametrize("block", [16, 32])
@pytest.mark.parametrize("D,N,decay", [(16, 40, 1.0), (33, 100, 1e-12), (100, 64, 1e-6), (257, 300, 1e-14),
                                       (700, 1500, 1e-9)])
def test_jacobi_svd_wide_blocks_known_spectrum(block, D, N, decay):
    # pairs of 32 or 64 rows (four-wave pair solves, a half or a quarter of the rounds per sweep):
    # the same checks
    import paper_1411_1994_amd as L
    require_gpu()
    with L.Context(0, n_slots=1) as c:
        c.set_option(L.OPT_JACOBI_BLOCK, block)
        _check_known_spectrum(c, D, N, decay)


def _check_known_spectrum(ctx, D, N, decay):
    rng = np.random.default_rng(D + N)
    r = min(D, N)
    U, _ = np.linalg.qr(rng.standard_normal((N, r)))
    V, _ = np.linalg.qr(rng.standard_normal((D, r)))
    s = np.geomspace(10.0, 10.0 * decay, r) if decay != 1.0 else np.linspace(3, 1, r)
    A = (U * s) @ V.T                     # N x D, columns a_j
    X = np.ascontiguousarray(A.T)         # rows = columns
    dX = dev(X)
    sig, sweeps = ctx.jacobi_svd(D, N, dX, N)
    Xr = host(dX).reshape(D, N)
    # singular values to absolute accuracy ~ eps_mach * sigma_max * sqrt(D)
    assert np.all(np.abs(sig[:r] - s) <= 1e-14 * s[0] * math.sqrt(D) * 4)
    assert np.all(sig[r:] <= 1e-13 * s[0])
    # rotated columns: mutually orthogonal, norms = sigma (descending)
    nr = np.linalg.norm(Xr, axis=1)
    assert np.allclose(nr, sig, rtol=1e-12, atol=1e-14 * s[0])
    k = int(np.sum(sig > 1e-10 * s[0]))
    Zk = Xr[:k] / sig[:k, None]
    assert np.max(np.abs(Zk @ Zk.T - np.eye(k))) < 1e-11
    # what the truncation relies on: projecting onto the leading r columns leaves exactly the
    # tail (sum_{j >= r} s_j^2)^(1/2), to the absolute accuracy eps * sigma_max
    for rr in sorted({1, k // 3, k // 2, k}):
        if rr < 1:
            continue
        Zr = Zk[:rr]
        res = np.linalg.norm(A - Zr.T @ (Zr @ A))
        tail = math.sqrt(np.sum(s[rr:] ** 2))
        assert abs(res - tail) <= 1e-12 * s[0] * math.sqrt(D), (rr, res, tail)
    assert sweeps < 40


def test_jacobi_svd_side_matrix_tails(ctx):
    # the normalised side matrix of a small defected lattice: tails of sigma^2 against the
    # oracle's LAPACK SVD, including far below sqrt(eps) * sigma_1
    rng = np.random.default_rng(9)
    blocks = [W.cubic_block(6)]
    p = W.Problem("jac", W.NEWTON, 0.0, 30, (129, 129, 129), 0.2, blocks,
                  W.draw_defects(rng, blocks, 10, 5))
    xi, A = O.canonical_terms(p)
    A0 = A[0]
    X = np.ascontiguousarray(A0.T)
    dX = dev(X)
    sig, _ = ctx.jacobi_svd(X.shape[0], X.shape[1], dX, X.shape[1])
    ref = np.linalg.svd(A0, compute_uv=False)
    n = len(ref)
    # one-sided Jacobi is backward stable: each column takes part in ~D rotations per sweep, so
    # singular values agree with LAPACK to a small multiple of eps * sigma_max * sqrt(D * sweeps)
    assert np.all(np.abs(sig[:n] - ref) <= 1e-12 * ref[0])
    tg, tr = O.tail_norms(sig[:n]), O.tail_norms(ref)
    assert np.all(np.abs(tg - tr) <= 1e-12 * ref[0])

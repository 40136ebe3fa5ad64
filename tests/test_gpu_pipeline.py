"""End-to-end parity of whole requests (submit -> results) against the CPU oracle."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    import paper_1411_1994_amd as L
    c = L.Context(0)
    yield c
    c.close()


def cells_xyz(p, pts):
    return np.stack([(pts[:, a] - (p.N[a] - 1) // 2) * p.h for a in range(3)], axis=1)


def run(ctx, p):
    r = ctx.submit(p)
    rc = r.wait()
    assert rc == 0, r.stats()
    return r


def test_cfg1_all_points_match_brute_force(ctx):
    # config 1: 4x4x4 Newton lattice, N = 129, M = 32; every one of the 129^3 cells vs O1
    p = W.config(1)
    r = run(ctx, p)
    g = np.stack(np.meshgrid(*[np.arange(n) for n in p.N], indexing="ij"), -1).reshape(-1, 3)
    got = r.sample(cells_xyz(p, g)).reshape(p.N)
    ref = O.brute_force_grid(p)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    assert err <= 1e-12, err
    # the canonical factors are the oracle's assembled vectors (unique given the nodes)
    U = r.canonical(0)
    Uo = O.assembled_canonical(p)[0]
    for a in range(3):
        # entries of the narrowest Gaussians underflow far from the charges: per-row floor
        floor = 1e-13 * np.max(np.abs(Uo[a]), axis=1, keepdims=True)
        assert np.all(np.abs(U[a] - Uo[a]) <= 1e-12 * np.abs(Uo[a]) + floor)
    st = r.stats()
    assert st["offsets"][0][0] == [48, 59, 69, 80]
    r.release()


def _shortest_period(c):
    c = np.sort(np.asarray(c))
    for p in range(1, len(c) // 2 + 1):
        d = c[p:] - c[:-p]
        if d[0] > 0 and np.all(d == d[0]):
            return p
    return 0


@pytest.mark.parametrize("kind,param", [(W.NEWTON, 0.0), (W.SLATER, 1.0)])
def test_served_mix_shape_canonical_matches_oracle(ctx, kind, param):
    # a served-mix-shaped lattice (b/h = (N - 1) / (L_max + 16) = 512 / 55): no axis has a comb
    # period of 8 or less (13, none, none), and runs of one stride need 10 terms per axis against
    # 13, 25 and 17, so the request's shift-sums read those runs as differences of strided
    # prefix / suffix sums.  Values at points within 1e-12 of the largest direct-sum
    # value; factors within 1e-12 relative of the oracle's site-by-site sums near the lattice,
    # and everywhere within 5 n u of the reference row's sum (each of at most n terms is within
    # two roundoffs of its chain's sum, a chain being part of the row, plus the additions)
    L = (39, 25, 17)
    h = 2.0 * (max(L) / 2 + 8) / 512
    N = tuple(513 if l == max(L) else int(2 * np.ceil((l / 2 + 8) / h) + 1) for l in L)
    p = W.Problem("mixshape", kind, param, 30, N, h, [W.Block(L, (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))], [])
    r = run(ctx, p)
    offs = r.stats()["offsets"][0]   # block 0: the sites of each axis
    assert all(_shortest_period(offs[a]) in (0, 13) for a in range(3))
    rng = np.random.default_rng(41 + kind)
    pts = np.stack([rng.integers(0, n, 400) for n in p.N], axis=1)
    got = r.sample(cells_xyz(p, pts))
    ref = O.brute_force_points(p, pts)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    t, w = O.quadrature_of(p)
    Nr = max(p.N)
    rowsum = np.sum(np.abs(O.reference_vectors(t, w, Nr, p.h)), axis=1, keepdims=True)
    U = r.canonical(0)
    Uo = O.assembled_canonical(p)[0]
    u = 2.0 ** -53
    for a in range(3):
        n = L[a]
        assert np.all(np.abs(U[a] - Uo[a]) <= 1.2e-16 * n * np.abs(Uo[a]) + 5 * n * u * rowsum)
        lo, hi = min(offs[a]), max(offs[a])
        near = slice(lo, hi + 1)
        floor = 1e-13 * np.max(np.abs(Uo[a]), axis=1, keepdims=True)
        assert np.all(np.abs(U[a][:, near] - Uo[a][:, near]) <= 1e-12 * np.abs(Uo[a][:, near]) + floor)
    r.release()


@pytest.mark.parametrize("kind,param", [(W.NEWTON, 0.0), (W.YUKAWA, 0.5), (W.SLATER, 1.0)])
def test_defects_and_blocks_canonical(ctx, kind, param):
    rng = np.random.default_rng(21 + kind)
    big = W.Block((6, 5, 4), (1.0, 1.1, 0.9), (0.13, -0.2, 0.07))
    second = W.Block((3, 3, 2), (1.0, 1.0, 1.0), (-1.5, 4.4, 3.1), charge=0.5)
    defects = W.draw_defects(rng, [big, second], 6, 4)
    p = W.Problem("def", kind, param, 28, (61, 67, 55), 0.21, [big, second], defects)
    r = run(ctx, p)
    pts = np.stack([rng.integers(0, n, 400) for n in p.N], axis=1)
    got = r.sample(cells_xyz(p, pts))
    ref = O.brute_force_points(p, pts)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    r.release()


@pytest.mark.parametrize("kind,param", [(W.NEWTON, 0.0), (W.SLATER, 1.0)])
def test_fp32_canonical_factors(ctx, kind, param):
    # FP32 precision on canonical output keeps the point-major factors rounded to FP32 and forms
    # products and sums in FP64.  Every factor entry is then within one rounding (2^-24 relative,
    # or the FP32 underflow threshold) of the oracle's assembled sums, and a sampled value is off
    # by at most 3 roundings per term: |err| <= 3.01 * 2^-24 * sum_b |lam_b| sum_q prod_l |U|,
    # which for these positive kernels and charges is the defect-free potential itself.  The
    # defect windows come from the FP64 reference rows and add only FP64 rounding.
    rng = np.random.default_rng(31 + kind)
    big = W.Block((6, 5, 4), (1.0, 1.1, 0.9), (0.13, -0.2, 0.07))
    second = W.Block((3, 3, 2), (1.0, 1.0, 1.0), (-1.5, 4.4, 3.1), charge=0.5)
    defects = W.draw_defects(rng, [big, second], 6, 4)
    p = W.Problem("f32", kind, param, 28, (61, 67, 55), 0.21, [big, second], defects, precision=W.FP32)
    r = run(ctx, p)
    u = 2.0 ** -24
    Uo = O.assembled_canonical(p)
    for b in range(2):
        U, wb = r.canonical(b, with_weight=True)
        assert wb == p.blocks[b].charge                 # the block's weight in eq. CP_form
        for a in range(3):
            # the FP64 sums agree with the oracle to 1e-12 (per-row floor for underflowing tails)
            floor = 1e-13 * np.max(np.abs(Uo[b][a]), axis=1, keepdims=True) + 2.0 ** -126
            assert np.all(np.abs(U[a] - Uo[b][a]) <= (u + 1e-12) * np.abs(Uo[b][a]) + floor)
    pts = np.stack([rng.integers(0, n, 400) for n in p.N], axis=1)
    got = r.sample(cells_xyz(p, pts))
    ref = O.brute_force_points(p, pts)
    clean = O.brute_force_points(W.Problem(**{**p.__dict__, "defects": []}), pts)
    assert np.all(clean > 0)
    err = np.abs(got - ref)
    assert np.all(err <= 3.01 * u * clean + 1e-12 * np.max(np.abs(ref))), np.max(err / clean)
    assert np.max(err / np.abs(ref)) <= 1e-6
    # FP32 factors take half the resident bytes of FP64 ones
    p64 = W.Problem(**{**p.__dict__, "precision": W.FP64})
    r64 = run(ctx, p64)
    assert r.stats()["bytes"]["canonical"] * 2 == r64.stats()["bytes"]["canonical"]
    r64.release()
    r.release()


def test_points_outside_grid_are_nan(ctx):
    p = W.Problem("nan", W.NEWTON, 0.0, 10, (21, 21, 21), 0.5, [W.cubic_block(2)])
    r = run(ctx, p)
    v = r.sample(np.array([[0.0, 0.0, 0.0], [5.26, 0.0, 0.0], [0.0, -5.3, 0.0]]))
    assert np.isfinite(v[0]) and np.isnan(v[1]) and np.isnan(v[2])
    r.release()


def _small_defected(kind=W.NEWTON, param=0.0, eps=1e-6, precision=W.FP64, seed=11, tile=True, n_vac=5, n_imp=3):
    rng = np.random.default_rng(seed)
    blocks = [W.Block((5, 4, 4), (1.0, 1.0, 1.0), (0.1, -0.2, 0.05))]
    defects = W.draw_defects(rng, blocks, n_vac, n_imp)
    N = (33, 37, 31)
    p = W.Problem("rh", kind, param, 20, N, 0.37, blocks, defects, eps=eps, precision=precision)
    if tile:
        p.tile_lo = (0, 0, 0)
        p.tile_T = N
    return p


@pytest.mark.parametrize("kind,param", [(W.NEWTON, 0.0), (W.YUKAWA, 0.5), (W.SLATER, 1.0)])
@pytest.mark.parametrize("eps", [1e-3, 1e-6, 1e-9])
def test_rhosvd_fp64_matches_oracle(ctx, kind, param, eps):
    p = _small_defected(kind, param, eps)
    r = run(ctx, p)
    inf = r.info()
    xi, A = O.canonical_terms(p)
    ref = O.rhosvd(xi, A, eps=eps)
    full = O.cp_full(xi, A)
    nA = np.linalg.norm(full)
    assert abs(inf.norm_A - nA) <= 1e-12 * nA
    assert abs(inf.norm_xi - ref.norm_xi) <= 1e-12 * ref.norm_xi
    # singular values of the (deduplicated, multiplicity-weighted) side matrices = oracle's literal
    # ones, for every value above the irrelevance floor (1% of thr / sqrt(D)); below it only the
    # tail sums matter and they are certified upper bounds
    thr = eps * nA / (3 * ref.norm_xi)
    irr = 1e-2 * thr / math.sqrt(max(inf.D))
    sig = r.sigma()
    for a in range(3):
        n = len(ref.sigma[a])
        s = np.zeros(max(n, len(sig[a])))
        s[:len(sig[a])] = sig[a]
        # a relevant column keeps the (unrotated) components of up to D sub-floor columns
        big = ref.sigma[a] > 10 * irr
        tol_s = 1e-12 * ref.sigma[a][0] + math.sqrt(inf.D[a]) * irr
        assert np.all(np.abs(s[:n][big] - ref.sigma[a][big]) <= tol_s)
        tg, tr = O.tail_norms(s[:n]), O.tail_norms(ref.sigma[a])
        k = min(n, ref.ranks[a] + 2)
        assert np.all(np.abs(tg[:k] - tr[:k]) <= 1e-3 * thr + 1e-12 * ref.sigma[a][0])
        # ranks: equal unless the threshold sits within that margin of a tail value
        if inf.r[a] != ref.ranks[a]:
            kk = min(inf.r[a], ref.ranks[a])
            assert abs(tr[kk] - thr) <= 2e-3 * thr
    tile = r.tile()
    err = np.linalg.norm(tile - full)
    assert err <= inf.bound * (1 + 1e-9) + 1e-12 * nA
    assert err <= eps * nA * (1 + 1e-9) + 1e-12 * nA
    if tuple(inf.r) == ref.ranks:
        # same ranks: the two rank-r projections differ by the subspace angle left by the Jacobi
        # stopping rule (relative coupling <= 1e-12), amplified by sigma_1 / gap (Davis-Kahan)
        Tref = O.tucker_full(ref.core, ref.Z)
        assert np.max(np.abs(tile - Tref)) <= 1e-10 * np.max(np.abs(Tref))
    # the Tucker factors are orthonormal and the core is their projection of the canonical sum
    Z, core = r.tucker()
    for a in range(3):
        assert np.max(np.abs(Z[a] @ Z[a].T - np.eye(Z[a].shape[0]))) < 1e-11
    mu = np.einsum("ijk,ai,bj,ck->abc", full, *Z, optimize=True)
    assert np.max(np.abs(mu - core)) <= 1e-11 * np.max(np.abs(mu))
    # points: Tucker sampling equals the tile values, for points in any order that share
    # mode-3 cells (each distinct cell is contracted once) or repeat, and points outside the
    # grid along any axis are NaN
    rng = np.random.default_rng(1)
    pts = np.stack([rng.integers(0, n, 64) for n in p.N], axis=1)
    pts = np.concatenate([pts, pts[::7]])
    far = np.array([[0.0, 0.0, 1e3], [1e3, 0.0, 0.0], [0.0, -1e3, 0.0]])
    xyz = np.concatenate([cells_xyz(p, pts)[:40], far, cells_xyz(p, pts)[40:]])
    v = r.sample(xyz)
    assert np.all(np.isnan(v[40:43]))
    v = np.concatenate([v[:40], v[43:]])
    assert np.allclose(v, tile[pts[:, 0], pts[:, 1], pts[:, 2]], rtol=1e-12, atol=1e-12 * np.max(np.abs(tile)))
    r.release()


@pytest.mark.parametrize("prec", [W.FP32, W.BF16X3])
def test_rhosvd_mixed_precision_error(ctx, prec):
    p64 = _small_defected(eps=1e-6)
    pm = _small_defected(eps=1e-6, precision=prec)
    r64, rm = run(ctx, p64), run(ctx, pm)
    t64 = r64.tile()
    tm = rm.tile().astype(np.float64)
    assert tuple(r64.info().r) == tuple(rm.info().r)        # SVD and truncation stay FP64
    rel = np.max(np.abs(tm - t64)) / np.max(np.abs(t64))
    # Accumulation is chunked (16 FP32 terms, then FP64), so the error comes from rounding the
    # stored operands: Z, the projections, the core and the two tile intermediates, about six
    # roundings of 2^-24 each, amplified by the cancellation inside the Tucker sum
    # (sum |mu||Z||Z||Z| / |V|, about 5 here).  Split-BF16x3 products are good to about 2^-16.
    tol = 6 * 2.0 ** -24 * 5 * 2 if prec == W.FP32 else 1e-4
    assert rel < tol, rel
    # against the oracle's full tensor (the canonical sum on the whole grid): within the certified
    # truncation bound (Frobenius) plus the arithmetic error above (max norm, per cell)
    xi, A = O.canonical_terms(pm)
    full = O.cp_full(xi, A)
    inf = rm.info()
    assert np.max(np.abs(tm - full)) <= inf.bound * (1 + 1e-9) + tol * np.max(np.abs(full))
    # values at points: the mode-3 contraction in the request's precision (Z3 rows, the core and
    # its product rounded to the element type, FP64 sums across chunks), the rest FP64
    rng = np.random.default_rng(17)
    cells = np.stack([rng.integers(0, n, 300) for n in p64.N], axis=1)
    v64, vm = r64.sample(cells_xyz(p64, cells)), rm.sample(cells_xyz(pm, cells))
    assert np.max(np.abs(vm - v64)) / np.max(np.abs(v64)) < tol
    r64.release()
    rm.release()


@pytest.mark.parametrize("prec", [W.FP64, W.FP32, W.BF16X3])
def test_result_states_its_error_against_the_oracle(ctx, prec):
    # Every Tucker result reports its max-norm relative deviation at seeded probe cells from the
    # untruncated canonical sum (the discrete tensor the oracle's direct sum gives): the stated
    # number is the deviation measured against the oracle at those cells, it respects the
    # certified Frobenius bound, and it grows with the rounding of the precision
    p = _small_defected(eps=1e-6, precision=prec)
    r = run(ctx, p)
    inf, st = r.info(), r.stats()
    cells = np.array(st["probe_cells"])
    assert inf.n_probe == st["n_probe"] == len(cells) == 32
    ref = O.brute_force_points(p, cells)
    v = r.sample(cells_xyz(p, cells))
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(v - ref)) / scale
    # the library's canonical sum and the oracle's direct sum agree to ~1e-14 of the values
    assert abs(inf.probe_err - err) <= 1e-12, (inf.probe_err, err)
    assert inf.probe_err * scale <= inf.bound * (1 + 1e-9) + (0 if prec == W.FP64 else 1e-4 * scale)
    tol = {W.FP64: 1e-6, W.FP32: 1e-5, W.BF16X3: 1e-4}[prec]
    assert inf.probe_err < tol, inf.probe_err
    r.release()


@pytest.mark.parametrize("prec", [W.FP64, W.FP32, W.BF16X3])
def test_grouped_core_matches_oracle(ctx, prec):
    # 20 defects on the 5 x 4 x 4 lattice share at most 4 mode-3 planes: the terms of each mode-3
    # column are summed before the mode-3 contraction (D3 <= K / 2).  The core against the
    # oracle's projection of the full tensor onto the GPU's factors, and the tile against the
    # full tensor within the certified bound
    p = _small_defected(eps=1e-8, precision=prec, n_vac=12, n_imp=8)
    assert 2 * (len(p.blocks) + len({(d.block, d.site[2]) for d in p.defects})) <= len(p.blocks) + len(p.defects)
    r = run(ctx, p)
    inf = r.info()
    xi, A = O.canonical_terms(p)
    full = O.cp_full(xi, A)
    nA = np.linalg.norm(full)
    Z, core = r.tucker()
    mu = np.einsum("ijk,ai,bj,ck->abc", full, *Z, optimize=True)
    tile = r.tile().astype(np.float64)
    err = np.linalg.norm(tile - full)
    r.release()
    if prec == W.FP64:
        assert np.max(np.abs(mu - core)) <= 1e-11 * np.max(np.abs(mu))
        assert err <= inf.bound * (1 + 1e-9) + 1e-12 * nA
    else:
        # FP32 operands (projections, Z) and an FP32 core; BF16x3 products good to about 2^-16
        tol = 1e-5 if prec == W.FP32 else 1e-4
        assert np.max(np.abs(mu - core.astype(np.float64))) <= tol * np.max(np.abs(mu))
        assert err <= inf.bound * (1 + 1e-9) + tol * nA


def test_concurrent_requests_equal_alone(ctx):
    import paper_1411_1994_amd as L
    probs = [_small_defected(kind=k, param=pp, eps=e, seed=s, tile=False)
             for (k, pp, e, s) in [(0, 0.0, 1e-6, 1), (1, 0.5, 1e-4, 2), (2, 1.0, 1e-6, 3), (0, 0.0, 1e-8, 4)]]
    pts = np.array([[0.1, 0.2, 0.3], [1.0, -2.0, 0.5], [3.0, 3.0, -3.0]])
    alone = []
    for p in probs:
        r = run(ctx, p)
        alone.append(r.sample(pts))
        r.release()
    reqs = [ctx.submit(p) for p in probs * 3]
    for i, r in enumerate(reqs):
        assert r.wait() == 0
        assert np.array_equal(r.sample(pts), alone[i % len(probs)])   # bitwise: batch-invariant kernels
        r.release()


def test_invalid_problems_are_rejected(ctx):
    import paper_1411_1994_amd as L
    good = W.Problem("bad", W.NEWTON, 0.0, 10, (21, 21, 21), 0.5, [W.cubic_block(2)])
    cases = [
        (dict(N=(20, 21, 21)), -1),
        (dict(M=0), -1),
        (dict(kind=9), -1),
        (dict(blocks=[W.cubic_block(40)]), -2),
        (dict(defects=[W.Defect(0, (0, 0, 0), -1.0), W.Defect(0, (0, 0, 0), 0.5)]), -3),
        (dict(defects=[W.Defect(0, (2, 0, 0), -1.0)]), -2),
        (dict(eps=1e-6, tile_lo=(0, 0, 10), tile_T=(21, 21, 21)), -1),
    ]
    for change, code in cases:
        q = W.Problem(**{**good.__dict__, **change})
        with pytest.raises(L.LsumError) as e:
            ctx.submit(q)
        assert e.value.code == code, (change, e.value)
    # a budget that can never hold the request
    small = L.Context(0, hbm_budget_bytes=1 << 20, n_slots=1)
    with pytest.raises(L.LsumError) as e:
        small.submit(good)
    assert e.value.code == -4
    small.close()


def _medium_defected(seed=11, eps=1e-2):
    # side matrices with min(D, N) above 512: D = R * (1 + distinct defect cells per axis); the
    # loose eps keeps the certified ranks well under the 256-vector range basis
    # (assert max(range_k) > 0 below)
    rng = np.random.default_rng(seed)
    blocks = [W.Block((24, 24, 24), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))]
    defects = W.draw_defects(rng, blocks, 40, 30)
    return W.Problem("med", W.NEWTON, 0.0, 24, (601, 601, 601), 1.0 / 15, blocks, defects, eps=eps)


def _large_defected(seed=12, eps=1e-2):
    # D ~ 900-990 distinct columns, N = 1025, certified ranks 344-366 (oracle): above one block
    # of 256 basis vectors and below min(D, N) / 2, so the range basis grows over two blocks
    rng = np.random.default_rng(seed)
    blocks = [W.Block((40, 40, 40), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))]
    defects = W.draw_defects(rng, blocks, 60, 30)
    return W.Problem("large", W.NEWTON, 0.0, 24, (1025, 1025, 1025), 56.0 / 1024, blocks, defects, eps=eps)


@pytest.mark.parametrize("problem", ["medium", "large"])
def test_range_basis_svd_matches_direct_jacobi(problem):
    # the randomized range basis (large side matrices) against the plain one-sided Jacobi on the
    # same request: same leading singular values, certified bounds, orthonormal factors, and
    # potentials that agree with each other and with the oracle's direct sum
    require_gpu()
    import paper_1411_1994_amd as L
    p = _medium_defected() if problem == "medium" else _large_defected()
    out = {}
    for name, rmin in (("range", 512), ("direct", 0)):
        with L.Context(0, n_slots=1) as c:
            c.set_option(L.OPT_RANGE_MIN, rmin)
            r = c.submit(p)
            assert r.wait() == 0, r.stats()
            inf, st = r.info(), r.stats()
            rng = np.random.default_rng(4)
            cells = np.stack([rng.integers(0, n, 24) for n in p.N], axis=1)
            Z, _ = r.tucker()
            out[name] = dict(inf=inf, st=st, sig=r.sigma(), Z=Z, v=r.sample(cells_xyz(p, cells)), cells=cells)
            r.release()
    a, b = out["range"], out["direct"]
    assert max(a["st"]["range_k"]) > 0 and max(b["st"]["range_k"]) == 0, (a["st"]["range_k"], a["inf"].r, a["inf"].D)
    if problem == "large":
        assert min(a["st"]["range_k"]) > 256 and min(b["inf"].r) > 256, (a["st"]["range_k"], b["inf"].r)
    nA = a["inf"].norm_A
    thr = p.eps * nA / (3 * a["inf"].norm_xi)
    for o in (a, b):
        assert o["inf"].bound <= p.eps * nA * (1 + 1e-12)
        for l in range(3):
            assert np.max(np.abs(o["Z"][l] @ o["Z"][l].T - np.eye(o["Z"][l].shape[0]))) < 1e-11
    for l in range(3):
        res = a["st"]["range_res"][l]
        assert res <= 0.1 * thr
        if a["st"]["range_k"][l] == 0:       # this mode took the direct solve
            assert a["inf"].r[l] == b["inf"].r[l]
            continue
        # the basis keeps the leading values; a few more vectors can be needed to absorb res
        assert b["inf"].r[l] <= a["inf"].r[l] <= b["inf"].r[l] + max(3, b["inf"].r[l] // 50)
        sa, sb = a["sig"][l], b["sig"][l]
        big = sb[:len(sa)] > 10 * thr
        assert np.all(np.abs(sa[big] - sb[:len(sa)][big]) <= 1e-10 * sb[0] + res)
    # pointwise errors are bounded by the certified Frobenius error eps * ||A||
    ref = O.brute_force_points(p, a["cells"])
    assert np.max(np.abs(a["v"] - ref)) <= p.eps * nA
    assert np.max(np.abs(b["v"] - ref)) <= p.eps * nA


def test_jacobi_rank_stop_matches_full_convergence():
    # the Jacobi stop rule (end once the certified rank repeats and the kept rows are orthogonal)
    # against sweeping to full convergence, on the direct solve of the same request: certified
    # bounds, orthonormal factors, the same leading singular values, ranks within a few, and
    # potentials that agree with the oracle's direct sum
    require_gpu()
    import paper_1411_1994_amd as L
    p = _medium_defected(eps=1e-4)
    out = {}
    for stop in (1, 0):
        with L.Context(0, n_slots=1) as c:
            c.set_option(L.OPT_RANGE_MIN, 0)
            c.set_option(L.OPT_JACOBI_STOP, stop)
            r = c.submit(p)
            assert r.wait() == 0, r.stats()
            rng = np.random.default_rng(5)
            cells = np.stack([rng.integers(0, n, 24) for n in p.N], axis=1)
            Z, _ = r.tucker()
            out[stop] = dict(inf=r.info(), st=r.stats(), sig=r.sigma(), Z=Z, v=r.sample(cells_xyz(p, cells)),
                             cells=cells)
            r.release()
    a, b = out[1], out[0]
    nA = b["inf"].norm_A
    thr = p.eps * nA / (3 * b["inf"].norm_xi)
    for o in (a, b):
        assert o["inf"].bound <= p.eps * nA * (1 + 1e-12)
        for l in range(3):
            assert np.max(np.abs(o["Z"][l] @ o["Z"][l].T - np.eye(o["Z"][l].shape[0]))) < 1e-11
    for l in range(3):
        assert a["st"]["sweeps"][l] <= b["st"]["sweeps"][l]
        # column norms in any sweep give tails that bound the converged ones from above
        assert b["inf"].r[l] <= a["inf"].r[l] <= b["inf"].r[l] + max(3, b["inf"].r[l] // 50)
        # the kept rows are orthogonal among themselves; what they still share with the tail rows
        # (at most the tail energy, <= thr^2) moves their norms by far less than thr
        sa, sb = a["sig"][l], b["sig"][l]
        big = sb > 10 * thr
        assert np.all(np.abs(sa[big] - sb[big]) <= 1e-10 * sb[0] + thr)
    ref = O.brute_force_points(p, a["cells"])
    for o in (a, b):
        assert np.max(np.abs(o["v"] - ref)) <= p.eps * nA


@pytest.mark.parametrize("L,N,src", [((4, 4, 4), (65, 65, 65), [0, 0, 0]),
                                     ((4, 4, 5), (65, 65, 67), [0, 0, 2]),
                                     ((3, 4, 3), (65, 65, 65), [0, 1, 0])])
def test_identical_axes_share_factors(ctx, L, N, src):
    # axes with the same cell count and snapped sites are summed once and shared; every axis's
    # factors still equal the oracle's assembled sums
    blocks = [W.Block(L, (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))]
    p = W.Problem("ax", W.NEWTON, 0.0, 20, N, 0.25, blocks)
    r = run(ctx, p)
    assert r.stats()["axis_src"] == src
    got = r.canonical(0)
    ref = O.assembled_canonical(p)[0]
    for a in range(3):
        assert np.max(np.abs(got[a] - ref[a])) <= 1e-13 * np.max(np.abs(ref[a]))
    r.release()


@pytest.mark.parametrize("kind,param,eps", [(W.NEWTON, 0.0, 1e-7), (W.YUKAWA, 0.5, 1e-6)])
def test_chosen_M_meets_its_tolerance_end_to_end(ctx, kind, param, eps):
    # Sec. 2.1 error control: M from the library's search; the potential of one unit charge
    # computed by the device path (collocation, shift-sum, sampling) against the exact
    # Galerkin entries of the oracle, in the max norm, at cells that are not probe cells
    import paper_1411_1994_amd as L
    N, h, hu = (257, 129, 129), 1 / 16, 0.25
    M, e = L.lsum_choose_M(kind, param, N, h, eps, 128, h_u=hu)
    assert e <= eps
    p = W.Problem("one-charge", kind, param, M, N, h, [W.Block((1, 1, 1), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))],
                  h_u=hu)
    rng = np.random.default_rng(W.SEED_BASE + 31)
    c = np.array([(n - 1) // 2 for n in N])
    near = np.array([[i, j, k] for i in range(-3, 4) for j in range(-3, 4) for k in range(-3, 4)]) + c
    far = np.stack([rng.integers(0, n, 400) for n in N], axis=1)
    pts = np.concatenate([near, far, [[0, 0, 0], [N[0] - 1, N[1] - 1, N[2] - 1]]])
    r = run(ctx, p)
    got = r.sample(cells_xyz(p, pts))
    r.release()
    exact = O.exact_cell_averages(kind, param, np.abs(pts - c), h)
    err = np.max(np.abs(got - exact)) / np.max(exact)
    assert err <= 1.05 * eps, (M, e, err)
    # the error at these cells is of the size the probes estimate (its peak, the charge's own
    # cell, is among them)
    assert err >= 0.5 * e


@pytest.mark.parametrize("sweeps", [1, 3])
def test_als_after_rhosvd_matches_oracle(ctx, sweeps):
    # Thm thm:C2Tucker (b): ALS sweeps from the RHOSVD factors, against the oracle's sweeps from
    # its own RHOSVD of the same terms: same ||core|| after every sweep and the same values
    rng = np.random.default_rng(71)
    big = W.Block((6, 5, 4), (1.0, 1.1, 0.9), (0.13, -0.2, 0.07))
    defects = W.draw_defects(rng, [big], 6, 4)
    p = W.Problem("als", W.NEWTON, 0.0, 24, (61, 67, 55), 0.21, [big], defects, eps=1e-3,
                  als_sweeps=sweeps)
    r = run(ctx, p)
    st = r.stats()
    xi, A = O.canonical_terms(p)
    res = O.rhosvd(xi, A, eps=1e-3)
    Z, core, hist = O.als_refine(xi, A, res.Z, sweeps)
    assert tuple(r.info().r) == res.ranks and st["als_skipped"] == 0
    assert np.allclose(st["als_core_norm"], hist, rtol=1e-10, atol=0)
    pts = np.stack([rng.integers(0, n, 300) for n in p.N], axis=1)
    got = r.sample(cells_xyz(p, pts))
    r.release()
    want = O.tucker_points(core, Z, pts)
    assert np.max(np.abs(got - want)) <= 1e-9 * np.max(np.abs(want))
    # never worse than the RHOSVD guess against the plain sum
    ref = O.brute_force_points(p, pts)
    rh = O.tucker_points(res.core, res.Z, pts)
    assert np.linalg.norm(got - ref) <= np.linalg.norm(rh - ref) * 1.01


def test_als_is_skipped_when_the_ranks_do_not_allow_it(ctx):
    # r_a r_b > 4096 for some pair of modes: the RHOSVD result stands and the skip is reported
    p = W.Problem("als-big", W.NEWTON, 0.0, 28, (129, 129, 129), 3 / 32,
                  [W.Block((8, 8, 8), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))],
                  W.draw_defects(np.random.default_rng(72), [W.Block((8, 8, 8), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))], 120, 40),
                  eps=1e-10, als_sweeps=2)
    r = run(ctx, p)
    st = r.stats()
    rr = r.info().r
    r.release()
    if max(rr[0] * rr[1], rr[0] * rr[2], rr[1] * rr[2]) > 4096:
        assert st["als_skipped"] == 1 and st["als_core_norm"] == []
    else:
        assert st["als_skipped"] == 0 and len(st["als_core_norm"]) == 2


@pytest.mark.parametrize("eps2", [0.0, 1e-4])
def test_tucker_to_canonical_matches_oracle(ctx, eps2):
    # Can -> Tuck -> Can: the canonical form of the device's Tucker result against the oracle's
    # conversion of the same Tucker tensor (same rank and weights; values at points)
    rng = np.random.default_rng(73)
    big = W.Block((5, 4, 4), (1.0, 1.1, 0.9), (0.13, -0.2, 0.07))
    p = W.Problem("c2t2c", W.NEWTON, 0.0, 24, (49, 45, 41), 0.25, [big], W.draw_defects(rng, [big], 5, 3),
                  eps=1e-3)
    r = run(ctx, p)
    Z, core = r.tucker()
    xi, U, err = r.tucker_to_canonical(eps2)
    xo, Ao, erro = O.tucker_to_canonical(core, [z.T for z in Z], eps2)
    assert len(xi) == len(xo) and abs(err - erro) <= 1e-9 * np.linalg.norm(core)
    assert np.allclose(xi, xo, rtol=1e-9, atol=1e-12 * xo[0])
    pts = np.stack([rng.integers(0, n, 200) for n in p.N], axis=1)
    got = O.canonical_eval([u for u in U], pts, xi)
    want = O.tucker_points(core, [z.T for z in Z], pts)
    assert np.max(np.abs(got - want)) <= 1e-9 * np.max(np.abs(want)) + 2 * erro
    r.release()


@pytest.mark.parametrize("eps", [0.0, 1e-6])
def test_parallelogram_lattice(ctx, eps):
    # case (B): x moves by 0.45 per step along y; the library's block decomposition, summed on the
    # canonical route (and reduced by RHOSVD), against the plain sum over the sheared sites
    import paper_1411_1994_amd as L
    base = W.Block((6, 5, 4), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))
    blocks = [W.Block(b.L, b.b, b.center, b.charge) for b in L.lsum_shear_blocks(base, 0, 1, 0.45)]
    p = W.Problem("shear", W.NEWTON, 0.0, 28, (81, 65, 57), 0.25, blocks, eps=eps)
    r = run(ctx, p)
    rng = np.random.default_rng(81)
    pts = np.stack([rng.integers(0, n, 300) for n in p.N], axis=1)
    got = r.sample(cells_xyz(p, pts))
    inf = r.info()
    r.release()
    pos = O.shear_sites(base, 0, 1, 0.45)
    ref = O.brute_force_points_at(p, pts, pos, np.ones(len(pos)))
    tol = 1e-12 if eps == 0.0 else 10 * eps
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))
    # axis 2 is the same in every sub-block: one lattice source there, one per sub-block on axis 1
    if eps > 0:
        assert inf.D[2] == inf.R and inf.D[1] == inf.R * base.L[1]


def test_vacancy_clusters_as_one_non_equidistant_block(ctx):
    # case (D): vacancy clusters of 2 x 2 x 2 sites on a 3 x 3 x 2 coarse lattice inside an
    # 8 x 8 x 6 lattice, as one block of charge -1 with explicit coordinates
    lat = W.Block((8, 8, 6), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))
    sites = [O.site_coords(lat.L[a], 1.0, 0.0) for a in range(3)]
    pick = [np.array([0, 1, 3, 4, 6, 7]), np.array([1, 2, 4, 5, 6, 7]), np.array([0, 1, 3, 4])]
    coords = tuple(sites[a][pick[a]] for a in range(3))
    vac = W.Block(tuple(len(c) for c in coords), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0), charge=-1.0, coords=coords)
    for eps in (0.0, 1e-6):
        p = W.Problem("clusters", W.NEWTON, 0.0, 28, (65, 65, 57), 0.25, [lat, vac], eps=eps)
        r = run(ctx, p)
        rng = np.random.default_rng(82)
        pts = np.stack([rng.integers(0, n, 300) for n in p.N], axis=1)
        got = r.sample(cells_xyz(p, pts))
        r.release()
        pos, Z = O.charge_positions(p)
        ref = O.brute_force_points_at(p, pts, pos, Z)
        tol = 1e-12 if eps == 0.0 else 10 * eps
        assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))


@pytest.mark.parametrize("lattice", [False, True])
def test_galerkin_matrix_matches_oracle(ctx, lattice):
    # eq. nuc_pot on the device's own Tucker result against the oracle's sum over its full tensor
    alpha = np.array([1.0, 2.0, 1.5, 0.8])
    A = np.array([[0.3, -0.2, 0.1], [-0.4, 0.5, 0.0], [0.0, 0.0, 0.6], [0.5, 0.5, -0.5]])
    N, h = (49, 45, 41), 1 / 6
    blk = W.Block((3, 2, 2), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0)) if lattice else W.Block((1, 1, 1), (1, 1, 1), (0, 0, 0))
    p = W.Problem("galerkin", W.NEWTON, 0.0, 32, N, h, [blk], eps=1e-9)
    r = run(ctx, p)
    x = [(np.arange(n) - (n - 1) // 2) * h for n in N]
    G = [np.exp(-alpha[:, None] * (x[l][None, :] - A[:, l][:, None]) ** 2) for l in range(3)]
    V = r.galerkin(G)
    Z, core = r.tucker()
    r.release()
    Vo = O.galerkin_matrix(O.tucker_full(core, [z.T for z in Z]), G, h)
    assert np.max(np.abs(V - Vo)) <= 1e-10 * np.max(np.abs(Vo))
    assert np.max(np.abs(V - V.T)) <= 1e-12 * np.max(np.abs(V))


def test_column_lattice(ctx):
    # case (C): columns of 6 sites along z at 20 scattered (x, y) points; canonical route against
    # the plain sum over the explicit sites
    import paper_1411_1994_amd as L
    rng = np.random.default_rng(83)
    base = W.Block((1, 1, 6), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))
    xy = rng.uniform(-5.0, 5.0, (20, 2))
    blocks = [W.Block(b.L, b.b, b.center, b.charge) for b in L.lsum_column_blocks(base, 2, xy)]
    p = W.Problem("columns", W.NEWTON, 0.0, 28, (65, 65, 41), 0.25, blocks)
    r = run(ctx, p)
    pts = np.stack([rng.integers(0, n, 300) for n in p.N], axis=1)
    got = r.sample(cells_xyz(p, pts))
    r.release()
    pos, Z = O.charge_positions(p)
    ref = O.brute_force_points_at(p, pts, pos, Z)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_galerkin_and_canonical_form_with_device_buffers(ctx):
    # the on_device variants read the basis from and write the results to device memory; they
    # equal the host variants bit for bit
    import ctypes
    import paper_1411_1994_amd as L
    from gpu_util import dev, host
    alpha = np.array([1.0, 2.0, 1.5])
    A = np.array([[0.3, -0.2, 0.1], [-0.4, 0.5, 0.0], [0.0, 0.0, 0.6]])
    N, h = (49, 45, 41), 1 / 6
    p = W.Problem("dev", W.NEWTON, 0.0, 32, N, h, [W.Block((3, 2, 2), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))],
                  eps=1e-6)
    r = run(ctx, p)
    x = [(np.arange(n) - (n - 1) // 2) * h for n in N]
    G = [np.exp(-alpha[:, None] * (x[l][None, :] - A[:, l][:, None]) ** 2) for l in range(3)]
    Vh = r.galerkin(G)
    Gd = [dev(g) for g in G]
    Vd = dev(np.zeros((3, 3)))
    rc = L._lib.lsum_galerkin(r.handle, 3, Gd[0].data_ptr(), Gd[1].data_ptr(), Gd[2].data_ptr(),
                              Vd.data_ptr(), 1)
    assert rc == 0 and np.array_equal(host(Vd), Vh)
    xi, U, err = r.tucker_to_canonical(1e-8)
    R = len(xi)
    xd = dev(np.zeros(R))
    Ud = [dev(np.zeros((R, n))) for n in N]
    Rc, ec = ctypes.c_int(0), ctypes.c_double(0.0)
    rc = L._lib.lsum_tucker_to_canonical(r.handle, 1e-8, R, ctypes.byref(Rc),
                                         ctypes.cast(xd.data_ptr(), ctypes.POINTER(ctypes.c_double)),
                                         *[ctypes.cast(u.data_ptr(), ctypes.POINTER(ctypes.c_double)) for u in Ud],
                                         ctypes.byref(ec), 1)
    r.release()
    assert rc == 0 and Rc.value == R and ec.value == err
    assert np.array_equal(host(xd), xi) and all(np.array_equal(host(Ud[l]), U[l]) for l in range(3))


@pytest.mark.parametrize("prec", [W.FP64, W.FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_grouped_core_in_each_mode_matches_direct_sum(ctx, axis, prec):
    # vacancies and impurities on one lattice plane across `axis`: that axis has the fewest
    # distinct defect columns (D = 2 R), so the core sums the terms sharing its columns first and
    # contracts over them (mode 3: one product over rows of the core; mode 1: over columns; mode
    # 2: one product per core slice); each placement against the oracle's direct sum
    rng = np.random.default_rng(40 + axis)
    blk = W.Block((4, 4, 4), (1.0, 1.0, 1.0), (0.1, -0.15, 0.05))
    sites = rng.choice(16, 10, replace=False)
    defects = []
    for k, f in enumerate(sites):
        s = [int(f // 4), int(f % 4)]
        s.insert(axis, 1)
        defects.append(W.Defect(0, tuple(s), -1.0 if k < 6 else 0.5))
    p = W.Problem("plane", W.NEWTON, 0.0, 20, (33, 35, 31), 0.37, [blk], defects, eps=1e-6, precision=prec)
    r = run(ctx, p)
    st = r.stats()
    assert st["core_mode"] == axis, st["core_mode"]
    inf = r.info()
    pts = np.stack([rng.integers(0, n, 200) for n in p.N], axis=1)
    got = r.sample(cells_xyz(p, pts))
    ref = O.brute_force_points(p, pts)
    slack = 1e-12 if prec == W.FP64 else 1e-5
    assert np.max(np.abs(got - ref)) <= inf.bound * (1 + 1e-9) + slack * np.max(np.abs(ref))
    r.release()


@pytest.mark.parametrize("prec", [W.FP64, W.FP32], ids=["fp64", "fp32"])
def test_own_gemm_kernels_match_the_library_path(prec):
    # the medium defected request (range bases, projections and core) with every product on the
    # library's own MFMA kernels and with the large FP64 ones on the ROCm BLAS DGEMM (the range
    # basis is FP64 at either precision): the same certified ranks, bounds within rounding, and
    # values within 1e-10 (FP64) or 2e-6 (FP32) of each other and within the bound of the
    # oracle's direct sum (FP32: plus 1e-5 of the largest value)
    require_gpu()
    import paper_1411_1994_amd as L
    p = _medium_defected(eps=1e-4)
    p.precision = prec
    rng = np.random.default_rng(8)
    cells = np.stack([rng.integers(0, n, 24) for n in p.N], axis=1)
    out = {}
    try:
        for lib in (0, 1):
            with L.Context(0, n_slots=1) as c:
                c.set_option(L.OPT_GEMM_LIBRARY, lib)
                r = c.submit(p)
                assert r.wait() == 0, r.stats()
                out[lib] = (r.info(), r.sample(cells_xyz(p, cells)))
                r.release()
    finally:
        with L.Context(0, n_slots=1) as c:
            c.set_option(L.OPT_GEMM_LIBRARY, 1)
    (ia, va), (ib, vb) = out[0], out[1]
    assert tuple(ia.r) == tuple(ib.r)
    assert abs(ia.bound - ib.bound) <= 1e-9 * ib.bound
    scale = np.max(np.abs(vb))
    assert np.max(np.abs(va - vb)) <= (1e-10 if prec == W.FP64 else 2e-6) * scale
    ref = O.brute_force_points(p, cells)
    slack = 1e-12 if prec == W.FP64 else 1e-5
    for v in (va, vb):
        assert np.max(np.abs(v - ref)) <= ib.bound * (1 + 1e-9) + slack * np.max(np.abs(ref))

"""Exact sites: lattices whose sites are not on cell centres, summed without snapping, against
the oracle's charge-by-charge sum at the exact positions."""
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


def points(p, n, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.integers(0, N, n) for N in p.N], axis=1)


def run(ctx, p):
    r = ctx.submit(p)
    rc = r.wait()
    assert rc == 0, r.stats()
    return r


def rel_err(got, ref):
    return np.max(np.abs(got - ref)) / np.max(np.abs(ref))


# b/h = 22/5 on axis 0 (5 classes), 13/4 on axis 1 (4), b/h = 3.6548 on axis 2 (every site its
# own class), sub-cell centres everywhere
H = 0.25
BIG = W.Block((6, 5, 4), (1.1, 0.8125, 0.9137), (0.071, -0.113, 0.029))
SECOND = W.Block((3, 3, 2), (0.55, 1.0, 0.6), (-1.53, 4.41, 3.12), charge=0.5)


@pytest.mark.parametrize("kind,param", [(W.NEWTON, 0.0), (W.YUKAWA, 0.5), (W.SLATER, 1.0)])
def test_canonical_exact_sites(ctx, kind, param):
    p = W.Problem("off", kind, param, 28, (61, 67, 55), H, [BIG, SECOND], exact_sites=True)
    r = run(ctx, p)
    pts = points(p, 400, 41 + kind)
    got = r.sample(cells_xyz(p, pts))
    r.release()
    ref = O.brute_force_points_exact(p, pts)
    assert rel_err(got, ref) <= 1e-12
    # the snapped sum differs at the O(h) level, so the comparison above is not vacuous
    assert rel_err(O.brute_force_points(p, pts), ref) > 1e-4


def test_exact_sites_with_defects(ctx):
    rng = np.random.default_rng(43)
    defects = W.draw_defects(rng, [BIG, SECOND], 7, 5)
    p = W.Problem("off-def", W.NEWTON, 0.0, 28, (61, 67, 55), H, [BIG, SECOND], defects, exact_sites=True)
    r = run(ctx, p)
    pts = points(p, 400, 44)
    got = r.sample(cells_xyz(p, pts))
    r.release()
    assert rel_err(got, O.brute_force_points_exact(p, pts)) <= 1e-12


@pytest.mark.parametrize("eps", [1e-5, 1e-8])
def test_exact_sites_rhosvd(ctx, eps):
    # Tucker output: certified relative Frobenius bound; pointwise within a few eps of the
    # maximum on these positive-dominated sums
    rng = np.random.default_rng(45)
    defects = W.draw_defects(rng, [BIG, SECOND], 7, 5)
    p = W.Problem("off-tucker", W.NEWTON, 0.0, 28, (61, 67, 55), H, [BIG, SECOND], defects, eps=eps,
                  exact_sites=True)
    r = run(ctx, p)
    info = r.info()
    assert info.rel_bound <= eps
    pts = points(p, 400, 46)
    got = r.sample(cells_xyz(p, pts))
    r.release()
    assert rel_err(got, O.brute_force_points_exact(p, pts)) <= 10 * eps


def test_exact_sites_large_lattice_uses_combs(ctx):
    # 24^3 sites with b/h = 5/2: two classes per axis, each a comb of stride 5 (window sums of the
    # class rows), against the charge-by-charge sum at sampled cells
    blk = W.Block((24, 24, 24), (0.625, 0.625, 0.625), (0.0, 0.0, 0.0))
    p = W.Problem("off-comb", W.NEWTON, 0.0, 32, (129, 129, 129), H, [blk], exact_sites=True)
    r = run(ctx, p)
    pts = points(p, 60, 47)
    got = r.sample(cells_xyz(p, pts))
    r.release()
    assert rel_err(got, O.brute_force_points_exact(p, pts)) <= 1e-12


def test_exact_sites_fp32_rows(ctx):
    # FP32 rows: every term within 3 roundings of its FP64 value (positive charges and kernel)
    p = W.Problem("off-f32", W.NEWTON, 0.0, 28, (61, 67, 55), H, [BIG, SECOND], precision=W.FP32,
                  exact_sites=True)
    r = run(ctx, p)
    pts = points(p, 300, 48)
    got = r.sample(cells_xyz(p, pts))
    r.release()
    ref = O.brute_force_points_exact(p, pts)
    assert np.all(np.abs(got - ref) <= 3.01 * 2.0 ** -24 * np.abs(ref) + 1e-13 * np.max(ref))


def test_exact_sites_on_centres_equal_snapped_results(ctx):
    # sites on cell centres: exact_sites takes the snapped path and gives the same bits
    blk = W.Block((5, 4, 3), (0.5, 1.0, 0.5), (0.25, 0.0, -0.5))
    base = W.Problem("on", W.NEWTON, 0.0, 28, (41, 41, 41), H, [blk])
    exact = W.Problem("on-x", W.NEWTON, 0.0, 28, (41, 41, 41), H, [blk], exact_sites=True)
    pts = points(base, 200, 49)
    r0, r1 = run(ctx, base), run(ctx, exact)
    a, b = r0.sample(cells_xyz(base, pts)), r1.sample(cells_xyz(base, pts))
    r0.release()
    r1.release()
    assert np.array_equal(a, b)


def test_mixed_batch_of_exact_and_snapped_requests(ctx):
    # one batch holding off-grid and on-grid requests: each equals its own single run
    probs = [W.Problem("mix%d" % k, W.NEWTON, 0.0, 28, (61, 67, 55), H, [BIG, SECOND], exact_sites=bool(k % 2))
             for k in range(4)]
    pts = points(probs[0], 200, 50)
    xyz = cells_xyz(probs[0], pts)
    rs = ctx.submit_many(probs)
    for r in rs:
        assert r.wait() == 0
    got = [r.sample(xyz) for r in rs]
    for r in rs:
        r.release()
    for k, p in enumerate(probs):
        ref = O.brute_force_points_exact(p, pts) if p.exact_sites else O.brute_force_points(p, pts)
        assert rel_err(got[k], ref) <= 1e-12
    assert np.array_equal(got[0], got[2]) and np.array_equal(got[1], got[3])


def test_exact_sites_table_cache_switch_gives_identical_results():
    # class rows and window sums from the context's row cache (shared by repeated problems) or
    # built for each request (cache disabled): the same bits
    require_gpu()
    import paper_1411_1994_amd as L
    rng = np.random.default_rng(51)
    defects = W.draw_defects(rng, [BIG, SECOND], 3, 2)
    p = W.Problem("cache", W.NEWTON, 0.0, 28, (61, 67, 55), H, [BIG, SECOND], defects, exact_sites=True)
    xyz = cells_xyz(p, points(p, 200, 52))
    got = []
    for cap in (None, 0):
        with L.Context(0) as c:
            if cap is not None:
                c.set_option(L.OPT_REF_CACHE_BYTES, cap)
            rs = [c.submit(p) for _ in range(3)]
            for r in rs:
                assert r.wait() == 0
            got += [r.sample(xyz) for r in rs]
            for r in rs:
                r.release()
    for g in got[1:]:
        assert np.array_equal(g, got[0])

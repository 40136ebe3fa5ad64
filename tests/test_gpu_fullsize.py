"""Parity at the benchmark's full sizes, in the launch configuration the bench times, on outputs
the oracle computes one by one (direct sums over all lattice charges at sampled points)."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import dev, empty, host, require_gpu

pytestmark = pytest.mark.gpu


def test_newton_64cubed_served_batch_matches_direct_sum():
    # 64^3 Newton lattice on the 4097 grid, 1e5 points per request, one batch of 32 requests with
    # FP32 factor rows (the served policy) on 4 slots, submitted and finished as one set; a request
    # with FP64 rows beside it.  At sampled points both match the oracle's direct sum over all
    # 262,144 charges: FP32 rows within 1e-6 relative (<= 3 roundings of 2^-24 per term of a sum
    # of positive terms), FP64 rows within 1e-12.
    require_gpu()
    import torch
    import paper_1411_1994_amd as L
    p64 = W.config(2)
    p32 = W.Problem(**{**p64.__dict__, "precision": W.FP32})
    n = 100_000
    xs = [W.sample_points(2, n, W.half_widths(p64)) if i == 0 else
          np.random.default_rng(900 + i).uniform(-1, 1, size=(n, 3)) * np.array(W.half_widths(p64))
          for i in range(4)]
    with L.Context(0, n_slots=4) as c:
        c.set_option(L.OPT_MAX_BATCH, 32)
        xd = [dev(x) for x in xs]
        outs = [empty(n, torch.float64) for _ in range(32)]
        prep = L.prepare(p32)
        reqs = c.submit_many([prep] * 32, points=[xd[i % 4] for i in range(32)], values=outs)
        res = L.finish_many(reqs)
        assert all(rc == 0 for rc, _ in res)
        r64 = c.submit(p64, points=xd[0], values=empty(n, torch.float64))
        assert r64.wait() == 0
        v64 = host(r64.values)
        r64.release()
    rng = np.random.default_rng(17)
    for i in (0, 1, 2, 3, 31):
        x = xs[i % 4]
        sel = rng.choice(n, 24 if i == 0 else 8, replace=False)   # direct sums: ~0.2 s per point
        ref = O.brute_force_points(p64, O.points_to_cells(x[sel], p64.h, p64.N))
        got = host(outs[i])[sel]
        assert np.max(np.abs(got - ref) / np.abs(ref)) <= 1e-6
        if i == 0:
            assert np.max(np.abs(v64[sel] - ref) / np.abs(ref)) <= 1e-12
    # every request of the batch gave the same values for the same points (batch invariance)
    for i in range(4, 32):
        assert np.array_equal(host(outs[i]), host(outs[i % 4]))


def test_defected_48cubed_rhosvd_full_size_matches_direct_sum():
    # the defected 48^3 Newton lattice (300 vacancies, 100 impurities) on the 2049 grid, reduced
    # at eps = 1e-6 with the FP32 core, sampled at the bench's 4096 points: within 1e-6 of the
    # largest value against the oracle's direct sum at sampled points, and the certified bound
    require_gpu()
    import paper_1411_1994_amd as L
    p = W.config(3)
    x = W.sample_points(3, 4096, W.half_widths(p))
    with L.Context(0) as c:
        r = c.submit(p, points=x)
        assert r.wait() == 0
        inf = r.info()
        v = r.values.copy()
        r.release()
    assert inf.is_tucker == 1 and inf.rel_bound <= p.eps * (1 + 1e-9)
    sel = np.random.default_rng(5).choice(len(x), 24, replace=False)
    ref = O.brute_force_points(p, O.points_to_cells(x[sel], p.h, p.N))
    assert np.max(np.abs(v[sel] - ref)) <= 1e-6 * np.max(np.abs(ref))


@pytest.mark.parametrize("L", [(1, 1, 1), (1, 1, 7), (1, 5, 3), (9, 1, 1)])
def test_degenerate_lattices_match_direct_sum(L):
    # single sites, lines and planes of charges: combs of one site, axes with a single offset
    require_gpu()
    import paper_1411_1994_amd as Lib
    blk = W.Block(L, (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))
    p = W.Problem("deg", W.NEWTON, 0.0, 24, (81, 83, 85), 0.2, [blk])
    rng = np.random.default_rng(sum(L))
    cells = np.stack([rng.integers(0, n, 200) for n in p.N], axis=1)
    xyz = np.stack([(cells[:, a] - (p.N[a] - 1) // 2) * p.h for a in range(3)], axis=1)
    with Lib.Context(0) as c:
        r = c.submit(p, points=xyz)
        assert r.wait() == 0
        v = r.values.copy()
        r.release()
    ref = O.brute_force_points(p, cells)
    assert np.max(np.abs(v - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("prec,tol", [(W.FP32, 1e-5), (W.BF16X3, 1e-4)])
def test_yukawa_step_lattice_512_tile_matches_direct_sum(prec, tol):
    # The Yukawa (kappa = 0.5) step lattice of three blocks (40x40x20, 40x20x20, 20x20x20; 56,000
    # sites) with 500 vacancies on the 2049 grid, reduced at eps = 1e-5 and reconstructed on the
    # centred 512^3 tile by three mode products (eq. Tucker_singePot), in FP32 and in split
    # BF16x3, as the bench runs it.  At 160 seeded tile cells and 24 of the 4096 sample points the
    # values are within tol of the oracle's direct sum over all 55,500 charges (relative to the
    # largest of those values): tol = eps (the certified Frobenius-relative truncation) for FP32,
    # whose rounding of Z, core and the two tile intermediates stays a few 1e-6; 1e-4 for BF16x3,
    # whose products are good to about 2^-16 amplified by the cancellation in the Tucker sum.
    require_gpu()
    import paper_1411_1994_amd as L
    p = W.Problem(**{**W.config(4).__dict__, "precision": prec})
    x = W.sample_points(4, 4096, W.half_widths(p))
    with L.Context(0) as c:
        r = c.submit(p, points=x)
        assert r.wait() == 0, r.stats()
        inf = r.info()
        v = r.values.copy()
        tile = r.tile()
        r.release()
    assert tile.shape == (512, 512, 512) and tile.dtype == np.float32
    assert inf.is_tucker == 1 and inf.rel_bound <= p.eps * (1 + 1e-9)
    rng = np.random.default_rng(44)
    loc = np.stack([rng.integers(0, 512, 160) for _ in range(3)], axis=1)
    loc[0] = (256, 256, 256)                                  # the centre cell (a lattice site)
    cells = loc + np.array(p.tile_lo)
    ref = O.brute_force_points(p, cells)
    got = tile[loc[:, 0], loc[:, 1], loc[:, 2]].astype(np.float64)
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref)), np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    sel = np.random.default_rng(5).choice(len(x), 24, replace=False)
    refp = O.brute_force_points(p, O.points_to_cells(x[sel], p.h, p.N))
    assert np.max(np.abs(v[sel] - refp)) <= tol * np.max(np.abs(refp))

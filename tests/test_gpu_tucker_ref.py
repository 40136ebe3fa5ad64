"""The Tucker-reference sum (Thm thm:sumCaseE (B)) on the device against the oracle's."""
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


def rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


@pytest.mark.parametrize("kind,param", [(W.NEWTON, 0.0), (W.YUKAWA, 0.5)])
@pytest.mark.parametrize("eps", [1e-5, 1e-8])
def test_tucker_reference_sum_matches_oracle(ctx, kind, param, eps):
    blk = W.Block((6, 5, 4), (1.0, 1.25, 0.75), (0.25, -0.5, 0.0))
    p = W.Problem("tref", kind, param, 28, (81, 75, 69), 0.25, [blk], eps=eps, method=1)
    r = run(ctx, p)
    core_o, Q_o, _, _ = O.tucker_lattice_sum(p)
    assert tuple(r.info().r) == core_o.shape          # the reference's ranks (Thm (B))
    pts = points(p, 300, 61)
    got = r.sample(cells_xyz(p, pts))
    want = O.tucker_points(core_o, Q_o, pts)
    assert rel(got, want) <= 1e-10
    # against the plain sum of every charge: the reference's Tucker error, summed over the sites
    assert rel(got, O.brute_force_points(p, pts)) <= 20 * eps
    r.release()


def test_tucker_reference_union_of_blocks_and_tile(ctx):
    blocks = [W.Block((4, 4, 3), (1.0, 1.0, 1.0), (-2.0, 0.0, 0.5)),
              W.Block((3, 2, 2), (0.75, 1.5, 1.0), (3.0, 2.0, -1.0), charge=-0.5)]
    p = W.Problem("tref2", W.NEWTON, 0.0, 28, (65, 61, 57), 0.25, blocks, eps=1e-7, method=1,
                  tile_lo=(10, 12, 14), tile_T=(24, 20, 16))
    r = run(ctx, p)
    core_o, Q_o, _, _ = O.tucker_lattice_sum(p)
    pts = points(p, 300, 62)
    got = r.sample(cells_xyz(p, pts))
    assert rel(got, O.tucker_points(core_o, Q_o, pts)) <= 1e-10
    tile = r.tile()
    want = O.tucker_full(core_o, [Q_o[0][10:34], Q_o[1][12:32], Q_o[2][14:30]])
    assert rel(tile, want) <= 1e-10
    r.release()


def test_tucker_reference_large_lattice(ctx):
    # 16^3 sites on N = 1025 (the smallest case of Table Table_timesL scaled down in N): values
    # against the plain sum at sampled cells
    blk = W.Block((16, 16, 16), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))
    p = W.Problem("tref-L16", W.NEWTON, 0.0, 36, (1025, 1025, 1025), 1.0 / 32, [blk], eps=1e-7, method=1)
    r = run(ctx, p)
    pts = points(p, 40, 63)
    got = r.sample(cells_xyz(p, pts))
    r.release()
    assert rel(got, O.brute_force_points(p, pts)) <= 1e-6


def test_tucker_reference_rejects_what_it_does_not_cover(ctx):
    import paper_1411_1994_amd as L
    blk = W.Block((3, 3, 3), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))
    bad = [W.Problem("x", W.NEWTON, 0.0, 24, (41, 41, 41), 0.25, [blk], eps=0.0, method=1),
           W.Problem("x", W.NEWTON, 0.0, 24, (41, 41, 41), 0.25, [blk], eps=1e-6, method=1, precision=W.FP32),
           W.Problem("x", W.NEWTON, 0.0, 24, (41, 41, 41), 0.25, [blk], [W.Defect(0, (1, 1, 1), -1.0)],
                     eps=1e-6, method=1),
           W.Problem("x", W.NEWTON, 0.0, 24, (41, 41, 41), 0.25, [blk], eps=1e-6, method=7)]
    for p in bad:
        with pytest.raises(L.LsumError) as e:
            ctx.submit(p)
        assert e.value.code == -1


def test_generalised_rhosvd_of_blocks_with_vacancy_and_impurity_blocks(ctx):
    # the setting of Fig. fig:Tuck_vac: a 16 x 16 x 1 lattice with a 2 x 2 x 1 block of vacancies
    # (charge -1) and a 2 x 2 x 1 block of impurities (Z = 1.5: charge change 0.5), summed as Tucker
    # tensors and truncated by the generalised RHOSVD (Thm thm:TSum2Tucker) at eps
    eps = 1e-6
    blocks = [W.Block((16, 16, 1), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0)),
              W.Block((2, 2, 1), (1.0, 1.0, 1.0), (-3.0, 2.0, 0.0), charge=-1.0),
              W.Block((2, 2, 1), (1.0, 1.0, 1.0), (4.0, -5.0, 0.0), charge=0.5)]
    p = W.Problem("tref-vac", W.NEWTON, 0.0, 28, (161, 161, 65), 0.125, blocks, eps=eps, method=1)
    r = run(ctx, p)
    core_o, Z_o, bound_o, norm_o = O.tucker_lattice_sum(p)
    info = r.info()
    assert tuple(info.r) == core_o.shape
    assert info.rel_bound <= eps and abs(info.norm_A - norm_o) <= 1e-10 * norm_o
    # the device's tail is ||W||^2 less the retained rows' norms after its Jacobi rotations, never
    # below the exact tail (Ky Fan) and looser where rows below the irrelevance floor stay unrotated
    assert bound_o * (1 - 1e-9) <= info.bound <= 2 * bound_o
    pts = points(p, 300, 64)
    got = r.sample(cells_xyz(p, pts))
    r.release()
    assert rel(got, O.tucker_points(core_o, Z_o, pts)) <= 1e-9
    assert rel(got, O.brute_force_points(p, pts)) <= 10 * eps


def test_tucker_reference_with_c2t_als(ctx):
    # the reference's Tucker form refined by ALS sweeps (the canonical-to-Tucker approximation of
    # Thm thm:C2Tucker), then assembled: against the oracle's same construction
    blk = W.Block((6, 5, 4), (1.0, 1.25, 0.75), (0.25, -0.5, 0.0))
    p = W.Problem("tref-als", W.NEWTON, 0.0, 28, (81, 75, 69), 0.25, [blk], eps=1e-5, method=1, als_sweeps=2)
    r = run(ctx, p)
    core_o, Q_o, _, _ = O.tucker_lattice_sum(p)
    assert tuple(r.info().r) == core_o.shape
    pts = points(p, 300, 65)
    got = r.sample(cells_xyz(p, pts))
    r.release()
    assert rel(got, O.tucker_points(core_o, Q_o, pts)) <= 1e-9

"""Pins of the oracle's lattice bookkeeping, assembled canonical sum (Thm thm:sumCaseE (A)),
defect algebra (Sec. 4.1) and RHOSVD (Def. def:RHOSVD, Appendix theorem).  CPU only."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def exact_snap(coord: Fraction, h: Fraction, N: int) -> int:
    """Round-half-away-from-zero of coord/h in exact rational arithmetic."""
    u = coord / h
    j = math.floor(abs(u) + Fraction(1, 2))
    return (j if u >= 0 else -j) + (N - 1) // 2


def small_problem(kind=W.NEWTON, param=0.0, L=(3, 4, 2), N=(33, 41, 29), h=0.37, M=12,
                  center=(0.1, -0.2, 0.05), defects=(), blocks=None):
    blocks = blocks or [W.Block(L, (1.0, 1.0, 1.0), center)]
    return W.Problem("small", kind, param, M, N, h, blocks, list(defects))


# ------------------------------------------------------------------------------------------
# bookkeeping
# ------------------------------------------------------------------------------------------

def test_cfg1_offsets_exact():
    p = W.config(1)
    offs = O.block_offsets(p.blocks[0], p.h, p.N)
    with open(os.path.join(GOLDEN, "closed_forms.json")) as f:
        g = json.load(f)["cfg1_snapped_offsets"]["value"]
    for a in range(3):
        assert offs[a].tolist() == g
    # and from first principles with rationals
    h = Fraction(3, 32)
    exp = [exact_snap(Fraction(2 * k - 3, 2), h, 129) for k in range(4)]
    assert exp == g


@pytest.mark.parametrize("c", [1, 2, 3, 4])
def test_config_offsets_match_rational_arithmetic(c):
    p = W.config(c)
    for blk in p.blocks:
        offs = O.block_offsets(blk, p.h, p.N)
        for a in range(3):
            h = Fraction(p.h)           # the double h exactly
            L = blk.L[a]
            exp = [exact_snap((Fraction(k) - Fraction(L - 1, 2)) * Fraction(blk.b[a]) + Fraction(blk.center[a]),
                              h, p.N[a]) for k in range(L)]
            assert offs[a].tolist() == exp


def test_centred_offsets_are_mirror_symmetric():
    for c in (1, 2, 3):
        p = W.config(c)
        o = O.block_offsets(p.blocks[0], p.h, p.N)[0]
        assert np.array_equal(o + o[::-1], np.full_like(o, p.N[0] - 1))


def test_out_of_box_raises():
    with pytest.raises(O.OutOfBox):
        O.snap(np.array([10.0]), 0.5, 21)          # cell 30 of a 21-cell axis
    assert O.snap(np.array([5.0, -5.0]), 0.5, 21).tolist() == [20, 0]


def test_charges_apply_defects():
    p = small_problem(defects=[W.Defect(0, (1, 2, 0), -1.0), W.Defect(0, (0, 0, 1), 0.75)])
    idx, Z = O.charges(p)
    assert len(Z) == 24 and Z.sum() == 24 - 1 + 0.75
    assert Z[(1 * 4 + 2) * 2 + 0] == 0.0 and Z[1] == 1.75


# ------------------------------------------------------------------------------------------
# Theorem A: the assembled rank-R canonical tensor equals the brute-force sum
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("kind,param", [(W.NEWTON, 0.0), (W.YUKAWA, 0.5), (W.SLATER, 1.0)])
def test_assembled_equals_brute_force_full_grid(kind, param):
    p = small_problem(kind, param)
    t, w = O.quadrature_of(p)
    fac = O.assembled_canonical(p, t, w)[0]
    assert all(f.shape == (len(t), n) for f, n in zip(fac, p.N))      # rank stays R
    V = np.einsum("qi,qj,qk->ijk", *fac)
    Vb = O.brute_force_grid(p, t=t, w=w)
    assert np.max(np.abs(V - Vb)) <= 1e-13 * np.max(np.abs(Vb))


def test_concatenation_to_sum_rule():
    # eq. conc2sum: CP tensors sharing two factor matrices add by adding the third factors
    rng = np.random.default_rng(0)
    A1, A2, A3, B3 = (rng.standard_normal((5, n)) for n in (4, 6, 7, 7))
    full = lambda X, Y, Z: np.einsum("qi,qj,qk->ijk", X, Y, Z)
    assert np.allclose(full(A1, A2, A3) + full(A1, A2, B3), full(A1, A2, A3 + B3), atol=1e-13)


def test_lattice_symmetry_cubic():
    p = W.Problem("sym", W.NEWTON, 0.0, 16, (41, 41, 41), 0.3, [W.cubic_block(5, 1.0)])
    t, w = O.quadrature_of(p)
    fac = O.assembled_canonical(p, t, w)[0]
    V = np.einsum("qi,qj,qk->ijk", *fac)
    scale = np.max(V)
    assert np.max(np.abs(V - V[::-1, :, :])) <= 1e-14 * scale
    assert np.max(np.abs(V - V.transpose(1, 0, 2))) <= 1e-14 * scale
    assert np.max(np.abs(V - V.transpose(2, 1, 0))) <= 1e-14 * scale


def test_far_field_matches_point_charges():
    # far from every charge the lattice potential is sum_c 1/|x - c| (snapped positions)
    p = W.Problem("ff", W.NEWTON, 0.0, 40, (257, 257, 257), 0.125, [W.cubic_block(3, 1.0)])
    t, w = O.quadrature_of(p)
    fac = O.assembled_canonical(p, t, w)[0]
    idx, Z = O.charges(p)
    pts = np.array([[0, 0, 0], [10, 200, 128], [250, 30, 60], [128, 128, 0]])
    got = O.canonical_eval(fac, pts)
    x = (pts - 128) * p.h
    c = (idx - 128) * p.h
    ref = np.array([np.sum(Z / np.linalg.norm(xi - c, axis=1)) for xi in x])
    assert np.max(np.abs(got / ref - 1)) < 2e-5


def test_canonical_pipeline_matches_brute_force_at_points():
    p = small_problem(L=(4, 3, 5), N=(45, 37, 51), h=0.29)
    B = W.half_widths(p)
    xyz = np.random.default_rng(3).uniform(-np.array(B), np.array(B), size=(40, 3))
    _, v = O.canonical_pipeline(p, xyz)
    pts = O.points_to_cells(xyz, p.h, p.N)
    vb = O.brute_force_points(p, pts)
    assert np.max(np.abs(v - vb)) <= 1e-13 * np.max(np.abs(vb))


# ------------------------------------------------------------------------------------------
# defects (Sec. 4.1, eq. Can_LatticeSum_full)
# ------------------------------------------------------------------------------------------

def test_vacancy_invariant():
    # full lattice minus vacancy windows equals the direct sum over the remaining charges
    rng = np.random.default_rng(5)
    base = small_problem(L=(4, 3, 3), N=(31, 27, 29), h=0.41)
    defects = W.draw_defects(rng, base.blocks, 5, 0)
    p = small_problem(L=(4, 3, 3), N=(31, 27, 29), h=0.41, defects=defects)
    xi, A = O.canonical_terms(p)
    V = O.cp_full(xi, A)
    Vb = O.brute_force_grid(p)
    assert np.max(np.abs(V - Vb)) <= 1e-13 * np.max(np.abs(Vb))
    R = len(O.quadrature_of(p)[0])
    assert len(xi) == R * (1 + len(defects))                  # eq. RankCan_def: r <= r0 + sum r_s


def test_linearity_in_charge_change():
    p0 = small_problem()
    pts = np.array([[3, 5, 7], [16, 20, 14], [30, 2, 25]])
    base = O.brute_force_points(p0, pts)
    vals = []
    for dz in (0.25, 0.5, 1.0):
        p = small_problem(defects=[W.Defect(0, (1, 1, 1), dz), W.Defect(0, (2, 3, 0), -dz)])
        xi, A = O.canonical_terms(p)
        vals.append(np.einsum("v,pv,pv,pv->p", xi, A[0][pts[:, 0]], A[1][pts[:, 1]], A[2][pts[:, 2]]) - base)
    assert np.allclose(vals[1], 2 * vals[0], rtol=1e-11, atol=1e-13)
    assert np.allclose(vals[2], 4 * vals[0], rtol=1e-11, atol=1e-13)


# ------------------------------------------------------------------------------------------
# RHOSVD
# ------------------------------------------------------------------------------------------

def _defected(nvac=4, nimp=3, kind=W.NEWTON, param=0.0, seed=11):
    rng = np.random.default_rng(seed)
    base = small_problem(kind, param, L=(4, 4, 3), N=(29, 31, 27), h=0.43)
    defects = W.draw_defects(rng, base.blocks, nvac, nimp)
    return small_problem(kind, param, L=(4, 4, 3), N=(29, 31, 27), h=0.43, defects=defects)


@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-6])
def test_rhosvd_bound_and_relative_error(eps):
    p = _defected()
    xi, A = O.canonical_terms(p)
    res = O.rhosvd(xi, A, eps=eps)
    Afull = O.cp_full(xi, A)
    T = O.tucker_full(res.core, res.Z)
    err = np.linalg.norm(Afull - T)
    nA = np.linalg.norm(Afull)
    assert abs(res.norm_A - nA) <= 1e-12 * nA
    assert err <= res.bound * (1 + 1e-9) + 1e-12 * nA        # Appendix theorem (d)
    assert err <= eps * nA * (1 + 1e-9)                        # the certified truncation rule
    for Z in res.Z:
        assert np.allclose(Z.T @ Z, np.eye(Z.shape[1]), atol=1e-13)
    # Pythagoras: the core is an orthogonal projection of A
    assert abs(np.linalg.norm(res.core) ** 2 + err ** 2 - nA ** 2) <= 1e-10 * nA ** 2


def test_rhosvd_core_is_projection_of_full_tensor():
    # Appendix (c): mu_k = <w1_k1 (x) w2_k2 (x) w3_k3, A>, computed here from the full tensor
    p = _defected(kind=W.YUKAWA, param=0.5)
    xi, A = O.canonical_terms(p)
    res = O.rhosvd(xi, A, eps=1e-5)
    Afull = O.cp_full(xi, A)
    mu = np.einsum("ijk,ia,jb,kc->abc", Afull, *res.Z, optimize=True)
    assert np.max(np.abs(mu - res.core)) <= 1e-12 * np.max(np.abs(mu))


def test_rhosvd_full_rank_is_exact():
    p = _defected(nvac=2, nimp=1)
    xi, A = O.canonical_terms(p)
    full = [min(a.shape) for a in A]
    res = O.rhosvd(xi, A, ranks=full)
    Afull = O.cp_full(xi, A)
    assert np.max(np.abs(O.tucker_full(res.core, res.Z) - Afull)) <= 1e-12 * np.max(np.abs(Afull))
    assert all(r <= np.linalg.matrix_rank(a) + 1 for r, a in zip(full, A))


def test_perfect_lattice_rank_at_most_R():
    # Thm A: a perfect lattice keeps the reference rank R in every mode
    p = small_problem(L=(4, 4, 3), N=(29, 31, 27), h=0.43)
    xi, A = O.canonical_terms(p)
    R = len(xi)
    res = O.rhosvd(xi, A, eps=1e-14)
    assert all(r <= R for r in res.ranks)


def test_sublattice_vacancies_rank_at_most_2R():
    # Sec. 4.4, class (D) / Fig. fig:Vacance_L_O: vacancies on a tensor sub-lattice, written as a
    # second block of charge -1, give Tucker ranks <= 2R; the sum equals the direct sum
    big = W.Block((8, 8, 2), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))
    vac = W.Block((2, 2, 1), (4.0, 4.0, 1.0), (0.5, 0.5, -0.5), charge=-1.0)
    p = W.Problem("sub", W.NEWTON, 0.0, 14, (45, 45, 29), 0.5, [big, vac])
    xi, A = O.canonical_terms(p)
    R = len(O.quadrature_of(p)[0])
    res = O.rhosvd(xi, A, eps=1e-12)
    assert all(r <= 2 * R for r in res.ranks)
    Afull = O.cp_full(xi, A)
    Vb = O.brute_force_grid(p)
    assert np.max(np.abs(Afull - Vb)) <= 1e-13 * np.max(np.abs(Vb))
    # equivalently: the same sites removed one by one as vacancies
    offs_big = O.block_offsets(big, p.h, p.N)
    offs_vac = O.block_offsets(vac, p.h, p.N)
    sites = []
    for i in offs_vac[0]:
        for j in offs_vac[1]:
            for k in offs_vac[2]:
                sites.append((int(np.where(offs_big[0] == i)[0][0]), int(np.where(offs_big[1] == j)[0][0]),
                              int(np.where(offs_big[2] == k)[0][0])))
    p2 = W.Problem("sub2", W.NEWTON, 0.0, 14, (45, 45, 29), 0.5, [big], [W.Defect(0, s, -1.0) for s in sites])
    xi2, A2 = O.canonical_terms(p2)
    assert np.max(np.abs(O.cp_full(xi2, A2) - Afull)) <= 1e-13 * np.max(np.abs(Vb))


def test_single_kernel_tucker_rank_ballpark():
    # soft pin from Table Table_Times: the Tucker rank of one Newton kernel at eps = 1e-6 is
    # about 6..12 on the paper's grids; RHOSVD (no ALS) of the centred reference
    with open(os.path.join(GOLDEN, "paper_numbers.json")) as f:
        ranks = json.load(f)["table_times"]["tucker_rank"]
    p = W.Problem("one", W.NEWTON, 0.0, 40, (257, 257, 257), 8.75 / 256, [W.cubic_block(1)])
    xi, A = O.canonical_terms(p)
    res = O.rhosvd(xi, A, eps=1e-6)
    assert min(ranks) - 2 <= max(res.ranks) <= 2 * max(ranks)


def test_tucker_evaluators_agree_with_direct_triple_sum():
    rng = np.random.default_rng(2)
    core = rng.standard_normal((3, 2, 4))
    Z = [rng.standard_normal((n, r)) for n, r in zip((5, 6, 7), core.shape)]
    full = O.tucker_full(core, Z)
    for (i, j, k) in [(0, 0, 0), (4, 5, 6), (2, 3, 1)]:
        s = 0.0
        for a in range(3):
            for b in range(2):
                for c in range(4):
                    s += core[a, b, c] * Z[0][i, a] * Z[1][j, b] * Z[2][k, c]
        assert abs(full[i, j, k] - s) < 1e-12
    pts = np.array([[1, 2, 3], [4, 0, 6]])
    assert np.allclose(O.tucker_points(core, Z, pts), full[pts[:, 0], pts[:, 1], pts[:, 2]], atol=1e-13)
    tile = O.tucker_tile(core, Z, [np.arange(1, 4), np.arange(2, 6), np.arange(0, 7)])
    assert np.allclose(tile, full[1:4, 2:6, 0:7], atol=1e-13)


def test_snap_rounds_halves_away_from_zero():
    # exact ties: x/h = +-2.5 -> +-3 (not banker's rounding), +-0.5 -> +-1
    assert O.snap(np.array([1.25, -1.25, 0.25, -0.25, 0.0]), 0.5, 21).tolist() == [13, 7, 11, 9, 10]


def test_truncation_rule_is_smallest_certified_rank():
    # the chosen r_l is the smallest rank whose discarded tail is <= eps ||A|| / (3 ||xi||);
    # singular values recomputed here from the eigenvalues of A A^T (a different route)
    p = _defected(nvac=5, nimp=2)
    xi, A = O.canonical_terms(p)
    for eps in (1e-3, 1e-5):
        res = O.rhosvd(xi, A, eps=eps)
        thr = eps * res.norm_A / (3.0 * np.linalg.norm(xi))
        for a in range(3):
            lam = np.sort(np.clip(np.linalg.eigvalsh(A[a] @ A[a].T), 0, None))[::-1]
            tail = lambda r: math.sqrt(lam[r:].sum())
            r = res.ranks[a]
            assert tail(r) <= thr * (1 + 1e-6) + 1e-12
            assert r == 1 or tail(r - 1) > thr * (1 - 1e-6)


# ---------------------------------------------------------------------------------------
# exact sites: every charge at its own position (no snapping)
# ---------------------------------------------------------------------------------------

def _cells(rng, N, n):
    return np.stack([rng.integers(0, N[a], n) for a in range(3)], axis=1)


def test_exact_sites_on_cell_centres_equal_snapped():
    # b/h even (so (k - (L-1)/2) b is a whole number of cells for even L too) and a centre on a
    # cell centre: the exact positions are the snapped ones
    h = 0.25
    p = W.Problem("on-grid", W.NEWTON, 0.0, 24, (41, 41, 41), h,
                  [W.Block((3, 4, 2), (1.0, 0.5, 1.5), (0.25, -0.5, 0.0)),
                   W.Block((2, 2, 3), (0.5, 1.0, 0.5), (-1.0, 1.25, 0.75), charge=-2.0)])
    pts = _cells(np.random.default_rng(3), p.N, 60)
    a = O.brute_force_points(p, pts)
    b = O.brute_force_points_exact(p, pts)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))


def test_exact_site_single_charge_against_exact_galerkin():
    # one charge at a sub-cell position: its entries are the exact cell averages of the kernel
    # about that position (eq. galten), up to the sinc error of the rule (M = 48: < 1e-6)
    N, h = (65, 65, 65), 0.25
    y = np.array([0.3, -0.45, 0.1]) * h + np.array([2, -1, 0]) * h
    p = W.Problem("one", W.NEWTON, 0.0, 48, N, h, [W.Block((1, 1, 1), (1.0, 1.0, 1.0), tuple(y))])
    pts = np.concatenate([np.array([[32 + i, 32 + j, 32 + k] for i in (1, 2, 3) for j in (-2, -1, 0)
                                    for k in (-1, 0, 1)]), _cells(np.random.default_rng(4), N, 20)])
    v = O.brute_force_points_exact(p, pts)
    centres = (pts - 32) * h
    exact = O.exact_cell_averages(W.NEWTON, 0.0, (centres - y) / h, h)
    assert np.max(np.abs(v - exact)) <= 1e-6 * np.max(exact)
    # the snapped charge (cell (2, -1, 0)) is off by O(h) near the charge
    snapped = O.brute_force_points(p, pts)
    assert np.max(np.abs(snapped - exact)) > 1e-2 * np.max(exact)


def test_exact_sites_far_field_matches_point_charges():
    # b/h = 22/5 and a sub-cell centre: far from the lattice every cell average is the point value
    h = 0.25
    blk = W.Block((3, 3, 3), (1.1, 1.1, 1.1), (0.07, -0.11, 0.13))
    p = W.Problem("far", W.NEWTON, 0.0, 40, (161, 161, 161), h, [blk])
    pos, Z = O.charge_positions(p)
    pts = np.array([[150, 80, 80], [10, 10, 150], [80, 155, 5], [2, 158, 79]])
    v = O.brute_force_points_exact(p, pts)
    x = (pts - 80) * h
    direct = np.array([np.sum(Z / np.linalg.norm(pos - xi, axis=1)) for xi in x])
    assert np.max(np.abs(v - direct) / direct) < 2e-5


def test_exact_sites_mirror_and_whole_cell_shift():
    # a lattice centred at +d and its mirror at -d give mirrored fields; moving the centre by one
    # whole cell moves the field by one cell (both exact up to rounding)
    h, N = 0.25, (45, 45, 45)
    d = (0.31, -0.17, 0.09)
    mk = lambda c: W.Problem("m", W.NEWTON, 0.0, 32, N, h, [W.Block((4, 3, 2), (0.8, 0.65, 1.1), c)])
    pts = _cells(np.random.default_rng(5), (40, 40, 40), 40) + 2
    v = O.brute_force_points_exact(mk(d), pts)
    vm = O.brute_force_points_exact(mk(tuple(-x for x in d)), (np.array(N) - 1) - pts)
    assert np.max(np.abs(v - vm)) <= 1e-12 * np.max(np.abs(v))
    vs = O.brute_force_points_exact(mk((d[0] + h, d[1], d[2])), pts + np.array([1, 0, 0]))
    assert np.max(np.abs(v - vs)) <= 1e-12 * np.max(np.abs(v))


# ---------------------------------------------------------------------------------------
# Thm thm:sumCaseE (B): the Tucker-reference sum
# ---------------------------------------------------------------------------------------

def _tref_problem(blocks, N=(33, 29, 25), h=0.25, eps=1e-6, M=24):
    return W.Problem("tref", W.NEWTON, 0.0, M, N, h, blocks, eps=eps, method=1)


def test_tucker_reference_sum_of_one_charge_is_the_windowed_reference():
    # one site: the assembled vectors are the reference vectors' windows, so the sum is the
    # reference Tucker tensor read at the displacements
    p = _tref_problem([W.Block((1, 1, 1), (1.0, 1.0, 1.0), (0.5, -0.75, 0.25))])
    core, Q, _, _ = O.tucker_lattice_sum(p)
    ref = O.tucker_reference(p)
    c = np.array([O.block_offsets(p.blocks[0], p.h, p.N)[a][0] for a in range(3)])
    pts = np.stack([np.random.default_rng(6).integers(0, n, 50) for n in p.N], axis=1)
    Nr = max(p.N)
    got = O.tucker_points(core, Q, pts)
    want = O.tucker_points(ref.core, ref.Z, pts - c + Nr - 1)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    for a in range(3):
        assert np.allclose(Q[a].T @ Q[a], np.eye(Q[a].shape[1]), atol=1e-12)


def test_tucker_reference_sum_error_is_bounded_by_the_reference_error():
    # T_cL - P_cL = sum_k W_k (T_ref - P_ref): each window is a sub-box of the reference, so
    # ||T_cL - P_cL||_F <= (number of sites) ||T_ref - P_ref||_F (plus, for two blocks, the
    # certified truncation of their sum), on the full (small) grid
    blocks = [W.Block((3, 3, 2), (1.0, 1.25, 1.5), (0.0, 0.25, -0.5)),
              W.Block((2, 1, 2), (0.75, 1.0, 1.0), (-2.0, 1.5, 1.0), charge=-0.5)]
    p = _tref_problem(blocks)
    core, Q, bound, _ = O.tucker_lattice_sum(p)
    T = O.tucker_full(core, Q)
    P = O.brute_force_grid(p)
    ref = O.tucker_reference(p)
    t, w = O.quadrature_of(p)
    Bv = O.reference_vectors(t, w, max(p.N), p.h)
    Pref = np.einsum("qi,qj,qk->ijk", Bv, Bv, Bv, optimize=True)
    e_ref = np.linalg.norm(O.tucker_full(ref.core, ref.Z) - Pref)
    n_sites = sum(abs(b.charge) * np.prod(b.L) for b in blocks)
    assert np.linalg.norm(T - P) <= n_sites * e_ref * (1 + 1e-9) + bound
    assert np.linalg.norm(T - P) <= 1e-5 * np.linalg.norm(P)
    # and the reference's own error obeys its certified RHOSVD bound
    assert e_ref <= ref.bound * (1 + 1e-9) and ref.bound <= p.eps * np.linalg.norm(Pref) * (1 + 1e-9)


def test_tucker_reference_sum_keeps_the_reference_ranks_for_every_L():
    # the rank of the assembled sum is the reference's whatever the lattice size (Thm (B))
    ranks = set()
    for L in (1, 2, 4, 8):
        p = _tref_problem([W.Block((L, L, L), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))], N=(41, 41, 41))
        core, Q, _, _ = O.tucker_lattice_sum(p)
        ranks.add(core.shape)
    assert len(ranks) == 1 and ranks.pop() == O.tucker_reference(p).ranks


def test_generalised_rhosvd_of_a_union_of_blocks():
    # Thm thm:TSum2Tucker on the sum of two blocks' Tucker tensors: the truncated result is within
    # its certified bound of the untruncated sum, the bound is <= eps ||U||, ||U|| is the full
    # tensor's norm, and the ranks drop below the stacked 2 r
    blocks = [W.Block((4, 4, 2), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0)),
              W.Block((2, 2, 1), (1.0, 1.0, 1.0), (0.5, 0.5, 0.0), charge=-1.0)]
    p = _tref_problem(blocks, eps=1e-4)
    core, Z, bound, norm = O.tucker_lattice_sum(p)
    parts = [O.tucker_lattice_sum(_tref_problem([b], eps=1e-4)) for b in blocks]
    U = sum(O.tucker_full(c, q) for c, q, _, _ in parts)
    T = O.tucker_full(core, Z)
    assert abs(np.linalg.norm(U) - norm) <= 1e-10 * norm
    assert np.linalg.norm(T - U) <= bound * (1 + 1e-9)
    assert 0 < bound <= p.eps * norm * (1 + 1e-9)
    r_ref = O.tucker_reference(p).ranks
    assert all(core.shape[a] < 2 * r_ref[a] for a in range(3))


# ---------------------------------------------------------------------------------------
# Thm thm:C2Tucker (b): ALS from the RHOSVD initial guess
# ---------------------------------------------------------------------------------------

def test_als_raises_the_core_norm_and_lowers_the_error():
    # the dual objective ||core|| never decreases, and ||A - T||^2 = ||A||^2 - ||core||^2 falls
    # below the RHOSVD error (projection onto orthonormal factors)
    xi, A = O.canonical_terms(_defected(nvac=5, nimp=3))
    res = O.rhosvd(xi, A, ranks=(6, 5, 4))
    Z, core, hist = O.als_refine(xi, A, res.Z, 4)
    full = O.cp_full(xi, A)
    e0 = np.linalg.norm(full - O.tucker_full(res.core, res.Z))
    e1 = np.linalg.norm(full - O.tucker_full(core, Z))
    assert np.all(np.diff(hist) >= -1e-12 * hist[0]) and hist[0] >= np.linalg.norm(res.core) * (1 - 1e-12)
    assert e1 <= e0 * (1 + 1e-12)
    assert abs(e1 ** 2 - (np.linalg.norm(full) ** 2 - hist[-1] ** 2)) <= 1e-9 * np.linalg.norm(full) ** 2
    for z in Z:
        assert np.allclose(z.T @ z, np.eye(z.shape[1]), atol=1e-12)


def test_als_recovers_an_exact_tucker_tensor():
    # a canonical tensor that is exactly of Tucker rank (3, 3, 2) (its terms are the core's entries
    # times products of orthonormal columns) is recovered to rounding from a perturbed guess
    rng = np.random.default_rng(17)
    N, r = (20, 18, 16), (3, 3, 2)
    Q = [np.linalg.qr(rng.standard_normal((N[a], r[a])))[0] for a in range(3)]
    B = rng.standard_normal(r)
    idx = [(i, j, k) for i in range(r[0]) for j in range(r[1]) for k in range(r[2])]
    xi = np.array([B[i, j, k] for i, j, k in idx])
    A = [np.stack([Q[a][:, t[a]] for t in idx], axis=1) for a in range(3)]
    guess = [np.linalg.qr(Q[a] + 0.3 * rng.standard_normal(Q[a].shape))[0] for a in range(3)]
    Z, core, hist = O.als_refine(xi, A, guess, 6)
    T = O.tucker_full(core, Z)
    assert np.linalg.norm(T - O.cp_full(xi, A)) <= 1e-10 * np.linalg.norm(B)


# ---------------------------------------------------------------------------------------
# Can -> Tuck -> Can
# ---------------------------------------------------------------------------------------

def test_tucker_to_canonical_exact_and_truncated():
    xi0, A0 = O.canonical_terms(_defected(nvac=6, nimp=2))
    res = O.rhosvd(xi0, A0, ranks=(8, 7, 5))
    T = O.tucker_full(res.core, res.Z)
    # eps = 0: the same tensor, rank <= r3 min(r1, r2), orthogonal rank-1 terms
    xi, A, err = O.tucker_to_canonical(res.core, res.Z, 0.0)
    assert len(xi) <= 5 * 7 and err == 0.0
    C = O.cp_full(xi, A)
    assert np.linalg.norm(C - T) <= 1e-12 * np.linalg.norm(T)
    assert abs(np.sum(xi ** 2) - np.linalg.norm(T) ** 2) <= 1e-12 * np.linalg.norm(T) ** 2
    for a in range(3):
        assert np.allclose(np.linalg.norm(A[a], axis=0), 1.0, atol=1e-12)
    # truncated: the error is the root of the dropped s^2 and at most eps ||core||
    for eps in (1e-3, 1e-6):
        xi2, A2, err2 = O.tucker_to_canonical(res.core, res.Z, eps)
        e = np.linalg.norm(O.cp_full(xi2, A2) - T)
        assert abs(e - err2) <= 1e-9 * np.linalg.norm(T) and err2 <= eps * np.linalg.norm(res.core)
        assert len(xi2) < len(xi) if eps == 1e-3 else len(xi2) <= len(xi)


def test_shear_sites_and_explicit_charge_sum_pins():
    # zero shear: the rectangular block itself; a shear moves each site by (k - (L-1)/2) shear
    base = W.Block((4, 3, 2), (1.0, 0.7, 1.3), (0.2, -0.1, 0.4))
    pos0 = O.shear_sites(base, 0, 1, 0.0)
    rect, _ = O.charge_positions(W.Problem("r", 0, 0.0, 8, (5, 5, 5), 1.0, [base]))
    assert np.array_equal(pos0, rect)
    pos = O.shear_sites(base, 0, 1, 0.5)
    k1 = np.repeat(np.tile(np.arange(3), 4), 2)           # the axis-1 index of each site (C order)
    assert np.allclose(pos[:, 0] - rect[:, 0], (k1 - 1.0) * 0.5) and np.array_equal(pos[:, 1:], rect[:, 1:])
    # the explicit-list sum over a block's own sites and charges is the block sum
    blocks = [base, W.Block((2, 2, 2), (1.0, 1.0, 1.0), (1.5, 1.0, -1.0), charge=-0.5)]
    p = W.Problem("e", W.NEWTON, 0.0, 24, (33, 33, 33), 0.25, blocks)
    pts = np.stack([np.random.default_rng(12).integers(0, 33, 40) for _ in range(3)], axis=1)
    posb, Z = O.charge_positions(p)
    assert np.allclose(O.brute_force_points_at(p, pts, posb, Z), O.brute_force_points(p, pts), rtol=1e-13, atol=0)

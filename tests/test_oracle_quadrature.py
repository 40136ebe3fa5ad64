"""Pins of the oracle's quadrature and collocation (Sec. 2.1-2.2) against closed forms and
independent numerics.  CPU only."""
import json
import math
import os

import mpmath
import numpy as np
import pytest
from scipy.integrate import dblquad
from scipy.special import erf

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kernel_err(kind, p, M, N, h):
    hu, s = O.default_quadrature(kind, (N, N, N), h)
    t, w = O.sinc_nodes(kind, p, M, hu, s)
    r_max = math.sqrt(3) * (N - 1) * h
    z = np.geomspace(h, r_max, 2000)
    approx = (w * np.exp(-np.outer(z * z, t * t))).sum(1)
    exact = O.kernel_value(kind, p, z)
    return np.max(np.abs(approx - exact)) / np.max(exact), approx, exact, z


@pytest.mark.parametrize("N,h,M", [(129, 3 / 32, 32), (4097, 5 / 256, 40), (2049, 1 / 32, 40)])
def test_newton_gauss_sum_matches_inverse_distance(N, h, M):
    # eq. LalpNewt: 1/z = 2/sqrt(pi) int exp(-t^2 z^2) dt; the folded sinc rule reproduces it
    err, approx, exact, z = _kernel_err(O.NEWTON, 0.0, M, N, h)
    assert err < 1e-4
    # at moderate distances the pointwise relative error is small as well
    mid = z <= math.sqrt(3) * (N - 1) * h / 4
    assert np.max(np.abs(approx - exact)[mid] / exact[mid]) < 1e-5


@pytest.mark.parametrize("N,h,M", [(129, 3 / 32, 32), (2049, 1 / 32, 40)])
def test_yukawa_exponent_reading(N, h, M):
    # the corrected transform reproduces exp(-k z)/z; the printed one would give exp(-2 k z)/z
    err, approx, exact, z = _kernel_err(O.YUKAWA, 0.5, M, N, h)
    assert err < 1e-4
    wrong = np.exp(-2 * 0.5 * z) / z
    assert np.max(np.abs(approx - wrong)) / np.max(wrong) > 1e-2


@pytest.mark.parametrize("N,h,M", [(129, 3 / 32, 32), (2049, 1 / 32, 40)])
def test_slater_transform(N, h, M):
    # eq. LalpSlater with rho = z^2, kappa = l^2/4
    err, *_ = _kernel_err(O.SLATER, 1.0, M, N, h)
    assert err < 1e-4


def test_yukawa_zero_screening_is_newton():
    t0, w0 = O.sinc_nodes(O.NEWTON, 0.0, 30, 0.35, 5.0)
    t1, w1 = O.sinc_nodes(O.YUKAWA, 0.0, 30, 0.35, 5.0)
    assert np.array_equal(t0, t1) and np.allclose(w0, w1, rtol=1e-15, atol=0)


def test_node_closed_forms():
    # u_k = k h_u, t_k = sinh(u_k)/s; Newton weights h_u/(sqrt(pi) s) at k=0, 2 h_u cosh(u_k)/(sqrt(pi) s)
    hu, s = 0.3, 7.0
    t, w = O.sinc_nodes(O.NEWTON, 0.0, 5, hu, s)
    for k in range(6):
        mp_t = mpmath.sinh(k * mpmath.mpf(hu)) / s
        mp_w = (1 if k == 0 else 2) * hu * mpmath.cosh(k * mpmath.mpf(hu)) / (mpmath.sqrt(mpmath.pi) * s)
        assert abs(t[k] - float(mp_t)) <= 4e-16 * max(1.0, abs(float(mp_t)))
        assert abs(w[k] - float(mp_w)) <= 4e-16 * float(mp_w)
    assert len(t) == 6                                       # rank M+1 for Newton
    t2, w2 = O.sinc_nodes(O.YUKAWA, 0.5, 5, hu, s)
    assert len(t2) <= 5 and np.all(t2 > 0)                  # t = 0 carries no Yukawa weight


def test_exponential_convergence_in_M():
    # eq. sinc_conv: error <= C/a exp(-beta sqrt(M)) with h_M = C0 log M / M (eq. hM)
    for kind, p in [(O.NEWTON, 0.0), (O.YUKAWA, 0.5), (O.SLATER, 1.0)]:
        errs = []
        for M in (8, 16, 32, 64):
            t, w = O.sinc_nodes(kind, p, M, 2.0 * math.log(M) / M, 4.0)
            z = np.geomspace(0.05, 20, 1500)
            ap = (w * np.exp(-np.outer(z * z, t * t))).sum(1)
            ex = O.kernel_value(kind, p, z)
            errs.append(np.max(np.abs(ap - ex)) / np.max(ex))
        assert errs[0] > errs[1] > errs[2] > errs[3]
        assert errs[3] < 1e-6 and errs[0] / errs[3] > 1e5


# ------------------------------------------------------------------------------------------
# collocation (cell averages of Gaussians)
# ------------------------------------------------------------------------------------------

def test_cell_average_against_high_precision():
    # independent arithmetic: 50-digit erfc differences (no cancellation for positive ends)
    mpmath.mp.dps = 50
    h = 1 / 32
    rng = np.random.default_rng(1)
    ts = np.concatenate([[1e-4, 0.01, 0.3, 1.0, 7.0, 40.0, 300.0], rng.uniform(0, 50, 10)])
    ds = np.concatenate([np.arange(0, 8), [31, 100, 1000, 2048, 4095]]) * h
    for t in ts:
        got = O.cell_average_gauss(np.full(ds.shape, t), ds, h)
        for d, g in zip(ds, got):
            T, D, H = mpmath.mpf(float(t)), mpmath.mpf(float(d)), mpmath.mpf(h)
            lo, hi = T * (D - H / 2), T * (D + H / 2)
            diff = mpmath.erfc(lo) - mpmath.erfc(hi) if lo > 0 else mpmath.erf(hi) - mpmath.erf(lo)
            ex = float(mpmath.sqrt(mpmath.pi) / (2 * T * H) * diff)
            if ex < 1e-290:
                assert g < 1e-280
                continue
            # erf differences lose at most log10((|d|+h)/h) digits when both ends are close;
            # the FP64 erfc itself is good to ~2e-14 relative deep in the tail
            tol = 5e-14 + 4e-16 * abs(d) / h
            assert abs(g - ex) <= tol * ex, (t, d, g, ex)


def test_collocation_row_at_t0_and_mirror_symmetry():
    t, w = O.sinc_nodes(O.NEWTON, 0.0, 20, 0.35, 3.0)
    N, h = 65, 0.125
    P = O.reference_vectors(t, w, N, h)
    assert np.all(P[0] == np.cbrt(w[0]))                    # t = 0: exp(0) averages to 1
    assert np.array_equal(P, P[:, ::-1])                      # exact mirror symmetry in m
    assert P.shape == (len(t), 2 * N - 1)


def test_collocation_sum_rule_telescopes():
    # h sum_m b(t; m h) = int_{-(N-1/2)h}^{(N-1/2)h} exp(-t^2 x^2) dx = sqrt(pi)/t erf(t (N - 1/2) h)
    t, w = O.sinc_nodes(O.NEWTON, 0.0, 40, 0.35, 30.0)
    N, h = 1025, 1 / 32
    B = O.reference_vectors(t, w, N, h, weighted=False)
    lhs = h * B.sum(axis=1)
    tp = np.where(t > 0, t, 1.0)
    rhs = np.where(t > 0, math.sqrt(math.pi) / tp * erf(t * (N - 0.5) * h), (2 * N - 1) * h)
    assert np.max(np.abs(lhs - rhs) / rhs) < 1e-13


def test_cube_constant_closed_form():
    # average of 1/|x| over the cube of side h centred at the origin = (3 ln(2+sqrt 3) - pi/2)/h
    c_closed = 3 * math.log(2 + math.sqrt(3)) - math.pi / 2
    # independent: int_[0,1]^3 dV/r = int_[0,1]^2 asinh(1/rho) dx dy; the centred cube is 2x that
    v = dblquad(lambda y, x: np.arcsinh(1 / np.sqrt(x * x + y * y)), 0, 1, 0, 1,
                epsabs=1e-13, epsrel=1e-13)[0]
    assert abs(2 * v - c_closed) < 1e-11
    with open(os.path.join(GOLDEN, "closed_forms.json")) as f:
        g = json.load(f)
    assert abs(g["newton_unit_cube_average"]["value"] - c_closed) < 1e-14
    # the exact Galerkin entry (O3) at the singular cell
    h = 0.1
    assert abs(O.exact_cell_average(O.NEWTON, 0.0, [0, 0, 0], h) * h - c_closed) < 1e-10


@pytest.mark.parametrize("kind,p", [(O.NEWTON, 0.0), (O.YUKAWA, 0.5), (O.SLATER, 1.0)])
def test_canonical_entry_against_exact_galerkin(kind, p):
    # P_R (eq. sinc_general) against the exact cell average (eq. galten), max-norm relative
    N, h, M = 129, 3 / 32, 32
    hu, s = O.default_quadrature(kind, (N, N, N), h)
    t, w = O.sinc_nodes(kind, p, M, hu, s)
    disps = [(0, 0, 0), (1, 0, 0), (1, 1, 1), (2, 1, 0), (5, 3, 2), (16, 0, 0), (40, 40, 40),
             (128, 0, 0), (128, 128, 128), (7, 100, 33)]
    ex = np.array([O.exact_cell_average(kind, p, [di * h for di in d], h) for d in disps])
    ap = np.array([np.sum(w * np.prod([O.cell_average_gauss(t, di * h, h) for di in d], axis=0))
                   for d in disps])
    assert np.max(np.abs(ap - ex)) / np.max(np.abs(ex)) < 1e-4


def test_far_field_cell_average_is_point_value():
    # 1/r is harmonic: the cube average equals the centre value up to O((h/r)^4)
    N, h, M = 2049, 1 / 32, 40
    hu, s = O.default_quadrature(O.NEWTON, (N, N, N), h)
    t, w = O.sinc_nodes(O.NEWTON, 0.0, M, hu, s)
    for d in [(20, 0, 0), (30, 40, 0), (64, 64, 64), (300, 10, 5)]:
        r = math.sqrt(sum((di * h) ** 2 for di in d))
        ap = np.sum(w * np.prod([O.cell_average_gauss(t, di * h, h) for di in d], axis=0))
        assert abs(ap * r - 1.0) < 2e-5 + 10 * (h * math.sqrt(3) / r) ** 4


def test_golden_paper_ranks_are_in_range():
    # soft pins from the paper's Table Table_Times (canonical rank R at eps = 1e-6 grows
    # logarithmically from 34 to 43 for n = 4608..73768); our rank is M+1
    with open(os.path.join(GOLDEN, "paper_numbers.json")) as f:
        g = json.load(f)
    R = g["table_times"]["canonical_rank"]
    assert R == sorted(R) and R[0] >= 30 and R[-1] <= 45
    # our M = 40 Newton rule is inside that range
    t, _ = O.sinc_nodes(O.NEWTON, 0.0, 40, 0.35, 10.0)
    assert R[0] <= len(t) <= R[-1]


# ---------------------------------------------------------------------------------------
# error control of the sinc rule (Sec. 2.1, max-norm bound after eq. sinc_general)
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("kind,p", [(O.NEWTON, 0.0), (O.YUKAWA, 0.5), (O.SLATER, 1.0)])
def test_vector_exact_averages_match_scalar(kind, p):
    # the shared-subdivision vector quadrature against the per-cell adaptive one (pinned above
    # by the cube constant)
    h = 0.1
    disps = [(0, 0, 0), (1, 0, 0), (2, 1, 1), (7, 3, 0), (40, 20, 10)]
    vec = O.exact_cell_averages(kind, p, disps, h)
    one = np.array([O.exact_cell_average(kind, p, [x * h for x in d], h) for d in disps])
    assert np.max(np.abs(vec - one) / np.abs(one)) < 1e-11


def _signed_box(N):
    lim = [n - 1 for n in N]
    return [(i, j, k) for i in range(-lim[0], lim[0] + 1) for j in range(-lim[1], lim[1] + 1)
            for k in range(-lim[2], lim[2] + 1)]


@pytest.mark.parametrize("kind,p", [(O.NEWTON, 0.0), (O.SLATER, 2.0)])
def test_probe_cells_hold_every_entry_of_a_small_box(kind, p):
    # with N <= 5 per axis every entry of the signed doubled box (2N-1 per axis, both signs and
    # all axis orders) has a probe cell with the same sorted |displacements|: same maximum
    N, h = (5, 5, 3), 0.3
    full = _signed_box(N)
    ex = O.exact_cell_averages(kind, p, full, h)
    for M in (4, 8, 16):
        e_full = O.sinc_error(kind, p, M, N, h, cells=full, exact=ex)
        e_probe = O.sinc_error(kind, p, M, N, h)
        assert e_probe == pytest.approx(e_full, rel=1e-9)


@pytest.mark.parametrize("kind,p", [(O.NEWTON, 0.0), (O.SLATER, 1.0)])
def test_probe_cells_find_the_box_maximum(kind, p):
    # a non-cubic box where the probes are a small subset (66 of the 5049 cells of the positive
    # octant, which holds every entry up to sign): their maximum reaches the box maximum
    N, h = (33, 17, 9), 0.1
    lim = [n - 1 for n in N]
    full = [(i, j, k) for i in range(lim[0] + 1) for j in range(lim[1] + 1) for k in range(lim[2] + 1)]
    ex = O.exact_cell_averages(kind, p, full, h)
    for M in (8, 16, 24):
        e_full = O.sinc_error(kind, p, M, N, h, cells=full, exact=ex)
        e_probe = O.sinc_error(kind, p, M, N, h)
        assert 0.999 * e_full <= e_probe <= e_full * (1 + 1e-12)


def test_chosen_rank_grows_like_the_papers_table():
    # soft pin, Table Table_Times: at eps = 1e-6 the canonical rank of one Newton kernel grows
    # by 2-3 per doubling of n (34, 37, 39, 41, 43 for n = 4608..73728).  Our rule (fixed step
    # h_u, s a quarter of the box diagonal) needs about 1.2x the paper's rank and grows alike.
    with open(os.path.join(GOLDEN, "paper_numbers.json")) as f:
        g = json.load(f)["table_times"]
    ranks = []
    for n, R_paper in zip(g["grid_n"], g["canonical_rank"]):
        N = (n + 1,) * 3
        M, e = O.choose_M(O.NEWTON, 0.0, N, 10.0 / n, 1e-6, 128)
        assert M is not None and e <= 1e-6
        assert O.sinc_error(O.NEWTON, 0.0, M - 1, N, 10.0 / n) > 1e-6
        R = len(O.sinc_nodes(O.NEWTON, 0.0, M, *O.default_quadrature(O.NEWTON, N, 10.0 / n))[0])
        assert R_paper <= R <= 1.35 * R_paper
        ranks.append(R)
    steps = np.diff(ranks)
    assert np.all(steps >= 1) and np.all(steps <= 3)


def test_choose_M_reports_the_floor_of_the_step():
    # the step h_u bounds the accuracy (discretisation error of the trapezoid rule, Sec. 2.1
    # eq. sinc_conv): below that floor no M suffices; a finer step lowers it
    N, h = (257,) * 3, 1 / 16
    M, e = O.choose_M(O.NEWTON, 0.0, N, h, 1e-9, 96)
    assert M is None and e > 1e-9
    M2, e2 = O.choose_M(O.NEWTON, 0.0, N, h, 1e-9, 160, h_u=0.2)
    assert M2 is not None and e2 <= 1e-9


# ---------------------------------------------------------------------------------------
# eq. nuc_pot: Galerkin matrix in a Gaussian basis against its closed form
# ---------------------------------------------------------------------------------------

def _gauss_coulomb(alpha, A, C):
    # int exp(-a|x-A|^2) exp(-b|x-B|^2) / |x - C| dx = exp(-ab/p |A-B|^2) (2 pi / p) F0(p |P-C|^2),
    # p = a + b, P = (a A + b B) / p, F0(t) = sqrt(pi / t) erf(sqrt t) / 2
    nb = len(alpha)
    V = np.zeros((nb, nb))
    for k in range(nb):
        for m in range(nb):
            p = alpha[k] + alpha[m]
            P = (alpha[k] * A[k] + alpha[m] * A[m]) / p
            t = p * float(np.sum((P - C) ** 2))
            F0 = 1.0 if t < 1e-14 else 0.5 * math.sqrt(math.pi / t) * erf(math.sqrt(t))
            V[k, m] = math.exp(-alpha[k] * alpha[m] / p * float(np.sum((A[k] - A[m]) ** 2))) * 2 * math.pi / p * F0
    return V


def test_galerkin_matrix_converges_to_the_gaussian_closed_form():
    # one Newton charge: the grid functional with the basis at cell centres converges at O(h^2)
    import workloads as W
    alpha = np.array([1.0, 2.0, 1.5])
    A = np.array([[0.3, -0.2, 0.1], [-0.4, 0.5, 0.0], [0.0, 0.0, 0.6]])
    Vc = _gauss_coulomb(alpha, A, np.zeros(3))
    errs = []
    for N, h in [(49, 1 / 6), (97, 1 / 12)]:
        c = (N - 1) // 2
        p = W.Problem("g", W.NEWTON, 0.0, 40, (N, N, N), h, [W.Block((1, 1, 1), (1, 1, 1), (0, 0, 0))])
        x = (np.arange(N) - c) * h
        G = [np.exp(-alpha[:, None] * (x[None, :] - A[:, l][:, None]) ** 2) for l in range(3)]
        V = O.galerkin_matrix(O.brute_force_grid(p), G, h)
        assert np.array_equal(V, V.T)
        errs.append(np.max(np.abs(V - Vc) / np.abs(Vc)))
    assert errs[1] < 2e-3 and 3.0 < errs[0] / errs[1] < 5.0

"""Plain FP64 CPU oracle for grid-based canonical/Tucker lattice sums.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or runs this
module; only the tests, the smoke check and the CPU-baseline leg of the benchmark use
it.  It shares no code with the GPU path: the only common dependency is the seeded
input description in ``workloads``.

Every function follows a passage of
V. Khoromskaia, B. N. Khoromskij, "Tucker tensor method for fast grid-based summation
of long-range potentials on 3D lattices with defects" (arXiv:1411.1994), cited by
section / equation label.  The code favours being checkable by eye over speed: no
blocking, no fusion, no reordering beyond the definitions.

Readings of passages that are silent, ambiguous or garbled (each one is tested):

* sinc quadrature (Sec. 2.1, eqs. ``laplace``/``hM``): the trapezoid rule with step
  h_u is applied after the substitution t = sinh(u)/s, which makes the integrand even
  in u; the sum over k = -M..M is folded onto k = 0..M, so the rank is M+1 for Newton
  (the t = 0 node carries weight) and M for Yukawa/Slater.
* Yukawa transform (Sec. 2.2, eq. ``LalpYukawa``): the exponent of the weight is read as
  kappa^2/(4 t^2); as printed (kappa^2/t^2) the transform gives exp(-2 kappa r)/r.
* Galerkin basis (Sec. 2.1, eq. ``galten``): psi_i is the cell indicator divided by the
  cell volume, so tensor entries are cell averages (values of a potential).
* grid: odd N per axis, cell i centred at (i - (N-1)/2) h; the reference vector of
  length 2N-1 (the doubled box of Sec. 3.1, eq. ``master_pot``) has entry m at
  displacement (m - (N-1)) h, and a charge in cell c contributes entry i - c + N - 1 at
  cell i (the windowing operator of eq. ``sub_tens``, whose printed index range is
  inconsistent with the index set I_0).
* lattice (Sec. 3.2): site k of an axis sits at (k - (L-1)/2) b + centre; sites that do
  not fall on a cell centre are snapped to the nearest one, rounding halves away from
  zero (the paper assumes on-grid sites and accepts O(h) error otherwise).  With exact
  sites (``brute_force_points_exact``) each charge keeps its position: its Galerkin entries
  are the cell averages of its own shifted Gaussians (Sec. 3.1 footnote: nuclei anywhere).
* RHOSVD truncation (Sec. 4.3 allows a threshold instead of fixed ranks): per mode the
  smallest r with (sum_{k>r} sigma_k^2)^{1/2} <= eps ||A|| / (3 ||xi||), which by the
  bound of the Appendix theorem (d) certifies ||A - A0|| <= eps ||A|| in Frobenius norm.
* quadrature nodes whose weight is below 1e-18 of the largest weight are dropped.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np
from scipy.special import erf, erfc

NEWTON, YUKAWA, SLATER = 0, 1, 2

SQRT_PI = math.sqrt(math.pi)


class OutOfBox(ValueError):
    """A snapped site or sample point lies outside the grid."""


# ---------------------------------------------------------------------------------------
# Sec. 2.1-2.2: sinc quadrature of the Laplace-Gauss transform
# ---------------------------------------------------------------------------------------

def default_quadrature(kind: int, N: Sequence[int], h: float) -> Tuple[float, float]:
    """Default (h_u, s): s is a quarter of the largest charge-to-cell distance in the box,
    h_u a per-kernel step chosen to minimise the max-norm error at M = 32..40."""
    r_max = h * math.sqrt(sum(float(n - 1) ** 2 for n in N))
    s = r_max / 4.0
    h_u = 0.30 if kind == SLATER else 0.35
    return h_u, s


def transform_density(kind: int, param: float, t: np.ndarray) -> np.ndarray:
    """a(t) with p(z) = int_0^inf a(t) exp(-t^2 z^2) dt (Sec. 2.2):

    * Newton 1/z:           a = 2/sqrt(pi)                           (eq. LalpNewt)
    * Yukawa exp(-k z)/z:   a = 2/sqrt(pi) exp(-k^2/(4 t^2))         (eq. LalpYukawa, read)
    * Slater exp(-l z):     a = l/sqrt(pi) t^-2 exp(-l^2/(4 t^2))    (eq. LalpSlater with
      rho = z^2, kappa = l^2/4 and the change of variable t_paper = t^2)
    """
    t = np.asarray(t, dtype=np.float64)
    a = np.zeros_like(t)
    pos = t > 0
    if kind == NEWTON or (kind == YUKAWA and param == 0.0):
        a[:] = 2.0 / SQRT_PI
    elif kind == YUKAWA:
        a[pos] = 2.0 / SQRT_PI * np.exp(-param * param / (4.0 * t[pos] ** 2))
    elif kind == SLATER:
        if param <= 0:
            raise ValueError("Slater exponent must be positive")
        a[pos] = param / SQRT_PI / t[pos] ** 2 * np.exp(-param * param / (4.0 * t[pos] ** 2))
    else:
        raise ValueError(f"unknown kernel {kind}")
    return a


def sinc_nodes(kind: int, param: float, M: int, h_u: float, s: float):
    """Nodes t_q and weights w_q with p(z) ~= sum_q w_q exp(-t_q^2 z^2) (Sec. 2.1, eqs.
    ``laplace``, ``hM``, ``sinc_Newt``): trapezoid rule in u with t = sinh(u)/s on
    u_k = k h_u, k = -M..M, folded onto k >= 0 (k = 0 keeps half of the full step)."""
    if M < 1 or h_u <= 0 or s <= 0:
        raise ValueError("need M >= 1, h_u > 0, s > 0")
    k = np.arange(M + 1, dtype=np.float64)
    u = k * h_u
    t = np.sinh(u) / s
    dtdu = np.cosh(u) / s
    step = np.where(k == 0, 0.5 * h_u, h_u)
    w = step * transform_density(kind, param, t) * dtdu
    keep = w > 1e-18 * np.max(w)
    return t[keep], w[keep]


def kernel_value(kind: int, param: float, z):
    """The kernel p(z) itself (Sec. 2.2)."""
    z = np.asarray(z, dtype=np.float64)
    if kind == NEWTON:
        return 1.0 / z
    if kind == YUKAWA:
        return np.exp(-param * z) / z
    if kind == SLATER:
        return np.exp(-param * z)
    raise ValueError(kind)


# ---------------------------------------------------------------------------------------
# Sec. 2.1: Galerkin (cell-average) collocation of the Gaussians; Sec. 3.1 reference tensor
# ---------------------------------------------------------------------------------------

def cell_average_gauss(t, d, h: float) -> np.ndarray:
    """b(t; d) = (1/h) int_{d-h/2}^{d+h/2} exp(-t^2 x^2) dx, the entries of the vectors
    b(t_k) of Sec. 2.1 for cell-average basis functions.  Closed form
    sqrt(pi)/(2 t h) [erf(t(d+h/2)) - erf(t(d-h/2))], evaluated with erfc when both ends
    lie in the tail (t(|d|-h/2) > 1); equals 1 at t = 0.  Uses |d| (mirror symmetry)."""
    t = np.asarray(t, dtype=np.float64)
    d = np.abs(np.asarray(d, dtype=np.float64))
    t, d = np.broadcast_arrays(t, d)
    out = np.ones(t.shape, dtype=np.float64)
    pos = t > 0
    tp, dp = t[pos], d[pos]
    lo = tp * (dp - 0.5 * h)
    hi = tp * (dp + 0.5 * h)
    diff = np.where(lo > 1.0, erfc(lo) - erfc(hi), erf(hi) - erf(lo))
    out[pos] = SQRT_PI / (2.0 * tp * h) * diff
    return out


def reference_vectors(t: np.ndarray, w: np.ndarray, N: int, h: float, weighted: bool = True):
    """Reference canonical vectors on the doubled box (Sec. 3.1, eq. ``master_pot``; Sec. 3.2,
    eq. ``CanMastSumNL``): row q, entry m = w_q^(1/3) b(t_q; (m-(N-1)) h), m = 0..2N-2
    (p_q = a_q^{1/3} b(t_q) of Sec. 2.1).  ``weighted=False`` omits w_q^(1/3)."""
    m = np.arange(2 * N - 1)
    d = (m - (N - 1)).astype(np.float64) * h
    B = cell_average_gauss(t[:, None], d[None, :], h)
    if weighted:
        B = np.cbrt(w)[:, None] * B
    return B


# ---------------------------------------------------------------------------------------
# Sec. 3.1-3.2: lattice bookkeeping (shift-and-windowing offsets)
# ---------------------------------------------------------------------------------------

def snap(coord, h: float, N: int) -> np.ndarray:
    """Cell index of coordinate(s): j = sign(x/h) floor(|x/h| + 1/2), i = j + (N-1)/2.
    Raises OutOfBox unless 0 <= i <= N-1."""
    u = np.asarray(coord, dtype=np.float64) / h
    j = np.sign(u) * np.floor(np.abs(u) + 0.5)
    i = j + (N - 1) // 2
    if np.any(i < 0) or np.any(i > N - 1):
        raise OutOfBox("site outside the grid")
    return i.astype(np.int64)


def site_coords(L: int, b: float, center: float) -> np.ndarray:
    """Coordinates of the L sites of a centred lattice axis: (k - (L-1)/2) b + centre
    (Sec. 3.2, the set K read as centred)."""
    k = np.arange(L, dtype=np.float64)
    return (k - (L - 1) / 2.0) * b + center


def block_axis_coords(block, a: int) -> np.ndarray:
    """The coordinates of the block's sites along axis a: its explicit list when it has one (a
    non-equidistant tensor lattice, Sec. 4.4 case (D)), else the centred equidistant sites."""
    coords = getattr(block, "coords", None)
    if coords is not None and coords[a] is not None:
        return np.asarray(coords[a], dtype=np.float64)
    return site_coords(block.L[a], block.b[a], block.center[a])


def block_offsets(block, h: float, N: Sequence[int]) -> List[np.ndarray]:
    """Per axis, the snapped cell indices of the block's sites."""
    return [snap(block_axis_coords(block, a), h, N[a]) for a in range(3)]


def shear_sites(base, shear_axis: int, along_axis: int, shear: float) -> np.ndarray:
    """All sites (C,3) of a parallelogram-type lattice (Sec. 4.4 case (B)): the sites of ``base``
    with coordinate ``shear_axis`` moved by (k - (L-1)/2) shear, k the index along ``along_axis``."""
    axes = [block_axis_coords(base, a) for a in range(3)]
    idx = np.stack(np.meshgrid(*[np.arange(len(x)) for x in axes], indexing="ij"), axis=-1).reshape(-1, 3)
    pos = np.stack([axes[a][idx[:, a]] for a in range(3)], axis=1)
    half = (base.L[along_axis] - 1) / 2.0
    pos[:, shear_axis] += (idx[:, along_axis] - half) * shear
    return pos


def brute_force_points_at(problem, pts: np.ndarray, pos: np.ndarray, Z: np.ndarray) -> np.ndarray:
    """The plain sum of eq. ``EwaldSumE`` projected on the grid for an explicit list of charges:
    each charge snapped to its cell (as for blocks), V[p] = sum_c Z_c sum_q w_q prod_l
    b(t_q; (p_l - c_l) h)."""
    t, w = quadrature_of(problem)
    Nr = max(problem.N)
    table = reference_vectors(t, w, Nr, problem.h, weighted=False)
    cidx = np.stack([snap(pos[:, a], problem.h, problem.N[a]) for a in range(3)], axis=1)
    out = np.empty(len(pts))
    for n, p in enumerate(np.asarray(pts)):
        prod = (table[:, p[0] - cidx[:, 0] + Nr - 1] * table[:, p[1] - cidx[:, 1] + Nr - 1]
                * table[:, p[2] - cidx[:, 2] + Nr - 1])
        out[n] = np.sum(Z * (w @ prod))
    return out


def charges(problem) -> Tuple[np.ndarray, np.ndarray]:
    """All charges of the problem as (cell index triples (C,3), charge Z (C,)): the block's
    charge on every site of every block, changed by dZ at defect sites (Sec. 4.1)."""
    idx, Z = [], []
    for bi, blk in enumerate(problem.blocks):
        offs = block_offsets(blk, problem.h, problem.N)
        g = np.stack(np.meshgrid(*offs, indexing="ij"), axis=-1).reshape(-1, 3)
        z = np.full(g.shape[0], float(blk.charge))
        L = blk.L
        for d in problem.defects:
            if d.block == bi:
                z[(d.site[0] * L[1] + d.site[1]) * L[2] + d.site[2]] += d.dZ
        idx.append(g)
        Z.append(z)
    return np.concatenate(idx), np.concatenate(Z)


def quadrature_of(problem):
    h_u, s = problem.h_u, problem.s
    if h_u <= 0 or s <= 0:
        dh, ds = default_quadrature(problem.kind, problem.N, problem.h)
        h_u = h_u if h_u > 0 else dh
        s = s if s > 0 else ds
    return sinc_nodes(problem.kind, problem.param, problem.M, h_u, s)


# ---------------------------------------------------------------------------------------
# O1: brute-force sum over every charge (the plain definition, eq. ``EwaldSumE`` projected
# onto the grid with the separable Gaussian sum of eq. ``sinc_Newt``)
# ---------------------------------------------------------------------------------------

def brute_force_points(problem, pts: np.ndarray, t=None, w=None) -> np.ndarray:
    """V[p] = sum_c Z_c sum_q w_q prod_l b(t_q; (p_l - c_l) h) at cell-index triples pts (P,3).
    No factorisation over lattice axes: every charge is visited for every point."""
    if t is None:
        t, w = quadrature_of(problem)
    Nr = max(problem.N)
    table = reference_vectors(t, w, Nr, problem.h, weighted=False)   # b(t_q; m h), unweighted
    cidx, Z = charges(problem)
    out = np.empty(len(pts))
    for n, p in enumerate(np.asarray(pts)):
        prod = (table[:, p[0] - cidx[:, 0] + Nr - 1]
                * table[:, p[1] - cidx[:, 1] + Nr - 1]
                * table[:, p[2] - cidx[:, 2] + Nr - 1])          # (R, C)
        per_charge = w @ prod                                    # q inside
        out[n] = np.sum(Z * per_charge)                          # charges outside
    return out


def charge_positions(problem) -> Tuple[np.ndarray, np.ndarray]:
    """All charges at their exact coordinates (C,3), without snapping, with their charges Z (C,)
    (the same order and defect changes as ``charges``)."""
    pos, Z = [], []
    for bi, blk in enumerate(problem.blocks):
        axes = [block_axis_coords(blk, a) for a in range(3)]
        g = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3)
        z = np.full(g.shape[0], float(blk.charge))
        L = blk.L
        for d in problem.defects:
            if d.block == bi:
                z[(d.site[0] * L[1] + d.site[1]) * L[2] + d.site[2]] += d.dZ
        pos.append(g)
        Z.append(z)
    return np.concatenate(pos), np.concatenate(Z)


def brute_force_points_exact(problem, pts: np.ndarray, t=None, w=None) -> np.ndarray:
    """Charges at their exact positions y_c (the paper's nuclei anywhere in the box, Sec. 3.1):
    V[p] = sum_c Z_c sum_q w_q prod_l b(t_q; x_l(p) - y_c,l), x(p) the centre of cell p, i.e.
    the cell averages of eq. ``galten`` of the sinc sum of every charge, one charge at a time.
    Every site must still lie in a cell of the grid (as for snapping)."""
    if t is None:
        t, w = quadrature_of(problem)
    for blk in problem.blocks:
        block_offsets(blk, problem.h, problem.N)          # raises OutOfBox like the snapped path
    pos, Z = charge_positions(problem)
    h = problem.h
    # the distinct coordinates of each axis, and each charge's index into them
    axes = [np.unique(pos[:, a], return_inverse=True) for a in range(3)]
    out = np.empty(len(pts))
    for n, p in enumerate(np.asarray(pts)):
        prod = np.ones((len(t), len(Z)))
        for a in range(3):
            xa = (p[a] - (problem.N[a] - 1) // 2) * h
            ya, inv = axes[a]
            prod *= cell_average_gauss(t[:, None], (xa - ya)[None, :], h)[:, inv.reshape(-1)]
        out[n] = np.sum(Z * (w @ prod))
    return out


def brute_force_grid(problem, ranges=None, t=None, w=None) -> np.ndarray:
    """V on a full box of cells (all cells, or index ranges per axis), charge by charge."""
    if t is None:
        t, w = quadrature_of(problem)
    Nr = max(problem.N)
    if ranges is None:
        ranges = [np.arange(n) for n in problem.N]
    table = reference_vectors(t, w, Nr, problem.h, weighted=False)
    cidx, Z = charges(problem)
    V = np.zeros(tuple(len(r) for r in ranges))
    for c in range(len(Z)):
        if Z[c] == 0.0:
            continue
        f = [table[:, ranges[a] - cidx[c, a] + Nr - 1] for a in range(3)]
        V += Z[c] * np.einsum("q,qi,qj,qk->ijk", w, f[0], f[1], f[2], optimize=True)
    return V


# ---------------------------------------------------------------------------------------
# Thm ``thm:sumCaseE`` (A), eq. ``EwaldTensorGl``: assembled canonical lattice sum
# ---------------------------------------------------------------------------------------

def window(P_ref: np.ndarray, c: int, N_axis: int, N_ref: int) -> np.ndarray:
    """Shift-and-windowing of the reference vectors to a charge in cell c of an axis with
    N_axis cells (Sec. 3.1, eq. ``sub_tens``): entry i is P_ref[:, i - c + N_ref - 1]."""
    i = np.arange(N_axis)
    return P_ref[:, i - c + N_ref - 1]


def shift_sum(P_ref: np.ndarray, sites: np.ndarray, N_axis: int, N_ref: int) -> np.ndarray:
    """sum_k W_(k) p_q over the sites of one axis (the 1D sums of eq. ``EwaldTensorGl``)."""
    U = np.zeros((P_ref.shape[0], N_axis))
    for c in sites:
        U += window(P_ref, int(c), N_axis, N_ref)
    return U


def assembled_canonical(problem, t=None, w=None):
    """Per block, the rank-R factors [U_1, U_2, U_3] (each R x N_l) of the block's lattice sum
    (the block's charge is not applied)."""
    if t is None:
        t, w = quadrature_of(problem)
    Nr = max(problem.N)
    P = reference_vectors(t, w, Nr, problem.h)
    out = []
    for blk in problem.blocks:
        offs = block_offsets(blk, problem.h, problem.N)
        out.append([shift_sum(P, offs[a], problem.N[a], Nr) for a in range(3)])
    return out


def canonical_eval(factors: Sequence[np.ndarray], pts: np.ndarray, lam=None) -> np.ndarray:
    """sum_q lam_q prod_l U_l[q, p_l] at cell-index triples (canonical format, eq. ``CP_form``)."""
    pts = np.asarray(pts)
    prod = factors[0][:, pts[:, 0]] * factors[1][:, pts[:, 1]] * factors[2][:, pts[:, 2]]
    if lam is None:
        return prod.sum(axis=0)
    return lam @ prod


# ---------------------------------------------------------------------------------------
# Sec. 4.1-4.2: defected lattice as a sum of canonical tensors (eq. ``Can_LatticeSum_full``)
# ---------------------------------------------------------------------------------------

def canonical_terms(problem, t=None, w=None):
    """The rank-1 terms of P_hat = P_0 + sum_s P_s in the normalised form of eq. ``CP_form``:
    xi (Rhat,) and side matrices A_l (N_l x Rhat) with unit columns.  Terms: for every block
    and node q the block's assembled vectors times the block's charge; for every defect s
    and node q the windows of the reference vectors at the defect's cell, times dZ_s."""
    if t is None:
        t, w = quadrature_of(problem)
    Nr = max(problem.N)
    P = reference_vectors(t, w, Nr, problem.h)
    cols = [[], [], []]
    xi = []
    offs_all = [block_offsets(blk, problem.h, problem.N) for blk in problem.blocks]
    for blk, offs in zip(problem.blocks, offs_all):
        U = [shift_sum(P, offs[a], problem.N[a], Nr) for a in range(3)]
        nrm = [np.linalg.norm(U[a], axis=1) for a in range(3)]
        xi.append(blk.charge * nrm[0] * nrm[1] * nrm[2])
        for a in range(3):
            cols[a].append(U[a] / nrm[a][:, None])
    for d in problem.defects:
        offs = offs_all[d.block]
        Wv = [window(P, int(offs[a][d.site[a]]), problem.N[a], Nr) for a in range(3)]
        nrm = [np.linalg.norm(Wv[a], axis=1) for a in range(3)]
        xi.append(d.dZ * nrm[0] * nrm[1] * nrm[2])
        for a in range(3):
            cols[a].append(Wv[a] / nrm[a][:, None])
    xi = np.concatenate(xi)
    A = [np.concatenate(cols[a], axis=0).T for a in range(3)]   # N_l x Rhat
    return xi, A


def cp_norm(xi: np.ndarray, A: Sequence[np.ndarray]) -> float:
    """Frobenius norm of sum_v xi_v a1_v (x) a2_v (x) a3_v from the factor Gram matrices."""
    G = (A[0].T @ A[0]) * (A[1].T @ A[1]) * (A[2].T @ A[2])
    return float(math.sqrt(max(xi @ G @ xi, 0.0)))


def cp_full(xi: np.ndarray, A: Sequence[np.ndarray]) -> np.ndarray:
    """The full tensor of a canonical sum (tiny sizes only)."""
    return np.einsum("v,iv,jv,kv->ijk", xi, A[0], A[1], A[2], optimize=True)


# ---------------------------------------------------------------------------------------
# Definition ``def:RHOSVD`` and Appendix theorem ``thm:C2Tucker`` (c), (d)
# ---------------------------------------------------------------------------------------

@dataclass
class TuckerResult:
    Z: List[np.ndarray]          # N_l x r_l orthonormal
    core: np.ndarray             # r1 x r2 x r3
    sigma: List[np.ndarray]      # singular values of each side matrix
    ranks: Tuple[int, int, int]
    tails: Tuple[float, float, float]
    bound: float                 # ||xi|| sum_l tail_l (absolute)
    norm_A: float
    norm_xi: float


def tail_norms(sig: np.ndarray) -> np.ndarray:
    """tail[r] = (sum_{k >= r} sigma_k^2)^{1/2} for r = 0..len(sig) (0-based: drops k = r..)."""
    sq = sig.astype(np.float64) ** 2
    suffix = np.concatenate([np.cumsum(sq[::-1])[::-1], [0.0]])
    return np.sqrt(suffix)


def rhosvd(xi: np.ndarray, A: Sequence[np.ndarray], eps: float = None, ranks=None,
           norm_A: float = None) -> TuckerResult:
    """RHOSVD of a canonical tensor: truncated SVD of each side matrix A_l, the dominant left
    singular vectors Z_l as Tucker factors, and the core by canonical projection
    mu = sum_v xi_v (Z_1^T a1_v) (x) (Z_2^T a2_v) (x) (Z_3^T a3_v) (Appendix, (c)).
    Ranks are given, or chosen by the eps rule of the module docstring."""
    norm_xi = float(np.linalg.norm(xi))
    if norm_A is None:
        norm_A = cp_norm(xi, A)
    Zs, sigs, rs, tails = [], [], [], []
    for a in range(3):
        U, S, _ = np.linalg.svd(A[a], full_matrices=False)
        tl = tail_norms(S)
        if ranks is not None:
            r = int(ranks[a])
        else:
            thr = eps * norm_A / (3.0 * norm_xi)
            r = int(np.argmax(tl <= thr))         # smallest r with tail(r) <= thr
            r = max(r, 1)
        Zs.append(U[:, :r])
        sigs.append(S)
        rs.append(r)
        tails.append(float(tl[r]))
    Y = [Zs[a].T @ A[a] for a in range(3)]
    core = np.einsum("v,av,bv,cv->abc", xi, Y[0], Y[1], Y[2], optimize=True)
    bound = norm_xi * sum(tails)
    return TuckerResult(Zs, core, sigs, tuple(rs), tuple(tails), bound, norm_A, norm_xi)


def als_refine(xi: np.ndarray, A: Sequence[np.ndarray], Z: Sequence[np.ndarray], sweeps: int):
    """Thm ``thm:C2Tucker`` (b): ALS for the dual maximisation of ||sum_v xi_v (Y_1^T a1_v) (x)
    (Y_2^T a2_v) (x) (Y_3^T a3_v)|| over orthonormal Y_l, from the RHOSVD factors Z: each sweep
    visits the modes in order and takes the leading r_l left singular vectors of the mode-l matrix
    sum_v xi_v a_l,v (Y_a^T a_a,v (x) Y_b^T a_b,v)^T (the other modes at their latest factors).
    Returns (Z, core, [||core|| after each sweep]); ||A - Tucker||^2 = ||A||^2 - ||core||^2."""
    Z = [np.array(z) for z in Z]
    history = []
    core = None
    for _ in range(sweeps):
        for l in range(3):
            a, b = [m for m in range(3) if m != l]
            Pa, Pb = Z[a].T @ A[a], Z[b].T @ A[b]                          # r x R
            KR = np.einsum("iv,jv->ijv", Pa, Pb).reshape(-1, len(xi))      # (r_a r_b) x R
            M = (A[l] * xi[None, :]) @ KR.T                                  # N_l x (r_a r_b)
            U, _, _ = np.linalg.svd(M, full_matrices=False)
            Z[l] = U[:, :Z[l].shape[1]]
        Y = [Z[m].T @ A[m] for m in range(3)]
        core = np.einsum("v,av,bv,cv->abc", xi, Y[0], Y[1], Y[2], optimize=True)
        history.append(float(np.linalg.norm(core)))
    return Z, core, history


def tucker_to_canonical(core: np.ndarray, Z: Sequence[np.ndarray], eps: float):
    """Can -> Tuck -> Can (the rank reduction of a defected canonical sum through its Tucker form,
    Sec. 4.2): each mode-3 slice of the core by its SVD, mu[:, :, k] = sum_i s_i u_i v_i^T, gives
    the rank-1 terms s_i (Z_1 u_i) (x) (Z_2 v_i) (x) z_3,k, so the canonical rank is at most
    r_3 min(r_1, r_2).  With orthonormal Z_l these terms are mutually orthogonal: dropping the
    smallest s (over all slices, ties by slice then index) while the dropped (sum s^2)^(1/2)
    stays <= eps ||core|| bounds the Frobenius error by that.  Returns (xi, [A_1, A_2, A_3],
    error), A_l (N_l x R) with unit columns, terms by decreasing s."""
    terms = []
    for k in range(core.shape[2]):
        U, S, Vt = np.linalg.svd(core[:, :, k], full_matrices=False)
        for i in range(len(S)):
            terms.append((float(S[i]), k, i, U[:, i], Vt[i]))
    terms.sort(key=lambda t: (-t[0], t[1], t[2]))
    budget = (eps * float(np.linalg.norm(core))) ** 2
    dropped = 0.0
    keep = len(terms)
    while keep > 1 and dropped + terms[keep - 1][0] ** 2 <= budget:
        dropped += terms[keep - 1][0] ** 2
        keep -= 1
    kept = terms[:keep]
    xi = np.array([t[0] for t in kept])
    A = [np.stack([Z[0] @ t[3] for t in kept], axis=1), np.stack([Z[1] @ t[4] for t in kept], axis=1),
         np.stack([Z[2][:, t[1]] for t in kept], axis=1)]
    return xi, A, math.sqrt(dropped)


def tucker_full(core: np.ndarray, Z: Sequence[np.ndarray]) -> np.ndarray:
    """B x_1 T1 x_2 T2 x_3 T3 (eq. ``Tucker_singePot``) on the full grid (tiny sizes)."""
    return np.einsum("abc,ia,jb,kc->ijk", core, Z[0], Z[1], Z[2], optimize=True)


def tucker_tile(core: np.ndarray, Z: Sequence[np.ndarray], ranges) -> np.ndarray:
    """The Tucker tensor restricted to index ranges per axis."""
    return tucker_full(core, [Z[a][ranges[a], :] for a in range(3)])


def tucker_points(core: np.ndarray, Z: Sequence[np.ndarray], pts: np.ndarray) -> np.ndarray:
    """Tucker values at cell-index triples: sum_abc B_abc T1[p1,a] T2[p2,b] T3[p3,c]."""
    pts = np.asarray(pts)
    return np.einsum("abc,pa,pb,pc->p", core, Z[0][pts[:, 0]], Z[1][pts[:, 1]], Z[2][pts[:, 2]],
                     optimize=True)


# ---------------------------------------------------------------------------------------
# Thm ``thm:sumCaseE`` (B): the lattice sum from the Tucker form of the reference
# ---------------------------------------------------------------------------------------

def tucker_reference(problem) -> TuckerResult:
    """The rank-r Tucker form of the reference tensor on the doubled box (eq. ``TuckRef_sum``):
    RHOSVD at ``problem.eps`` of its canonical form (eq. ``CanMastSumNL``, the same R weighted
    reference vectors in every mode) written as in eq. ``CP_form``: unit columns, their norms
    in xi (as ``canonical_terms`` writes the lattice sum); with ``problem.als_sweeps`` ALS sweeps
    from that guess (the canonical-to-Tucker approximation of Thm ``thm:C2Tucker``)."""
    t, w = quadrature_of(problem)
    B = reference_vectors(t, w, max(problem.N), problem.h)           # R x (2 N_ref - 1)
    nrm = np.linalg.norm(B, axis=1)
    A = (B / nrm[:, None]).T
    res = rhosvd(nrm ** 3, [A, A, A], eps=problem.eps)
    sweeps = getattr(problem, "als_sweeps", 0)
    if sweeps:                                  # C2T: ALS from the RHOSVD guess (Thm C2Tucker (b))
        Z, core, _ = als_refine(nrm ** 3, [A, A, A], res.Z, sweeps)
        res = TuckerResult(Z, core, res.sigma, res.ranks, res.tails, res.bound, res.norm_A, res.norm_xi)
    return res


def tucker_lattice_sum(problem):
    """eq. ``Tuck_LatticeSum`` per block: the windowed sums of the reference Tucker vectors over
    the block's sites, made orthonormal by Gram-Schmidt (QR) with the triangular factors carried
    into the block's core (times its charge).  One block: that Tucker tensor.  Several blocks
    (the sum of Tucker tensors of eq. ``WindowTuck_sum``): the generalised RHOSVD of Thm
    ``thm:TSum2Tucker``, i.e. per mode the truncated SVD of the blocks' stacked factor columns
    (eq. ``SideMTuckS``), the smallest rank whose tail is <= eps ||U|| / (3 |B|) with
    |B|^2 = sum_b ||B_b||^2, so that the bound |B| sum_l tail_l of the theorem is <= eps ||U||,
    and the core by projection.  Returns (core, [Z_1, Z_2, Z_3], bound, norm), Z_l (N_l x k_l)
    with orthonormal columns, norm = ||U|| of the untruncated sum."""
    ref = tucker_reference(problem)
    Nr = max(problem.N)
    terms = []                                         # (core B_b, [Q_1, Q_2, Q_3])
    for blk in problem.blocks:
        offs = block_offsets(blk, problem.h, problem.N)
        Q, Rt = [], []
        for a in range(3):
            F = shift_sum(ref.Z[a].T, offs[a], problem.N[a], Nr)      # r_a x N_a
            q, rr = np.linalg.qr(F.T)
            Q.append(q)
            Rt.append(rr)
        B = blk.charge * np.einsum("ijk,ai,bj,ck->abc", ref.core, Rt[0], Rt[1], Rt[2], optimize=True)
        terms.append((B, Q))
    if len(terms) == 1:
        B, Q = terms[0]
        return B, Q, 0.0, float(np.linalg.norm(B))
    # ||U||^2 = sum_{b,b'} <T_b, T_b'>, each from the cross Grams of the factors
    norm2 = 0.0
    for Bb, Qb in terms:
        for Bc, Qc in terms:
            G = [Qb[a].T @ Qc[a] for a in range(3)]
            norm2 += float(np.einsum("ijk,abc,ia,jb,kc->", Bb, Bc, G[0], G[1], G[2], optimize=True))
    norm = math.sqrt(max(norm2, 0.0))
    Bhat = math.sqrt(sum(float(np.linalg.norm(B)) ** 2 for B, _ in terms))
    thr = problem.eps * norm / (3.0 * Bhat)
    Z, tails = [], []
    for a in range(3):
        U, S, _ = np.linalg.svd(np.concatenate([Q[a] for _, Q in terms], axis=1), full_matrices=False)
        tl = tail_norms(S)
        r = max(int(np.argmax(tl <= thr)), 1)
        Z.append(U[:, :r])
        tails.append(float(tl[r]))
    core = sum(np.einsum("ijk,ai,bj,ck->abc", B, Z[0].T @ Q[0], Z[1].T @ Q[1], Z[2].T @ Q[2], optimize=True)
               for B, Q in terms)
    return core, Z, Bhat * sum(tails), norm


# ---------------------------------------------------------------------------------------
# eq. ``nuc_pot``: the Galerkin matrix of the summed potential in a separable basis
# ---------------------------------------------------------------------------------------

def galerkin_matrix(T: np.ndarray, G: Sequence[np.ndarray], h: float) -> np.ndarray:
    """V[k, m] = h^3 sum_i T_i g_k(x_i) g_m(x_i) over every cell i of the full tensor T, with the
    separable basis functions given by their per-axis values at the cell centres, G[l]
    (nb x N_l): eq. ``nuc_pot`` read as the midpoint rule for the integral of v g_k g_m."""
    nb = G[0].shape[0]
    V = np.zeros((nb, nb))
    for k in range(nb):
        for m in range(nb):
            gkm = np.einsum("i,j,k->ijk", G[0][k] * G[0][m], G[1][k] * G[1][m], G[2][k] * G[2][m])
            V[k, m] = h ** 3 * float(np.sum(T * gkm))
    return V


# ---------------------------------------------------------------------------------------
# O3: the exact Galerkin entry (no sinc quadrature), by adaptive Gauss-Kronrod
# ---------------------------------------------------------------------------------------

def exact_cell_average(kind: int, param: float, d: Sequence[float], h: float) -> float:
    """(1/h^3) int_cell p(|x|) dx for the cell centred at displacement d (eq. ``galten`` with
    cell averages) written as int_0^inf a(t) prod_l b(t; d_l) dt (Sec. 2.1-2.2) and
    integrated numerically in v = log t."""
    from scipy.integrate import quad

    def f(v):
        t = math.exp(v)
        a = float(transform_density(kind, param, np.array([t]))[0])
        if a == 0.0:
            return 0.0
        b = 1.0
        for dl in d:
            b *= float(cell_average_gauss(np.array([t]), np.array([dl]), h)[0])
        return a * b * t

    edges = np.linspace(-30.0, 30.0, 61)
    total = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        total += quad(f, lo, hi, epsabs=0.0, epsrel=1e-12, limit=200)[0]
    return total


def exact_cell_averages(kind: int, param: float, disps, h: float) -> np.ndarray:
    """``exact_cell_average`` for many cells at once: the same integral in v = log t, done by
    scipy's adaptive vector quadrature (one subdivision shared by all cells).  ``disps`` holds
    displacements in units of h, one row per cell."""
    from scipy.integrate import quad_vec

    D = np.asarray(disps, dtype=np.float64) * h

    def f(v):
        t = math.exp(v)
        a = float(transform_density(kind, param, np.array([t]))[0])
        if a == 0.0:
            return np.zeros(len(D))
        return a * np.prod(cell_average_gauss(t, D, h), axis=1) * t

    return quad_vec(f, -40.0, 40.0, epsabs=0.0, epsrel=1e-13, limit=20000,
                    points=np.linspace(-40.0, 40.0, 81))[0]


# ---------------------------------------------------------------------------------------
# Sec. 2.1: error control of the sinc rule (max-norm bound after eq. sinc_general)
# ---------------------------------------------------------------------------------------

def sinc_probe_cells(N: Sequence[int]) -> List[Tuple[int, int, int]]:
    """Cells at which the max norm of P - P_R is taken (reading: the maximum over the whole
    doubled reference box, |i_l| <= N_l - 1, is estimated on these).  An entry depends only on
    the sorted absolute displacements, so cells are sorted triples a >= b >= c within the
    sorted limits: all with a <= 4, and along the directions (1, 0, 0), (1, 1, 0), (1, 1, 1),
    (1, 1/2, 0), (1, 1/2, 1/2), (1, 1, 1/2) the cells (m, floor(m d_2), floor(m d_3)), clipped
    to the limits, for m = 5, 8, 12, 18, ... (ceil(3m/2)) below the largest limit and at it."""
    lim = sorted((n - 1 for n in N), reverse=True)
    cells = set()
    for a in range(min(4, lim[0]) + 1):
        for b in range(min(a, lim[1]) + 1):
            for c in range(min(b, lim[2]) + 1):
                cells.add((a, b, c))
    ms = []
    m = 5
    while m < lim[0]:
        ms.append(m)
        m = math.ceil(3 * m / 2)
    ms.append(lim[0])
    halves = [(0, 0), (2, 0), (2, 2), (1, 0), (1, 1), (2, 1)]
    for m in ms:
        for d2, d3 in halves:
            cells.add((min(m, lim[0]), min(m * d2 // 2, lim[1]), min(m * d3 // 2, lim[2])))
    return sorted(cells)


def sinc_error(kind: int, param: float, M: int, N: Sequence[int], h: float, h_u=None, s=None,
               cells=None, exact=None) -> float:
    """max |P - P_R| / max |P| over ``cells`` (default: the probe cells), P the exact Galerkin
    entries of one unit charge, P_R the rule with M (Sec. 2.1 eq. sinc_general)."""
    du, ds = default_quadrature(kind, N, h)
    h_u = du if h_u is None else h_u
    s = ds if s is None else s
    cells = np.asarray(sinc_probe_cells(N) if cells is None else cells, dtype=np.float64)
    if exact is None:
        exact = exact_cell_averages(kind, param, cells, h)
    t, w = sinc_nodes(kind, param, M, h_u, s)
    approx = np.array([np.sum(w * np.prod(cell_average_gauss(t[:, None], c[None, :] * h, h), axis=1))
                       for c in cells])
    return float(np.max(np.abs(exact - approx)) / np.max(np.abs(exact)))


def choose_M(kind: int, param: float, N: Sequence[int], h: float, eps: float, M_max: int = 256,
             h_u=None, s=None):
    """The minimal M with sinc_error <= eps (Sec. 2.1), found by trying M = 1, 2, ...; returns
    (M, error), or (None, smallest error seen) when no M <= M_max reaches eps."""
    cells = sinc_probe_cells(N)
    exact = exact_cell_averages(kind, param, cells, h)
    best = math.inf
    for M in range(1, M_max + 1):
        e = sinc_error(kind, param, M, N, h, h_u, s, cells, exact)
        if e <= eps:
            return M, e
        best = min(best, e)
    return None, best


# ---------------------------------------------------------------------------------------
# the same method end to end (CPU, FP64)
# ---------------------------------------------------------------------------------------

def points_to_cells(xyz: np.ndarray, h: float, N: Sequence[int]) -> np.ndarray:
    """Cell index triples of sample points (same rounding as the sites)."""
    xyz = np.asarray(xyz, dtype=np.float64)
    return np.stack([snap(xyz[:, a], h, N[a]) for a in range(3)], axis=1)


def canonical_pipeline(problem, xyz: np.ndarray):
    """Nodes -> reference vectors -> 1D shift-sums -> potential at sample points, for a
    defect-free problem (the steps of Thm ``thm:sumCaseE`` (A))."""
    t, w = quadrature_of(problem)
    fac = assembled_canonical(problem, t, w)
    pts = points_to_cells(xyz, problem.h, problem.N)
    v = np.zeros(len(pts))
    for blk, f in zip(problem.blocks, fac):
        v += blk.charge * canonical_eval(f, pts)
    return fac, v

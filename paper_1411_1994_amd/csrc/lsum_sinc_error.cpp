// Error control of the sinc quadrature (Sec. 2.1, the max-norm bound that follows eq.
// sinc_general): the relative max-norm distance between the Galerkin tensor P of one unit
// charge and its R-term sinc approximation P_R, and the smallest M that brings it under a
// tolerance.  Host only, FP64.
//
// P is taken on the doubled reference box that the shift-and-windowing step reads (Sec. 3.1,
// eq. master_pot): every displacement (i, j, k) h with |i| <= N_1 - 1, |j| <= N_2 - 1,
// |k| <= N_3 - 1.  An entry depends only on the multiset {|i|, |j|, |k|} (isotropic kernel,
// cubic cells), so the maximum is estimated over sorted "probe" triples a >= b >= c that fit
// the sorted limits n_1 >= n_2 >= n_3 (n = N - 1):
//   * every triple with a <= 4 (the near field, where the truncation at large t shows), and
//   * along six directions (2, 0, 0), (2, 2, 0), (2, 2, 2), (2, 1, 0), (2, 1, 1), (2, 2, 1),
//     halved, the triples (m, floor(m d_2 / 2), floor(m d_3 / 2)) clipped per component to the
//     limits, for m = 5, then m <- ceil(3 m / 2) while m < n_1, and m = n_1 (the far field,
//     where the resolution of small t shows).
// The exact entries P(d) = int_0^inf a(t) prod_l b(t; d_l) dt (Sec. 2.1-2.2) are integrated by
// the trapezoid rule in v = log t: the integrand is analytic and decaying in the strip
// |Im v| < pi/4, where the rule with step 1/10 is accurate far below FP64 rounding; the range
// [log(1e-19 / D), log(1e10 / h)] (D the box diagonal) leaves tails below 1e-19 of max P.
#include <algorithm>
#include <array>
#include <cmath>
#include <vector>

#include "lsum_internal.h"

namespace lsum {
namespace {

// (1/h) int_{d-h/2}^{d+h/2} exp(-t^2 x^2) dx: the cell-average entry of the Gaussian (Sec. 2.1),
// from the error function (erfc when both ends lie in the tail); 1 at t = 0.
double gauss_cell_average(double t, double d, double h) {
    if (!(t > 0.0)) return 1.0;
    d = std::fabs(d);
    const double lo = t * (d - 0.5 * h), hi = t * (d + 0.5 * h);
    const double diff = lo > 1.0 ? std::erfc(lo) - std::erfc(hi) : std::erf(hi) - std::erf(lo);
    return std::sqrt(M_PI) / (2.0 * t * h) * diff;
}

struct Probes {
    std::vector<double> d;   // 3 displacements (times h) per probe
    int n = 0;
};

Probes probe_cells(const int N[3], double h) {
    int lim[3] = {N[0] - 1, N[1] - 1, N[2] - 1};
    std::sort(lim, lim + 3, [](int x, int y) { return x > y; });
    std::vector<std::array<int, 3>> cells;
    for (int a = 0; a <= std::min(4, lim[0]); ++a)
        for (int b = 0; b <= std::min(a, lim[1]); ++b)
            for (int c = 0; c <= std::min(b, lim[2]); ++c) cells.push_back({a, b, c});
    std::vector<int> ms;
    for (int m = 5; m < lim[0]; m = (3 * m + 1) / 2) ms.push_back(m);
    ms.push_back(lim[0]);
    static const int dir[6][2] = {{0, 0}, {2, 0}, {2, 2}, {1, 0}, {1, 1}, {2, 1}};
    for (int m : ms)
        for (const auto& e : dir)
            cells.push_back({std::min(m, lim[0]), std::min(m * e[0] / 2, lim[1]), std::min(m * e[1] / 2, lim[2])});
    std::sort(cells.begin(), cells.end());
    cells.erase(std::unique(cells.begin(), cells.end()), cells.end());
    Probes p;
    p.n = (int)cells.size();
    p.d.resize(3 * (size_t)p.n);
    for (int i = 0; i < p.n; ++i)
        for (int l = 0; l < 3; ++l) p.d[3 * (size_t)i + l] = (double)cells[i][l] * h;
    return p;
}

// prod_l b(t; d_l) for every probe
void gauss_products(double t, double h, const Probes& p, double* g) {
    for (int i = 0; i < p.n; ++i) {
        const double* d = &p.d[3 * (size_t)i];
        g[i] = gauss_cell_average(t, d[0], h) * gauss_cell_average(t, d[1], h) * gauss_cell_average(t, d[2], h);
    }
}

void exact_entries(int kind, double param, const int N[3], double h, const Probes& p, std::vector<double>& P) {
    double diag = 0.0;
    for (int l = 0; l < 3; ++l) diag += (double)N[l] * (double)N[l];
    diag = h * std::sqrt(diag);
    const double step = 0.1;
    const double v0 = std::log(1e-19 / diag), v1 = std::log(1e10 / h);
    const int n = (int)std::ceil((v1 - v0) / step);
    P.assign(p.n, 0.0);
    std::vector<double> g(p.n);
    for (int k = 0; k <= n; ++k) {
        const double t = std::exp(v0 + k * step);
        const double a = laplace_density(kind, param, t);
        if (a == 0.0) continue;
        gauss_products(t, h, p, g.data());
        const double f = step * a * t;   // dt = t dv
        for (int i = 0; i < p.n; ++i) P[i] += f * g[i];
    }
}

double max_rel_error(const std::vector<double>& P, const std::vector<double>& PR, double Pmax) {
    double e = 0.0;
    for (size_t i = 0; i < P.size(); ++i) e = std::max(e, std::fabs(P[i] - PR[i]));
    return e / Pmax;
}

int check_args(const lsum_kernel* k, const int N[3], double h) {
    if (!k || !N) return fail(LSUM_E_INVALID, "null argument");
    for (int l = 0; l < 3; ++l)
        if (N[l] < 1 || (N[l] % 2) == 0) return fail(LSUM_E_INVALID, "N must be odd");
    if (!(h > 0.0) || !std::isfinite(h)) return fail(LSUM_E_INVALID, "h must be positive");
    return LSUM_OK;
}

}  // namespace

int sinc_error_scan(const lsum_kernel& k, const int N[3], double h, double eps, int M_lo, int M_hi, int* M_out,
                    double* err_out) {
    double h_u = k.h_u, s = k.s, dh, ds;
    default_quadrature(k.kind, N, h, &dh, &ds);
    if (!(h_u > 0.0)) h_u = dh;
    if (!(s > 0.0)) s = ds;
    // validates kind, param, h_u, s and M_hi
    std::vector<double> t_all, w_all;
    int rc = sinc_nodes(k.kind, k.param, M_hi, h_u, s, t_all, w_all);
    if (rc != LSUM_OK) return rc;
    const Probes pr = probe_cells(N, h);
    std::vector<double> P;
    exact_entries(k.kind, k.param, N, h, pr, P);
    double Pmax = 0.0;
    for (double v : P) Pmax = std::max(Pmax, std::fabs(v));
    if (!(Pmax > 0.0)) return fail(LSUM_E_INVALID, "the kernel vanishes on the grid");

    // the folded rule of every M <= M_hi is the prefix j <= M of the rule of M_hi, with the
    // nodes below 1e-18 of its largest weight dropped (as the plan drops them)
    std::vector<double> tj(M_hi + 1), wj(M_hi + 1);
    sinc_rule(k.kind, k.param, M_hi, h_u, s, tj.data(), wj.data());
    std::vector<std::vector<double>> g(M_hi + 1);
    std::vector<double> PR(pr.n);
    int best_M = M_lo;
    double best = INFINITY;
    for (int M = M_lo; M <= M_hi; ++M) {
        double wmax = 0.0;
        for (int j = 0; j <= M; ++j) wmax = std::max(wmax, wj[j]);
        std::fill(PR.begin(), PR.end(), 0.0);
        for (int j = 0; j <= M; ++j) {
            if (!(wj[j] > 1e-18 * wmax)) continue;
            if (g[j].empty()) {
                g[j].resize(pr.n);
                gauss_products(tj[j], h, pr, g[j].data());
            }
            for (int i = 0; i < pr.n; ++i) PR[i] += wj[j] * g[j][i];
        }
        const double e = max_rel_error(P, PR, Pmax);
        if (e < best) {
            best = e;
            best_M = M;
        }
        if (e <= eps) {
            *M_out = M;
            *err_out = e;
            return LSUM_OK;
        }
    }
    *M_out = best_M;
    *err_out = best;
    return eps < 0.0 ? LSUM_OK : LSUM_E_NOCONV;
}

}  // namespace lsum

extern "C" {

int lsum_sinc_error(const lsum_kernel* k, const int N[3], double h, double* err) {
    int rc = lsum::check_args(k, N, h);
    if (rc != LSUM_OK) return rc;
    if (!err) return lsum::fail(LSUM_E_INVALID, "null argument");
    int M = 0;
    return lsum::sinc_error_scan(*k, N, h, -1.0, k->M, k->M, &M, err);
}

int lsum_choose_M(const lsum_kernel* k, const int N[3], double h, double eps, int M_max, int* M, double* err) {
    int rc = lsum::check_args(k, N, h);
    if (rc != LSUM_OK) return rc;
    if (!M || !err) return lsum::fail(LSUM_E_INVALID, "null argument");
    if (!(eps > 0.0)) return lsum::fail(LSUM_E_INVALID, "eps must be positive");
    if (M_max < 1 || M_max > 4096) return lsum::fail(LSUM_E_INVALID, "M_max must be in [1, 4096]");
    rc = lsum::sinc_error_scan(*k, N, h, eps, 1, M_max, M, err);
    if (rc == LSUM_E_NOCONV) lsum::fail(rc, "no M <= M_max reaches eps (the step h_u sets the error floor)");
    return rc;
}

}  // extern "C"

// Host-side steps of the lattice-sum path: FP64 quadrature nodes, integer snapping and the
// bookkeeping plan (side-matrix column sources, term groups, multiplicities).
// Compiled with -ffp-contract=off: every FP64 operation here is a single IEEE operation, so
// the snapped indices are reproducible bit for bit.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <set>
#include <tuple>
#include <vector>

#include "lsum_internal.h"

namespace lsum {

static thread_local std::string g_last_error;
static thread_local hipStream_t g_fail_stream = nullptr;

void set_error(const std::string& msg) { g_last_error = msg; }

// An error is raised where it is detected, before the caller unwinds: waiting here for the
// thread's stream means every kernel queued so far has finished before the unwinding returns
// its device buffers to the shared pool, from which another slot may take them at once.
int fail(int code, const std::string& msg) {
    g_last_error = msg;
    if (g_fail_stream) {
        (void)hipStreamSynchronize(g_fail_stream);
        (void)hipGetLastError();
    }
    return code;
}

FailStream::FailStream(hipStream_t st) : prev_(g_fail_stream) { g_fail_stream = st; }
FailStream::~FailStream() { g_fail_stream = prev_; }

const char* last_error() { return g_last_error.c_str(); }

// Default quadrature parameters: s is a quarter of the largest charge-to-cell distance of the
// box, h_u a per-kernel trapezoid step (chosen for the max-norm error at M = 32..40).
void default_quadrature(int kind, const int N[3], double h, double* h_u, double* s) {
    double acc = 0.0;
    for (int l = 0; l < 3; ++l) {
        double d = (double)(N[l] - 1);
        acc += d * d;
    }
    *s = h * std::sqrt(acc) / 4.0;
    *h_u = (kind == LSUM_SLATER) ? 0.30 : 0.35;
}

// Laplace-Gauss density a(t), p(z) = int_0^inf a(t) exp(-t^2 z^2) dt (Sec. 2.2):
// Newton 2/sqrt(pi); Yukawa 2/sqrt(pi) exp(-k^2/(4t^2)); Slater l/sqrt(pi) t^-2 exp(-l^2/(4t^2)).
double laplace_density(int kind, double param, double t) {
    const double two_over_sqrt_pi = 2.0 / std::sqrt(M_PI);
    if (kind == LSUM_NEWTON || (kind == LSUM_YUKAWA && param == 0.0)) return two_over_sqrt_pi;
    if (t <= 0.0) return 0.0;
    double e = std::exp(-param * param / (4.0 * (t * t)));
    if (kind == LSUM_YUKAWA) return two_over_sqrt_pi * e;
    return param / std::sqrt(M_PI) / (t * t) * e;   // Slater
}

void sinc_rule(int kind, double param, int M, double h_u, double s, double* t, double* w) {
    for (int k = 0; k <= M; ++k) {
        double u = (double)k * h_u;
        t[k] = std::sinh(u) / s;
        double step = (k == 0) ? 0.5 * h_u : h_u;
        w[k] = step * laplace_density(kind, param, t[k]) * (std::cosh(u) / s);
    }
}

// Sinc quadrature (Sec. 2.1, eqs. laplace, hM): trapezoid rule with step h_u in u after the
// substitution t = sinh(u)/s (even integrand), folded onto u_k = k h_u, k = 0..M.
int sinc_nodes(int kind, double param, int M, double h_u, double s, std::vector<double>& t,
               std::vector<double>& w) {
    if (kind < LSUM_NEWTON || kind > LSUM_SLATER) return fail(LSUM_E_INVALID, "unknown kernel");
    if (M < 1 || M > 4096) return fail(LSUM_E_INVALID, "M must be in [1, 4096]");
    if (!(h_u > 0.0) || !(s > 0.0)) return fail(LSUM_E_INVALID, "h_u and s must be positive");
    if (kind != LSUM_NEWTON && !(param >= 0.0)) return fail(LSUM_E_INVALID, "negative kernel parameter");
    if (kind == LSUM_SLATER && !(param > 0.0)) return fail(LSUM_E_INVALID, "Slater needs param > 0");
    std::vector<double> tt(M + 1), ww(M + 1);
    sinc_rule(kind, param, M, h_u, s, tt.data(), ww.data());
    double wmax = 0.0;
    for (int k = 0; k <= M; ++k) wmax = std::max(wmax, ww[k]);
    t.clear();
    w.clear();
    for (int k = 0; k <= M; ++k) {
        if (ww[k] > 1e-18 * wmax) {
            t.push_back(tt[k]);
            w.push_back(ww[k]);
        }
    }
    if (t.empty()) return fail(LSUM_E_INVALID, "no quadrature node carries weight");
    return LSUM_OK;
}

// Cell of a coordinate: j = sign(x/h) floor(|x/h| + 1/2) (halves away from zero), i = j + (N-1)/2.
int snap_coord(double x, double h, int N, int32_t* idx) {
    double u = x / h;
    double j = std::floor(std::fabs(u) + 0.5);
    if (u < 0.0) j = -j;
    double i = j + (double)((N - 1) / 2);
    if (!(i >= 0.0 && i <= (double)(N - 1))) return LSUM_E_OUT_OF_BOX;
    *idx = (int32_t)i;
    return LSUM_OK;
}

double site_x(const lsum_block& blk, int l, int k) {
    if (blk.x[l]) return blk.x[l][k];
    double half = (double)(blk.L[l] - 1) / 2.0;
    return ((double)k - half) * blk.b[l] + blk.center[l];
}

int block_offsets(const lsum_block& blk, const int N[3], double h, std::vector<int32_t> offs[3]) {
    for (int l = 0; l < 3; ++l) {
        if (blk.L[l] < 1) return fail(LSUM_E_INVALID, "block with L < 1");
        offs[l].resize(blk.L[l]);
        for (int k = 0; k < blk.L[l]; ++k) {
            double x = site_x(blk, l, k);
            if (!std::isfinite(x)) return fail(LSUM_E_INVALID, "site coordinate is not finite");
            int rc = snap_coord(x, h, N[l], &offs[l][k]);
            if (rc != LSUM_OK) return fail(rc, "lattice site outside the grid");
        }
    }
    return LSUM_OK;
}

void block_subcell(const lsum_block& blk, double h, std::vector<double> f[3]) {
    for (int l = 0; l < 3; ++l) {
        f[l].resize(blk.L[l]);
        for (int k = 0; k < blk.L[l]; ++k) {
            double x = site_x(blk, l, k);
            double u = x / h;
            double j = std::floor(std::fabs(u) + 0.5);
            if (u < 0.0) j = -j;
            f[l][k] = u - j;
        }
    }
}

void small_svd(const double* M, int m, int n, std::vector<double>& Ul, std::vector<double>& S,
               std::vector<double>& Vr) {
    // one-sided Jacobi on the columns of A = M (m >= n) or A = M^T (m < n), column-major
    const bool tr = m < n;
    const int rows = tr ? n : m, cols = tr ? m : n;
    std::vector<double> W((size_t)rows * cols), V((size_t)cols * cols, 0.0);
    for (int j = 0; j < cols; ++j) {
        V[(size_t)j * cols + j] = 1.0;
        for (int i = 0; i < rows; ++i) W[(size_t)j * rows + i] = tr ? M[(size_t)j * n + i] : M[(size_t)i * n + j];
    }
    for (int sweep = 0; sweep < 60; ++sweep) {
        bool rotated = false;
        for (int p = 0; p < cols; ++p)
            for (int q = p + 1; q < cols; ++q) {
                double* wp = &W[(size_t)p * rows];
                double* wq = &W[(size_t)q * rows];
                double alpha = 0.0, beta = 0.0, gamma = 0.0;
                for (int i = 0; i < rows; ++i) {
                    alpha += wp[i] * wp[i];
                    beta += wq[i] * wq[i];
                    gamma += wp[i] * wq[i];
                }
                if (!(std::fabs(gamma) > 1e-15 * std::sqrt(alpha * beta))) continue;
                rotated = true;
                const double zeta = (beta - alpha) / (2.0 * gamma);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
                for (int i = 0; i < rows; ++i) {
                    const double a = wp[i], b = wq[i];
                    wp[i] = c * a - sn * b;
                    wq[i] = sn * a + c * b;
                }
                double* vp = &V[(size_t)p * cols];
                double* vq = &V[(size_t)q * cols];
                for (int i = 0; i < cols; ++i) {
                    const double a = vp[i], b = vq[i];
                    vp[i] = c * a - sn * b;
                    vq[i] = sn * a + c * b;
                }
            }
        if (!rotated) break;
    }
    std::vector<double> nrm(cols);
    std::vector<int> ord(cols);
    for (int j = 0; j < cols; ++j) {
        double a = 0.0;
        for (int i = 0; i < rows; ++i) a += W[(size_t)j * rows + i] * W[(size_t)j * rows + i];
        nrm[j] = std::sqrt(a);
        ord[j] = j;
    }
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return nrm[x] > nrm[y]; });
    // A = U S V^T with U = W / S (rows x cols) and V (cols x cols); M = A or A^T
    const int k = cols;
    S.resize(k);
    Ul.assign((size_t)m * k, 0.0);
    Vr.assign((size_t)n * k, 0.0);
    for (int e = 0; e < k; ++e) {
        const int j = ord[e];
        S[e] = nrm[j];
        const double inv = nrm[j] > 0.0 ? 1.0 / nrm[j] : 0.0;
        for (int i = 0; i < rows; ++i) {
            const double u = W[(size_t)j * rows + i] * inv;
            if (tr) Vr[(size_t)e * n + i] = u;
            else Ul[(size_t)e * m + i] = u;
        }
        for (int i = 0; i < cols; ++i) {
            const double v = V[(size_t)j * cols + i];
            if (tr) Ul[(size_t)e * m + i] = v;
            else Vr[(size_t)e * n + i] = v;
        }
    }
}

size_t Plan::planned_bytes() const {
    size_t b = 0;
    size_t sumN = (size_t)N[0] + N[1] + N[2];
    b += (size_t)R * ldg * 8;                                  // reference rows (if not cached)
    if (off_grid()) b += 3 * cls_f.size() * (size_t)R * ldg * 8;   // class rows and their window sums
    if (tucker_ref()) b += 16 * (size_t)R * (4 * (size_t)N_ref) * 8;   // the reference's own RHOSVD
    b += blocks.size() * (size_t)ldt * sumN * 8;               // canonical factors (FP64 bound)
    if (tucker()) {
        size_t rmax[3];
        for (int l = 0; l < 3; ++l) {
            b += 2 * (size_t)D[l] * N[l] * 8;                  // raw + weighted columns
            rmax[l] = std::min<size_t>(std::min(D[l], N[l]), 1024);
            b += rmax[l] * N[l] * 8 * 2 + rmax[l] * D[l] * 8 * 2;   // Z, Y
            b += (size_t)n_groups * R * (rmax[l] + 4) * 8;         // term-major core operand
            b += (size_t)D[l] * D[l] * 8;                      // column Gram
        }
        b += rmax[0] * rmax[1] * rmax[2] * 8;                  // core
        if (2 * (size_t)D[2] <= (size_t)n_groups * R)          // grouped core terms (<= 2 GiB chunks of rows)
            b += std::min<size_t>(rmax[0] * rmax[1] * D[2] * 8, std::max<size_t>(2ull << 30, rmax[1] * (size_t)D[2] * 8));
        if (has_tile()) {
            size_t T0 = tile_T[0], T1 = tile_T[1], T2 = tile_T[2];
            size_t e = precision == LSUM_FP64 ? 8 : 4;
            b += (T0 * T1 * T2 + rmax[0] * rmax[1] * T2 + rmax[0] * T1 * T2) * e;
        }
    }
    return b + (16u << 20);
}

int comb_period(const int32_t* c, int n, int max_p, int* stride) {
    for (int p = 1; p <= max_p && p < n; ++p) {
        const int S = c[p] - c[0];
        if (S <= 0) continue;
        bool ok = true;
        for (int k = 0; k + p < n && ok; ++k) ok = (c[k + p] - c[k] == S);
        if (ok) {
            *stride = S;
            return p;
        }
    }
    return 0;
}

// Thm thm:sumCaseE (A) sums the reference row over every site of an axis.  Sites snapped from
// a lattice of spacing b on a grid of step h repeat with period p whenever b/h = S/p is
// rational: the axis is then p interleaved combs of stride S, and each comb is one window of
// the strided sums of the reference row (one term instead of n_j).
//
// When b/h has a large denominator (no period below n/2) the snapped sites still split into a
// few runs of one stride S (a convergent of b/h: the rounding drifts by one cell only every so
// many sites).  A run a, a + S, ..., a + (n - 1) S is the difference of two strided prefix sums
// Pb[x] = sum_{m >= 0, x - mS >= 0} g[x - mS] (two terms, whatever n), or of two strided suffix
// sums Pu[x] = sum_{m >= 0, x + mS < ldg} g[x + mS] when the prefix difference would read below
// the row; a run that fits neither is split between them.  This form is taken when it needs
// fewer terms than the sites (or the periodic combs).
namespace {

// the runs of stride S over the ascending sites u[0..n) (each in [0, expect.size() - S)):
// (first site, count), in order of their first site (greedy: a site extends the open run that
// expects it, else opens a run).  `expect` (site -> open run expecting it, or -1) enters and
// leaves all -1.
void stride_runs(const std::vector<int32_t>& u, int S, std::vector<int2>& runs, std::vector<int>& expect) {
    runs.clear();
    for (int32_t v : u) {
        int r = expect[v];
        if (r >= 0) {
            expect[v] = -1;
            ++runs[r].y;
        } else {
            r = (int)runs.size();
            runs.push_back(make_int2(v, 1));
        }
        if (expect[v + S] < 0) expect[v + S] = r;   // a run already expecting v + S keeps it (equal sites)
    }
    for (const int2& r : runs) expect[r.x + r.y * S] = -1;
}

// terms of one run of stride S on the prefix (tab 0) and suffix (tab 1) tables; bit 1 of tab
// marks a term that is subtracted.  lo_suffix is the first site a suffix run may start at.
// With S within the bound shift_terms sets, every term read i + off stays in [0, ldg) for
// i < max(N_axis, 2), and a run that fits neither form splits into one of each.
void run_terms(int a, int n, int S, int N_ref, int lo_suffix, std::vector<int2>& terms) {
    const int last = a + (n - 1) * S;
    if (last + S <= N_ref - 1) {   // prefix: Pb[y] - Pb[y - nS], y - nS >= 0
        terms.push_back(make_int2(N_ref - 1 - a, 0));
        terms.push_back(make_int2(N_ref - 1 - last - S, 2));
    } else if (a >= lo_suffix) {   // suffix: Pu[y - (n - 1) S] - Pu[y + S], y + S inside the row
        terms.push_back(make_int2(N_ref - 1 - last, 1));
        terms.push_back(make_int2(N_ref - 1 - a + S, 3));
    } else {                       // the sites up to N_ref - 1 - S on the prefix, the rest on the suffix
        const int j = (N_ref - 1 - S - a) / S;   // >= 0: a <= N_ref - 1 - S here
        run_terms(a, j + 1, S, N_ref, lo_suffix, terms);
        run_terms(a + (j + 1) * S, n - j - 1, S, N_ref, lo_suffix, terms);
    }
}

}  // namespace

void shift_terms(const int32_t* c, int n, int N_ref, int N_axis, int ldg, std::vector<int2>& terms, int* stride,
                 int n_tab[2], bool* two_tables) {
    terms.clear();
    *stride = 0;
    n_tab[0] = n_tab[1] = 0;
    *two_tables = false;
    int S = 0;
    const int period = n >= 4 ? comb_period(c, n, n / 2, &S) : 0;
    int best = period > 0 ? period : n;   // terms of the periodic combs, or of the sites
    int bestS = 0;
    std::vector<int2> runs;
    // strided runs: a stride S <= (ldg + 1 - max(N, 2)) / 2 lets every run take the prefix or the
    // suffix form (split at most once).  The search (tens of microseconds for ~100 sites) is
    // skipped where it cannot pay: few sites, or a short period whose comb form already reads at
    // most 8 entries (a stream of small canonical requests spends a few microseconds of host time
    // per request in all).
    const int Nr = std::max(N_axis, 2);
    const int S_max = (ldg + 1 - Nr) / 2;
    const int lo_suffix = N_ref + Nr - 1 - ldg;   // + S: the first site a suffix run may start at
    if (n >= 6 && !(period > 0 && period <= 8) && S_max >= 1) {
        std::vector<int32_t> u(c, c + n);
        std::sort(u.begin(), u.end());
        // candidate strides: the distances from three anchor sites to the next 16 (an outlying
        // first site does not hide the lattice's stride; a stride of a few lattice spacings, a
        // convergent of b/h, is among them)
        std::vector<int> cand;
        for (int a : {0, n / 3, (2 * n) / 3})
            for (int p = 1; p <= 16 && a + p < n; ++p) {
                const int d = u[a + p] - u[a];
                if (d >= 1 && d <= S_max && std::find(cand.begin(), cand.end(), d) == cand.end()) cand.push_back(d);
            }
        int S_top = 0;
        for (int d : cand) S_top = std::max(S_top, d);
        std::vector<int> expect((size_t)u.back() + S_top + 2, -1);
        for (int d : cand) {
            stride_runs(u, d, runs, expect);
            int cost = 0;
            for (const int2& r : runs) {
                const int last = r.x + (r.y - 1) * d;
                cost += (last + d <= N_ref - 1 || r.x >= lo_suffix + d) ? 2 : 4;
            }
            if (cost < best) {
                best = cost;
                bestS = d;
            }
        }
        if (bestS > 0) {
            stride_runs(u, bestS, runs, expect);
            for (const int2& r : runs) run_terms(r.x, r.y, bestS, N_ref, lo_suffix + bestS, terms);
            *stride = bestS;
            n_tab[0] = kPrefixSums;
            n_tab[1] = kSuffixSums;
            for (const int2& t : terms) *two_tables = *two_tables || (t.y & 1);
            return;
        }
    }
    if (period > 0) {
        const int hi = (n + period - 1) / period;
        for (int j = 0; j < period; ++j) {
            const int nj = (n - j + period - 1) / period;
            terms.push_back(make_int2(N_ref - 1 - c[j], nj == hi ? 0 : 1));
            if (nj != hi) *two_tables = true;
        }
        *stride = S;
        n_tab[0] = hi;
        n_tab[1] = hi - 1;
        return;
    }
    for (int k = 0; k < n; ++k) terms.push_back(make_int2(N_ref - 1 - c[k], 0));
}

int make_plan(const lsum_problem& p, Plan& plan) {
    plan = Plan();
    plan.kernel = p.kernel;
    for (int l = 0; l < 3; ++l) {
        if (p.N[l] < 1 || (p.N[l] % 2) == 0) return fail(LSUM_E_INVALID, "N must be odd and positive");
        if (p.N[l] > (1 << 20)) return fail(LSUM_E_INVALID, "N too large");
        plan.N[l] = p.N[l];
        plan.tile_lo[l] = p.tile_lo[l];
        plan.tile_T[l] = p.tile_T[l];
    }
    if (!(p.h > 0.0) || !std::isfinite(p.h)) return fail(LSUM_E_INVALID, "h must be positive");
    plan.h = p.h;
    if (p.n_blocks < 1 || !p.blocks) return fail(LSUM_E_INVALID, "need at least one block");
    if (p.n_defects < 0 || (p.n_defects > 0 && !p.defects)) return fail(LSUM_E_INVALID, "bad defect list");
    if (!(p.eps < 1.0) || std::isnan(p.eps)) return fail(LSUM_E_INVALID, "eps must be < 1");
    if (p.precision < LSUM_FP64 || p.precision > LSUM_BF16X3) return fail(LSUM_E_INVALID, "bad precision");
    plan.eps = p.eps;
    plan.precision = p.precision;
    if (p.method != LSUM_SUM_CANONICAL && p.method != LSUM_SUM_TUCKER_REF) return fail(LSUM_E_INVALID, "unknown method");
    plan.method = p.method;
    if (p.als_sweeps < 0 || p.als_sweeps > 64) return fail(LSUM_E_INVALID, "als_sweeps must be in [0, 64]");
    plan.als_sweeps = p.als_sweeps;
    if (p.method == LSUM_SUM_TUCKER_REF &&
        (!(p.eps > 0.0) || p.precision != LSUM_FP64 || p.n_defects > 0 || p.exact_sites))
        return fail(LSUM_E_INVALID, "the Tucker-reference sum needs eps > 0, FP64, no defects and snapped sites");
    plan.blocks.assign(p.blocks, p.blocks + p.n_blocks);
    for (auto& b : plan.blocks)   // explicit coordinates are read below, while the caller's arrays live
        for (int l = 0; l < 3; ++l) b.x[l] = nullptr;
    plan.defects.assign(p.defects, p.defects + p.n_defects);
    if (plan.has_tile()) {
        if (!plan.tucker()) return fail(LSUM_E_INVALID, "a tile needs eps > 0 (Tucker output)");
        for (int l = 0; l < 3; ++l)
            if (p.tile_lo[l] < 0 || p.tile_lo[l] + p.tile_T[l] > p.N[l])
                return fail(LSUM_E_INVALID, "tile outside the grid");
    }

    // quadrature
    double h_u = p.kernel.h_u, s = p.kernel.s, dh, ds;
    default_quadrature(p.kernel.kind, p.N, p.h, &dh, &ds);
    if (!(h_u > 0.0)) h_u = dh;
    if (!(s > 0.0)) s = ds;
    plan.h_u = h_u;
    plan.s = s;
    int rc = sinc_nodes(p.kernel.kind, p.kernel.param, p.kernel.M, h_u, s, plan.t, plan.w);
    if (rc != LSUM_OK) return rc;
    plan.R = (int)plan.t.size();
    plan.N_ref = std::max(p.N[0], std::max(p.N[1], p.N[2]));
    plan.ldg = ((2 * plan.N_ref - 1) + 7) / 8 * 8;
    plan.ldt = (plan.R + 15) / 16 * 16;

    // snapping
    const int nb = p.n_blocks;
    for (int l = 0; l < 3; ++l) plan.offs[l].resize(nb);
    for (int b = 0; b < nb; ++b) {
        if (!std::isfinite(p.blocks[b].charge)) return fail(LSUM_E_INVALID, "bad block charge");
        std::vector<int32_t> o[3];
        rc = block_offsets(p.blocks[b], p.N, p.h, o);
        if (rc != LSUM_OK) return rc;
        for (int l = 0; l < 3; ++l) plan.offs[l][b] = std::move(o[l]);
    }
    // exact sites: classes of sub-cell offsets, shared by all axes (the rows depend on f only).
    // Offsets within kClassTol of 0 are on the cell centre (class 0); the others, sorted, form
    // classes that start at their smallest offset and take every offset within kClassTol of it,
    // so sites that differ only by the rounding of x / h share rows (the class's first offset).
    plan.exact_sites = p.exact_sites ? 1 : 0;
    if (plan.exact_sites) {
        const double kClassTol = 1.0 / 1073741824.0;   // 2^-30
        std::vector<std::vector<double>> f[3];
        for (int l = 0; l < 3; ++l) f[l].resize(nb);
        std::vector<double> all;
        for (int b = 0; b < nb; ++b) {
            std::vector<double> fb[3];
            block_subcell(p.blocks[b], p.h, fb);
            for (int l = 0; l < 3; ++l) {
                for (double v : fb[l])
                    if (std::fabs(v) > kClassTol) all.push_back(v);
                f[l][b] = std::move(fb[l]);
            }
        }
        std::sort(all.begin(), all.end());
        std::vector<double> starts;
        for (double v : all)
            if (starts.empty() || v - starts.back() > kClassTol) starts.push_back(v);
        if (!starts.empty()) {
            plan.cls_f.assign(1, 0.0);
            plan.cls_f.insert(plan.cls_f.end(), starts.begin(), starts.end());
            if ((double)plan.cls_f.size() * plan.R * plan.ldg > (double)(1 << 30))
                return fail(LSUM_E_INVALID, "too many sub-cell offset classes for the row tables");
            for (int l = 0; l < 3; ++l) {
                plan.cls[l].resize(nb);
                for (int b = 0; b < nb; ++b) {
                    plan.cls[l][b].resize(f[l][b].size());
                    for (size_t k = 0; k < f[l][b].size(); ++k) {
                        const double v = f[l][b][k];
                        plan.cls[l][b][k] =
                            std::fabs(v) <= kClassTol
                                ? 0
                                : (int)(std::upper_bound(starts.begin(), starts.end(), v) - starts.begin());
                    }
                }
            }
        }
    }
    // defects: validation and duplicate detection
    std::set<std::tuple<int, int, int, int>> seen;
    for (const auto& d : plan.defects) {
        if (d.block < 0 || d.block >= nb) return fail(LSUM_E_INVALID, "defect block out of range");
        for (int l = 0; l < 3; ++l)
            if (d.site[l] < 0 || d.site[l] >= p.blocks[d.block].L[l])
                return fail(LSUM_E_OUT_OF_BOX, "defect site outside its block");
        if (!std::isfinite(d.dZ)) return fail(LSUM_E_INVALID, "bad defect charge");
        auto key = std::make_tuple(d.block, d.site[0], d.site[1], d.site[2]);
        if (!seen.insert(key).second) return fail(LSUM_E_DUP_DEFECT, "two defects at the same site");
    }

    // column sources per mode and term groups (blocks, then defects)
    plan.n_groups = nb + (int)plan.defects.size();
    plan.g_scale.resize(plan.n_groups);
    for (int b = 0; b < nb; ++b) plan.g_scale[b] = p.blocks[b].charge;
    for (size_t s2 = 0; s2 < plan.defects.size(); ++s2) plan.g_scale[nb + s2] = plan.defects[s2].dZ;
    for (int l = 0; l < 3; ++l) {
        plan.g_src[l].assign(plan.n_groups, -1);
        // lattice sources: distinct offset lists (cells, then classes when off grid)
        std::map<std::vector<int32_t>, int> lat;
        for (int b = 0; b < nb; ++b) {
            std::vector<int32_t> key = plan.offs[l][b];
            if (plan.off_grid()) key.insert(key.end(), plan.cls[l][b].begin(), plan.cls[l][b].end());
            auto it = lat.find(key);
            if (it == lat.end()) {
                int id = (int)plan.lat_block[l].size();
                lat.emplace(std::move(key), id);
                plan.lat_block[l].push_back(b);
                plan.g_src[l][b] = id;
            } else {
                plan.g_src[l][b] = it->second;
            }
        }
        plan.n_lat[l] = (int)plan.lat_block[l].size();
        // window sources: distinct defect (cell, class) pairs
        std::map<std::pair<int32_t, int32_t>, int> win;
        for (size_t s2 = 0; s2 < plan.defects.size(); ++s2) {
            const auto& d = plan.defects[s2];
            int32_t cell = plan.offs[l][d.block][d.site[l]];
            int32_t cl = plan.site_cls(l, d.block, d.site[l]);
            auto it = win.find({cell, cl});
            int id;
            if (it == win.end()) {
                id = (int)plan.win_cell[l].size();
                win.emplace(std::make_pair(cell, cl), id);
                plan.win_cell[l].push_back(cell);
                plan.win_cls[l].push_back(cl);
            } else {
                id = it->second;
            }
            plan.g_src[l][nb + s2] = plan.n_lat[l] + id;
        }
        plan.n_win[l] = (int)plan.win_cell[l].size();
        plan.src_mult[l].assign(plan.n_lat[l] + plan.n_win[l], 0);
        for (int g = 0; g < plan.n_groups; ++g) plan.src_mult[l][plan.g_src[l][g]] += 1;
        plan.D[l] = plan.R * (plan.n_lat[l] + plan.n_win[l]);
    }
    return LSUM_OK;
}

}  // namespace lsum

// ------------------------------------------------------------------------------------------
// C ABI: host-side steps
// ------------------------------------------------------------------------------------------
extern "C" {

const char* lsum_last_error(void) { return lsum::last_error(); }

int lsum_nodes(const lsum_kernel* k, const int N[3], double h, double* t, double* w, int cap, int* R) {
    if (!k || !N || !t || !w || !R) return lsum::fail(LSUM_E_INVALID, "null argument");
    double h_u = k->h_u, s = k->s, dh, ds;
    lsum::default_quadrature(k->kind, N, h, &dh, &ds);
    if (!(h_u > 0.0)) h_u = dh;
    if (!(s > 0.0)) s = ds;
    std::vector<double> tt, ww;
    int rc = lsum::sinc_nodes(k->kind, k->param, k->M, h_u, s, tt, ww);
    if (rc != LSUM_OK) return rc;
    if ((int)tt.size() > cap) return lsum::fail(LSUM_E_INVALID, "output capacity too small");
    std::memcpy(t, tt.data(), tt.size() * sizeof(double));
    std::memcpy(w, ww.data(), ww.size() * sizeof(double));
    *R = (int)tt.size();
    return LSUM_OK;
}

int lsum_shear_blocks(const lsum_block* base, int shear_axis, int along_axis, double shear, int cap,
                      lsum_block* out, int* n) {
    if (!base || !n) return lsum::fail(LSUM_E_INVALID, "null argument");
    if (shear_axis < 0 || shear_axis > 2 || along_axis < 0 || along_axis > 2 || shear_axis == along_axis)
        return lsum::fail(LSUM_E_INVALID, "the shear and along axes must be two different axes");
    if (base->x[shear_axis]) return lsum::fail(LSUM_E_INVALID, "explicit coordinates on the sheared axis");
    if (!std::isfinite(shear)) return lsum::fail(LSUM_E_INVALID, "shear is not finite");
    const int La = base->L[along_axis];
    if (La < 1) return lsum::fail(LSUM_E_INVALID, "block with L < 1");
    *n = La;
    if (!out) return LSUM_OK;
    if (cap < La) return lsum::fail(LSUM_E_INVALID, "output capacity below the number of blocks");
    const double half = (double)(La - 1) / 2.0;
    for (int k = 0; k < La; ++k) {
        lsum_block b = *base;
        b.L[along_axis] = 1;
        b.center[along_axis] = lsum::site_x(*base, along_axis, k);
        b.x[along_axis] = nullptr;
        b.center[shear_axis] = base->center[shear_axis] + ((double)k - half) * shear;
        out[k] = b;
    }
    return LSUM_OK;
}

int lsum_column_blocks(const lsum_block* base, int axis, int n, const double* pts, int cap, lsum_block* out) {
    if (!base || (n > 0 && (!pts || !out))) return lsum::fail(LSUM_E_INVALID, "null argument");
    if (axis < 0 || axis > 2) return lsum::fail(LSUM_E_INVALID, "bad axis");
    if (n < 0 || cap < n) return lsum::fail(LSUM_E_INVALID, "output capacity below the number of points");
    const int a = axis == 0 ? 1 : 0, b = axis == 2 ? 1 : 2;
    for (int k = 0; k < n; ++k) {
        if (!std::isfinite(pts[2 * k]) || !std::isfinite(pts[2 * k + 1]))
            return lsum::fail(LSUM_E_INVALID, "point coordinate is not finite");
        lsum_block blk = *base;
        blk.L[a] = blk.L[b] = 1;
        blk.x[a] = blk.x[b] = nullptr;
        blk.center[a] = pts[2 * k];
        blk.center[b] = pts[2 * k + 1];
        out[k] = blk;
    }
    return LSUM_OK;
}

int lsum_block_offsets(const lsum_block* blk, const int N[3], double h, int32_t* offs) {
    if (!blk || !N || !offs) return lsum::fail(LSUM_E_INVALID, "null argument");
    for (int l = 0; l < 3; ++l)
        if (N[l] < 1 || (N[l] % 2) == 0) return lsum::fail(LSUM_E_INVALID, "N must be odd");
    std::vector<int32_t> o[3];
    int rc = lsum::block_offsets(*blk, N, h, o);
    if (rc != LSUM_OK) return rc;
    size_t pos = 0;
    for (int l = 0; l < 3; ++l) {
        std::memcpy(offs + pos, o[l].data(), o[l].size() * sizeof(int32_t));
        pos += o[l].size();
    }
    return LSUM_OK;
}

}  // extern "C"

// Host self-test of the library's host-side steps, built with AddressSanitizer and
// UndefinedBehaviorSanitizer (host code only, no device work): the sinc quadrature (Sec. 2.1,
// 2.2), the snapped site offsets (Sec. 3.2), the lattice classes (Sec. 4.4 cases (B), (C), (D)),
// the sinc error control and choice of M, the request plan a context builds from a problem
// (deduplicated side-matrix sources, comb decomposition of the shift-sums, defect windows,
// exact-site classes), and the autotuner's decision file.  Every entry point is called with
// valid and with invalid arguments; the checks below are properties any correct result has.
// Exit status 0 when every check holds; the sanitizers abort on the first memory or undefined-
// behaviour error.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "lsum_internal.h"

namespace {

using lsum::make_plan;
using lsum::Plan;
using lsum::Tuner;

int g_checks = 0, g_failed = 0;

void check(bool ok, const char* what) {
    ++g_checks;
    if (!ok) {
        ++g_failed;
        std::fprintf(stderr, "FAILED: %s (%s)\n", what, lsum_last_error());
    }
}

lsum_kernel kernel(int kind, double param, int M) {
    lsum_kernel k{};
    k.kind = kind;
    k.param = param;
    k.M = M;
    return k;
}

lsum_block block(int L0, int L1, int L2, double b, double cx, double cy, double cz, double charge = 1.0) {
    lsum_block blk{};
    blk.L[0] = L0;
    blk.L[1] = L1;
    blk.L[2] = L2;
    blk.b[0] = blk.b[1] = blk.b[2] = b;
    blk.center[0] = cx;
    blk.center[1] = cy;
    blk.center[2] = cz;
    blk.charge = charge;
    return blk;
}

lsum_problem problem(const lsum_kernel& k, const int N[3], double h, const std::vector<lsum_block>& blocks,
                     const std::vector<lsum_defect>& defects, double eps) {
    lsum_problem p{};
    p.kernel = k;
    for (int l = 0; l < 3; ++l) p.N[l] = N[l];
    p.h = h;
    p.n_blocks = (int)blocks.size();
    p.blocks = blocks.empty() ? nullptr : blocks.data();
    p.n_defects = (int)defects.size();
    p.defects = defects.empty() ? nullptr : defects.data();
    p.eps = eps;
    p.precision = LSUM_FP64;
    return p;
}

void test_nodes() {
    const int N[3] = {65, 63, 61};
    for (int kind : {LSUM_NEWTON, LSUM_YUKAWA, LSUM_SLATER}) {
        for (int M : {1, 8, 32, 64}) {
            const lsum_kernel k = kernel(kind, kind == LSUM_NEWTON ? 0.0 : 0.7, M);
            std::vector<double> t(M + 1), w(M + 1);
            int R = -1;
            check(lsum_nodes(&k, N, 0.2, t.data(), w.data(), M + 1, &R) == LSUM_OK, "nodes");
            check(R >= 1 && R <= M + 1, "node count within M + 1");
            bool pos = true, inc = true;
            for (int q = 0; q < R; ++q) {
                pos = pos && w[q] > 0.0 && std::isfinite(w[q]) && t[q] >= 0.0;
                if (q > 0) inc = inc && t[q] > t[q - 1];
            }
            check(pos, "positive finite weights");
            check(inc, "increasing nodes");
            int R2 = -1;
            check(lsum_nodes(&k, N, 0.2, t.data(), w.data(), 0, &R2) != LSUM_OK || R2 == 0, "zero capacity");
        }
    }
    const lsum_kernel bad = kernel(7, 0.0, 10);
    double t[16], w[16];
    int R = 0;
    check(lsum_nodes(&bad, N, 0.2, t, w, 16, &R) != LSUM_OK, "unknown kernel rejected");
    check(lsum_nodes(nullptr, N, 0.2, t, w, 16, &R) != LSUM_OK, "null kernel rejected");
}

void test_offsets(std::mt19937_64& rng) {
    std::uniform_int_distribution<int> Ld(1, 40);
    std::uniform_real_distribution<double> bd(0.3, 2.5), cd(-3.0, 3.0);
    const int N[3] = {257, 255, 129};
    const double h = 0.1;
    for (int trial = 0; trial < 300; ++trial) {
        lsum_block blk = block(Ld(rng), Ld(rng), Ld(rng), bd(rng), cd(rng), cd(rng), cd(rng));
        std::vector<int32_t> offs(blk.L[0] + blk.L[1] + blk.L[2], -7);
        const int rc = lsum_block_offsets(&blk, N, h, offs.data());
        if (rc != LSUM_OK) continue;   // a lattice wider than the grid is rejected
        bool in = true, mono = true;
        int base = 0;
        for (int l = 0; l < 3; ++l) {
            for (int k = 0; k < blk.L[l]; ++k) {
                in = in && offs[base + k] >= 0 && offs[base + k] < N[l];
                if (k > 0) mono = mono && offs[base + k] >= offs[base + k - 1];
            }
            base += blk.L[l];
        }
        check(in, "offsets inside the grid");
        check(mono, "offsets non-decreasing along an axis");
    }
    // explicit coordinates (Sec. 4.4 case (D))
    std::vector<double> xs = {-1.0, -0.25, 0.5, 2.0};
    lsum_block blk = block(4, 1, 1, 1.0, 0, 0, 0);
    blk.x[0] = xs.data();
    int32_t offs[6];
    check(lsum_block_offsets(&blk, N, h, offs) == LSUM_OK, "explicit coordinates");
    check(offs[0] < offs[1] && offs[1] < offs[2] && offs[2] < offs[3], "explicit coordinates ordered");
    lsum_block wide = block(4000, 1, 1, 1.0, 0, 0, 0);
    std::vector<int32_t> big(4002);
    check(lsum_block_offsets(&wide, N, h, big.data()) != LSUM_OK, "lattice beyond the grid rejected");
    check(lsum_block_offsets(nullptr, N, h, offs) != LSUM_OK, "null block rejected");
}

void test_classes() {
    const lsum_block base = block(5, 4, 3, 1.0, 0.1, -0.2, 0.3);
    std::vector<lsum_block> out(8);
    int n = 0;
    check(lsum_shear_blocks(&base, 0, 1, 0.5, (int)out.size(), out.data(), &n) == LSUM_OK, "shear blocks");
    check(n == base.L[1], "one block per site along the along-axis");
    bool ok = true;
    for (int k = 0; k < n; ++k) ok = ok && out[k].L[1] == 1 && out[k].L[0] == base.L[0] && out[k].L[2] == base.L[2];
    check(ok, "shear blocks are single-site rows");
    check(lsum_shear_blocks(&base, 0, 0, 0.5, (int)out.size(), out.data(), &n) != LSUM_OK, "equal axes rejected");
    check(lsum_shear_blocks(&base, 0, 1, 0.5, 2, out.data(), &n) != LSUM_OK, "capacity below the block count rejected");
    const double pts[6] = {0.0, 0.0, 1.5, -0.5, -2.0, 1.0};
    check(lsum_column_blocks(&base, 2, 3, pts, (int)out.size(), out.data()) == LSUM_OK, "column blocks");
    check(out[1].L[0] == 1 && out[1].L[1] == 1 && out[1].L[2] == base.L[2], "column blocks keep the column axis");
    check(lsum_column_blocks(&base, 2, 3, pts, 2, out.data()) != LSUM_OK, "column capacity rejected");
}

void test_sinc_error() {
    const int N[3] = {33, 33, 33};
    for (int kind : {LSUM_NEWTON, LSUM_YUKAWA, LSUM_SLATER}) {
        const lsum_kernel k = kernel(kind, kind == LSUM_NEWTON ? 0.0 : 0.5, 16);
        double e16 = -1.0, e32 = -1.0;
        check(lsum_sinc_error(&k, N, 0.25, &e16) == LSUM_OK && e16 >= 0.0 && std::isfinite(e16), "sinc error");
        const lsum_kernel k32 = kernel(kind, k.param, 32);
        check(lsum_sinc_error(&k32, N, 0.25, &e32) == LSUM_OK && e32 <= e16 * 1.0001 + 1e-15, "more nodes, no larger error");
        int M = 0;
        double err = -1.0;
        const int rc = lsum_choose_M(&k, N, 0.25, 1e-6, 256, &M, &err);
        check((rc == LSUM_OK && err <= 1e-6) || rc == LSUM_E_NOCONV, "choice of M");
        check(M >= 1 && M <= 256, "chosen M in range");
    }
}

void test_plans(std::mt19937_64& rng) {
    const int N[3] = {129, 127, 121};
    const lsum_kernel k = kernel(LSUM_NEWTON, 0.0, 24);
    std::vector<lsum_block> blocks = {block(8, 7, 6, 1.0, 0.05, -0.1, 0.2), block(3, 3, 2, 1.3, 2.0, -1.5, 1.0, 0.5)};
    std::vector<lsum_defect> defects;   // 40 distinct sites of block 0
    std::vector<int> sites(8 * 7 * 6);
    for (int i = 0; i < (int)sites.size(); ++i) sites[i] = i;
    std::shuffle(sites.begin(), sites.end(), rng);
    for (int d = 0; d < 40; ++d) {
        lsum_defect df{};
        df.block = 0;
        df.site[0] = sites[d] / 42;
        df.site[1] = (sites[d] / 6) % 7;
        df.site[2] = sites[d] % 6;
        df.dZ = d % 2 ? -1.0 : 0.4;
        defects.push_back(df);
    }
    for (int exact : {0, 1}) {
        for (double eps : {0.0, 1e-6}) {
            lsum_problem p = problem(k, N, 0.11, blocks, defects, eps);
            p.exact_sites = exact;
            Plan plan;
            check(make_plan(p, plan) == LSUM_OK, "plan of a valid problem");
            check(plan.R >= 1 && (int)plan.t.size() == plan.R && (int)plan.w.size() == plan.R, "plan quadrature");
            check(plan.n_groups >= (int)blocks.size(), "term groups cover the blocks");
            bool src_ok = true;
            for (int l = 0; l < 3; ++l)
                for (int g = 0; g < plan.n_groups; ++g)
                    src_ok = src_ok && plan.g_src[l][g] >= 0 && plan.g_src[l][g] < plan.n_lat[l] + plan.n_win[l];
            check(src_ok, "every group's sources exist");
            check(plan.planned_bytes() > 0, "planned bytes");
        }
    }
    // invalid problems: each one rejected with an error, none read out of bounds
    {
        lsum_problem p = problem(k, N, 0.11, blocks, defects, 0.0);
        Plan plan;
        int even[3] = {128, 127, 121};
        lsum_problem q = p;
        for (int l = 0; l < 3; ++l) q.N[l] = even[l];
        check(make_plan(q, plan) != LSUM_OK, "even N rejected");
        q = p;
        q.h = -1.0;
        check(make_plan(q, plan) != LSUM_OK, "negative h rejected");
        q = p;
        q.n_blocks = 0;
        check(make_plan(q, plan) != LSUM_OK, "no blocks rejected");
        q = p;
        q.eps = 1.5;
        check(make_plan(q, plan) != LSUM_OK, "eps >= 1 rejected");
        q = p;
        q.precision = 9;
        check(make_plan(q, plan) != LSUM_OK, "unknown precision rejected");
        std::vector<lsum_defect> bad = defects;
        bad[3].site[0] = 99;
        q = problem(k, N, 0.11, blocks, bad, 0.0);
        check(make_plan(q, plan) != LSUM_OK, "defect site outside its block rejected");
        bad = defects;
        bad[9] = bad[8];
        q = problem(k, N, 0.11, blocks, bad, 0.0);
        check(make_plan(q, plan) != LSUM_OK, "two defects at one site rejected");
        bad = defects;
        bad[5].block = 7;
        q = problem(k, N, 0.11, blocks, bad, 0.0);
        check(make_plan(q, plan) != LSUM_OK, "defect of a missing block rejected");
        q = p;
        q.method = LSUM_SUM_TUCKER_REF;   // needs eps > 0 and no defects
        check(make_plan(q, plan) != LSUM_OK, "Tucker-reference sum with defects and eps 0 rejected");
        q = p;
        q.als_sweeps = 65;
        check(make_plan(q, plan) != LSUM_OK, "too many ALS sweeps rejected");
    }
}

void test_tuner() {
    const std::string path = std::string(std::getenv("TMPDIR") ? std::getenv("TMPDIR") : "/tmp") + "/lsum_selftest_tune.txt";
    std::remove(path.c_str());
    {
        Tuner t;
        t.set_device_tag("dev-a");
        check(t.use_file(path) == LSUM_OK, "tuner file (absent)");
        check(t.get("bucket/1") == -1, "no decision yet");
        check(t.put("bucket/1", {3.0, 1.0, -1.0, 2.0}) == 1, "fastest variant chosen");
        check(t.put("bucket/2", {-1.0, 5.0}) == 1, "unmeasured variants skipped");
        check(t.get("bucket/1") == 1, "decision kept");
    }
    {
        Tuner t;
        t.set_device_tag("dev-a");
        check(t.use_file(path) == LSUM_OK, "tuner file read back");
        check(t.get("bucket/1") == 1 && t.get("bucket/2") == 1, "decisions read back");
        check(t.json().find("bucket/2") != std::string::npos, "decisions in JSON");
    }
    {
        Tuner t;
        t.set_device_tag("dev-b");   // another device's decisions are not taken
        check(t.use_file(path) == LSUM_OK && t.get("bucket/1") == -1, "other device ignored");
    }
    if (FILE* f = std::fopen(path.c_str(), "a")) {   // malformed lines are skipped
        std::fputs("dev-a bucket/3\ndev-a bucket/4 7 1.0 2.0\ngarbage\n\n", f);
        std::fclose(f);
    }
    {
        Tuner t;
        t.set_device_tag("dev-a");
        check(t.use_file(path) == LSUM_OK && t.get("bucket/3") == -1 && t.get("bucket/4") == -1, "malformed lines skipped");
    }
    std::remove(path.c_str());
}

}  // namespace

// The terms of an axis (Thm thm:sumCaseE (A)) reproduce the direct sum over its sites exactly:
// rows of integers (exact in FP64), the tables built here from their stated definitions (window
// sums, strided prefix and suffix sums), every term read checked inside the row, and the terms
// never more than the sites.  Site lists: snapped lattices with b/h of small and of large
// denominator (the served mix's b/h = (N - 1) / (L + 16)), periodic combs, and random sites
// with repeats.
void test_shift_terms(std::mt19937_64& rng) {
    auto table = [](const std::vector<double>& g, int R, int ldg, int S, int n) {
        std::vector<double> Q((size_t)R * ldg, 0.0);
        for (int q = 0; q < R; ++q)
            for (int x = 0; x < ldg; ++x) {
                double a = 0.0;
                if (n > 0) {
                    for (int m = 0; m < n && x - m * S >= 0; ++m) a += g[(size_t)q * ldg + x - m * S];
                } else if (n == lsum::kPrefixSums) {
                    for (int y = x; y >= 0; y -= S) a += g[(size_t)q * ldg + y];
                } else {
                    for (int y = x; y < ldg; y += S) a += g[(size_t)q * ldg + y];
                }
                Q[(size_t)q * ldg + x] = a;
            }
        return Q;
    };
    int fewer = 0, strided = 0;
    for (int it = 0; it < 160; ++it) {
        const int N_ref = 2 * (int)(rng() % 700) + 1 + (it % 7 == 0 ? 0 : 4);
        const int N_axis = std::max(1, N_ref - 2 * (int)(rng() % 40));
        const int ldg = std::max(2, 2 * N_ref - 1) + (int)(rng() % 8);
        std::vector<int32_t> c;
        const int kind = it % 4;
        if (kind == 0 || kind == 1) {
            // a snapped lattice: L sites at spacing beta cells (kind 1: b/h = (N - 1) / (L + 16))
            const int L = 3 + (int)(rng() % 100);
            const double beta = kind == 1 ? (double)(N_axis - 1) / (L + 16)
                                          : 1.0 + std::uniform_real_distribution<double>(0.0, 40.0)(rng);
            const double c0 = 0.5 * (N_axis - 1);
            for (int k = 0; k < L; ++k) {
                const double x = (k - 0.5 * (L - 1)) * beta;
                const long v = std::lround(c0 + x);
                if (v >= 0 && v < N_axis) c.push_back((int32_t)v);
            }
        } else if (kind == 2) {   // periodic combs: b/h = P / Q
            const int P = 1 + (int)(rng() % 60), Qd = 1 + (int)(rng() % 6), L = 4 + (int)(rng() % 60);
            for (int k = 0; k < L; ++k) {
                const long v = (long)k * P / Qd;
                if (v < N_axis) c.push_back((int32_t)v);
            }
        } else {                  // random sites, repeats allowed, unsorted
            const int n = (int)(rng() % 90);
            for (int k = 0; k < n; ++k) c.push_back((int32_t)(rng() % N_axis));
        }
        const int n = (int)c.size();
        std::vector<int2> terms;
        int stride = 0, n_tab[2] = {0, 0};
        bool two = false;
        lsum::shift_terms(c.data(), n, N_ref, N_axis, ldg, terms, &stride, n_tab, &two);
        check((int)terms.size() <= std::max(n, 0), "no more terms than sites");
        if ((int)terms.size() < n) ++fewer;
        if (n_tab[0] == lsum::kPrefixSums) ++strided;
        const int R = 2;
        std::vector<double> g((size_t)R * ldg, 0.0);
        for (int q = 0; q < R; ++q)
            for (int x = 0; x < 2 * N_ref - 1; ++x) g[(size_t)q * ldg + x] = (double)((long)(rng() % 2001) - 1000);
        std::vector<double> T0 = g, T1 = g;
        if (stride > 0) {
            T0 = table(g, R, ldg, stride, n_tab[0]);
            T1 = table(g, R, ldg, stride, n_tab[1]);
        }
        bool inside = true, exact = true, tab_ok = true;
        const int Nr = std::max(N_axis, 2);
        for (const int2& t : terms) {
            inside = inside && t.x >= 0 && t.x + Nr - 1 < ldg;
            tab_ok = tab_ok && t.y >= 0 && t.y <= 3 && (two || !(t.y & 1)) && (stride > 0 || t.y == 0);
        }
        check(inside, "every term reads inside the row");
        check(tab_ok, "term tables and signs as announced");
        if (!inside || !tab_ok) continue;
        for (int q = 0; q < R; ++q)
            for (int i = 0; i < N_axis; ++i) {
                double direct = 0.0, sum = 0.0;
                for (int k = 0; k < n; ++k) direct += g[(size_t)q * ldg + i + N_ref - 1 - c[k]];
                for (const int2& t : terms) {
                    const double v = ((t.y & 1) ? T1 : T0)[(size_t)q * ldg + i + t.x];
                    sum += (t.y & 2) ? -v : v;
                }
                exact = exact && sum == direct;
            }
        check(exact, "terms reproduce the direct sum over the sites");
    }
    // a lattice whose snapped sites repeat with a short period keeps its comb form, one term per
    // comb (the 64^3 lattice on the 4097 grid: b/h = 51.2, five combs of 64 sites)
    {
        std::vector<int32_t> c;
        for (int k = 0; k < 64; ++k) {
            const double x = (k - 31.5) * 51.2;
            const double j = std::floor(std::fabs(x) + 0.5);
            c.push_back((int32_t)((x < 0 ? -j : j) + 2048));
        }
        std::vector<int2> terms;
        int stride = 0, n_tab[2] = {0, 0};
        bool two = false;
        lsum::shift_terms(c.data(), 64, 4097, 4097, 8200, terms, &stride, n_tab, &two);
        check(terms.size() == 5 && stride == 256 && n_tab[0] == 13 && n_tab[1] == 12,
              "a period-5 lattice keeps its five combs");
    }
    std::printf("shift terms: %d of 160 axes with fewer terms than sites, %d on strided runs\n", fewer, strided);
    check(fewer > 40, "most lattices need fewer terms than sites");
    check(strided > 10, "strided runs are taken for lattices without a short period");
}

int main() {
    std::mt19937_64 rng(1411);
    test_nodes();
    test_offsets(rng);
    test_classes();
    test_sinc_error();
    test_plans(rng);
    test_shift_terms(rng);
    test_tuner();
    std::printf("host self-test: %d checks, %d failed\n", g_checks, g_failed);
    return g_failed ? 1 : 0;
}

// C ABI of the lattice-sum library (include/lsum.h): context and request lifecycle, results,
// options, profile, and the stage-level entry points used to test each kernel family.
#include "lsum_runtime.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <sstream>

using namespace lsum;

struct lsum_ctx_s {
    std::shared_ptr<Context> sp;
    Context& c;
    lsum_ctx_s() : sp(std::make_shared<Context>()), c(*sp) {}
};
struct lsum_req_s {
    Request q;
};

extern "C" {

int lsum_create(lsum_ctx* out, int device, size_t budget, int n_slots) {
    if (!out) return fail(LSUM_E_INVALID, "null ctx pointer");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        return fail(LSUM_E_DEVICE, "no HIP device available");
    }
    if (device < 0 || device >= ndev) return fail(LSUM_E_INVALID, "bad device index");
    LSUM_HIP(hipSetDevice(device));
    size_t fr = 0, tot = 0;
    LSUM_HIP(hipMemGetInfo(&fr, &tot));
    auto* x = new lsum_ctx_s();
    Context& c = x->c;
    c.device = device;
    c.budget = budget ? budget : (size_t)(0.8 * (double)fr);
    c.n_slots = n_slots > 0 ? n_slots : 4;
    c.pool = new DevPool();
    {
        // the autotuner's decisions hold for devices of the same architecture and size
        hipDeviceProp_t prop{};
        if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
            std::string arch(prop.gcnArchName);
            const size_t colon = arch.find(':');
            if (colon != std::string::npos) arch.resize(colon);
            c.tuner.set_device_tag(arch + "-" + std::to_string(prop.multiProcessorCount) + "cu");
        } else {
            (void)hipGetLastError();
            c.tuner.set_device_tag("unknown");
        }
    }
    if (hipStreamCreateWithFlags(&c.own_stream, hipStreamNonBlocking) != hipSuccess) {
        c.own_stream = nullptr;
        delete x;
        return fail(LSUM_E_DEVICE, "stream creation failed");
    }
    for (int i = 0; i < c.n_slots; ++i) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            delete x;
            return fail(LSUM_E_DEVICE, "stream creation failed");
        }
        c.streams.push_back(s);
    }
    // auxiliary streams after the slot streams: HIP spreads streams over its hardware queues in
    // creation order, so the slots take distinct queues first
    for (int i = 0; i < 3 * c.n_slots; ++i) {
        hipStream_t a = nullptr;
        if (hipStreamCreateWithFlags(&a, hipStreamNonBlocking) != hipSuccess) {
            delete x;
            return fail(LSUM_E_DEVICE, "stream creation failed");
        }
        c.aux.push_back(a);
    }
    for (int i = 0; i < c.n_slots; ++i) c.workers.emplace_back(worker, &c, i);
    *out = x;
    return LSUM_OK;
}

int lsum_destroy(lsum_ctx x) {
    if (!x) return LSUM_OK;
    Context& c = x->c;
    {
        std::lock_guard<std::mutex> lk(c.mu);
        c.stopping = true;
    }
    c.cv.notify_all();
    for (auto& t : c.workers) t.join();
    c.workers.clear();
    // streams, caches and the pool go when the last unreleased request lets go of the context
    delete x;
    return LSUM_OK;
}

// a validated, planned request that is not queued yet
// The fields make_plan reads, appended one by one (no struct padding), as a cache key.
static bool plan_key(const lsum_problem& p, std::string& key) {
    if (p.n_blocks < 1 || !p.blocks || p.n_blocks > 64 || p.n_defects < 0 || p.n_defects > 4096 ||
        (p.n_defects > 0 && !p.defects))
        return false;
    auto put = [&](const void* v, size_t n) { key.append((const char*)v, n); };
    put(&p.kernel.kind, sizeof(int));
    put(&p.kernel.param, sizeof(double));
    put(&p.kernel.M, sizeof(int));
    put(&p.kernel.h_u, sizeof(double));
    put(&p.kernel.s, sizeof(double));
    put(p.N, sizeof(p.N));
    put(&p.h, sizeof(double));
    put(&p.eps, sizeof(double));
    put(&p.precision, sizeof(int));
    put(p.tile_lo, sizeof(p.tile_lo));
    put(p.tile_T, sizeof(p.tile_T));
    put(&p.exact_sites, sizeof(int));
    put(&p.method, sizeof(int));
    put(&p.als_sweeps, sizeof(int));
    put(&p.n_blocks, sizeof(int));
    for (int b = 0; b < p.n_blocks; ++b) {
        const lsum_block& k = p.blocks[b];
        put(k.L, sizeof(k.L));
        put(k.b, sizeof(k.b));
        put(k.center, sizeof(k.center));
        put(&k.charge, sizeof(double));
        for (int l = 0; l < 3; ++l) {
            const char f = k.x[l] ? 1 : 0;
            put(&f, 1);
            if (k.x[l]) put(k.x[l], (size_t)std::max(0, k.L[l]) * sizeof(double));
        }
    }
    put(&p.n_defects, sizeof(int));
    for (int d = 0; d < p.n_defects; ++d) {
        const lsum_defect& k = p.defects[d];
        put(&k.block, sizeof(int));
        put(k.site, sizeof(k.site));
        put(&k.dZ, sizeof(double));
    }
    return true;
}

// The plan of a problem: from the context's cache when the same problem was planned before.
static int plan_for(Context& c, const lsum_problem& p, std::shared_ptr<const Plan>& out) {
    std::string key;
    const bool cacheable = plan_key(p, key);
    if (cacheable) {
        std::lock_guard<std::mutex> lk(c.plan_mu);
        auto it = c.plans.find(key);
        if (it != c.plans.end()) {
            out = it->second;
            return LSUM_OK;
        }
    }
    auto made = std::make_shared<Plan>();
    const int rc = make_plan(p, *made);
    if (rc != LSUM_OK) return rc;
    out = made;
    if (!cacheable) return LSUM_OK;
    std::lock_guard<std::mutex> lk(c.plan_mu);
    if (c.plans.size() >= 256) c.plans.clear();
    c.plans.emplace(std::move(key), out);
    return LSUM_OK;
}

static int prepare_request(lsum_ctx x, const lsum_problem* p, lsum_req_s** out) {
    auto* r = new lsum_req_s();
    Request& q = r->q;
    q.ctx_ref = x->sp;
    q.ctx = &x->c;
    int rc = plan_for(x->c, *p, q.plan_sp);
    if (rc != LSUM_OK) {
        delete r;
        return rc;
    }
    if (p->n_points < 0 || (p->n_points > 0 && (!p->points || !p->values))) {
        delete r;
        return fail(LSUM_E_INVALID, "bad sample point arguments");
    }
    q.n_points = p->n_points;
    q.points = p->points;
    q.values = p->values;
    q.points_on_device = p->points_on_device;
    q.reserved = q.plan().planned_bytes() + (q.points_on_device ? 0 : (size_t)q.n_points * 32);
    if (q.reserved > x->c.budget) {
        delete r;
        return fail(LSUM_E_NOMEM, "the request can never fit the HBM budget");
    }
    *out = r;
    return LSUM_OK;
}

int lsum_submit(lsum_ctx x, const lsum_problem* p, int nonblocking, lsum_req* out) {
    return lsum_submit_many(x, 1, p, nonblocking, out);
}

int lsum_submit_many(lsum_ctx x, int n, const lsum_problem* p, int nonblocking, lsum_req* out) {
    if (!x || (n > 0 && (!p || !out)) || n < 0) return fail(LSUM_E_INVALID, "null argument");
    std::vector<lsum_req_s*> rs(n, nullptr);
    for (int i = 0; i < n; ++i) {
        const int rc = prepare_request(x, p + i, &rs[i]);
        if (rc != LSUM_OK) {
            for (int k = 0; k < i; ++k) delete rs[k];
            return rc;
        }
    }
    Context& c = x->c;
    {
        std::lock_guard<std::mutex> lk(c.mu);
        if (c.stopping) {
            for (auto* r : rs) delete r;
            return fail(LSUM_E_STATE, "context is shutting down");
        }
        if (nonblocking && c.queue.size() + n > c.max_queue) {
            for (auto* r : rs) delete r;
            return fail(LSUM_E_BUSY, "queue full");
        }
        const auto now = Clock::now();
        for (auto* r : rs) {
            r->q.t_submit = now;
            c.queue.push_back(&r->q);
        }
    }
    c.cv.notify_all();
    for (int i = 0; i < n; ++i) out[i] = rs[i];
    return LSUM_OK;
}

int lsum_wait(lsum_req r, int timeout_ms) {
    if (!r) return fail(LSUM_E_INVALID, "null request");
    Request& q = r->q;
    std::unique_lock<std::mutex> lk(q.mu);
    if (timeout_ms < 0) {
        q.cv.wait(lk, [&] { return q.done; });
    } else if (!q.cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), [&] { return q.done; })) {
        return LSUM_E_TIMEOUT;
    }
    return q.status.load();
}

int lsum_cancel(lsum_req r) {
    if (!r) return fail(LSUM_E_INVALID, "null request");
    Request& q = r->q;
    Context& c = *q.ctx;
    {
        std::lock_guard<std::mutex> lk(c.mu);
        auto it = std::find(c.queue.begin(), c.queue.end(), &q);
        if (it == c.queue.end()) return fail(LSUM_E_STATE, "request already started or finished");
        c.queue.erase(it);
    }
    c.cv.notify_all();
    finish(&q, LSUM_E_CANCELLED);
    return LSUM_OK;
}

static int l_max(const Plan& P) { return P.N[0] >= P.N[1] ? (P.N[0] >= P.N[2] ? 0 : 2) : (P.N[1] >= P.N[2] ? 1 : 2); }

static int need_done(lsum_req r) {
    if (!r) return fail(LSUM_E_INVALID, "null request");
    std::lock_guard<std::mutex> lk(r->q.mu);
    if (!r->q.done) return fail(LSUM_E_STATE, "request not finished");
    if (r->q.status.load() != LSUM_OK) return fail(LSUM_E_STATE, "request failed");
    return LSUM_OK;
}

int lsum_get_info(lsum_req r, lsum_info* info) {
    if (!r || !info) return fail(LSUM_E_INVALID, "null argument");
    Request& q = r->q;
    std::lock_guard<std::mutex> lk(q.mu);
    std::memset(info, 0, sizeof(*info));
    info->status = q.done ? q.status.load() : 1;
    const Plan& P = q.plan();
    info->R = P.R;
    info->n_terms = P.R * P.n_groups;
    info->is_tucker = P.tucker() ? 1 : 0;
    for (int l = 0; l < 3; ++l) {
        info->r[l] = q.r[l];
        info->D[l] = P.D[l];
    }
    info->norm_A = q.norm_A;
    info->norm_xi = q.norm_xi;
    info->bound = q.bound;
    info->rel_bound = q.norm_A > 0 ? q.bound / q.norm_A : 0.0;
    info->probe_err = q.probe_err;
    info->n_probe = q.n_probe;
    if (q.started) info->t_queue_ms = ms_since(q.t_submit, q.t_start);
    if (q.done && q.started) info->t_run_ms = ms_since(q.t_start, q.t_end);
    return LSUM_OK;
}

static int copy_out(void* dst, const void* src, size_t bytes, int on_device, int device) {
    LSUM_HIP(hipSetDevice(device));
    LSUM_HIP(hipMemcpy(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
    return LSUM_OK;
}

int lsum_get_canonical(lsum_req r, int block, double* U0, double* U1, double* U2, double* weight,
                       int on_device) {
    int rc = need_done(r);
    if (rc) return rc;
    Request& q = r->q;
    const Plan& P = q.plan();
    if (block < 0 || block >= (int)P.blocks.size()) return fail(LSUM_E_INVALID, "bad block index");
    if (P.tucker_ref()) return fail(LSUM_E_STATE, "a Tucker-reference sum keeps no canonical factors");
    if (weight) *weight = P.blocks[block].charge;
    double* dst[3] = {U0, U1, U2};
    const bool have_vm = q.U[block].p != nullptr;
    DevBuf tmp;
    if (!have_vm) {
        LSUM_HIP(hipSetDevice(q.ctx->device));
        if ((rc = tmp.get(q.ctx->pool, (size_t)P.R * P.N[l_max(P)] * 8))) return rc;
    }
    for (int l = 0; l < 3; ++l) {
        if (!dst[l]) continue;
        const double* src = have_vm ? q.U[block].as<double>() + q.U_axis_off[l] : nullptr;
        if (!have_vm) {
            // factors are kept point-major (N x R); transpose back to R x N
            if (P.rows_f32())
                launch_transpose(q.ctx->own_stream, P.N[l], P.R, q.UT[block].as<float>() + q.UT_axis_off[l], P.ldt,
                                 tmp.as<double>());
            else
                launch_transpose(q.ctx->own_stream, P.N[l], P.R, q.UT[block].as<double>() + q.UT_axis_off[l], P.ldt,
                                 tmp.as<double>());
            LSUM_HIP(hipStreamSynchronize(q.ctx->own_stream));
            src = tmp.as<double>();
        }
        rc = copy_out(dst[l], src, (size_t)P.R * P.N[l] * 8, on_device, q.ctx->device);
        if (rc) return rc;
    }
    return LSUM_OK;
}

int lsum_tucker_to_canonical(lsum_req r, double eps, int cap, int* R, double* xi, double* U0, double* U1,
                             double* U2, double* err, int on_device) {
    int rc = need_done(r);
    if (rc) return rc;
    if (!R || !err) return fail(LSUM_E_INVALID, "null argument");
    if (!(eps >= 0.0)) return fail(LSUM_E_INVALID, "eps must be >= 0");
    Request& q = r->q;
    const Plan& P = q.plan();
    if (!P.tucker()) return fail(LSUM_E_STATE, "request has no Tucker output");
    const int r1 = q.r[0], r2 = q.r[1], r3 = q.r[2];
    if (std::max(r1, r2) > 128) return fail(LSUM_E_INVALID, "core slices above 128 x 128");
    Context& c = *q.ctx;
    LSUM_HIP(hipSetDevice(c.device));
    hipStream_t st = c.own_stream;
    FailStream fs(st);
    // the core on the host in FP64 (it is FP32 at FP32 / BF16X3 precision)
    const size_t plane = (size_t)r1 * r2 * r3;
    std::vector<double> mu(plane);
    if (P.precision == LSUM_FP64) {
        LSUM_HIP(hipMemcpy(mu.data(), q.core.p, plane * 8, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> f(plane);
        LSUM_HIP(hipMemcpy(f.data(), q.core.p, plane * 4, hipMemcpyDeviceToHost));
        for (size_t k = 0; k < plane; ++k) mu[k] = f[k];
    }
    // per mode-3 slice its SVD: terms s u (x) v (x) e_k
    struct Term {
        double s;
        int k, i;
    };
    std::vector<Term> terms;
    std::vector<std::vector<double>> Us(r3), Vs(r3);
    std::vector<double> slice((size_t)r1 * r2), S;
    double mu2 = 0.0;
    for (double v : mu) mu2 += v * v;
    for (int k = 0; k < r3; ++k) {
        for (int a = 0; a < r1; ++a)
            for (int b = 0; b < r2; ++b) slice[(size_t)a * r2 + b] = mu[((size_t)a * r2 + b) * r3 + k];
        lsum::small_svd(slice.data(), r1, r2, Us[k], S, Vs[k]);
        for (int i = 0; i < (int)S.size(); ++i) terms.push_back(Term{S[i], k, i});
    }
    std::stable_sort(terms.begin(), terms.end(), [](const Term& x, const Term& y) {
        if (x.s != y.s) return x.s > y.s;
        return x.k != y.k ? x.k < y.k : x.i < y.i;
    });
    // drop the smallest while the dropped (sum s^2)^(1/2) stays <= eps ||core||
    const double budget = eps * eps * mu2;
    double dropped = 0.0;
    size_t keep = terms.size();
    while (keep > 1 && dropped + terms[keep - 1].s * terms[keep - 1].s <= budget) {
        dropped += terms[keep - 1].s * terms[keep - 1].s;
        --keep;
    }
    *R = (int)keep;
    *err = std::sqrt(dropped);
    if (!xi) return LSUM_OK;
    if (cap < (int)keep) return fail(LSUM_E_INVALID, "output capacity below the canonical rank");
    // factor rows: U_l (keep x N_l) = coefficients (keep x r_l) x Z_l (r_l x N_l), by MFMA GEMMs
    std::vector<double> xs(keep), C[3];
    C[0].assign(keep * (size_t)r1, 0.0);
    C[1].assign(keep * (size_t)r2, 0.0);
    C[2].assign(keep * (size_t)r3, 0.0);
    for (size_t t = 0; t < keep; ++t) {
        const Term& e = terms[t];
        xs[t] = e.s;
        for (int a = 0; a < r1; ++a) C[0][t * r1 + a] = Us[e.k][(size_t)e.i * r1 + a];
        for (int b = 0; b < r2; ++b) C[1][t * r2 + b] = Vs[e.k][(size_t)e.i * r2 + b];
        C[2][t * r3 + e.k] = 1.0;
    }
    double* dst[3] = {U0, U1, U2};
    for (int l = 0; l < 3; ++l) {
        if (!dst[l]) continue;
        const int rl = q.r[l], N = P.N[l];
        DevBuf Cd, Out;
        if ((rc = Cd.get(c.pool, C[l].size() * 8)) || (rc = Out.get(c.pool, keep * (size_t)N * 8))) return rc;
        LSUM_HIP(hipMemcpyAsync(Cd.p, C[l].data(), C[l].size() * 8, hipMemcpyHostToDevice, st));
        GemmArgs a{};
        a.m = (int)keep; a.n = N; a.k = rl;
        a.A = Cd.p; a.sam = rl; a.sak = 1;
        a.B = q.Z[l].p; a.sbk = N; a.sbn = 1;
        a.C = Out.p; a.scm = N; a.scn = 1;
        a.alpha = 1.0; a.beta = 0.0; a.batch = 1;
        launch_gemm(st, GEMM_F64, a);
        LSUM_HIP(hipGetLastError());
        LSUM_HIP(hipStreamSynchronize(st));
        if ((rc = copy_out(dst[l], Out.p, keep * (size_t)N * 8, on_device, c.device))) return rc;
    }
    if (on_device) {
        LSUM_HIP(hipMemcpy(xi, xs.data(), keep * 8, hipMemcpyHostToDevice));
    } else {
        std::memcpy(xi, xs.data(), keep * 8);
    }
    return LSUM_OK;
}

int lsum_galerkin(lsum_req r, int nb, const double* G0, const double* G1, const double* G2, double* V,
                  int on_device) {
    int rc = need_done(r);
    if (rc) return rc;
    if (!G0 || !G1 || !G2 || !V) return fail(LSUM_E_INVALID, "null argument");
    if (nb < 1 || nb > 255) return fail(LSUM_E_INVALID, "nb must be in [1, 255]");
    Request& q = r->q;
    const Plan& P = q.plan();
    if (!P.tucker()) return fail(LSUM_E_STATE, "the Galerkin functional needs a Tucker result");
    Context& c = *q.ctx;
    LSUM_HIP(hipSetDevice(c.device));
    hipStream_t st = c.own_stream;
    FailStream fs(st);
    const int r1 = q.r[0], r2 = q.r[1], r3 = q.r[2];
    const long Pn = (long)nb * nb;
    const double* G[3] = {G0, G1, G2};
    DevBuf Gd[3], H, Y[3], X, mu, v;
    // per mode: the pairs' Hadamard rows and their projections Y_l = H_l Z_l^T (Pn x r_l)
    for (int l = 0; l < 3; ++l) {
        const int N = P.N[l], rl = q.r[l];
        const double* g = G[l];
        if (!on_device) {
            if ((rc = Gd[l].get(c.pool, (size_t)nb * N * 8))) return rc;
            LSUM_HIP(hipMemcpyAsync(Gd[l].p, G[l], (size_t)nb * N * 8, hipMemcpyHostToDevice, st));
            g = Gd[l].as<double>();
        }
        if ((rc = H.get(c.pool, (size_t)Pn * N * 8))) return rc;
        launch_hadamard_pairs(st, nb, N, g, H.as<double>());
        if ((rc = Y[l].get(c.pool, (size_t)Pn * rl * 8))) return rc;
        GemmArgs a{};
        a.m = (int)Pn; a.n = rl; a.k = N;
        a.A = H.p; a.sam = N; a.sak = 1;
        a.B = q.Z[l].p; a.sbk = 1; a.sbn = N;
        a.C = Y[l].p; a.scm = rl; a.scn = 1;
        a.alpha = 1.0; a.beta = 0.0; a.batch = 1;
        if ((rc = gemm_auto(&c, st, GEMM_F64, a))) return rc;
        LSUM_HIP(hipStreamSynchronize(st));   // H is reused by the next mode
        H.reset();
    }
    // the core in FP64 (FP32 at FP32 / BF16X3 precision), then X = Y_3 mu^T (Pn x r1 r2)
    const long plane = (long)r1 * r2 * r3;
    const double* mud = q.core.as<double>();
    if (P.precision != LSUM_FP64) {
        if ((rc = mu.get(c.pool, (size_t)plane * 8))) return rc;
        launch_f32_to_f64(st, plane, q.core.as<float>(), mu.as<double>());
        mud = mu.as<double>();
    }
    if ((rc = X.get(c.pool, (size_t)Pn * r1 * r2 * 8))) return rc;
    GemmArgs a{};
    a.m = (int)Pn; a.n = r1 * r2; a.k = r3;
    a.A = Y[2].p; a.sam = r3; a.sak = 1;
    a.B = mud; a.sbk = 1; a.sbn = r3;
    a.C = X.p; a.scm = (long)r1 * r2; a.scn = 1;
    a.alpha = 1.0; a.beta = 0.0; a.batch = 1;
    if ((rc = gemm_auto(&c, st, GEMM_F64, a))) return rc;
    double* out = V;
    if (!on_device) {
        if ((rc = v.get(c.pool, (size_t)Pn * 8))) return rc;
        out = v.as<double>();
    }
    launch_galerkin_finish(st, (int)Pn, r1, r2, X.as<double>(), Y[0].as<double>(), Y[1].as<double>(),
                           P.h * P.h * P.h, out);
    LSUM_HIP(hipGetLastError());
    if (!on_device) LSUM_HIP(hipMemcpyAsync(V, out, (size_t)Pn * 8, hipMemcpyDeviceToHost, st));
    LSUM_HIP(hipStreamSynchronize(st));
    return LSUM_OK;
}

int lsum_get_tucker(lsum_req r, double* Z0, double* Z1, double* Z2, double* core, int on_device) {
    int rc = need_done(r);
    if (rc) return rc;
    Request& q = r->q;
    const Plan& P = q.plan();
    if (!P.tucker()) return fail(LSUM_E_STATE, "request has no Tucker output");
    double* dst[3] = {Z0, Z1, Z2};
    for (int l = 0; l < 3; ++l) {
        if (!dst[l]) continue;
        rc = copy_out(dst[l], q.Z[l].p, (size_t)q.r[l] * P.N[l] * 8, on_device, q.ctx->device);
        if (rc) return rc;
    }
    if (core) {
        const size_t n = (size_t)q.r[0] * q.r[1] * q.r[2];
        if (P.precision == LSUM_FP64) return copy_out(core, q.core.p, n * 8, on_device, q.ctx->device);
        LSUM_HIP(hipSetDevice(q.ctx->device));
        DevBuf tmp;
        if ((rc = tmp.get(q.ctx->pool, n * 8))) return rc;
        launch_f32_to_f64(q.ctx->own_stream, (long)n, q.core.as<float>(), tmp.as<double>());
        LSUM_HIP(hipStreamSynchronize(q.ctx->own_stream));
        return copy_out(core, tmp.p, n * 8, on_device, q.ctx->device);
    }
    return LSUM_OK;
}

int lsum_get_sigma(lsum_req r, double* s0, double* s1, double* s2) {
    int rc = need_done(r);
    if (rc) return rc;
    Request& q = r->q;
    double* dst[3] = {s0, s1, s2};
    for (int l = 0; l < 3; ++l)
        if (dst[l]) std::copy(q.sigma[l].begin(), q.sigma[l].end(), dst[l]);
    return LSUM_OK;
}

int lsum_sample(lsum_req r, int n, const double* xyz, double* out, int on_device) {
    int rc = need_done(r);
    if (rc) return rc;
    if (n < 0 || (n > 0 && (!xyz || !out))) return fail(LSUM_E_INVALID, "bad point arguments");
    if (n == 0) return LSUM_OK;
    Request& q = r->q;
    Context& c = *q.ctx;
    const Plan& P = q.plan();
    LSUM_HIP(hipSetDevice(c.device));
    hipStream_t st = c.own_stream;
    FailStream fs(st);
    DevBuf xd, od;
    const double* xyz_d = xyz;
    double* out_d = out;
    if (!on_device) {
        if ((rc = xd.get(c.pool, (size_t)n * 24))) return rc;
        if ((rc = od.get(c.pool, (size_t)n * 8))) return rc;
        LSUM_HIP(hipMemcpyAsync(xd.p, xyz, (size_t)n * 24, hipMemcpyHostToDevice, st));
        xyz_d = xd.as<double>();
        out_d = od.as<double>();
    }
    (void)P;
    rc = sample_points(&q, st, n, xyz_d, out_d);
    if (rc) return rc;
    LSUM_HIP(hipGetLastError());
    if (!on_device) LSUM_HIP(hipMemcpyAsync(out, out_d, (size_t)n * 8, hipMemcpyDeviceToHost, st));
    LSUM_HIP(hipStreamSynchronize(st));
    return LSUM_OK;
}

int lsum_get_tile(lsum_req r, void* out, int elem_size, int on_device) {
    int rc = need_done(r);
    if (rc) return rc;
    Request& q = r->q;
    const Plan& P = q.plan();
    if (!P.has_tile()) return fail(LSUM_E_STATE, "request has no tile");
    const int want = P.precision == LSUM_FP64 ? 8 : 4;
    if (elem_size != want) return fail(LSUM_E_INVALID, "tile element size does not match the precision");
    const size_t n = (size_t)P.tile_T[0] * P.tile_T[1] * P.tile_T[2];
    return copy_out(out, q.tile.p, n * want, on_device, q.ctx->device);
}

int lsum_get_stats(lsum_req r, char* buf, size_t len) {
    if (!r) return fail(LSUM_E_INVALID, "null request");
    Request& q = r->q;
    std::ostringstream o;
    o.precision(17);
    const Plan& P = q.plan();
    {
        std::lock_guard<std::mutex> lk(q.mu);
        o << "{\"status\":" << (q.done ? q.status.load() : 1) << ",\"R\":" << P.R << ",\"n_groups\":" << P.n_groups
          << ",\"h_u\":" << P.h_u << ",\"s\":" << P.s << ",\"N\":[" << P.N[0] << "," << P.N[1] << "," << P.N[2]
          << "],\"D\":[" << P.D[0] << "," << P.D[1] << "," << P.D[2] << "],\"r\":[" << q.r[0] << "," << q.r[1]
          << "," << q.r[2] << "],\"sweeps\":[" << q.sweeps[0] << "," << q.sweeps[1] << "," << q.sweeps[2]
          << "],\"tails\":[" << q.tails[0] << "," << q.tails[1] << "," << q.tails[2]
          << "],\"axis_src\":[" << q.axis_src[0] << "," << q.axis_src[1] << "," << q.axis_src[2]
          << "],\"range_k\":[" << q.range_k[0] << "," << q.range_k[1] << "," << q.range_k[2]
          << "],\"range_res\":[" << q.range_res[0] << "," << q.range_res[1] << "," << q.range_res[2]
          << "],\"core_mode\":" << q.core_mode << ",\"norm_A\":" << q.norm_A
          << ",\"norm_xi\":" << q.norm_xi << ",\"bound\":" << q.bound << ",\"probe_err\":" << q.probe_err
          << ",\"n_probe\":" << q.n_probe << ",\"batch\":" << q.batch_size
          << ",\"als_skipped\":" << q.als_skipped << ",\"jacobi_persistent\":[" << q.jacobi_persistent[0] << ","
          << q.jacobi_persistent[1] << "," << q.jacobi_persistent[2] << "],\"jacobi_aborted\":["
          << q.jacobi_aborted[0] << "," << q.jacobi_aborted[1] << "," << q.jacobi_aborted[2]
          << "],\"jacobi_tuned\":[" << q.jacobi_tuned[0] << "," << q.jacobi_tuned[1] << "," << q.jacobi_tuned[2]
          << "],\"als_core_norm\":[";
        for (size_t k = 0; k < q.als_core_norm.size(); ++k) o << (k ? "," : "") << q.als_core_norm[k];
        o << "],\"probe_cells\":[";
        for (size_t k = 0; k + 2 < q.probe_cells.size(); k += 3)
            o << (k ? "," : "") << "[" << q.probe_cells[k] << "," << q.probe_cells[k + 1] << "," << q.probe_cells[k + 2]
              << "]";
        o << "],\"offsets\":[";
        for (int b = 0; b < (int)P.blocks.size(); ++b) {
            o << (b ? "," : "") << "[";
            for (int l = 0; l < 3; ++l) {
                o << (l ? "," : "") << "[";
                for (size_t k = 0; k < P.offs[l][b].size(); ++k) o << (k ? "," : "") << P.offs[l][b][k];
                o << "]";
            }
            o << "]";
        }
        o << "],\"t_ms\":{";
        bool first = true;
        static const std::map<std::string, double> none;
        for (auto& kv : (q.t_ms ? *q.t_ms : none)) {
            o << (first ? "" : ",") << "\"" << kv.first << "\":" << kv.second;
            first = false;
        }
        o << "},\"bytes\":{";
        first = true;
        if (q.canonical_bytes > 0) {
            o << "\"canonical\":" << q.canonical_bytes;
            first = false;
        }
        for (auto& kv : q.bytes) {
            o << (first ? "" : ",") << "\"" << kv.first << "\":" << kv.second;
            first = false;
        }
        o << "}";
        if (!q.error.empty()) {
            o << ",\"error\":\"";
            for (char ch : q.error) {
                if (ch == '"' || ch == '\\') o << '\\' << ch;
                else if ((unsigned char)ch < 0x20) o << ' ';
                else o << ch;
            }
            o << "\"";
        }
        if (q.started) o << ",\"t_queue_ms\":" << ms_since(q.t_submit, q.t_start);
        if (q.done && q.started) o << ",\"t_run_ms\":" << ms_since(q.t_start, q.t_end);
        o << "}";
    }
    const std::string s = o.str();
    if (buf && len > 0) {
        const size_t n = std::min(len - 1, s.size());
        std::memcpy(buf, s.data(), n);
        buf[n] = 0;
    }
    return (int)s.size() + 1;
}

int lsum_release(lsum_req r) {
    if (!r) return LSUM_OK;
    Request& q = r->q;
    {
        std::unique_lock<std::mutex> lk(q.mu);
        if (!q.done) {
            lk.unlock();
            if (lsum_cancel(r) != LSUM_OK) lsum_wait(r, -1);
        }
    }
    Context& c = *q.ctx;
    (void)hipSetDevice(c.device);
    drop_reference(&q);
    bool waiting;   // queued requests may be waiting for the memory this one frees
    {
        std::lock_guard<std::mutex> lk(c.mu);
        c.used -= std::min(c.used, q.retained);
        waiting = !c.queue.empty() && q.retained > 0;
    }
    if (waiting) c.cv.notify_all();
    delete r;
    return LSUM_OK;
}

int lsum_finish_many(int n, lsum_req* r, int* status, lsum_info* info) {
    if (n < 0 || (n > 0 && (!r || !status))) return fail(LSUM_E_INVALID, "null argument");
    for (int i = 0; i < n; ++i)
        if (!r[i]) return fail(LSUM_E_INVALID, "null request");
    for (int i = 0; i < n; ++i) {
        status[i] = lsum_wait(r[i], -1);
        if (info) lsum_get_info(r[i], info + i);
        lsum_release(r[i]);
        r[i] = nullptr;
    }
    return LSUM_OK;
}

int lsum_set_option(lsum_ctx x, int key, double value) {
    if (!x) return fail(LSUM_E_INVALID, "null ctx");
    Context& c = x->c;
    std::lock_guard<std::mutex> lk(c.mu);
    switch (key) {
        case LSUM_OPT_MAX_BATCH:
            if (!(value >= 1 && value <= 4096)) return fail(LSUM_E_INVALID, "batch size must be in [1, 4096]");
            c.max_batch = (int)value;
            return LSUM_OK;
        case LSUM_OPT_REF_CACHE_BYTES: {
            if (!(value >= 0)) return fail(LSUM_E_INVALID, "negative cache size");
            std::lock_guard<std::mutex> lr(c.ref_mu);
            c.ref_cap = (size_t)value;
            if (c.ref_cap == 0) {
                for (auto it = c.refs.begin(); it != c.refs.end();)
                    if (it->second->users.load() == 0) {
                        c.ref_bytes -= it->second->bytes;
                        it = c.refs.erase(it);
                    } else {
                        ++it;
                    }
            }
            return LSUM_OK;
        }
        case LSUM_OPT_RANGE_MIN:
            if (!(value >= 0 && value <= 1e9)) return fail(LSUM_E_INVALID, "range threshold out of range");
            c.range_min = (int)value;
            return LSUM_OK;
        case LSUM_OPT_JACOBI_STOP:
            if (!(value == 0 || value == 1)) return fail(LSUM_E_INVALID, "Jacobi stop rule must be 0 or 1");
            c.jacobi_rank_stop = value == 1;
            return LSUM_OK;
        case LSUM_OPT_JACOBI_MAX_SWEEPS:
            if (!(value >= 1 && value <= 1000)) return fail(LSUM_E_INVALID, "Jacobi sweep limit must be in [1, 1000]");
            c.jacobi_max_sweeps.store((int)value);
            return LSUM_OK;
        case LSUM_OPT_GRAPHS:
            if (!(value == 0 || value == 1)) return fail(LSUM_E_INVALID, "graph option must be 0 or 1");
            c.graphs.store((int)value);
            return LSUM_OK;
        case LSUM_OPT_JACOBI_PERSISTENT:
            if (!(value == 0 || value == 1 || value == 2))
                return fail(LSUM_E_INVALID, "persistent option must be 0, 1 or 2");
            c.persistent.store((int)value);
            return LSUM_OK;
        case LSUM_OPT_AUTOTUNE:
            if (!(value == 0 || value == 1)) return fail(LSUM_E_INVALID, "autotune option must be 0 or 1");
            c.tuner.enable(value == 1);
            return LSUM_OK;
        case LSUM_OPT_JACOBI_SKIP:
            if (!(value == 0 || value == 1)) return fail(LSUM_E_INVALID, "Jacobi skip option must be 0 or 1");
            c.jacobi_skip.store((int)value);
            return LSUM_OK;
        case LSUM_OPT_JACOBI_BLOCK:
            if (!(value == 0 || value == 8 || value == 16 || value == 32))
                return fail(LSUM_E_INVALID, "Jacobi block must be 0 (by size), 8, 16 or 32 columns");
            c.jacobi_block.store((int)value);
            return LSUM_OK;
        case LSUM_OPT_GEMM_LIBRARY:
            if (!(value == 0 || value == 1)) return fail(LSUM_E_INVALID, "GEMM library option must be 0 or 1");
            set_gemm_library(value == 1);
            return LSUM_OK;
        case LSUM_OPT_JACOBI_WAIT_US:
            if (!(value >= 0 && value <= 1e8)) return fail(LSUM_E_INVALID, "wait bound must be in [0, 1e8] us");
            c.jacobi_wait_us.store((long long)value);
            return LSUM_OK;
        default:
            return fail(LSUM_E_INVALID, "unknown option");
    }
}

int lsum_tune_file(lsum_ctx x, const char* path) {
    if (!x || !path) return fail(LSUM_E_INVALID, "null argument");
    return x->c.tuner.use_file(path);
}

int lsum_get_tuning(lsum_ctx x, char* buf, size_t len) {
    if (!x) return fail(LSUM_E_INVALID, "null ctx");
    const std::string j = x->c.tuner.json();
    if (buf && len > 0) {
        const size_t n = std::min(len - 1, j.size());
        std::memcpy(buf, j.data(), n);
        buf[n] = 0;
    }
    return (int)j.size();
}

int lsum_get_profile(lsum_ctx x, char* buf, size_t len) {
    if (!x) return fail(LSUM_E_INVALID, "null ctx");
    Context& c = x->c;
    std::ostringstream o;
    o.precision(17);
    {
        std::lock_guard<std::mutex> lk(c.prof_mu);
        o << "{";
        bool first = true;
        for (auto& kv : c.profile) {
            o << (first ? "" : ",") << "\"" << kv.first << "\":{\"ms\":" << kv.second.ms << ",\"launches\":"
              << kv.second.launches << ",\"bytes\":" << kv.second.bytes << ",\"flops\":" << kv.second.flops << "}";
            first = false;
        }
        o << "}";
    }
    const std::string s = o.str();
    if (buf && len > 0) {
        const size_t n = std::min(len - 1, s.size());
        std::memcpy(buf, s.data(), n);
        buf[n] = 0;
    }
    return (int)s.size() + 1;
}

int lsum_reset_profile(lsum_ctx x) {
    if (!x) return fail(LSUM_E_INVALID, "null ctx");
    std::lock_guard<std::mutex> lk(x->c.prof_mu);
    x->c.profile.clear();
    return LSUM_OK;
}

// ---- stage entry points (synchronous) -----------------------------------------------------

static hipStream_t pick(lsum_ctx x, void* s) { return s ? (hipStream_t)s : x->c.own_stream; }

int lsum_collocate(lsum_ctx x, void* stream, int R, const double* t, const double* w, int N_ref, double h,
                   double* G_dev, int ldg) {
    if (!x || !t || !w || !G_dev) return fail(LSUM_E_INVALID, "null argument");
    if (R < 1 || N_ref < 1 || ldg < 2 * N_ref - 1 || !(h > 0)) return fail(LSUM_E_INVALID, "bad sizes");
    LSUM_HIP(hipSetDevice(x->c.device));
    hipStream_t st = pick(x, stream);
    FailStream fs(st);
    std::vector<double> w13(R);
    for (int q = 0; q < R; ++q) {
        if (!(w[q] > 0.0) || !(t[q] >= 0.0)) return fail(LSUM_E_INVALID, "weights must be positive, nodes non-negative");
        w13[q] = std::cbrt(w[q]);
    }
    DevBuf tw;
    int rc = tw.get(x->c.pool, 2 * (size_t)R * 8);
    if (rc) return rc;
    LSUM_HIP(hipMemcpyAsync(tw.as<double>(), t, R * 8, hipMemcpyHostToDevice, st));
    LSUM_HIP(hipMemcpyAsync(tw.as<double>() + R, w13.data(), R * 8, hipMemcpyHostToDevice, st));
    launch_collocate(st, R, tw.as<double>(), tw.as<double>() + R, N_ref, h, G_dev, ldg);
    LSUM_HIP(hipGetLastError());
    LSUM_HIP(hipStreamSynchronize(st));
    return LSUM_OK;
}

static int check_shift_sum_args(lsum_ctx x, int R, const double* G_dev, int ldg, int N_ref, int N_axis,
                                int n_sites, const int32_t* sites, const double* U_dev, int ldu) {
    if (!x || !G_dev || !U_dev || (n_sites > 0 && !sites)) return fail(LSUM_E_INVALID, "null argument");
    if (R < 1 || N_axis < 1 || N_axis > N_ref || ldg < std::max(2, 2 * N_ref - 1) || ldu < N_axis || n_sites < 0)
        return fail(LSUM_E_INVALID, "bad sizes");
    for (int k = 0; k < n_sites; ++k)
        if (sites[k] < 0 || sites[k] >= N_axis) return fail(LSUM_E_OUT_OF_BOX, "site index outside the axis");
    return LSUM_OK;
}

int lsum_shift_sum(lsum_ctx x, void* stream, int R, const double* G_dev, int ldg, int N_ref, int N_axis,
                   int n_sites, const int32_t* sites, double* U_dev, int ldu) {
    if (int rc0 = check_shift_sum_args(x, R, G_dev, ldg, N_ref, N_axis, n_sites, sites, U_dev, ldu)) return rc0;
    LSUM_HIP(hipSetDevice(x->c.device));
    hipStream_t st = pick(x, stream);
    FailStream fs(st);
    // terms: one per site, one per comb on windowed strided sums of the rows, or two per run of
    // one stride on strided prefix / suffix sums of the rows
    std::vector<int2> terms;
    int stride = 0, n_tab[2] = {0, 0};
    bool two = false;
    shift_terms(sites, n_sites, N_ref, N_axis, ldg, terms, &stride, n_tab, &two);
    DevBuf td, jd, w0, w1;
    int rc = td.get(x->c.pool, std::max<size_t>(1, terms.size()) * sizeof(int2));
    if (rc) return rc;
    if ((rc = jd.get(x->c.pool, sizeof(ShiftJob)))) return rc;
    ShiftJob j{};
    j.T0 = G_dev;
    if (stride > 0) {
        if ((rc = w0.get(x->c.pool, (size_t)R * ldg * 8))) return rc;
        launch_window_sums(st, R, G_dev, ldg, stride, n_tab[0], w0.as<double>());
        j.T0 = w0.as<double>();
        if (two) {
            if ((rc = w1.get(x->c.pool, (size_t)R * ldg * 8))) return rc;
            launch_window_sums(st, R, G_dev, ldg, stride, n_tab[1], w1.as<double>());
            j.T1 = w1.as<double>();
        }
    }
    j.terms = td.as<int2>();
    j.n_terms = (int)terms.size();
    j.U = U_dev;
    j.ldu = ldu;
    j.N_axis = N_axis;
    j.ldg = ldg;
    j.R = R;
    if (!terms.empty())
        LSUM_HIP(hipMemcpyAsync(td.p, terms.data(), terms.size() * sizeof(int2), hipMemcpyHostToDevice, st));
    LSUM_HIP(hipMemcpyAsync(jd.p, &j, sizeof(j), hipMemcpyHostToDevice, st));
    launch_shift_sum(st, jd.as<ShiftJob>(), 1, N_axis, R);
    LSUM_HIP(hipGetLastError());
    LSUM_HIP(hipStreamSynchronize(st));
    return LSUM_OK;
}

// The same steps and kernels as lsum_shift_sum, with the job descriptor, the terms and the
// window tables in the device's static scratch array instead of pool memory: no allocation.
int lsum_shift_sum_noalloc(lsum_ctx x, void* stream, int R, const double* G_dev, int ldg, int N_ref, int N_axis,
                           int n_sites, const int32_t* sites, double* U_dev, int ldu) {
    if (int rc0 = check_shift_sum_args(x, R, G_dev, ldg, N_ref, N_axis, n_sites, sites, U_dev, ldu)) return rc0;
    LSUM_HIP(hipSetDevice(x->c.device));
    hipStream_t st = pick(x, stream);
    FailStream fs(st);
    std::vector<int2> terms;
    int stride = 0, n_tab[2] = {0, 0};
    bool two = false;
    shift_terms(sites, n_sites, N_ref, N_axis, ldg, terms, &stride, n_tab, &two);
    // scratch layout (256-byte aligned parts): job | terms | window table 0 | window table 1
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t off_terms = up(sizeof(ShiftJob));
    const size_t off_w0 = off_terms + up(std::max<size_t>(1, terms.size()) * sizeof(int2));
    const size_t tab = up((size_t)R * ldg * 8);
    const size_t need = off_w0 + (stride > 0 ? (two ? 2 : 1) * tab : 0);
    if (need > kNoallocScratchBytes)
        return fail(LSUM_E_NOMEM, "lsum_shift_sum_noalloc needs " + std::to_string(need) +
                                      " bytes of scratch; the static array holds " +
                                      std::to_string(kNoallocScratchBytes));
    void* base = nullptr;
    if (int rc = noalloc_scratch(x->c.device, &base)) return rc;
    unsigned char* sp = static_cast<unsigned char*>(base);
    ShiftJob j{};
    j.T0 = G_dev;
    if (stride > 0) {
        double* w0 = reinterpret_cast<double*>(sp + off_w0);
        launch_window_sums(st, R, G_dev, ldg, stride, n_tab[0], w0);
        j.T0 = w0;
        if (two) {
            double* w1 = reinterpret_cast<double*>(sp + off_w0 + tab);
            launch_window_sums(st, R, G_dev, ldg, stride, n_tab[1], w1);
            j.T1 = w1;
        }
    }
    j.terms = reinterpret_cast<const int2*>(sp + off_terms);
    j.n_terms = (int)terms.size();
    j.U = U_dev;
    j.ldu = ldu;
    j.N_axis = N_axis;
    j.ldg = ldg;
    j.R = R;
    if (!terms.empty())
        LSUM_HIP(hipMemcpyAsync(sp + off_terms, terms.data(), terms.size() * sizeof(int2), hipMemcpyHostToDevice, st));
    LSUM_HIP(hipMemcpyAsync(sp, &j, sizeof(j), hipMemcpyHostToDevice, st));
    launch_shift_sum(st, reinterpret_cast<const ShiftJob*>(sp), 1, N_axis, R);
    LSUM_HIP(hipGetLastError());
    LSUM_HIP(hipStreamSynchronize(st));   // the host job and terms are read before return
    return LSUM_OK;
}

int lsum_sample_canonical(lsum_ctx x, void* stream, int n_fac, int R, const double* U_dev, int ldu,
                          const double* lam, const int N[3], double h, int n_pts, const double* xyz_dev,
                          double* out_dev) {
    if (!x || !U_dev || !lam || !N || (n_pts > 0 && (!xyz_dev || !out_dev))) return fail(LSUM_E_INVALID, "null argument");
    if (n_fac < 1 || R < 1 || ldu < std::max(N[0], std::max(N[1], N[2])) || n_pts < 0) return fail(LSUM_E_INVALID, "bad sizes");
    LSUM_HIP(hipSetDevice(x->c.device));
    hipStream_t st = pick(x, stream);
    FailStream fs(st);
    DevBuf ld;
    int rc = ld.get(x->c.pool, n_fac * 8);
    if (rc) return rc;
    LSUM_HIP(hipMemcpyAsync(ld.p, lam, n_fac * 8, hipMemcpyHostToDevice, st));
    launch_sample_cp(st, n_fac, R, U_dev, ldu, ld.as<double>(), N[0], N[1], N[2], h, n_pts, xyz_dev, out_dev);
    LSUM_HIP(hipGetLastError());
    LSUM_HIP(hipStreamSynchronize(st));
    return LSUM_OK;
}

int lsum_contract(lsum_ctx x, void* stream, int prec, int m, int n, int k, const void* A_dev, long sam, long sak,
                  const void* B_dev, long sbk, long sbn, void* C_dev, long scm, long scn, double alpha,
                  double beta) {
    if (!x || !A_dev || !B_dev || !C_dev) return fail(LSUM_E_INVALID, "null argument");
    if (m < 0 || n < 0 || k < 0 || prec < LSUM_FP64 || prec > LSUM_BF16X3) return fail(LSUM_E_INVALID, "bad sizes");
    LSUM_HIP(hipSetDevice(x->c.device));
    hipStream_t st = pick(x, stream);
    FailStream fs(st);
    GemmArgs a{};
    a.m = m; a.n = n; a.k = k;
    a.A = A_dev; a.sam = sam; a.sak = sak;
    a.B = B_dev; a.sbk = sbk; a.sbn = sbn;
    a.C = C_dev; a.scm = scm; a.scn = scn;
    a.alpha = alpha; a.beta = beta; a.batch = 1;
    int rc = gemm_auto(&x->c, st, prec == LSUM_FP64 ? GEMM_F64 : (prec == LSUM_FP32 ? GEMM_F32 : GEMM_BF16X3), a);
    if (rc) return rc;
    LSUM_HIP(hipGetLastError());
    LSUM_HIP(hipStreamSynchronize(st));
    return LSUM_OK;
}

int lsum_jacobi_svd(lsum_ctx x, void* stream, int D, int N, double* A_dev, int lda, double tol, double irrelevant,
                    int max_sweeps, double* sigma, int* sweeps) {
    if (!x || !A_dev || !sigma || !sweeps) return fail(LSUM_E_INVALID, "null argument");
    if (D < 1 || N < 1 || lda < N || !(tol > 0) || max_sweeps < 1) return fail(LSUM_E_INVALID, "bad sizes");
    LSUM_HIP(hipSetDevice(x->c.device));
    hipStream_t st = pick(x, stream);
    FailStream fs(st);
    DevBuf work;
    const size_t wb = jacobi_work_bytes(D, N);
    int rc = work.get(x->c.pool, wb);
    if (rc) return rc;
    std::vector<double> s;
    JacobiRun jr = jacobi_run(&x->c);
    rc = jacobi_svd(st, D, N, A_dev, lda, tol, irrelevant, max_sweeps, s, sweeps, work.as<double>(), wb, 0, 0.0, &jr);
    std::copy(s.begin(), s.end(), sigma);
    return rc;
}

}  // extern "C"

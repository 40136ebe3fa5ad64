// Runtime of the lattice-sum library: contexts, request slots, HBM-budget admission, the device
// buffer pool, the shared reference-vector cache and the per-request pipeline
//   quadrature -> collocation -> shift-sums -> (defect columns -> Jacobi SVD -> truncation ->
//   projection -> core -> tile) -> results,
// plus the C ABI around them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <sstream>
#include <thread>
#include <tuple>
#include <set>

#include "lsum_internal.h"

namespace lsum {

using Clock = std::chrono::steady_clock;

static double ms_since(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

// ------------------------------------------------------------------------------------------
// device buffer pool: size-bucketed free lists, buffers are returned only after the owning
// stream has been synchronised, so reuse on another stream is safe
// ------------------------------------------------------------------------------------------
class DevPool {
  public:
    explicit DevPool(int device) : device_(device) {}
    int device() const { return device_; }
    ~DevPool() {
        for (auto& kv : free_) (void)hipFree(kv.second);
    }
    static size_t round(size_t n) {
        if (n <= (1u << 20)) {
            size_t r = 256;
            while (r < n) r <<= 1;
            return r;
        }
        return (n + (2u << 20) - 1) / (2u << 20) * (2u << 20);
    }
    int alloc(size_t n, void** p, size_t* got) {
        n = round(std::max<size_t>(n, 1));
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto it = free_.lower_bound(n);
            if (it != free_.end() && it->first <= n + n / 4) {
                *p = it->second;
                *got = it->first;
                cached_ -= it->first;
                free_.erase(it);
                return LSUM_OK;
            }
        }
        hipError_t e = hipMalloc(p, n);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            trim();
            e = hipMalloc(p, n);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return fail(LSUM_E_NOMEM, "device allocation of " + std::to_string(n) + " bytes failed");
            }
        }
        *got = n;
        return LSUM_OK;
    }
    void release(void* p, size_t n) {
        if (!p) return;
        std::lock_guard<std::mutex> lk(mu_);
        free_.emplace(n, p);
        cached_ += n;
        if (cached_ > cap_) trim_locked();
    }
    void trim() {
        std::lock_guard<std::mutex> lk(mu_);
        trim_locked();
    }

  private:
    void trim_locked() {
        for (auto& kv : free_) (void)hipFree(kv.second);
        free_.clear();
        cached_ = 0;
    }
    int device_;
    std::mutex mu_;
    std::multimap<size_t, void*> free_;
    size_t cached_ = 0;
    size_t cap_ = (size_t)24 << 30;
};

struct DevBuf {
    DevPool* pool = nullptr;
    void* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept { *this = std::move(o); }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) {
            reset();
            pool = o.pool; p = o.p; n = o.n;
            o.p = nullptr; o.n = 0;
        }
        return *this;
    }
    ~DevBuf() { reset(); }
    void reset() {
        if (p && pool) pool->release(p, n);
        p = nullptr;
        n = 0;
    }
    int get(DevPool* pl, size_t bytes) {
        reset();
        pool = pl;
        return pl->alloc(bytes, &p, &n);
    }
    template <typename T> T* as() const { return (T*)p; }
};

// ------------------------------------------------------------------------------------------
// reference-vector cache ("precompute once, store for multiple use", Sec. 2.1)
// ------------------------------------------------------------------------------------------
struct RefEntry {
    DevBuf G;
    int R = 0, ldg = 0, N_ref = 0;
    hipEvent_t ready = nullptr;
    std::atomic<int> users{0};
    size_t bytes = 0;
    uint64_t last_use = 0;
};
using RefKey = std::tuple<int, double, int, double, double, double, int>;

struct Request;

struct Context {
    int device = 0;
    size_t budget = 0;
    size_t used = 0;                 // bytes reserved by admitted requests and retained results
    int n_slots = 0;
    std::vector<hipStream_t> streams;
    std::vector<std::thread> workers;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request*> queue;
    size_t max_queue = 1 << 16;
    bool stopping = false;
    DevPool* pool = nullptr;
    hipStream_t own_stream = nullptr;
    // reference cache
    std::mutex ref_mu;
    std::map<RefKey, std::shared_ptr<RefEntry>> refs;
    size_t ref_bytes = 0, ref_cap = (size_t)4 << 30;
    uint64_t ref_clock = 0;
    // Released when the creator has destroyed the context and every request is released.
    ~Context() {
        (void)hipSetDevice(device);
        for (auto s : streams) (void)hipStreamSynchronize(s);
        if (own_stream) (void)hipStreamSynchronize(own_stream);
        for (auto& kv : refs) (void)hipEventDestroy(kv.second->ready);
        refs.clear();
        for (auto s : streams) (void)hipStreamDestroy(s);
        if (own_stream) (void)hipStreamDestroy(own_stream);
        delete pool;
    }
};

// ------------------------------------------------------------------------------------------
// a request and its results
// ------------------------------------------------------------------------------------------
struct Request {
    std::shared_ptr<Context> ctx_ref;   // keeps the pool and streams alive until release
    Context* ctx = nullptr;
    Plan plan;
    std::atomic<int> status{1};
    std::mutex mu;
    std::condition_variable cv;
    bool done = false;
    bool started = false;
    size_t reserved = 0, retained = 0;
    Clock::time_point t_submit, t_start, t_end;
    std::shared_ptr<RefEntry> ref;
    // canonical factors: per block, 3 axes of R x N[l]
    std::vector<DevBuf> U;             // one buffer per block
    size_t U_axis_off[3]{};
    DevBuf def_cells, def_scale;       // defects for sampling (n_def x 3, n_def)
    DevBuf lam;                        // block charges
    // Tucker
    int r[3]{};
    std::vector<double> sigma[3];
    int sweeps[3]{};
    double tails[3]{};
    double norm_A = 0, norm_xi = 0, bound = 0;
    DevBuf Z[3];                       // r_l x N_l FP64
    DevBuf core;                       // r1 r2 r3, FP64 or FP32 (precision)
    DevBuf tile;
    std::map<std::string, double> t_ms;
    std::map<std::string, double> bytes;
};

static void finish(Request* q, int status) {
    // notify under the lock: a waiter may free the request as soon as it sees `done`
    std::lock_guard<std::mutex> lk(q->mu);
    q->t_end = Clock::now();
    q->status.store(status);
    q->done = true;
    q->cv.notify_all();
}

// stage timer on a stream
struct StageTimer {
    hipStream_t st;
    std::vector<std::pair<std::string, std::pair<hipEvent_t, hipEvent_t>>> ev;
    explicit StageTimer(hipStream_t s) : st(s) {}
    ~StageTimer() {
        for (auto& e : ev) {
            (void)hipEventDestroy(e.second.first);
            (void)hipEventDestroy(e.second.second);
        }
    }
    void begin(const std::string& name) {
        hipEvent_t a, b;
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
        (void)hipEventRecord(a, st);
        ev.push_back({name, {a, b}});
    }
    void end() { (void)hipEventRecord(ev.back().second.second, st); }
    void collect(std::map<std::string, double>& out) {
        for (auto& e : ev) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, e.second.first, e.second.second) == hipSuccess) out[e.first] += ms;
        }
    }
};

// ------------------------------------------------------------------------------------------
// reference vectors: cached per (kernel, quadrature, grid)
// ------------------------------------------------------------------------------------------
static int get_reference(Context* c, const Plan& P, hipStream_t st, std::shared_ptr<RefEntry>& out) {
    RefKey key{P.kernel.kind, P.kernel.param, P.kernel.M, P.h_u, P.s, P.h, P.N_ref};
    std::shared_ptr<RefEntry> e;
    bool build = false;
    {
        std::lock_guard<std::mutex> lk(c->ref_mu);
        auto it = c->refs.find(key);
        if (it != c->refs.end()) {
            e = it->second;
        } else {
            // evict unused entries beyond the cap
            size_t need = (size_t)P.R * P.ldg * 8;
            while (c->ref_bytes + need > c->ref_cap) {
                auto victim = c->refs.end();
                for (auto jt = c->refs.begin(); jt != c->refs.end(); ++jt)
                    if (jt->second->users.load() == 0 &&
                        (victim == c->refs.end() || jt->second->last_use < victim->second->last_use))
                        victim = jt;
                if (victim == c->refs.end()) break;
                c->ref_bytes -= victim->second->bytes;
                c->refs.erase(victim);
            }
            e = std::make_shared<RefEntry>();
            e->R = P.R;
            e->ldg = P.ldg;
            e->N_ref = P.N_ref;
            e->bytes = need;
            int rc = e->G.get(c->pool, need);
            if (rc) return rc;
            LSUM_HIP(hipEventCreateWithFlags(&e->ready, hipEventDisableTiming));
            c->refs[key] = e;
            c->ref_bytes += need;
            build = true;
        }
        e->users.fetch_add(1);
        e->last_use = ++c->ref_clock;
    }
    if (build) {
        std::vector<double> w13(P.R);
        for (int q = 0; q < P.R; ++q) w13[q] = std::cbrt(P.w[q]);
        DevBuf tw;
        int rc = tw.get(c->pool, 2 * P.R * sizeof(double));
        if (rc) return rc;
        LSUM_HIP(hipMemcpyAsync(tw.as<double>(), P.t.data(), P.R * 8, hipMemcpyHostToDevice, st));
        LSUM_HIP(hipMemcpyAsync(tw.as<double>() + P.R, w13.data(), P.R * 8, hipMemcpyHostToDevice, st));
        launch_collocate(st, P.R, tw.as<double>(), tw.as<double>() + P.R, P.N_ref, P.h, e->G.as<double>(), P.ldg);
        LSUM_HIP(hipGetLastError());
        LSUM_HIP(hipEventRecord(e->ready, st));
        LSUM_HIP(hipStreamSynchronize(st));   // tw is released after this
    } else {
        LSUM_HIP(hipStreamWaitEvent(st, e->ready, 0));
    }
    out = e;
    return LSUM_OK;
}

static void drop_reference(Request* q) {
    if (q->ref) {
        q->ref->users.fetch_sub(1);
        q->ref.reset();
    }
}

// ------------------------------------------------------------------------------------------
// the pipeline of one request
// ------------------------------------------------------------------------------------------
static int run_request(Request* q, hipStream_t st) {
    Context* c = q->ctx;
    Plan& P = q->plan;
    StageTimer tm(st);
    int rc;
    // (1)-(2) quadrature (host, done in the plan) and reference vectors
    tm.begin("reference");
    rc = get_reference(c, P, st, q->ref);
    tm.end();
    if (rc) return rc;
    const double* G = q->ref->G.as<double>();

    // (3) assembled shift-sums for every block and axis in one launch
    const int nb = (int)P.blocks.size();
    const size_t sumN = (size_t)P.N[0] + P.N[1] + P.N[2];
    q->U_axis_off[0] = 0;
    q->U_axis_off[1] = (size_t)P.R * P.N[0];
    q->U_axis_off[2] = (size_t)P.R * (P.N[0] + P.N[1]);
    q->U.resize(nb);
    std::vector<int32_t> sites_h;
    std::vector<size_t> site_off;
    for (int b = 0; b < nb; ++b)
        for (int l = 0; l < 3; ++l) {
            site_off.push_back(sites_h.size());
            sites_h.insert(sites_h.end(), P.offs[l][b].begin(), P.offs[l][b].end());
        }
    DevBuf sites_d, jobs_d;
    if ((rc = sites_d.get(c->pool, sites_h.size() * 4))) return rc;
    std::vector<ShiftJob> jobs;
    int maxN = 0;
    for (int b = 0; b < nb; ++b) {
        if ((rc = q->U[b].get(c->pool, (size_t)P.R * sumN * 8))) return rc;
        for (int l = 0; l < 3; ++l) {
            ShiftJob j;
            j.G = G;
            j.U = q->U[b].as<double>() + q->U_axis_off[l];
            j.sites = sites_d.as<int32_t>() + site_off[3 * b + l];
            j.n_sites = (int)P.offs[l][b].size();
            j.N_axis = P.N[l];
            j.ldu = P.N[l];
            j.ldg = P.ldg;
            j.N_ref = P.N_ref;
            j.R = P.R;
            jobs.push_back(j);
            maxN = std::max(maxN, P.N[l]);
        }
    }
    if ((rc = jobs_d.get(c->pool, jobs.size() * sizeof(ShiftJob)))) return rc;
    tm.begin("shift_sum");
    LSUM_HIP(hipMemcpyAsync(sites_d.p, sites_h.data(), sites_h.size() * 4, hipMemcpyHostToDevice, st));
    LSUM_HIP(hipMemcpyAsync(jobs_d.p, jobs.data(), jobs.size() * sizeof(ShiftJob), hipMemcpyHostToDevice, st));
    launch_shift_sum(st, jobs_d.as<ShiftJob>(), (int)jobs.size(), maxN, P.R);
    LSUM_HIP(hipGetLastError());
    tm.end();
    q->bytes["canonical"] = (double)nb * P.R * sumN * 8;

    // block charges and defect table (for canonical sampling)
    {
        std::vector<double> lam(nb);
        for (int b = 0; b < nb; ++b) lam[b] = P.blocks[b].charge;
        if ((rc = q->lam.get(c->pool, nb * 8))) return rc;
        LSUM_HIP(hipMemcpyAsync(q->lam.p, lam.data(), nb * 8, hipMemcpyHostToDevice, st));
        const int nd = (int)P.defects.size();
        if (nd > 0) {
            std::vector<int32_t> cells(3 * nd);
            std::vector<double> sc(nd);
            for (int s = 0; s < nd; ++s) {
                const auto& d = P.defects[s];
                for (int l = 0; l < 3; ++l) cells[3 * s + l] = P.offs[l][d.block][d.site[l]];
                sc[s] = d.dZ;
            }
            if ((rc = q->def_cells.get(c->pool, cells.size() * 4))) return rc;
            if ((rc = q->def_scale.get(c->pool, nd * 8))) return rc;
            LSUM_HIP(hipMemcpyAsync(q->def_cells.p, cells.data(), cells.size() * 4, hipMemcpyHostToDevice, st));
            LSUM_HIP(hipMemcpyAsync(q->def_scale.p, sc.data(), nd * 8, hipMemcpyHostToDevice, st));
        }
    }
    if (!P.tucker()) {
        LSUM_HIP(hipStreamSynchronize(st));
        tm.collect(q->t_ms);
        return LSUM_OK;
    }

    // (4) side matrices per mode: lattice sources and defect windows (unnormalised)
    DevBuf cols[3], W[3], nrm[3], C[3], aux;
    std::vector<double> nrm_h[3];
    const GemmPrec prec = P.precision == LSUM_FP64 ? GEMM_F64 : (P.precision == LSUM_FP32 ? GEMM_F32 : GEMM_BF16X3);
    tm.begin("columns");
    for (int l = 0; l < 3; ++l) {
        const int D = P.D[l], N = P.N[l];
        if ((rc = cols[l].get(c->pool, (size_t)D * N * 8))) return rc;
        if ((rc = nrm[l].get(c->pool, (size_t)D * 8))) return rc;
        std::vector<const double*> latp(P.n_lat[l]);
        for (int s = 0; s < P.n_lat[l]; ++s) latp[s] = q->U[P.lat_block[l][s]].as<double>() + q->U_axis_off[l];
        DevBuf lp, wc;
        if ((rc = lp.get(c->pool, std::max<size_t>(1, latp.size()) * sizeof(void*)))) return rc;
        if ((rc = wc.get(c->pool, std::max<size_t>(1, P.win_cell[l].size()) * 4))) return rc;
        LSUM_HIP(hipMemcpyAsync(lp.p, latp.data(), latp.size() * sizeof(void*), hipMemcpyHostToDevice, st));
        if (!P.win_cell[l].empty())
            LSUM_HIP(hipMemcpyAsync(wc.p, P.win_cell[l].data(), P.win_cell[l].size() * 4, hipMemcpyHostToDevice, st));
        launch_gather_columns(st, P.R, P.n_lat[l], lp.as<const double*>(), P.N[l], P.n_win[l],
                              wc.as<int32_t>(), G, P.ldg, P.N_ref, N, cols[l].as<double>(), N);
        launch_row_norms(st, D, N, cols[l].as<double>(), N, nrm[l].as<double>());
        nrm_h[l].resize(D);
        LSUM_HIP(hipMemcpyAsync(nrm_h[l].data(), nrm[l].p, D * 8, hipMemcpyDeviceToHost, st));
        LSUM_HIP(hipStreamSynchronize(st));   // lp, wc released after the kernels ran
    }
    tm.end();
    for (int l = 0; l < 3; ++l)
        for (double v : nrm_h[l])
            if (!(v > 0.0)) return fail(LSUM_E_INVALID, "a side-matrix column vanishes on the grid");

    // weighted, normalised side matrices: row j = col_j / |col_j| * sqrt(multiplicity)
    tm.begin("svd");
    for (int l = 0; l < 3; ++l) {
        const int D = P.D[l], N = P.N[l];
        std::vector<double> sc(D);
        for (int j = 0; j < D; ++j) sc[j] = std::sqrt((double)P.src_mult[l][j / P.R]) / nrm_h[l][j];
        DevBuf scd;
        if ((rc = scd.get(c->pool, D * 8))) return rc;
        if ((rc = W[l].get(c->pool, (size_t)D * N * 8))) return rc;
        LSUM_HIP(hipMemcpyAsync(scd.p, sc.data(), D * 8, hipMemcpyHostToDevice, st));
        launch_scale_rows(st, D, N, cols[l].as<double>(), N, scd.as<double>(), W[l].as<double>(), N);
        DevBuf work;
        size_t wb = jacobi_work_bytes(D, N);
        if ((rc = work.get(c->pool, wb))) return rc;
        std::vector<int32_t> order;
        rc = jacobi_svd(st, D, N, W[l].as<double>(), N, 1e-12, 40, q->sigma[l], order, &q->sweeps[l],
                        work.as<double>(), wb);
        if (rc) return rc;
    }
    tm.end();

    // (5) ||A|| from the column Grams, ||xi|| from the norms, truncation (host FP64)
    tm.begin("norm");
    for (int l = 0; l < 3; ++l) {
        const int D = P.D[l], N = P.N[l];
        if ((rc = C[l].get(c->pool, (size_t)D * D * 8))) return rc;
        GemmArgs a{};
        a.m = D; a.n = D; a.k = N;
        a.A = cols[l].p; a.sam = N; a.sak = 1;
        a.B = cols[l].p; a.sbk = 1; a.sbn = N;
        a.C = C[l].p; a.scm = D; a.scn = 1;
        a.alpha = 1.0; a.beta = 0.0; a.batch = 1;
        launch_gemm(st, GEMM_F64, a);
    }
    DevBuf src_d, scale_d, part_d;
    const int ng = P.n_groups;
    std::vector<int32_t> srcs(3 * (size_t)ng);
    for (int l = 0; l < 3; ++l) std::copy(P.g_src[l].begin(), P.g_src[l].end(), srcs.begin() + (size_t)l * ng);
    if ((rc = src_d.get(c->pool, srcs.size() * 4))) return rc;
    if ((rc = scale_d.get(c->pool, ng * 8))) return rc;
    if ((rc = part_d.get(c->pool, ng * 8))) return rc;
    LSUM_HIP(hipMemcpyAsync(src_d.p, srcs.data(), srcs.size() * 4, hipMemcpyHostToDevice, st));
    LSUM_HIP(hipMemcpyAsync(scale_d.p, P.g_scale.data(), ng * 8, hipMemcpyHostToDevice, st));
    const int32_t* s1 = src_d.as<int32_t>();
    const int32_t* s2 = s1 + ng;
    const int32_t* s3 = s2 + ng;
    launch_cp_norm2(st, P.R, ng, s1, s2, s3, scale_d.as<double>(), C[0].as<double>(), C[1].as<double>(),
                    C[2].as<double>(), P.D[0], P.D[1], P.D[2], part_d.as<double>(), ng);
    std::vector<double> part(ng);
    LSUM_HIP(hipMemcpyAsync(part.data(), part_d.p, ng * 8, hipMemcpyDeviceToHost, st));
    LSUM_HIP(hipStreamSynchronize(st));
    tm.end();
    for (int l = 0; l < 3; ++l) C[l].reset();
    double nA2 = 0.0;
    for (double v : part) nA2 += v;
    q->norm_A = std::sqrt(std::max(nA2, 0.0));
    double nxi2 = 0.0;
    for (int g = 0; g < ng; ++g)
        for (int k = 0; k < P.R; ++k) {
            double xi = P.g_scale[g];
            for (int l = 0; l < 3; ++l) xi *= nrm_h[l][(size_t)P.g_src[l][g] * P.R + k];
            nxi2 += xi * xi;
        }
    q->norm_xi = std::sqrt(nxi2);
    const double thr = P.eps * q->norm_A / (3.0 * q->norm_xi);
    q->bound = 0.0;
    for (int l = 0; l < 3; ++l) {
        const auto& sg = q->sigma[l];
        const int D = (int)sg.size();
        std::vector<double> tail(D + 1, 0.0);
        for (int k = D - 1; k >= 0; --k) tail[k] = tail[k + 1] + sg[k] * sg[k];
        int r = D;
        for (int k = 1; k <= D; ++k)
            if (std::sqrt(tail[k]) <= thr) { r = k; break; }
        r = std::min(r, P.N[l]);
        q->r[l] = r;
        q->tails[l] = std::sqrt(tail[r]);
        q->bound += q->tails[l];
    }
    q->bound *= q->norm_xi;

    // Tucker factors Z_l = leading rotated columns / sigma
    for (int l = 0; l < 3; ++l) {
        const int r = q->r[l], N = P.N[l];
        std::vector<double> inv(r);
        std::vector<int32_t> ord(r);
        for (int a = 0; a < r; ++a) { inv[a] = 1.0 / q->sigma[l][a]; ord[a] = a; }
        DevBuf od, iv;
        if ((rc = od.get(c->pool, r * 4))) return rc;
        if ((rc = iv.get(c->pool, r * 8))) return rc;
        if ((rc = q->Z[l].get(c->pool, (size_t)r * N * 8))) return rc;
        LSUM_HIP(hipMemcpyAsync(od.p, ord.data(), r * 4, hipMemcpyHostToDevice, st));
        LSUM_HIP(hipMemcpyAsync(iv.p, inv.data(), r * 8, hipMemcpyHostToDevice, st));
        launch_gather_scale_rows(st, r, N, W[l].as<double>(), N, od.as<int32_t>(), iv.as<double>(),
                                 q->Z[l].as<double>(), N);
        LSUM_HIP(hipStreamSynchronize(st));
        W[l].reset();
    }

    // (6) projections Y_l = Z_l cols_l^T (r_l x D_l) in the problem's precision
    const size_t es = (prec == GEMM_F64) ? 8 : 4;
    DevBuf Y[3];
    tm.begin("projection");
    for (int l = 0; l < 3; ++l) {
        const int r = q->r[l], D = P.D[l], N = P.N[l];
        if ((rc = Y[l].get(c->pool, (size_t)r * D * es))) return rc;
        const void* Zp = q->Z[l].p;
        const void* Cp = cols[l].p;
        DevBuf Zf, Cf;
        if (prec != GEMM_F64) {
            if ((rc = Zf.get(c->pool, (size_t)r * N * 4))) return rc;
            if ((rc = Cf.get(c->pool, (size_t)D * N * 4))) return rc;
            launch_f64_to_f32(st, (long)r * N, q->Z[l].as<double>(), Zf.as<float>());
            launch_f64_to_f32(st, (long)D * N, cols[l].as<double>(), Cf.as<float>());
            Zp = Zf.p;
            Cp = Cf.p;
        }
        GemmArgs a{};
        a.m = r; a.n = D; a.k = N;
        a.A = Zp; a.sam = N; a.sak = 1;
        a.B = Cp; a.sbk = 1; a.sbn = N;
        a.C = Y[l].p; a.scm = D; a.scn = 1;
        a.alpha = 1.0; a.beta = 0.0; a.batch = 1;
        launch_gemm(st, prec, a);
        LSUM_HIP(hipStreamSynchronize(st));
    }
    tm.end();
    for (int l = 0; l < 3; ++l) cols[l].reset();

    // (7) core mu = sum_nu xi_nu y1 (x) y2 (x) y3 (eq. C-core), unnormalised columns: xi = scale
    tm.begin("core");
    {
        const long plane = (long)q->r[0] * q->r[1] * q->r[2];
        if ((rc = q->core.get(c->pool, (size_t)plane * es))) return rc;
        CoreArgs ca{};
        ca.r1 = q->r[0]; ca.r2 = q->r[1]; ca.r3 = q->r[2]; ca.R = P.R; ca.n_groups = ng;
        ca.Y1 = Y[0].p; ca.Y2 = Y[1].p; ca.Y3 = Y[2].p;
        ca.ldy1 = P.D[0]; ca.ldy2 = P.D[1]; ca.ldy3 = P.D[2];
        ca.src1 = s1; ca.src2 = s2; ca.src3 = s3;
        ca.scale = scale_d.as<double>();
        ca.core = q->core.p;
        const long tiles = (long)((ca.r3 + 63) / 64) * ((ca.r1 + 7) / 8) * ((ca.r2 + 7) / 8);
        const long K = (long)ng * P.R;
        int ks = 1;
        while (tiles * ks < 1024 && ks < 64 && K / (ks * 2) >= 256) ks *= 2;
        DevBuf work;
        if (ks > 1 && (rc = work.get(c->pool, (size_t)plane * ks * es))) return rc;
        launch_core(st, prec, ca, ks, work.p);
        LSUM_HIP(hipGetLastError());
        LSUM_HIP(hipStreamSynchronize(st));
        q->bytes["core"] = (double)plane * es;
    }
    tm.end();

    // (8) optional tile: V = mu x_3 Z3 x_2 Z2 x_1 Z1 restricted to [lo, lo+T)
    if (P.has_tile()) {
        tm.begin("tile");
        const int r1 = q->r[0], r2 = q->r[1], r3 = q->r[2];
        const int T1 = P.tile_T[0], T2 = P.tile_T[1], T3 = P.tile_T[2];
        const void* Zp[3];
        DevBuf Zf[3];
        for (int l = 0; l < 3; ++l) {
            Zp[l] = q->Z[l].p;
            if (prec != GEMM_F64) {
                if ((rc = Zf[l].get(c->pool, (size_t)q->r[l] * P.N[l] * 4))) return rc;
                launch_f64_to_f32(st, (long)q->r[l] * P.N[l], q->Z[l].as<double>(), Zf[l].as<float>());
                Zp[l] = Zf[l].p;
            }
        }
        DevBuf X1, X2;
        if ((rc = X1.get(c->pool, (size_t)r1 * r2 * T3 * es))) return rc;
        if ((rc = X2.get(c->pool, (size_t)r1 * T2 * T3 * es))) return rc;
        if ((rc = q->tile.get(c->pool, (size_t)T1 * T2 * T3 * es))) return rc;
        const long e = (long)es;
        GemmArgs a{};
        // X1[(a,b), n] = sum_c mu[(a,b), c] Z3[c, lo3 + n]
        a.m = r1 * r2; a.n = T3; a.k = r3;
        a.A = q->core.p; a.sam = r3; a.sak = 1;
        a.B = (const char*)Zp[2] + (long)P.tile_lo[2] * e; a.sbk = P.N[2]; a.sbn = 1;
        a.C = X1.p; a.scm = T3; a.scn = 1;
        a.alpha = 1.0; a.beta = 0.0; a.batch = 1;
        launch_gemm(st, prec, a);
        // X2[a][m, n] = sum_b Z2[b, lo2 + m] X1[(a,b), n]
        a = GemmArgs{};
        a.m = T2; a.n = T3; a.k = r2;
        a.A = (const char*)Zp[1] + (long)P.tile_lo[1] * e; a.sam = 1; a.sak = P.N[1];
        a.B = X1.p; a.sbk = T3; a.sbn = 1;
        a.C = X2.p; a.scm = T3; a.scn = 1;
        a.alpha = 1.0; a.beta = 0.0; a.batch = r1; a.bA = 0; a.bB = (long)r2 * T3; a.bC = (long)T2 * T3;
        launch_gemm(st, prec, a);
        // V[m, (n2,n3)] = sum_a Z1[a, lo1 + m] X2[a, (n2,n3)]
        a = GemmArgs{};
        a.m = T1; a.n = T2 * T3; a.k = r1;
        a.A = (const char*)Zp[0] + (long)P.tile_lo[0] * e; a.sam = 1; a.sak = P.N[0];
        a.B = X2.p; a.sbk = (long)T2 * T3; a.sbn = 1;
        a.C = q->tile.p; a.scm = (long)T2 * T3; a.scn = 1;
        a.alpha = 1.0; a.beta = 0.0; a.batch = 1;
        launch_gemm(st, prec, a);
        LSUM_HIP(hipGetLastError());
        LSUM_HIP(hipStreamSynchronize(st));
        tm.end();
        q->bytes["tile"] = (double)T1 * T2 * T3 * es;
    }
    LSUM_HIP(hipStreamSynchronize(st));
    tm.collect(q->t_ms);
    return LSUM_OK;
}

size_t retained_bytes(const Request* q) {
    size_t b = 0;
    for (const auto& u : q->U) b += u.n;
    for (int l = 0; l < 3; ++l) b += q->Z[l].n;
    return b + q->core.n + q->tile.n + q->lam.n + q->def_cells.n + q->def_scale.n;
}

static void worker(Context* c, int slot) {
    (void)hipSetDevice(c->device);
    hipStream_t st = c->streams[slot];
    for (;;) {
        Request* q = nullptr;
        {
            std::unique_lock<std::mutex> lk(c->mu);
            c->cv.wait(lk, [&] {
                if (c->stopping) return true;
                if (c->queue.empty()) return false;
                Request* h = c->queue.front();
                return h->reserved <= c->budget - std::min(c->used, c->budget) || c->used == 0;
            });
            if (c->stopping && c->queue.empty()) return;
            if (c->stopping) {
                q = c->queue.front();
                c->queue.pop_front();
                lk.unlock();
                finish(q, LSUM_E_CANCELLED);
                continue;
            }
            q = c->queue.front();
            c->queue.pop_front();
            c->used += q->reserved;
            q->started = true;
        }
        c->cv.notify_all();
        q->t_start = Clock::now();
        int rc;
        try {
            rc = run_request(q, st);
        } catch (const std::exception& ex) {
            rc = fail(LSUM_E_DEVICE, std::string("exception: ") + ex.what());
        }
        if (rc != LSUM_OK) {
            (void)hipStreamSynchronize(st);
            (void)hipGetLastError();
        }
        const size_t keep = rc == LSUM_OK ? retained_bytes(q) : 0;
        {
            std::lock_guard<std::mutex> lk(c->mu);
            c->used -= q->reserved;
            c->used += keep;
            q->retained = keep;
        }
        c->cv.notify_all();
        finish(q, rc);
    }
}

}  // namespace lsum

// ------------------------------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------------------------------
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
    c.pool = new DevPool(device);
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

int lsum_submit(lsum_ctx x, const lsum_problem* p, int nonblocking, lsum_req* out) {
    if (!x || !p || !out) return fail(LSUM_E_INVALID, "null argument");
    auto* r = new lsum_req_s();
    Request& q = r->q;
    q.ctx_ref = x->sp;
    q.ctx = &x->c;
    int rc = make_plan(*p, q.plan);
    if (rc != LSUM_OK) {
        delete r;
        return rc;
    }
    q.reserved = q.plan.planned_bytes();
    Context& c = x->c;
    if (q.reserved > c.budget) {
        delete r;
        return fail(LSUM_E_NOMEM, "the request can never fit the HBM budget");
    }
    {
        std::lock_guard<std::mutex> lk(c.mu);
        if (c.stopping) {
            delete r;
            return fail(LSUM_E_STATE, "context is shutting down");
        }
        if (c.queue.size() >= c.max_queue) {
            if (nonblocking) {
                delete r;
                return fail(LSUM_E_BUSY, "queue full");
            }
        }
        q.t_submit = Clock::now();
        c.queue.push_back(&q);
    }
    c.cv.notify_all();
    *out = r;
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
    const Plan& P = q.plan;
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
    if (q.started) info->t_queue_ms = ms_since(q.t_submit, q.t_start);
    if (q.done && q.started) info->t_run_ms = ms_since(q.t_start, q.t_end);
    return LSUM_OK;
}

static int copy_out(void* dst, const void* src, size_t bytes, int on_device, int device) {
    LSUM_HIP(hipSetDevice(device));
    LSUM_HIP(hipMemcpy(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
    return LSUM_OK;
}

int lsum_get_canonical(lsum_req r, int block, double* U0, double* U1, double* U2, int on_device) {
    int rc = need_done(r);
    if (rc) return rc;
    Request& q = r->q;
    const Plan& P = q.plan;
    if (block < 0 || block >= (int)P.blocks.size()) return fail(LSUM_E_INVALID, "bad block index");
    double* dst[3] = {U0, U1, U2};
    for (int l = 0; l < 3; ++l) {
        if (!dst[l]) continue;
        rc = copy_out(dst[l], q.U[block].as<double>() + q.U_axis_off[l], (size_t)P.R * P.N[l] * 8, on_device,
                      q.ctx->device);
        if (rc) return rc;
    }
    return LSUM_OK;
}

int lsum_get_tucker(lsum_req r, double* Z0, double* Z1, double* Z2, double* core, int on_device) {
    int rc = need_done(r);
    if (rc) return rc;
    Request& q = r->q;
    const Plan& P = q.plan;
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
    const Plan& P = q.plan;
    LSUM_HIP(hipSetDevice(c.device));
    hipStream_t st = c.own_stream;
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
    if (!P.tucker()) {
        // canonical: the blocks' assembled factors (weighted by the block charge), then the
        // defect windows straight from the reference rows
        LSUM_HIP(hipMemsetAsync(out_d, 0, (size_t)n * 8, st));
        for (int b = 0; b < (int)P.blocks.size(); ++b)
            launch_sample_block(st, P.R, q.U[b].as<double>(), q.U[b].as<double>() + q.U_axis_off[1],
                                q.U[b].as<double>() + q.U_axis_off[2], P.N[0], P.N[1], P.N[2], P.h,
                                P.blocks[b].charge, n, xyz_d, out_d);
        if (!P.defects.empty())
            launch_sample_windows(st, P.R, q.ref->G.as<double>(), P.ldg, P.N_ref, (int)P.defects.size(),
                                  q.def_cells.as<int32_t>(), q.def_scale.as<double>(), P.N[0], P.N[1],
                                  P.N[2], P.h, n, xyz_d, out_d);
    } else {
        // Tucker: snap, contract mode 3 with a GEMM per chunk of points, finish modes 1, 2
        const int r1 = q.r[0], r2 = q.r[1], r3 = q.r[2];
        const size_t ncore = (size_t)r1 * r2 * r3;
        DevBuf core64, idx, W, Z3s;
        const double* core_d = q.core.as<double>();
        if (P.precision != LSUM_FP64) {
            if ((rc = core64.get(c.pool, ncore * 8))) return rc;
            launch_f32_to_f64(st, (long)ncore, q.core.as<float>(), core64.as<double>());
            core_d = core64.as<double>();
        }
        if ((rc = idx.get(c.pool, (size_t)n * 12))) return rc;
        launch_snap_points(st, n, xyz_d, P.N[0], P.N[1], P.N[2], P.h, idx.as<int32_t>());
        // points outside the grid get index -1; clamp for the gather and mark in the finish
        int chunk = (int)std::max<size_t>(1, std::min<size_t>((size_t)n, ((size_t)1 << 28) / std::max<size_t>(1, (size_t)r1 * r2)));
        chunk = std::min(chunk, 4096);
        if ((rc = W.get(c.pool, (size_t)r1 * r2 * chunk * 8))) return rc;
        if ((rc = Z3s.get(c.pool, (size_t)r3 * chunk * 8))) return rc;
        std::vector<int32_t> idx_h((size_t)3 * n);
        LSUM_HIP(hipMemcpyAsync(idx_h.data(), idx.p, (size_t)n * 12, hipMemcpyDeviceToHost, st));
        LSUM_HIP(hipStreamSynchronize(st));
        DevBuf i3c;
        if ((rc = i3c.get(c.pool, (size_t)chunk * 4))) return rc;
        for (int p0 = 0; p0 < n; p0 += chunk) {
            const int P_ = std::min(chunk, n - p0);
            std::vector<int32_t> i3(P_);
            for (int p = 0; p < P_; ++p) i3[p] = std::max(0, idx_h[(size_t)2 * n + p0 + p]);
            LSUM_HIP(hipMemcpyAsync(i3c.p, i3.data(), P_ * 4, hipMemcpyHostToDevice, st));
            launch_select_cols(st, r3, P_, q.Z[2].p, P.N[2], i3c.as<int32_t>(), Z3s.p, 8);
            GemmArgs a{};
            a.m = r1 * r2; a.n = P_; a.k = r3;
            a.A = core_d; a.sam = r3; a.sak = 1;
            a.B = Z3s.p; a.sbk = P_; a.sbn = 1;
            a.C = W.p; a.scm = P_; a.scn = 1;
            a.alpha = 1.0; a.beta = 0.0; a.batch = 1;
            launch_gemm(st, GEMM_F64, a);
            launch_tucker_finish(st, r1, r2, P_, W.as<double>(), q.Z[0].as<double>(), P.N[0],
                                 q.Z[1].as<double>(), P.N[1], idx.as<int32_t>() + p0,
                                 idx.as<int32_t>() + n + p0, out_d + p0);
            LSUM_HIP(hipStreamSynchronize(st));
        }
        // mark points whose third index was outside the grid
        bool any_out = false;
        for (int p = 0; p < n; ++p) any_out |= idx_h[(size_t)2 * n + p] < 0;
        if (any_out) {
            std::vector<double> o(n);
            LSUM_HIP(hipMemcpyAsync(o.data(), out_d, (size_t)n * 8, hipMemcpyDeviceToHost, st));
            LSUM_HIP(hipStreamSynchronize(st));
            for (int p = 0; p < n; ++p)
                if (idx_h[(size_t)2 * n + p] < 0) o[p] = std::nan("");
            LSUM_HIP(hipMemcpyAsync(out_d, o.data(), (size_t)n * 8, hipMemcpyHostToDevice, st));
        }
    }
    LSUM_HIP(hipGetLastError());
    if (!on_device) LSUM_HIP(hipMemcpyAsync(out, out_d, (size_t)n * 8, hipMemcpyDeviceToHost, st));
    LSUM_HIP(hipStreamSynchronize(st));
    return LSUM_OK;
}

int lsum_get_tile(lsum_req r, void* out, int elem_size, int on_device) {
    int rc = need_done(r);
    if (rc) return rc;
    Request& q = r->q;
    const Plan& P = q.plan;
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
    const Plan& P = q.plan;
    {
        std::lock_guard<std::mutex> lk(q.mu);
        o << "{\"status\":" << (q.done ? q.status.load() : 1) << ",\"R\":" << P.R << ",\"n_groups\":" << P.n_groups
          << ",\"h_u\":" << P.h_u << ",\"s\":" << P.s << ",\"N\":[" << P.N[0] << "," << P.N[1] << "," << P.N[2]
          << "],\"D\":[" << P.D[0] << "," << P.D[1] << "," << P.D[2] << "],\"r\":[" << q.r[0] << "," << q.r[1]
          << "," << q.r[2] << "],\"sweeps\":[" << q.sweeps[0] << "," << q.sweeps[1] << "," << q.sweeps[2]
          << "],\"tails\":[" << q.tails[0] << "," << q.tails[1] << "," << q.tails[2] << "],\"norm_A\":" << q.norm_A
          << ",\"norm_xi\":" << q.norm_xi << ",\"bound\":" << q.bound << ",\"offsets\":[";
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
        for (auto& kv : q.t_ms) {
            o << (first ? "" : ",") << "\"" << kv.first << "\":" << kv.second;
            first = false;
        }
        o << "},\"bytes\":{";
        first = true;
        for (auto& kv : q.bytes) {
            o << (first ? "" : ",") << "\"" << kv.first << "\":" << kv.second;
            first = false;
        }
        o << "}";
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
    {
        std::lock_guard<std::mutex> lk(c.mu);
        c.used -= std::min(c.used, q.retained);
    }
    c.cv.notify_all();
    delete r;
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

int lsum_shift_sum(lsum_ctx x, void* stream, int R, const double* G_dev, int ldg, int N_ref, int N_axis,
                   int n_sites, const int32_t* sites, double* U_dev, int ldu) {
    if (!x || !G_dev || !U_dev || (n_sites > 0 && !sites)) return fail(LSUM_E_INVALID, "null argument");
    if (R < 1 || N_axis < 1 || N_axis > N_ref || ldg < 2 * N_ref - 1 || ldu < N_axis || n_sites < 0)
        return fail(LSUM_E_INVALID, "bad sizes");
    for (int k = 0; k < n_sites; ++k)
        if (sites[k] < 0 || sites[k] >= N_axis) return fail(LSUM_E_OUT_OF_BOX, "site index outside the axis");
    LSUM_HIP(hipSetDevice(x->c.device));
    hipStream_t st = pick(x, stream);
    DevBuf sd, jd;
    int rc = sd.get(x->c.pool, std::max(1, n_sites) * 4);
    if (rc) return rc;
    if ((rc = jd.get(x->c.pool, sizeof(ShiftJob)))) return rc;
    ShiftJob j{G_dev, U_dev, sd.as<int32_t>(), n_sites, N_axis, ldu, ldg, N_ref, R};
    if (n_sites > 0) LSUM_HIP(hipMemcpyAsync(sd.p, sites, n_sites * 4, hipMemcpyHostToDevice, st));
    LSUM_HIP(hipMemcpyAsync(jd.p, &j, sizeof(j), hipMemcpyHostToDevice, st));
    launch_shift_sum(st, jd.as<ShiftJob>(), 1, N_axis, R);
    LSUM_HIP(hipGetLastError());
    LSUM_HIP(hipStreamSynchronize(st));
    return LSUM_OK;
}

int lsum_sample_canonical(lsum_ctx x, void* stream, int n_fac, int R, const double* U_dev, int ldu,
                          const double* lam, const int N[3], double h, int n_pts, const double* xyz_dev,
                          double* out_dev) {
    if (!x || !U_dev || !lam || !N || (n_pts > 0 && (!xyz_dev || !out_dev))) return fail(LSUM_E_INVALID, "null argument");
    if (n_fac < 1 || R < 1 || ldu < std::max(N[0], std::max(N[1], N[2])) || n_pts < 0) return fail(LSUM_E_INVALID, "bad sizes");
    LSUM_HIP(hipSetDevice(x->c.device));
    hipStream_t st = pick(x, stream);
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
    GemmArgs a{};
    a.m = m; a.n = n; a.k = k;
    a.A = A_dev; a.sam = sam; a.sak = sak;
    a.B = B_dev; a.sbk = sbk; a.sbn = sbn;
    a.C = C_dev; a.scm = scm; a.scn = scn;
    a.alpha = alpha; a.beta = beta; a.batch = 1;
    launch_gemm(st, prec == LSUM_FP64 ? GEMM_F64 : (prec == LSUM_FP32 ? GEMM_F32 : GEMM_BF16X3), a);
    LSUM_HIP(hipGetLastError());
    LSUM_HIP(hipStreamSynchronize(st));
    return LSUM_OK;
}

int lsum_jacobi_svd(lsum_ctx x, void* stream, int D, int N, double* A_dev, int lda, double tol, int max_sweeps,
                    double* sigma, int* sweeps) {
    if (!x || !A_dev || !sigma || !sweeps) return fail(LSUM_E_INVALID, "null argument");
    if (D < 1 || N < 1 || lda < N || !(tol > 0) || max_sweeps < 1) return fail(LSUM_E_INVALID, "bad sizes");
    LSUM_HIP(hipSetDevice(x->c.device));
    hipStream_t st = pick(x, stream);
    DevBuf work;
    const size_t wb = jacobi_work_bytes(D, N);
    int rc = work.get(x->c.pool, wb);
    if (rc) return rc;
    std::vector<double> s;
    std::vector<int32_t> order;
    rc = jacobi_svd(st, D, N, A_dev, lda, tol, max_sweeps, s, order, sweeps, work.as<double>(), wb);
    std::copy(s.begin(), s.end(), sigma);
    return rc;
}

}  // extern "C"

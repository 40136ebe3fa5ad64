// Runtime of the lattice-sum library: device buffer pool, reference-vector cache, stage timing
// and the request workers.  Each context owns n_slots workers, each with its own HIP stream;
// a worker admits requests from the shared FIFO queue when their planned HBM footprint fits the
// free budget, and fuses consecutive canonical (no-reduction) requests into one batch so that
// their shift-sums run as a single launch.  Requests on different slots overlap on the device.
#include "lsum_runtime.h"

#include <functional>

#include <algorithm>
#include <cmath>
#include <cstring>

namespace lsum {

// ------------------------------------------------------------------------------------------
// DevPool
// ------------------------------------------------------------------------------------------
DevPool::~DevPool() {
    for (auto& kv : free_) (void)hipFree(kv.second);
}

size_t DevPool::round(size_t n) {
    if (n <= (1u << 20)) {
        size_t r = 256;
        while (r < n) r <<= 1;
        return r;
    }
    return (n + (2u << 20) - 1) / (2u << 20) * (2u << 20);
}

int DevPool::alloc(size_t n, void** p, size_t* got) {
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

void DevPool::release(void* p, size_t n) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu_);
    free_.emplace(n, p);
    cached_ += n;
    if (cached_ > cap_) trim_locked();
}

void DevPool::trim() {
    std::lock_guard<std::mutex> lk(mu_);
    trim_locked();
}

void DevPool::trim_locked() {
    for (auto& kv : free_) (void)hipFree(kv.second);
    free_.clear();
    cached_ = 0;
}

// ------------------------------------------------------------------------------------------
// Context teardown: runs when the creator has destroyed the context and the last request has
// been released (requests keep the pool and streams alive)
// ------------------------------------------------------------------------------------------
Context::~Context() {
    (void)hipSetDevice(device);
    for (auto s : streams) (void)hipStreamSynchronize(s);
    for (auto s : aux) (void)hipStreamSynchronize(s);
    if (own_stream) (void)hipStreamSynchronize(own_stream);
    refs.clear();
    for (auto s : streams) (void)hipStreamDestroy(s);
    for (auto s : aux) (void)hipStreamDestroy(s);
    if (own_stream) (void)hipStreamDestroy(own_stream);
    delete pool;
}

// ------------------------------------------------------------------------------------------
// StageTimer
// ------------------------------------------------------------------------------------------
StageTimer::~StageTimer() {
    for (auto& e : ev_) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
}

void StageTimer::begin(const std::string& name, double bytes, double flops) {
    Ev e{name, nullptr, nullptr, bytes, flops, false};
    (void)hipEventCreate(&e.a);
    (void)hipEventCreate(&e.b);
    (void)hipEventRecord(e.a, st_);
    ev_.push_back(e);
}

void StageTimer::end() {
    (void)hipEventRecord(ev_.back().b, st_);
    ev_.back().closed = true;
}

KTime StageTimer::kernels(const std::string& name, double bytes, double flops) {
    Ev e{name, nullptr, nullptr, bytes, flops, true};
    (void)hipEventCreate(&e.a);
    (void)hipEventCreate(&e.b);
    ev_.push_back(e);
    KTime k;
    k.start = e.a;
    k.stop = e.b;
    return k;
}

void StageTimer::collect(std::map<std::string, double>& out, Context* c) {
    std::lock_guard<std::mutex> lk(c->prof_mu);
    for (auto& e : ev_) {
        // a stage left open by an error has no stop event; an event that a failed launch never
        // recorded makes the query fail, and the error it leaves on this thread is cleared so
        // that the worker's next batch does not report it as its own
        if (!e.closed) continue;
        float ms = 0;
        if (hipEventElapsedTime(&ms, e.a, e.b) != hipSuccess) {
            (void)hipGetLastError();
            continue;
        }
        out[e.name] += ms;
        StageStat& s = c->profile[e.name];
        s.ms += ms;
        s.bytes += e.bytes;
        s.flops += e.flops;
        s.launches += 1;
    }
}

void finish(Request* q, int status) {
    // notify under the lock: a waiter may free the request as soon as it sees `done`
    std::lock_guard<std::mutex> lk(q->mu);
    q->t_end = Clock::now();
    q->status.store(status);
    q->done = true;
    q->cv.notify_all();
}

// ------------------------------------------------------------------------------------------
// reference vectors: cached per (kernel, quadrature, grid) unless the cache is disabled
// ------------------------------------------------------------------------------------------
static int build_reference(Context* c, const Plan& P, hipStream_t st, RefEntry& e) {
    std::vector<double> w13(P.R);
    for (int q = 0; q < P.R; ++q) w13[q] = std::cbrt(P.w[q]);
    DevBuf tw;
    int rc = tw.get(c->pool, 2 * (size_t)P.R * sizeof(double));
    if (rc) return rc;
    LSUM_HIP(hipMemcpyAsync(tw.as<double>(), P.t.data(), P.R * 8, hipMemcpyHostToDevice, st));
    LSUM_HIP(hipMemcpyAsync(tw.as<double>() + P.R, w13.data(), P.R * 8, hipMemcpyHostToDevice, st));
    StageTimer tm(st);
    tm.begin("collocate", (double)P.R * (2 * P.N_ref - 1) * 8, 0);
    launch_collocate(st, P.R, tw.as<double>(), tw.as<double>() + P.R, P.N_ref, P.h, e.G.as<double>(), P.ldg);
    tm.end();
    LSUM_HIP(hipGetLastError());
    LSUM_HIP(hipStreamSynchronize(st));   // the rows are complete for every stream; tw is released
    std::map<std::string, double> dummy;
    tm.collect(dummy, c);
    return LSUM_OK;
}

static RefKey ref_key(const Plan& P) {
    RefKey k;
    auto put = [&](const void* v, size_t n) { k.append((const char*)v, n); };
    put(&P.kernel.kind, sizeof(int));
    put(&P.kernel.param, sizeof(double));
    put(&P.kernel.M, sizeof(int));
    put(&P.h_u, sizeof(double));
    put(&P.s, sizeof(double));
    put(&P.h, sizeof(double));
    put(&P.N_ref, sizeof(int));
    return k;
}

// A cached set of R x ldg row tables under `key` (need bytes), built by `build` on st the first
// time; uncached (owned by the caller alone) when the cache is disabled.
static int cached_rows(Context* c, const RefKey& key, const Plan& P, size_t need, hipStream_t st,
                       const std::function<int(RefEntry&)>& build_fn, std::shared_ptr<RefEntry>& out) {
    if (c->ref_cap == 0) {
        auto e = std::make_shared<RefEntry>();
        e->R = P.R;
        e->ldg = P.ldg;
        e->N_ref = P.N_ref;
        e->bytes = need;
        e->cached = false;
        int rc = e->G.get(c->pool, need);
        if (rc) return rc;
        rc = build_fn(*e);
        if (rc) return rc;
        e->built.set(1);
        e->users.fetch_add(1);
        out = e;
        return LSUM_OK;
    }
    std::shared_ptr<RefEntry> e;
    bool build = false;
    {
        std::lock_guard<std::mutex> lk(c->ref_mu);
        auto it = c->refs.find(key);
        if (it != c->refs.end()) {
            e = it->second;
        } else {
            while (c->ref_bytes + need > c->ref_cap) {   // evict unused entries beyond the cap
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
            c->refs[key] = e;
            c->ref_bytes += need;
            build = true;
        }
        e->users.fetch_add(1);
        e->last_use = ++c->ref_clock;
    }
    int rc;
    if (build) {
        rc = build_fn(*e);
        if (rc) {
            std::lock_guard<std::mutex> lk(c->ref_mu);   // a failed entry leaves the cache
            auto it = c->refs.find(key);
            if (it != c->refs.end() && it->second == e) {
                c->ref_bytes -= e->bytes;
                c->refs.erase(it);
            }
        }
        e->built.set(rc ? rc : 1);
    } else {
        const int s = e->built.wait();
        rc = s < 0 ? s : LSUM_OK;
    }
    if (rc) {
        e->users.fetch_sub(1);
        return rc;
    }
    out = e;
    return LSUM_OK;
}

int get_reference(Context* c, const Plan& P, hipStream_t st, std::shared_ptr<RefEntry>& out) {
    return cached_rows(c, ref_key(P), P, (size_t)P.R * P.ldg * 8, st,
                       [&](RefEntry& e) { return build_reference(c, P, st, e); }, out);
}

// The class rows (k_collocate at each class's sub-cell offset) and their window sums.
static int build_tables(Context* c, const Plan& P, const std::vector<std::tuple<int, int, int>>& wins,
                        hipStream_t st, RefEntry& e) {
    const int C = (int)P.cls_f.size();
    const size_t tab = (size_t)P.R * P.ldg;
    std::vector<double> tw(2 * (size_t)P.R);
    for (int q = 0; q < P.R; ++q) {
        tw[q] = P.t[q];
        tw[P.R + q] = std::cbrt(P.w[q]);
    }
    DevBuf twd;
    int rc = twd.get(c->pool, tw.size() * 8);
    if (rc) return rc;
    LSUM_HIP(hipMemcpyAsync(twd.p, tw.data(), tw.size() * 8, hipMemcpyHostToDevice, st));
    double* T = e.G.as<double>();
    StageTimer tm(st);
    tm.begin("collocate", (double)(C + wins.size()) * P.R * (2 * P.N_ref - 1) * 8, 0);
    for (int cl = 0; cl < C; ++cl)
        launch_collocate(st, P.R, twd.as<double>(), twd.as<double>() + P.R, P.N_ref, P.h, T + cl * tab, P.ldg,
                         P.cls_f[cl] * P.h);
    for (size_t w = 0; w < wins.size(); ++w)
        launch_window_sums(st, P.R, T + std::get<0>(wins[w]) * tab, P.ldg, std::get<1>(wins[w]),
                           std::get<2>(wins[w]), T + (C + w) * tab);
    tm.end();
    LSUM_HIP(hipGetLastError());
    LSUM_HIP(hipStreamSynchronize(st));   // complete for every stream; twd is released
    std::map<std::string, double> dummy;
    tm.collect(dummy, c);
    return LSUM_OK;
}

int get_tucker_ref(Context* c, const Plan& P, hipStream_t st, const std::function<int(RefEntry&)>& make,
                   std::shared_ptr<RefEntry>& out) {
    RefKey key = ref_key(P);
    key += "tucker";
    key.append((const char*)&P.eps, sizeof(double));
    key.append((const char*)&P.als_sweeps, sizeof(int));
    return cached_rows(c, key, P, 3 * (size_t)P.R * P.ldg * 8, st, make, out);
}

int get_tables(Context* c, const Plan& P, const std::vector<std::tuple<int, int, int>>& wins, hipStream_t st,
               std::shared_ptr<RefEntry>& out) {
    RefKey key = ref_key(P);
    auto put = [&](const void* v, size_t n) { key.append((const char*)v, n); };
    const int C = (int)P.cls_f.size(), nw = (int)wins.size();
    put(&C, sizeof(int));
    put(P.cls_f.data(), P.cls_f.size() * sizeof(double));
    put(&nw, sizeof(int));
    for (const auto& w : wins) {
        const int v[3] = {std::get<0>(w), std::get<1>(w), std::get<2>(w)};
        put(v, sizeof(v));
    }
    const size_t need = (size_t)(C + nw) * P.R * P.ldg * 8;
    return cached_rows(c, key, P, need, st, [&](RefEntry& e) { return build_tables(c, P, wins, st, e); }, out);
}

int get_windows(Context* c, RefEntry& e, int stride, int n, hipStream_t st, const double** out) {
    WindowRows* wr = nullptr;
    bool build = false;
    {
        std::lock_guard<std::mutex> lk(e.win_mu);
        auto it = e.windows.find({stride, n});
        if (it == e.windows.end()) {
            auto nw = std::make_unique<WindowRows>();
            int rc = nw->Q.get(c->pool, (size_t)e.R * e.ldg * 8);
            if (rc) return rc;
            wr = nw.get();
            e.windows.emplace(std::make_pair(stride, n), std::move(nw));
            build = true;
        } else {
            wr = it->second.get();
        }
    }
    if (build) {
        StageTimer tm(st);
        // additions: n per entry, or half a chain of ldg / stride for the prefix and suffix sums
        tm.begin("windows", 2.0 * e.R * e.ldg * 8, (double)e.R * e.ldg * (n > 0 ? n : 0.5 * e.ldg / stride));
        launch_window_sums(st, e.R, e.G.as<double>(), e.ldg, stride, n, wr->Q.as<double>());
        tm.end();
        hipError_t err = hipGetLastError();
        if (err == hipSuccess) err = hipStreamSynchronize(st);
        if (err != hipSuccess) {
            wr->built.set(LSUM_E_DEVICE);
            return fail(LSUM_E_DEVICE, std::string("window sums: ") + hipGetErrorString(err));
        }
        std::map<std::string, double> dummy;
        tm.collect(dummy, c);
        wr->built.set(1);
    } else {
        const int s = wr->built.wait();
        if (s < 0) return fail(s, "window sums failed to build");
    }
    *out = wr->Q.as<const double>();
    return LSUM_OK;
}

void drop_reference(Request* q) {
    if (q->ref) {
        q->ref->users.fetch_sub(1);
        q->ref.reset();
    }
    if (q->tabs) {
        q->tabs->users.fetch_sub(1);
        q->tabs.reset();
    }
}

size_t retained_bytes(const Request* q) {
    size_t b = 0;
    for (const auto& u : q->U) b += u.n;
    for (const auto& u : q->UT) b += u.n;
    for (int l = 0; l < 3; ++l) b += q->Z[l].n;
    return b + q->core.n + q->tile.n + q->def_offs.n + q->def_scale.n +
           (q->tabs && !q->tabs->cached ? q->tabs->bytes : 0);
}

// ------------------------------------------------------------------------------------------
// workers
// ------------------------------------------------------------------------------------------
static bool fits(const Context* c, const Request* q) {
    return c->used == 0 || q->reserved <= c->budget - std::min(c->used, c->budget);
}

void worker(Context* c, int slot) {
    (void)hipSetDevice(c->device);
    hipStream_t st = c->streams[slot];
    FailStream fs(st);   // an error inside a batch waits for the slot's queued kernels
    for (;;) {
        std::vector<Request*> batch;
        {
            std::unique_lock<std::mutex> lk(c->mu);
            c->cv.wait(lk, [&] { return c->stopping || (!c->queue.empty() && fits(c, c->queue.front())); });
            if (c->stopping) {
                if (c->queue.empty()) return;
                Request* q = c->queue.front();
                c->queue.pop_front();
                lk.unlock();
                finish(q, LSUM_E_CANCELLED);
                continue;
            }
            // the head, then following canonical requests while they fit (continuous batching)
            Request* h = c->queue.front();
            c->queue.pop_front();
            c->used += h->reserved;
            h->started = true;
            batch.push_back(h);
            while (!h->plan().tucker() && (int)batch.size() < c->max_batch && !c->queue.empty()) {
                Request* n = c->queue.front();
                if (n->plan().tucker() || !fits(c, n)) break;
                c->queue.pop_front();
                c->used += n->reserved;
                n->started = true;
                batch.push_back(n);
            }
        }
        c->cv.notify_all();
        const auto t0 = Clock::now();
        for (auto* q : batch) {
            q->t_start = t0;
            q->batch_size = (int)batch.size();
        }
        int rc;
        try {
            rc = run_batch(batch, st, c->aux.size() >= 3 * (size_t)(slot + 1) ? &c->aux[3 * slot] : nullptr);
        } catch (const std::exception& ex) {
            rc = fail(LSUM_E_DEVICE, std::string("exception: ") + ex.what());
        }
        if (rc != LSUM_OK) {
            (void)hipStreamSynchronize(st);
            (void)hipGetLastError();
        }
        for (auto* q : batch) {
            // a batch fails as a whole only on a device error; per-request errors are recorded
            int qrc = q->status.load() < 0 ? q->status.load() : rc;
            const size_t keep = qrc == LSUM_OK ? retained_bytes(q) : 0;
            if (qrc != LSUM_OK) {
                std::lock_guard<std::mutex> lk(q->mu);
                if (q->error.empty()) q->error = last_error();
            }
            {
                std::lock_guard<std::mutex> lk(c->mu);
                c->used -= q->reserved;
                c->used += keep;
                q->retained = keep;
            }
            finish(q, qrc);
        }
        c->cv.notify_all();
    }
}

}  // namespace lsum

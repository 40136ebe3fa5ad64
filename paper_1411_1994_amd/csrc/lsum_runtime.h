// Runtime structures of the lattice-sum library: the device buffer pool, the reference-vector
// cache, the stage profile, contexts and requests.  Internal (see include/lsum.h for the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <functional>
#include <map>
#include <unordered_map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "lsum_internal.h"

namespace lsum {

using Clock = std::chrono::steady_clock;

inline double ms_since(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

// ------------------------------------------------------------------------------------------
// device buffer pool: size-bucketed free lists; buffers come back only after the owning stream
// has been synchronised, so reuse on another stream is safe
// ------------------------------------------------------------------------------------------
class DevPool {
  public:
    DevPool() = default;
    ~DevPool();
    static size_t round(size_t n);
    int alloc(size_t n, void** p, size_t* got);
    void release(void* p, size_t n);
    void trim();

  private:
    void trim_locked();
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
            pool = o.pool;
            p = o.p;
            n = o.n;
            o.p = nullptr;
            o.n = 0;
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

// Build state of a cached device table: the first user builds it on its stream and
// synchronises; later users wait on the host until it is ready (or failed).
struct BuildState {
    std::mutex mu;
    std::condition_variable cv;
    int state = 0;                   // 0 building, 1 ready, < 0 the build's error code
    void set(int s) {
        std::lock_guard<std::mutex> lk(mu);
        state = s;
        cv.notify_all();
    }
    int wait() {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return state != 0; });
        return state;
    }
};

// windowed strided sums of the reference rows for one (stride, comb length)
struct WindowRows {
    DevBuf Q;
    BuildState built;
};

// reference vectors of one (kernel, quadrature, grid): "precomputed once, stored for multiple
// use" (Sec. 2.1)
struct RefEntry {
    DevBuf G;
    int R = 0, ldg = 0, N_ref = 0;
    BuildState built;
    std::atomic<int> users{0};
    size_t bytes = 0;
    uint64_t last_use = 0;
    bool cached = true;
    std::mutex win_mu;
    std::map<std::pair<int, int>, std::unique_ptr<WindowRows>> windows;   // by (stride, n)
    // a reference Tucker form: G holds the three modes' vectors as zero-padded rows (mode l at
    // element l * R * ldg, r[l] rows of ldg), `core` its r1 r2 r3 core (host FP64)
    int r[3]{};
    std::vector<double> core;
    double norm_A = 0, norm_xi = 0, bound = 0;
};
// bytes of (kind, param, M, h_u, s, h, N_ref), followed for class tables by their layout
using RefKey = std::string;

// event-timed GPU duration and algorithmic bytes/flops of each stage, summed over launches
struct StageStat {
    double ms = 0, bytes = 0, flops = 0;
    long launches = 0;
};

struct Request;

struct Context {
    int device = 0;
    size_t budget = 0;
    size_t used = 0;                 // bytes reserved by admitted requests and retained results
    int n_slots = 0;
    int max_batch = 32;              // canonical requests fused into one batch
    int range_min = 64;              // min(D, N) from which side matrices use the range basis
    bool jacobi_rank_stop = true;    // Jacobi SVDs of side matrices end once the certified rank is settled
    std::atomic<int> jacobi_max_sweeps{40};   // sweeps before a side-matrix SVD fails (LSUM_E_NOCONV)
    std::atomic<int> graphs{0};               // round-by-round Jacobi sweeps captured in HIP graphs
    std::atomic<int> jacobi_block{0};         // Jacobi columns per block (0: by size; 8, 16, 32)
    std::atomic<int> jacobi_skip{1};          // 16-column pair solves skip rotations below tol / 10
    std::atomic<int> persistent{0};           // Jacobi sweeps as one persistent launch each
    std::atomic<long long> jacobi_wait_us{20000};    // bound on a persistent sweep's waits
    std::atomic<int> persistent_wgs{0};       // workgroups of persistent sweeps now on the device
    Tuner tuner;                              // launch variants per shape bucket
    std::vector<hipStream_t> streams;
    std::vector<hipStream_t> aux;    // three per slot: the per-mode SVDs of a request run concurrently
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
    // plans of recently submitted problems, keyed by the problem's contents (a server sees the
    // same lattice many times); a plan depends on nothing else
    std::mutex plan_mu;
    std::unordered_map<std::string, std::shared_ptr<const Plan>> plans;
    // stage profile
    std::mutex prof_mu;
    std::map<std::string, StageStat> profile;
    ~Context();
};

// how the context runs Jacobi sweeps
inline JacobiRun jacobi_run(Context* c) {
    JacobiRun r;
    r.graphs = c->graphs.load();
    r.block = c->jacobi_block.load();
    r.skip_rel = c->jacobi_skip.load() ? 0.1 : 0.0;
    r.persistent = c->persistent.load();
    r.wait_us = (double)c->jacobi_wait_us.load();
    r.wg_in_use = &c->persistent_wgs;
    r.tuner = &c->tuner;
    return r;
}

// a request and its results
struct Request {
    std::shared_ptr<Context> ctx_ref;  // keeps the pool and streams alive until release
    Context* ctx = nullptr;
    // the plan, shared with the context's plan cache (immutable once made)
    std::shared_ptr<const Plan> plan_sp;
    const Plan& plan() const { return *plan_sp; }
    std::atomic<int> status{1};
    std::mutex mu;
    std::condition_variable cv;
    bool done = false;
    bool started = false;
    size_t reserved = 0, retained = 0;
    Clock::time_point t_submit, t_start, t_end;
    int batch_size = 1;
    std::shared_ptr<RefEntry> ref;
    // completion sampling (caller-owned memory)
    int n_points = 0;
    const double* points = nullptr;
    double* values = nullptr;
    int points_on_device = 0;
    // canonical factors: per block, 3 axes of R x N[l] (vector-major) and N[l] x R (point-major)
    std::vector<DevBuf> U, UT;
    size_t U_axis_off[3]{};           // element offsets of the axes in U (R x N_l each)
    size_t UT_axis_off[3]{};          // element offsets of the axes in UT (N_l x ldt each)
    int axis_src[3]{0, 1, 2};         // axis whose factors this axis shares (itself if distinct)
    DevBuf def_offs, def_scale;        // defects for sampling: window offsets (n_def x 3), dZ
    // exact sites off their cell centres: the request's row tables (the class rows, then the
    // window sums of its combs), R x ldg each with stride R * ldg, then t and w^(1/3)
    std::shared_ptr<RefEntry> tabs;
    const double* rows() const { return plan().off_grid() ? tabs->G.as<double>() : ref->G.as<double>(); }
    // Tucker
    int r[3]{};
    std::vector<double> sigma[3];
    int sweeps[3]{};
    double tails[3]{};
    double norm_A = 0, norm_xi = 0, bound = 0;
    double range_res[3]{};             // residual outside the range basis per mode (0: direct)
    int range_k[3]{};                  // size of the range basis per mode (0: direct)
    int core_mode = -1;                // mode whose shared columns grouped the core's terms (-1: none)
    std::vector<double> als_core_norm;  // ||core|| after each ALS sweep
    int als_skipped = 0;               // 1: ALS asked for but the ranks do not allow it
    double probe_err = -1.0;           // Tucker result vs the FP64 canonical sum at probe cells
    int n_probe = 0;
    std::vector<int32_t> probe_cells;  // 3 * n_probe cell indices
    int jacobi_persistent[3]{};        // per mode: sweeps launched persistently
    int jacobi_aborted[3]{};           // per mode: persistent sweeps that aborted
    int jacobi_tuned[3]{};             // per mode: 1 if the SVD timed the ways of launching a sweep
    std::string error;                 // message of a failed request (the worker's last error)
    DevBuf Z[3];                       // r_l x N_l FP64
    DevBuf core;                       // r1 r2 r3, FP64 or FP32 (precision)
    DevBuf tile;
    // stage times of the request's batch (shared by its requests) and result sizes by name
    std::shared_ptr<const std::map<std::string, double>> t_ms;
    double canonical_bytes = 0;
    std::map<std::string, double> bytes;
};

// stage timer on a stream; collects into requests and the context profile
class StageTimer {
  public:
    explicit StageTimer(hipStream_t s) : st_(s) {}
    ~StageTimer();
    void begin(const std::string& name, double bytes = 0, double flops = 0);
    // the algorithmic work of the open stage, when it is known only once its kernels are queued
    void work(double bytes, double flops) {
        if (!ev_.empty()) {
            ev_.back().bytes = bytes;
            ev_.back().flops = flops;
        }
    }
    void end();
    // a stage of kernels timed by their own dispatches: pass `start` to the first kernel's
    // launch and `stop` to the last one's (instead of begin/end)
    KTime kernels(const std::string& name, double bytes = 0, double flops = 0);
    // elapsed times (call after the stream has been synchronised)
    void collect(std::map<std::string, double>& out, Context* c);

  private:
    struct Ev {
        std::string name;
        hipEvent_t a, b;
        double bytes, flops;
        bool closed;   // the stop event was recorded (or handed to the stage's last launch)
    };
    hipStream_t st_;
    std::vector<Ev> ev_;
};

void finish(Request* q, int status);
int get_reference(Context* c, const Plan& P, hipStream_t st, std::shared_ptr<RefEntry>& out);
// Row tables of an off-grid plan, cached like the reference rows: the rows of every sub-cell
// class (R x ldg each, stride R * ldg, in class order), then the window sums (class, stride, n)
// of `wins` in order, each R x ldg.
int get_tables(Context* c, const Plan& P, const std::vector<std::tuple<int, int, int>>& wins, hipStream_t st,
               std::shared_ptr<RefEntry>& out);
// The rank-r Tucker form of a plan's reference (RHOSVD at the plan's eps of one unit charge on
// the doubled box), cached like the reference rows; `make` computes it on a miss.
int get_tucker_ref(Context* c, const Plan& P, hipStream_t st, const std::function<int(RefEntry&)>& make,
                   std::shared_ptr<RefEntry>& out);
// windowed strided sums of a reference (stride, comb length n), computed on st on first use;
// complete on return
int get_windows(Context* c, RefEntry& e, int stride, int n, hipStream_t st, const double** out);
void drop_reference(Request* q);
size_t retained_bytes(const Request* q);
void worker(Context* c, int slot);

// pipeline stages (lsum_pipeline.cpp)
// aux: three streams for the concurrent per-mode SVDs (nullptr: everything on st)
int run_batch(std::vector<Request*>& reqs, hipStream_t st, const hipStream_t* aux = nullptr);
// A GEMM that splits a long FP64 reduction over many workgroups when the output has few tiles
// (synchronous in that case); otherwise one asynchronous launch.
int gemm_auto(Context* c, hipStream_t st, GemmPrec prec, const GemmArgs& a);
// one canonical request's points for a batched sampling launch (device pointers)
struct CanonSample {
    Request* q;
    int n;
    const double* xyz;
    double* out;
};
int sample_canonical(Context* c, hipStream_t st, const std::vector<CanonSample>& items, const KTime* kt);
// kt (canonical requests only): kernel-bound timing of the sampling kernels; flops (Tucker
// requests, added to): the algorithmic flops of the contraction with the points' factor rows,
// run in the request's precision with FP64 final sums
int sample_points(Request* q, hipStream_t st, int n, const double* xyz_dev, double* out_dev,
                  const KTime* kt = nullptr, double* flops = nullptr);

}  // namespace lsum

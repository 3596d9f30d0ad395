// Batched stepping (lbm_group_*) and the continuous-batching server
// (lbm_server_*, lbm_batch_*) of the HMCSC library.
//
// Both drive the batched step kernel through a BatchRunner: two device copies
// of the domain table (double-buffered so the host can encode tick k+1 while
// tick k still reads its table), pinned staging, and two captured HIP graphs
// of K launches (one per table copy).  A launch k advances every domain whose
// step count for the tick exceeds k, so domains with different remaining
// budgets share one graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lbm_internal.h"

namespace {

#define HIP_TRY(expr)                                  \
    do {                                               \
        if ((expr) != hipSuccess) return LBM_EDEVICE;  \
    } while (0)

class BatchRunner {
  public:
    ~BatchRunner() { release(); }

    int init(int storage, int ncomp, int c_ns, int tile_x, int tile_y, int max_domains, int k_graph,
             hipStream_t st)
    {
        storage_ = storage;
        ncomp_ = ncomp;
        c_ns_ = c_ns;
        tx_ = tile_x;
        ty_ = tile_y;
        kmax_ = std::max(1, k_graph);
        stream_ = st;
        bytes_ = hm::batch_table_bytes(storage, max_domains);
        if (!hm::batch_tile_supported(storage, ncomp, tx_, ty_)) return LBM_EINVAL;
        int dev = 0, cus = 0;
        HIP_TRY(hipGetDevice(&dev));
        HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        // every block resident from the start: blocks stride over the tiles in
        // table order, so a block that had to wait for a CU would start its
        // whole share late
        grid_ = std::max(8, cus * hm::batch_blocks_per_cu(storage, ncomp, c_ns, tile_x, tile_y));
        cus_ = std::max(cus, 1);
        tpc_ = std::max(0, hm_rt::env_int("LBM_BATCH_TILES_PER_CU", 0));  // 0: planned per launch
        maxc_ = std::max(4, hm_rt::env_int("LBM_BATCH_MAX_CHUNK", 64));
        for (int j = 0; j < 2; ++j) {
            if (hipMalloc(&dev_[j], bytes_) != hipSuccess) return LBM_ENOMEM;
            if (hipHostMalloc(reinterpret_cast<void**>(&host_[j]), bytes_, hipHostMallocDefault) != hipSuccess)
                return LBM_ENOMEM;
            std::memset(host_[j], 0, bytes_);
            HIP_TRY(hipMemcpy(dev_[j], host_[j], bytes_, hipMemcpyHostToDevice));
            HIP_TRY(hipEventCreateWithFlags(&copied_[j], hipEventDisableTiming));
            HIP_TRY(hipEventRecord(copied_[j], stream_));
        }
        HIP_TRY(hipEventCreate(&t0_));
        HIP_TRY(hipEventCreate(&t1_));
        // graphs of kmax launches, one per table copy
        graphs_ok_ = true;
        for (int j = 0; j < 2 && graphs_ok_; ++j) {
            hipGraph_t g = nullptr;
            if (hipStreamBeginCapture(stream_, hipStreamCaptureModeRelaxed) != hipSuccess) {
                graphs_ok_ = false;
                break;
            }
            bool ok = true;
            for (int k = 0; k < kmax_; ++k)
                ok = ok && hm::launch_step_batch(storage_, ncomp_, c_ns_, tx_, ty_, dev_[j], k, grid_, stream_) ==
                               hipSuccess;
            if (hipStreamEndCapture(stream_, &g) != hipSuccess || !ok || !g) {
                graphs_ok_ = false;
                if (g) (void)hipGraphDestroy(g);
                (void)hipGetLastError();
                break;
            }
            if (hipGraphInstantiate(&exec_[j], g, nullptr, nullptr, 0) != hipSuccess) graphs_ok_ = false;
            (void)hipGraphDestroy(g);
        }
        (void)hipGetLastError();
        return LBM_OK;
    }

    // k launches over the n domains (k <= kmax uses the graph when k == kmax).
    int run(const hm::BatchDomain* d, int n, int k)
    {
        const int j = slot_;
        slot_ ^= 1;
        HIP_TRY(hipEventSynchronize(copied_[j]));  // host copy j is free again
        // z-chunks from the batch as a whole, none longer than maxc_ planes,
        // none shorter than 16 (each chunk re-reads two halo planes) unless
        // the batch would then give fewer than two tiles per CU (a few small
        // domains alone would leave most of the GPU idle, and the halo
        // re-reads cost little there)
        balanced_.assign(d, d + n);
        int64_t cols = 0, tiles16 = 0;
        for (const hm::BatchDomain& b : balanced_) {
            const int64_t c = static_cast<int64_t>((b.prob.nx + tx_ - 1) / tx_) * ((b.prob.ny + ty_ - 1) / ty_);
            cols += c;
            tiles16 += c * ((b.prob.nz + 15) / 16);
        }
        const int64_t min_chunk = tiles16 >= 2 * static_cast<int64_t>(cus_) ? 16 : 4;
        auto chunk_of = [&](const hm::BatchDomain& b, int64_t per_cols) {
            const int64_t chunks = std::max<int64_t>(per_cols, (b.prob.nz + maxc_ - 1) / maxc_);
            return static_cast<int>(
                std::min<int64_t>(b.prob.nz, std::max<int64_t>(min_chunk, (b.prob.nz + chunks - 1) / chunks)));
        };
        int64_t per_cols = 1;
        if (tpc_ > 0) {
            // fixed aim of tpc_ tiles per CU (LBM_BATCH_TILES_PER_CU)
            per_cols = std::max<int64_t>(1, (tpc_ * static_cast<int64_t>(cus_) + cols - 1) / std::max<int64_t>(cols, 1));
        } else {
            per_cols = plan_chunks(chunk_of, min_chunk);
        }
        for (hm::BatchDomain& b : balanced_) b.zchunk = chunk_of(b, per_cols);
        // longest tiles first: blocks take tiles in table order, so the
        // short ones fill in at the end (longest-processing-time order)
        std::stable_sort(balanced_.begin(), balanced_.end(), [](const hm::BatchDomain& a, const hm::BatchDomain& b) {
            return a.zchunk > b.zchunk;
        });
        hm::batch_encode(storage_, balanced_.data(), n, tx_, ty_, host_[j]);
        HIP_TRY(hipMemcpyAsync(dev_[j], host_[j], bytes_, hipMemcpyHostToDevice, stream_));
        HIP_TRY(hipEventRecord(copied_[j], stream_));
        HIP_TRY(hipEventRecord(t0_, stream_));
        if (k == kmax_ && graphs_ok_) {
            HIP_TRY(hipGraphLaunch(exec_[j], stream_));
        } else {
            for (int kk = 0; kk < k; ++kk)
                HIP_TRY(hm::launch_step_batch(storage_, ncomp_, c_ns_, tx_, ty_, dev_[j], kk, grid_, stream_));
        }
        HIP_TRY(hipEventRecord(t1_, stream_));
        last_k_ = k;
        return LBM_OK;
    }

    double last_launch_ms()
    {
        if (last_k_ <= 0 || hipEventSynchronize(t1_) != hipSuccess) return 0.0;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, t0_, t1_) != hipSuccess) return 0.0;
        return ms / last_k_;
    }

    int kmax() const { return kmax_; }
    int tile_x() const { return tx_; }
    int tile_y() const { return ty_; }

    void release()
    {
        if (stream_) (void)hipStreamSynchronize(stream_);
        for (int j = 0; j < 2; ++j) {
            if (exec_[j]) (void)hipGraphExecDestroy(exec_[j]);
            if (dev_[j]) (void)hipFree(dev_[j]);
            if (host_[j]) (void)hipHostFree(host_[j]);
            if (copied_[j]) (void)hipEventDestroy(copied_[j]);
            exec_[j] = nullptr;
            dev_[j] = nullptr;
            host_[j] = nullptr;
            copied_[j] = nullptr;
        }
        if (t0_) (void)hipEventDestroy(t0_);
        if (t1_) (void)hipEventDestroy(t1_);
        t0_ = t1_ = nullptr;
    }

  private:
    // Chunks per tile column shared by the domains of balanced_ (each capped
    // by chunk_of).  Blocks take tiles w, w + G, w + 2G, ... of the table
    // (G = grid_, tiles ordered longest first, each domain's tiles chunk by
    // chunk), so a launch lasts about as long as the most loaded of the G
    // block classes.  Each candidate is priced by that load in planes, a
    // tile adding kTileCost planes for its two halo planes and its pipeline
    // fill; the cheapest wins, ties going to fewer tiles.  The choice
    // depends only on the domains' shapes and is kept until they change.
    template <typename ChunkOf>
    int64_t plan_chunks(ChunkOf chunk_of, int64_t min_chunk)
    {
        constexpr int64_t kTileCost = 3;
        shapes_now_.clear();
        for (const hm::BatchDomain& b : balanced_) {
            shapes_now_.push_back(b.prob.nx);
            shapes_now_.push_back(b.prob.ny);
            shapes_now_.push_back(b.prob.nz);
        }
        shapes_now_.push_back(static_cast<int>(min_chunk));
        if (shapes_now_ == shapes_planned_) return planned_;
        int64_t cmax = 1;
        for (const hm::BatchDomain& b : balanced_)
            cmax = std::max<int64_t>(cmax, (b.prob.nz + min_chunk - 1) / min_chunk);
        cmax = std::min<int64_t>(cmax, 256);
        std::vector<int64_t> load(static_cast<size_t>(std::max(grid_, 1)));
        std::vector<std::pair<int, int64_t>> order;  // (zchunk, domain index)
        int64_t best = 1, best_cost = -1, best_tiles = 0;
        std::vector<int> zcs, prev_zcs;
        for (int64_t c = 1; c <= cmax; ++c) {
            order.clear();
            zcs.clear();
            for (size_t i = 0; i < balanced_.size(); ++i) {
                const int zc = chunk_of(balanced_[i], c);
                order.emplace_back(zc, static_cast<int64_t>(i));
                zcs.push_back(zc);
            }
            if (zcs == prev_zcs) continue;  // same chunking as the previous candidate
            prev_zcs = zcs;
            std::stable_sort(order.begin(), order.end(),
                             [](const std::pair<int, int64_t>& a, const std::pair<int, int64_t>& b) {
                                 return a.first > b.first;
                             });
            std::fill(load.begin(), load.end(), 0);
            int64_t w = 0;
            for (const auto& o : order) {
                const hm::BatchDomain& b = balanced_[static_cast<size_t>(o.second)];
                const int64_t tcols = static_cast<int64_t>((b.prob.nx + tx_ - 1) / tx_) * ((b.prob.ny + ty_ - 1) / ty_);
                for (int64_t z0 = 0; z0 < b.prob.nz; z0 += o.first) {
                    const int64_t len = std::min<int64_t>(o.first, b.prob.nz - z0) + kTileCost;
                    for (int64_t t = 0; t < tcols; ++t, ++w) load[static_cast<size_t>(w % grid_)] += len;
                }
            }
            const int64_t cost = *std::max_element(load.begin(), load.end());
            if (best_cost < 0 || cost < best_cost || (cost == best_cost && w < best_tiles)) {
                best = c;
                best_cost = cost;
                best_tiles = w;
            }
        }
        shapes_planned_ = shapes_now_;
        planned_ = best;
        return best;
    }

    int storage_ = 0, ncomp_ = 0, c_ns_ = 0, tx_ = 64, ty_ = 8, kmax_ = 1, grid_ = 512, cus_ = 256;
    int tpc_ = 0, maxc_ = 64;  // tiles per CU aimed at (0: planned), longest z-chunk
    std::vector<int> shapes_now_, shapes_planned_;
    int64_t planned_ = 1;
    std::vector<hm::BatchDomain> balanced_;
    size_t bytes_ = 0;
    hipStream_t stream_ = nullptr;
    void* dev_[2] = {nullptr, nullptr};
    char* host_[2] = {nullptr, nullptr};
    hipEvent_t copied_[2] = {nullptr, nullptr};
    hipGraphExec_t exec_[2] = {nullptr, nullptr};
    bool graphs_ok_ = false;
    int slot_ = 0;
    hipEvent_t t0_ = nullptr, t1_ = nullptr;
    int last_k_ = 0;
};

hm::BatchDomain domain_of(const lbm_ctx* c, int steps)
{
    hm::BatchDomain d{};
    d.prob = c->prob;
    d.zchunk = c->prob.nz;  // set per launch by BatchRunner::run
    d.buf[0] = c->buf[0];
    d.buf[1] = c->buf[1];
    d.ns = c->ns;
    d.parity = c->cur;
    d.t = c->t;
    d.steps = steps;
    return d;
}

void advance(lbm_ctx* c, int steps)
{
    if (steps & 1) c->cur = 1 - c->cur;
    c->t += steps;
}

double now_s(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

// ---------------------------------------------------------------------------
// Groups.

struct lbm_group {
    std::vector<lbm_ctx*> ctx;
    BatchRunner runner;
    std::vector<hm::BatchDomain> doms;
};

extern "C" {

int lbm_group_create(lbm_ctx* const* ctxs, int32_t n, lbm_group** out)
{
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    if (!ctxs || n < 1) return LBM_EINVAL;
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i]) return LBM_EINVAL;
        // one format per batched kernel, which runs the HMCSC only; one stream,
        // so the group's launches and each context's own calls stay ordered;
        // no health check (the group has no per-step totals)
        if (ctxs[i]->prm.storage != ctxs[0]->prm.storage || ctxs[i]->prm.ncomp != ctxs[0]->prm.ncomp ||
            ctxs[i]->prm.c_ns != ctxs[0]->prm.c_ns || ctxs[i]->device != ctxs[0]->device ||
            ctxs[i]->stream != ctxs[0]->stream || ctxs[i]->prm.forcing != LBM_FORCING_SHAN_CHEN ||
            ctxs[i]->prm.check_every != 0)
            return LBM_EINVAL;
    }
    lbm_group* g = new (std::nothrow) lbm_group();
    if (!g) return LBM_ENOMEM;
    g->ctx.assign(ctxs, ctxs + n);
    const lbm_params& p = ctxs[0]->prm;
    int tx = 64, ty = 8;
    hm::batch_default_tile(p.storage, p.ncomp, &tx, &ty);
    tx = hm_rt::env_int("LBM_BATCH_TILE_X", tx);
    ty = hm_rt::env_int("LBM_BATCH_TILE_Y", ty);
    const int rc = g->runner.init(p.storage, p.ncomp, p.c_ns, tx, ty, n, hm_rt::env_int("LBM_GRAPH_STEPS", 16),
                                  ctxs[0]->stream);
    if (rc) {
        delete g;
        return rc;
    }
    *out = g;
    return LBM_OK;
}

int lbm_group_step(lbm_group* g, int64_t nsteps)
{
    if (!g || nsteps < 0) return LBM_EINVAL;
    while (nsteps > 0) {
        const int k = static_cast<int>(std::min<int64_t>(nsteps, g->runner.kmax()));
        g->doms.clear();
        for (lbm_ctx* c : g->ctx) g->doms.push_back(domain_of(c, k));
        const int rc = g->runner.run(g->doms.data(), static_cast<int>(g->doms.size()), k);
        if (rc) return rc;
        for (lbm_ctx* c : g->ctx) advance(c, k);
        nsteps -= k;
    }
    return LBM_OK;
}

double lbm_group_last_step_ms(const lbm_group* g)
{
    return g ? const_cast<lbm_group*>(g)->runner.last_launch_ms() : 0.0;
}

void lbm_group_destroy(lbm_group* g) { delete g; }

}  // extern "C"

// ---------------------------------------------------------------------------
// Server.
//
// The worker thread runs ticks back to back on the main stream without
// waiting for them: it launches tick k, then waits for tick k-1 (already done
// or about to be), reads that tick's convergence data, and retires what has
// finished, while tick k runs.  A request's state lives in a block of a
// device memory pool (grown in chunks up to the budget, never returned to the
// device before the server ends).  Admission copies a request's arrays to
// pinned staging, uploads them and initialises the state on a second stream,
// overlapping the ticks; the request joins the ticks once that is done.
// Retirement reads the final state on a third stream.  All streams have the
// default priority.

namespace {

struct Request {
    uint64_t id = 0;
    lbm_domain dom{};
    std::vector<float> ns;
    std::vector<double> rho;
    lbm_params prm{};
    int64_t max_steps = 0;
    double tol = 0.0;
    int window = 1;
    int noise = 0;
    double* rho_out = nullptr;
    double t_submit = 0.0;
    uint64_t bytes = 0;
};

// Device memory of the resident requests: chunks from hipMalloc, at most the
// budget in total, allocated when first needed and kept; first-fit blocks,
// neighbours merged on release.
class DevicePool {
  public:
    void init(uint64_t budget, uint64_t chunk)
    {
        budget_ = budget;
        chunk_ = chunk;
    }
    void* alloc(uint64_t bytes)
    {
        bytes = hm_rt::align_up(bytes);
        for (Chunk& c : chunks_)
            for (auto it = c.free.begin(); it != c.free.end(); ++it)
                if (it->second >= bytes) {
                    const uint64_t off = it->first, sz = it->second;
                    c.free.erase(it);
                    if (sz > bytes) c.free[off + bytes] = sz - bytes;
                    return c.base + off;
                }
        if (reserved_ + bytes > budget_) return nullptr;
        const uint64_t size = std::max(bytes, std::min(chunk_, budget_ - reserved_));
        void* base = nullptr;
        if (hipMalloc(&base, size) != hipSuccess) {
            (void)hipGetLastError();
            budget_ = reserved_;  // the device is full: stop growing
            return nullptr;
        }
        reserved_ += size;
        Chunk c;
        c.base = static_cast<char*>(base);
        c.size = size;
        if (size > bytes) c.free[bytes] = size - bytes;
        chunks_.push_back(std::move(c));
        return base;
    }
    void release(void* p, uint64_t bytes)
    {
        bytes = hm_rt::align_up(bytes);
        char* q = static_cast<char*>(p);
        for (Chunk& c : chunks_) {
            if (q < c.base || q >= c.base + c.size) continue;
            uint64_t off = static_cast<uint64_t>(q - c.base), sz = bytes;
            auto next = c.free.lower_bound(off);
            if (next != c.free.end() && off + sz == next->first) {
                sz += next->second;
                next = c.free.erase(next);
            }
            if (next != c.free.begin()) {
                auto prev = std::prev(next);
                if (prev->first + prev->second == off) {
                    off = prev->first;
                    sz += prev->second;
                    c.free.erase(prev);
                }
            }
            c.free[off] = sz;
            return;
        }
    }
    void destroy()
    {
        for (Chunk& c : chunks_) (void)hipFree(c.base);
        chunks_.clear();
        reserved_ = 0;
    }
    uint64_t reserved() const { return reserved_; }

  private:
    struct Chunk {
        char* base = nullptr;
        uint64_t size = 0;
        std::map<uint64_t, uint64_t> free;  // offset -> bytes
    };
    std::vector<Chunk> chunks_;
    uint64_t budget_ = 0, chunk_ = 0, reserved_ = 0;
};

struct Slot {
    Request req;
    lbm_ctx* ctx = nullptr;
    void* mem = nullptr;      // f_a | f_b | n_s in one pool block
    uint64_t mem_bytes = 0;
    int64_t issued = 0;       // steps launched
    int64_t last_tick = -1;   // the last tick that stepped it
    bool stop = false;        // converged or failed: no further ticks
    bool converged = false;
    int status = LBM_OK;
    std::vector<std::array<double, 3>> hist;  // convergence monitor samples
    double t_admit = 0.0;
};

// What a tick launched: the slots it stepped and, for those it monitored,
// their position in the tick's monitor output.
struct TickRecord {
    int64_t index = -1;
    std::vector<Slot*> monitored;
    hipEvent_t done = nullptr;
};

void ctx_release(lbm_ctx* c)
{
    if (!c) return;
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    delete c;
}

}  // namespace

struct lbm_server {
    lbm_server_cfg cfg{};
    int device = 0;
    hipStream_t stream = nullptr;         // ticks and their monitors
    hipStream_t admit_stream = nullptr;   // uploads and initial states
    hipStream_t retire_stream = nullptr;  // final moments
    void* scratch = nullptr;              // FP64 fields and reductions of retirements
    uint64_t scratch_bytes = 0;
    uint64_t budget = 0;
    DevicePool pool;
    BatchRunner runner;
    std::chrono::steady_clock::time_point t0;

    // admission staging: pinned host arrays and the device densities
    char* stage_host = nullptr;
    double* stage_rho = nullptr;
    hipEvent_t admit_done = nullptr;
    std::unique_ptr<Slot> admitting;

    // convergence monitor: tables, partial sums and outputs per tick parity
    void* mon_dev[2] = {nullptr, nullptr};
    char* mon_host[2] = {nullptr, nullptr};
    double* mon_part = nullptr;
    double* mon_out_dev[2] = {nullptr, nullptr};
    double* mon_out_host[2] = {nullptr, nullptr};
    size_t mon_bytes = 0;
    TickRecord rec[2];

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> queue;
    std::unordered_map<uint64_t, lbm_result> done;
    std::unordered_map<uint64_t, int> live;  // submitted and not final
    uint64_t next_id = 1;
    bool stop = false;
    std::thread worker;

    // worker-owned
    std::vector<std::unique_ptr<Slot>> active;
    std::vector<hm::BatchDomain> doms;
    std::vector<hm::MonitorDomain> mdoms;
    uint64_t resident = 0;

    // statistics (guarded by mu)
    lbm_server_stats st{};
    double busy_since = -1.0;

    void run();
    bool start_admission();
    bool finish_admission(bool block);
    void process_tick(TickRecord& r, int parity);
    void retire(size_t i, int status, bool converged);
    void fail_request(Request& r, int status);
};

namespace {

uint64_t state_bytes(const lbm_domain& d, const lbm_params& p)
{
    lbm_sizes s{};
    if (lbm_required_bytes(&d, &p, &s)) return 0;
    return 2 * s.pop_bytes + s.ns_bytes;
}

// Convergence of one monitored request after a new sample J (the local
// mixture momentum of its state): with a window of 1, |J - J_prev| <= tol |J|
// over the last two samples; with a window W > 1, the means of the last two
// windows of W samples differ by at most tol times the newer mean, or (noise
// floor on) by at most twice the standard error of their difference estimated
// from the spread within the windows (the state no longer drifts beyond its
// own rounding noise).
bool converged_now(const Slot& s)
{
    const int W = std::max(1, s.req.window);
    const size_t n = s.hist.size();
    if (n < static_cast<size_t>(2 * W)) return false;
    double m1[3] = {0, 0, 0}, m0[3] = {0, 0, 0};
    for (int k = 0; k < W; ++k)
        for (int a = 0; a < 3; ++a) {
            m1[a] += s.hist[n - 1 - k][a] / W;
            m0[a] += s.hist[n - 1 - W - k][a] / W;
        }
    double d2 = 0, n2 = 0;
    for (int a = 0; a < 3; ++a) {
        d2 += (m1[a] - m0[a]) * (m1[a] - m0[a]);
        n2 += m1[a] * m1[a];
    }
    if (std::sqrt(d2) <= s.req.tol * std::sqrt(n2)) return true;
    if (!s.req.noise || W < 2) return false;
    double v1 = 0, v0 = 0;
    for (int k = 0; k < W; ++k)
        for (int a = 0; a < 3; ++a) {
            v1 += (s.hist[n - 1 - k][a] - m1[a]) * (s.hist[n - 1 - k][a] - m1[a]);
            v0 += (s.hist[n - 1 - W - k][a] - m0[a]) * (s.hist[n - 1 - W - k][a] - m0[a]);
        }
    const double se2 = (v1 + v0) / (W - 1) / W;
    return d2 <= 4.0 * se2;
}

}  // namespace

void lbm_server::fail_request(Request& r, int status)
{
    lbm_result res{};
    res.status = status;
    res.t_submit = r.t_submit;
    res.t_done = now_s(t0);
    std::lock_guard<std::mutex> lk(mu);
    done[r.id] = res;
    live.erase(r.id);
    st.completed += 1;
    cv_done.notify_all();
}

// Take the next queued request into the admission stage if a slot and pool
// memory are free: upload its arrays and initialise its state on the
// admission stream.  Returns true if an admission started.
bool lbm_server::start_admission()
{
    if (admitting) return false;
    Request r;
    {
        std::lock_guard<std::mutex> lk(mu);
        if (queue.empty() || static_cast<int>(active.size()) >= cfg.max_slots) return false;
        if (resident + queue.front().bytes > budget) return false;
        r = std::move(queue.front());
        queue.pop_front();
        st.queued = static_cast<int64_t>(queue.size());
    }
    lbm_sizes sz{};
    lbm_required_bytes(&r.dom, &r.prm, &sz);
    const uint64_t total = sz.pop_bytes * 2 + sz.ns_bytes;
    void* mem = pool.alloc(total);
    if (!mem) {  // fragmented or the device is full: wait for a retirement
        std::lock_guard<std::mutex> lk(mu);
        queue.push_front(std::move(r));
        st.queued = static_cast<int64_t>(queue.size());
        return false;
    }
    std::unique_ptr<Slot> sl(new Slot());
    sl->req = std::move(r);
    sl->mem = mem;
    sl->mem_bytes = total;
    char* m = static_cast<char*>(mem);
    lbm_device_buffers b{m, m + sz.pop_bytes, m + 2 * sz.pop_bytes, scratch};
    int rc = hm_rt::ctx_bind(&sl->req.dom, &sl->req.prm, &b, stream, &sl->ctx);
    const int64_t N = sl->ctx ? sl->ctx->prob.N : 0;
    const size_t ns_b = sizeof(float) * static_cast<size_t>(sl->req.prm.c_ns) * N;
    const size_t rho_b = sizeof(double) * static_cast<size_t>(sl->req.prm.ncomp) * N;
    if (rc == LBM_OK) {
        std::memcpy(stage_host, sl->req.rho.data(), rho_b);
        std::memcpy(stage_host + hm_rt::align_up(rho_b), sl->req.ns.data(), ns_b);
        if (hipMemcpyAsync(stage_rho, stage_host, rho_b, hipMemcpyHostToDevice, admit_stream) != hipSuccess ||
            hipMemcpyAsync(sl->ctx->ns, stage_host + hm_rt::align_up(rho_b), ns_b, hipMemcpyHostToDevice,
                           admit_stream) != hipSuccess ||
            hm::launch_init(sl->ctx->prob, stage_rho, sl->ctx->buf[0], admit_stream) != hipSuccess ||
            hipEventRecord(admit_done, admit_stream) != hipSuccess)
            rc = LBM_EDEVICE;
    }
    if (rc) {
        ctx_release(sl->ctx);
        pool.release(mem, total);
        fail_request(sl->req, rc);
        return false;
    }
    sl->req.ns.clear();
    sl->req.ns.shrink_to_fit();
    sl->req.rho.clear();
    sl->req.rho.shrink_to_fit();
    sl->t_admit = now_s(t0);
    resident += sl->req.bytes;
    admitting = std::move(sl);
    return true;
}

// Move the admitted request into the resident set once its state is ready
// (waiting for it if block).  Returns true if it joined.
bool lbm_server::finish_admission(bool block)
{
    if (!admitting) return false;
    const hipError_t e = block ? hipEventSynchronize(admit_done) : hipEventQuery(admit_done);
    if (e == hipErrorNotReady) return false;
    if (e != hipSuccess) {
        (void)hipGetLastError();
        Slot* s = admitting.get();
        resident -= s->req.bytes;
        ctx_release(s->ctx);
        pool.release(s->mem, s->mem_bytes);
        fail_request(s->req, LBM_EDEVICE);
        admitting.reset();
        return false;
    }
    active.push_back(std::move(admitting));
    return true;
}

// Read the convergence samples of a finished tick.
void lbm_server::process_tick(TickRecord& r, int parity)
{
    if (r.index < 0) return;
    if (hipEventSynchronize(r.done) != hipSuccess) {
        (void)hipGetLastError();
        for (Slot* s : r.monitored) {
            s->stop = true;
            s->status = LBM_EDEVICE;
        }
    } else {
        for (size_t k = 0; k < r.monitored.size(); ++k) {
            Slot* s = r.monitored[k];
            const double* o = mon_out_host[parity] + 4 * k;
            if (!(std::isfinite(o[0]) && std::isfinite(o[1]) && std::isfinite(o[2]) && std::isfinite(o[3]))) {
                s->stop = true;
                s->status = LBM_EUNSTABLE;
                continue;
            }
            s->hist.push_back({o[0], o[1], o[2]});
            if (s->hist.size() > static_cast<size_t>(4 * std::max(1, s->req.window)))
                s->hist.erase(s->hist.begin());
            if (converged_now(*s)) {
                s->stop = true;
                s->converged = true;
            }
        }
    }
    r.monitored.clear();
    r.index = -1;
}

void lbm_server::retire(size_t i, int status, bool converged)
{
    Slot& sl = *active[i];
    lbm_result res{};
    res.status = status;
    res.converged = converged ? 1 : 0;
    res.steps_done = sl.issued;
    res.t_submit = sl.req.t_submit;
    res.t_admit = sl.t_admit;
    if (status == LBM_OK) {
        // final FP64 moments, as lbm_moments computes them, on the retire stream
        lbm_ctx* c = sl.ctx;
        double* rho = reinterpret_cast<double*>(c->scratch + c->sl.rho);
        double* part = reinterpret_cast<double*>(c->scratch + c->sl.partials);
        double* tots = reinterpret_cast<double*>(c->scratch + c->sl.totals);
        double h[5];
        if (hm::launch_diagnostics(c->prob, c->buf[c->cur], c->ns, true, rho, nullptr, nullptr, part, tots,
                                   retire_stream) != hipSuccess ||
            hipMemcpyAsync(h, tots, sizeof(h), hipMemcpyDeviceToHost, retire_stream) != hipSuccess ||
            (sl.req.rho_out &&
             hipMemcpyAsync(sl.req.rho_out, rho, sizeof(double) * c->prm.ncomp * c->prob.N, hipMemcpyDeviceToHost,
                            retire_stream) != hipSuccess) ||
            hipStreamSynchronize(retire_stream) != hipSuccess) {
            (void)hipGetLastError();
            res.status = LBM_EDEVICE;
        } else {
            res.totals.mass[0] = h[0];
            res.totals.mass[1] = c->prm.ncomp == 2 ? h[1] : 0.0;
            for (int a = 0; a < 3; ++a) res.totals.momentum[a] = h[2 + a];
            res.totals.time = c->t;
            int fin = 1;
            for (double v : h) fin &= std::isfinite(v) ? 1 : 0;
            res.totals.finite = fin;
        }
    }
    res.t_done = now_s(t0);
    ctx_release(sl.ctx);
    pool.release(sl.mem, sl.mem_bytes);
    resident -= sl.req.bytes;
    const uint64_t id = sl.req.id;
    active.erase(active.begin() + static_cast<long>(i));
    {
        std::lock_guard<std::mutex> lk(mu);
        done[id] = res;
        live.erase(id);
        st.completed += 1;
        st.active = static_cast<int64_t>(active.size());
        st.bytes_resident = resident;
    }
    cv_done.notify_all();
}

void lbm_server::run()
{
    (void)hipSetDevice(device);
    int64_t tick = 0;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(mu);
            const bool idle = active.empty() && !admitting && queue.empty() && rec[0].index < 0 && rec[1].index < 0;
            if (idle && !stop) {
                if (busy_since >= 0) {
                    st.busy_seconds += now_s(t0) - busy_since;
                    busy_since = -1.0;
                }
                cv_work.wait_for(lk, std::chrono::milliseconds(20));
            }
            if (stop) break;
            if (busy_since < 0 && (!active.empty() || admitting || !queue.empty())) busy_since = now_s(t0);
        }
        // one tick over the resident requests that have steps left
        const int K = runner.kmax();
        const int par = static_cast<int>(tick & 1);
        std::vector<int> steps(active.size(), 0);
        for (size_t i = 0; i < active.size(); ++i) {
            const Slot& s = *active[i];
            if (!s.stop) steps[i] = static_cast<int>(std::min<int64_t>(K, s.req.max_steps - s.issued));
        }
        if (cfg.policy == LBM_SERVE_SHORTEST_FIRST) {
            std::vector<size_t> order;
            for (size_t i = 0; i < active.size(); ++i)
                if (steps[i] > 0) order.push_back(i);
            std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
                const Slot &sa = *active[a], &sb = *active[b];
                return static_cast<double>(sa.ctx->prob.N) * static_cast<double>(sa.req.max_steps - sa.issued) <
                       static_cast<double>(sb.ctx->prob.N) * static_cast<double>(sb.req.max_steps - sb.issued);
            });
            int64_t stepped = 0;
            for (size_t i : order) {
                if (stepped >= cfg.run_cells) steps[i] = 0;
                else stepped += active[i]->ctx->prob.N;
            }
        }
        doms.clear();
        mdoms.clear();
        std::vector<Slot*> monitored;
        double cells = 0.0;
        for (size_t i = 0; i < active.size(); ++i) {
            if (!steps[i]) continue;
            Slot& s = *active[i];
            doms.push_back(domain_of(s.ctx, steps[i]));
            cells += static_cast<double>(s.ctx->prob.N) * steps[i];
        }
        int rc = LBM_OK;
        if (!doms.empty()) {
            rc = runner.run(doms.data(), static_cast<int>(doms.size()), K);
            for (size_t i = 0; i < active.size(); ++i) {
                if (!steps[i]) continue;
                Slot& s = *active[i];
                advance(s.ctx, steps[i]);
                s.issued += steps[i];
                s.last_tick = tick;
                if (s.req.tol > 0.0) {
                    monitored.push_back(&s);
                    mdoms.push_back({s.ctx->prob, s.ctx->buf[s.ctx->cur], s.ctx->ns});
                }
            }
            if (rc == LBM_OK && !mdoms.empty()) {
                // the monitor table of the other parity's tick is no longer read
                const int blocks = hm::monitor_encode(cfg.storage, mdoms.data(), static_cast<int>(mdoms.size()),
                                                      mon_host[par]);
                if (hipMemcpyAsync(mon_dev[par], mon_host[par], mon_bytes, hipMemcpyHostToDevice, stream) !=
                        hipSuccess ||
                    hm::launch_monitor(cfg.storage, mon_dev[par], static_cast<int>(mdoms.size()), blocks, mon_part,
                                       mon_out_dev[par], stream) != hipSuccess ||
                    hipMemcpyAsync(mon_out_host[par], mon_out_dev[par], sizeof(double) * 4 * mdoms.size(),
                                   hipMemcpyDeviceToHost, stream) != hipSuccess)
                    rc = LBM_EDEVICE;
            }
            if (rc == LBM_OK && hipEventRecord(rec[par].done, stream) != hipSuccess) rc = LBM_EDEVICE;
            rec[par].index = tick;
            rec[par].monitored = std::move(monitored);
            {
                std::lock_guard<std::mutex> lk(mu);
                st.cell_updates += cells;
                st.ticks += 1;
                st.active = static_cast<int64_t>(active.size());
                st.bytes_resident = resident;
            }
            ++tick;
        }
        if (rc) {
            (void)hipStreamSynchronize(stream);
            for (auto& s : active) {
                s->stop = true;
                if (s->status == LBM_OK) s->status = rc;
            }
        }
        // admissions while the tick runs (uploads and initial states on the
        // admission stream): every queued request that has a slot and fits
        // joins the next tick
        for (int k = 0; k < cfg.max_slots && start_admission(); ++k) finish_admission(true);
        // the previous tick (or, with nothing launched now, the last one): its
        // convergence samples, then every request whose final state it holds
        const int prev = doms.empty() ? par ^ 1 : par ^ 1;
        int64_t completed = -1;
        if (rec[prev].index >= 0) {
            completed = rec[prev].index;
            process_tick(rec[prev], prev);
        }
        if (doms.empty() && rec[par].index >= 0) {
            completed = rec[par].index;
            process_tick(rec[par], par);
        }
        for (size_t i = active.size(); i-- > 0;) {
            Slot& s = *active[i];
            const bool finished = s.stop || s.issued >= s.req.max_steps;
            if (finished && s.last_tick <= completed) retire(i, s.status, s.converged);
        }
    }
    // shutting down: everything resident ends unfinished
    (void)hipStreamSynchronize(stream);
    (void)hipStreamSynchronize(admit_stream);
    if (admitting) active.push_back(std::move(admitting));
    for (size_t i = active.size(); i-- > 0;) retire(i, LBM_EAGAIN, false);
}

extern "C" {

int lbm_server_create(const lbm_server_cfg* cfg, void* reserved, lbm_server** out)
{
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    if (!cfg || reserved) return LBM_EINVAL;
    if (cfg->max_slots < 1 || cfg->steps_per_tick < 1 || cfg->max_cells < 1) return LBM_EINVAL;
    if (cfg->storage < LBM_F64 || cfg->storage > LBM_BF16S) return LBM_EINVAL;
    if (cfg->ncomp < 1 || cfg->ncomp > 2 || cfg->c_ns < 1 || cfg->c_ns > cfg->ncomp) return LBM_EINVAL;
    if (cfg->policy < LBM_SERVE_FAIR || cfg->policy > LBM_SERVE_SHORTEST_FIRST || cfg->pad != 0 ||
        cfg->run_cells < 0)
        return LBM_EINVAL;
    int tx = 64, ty = 8;
    hm::batch_default_tile(cfg->storage, cfg->ncomp, &tx, &ty);
    if (cfg->tile_x) tx = cfg->tile_x;
    if (cfg->tile_y) ty = cfg->tile_y;
    if (!hm::batch_tile_supported(cfg->storage, cfg->ncomp, tx, ty)) return LBM_EINVAL;
    lbm_server* s = new (std::nothrow) lbm_server();
    if (!s) return LBM_ENOMEM;
    s->cfg = *cfg;
    s->cfg.tile_x = tx;
    s->cfg.tile_y = ty;
    if (!s->cfg.run_cells) s->cfg.run_cells = int64_t(1) << 24;
    s->t0 = std::chrono::steady_clock::now();
    auto fail = [&](int rc) {
        lbm_server_destroy(s);
        return rc;
    };
    if (hipGetDevice(&s->device) != hipSuccess || hipStreamCreate(&s->stream) != hipSuccess ||
        hipStreamCreate(&s->admit_stream) != hipSuccess || hipStreamCreate(&s->retire_stream) != hipSuccess ||
        hipEventCreateWithFlags(&s->admit_done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&s->rec[0].done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&s->rec[1].done, hipEventDisableTiming) != hipSuccess)
        return fail(LBM_EDEVICE);
    s->scratch_bytes = hm_rt::scratch_layout(cfg->max_cells, cfg->ncomp).bytes;
    const size_t rho_b = hm_rt::align_up(sizeof(double) * cfg->ncomp * static_cast<size_t>(cfg->max_cells));
    const size_t ns_b = hm_rt::align_up(sizeof(float) * cfg->c_ns * static_cast<size_t>(cfg->max_cells));
    s->mon_bytes = hm::monitor_table_bytes(cfg->storage, cfg->max_slots);
    if (hipMalloc(&s->scratch, s->scratch_bytes) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&s->stage_rho), rho_b) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&s->stage_host), rho_b + ns_b, hipHostMallocDefault) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&s->mon_part),
                  sizeof(double) * 4 * hm::monitor_max_blocks(cfg->max_slots)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(LBM_ENOMEM);
    }
    for (int j = 0; j < 2; ++j)
        if (hipMalloc(&s->mon_dev[j], s->mon_bytes) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void**>(&s->mon_host[j]), s->mon_bytes, hipHostMallocDefault) !=
                hipSuccess ||
            hipMalloc(reinterpret_cast<void**>(&s->mon_out_dev[j]), sizeof(double) * 4 * cfg->max_slots) !=
                hipSuccess ||
            hipHostMalloc(reinterpret_cast<void**>(&s->mon_out_host[j]), sizeof(double) * 4 * cfg->max_slots,
                          hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return fail(LBM_ENOMEM);
        }
    size_t free_b = 0, total_b = 0;
    (void)hipMemGetInfo(&free_b, &total_b);
    s->budget = cfg->hbm_budget_bytes ? cfg->hbm_budget_bytes : static_cast<uint64_t>(0.9 * free_b);
    s->pool.init(s->budget, uint64_t(8) << 30);
    const int rc = s->runner.init(cfg->storage, cfg->ncomp, cfg->c_ns, tx, ty, cfg->max_slots, cfg->steps_per_tick,
                                  s->stream);
    if (rc) return fail(rc);
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return LBM_OK;
}

int lbm_batch_submit(lbm_server* s, const lbm_request* rq, uint64_t* ticket)
{
    if (!s || !rq || !ticket) return LBM_EINVAL;
    *ticket = 0;
    const lbm_params& p = rq->params;
    if (p.storage != s->cfg.storage || p.ncomp != s->cfg.ncomp || p.c_ns != s->cfg.c_ns) return LBM_EINVAL;
    if (rq->max_steps < 1 || !(rq->conv_tol >= 0.0) || !rq->n_s || !rq->rho_init) return LBM_EINVAL;
    if (rq->conv_window < 0 || rq->conv_window > 1024 || (rq->conv_noise != 0 && rq->conv_noise != 1))
        return LBM_EINVAL;
    if (p.check_every != 0) return LBM_EINVAL;
    if (p.forcing != LBM_FORCING_SHAN_CHEN) return LBM_EINVAL;  // the batched kernel runs the HMCSC only
    lbm_sizes sz{};
    const int vrc = lbm_required_bytes(&rq->dom, &p, &sz);
    if (vrc) return vrc;
    const int64_t N = static_cast<int64_t>(rq->dom.nx) * rq->dom.ny * rq->dom.nz;
    if (N > s->cfg.max_cells) return LBM_ENOMEM;
    Request r;
    r.dom = rq->dom;
    r.prm = p;
    r.max_steps = rq->max_steps;
    r.tol = rq->conv_tol;
    r.window = std::max(1, static_cast<int>(rq->conv_window));
    r.noise = rq->conv_noise;
    r.rho_out = rq->rho_out;
    r.bytes = state_bytes(rq->dom, p);
    if (r.bytes > s->budget) return LBM_ENOMEM;
    r.ns.assign(rq->n_s, rq->n_s + static_cast<size_t>(p.c_ns) * N);
    r.rho.assign(rq->rho_init, rq->rho_init + static_cast<size_t>(p.ncomp) * N);
    for (float v : r.ns)
        if (!(v >= 0.0f && v <= 1.0f)) return LBM_EINVAL;
    for (double v : r.rho)
        if (!std::isfinite(v)) return LBM_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return LBM_EINVAL;
        r.id = s->next_id++;
        r.t_submit = now_s(s->t0);
        *ticket = r.id;
        s->live[r.id] = 1;
        s->queue.push_back(std::move(r));
        s->st.submitted += 1;
        s->st.queued = static_cast<int64_t>(s->queue.size());
    }
    s->cv_work.notify_one();
    return LBM_OK;
}

int lbm_batch_poll(lbm_server* s, uint64_t ticket, lbm_result* out)
{
    if (!s || !out) return LBM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->done.find(ticket);
    if (it != s->done.end()) {
        *out = it->second;
        return LBM_OK;
    }
    return s->live.count(ticket) ? LBM_EAGAIN : LBM_ENOTFOUND;
}

int lbm_batch_wait(lbm_server* s, uint64_t ticket, double timeout_s, lbm_result* out)
{
    if (!s || !out) return LBM_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto ready = [&] { return s->done.count(ticket) || !s->live.count(ticket); };
    if (timeout_s < 0) {
        s->cv_done.wait(lk, ready);
    } else {
        s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready);
    }
    auto it = s->done.find(ticket);
    if (it != s->done.end()) {
        *out = it->second;
        return LBM_OK;
    }
    return s->live.count(ticket) ? LBM_EAGAIN : LBM_ENOTFOUND;
}

int lbm_server_stats_get(lbm_server* s, lbm_server_stats* out)
{
    if (!s || !out) return LBM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    out->uptime_seconds = now_s(s->t0);
    if (s->busy_since >= 0) out->busy_seconds += out->uptime_seconds - s->busy_since;
    return LBM_OK;
}

void lbm_server_destroy(lbm_server* s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (Request& r : s->queue) {
            lbm_result res{};
            res.status = LBM_EAGAIN;
            res.t_submit = r.t_submit;
            s->done[r.id] = res;
            s->live.erase(r.id);
        }
        s->queue.clear();
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    s->cv_done.notify_all();
    s->runner.release();
    for (hipStream_t q : {s->stream, s->admit_stream, s->retire_stream})
        if (q) (void)hipStreamSynchronize(q);
    s->pool.destroy();
    if (s->scratch) (void)hipFree(s->scratch);
    if (s->stage_rho) (void)hipFree(s->stage_rho);
    if (s->stage_host) (void)hipHostFree(s->stage_host);
    if (s->mon_part) (void)hipFree(s->mon_part);
    for (int j = 0; j < 2; ++j) {
        if (s->mon_dev[j]) (void)hipFree(s->mon_dev[j]);
        if (s->mon_host[j]) (void)hipHostFree(s->mon_host[j]);
        if (s->mon_out_dev[j]) (void)hipFree(s->mon_out_dev[j]);
        if (s->mon_out_host[j]) (void)hipHostFree(s->mon_out_host[j]);
        if (s->rec[j].done) (void)hipEventDestroy(s->rec[j].done);
    }
    if (s->admit_done) (void)hipEventDestroy(s->admit_done);
    for (hipStream_t q : {s->stream, s->admit_stream, s->retire_stream})
        if (q) (void)hipStreamDestroy(q);
    delete s;
}

}  // extern "C"

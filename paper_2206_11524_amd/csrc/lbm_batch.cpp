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
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
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
        tpc_ = std::max(1, hm_rt::env_int("LBM_BATCH_TILES_PER_CU", 2));
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
        // z-chunks from the batch as a whole: about tpc_ tiles per CU, none
        // longer than maxc_ planes (blocks stride over tiles of unequal
        // domains, shorter tiles balance them; longer tiles pay the pipeline
        // fill of a tile less often), none shorter than 16 (each chunk
        // re-reads two halo planes) unless the batch would then give fewer
        // than two tiles per CU: a few small domains alone would leave most
        // of the GPU idle, and the halo re-reads cost little there
        balanced_.assign(d, d + n);
        int64_t cols = 0, tiles16 = 0;
        for (const hm::BatchDomain& b : balanced_) {
            const int64_t c = static_cast<int64_t>((b.prob.nx + tx_ - 1) / tx_) * ((b.prob.ny + ty_ - 1) / ty_);
            cols += c;
            tiles16 += c * ((b.prob.nz + 15) / 16);
        }
        const int64_t min_chunk = tiles16 >= 2 * static_cast<int64_t>(cus_) ? 16 : 4;
        const int64_t per_cols =
            std::max<int64_t>(1, (tpc_ * static_cast<int64_t>(cus_) + cols - 1) / std::max<int64_t>(cols, 1));
        for (hm::BatchDomain& b : balanced_) {
            const int64_t chunks = std::max<int64_t>(per_cols, (b.prob.nz + maxc_ - 1) / maxc_);
            b.zchunk = static_cast<int>(
                std::min<int64_t>(b.prob.nz, std::max<int64_t>(min_chunk, (b.prob.nz + chunks - 1) / chunks)));
        }
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
    int storage_ = 0, ncomp_ = 0, c_ns_ = 0, tx_ = 64, ty_ = 8, kmax_ = 1, grid_ = 512, cus_ = 256;
    int tpc_ = 2, maxc_ = 64;  // tiles per CU aimed at, longest z-chunk
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

namespace {

struct Request {
    uint64_t id = 0;
    lbm_domain dom{};
    std::vector<float> ns;
    std::vector<double> rho;
    lbm_params prm{};
    int64_t max_steps = 0;
    double tol = 0.0;
    double* rho_out = nullptr;
    double t_submit = 0.0;
    uint64_t bytes = 0;
};

struct Slot {
    Request req;
    lbm_ctx* ctx = nullptr;
    void* mem[3] = {nullptr, nullptr, nullptr};  // f_a, f_b, n_s
    int64_t steps_done = 0;
    double J_prev[3] = {0, 0, 0};
    bool have_prev = false;
    double t_admit = 0.0;
};

}  // namespace

struct lbm_server {
    lbm_server_cfg cfg{};
    int device = 0;
    hipStream_t stream = nullptr;
    void* scratch = nullptr;
    uint64_t scratch_bytes = 0;
    uint64_t budget = 0;
    BatchRunner runner;
    std::chrono::steady_clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> queue;
    std::unordered_map<uint64_t, lbm_result> done;
    std::unordered_map<uint64_t, int> live;  // submitted and not final
    uint64_t next_id = 1;
    bool stop = false;
    std::thread worker;

    // worker-owned
    std::vector<Slot> active;
    std::vector<hm::BatchDomain> doms;
    uint64_t resident = 0;

    // statistics (guarded by mu)
    lbm_server_stats st{};
    double busy_since = -1.0;

    void run();
    int admit(Request&& r);
    void retire(size_t i, int status, bool converged);
};

namespace {

uint64_t state_bytes(const lbm_domain& d, const lbm_params& p)
{
    lbm_sizes s{};
    if (lbm_required_bytes(&d, &p, &s)) return 0;
    return 2 * s.pop_bytes + s.ns_bytes;
}

}  // namespace

int lbm_server::admit(Request&& r)
{
    Slot sl;
    sl.req = std::move(r);
    lbm_sizes sz{};
    lbm_required_bytes(&sl.req.dom, &sl.req.prm, &sz);
    if (hipMalloc(&sl.mem[0], sz.pop_bytes) != hipSuccess || hipMalloc(&sl.mem[1], sz.pop_bytes) != hipSuccess ||
        hipMalloc(&sl.mem[2], sz.ns_bytes) != hipSuccess) {
        (void)hipGetLastError();
        for (void* m : sl.mem)
            if (m) (void)hipFree(m);
        return LBM_ENOMEM;
    }
    lbm_device_buffers b{sl.mem[0], sl.mem[1], sl.mem[2], scratch};
    const int rc = lbm_create(&sl.req.dom, sl.req.ns.data(), sl.req.rho.data(), &sl.req.prm, &b, stream, &sl.ctx);
    if (rc) {
        for (void* m : sl.mem)
            if (m) (void)hipFree(m);
        return rc;
    }
    sl.req.ns.clear();
    sl.req.ns.shrink_to_fit();
    sl.req.rho.clear();
    sl.req.rho.shrink_to_fit();
    sl.t_admit = now_s(t0);
    resident += sl.req.bytes;
    active.push_back(std::move(sl));
    return LBM_OK;
}

void lbm_server::retire(size_t i, int status, bool converged)
{
    Slot& sl = active[i];
    lbm_result res{};
    res.status = status;
    res.converged = converged ? 1 : 0;
    res.steps_done = sl.steps_done;
    res.t_submit = sl.req.t_submit;
    res.t_admit = sl.t_admit;
    if (status == LBM_OK) {
        const int rc = lbm_moments(sl.ctx, sl.req.rho_out, nullptr, nullptr, &res.totals);
        if (rc) res.status = rc;
    }
    res.t_done = now_s(t0);
    lbm_destroy(sl.ctx);
    for (void* m : sl.mem)
        if (m) (void)hipFree(m);
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
    for (;;) {
        std::vector<Request> admitted;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (active.empty() && queue.empty() && !stop) {
                if (busy_since >= 0) {
                    st.busy_seconds += now_s(t0) - busy_since;
                    busy_since = -1.0;
                }
                cv_work.wait_for(lk, std::chrono::milliseconds(20));
            }
            if (stop) break;
            // admission: in arrival order while a slot is free and the state fits
            uint64_t planned = resident;
            while (!queue.empty() && static_cast<int>(active.size() + admitted.size()) < cfg.max_slots &&
                   planned + queue.front().bytes <= budget) {
                planned += queue.front().bytes;
                admitted.push_back(std::move(queue.front()));
                queue.pop_front();
            }
            st.queued = static_cast<int64_t>(queue.size());
        }
        for (Request& r : admitted) {
            const uint64_t id = r.id;
            const double ts = r.t_submit;
            const int rc = admit(std::move(r));
            if (rc) {
                lbm_result res{};
                res.status = rc;
                res.t_submit = ts;
                res.t_done = now_s(t0);
                std::lock_guard<std::mutex> lk(mu);
                done[id] = res;
                live.erase(id);
                st.completed += 1;
                cv_done.notify_all();
            }
        }
        if (active.empty()) continue;
        {
            std::lock_guard<std::mutex> lk(mu);
            if (busy_since < 0) busy_since = now_s(t0);
            st.active = static_cast<int64_t>(active.size());
            st.bytes_resident = resident;
        }
        // one tick: K launches over the resident domains this tick steps
        const int K = runner.kmax();
        std::vector<int> steps(active.size());
        for (size_t i = 0; i < active.size(); ++i)
            steps[i] = static_cast<int>(std::min<int64_t>(K, active[i].req.max_steps - active[i].steps_done));
        if (cfg.policy == LBM_SERVE_SHORTEST_FIRST) {
            std::vector<size_t> order(active.size());
            std::vector<double> work(active.size());
            for (size_t i = 0; i < active.size(); ++i) {
                order[i] = i;
                work[i] = static_cast<double>(active[i].ctx->prob.N) *
                          static_cast<double>(active[i].req.max_steps - active[i].steps_done);
            }
            std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return work[a] < work[b]; });
            int64_t stepped = 0;
            for (size_t i : order) {
                if (stepped >= cfg.run_cells) steps[i] = 0;
                else stepped += active[i].ctx->prob.N;
            }
        }
        doms.clear();
        double cells = 0.0;
        for (size_t i = 0; i < active.size(); ++i) {
            if (!steps[i]) continue;
            doms.push_back(domain_of(active[i].ctx, steps[i]));
            cells += static_cast<double>(active[i].ctx->prob.N) * steps[i];
        }
        int rc = runner.run(doms.data(), static_cast<int>(doms.size()), K);
        if (rc == LBM_OK && hipStreamSynchronize(stream) != hipSuccess) rc = LBM_EDEVICE;
        for (size_t i = 0; i < active.size(); ++i) {
            advance(active[i].ctx, steps[i]);
            active[i].steps_done += steps[i];
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            st.cell_updates += cells;
            st.ticks += 1;
        }
        // retire finished, converged or failed domains
        for (size_t i = active.size(); i-- > 0;) {
            Slot& sl = active[i];
            if (rc) {
                retire(i, rc, false);
                continue;
            }
            if (sl.steps_done >= sl.req.max_steps) {
                retire(i, LBM_OK, false);
                continue;
            }
            if (sl.req.tol > 0.0 && steps[i] > 0) {
                lbm_totals tt{};
                const int trc = lbm_totals_get(sl.ctx, &tt);
                if (trc || !tt.finite) {
                    retire(i, trc ? trc : LBM_EUNSTABLE, false);
                    continue;
                }
                const double nJ = std::sqrt(tt.momentum[0] * tt.momentum[0] + tt.momentum[1] * tt.momentum[1] +
                                            tt.momentum[2] * tt.momentum[2]);
                double dJ = 0.0;
                for (int a = 0; a < 3; ++a) dJ += (tt.momentum[a] - sl.J_prev[a]) * (tt.momentum[a] - sl.J_prev[a]);
                dJ = std::sqrt(dJ);
                const bool conv = sl.have_prev && dJ <= sl.req.tol * nJ;
                for (int a = 0; a < 3; ++a) sl.J_prev[a] = tt.momentum[a];
                sl.have_prev = true;
                if (conv) retire(i, LBM_OK, true);
            }
        }
    }
    // shutting down: everything still queued or resident ends unfinished
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
    if (hipGetDevice(&s->device) != hipSuccess || hipStreamCreate(&s->stream) != hipSuccess) {
        delete s;
        return LBM_EDEVICE;
    }
    s->scratch_bytes = hm_rt::scratch_layout(cfg->max_cells, cfg->ncomp).bytes;
    if (hipMalloc(&s->scratch, s->scratch_bytes) != hipSuccess) {
        (void)hipStreamDestroy(s->stream);
        delete s;
        return LBM_ENOMEM;
    }
    size_t free_b = 0, total_b = 0;
    (void)hipMemGetInfo(&free_b, &total_b);
    s->budget = cfg->hbm_budget_bytes ? cfg->hbm_budget_bytes : static_cast<uint64_t>(0.9 * free_b);
    const int rc = s->runner.init(cfg->storage, cfg->ncomp, cfg->c_ns, tx, ty, cfg->max_slots, cfg->steps_per_tick,
                                  s->stream);
    if (rc) {
        s->runner.release();
        (void)hipFree(s->scratch);
        (void)hipStreamDestroy(s->stream);
        delete s;
        return rc;
    }
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
    r.rho_out = rq->rho_out;
    r.bytes = state_bytes(rq->dom, p);
    if (r.bytes > s->budget) return LBM_ENOMEM;
    r.ns.assign(rq->n_s, rq->n_s + static_cast<size_t>(p.c_ns) * N);
    r.rho.assign(rq->rho_init, rq->rho_init + static_cast<size_t>(p.ncomp) * N);
    for (float v : r.ns)
        if (!(v >= 0.0f && v <= 1.0f)) return LBM_EINVAL;
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
    if (s->scratch) (void)hipFree(s->scratch);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // extern "C"

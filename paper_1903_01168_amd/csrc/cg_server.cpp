// cg_server.cpp -- continuous-batching solve server (include/cglbm_serve.h).
//
// A server thread owns the scheduling loop: admit queued requests in arrival
// order while slots and the HBM budget allow (head of line waits: no request
// is overtaken, so none starves), run one chunk of batched steps over every
// active lattice, retire the finished ones, repeat.  The GPU backend advances
// all active lattices with one k_step launch per step, a chunk being a
// captured HIP graph of chunk_steps launches; the fake backend does the same
// bookkeeping on a virtual clock without touching a GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "cg_capi_internal.hpp"
#include "cg_kernels.hpp"
#include "cg_schedule.hpp"
#include "cglbm.h"
#include "cglbm_serve.h"

namespace {

struct Request {
    lbm_req id = 0;
    lbm_params p{};
    int32_t kind = LBM_INIT_FIELDS;
    std::vector<double> f[4];            // FIELDS inputs
    lbm_init_desc geo{};                 // DISK / BANDS scalars (pointers cleared)
    std::vector<int32_t> edges;
    std::vector<int8_t> inlet;
    int64_t steps = 0, done = 0;
    bool keep = false;
    bool fail_flag = false;
    int status = LBM_E_BUSY;
    int slot = -1;
    double t_arrive = 0, t_admit = 0, t_done = 0;
    lbm_diag_t diag{};
    std::vector<double> out[5];
    size_t bytes = 0;
    lbm_ctx *ctx = nullptr;
    long long nodes() const { return (long long)p.nx * p.ny; }
};

// Sharp initial colour densities of a request, on the host.
void init_fields(const Request &r, std::vector<double> &rr, std::vector<double> &rb)
{
    const int nx = r.p.nx, ny = r.p.ny;
    const size_t n = (size_t)nx * ny;
    rr.assign(n, 0.0);
    rb.assign(n, 0.0);
    if (r.kind == LBM_INIT_FIELDS) {
        rr = r.f[0];
        rb = r.f[1];
        return;
    }
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const size_t c = (size_t)y * nx + x;
            if (r.kind == LBM_INIT_DISK) {
                const double dx = x + 0.5 - r.geo.cx, dy = y + 0.5 - r.geo.cy;
                const bool in = dx * dx + dy * dy < r.geo.radius * r.geo.radius;
                rr[c] = in ? r.geo.rho_r_in : r.geo.rho_r_out;
                rb[c] = in ? r.geo.rho_b_in : r.geo.rho_b_out;
            } else {
                int band = 0;
                while (band + 1 < (int)r.edges.size() && x >= r.edges[band + 1]) ++band;
                const bool red = (band % 2) == 0;
                rr[c] = red ? r.geo.rho_band_r : 0.0;
                rb[c] = red ? 0.0 : r.geo.rho_band_b;
            }
        }
}

struct Backend {
    virtual ~Backend() = default;
    virtual size_t bytes(const lbm_params &p) = 0;
    virtual int admit(Request &r, std::string &err) = 0;
    // launch one chunk of K steps over `act` (asynchronous on the GPU)...
    virtual int launch_chunk(const std::vector<Request *> &act, int K, std::string &err) = 0;
    // ... and wait for it; then the step counts of `act` are advanced
    virtual int wait_chunk(const std::vector<Request *> &act, int K, std::string &err) = 0;
    virtual void retire(Request &r) = 0;
    virtual double now() = 0;
};

struct FakeBackend : Backend {
    double mlups;
    std::atomic<double> vt{0.0};      // virtual clock, advanced by the server thread
    explicit FakeBackend(double m) : mlups(m) {}
    size_t bytes(const lbm_params &p) override { return lbm_bytes_required(&p); }
    int admit(Request &, std::string &) override { return LBM_OK; }
    int launch_chunk(const std::vector<Request *> &, int, std::string &) override { return LBM_OK; }
    int wait_chunk(const std::vector<Request *> &act, int K, std::string &) override
    {
        double lu = 0.0;
        for (auto *r : act) {
            const int64_t k = std::min<int64_t>(K, r->steps - r->done);
            r->done += k;
            lu += (double)r->nodes() * (double)k;
        }
        vt.store(vt.load() + lu / (mlups * 1e6));
        return LBM_OK;
    }
    void retire(Request &r) override
    {
        r.diag = lbm_diag_t{};
        r.diag.step = r.done;
        r.diag.mass_r = (double)r.nodes();
    }
    double now() override { return vt.load(); }
};

struct GpuBackend : Backend {
    int storage, tx, device = 0, max_slots;
    hipStream_t stream = nullptr, cap = nullptr;
    // two lanes (streams) step two cache groups of a chunk at a time; the
    // server stream forks to them after the table upload and joins them
    hipStream_t lane[2] = {nullptr, nullptr};
    hipEvent_t ev_fork = nullptr, ev_lane[2] = {nullptr, nullptr};
    bool own_stream = false;
    cgd::SlotDesc *d_slots = nullptr;
    std::vector<cgd::SlotDesc> table;
    // one captured chunk per cache group, re-captured when its shape changes
    struct Chunk {
        hipGraphExec_t graph = nullptr;
        int off = -1, nslots = -1, tiles = -1, K = -1;
        int variant = 0, tx = 0;
    };
    std::vector<Chunk> chunks;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    GpuBackend(int st, int t, int ms) : storage(st), tx(t), max_slots(ms) {}
    ~GpuBackend() override
    {
        if (stream) (void)hipStreamSynchronize(stream);
        for (hipStream_t l : lane)
            if (l) (void)hipStreamSynchronize(l);
        for (auto &c : chunks)
            if (c.graph) (void)hipGraphExecDestroy(c.graph);
        if (d_slots) (void)hipFree(d_slots);
        if (cap) (void)hipStreamDestroy(cap);
        for (hipStream_t l : lane)
            if (l) (void)hipStreamDestroy(l);
        for (hipEvent_t ev : {ev_fork, ev_lane[0], ev_lane[1]})
            if (ev) (void)hipEventDestroy(ev);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
    int setup(void *user_stream, std::string &err)
    {
        (void)hipGetDevice(&device);
        hipError_t e;
        if (user_stream) {
            stream = (hipStream_t)user_stream;
        } else {
            if ((e = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking)) != hipSuccess) {
                err = hipGetErrorString(e);
                return LBM_E_DEVICE;
            }
            own_stream = true;
        }
        if ((e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipMalloc(&d_slots, (size_t)max_slots * sizeof(cgd::SlotDesc))) != hipSuccess) {
            d_slots = nullptr;
            err = hipGetErrorString(e);
            return LBM_E_DEVICE;
        }
        for (hipStream_t &l : lane)
            if (e == hipSuccess) e = hipStreamCreateWithFlags(&l, hipStreamNonBlocking);
        for (hipEvent_t *ev : {&ev_fork, &ev_lane[0], &ev_lane[1]})
            if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            err = hipGetErrorString(e);
            return LBM_E_DEVICE;
        }
        return LBM_OK;
    }
    size_t bytes(const lbm_params &p) override { return lbm_bytes_required(&p); }
    int admit(Request &r, std::string &err) override
    {
        (void)hipSetDevice(device);
        int rc = lbm_create(&r.p, stream, &r.ctx);
        if (rc != LBM_OK) {
            err = lbm_last_error(nullptr);
            return rc;
        }
        std::vector<double> rr, rb;
        init_fields(r, rr, rb);
        const double *ux = r.kind == LBM_INIT_FIELDS && !r.f[2].empty() ? r.f[2].data() : nullptr;
        const double *uy = r.kind == LBM_INIT_FIELDS && !r.f[3].empty() ? r.f[3].data() : nullptr;
        rc = lbm_init_fields(r.ctx, rr.data(), rb.data(), ux, uy);
        if (rc == LBM_OK && !r.inlet.empty()) rc = lbm_set_inlet_color(r.ctx, r.inlet.data());
        if (rc != LBM_OK) {
            err = lbm_last_error(r.ctx);
            lbm_destroy(r.ctx);
            r.ctx = nullptr;
        }
        return rc;
    }
    // Chunk of K steps over the active lattices: groups (in admission order)
    // sized so that two fit the cache together, each running its K launches
    // from its own graph; with several groups, two lanes take whole groups
    // (largest first, to the lane with less work queued), so that two
    // groups are in flight at a time.
    int launch_chunk(const std::vector<Request *> &act, int K, std::string &err) override
    {
        (void)hipSetDevice(device);
        table.clear();
        std::vector<size_t> bytes;
        std::vector<char> kind;
        for (auto *r : act) {
            bytes.push_back(2 * r->ctx->buf_bytes);
            kind.push_back((char)cgd::step_variant(r->ctx->desc));
        }
        const std::vector<int> first = cgi::cache_groups(bytes, kind, cgi::kPairBudget / 2, 2);
        const int ng = (int)first.size() - 1;
        std::vector<int> gtiles(ng, 0);
        std::vector<int> gvar(ng, 0);      // the group's step-kernel variant (KV_XCH included)
        std::vector<int> gtx(ng, 0);       // its threads per workgroup
        std::vector<long long> gnodes(ng, 0);
        for (int g = 0; g < ng; ++g)
            for (int i = first[g]; i < first[g + 1]; ++i) gnodes[g] += act[i]->nodes();
        // strips planned for what shares the chip: the two largest groups
        long long pair_nodes = 0;
        {
            std::vector<long long> srt(gnodes);
            std::sort(srt.begin(), srt.end());
            pair_nodes = srt.back() + (ng > 1 ? srt[ng - 2] : 0);
        }
        for (int g = 0; g < ng; ++g) {
            long long tiles = 0;
            size_t gbytes = 0;
            std::vector<lbm_ctx *> gctx;
            for (int i = first[g]; i < first[g + 1]; ++i) {
                gbytes += bytes[i];
                gctx.push_back(act[i]->ctx);
            }
            const cgi::GroupPlan gp = cgi::plan_group(gbytes, storage, kind[first[g]], tx, gctx.data(), (int)gctx.size());
            gvar[g] = gp.variant;
            gtx[g] = gp.tx;
            const bool xch = gp.variant & cgd::KV_XCH;
            for (int i = first[g]; i < first[g + 1]; ++i) {
                const Request *r = act[i];
                lbm_ctx *c = r->ctx;
                cgd::SlotDesc d = c->desc;
                cgi::set_geometry(d, &c->p, c->lay, gp.tx, 1, xch);
                cgi::set_geometry(d, &c->p, c->lay, gp.tx,
                                  cgi::plan_strip(pair_nodes, c->p.ny, d.tiles_x, c->p.storage, 0, ng > 1, xch), xch);
                d.tile_begin = (int)tiles;
                d.active_steps = (int)std::min<int64_t>(K, r->steps - r->done);
                if (c->steps & 1) std::swap(d.buf[0], d.buf[1]);   // launch 0 reads the current buffer
                tiles += (long long)d.tiles_x * d.tiles_y;
                table.push_back(d);
            }
            if (tiles > INT_MAX / 2) {
                err = "too many tiles in one chunk";
                return LBM_E_INVAL;
            }
            gtiles[g] = (int)tiles;
        }
        hipError_t e = hipMemcpyAsync(d_slots, table.data(), table.size() * sizeof(cgd::SlotDesc),
                                      hipMemcpyHostToDevice, stream);
        if ((int)chunks.size() < ng) chunks.resize(ng);
        const std::vector<int> glane = cgs::assign_whole(gnodes);
        if (ng > 1) {
            if (e == hipSuccess) e = hipEventRecord(ev_fork, stream);
            for (hipStream_t l : lane)
                if (e == hipSuccess) e = hipStreamWaitEvent(l, ev_fork, 0);
        }
        for (int g = 0; g < ng && e == hipSuccess; ++g) {
            Chunk &ch = chunks[g];
            const int off = first[g], ns = first[g + 1] - first[g], nt = gtiles[g];
            const int var = gvar[g], gt = gtx[g];
            if (ch.off != off || ch.nslots != ns || ch.tiles != nt || ch.K != K || ch.variant != var || ch.tx != gt) {
                if (ch.graph) (void)hipGraphExecDestroy(ch.graph);
                ch = Chunk{};
                hipGraph_t gr = nullptr;
                e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
                hipError_t le = hipSuccess;
                for (int j = 0; j < K && e == hipSuccess && le == hipSuccess; ++j)
                    le = cgd::launch_step(storage, gt, d_slots + off, ns, nt, j & 1, j, cap, var);
                if (e == hipSuccess) e = hipStreamEndCapture(cap, &gr);
                if (e == hipSuccess) e = le;
                if (e == hipSuccess) e = hipGraphInstantiate(&ch.graph, gr, nullptr, nullptr, 0);
                if (gr) (void)hipGraphDestroy(gr);
                if (e == hipSuccess) ch = Chunk{ch.graph, off, ns, nt, K, var, gt};
                else ch = Chunk{};
            }
            if (e == hipSuccess) e = hipGraphLaunch(ch.graph, ng > 1 ? lane[glane[g]] : stream);
        }
        if (ng > 1) {   // join (also after a failure): the server stream waits for both lanes
            hipError_t je = hipSuccess;
            for (int l = 0; l < 2 && je == hipSuccess; ++l) je = hipEventRecord(ev_lane[l], lane[l]);
            for (int l = 0; l < 2 && je == hipSuccess; ++l) je = hipStreamWaitEvent(stream, ev_lane[l], 0);
            if (e == hipSuccess) e = je;
        }
        if (e != hipSuccess) {
            err = hipGetErrorString(e);
            return LBM_E_DEVICE;
        }
        return LBM_OK;
    }
    int wait_chunk(const std::vector<Request *> &act, int K, std::string &err) override
    {
        const hipError_t e = hipStreamSynchronize(stream);   // the table is reused by the next chunk
        if (e != hipSuccess) {
            err = hipGetErrorString(e);
            return LBM_E_DEVICE;
        }
        for (auto *r : act) {
            const int64_t k = std::min<int64_t>(K, r->steps - r->done);
            r->done += k;
            r->ctx->steps += k;
        }
        return LBM_OK;
    }
    void retire(Request &r) override
    {
        if (!r.ctx) return;
        (void)hipSetDevice(device);
        lbm_diag_t d{};
        int rc = lbm_diag(r.ctx, nullptr, &d);
        if (rc == LBM_OK && r.kind == LBM_INIT_DISK && d.area_r > 0) {
            // Laplace sampling of a bubble: mean pressure inside r < R - 4 and
            // outside r > R + 4, R the radius of a disk of the red area
            const double R = std::sqrt(d.area_r / M_PI);
            const double circle[4] = {r.geo.cx, r.geo.cy, R - 4.0, R + 4.0};
            rc = lbm_diag(r.ctx, circle, &d);
        }
        r.diag = d;
        if (rc == LBM_E_UNSTABLE && r.status == LBM_E_BUSY) r.status = LBM_E_UNSTABLE;
        else if (rc != LBM_OK && r.status == LBM_E_BUSY) r.status = rc;
        if (r.keep) {
            const size_t n = (size_t)r.nodes();
            for (auto &o : r.out) o.assign(n, 0.0);
            (void)lbm_moments(r.ctx, r.out[0].data(), r.out[1].data(), r.out[2].data(), r.out[3].data(),
                              r.out[4].data(), nullptr);
        }
        lbm_destroy(r.ctx);
        r.ctx = nullptr;
    }
    double now() override
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

}  // namespace

struct lbm_server {
    std::unique_ptr<Backend> be;
    size_t budget = 0, held = 0;
    int max_slots = 0, chunk = 0;
    int storage = 0;
    std::mutex m;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> pending;
    std::vector<Request *> active;
    std::vector<int> free_slots;
    std::map<lbm_req, std::unique_ptr<Request>> reqs;
    lbm_req next_id = 1;
    bool stop = false;
    lbm_server_stats st{};
    std::thread worker;
    std::string err;

    void finish(Request *r, int status)
    {
        if (r->status == LBM_E_BUSY) r->status = status;
        r->t_done = be->now();
        if (r->status == LBM_OK) st.completed++;
        else st.failed++;
        cv_done.notify_all();
    }

    // Admission: arrival order, the head of the queue waits for capacity.
    // Called with the lock held; the backend's work runs unlocked.
    void admit_pending(std::unique_lock<std::mutex> &lk)
    {
        while (!pending.empty() && (int)active.size() < max_slots && !stop) {
            Request *r = pending.front();
            if (r->bytes > budget) {
                pending.pop_front();
                finish(r, LBM_E_NOMEM);
                continue;
            }
            if (held + r->bytes > budget) break;
            pending.pop_front();
            r->slot = free_slots.back();
            free_slots.pop_back();
            held += r->bytes;
            lk.unlock();
            std::string e;
            const auto t = std::chrono::steady_clock::now();
            const int rc = be->admit(*r, e);
            const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t).count();
            lk.lock();
            st.admit_s += dt;
            if (rc != LBM_OK) {
                held -= r->bytes;
                free_slots.push_back(r->slot);
                err = e;
                finish(r, rc);
                continue;
            }
            r->t_admit = be->now();
            active.push_back(r);
            st.admitted++;
            st.peak_active = std::max<int64_t>(st.peak_active, (int64_t)active.size());
            st.peak_bytes = std::max<uint64_t>(st.peak_bytes, held);
        }
    }

    // One round: launch a chunk over the runnable lattices, admit arrivals
    // while it runs on the device (their set-up is host work and device work
    // queued behind the chunk), wait for the chunk, retire what finished.
    void loop()
    {
        std::unique_lock<std::mutex> lk(m);
        for (;;) {
            cv_work.wait(lk, [&] { return stop || !pending.empty() || !active.empty(); });
            if (stop) break;
            std::vector<Request *> act;
            for (auto *r : active)
                if (!r->fail_flag && r->done < r->steps) act.push_back(r);
            int rc = LBM_OK;
            bool launched = false;
            double t_launch = 0.0;
            if (!act.empty()) {
                lk.unlock();
                std::string e;
                t_launch = be->now();
                rc = be->launch_chunk(act, chunk, e);
                lk.lock();
                launched = rc == LBM_OK;
                if (rc != LBM_OK) err = e;
            }
            admit_pending(lk);
            if (launched) {
                lk.unlock();
                std::string e;
                rc = be->wait_chunk(act, chunk, e);
                const double dt = be->now() - t_launch;
                lk.lock();
                st.busy_s += dt;
                st.chunks++;
                st.launches += chunk;
                if (rc != LBM_OK) err = e;
            }
            // retire finished, failed and injected-failure lattices (a failed
            // chunk fails the lattices that were in it)
            std::vector<Request *> keep;
            for (auto *r : active) {
                const bool in_chunk = std::find(act.begin(), act.end(), r) != act.end();
                const bool fin = r->done >= r->steps;
                const bool chunk_failed = rc != LBM_OK && in_chunk;
                if (!fin && !r->fail_flag && !chunk_failed) {
                    keep.push_back(r);
                    continue;
                }
                if (r->fail_flag) r->status = LBM_E_UNSTABLE;
                else if (chunk_failed) r->status = rc;
                lk.unlock();
                const auto t = std::chrono::steady_clock::now();
                be->retire(*r);
                const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t).count();
                lk.lock();
                st.retire_s += dt;
                st.lattice_updates += (double)r->nodes() * (double)r->done;
                held -= r->bytes;
                free_slots.push_back(r->slot);
                finish(r, LBM_OK);
            }
            active.swap(keep);
        }
        // shutdown: release running lattices, drop the queue
        for (auto *r : active) {
            lk.unlock();
            be->retire(*r);
            lk.lock();
        }
        active.clear();
        pending.clear();
        cv_done.notify_all();
    }
};

static thread_local std::string g_serr;

static int sfail(lbm_server *s, int code, const std::string &msg)
{
    if (s) {
        std::lock_guard<std::mutex> g(s->m);
        s->err = msg;
    }
    g_serr = msg;
    return code;
}

static int create_server(std::unique_ptr<Backend> be, size_t budget, int32_t max_slots, int32_t chunk, int32_t storage,
                         lbm_server **out)
{
    lbm_server *s = new (std::nothrow) lbm_server();
    if (!s) return sfail(nullptr, LBM_E_NOMEM, "host allocation failed");
    s->be = std::move(be);
    s->budget = budget;
    s->max_slots = max_slots;
    s->chunk = chunk;
    s->storage = storage;
    for (int i = max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
    s->worker = std::thread([s] { s->loop(); });
    *out = s;
    return LBM_OK;
}

static int check_create(size_t budget, int32_t max_slots, int32_t chunk, lbm_server **out)
{
    if (!out) return sfail(nullptr, LBM_E_INVAL, "out is NULL");
    *out = nullptr;
    if (budget == 0) return sfail(nullptr, LBM_E_INVAL, "hbm_budget must be > 0");
    if (max_slots < 1 || max_slots > 4096) return sfail(nullptr, LBM_E_INVAL, "max_slots must be in 1..4096");
    if (chunk < 2 || (chunk & 1)) return sfail(nullptr, LBM_E_INVAL, "chunk_steps must be even and >= 2");
    return LBM_OK;
}

extern "C" {

const char *lbm_server_last_error(const lbm_server *s) { return s ? s->err.c_str() : g_serr.c_str(); }

int lbm_server_create(size_t hbm_budget, int32_t max_slots, int32_t chunk_steps, int32_t storage, int32_t tile_x,
                      void *hip_stream, lbm_server **out)
{
    int rc = check_create(hbm_budget, max_slots, chunk_steps, out);
    if (rc != LBM_OK) return rc;
    if (storage < LBM_STORE_F32 || storage > LBM_STORE_BF16S) return sfail(nullptr, LBM_E_INVAL, "unknown storage");
    if (tile_x != 0 && tile_x != 64 && tile_x != 128 && tile_x != 256)
        return sfail(nullptr, LBM_E_INVAL, "tile_x must be 0, 64, 128 or 256");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return sfail(nullptr, LBM_E_DEVICE, "no HIP device");
    auto be = std::make_unique<GpuBackend>(storage, tile_x, max_slots);   // tile_x 0: planned per group
    std::string e;
    if ((rc = be->setup(hip_stream, e)) != LBM_OK) return sfail(nullptr, rc, e);
    return create_server(std::move(be), hbm_budget, max_slots, chunk_steps, storage, out);
}

int lbm_server_create_fake(size_t hbm_budget, int32_t max_slots, int32_t chunk_steps, double mlups,
                           lbm_server **out)
{
    int rc = check_create(hbm_budget, max_slots, chunk_steps, out);
    if (rc != LBM_OK) return rc;
    if (!(mlups > 0)) return sfail(nullptr, LBM_E_INVAL, "mlups must be > 0");
    return create_server(std::make_unique<FakeBackend>(mlups), hbm_budget, max_slots, chunk_steps, LBM_STORE_F32, out);
}

int lbm_enqueue_solve(lbm_server *s, const lbm_params *p, const lbm_init_desc *init, int64_t steps,
                      int32_t keep_fields, lbm_req *id)
{
    if (!s || !p || !init || !id) return sfail(s, LBM_E_INVAL, "NULL argument");
    if (steps < 0) return sfail(s, LBM_E_INVAL, "steps must be >= 0");
    auto r = std::make_unique<Request>();
    r->p = *p;
    r->p.storage = s->storage;
    std::string msg;
    int rc = cgi::validate(&r->p, msg);
    if (rc != LBM_OK) return sfail(s, rc, msg);
    const size_t n = (size_t)p->nx * p->ny;
    r->kind = init->kind;
    if (init->kind == LBM_INIT_FIELDS) {
        if (!init->rho_r || !init->rho_b) return sfail(s, LBM_E_INVAL, "FIELDS needs rho_r and rho_b");
        r->f[0].assign(init->rho_r, init->rho_r + n);
        r->f[1].assign(init->rho_b, init->rho_b + n);
        if (init->ux) r->f[2].assign(init->ux, init->ux + n);
        if (init->uy) r->f[3].assign(init->uy, init->uy + n);
    } else if (init->kind == LBM_INIT_DISK) {
        if (!(init->radius > 0)) return sfail(s, LBM_E_INVAL, "DISK needs radius > 0");
    } else if (init->kind == LBM_INIT_BANDS) {
        if (init->n_edges < 1 || !init->edges || init->edges[0] != 0)
            return sfail(s, LBM_E_INVAL, "BANDS needs edges starting at 0");
        r->edges.assign(init->edges, init->edges + init->n_edges);
        for (size_t i = 1; i < r->edges.size(); ++i)
            if (r->edges[i] <= r->edges[i - 1]) return sfail(s, LBM_E_INVAL, "BANDS edges must increase");
    } else {
        return sfail(s, LBM_E_INVAL, "unknown init kind");
    }
    r->geo = *init;
    r->geo.rho_r = r->geo.rho_b = r->geo.ux = r->geo.uy = nullptr;
    r->geo.edges = nullptr;
    r->geo.inlet_color = nullptr;
    if (init->inlet_color) r->inlet.assign(init->inlet_color, init->inlet_color + p->ny);
    r->steps = steps;
    r->keep = keep_fields != 0;
    r->bytes = s->be->bytes(r->p);
    std::lock_guard<std::mutex> g(s->m);
    if (s->stop) return sfail(nullptr, LBM_E_INVAL, "server is shutting down");
    r->id = s->next_id++;
    r->t_arrive = s->be->now();
    *id = r->id;
    s->pending.push_back(r.get());
    s->reqs[r->id] = std::move(r);
    s->st.enqueued++;
    s->cv_work.notify_one();
    return LBM_OK;
}

static int fill_result(const Request &r, lbm_result *out)
{
    if (!out) return r.status;
    out->status = r.status;
    out->slot = r.slot;
    out->steps_done = r.done;
    out->t_arrive = r.t_arrive;
    out->t_admit = r.t_admit;
    out->t_done = r.t_done;
    out->diag = r.diag;
    double *dst[5] = {out->rho_r, out->rho_b, out->ux, out->uy, out->p};
    if (r.status != LBM_E_BUSY)
        for (int f = 0; f < 5; ++f)
            if (dst[f] && r.out[f].size() == (size_t)r.nodes()) std::memcpy(dst[f], r.out[f].data(), r.out[f].size() * 8);
    return r.status;
}

int lbm_poll(lbm_server *s, lbm_req id, lbm_result *r)
{
    if (!s) return sfail(nullptr, LBM_E_INVAL, "server is NULL");
    std::lock_guard<std::mutex> g(s->m);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return LBM_E_NOTFOUND;
    return fill_result(*it->second, r);
}

int lbm_wait(lbm_server *s, lbm_req id, lbm_result *r)
{
    if (!s) return sfail(nullptr, LBM_E_INVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(s->m);
    for (;;) {
        auto it = s->reqs.find(id);
        if (it == s->reqs.end()) return LBM_E_NOTFOUND;
        if (it->second->status != LBM_E_BUSY) return fill_result(*it->second, r);
        if (s->stop) return LBM_E_NOTFOUND;
        s->cv_done.wait(lk);
    }
}

int lbm_release(lbm_server *s, lbm_req id)
{
    if (!s) return sfail(nullptr, LBM_E_INVAL, "server is NULL");
    std::lock_guard<std::mutex> g(s->m);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return LBM_E_NOTFOUND;
    if (it->second->status == LBM_E_BUSY) return LBM_E_BUSY;
    s->reqs.erase(it);
    return LBM_OK;
}

int lbm_server_stats_get(lbm_server *s, lbm_server_stats *st)
{
    if (!s || !st) return sfail(s, LBM_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> g(s->m);
    *st = s->st;
    return LBM_OK;
}

int lbm_server_inject_failure(lbm_server *s, lbm_req id)
{
    if (!s) return sfail(nullptr, LBM_E_INVAL, "server is NULL");
    std::lock_guard<std::mutex> g(s->m);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return LBM_E_NOTFOUND;
    it->second->fail_flag = true;
    s->cv_work.notify_one();
    return LBM_OK;
}

int lbm_server_destroy(lbm_server *s)
{
    if (!s) return LBM_OK;
    {
        std::lock_guard<std::mutex> g(s->m);
        s->stop = true;
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
    if (s->worker.joinable()) s->worker.join();
    delete s;
    return LBM_OK;
}

}  // extern "C"

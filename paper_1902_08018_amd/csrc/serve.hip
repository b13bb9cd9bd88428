// serve.hip -- the real-time request loop (wh_submit / wh_poll).
//
// The paper's loop evaluates the deformation product every light-stage
// millisecond against resident field matrices, under a firm deadline: a late
// result is still delivered but counts as a miss (Sec. 1, Sec. 2.1, Fig. 2).
// Here many such dose-vector requests, against several resident matrices of
// different sizes, share one GPU:
//
//   submit      any thread; the request is validated, stamped and queued
//   admission   each matrix gets device slots (U, Y and the FP64 slab
//               partials of one batch) carved out of the context's HBM
//               budget: one on first use, a second (one batch runs while the
//               next is staged) if the budget still holds the first slots of
//               every other resident matrix; a batch waits for a free slot;
//               a request that can never fit is rejected at submit
//   batching    continuous: whenever a slot of a matrix is free, all queued
//               requests of that matrix (FIFO, up to 64 right-hand sides) form
//               one batch; requests that arrive while it runs form the next
//   launch      U rows are copied into the slot, the slot's pre-instantiated
//               hipGraph for the batch's k-bucket (1, 2, 4, 8, 16, 32, 64) is
//               replayed on the matrix's own stream, Y rows are copied back,
//               an event is recorded.  A graph is a chain of fused
//               decode+GEMV launches over consecutive row chunks of at most
//               ctx->serve_chunk_values values: a long pass over a big matrix
//               does not hold every compute unit until it ends, and batches
//               of other matrices start between its chunks
//   completion  the worker polls the events; a finished batch stamps t_done
//               on its requests and frees the slot
//   poll        never blocks: WH_PENDING, or the result once (then retired)
//
// Streams of different matrices run concurrently on the device.  All streams
// keep the default priority.
#include <hip/hip_runtime.h>

#include <time.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "wh_ctx.hpp"
#include "wh_internal.hpp"

namespace wh {

namespace {

uint64_t now_ns()
{
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

constexpr uint32_t kBuckets[] = {1, 2, 4, 8, 16, 32, 64};
constexpr int kNumBuckets = sizeof(kBuckets) / sizeof(kBuckets[0]);
constexpr int kMaxSlotsPerMatrix = 2;

int bucket_index(uint32_t k)
{
    for (int i = 0; i < kNumBuckets; ++i)
        if (k <= kBuckets[i])
            return i;
    return -1;
}

struct Req {
    wh_request r;
    uint64_t t_arrive = 0, t_start = 0, t_done = 0;
    wh_status status = WH_PENDING;
    uint32_t batch_size = 0;
    uint32_t row_off = 0; // first right-hand side of this request in its batch
};

struct Slot {
    float* U = nullptr;    // kMaxRhs x cols
    float* Y = nullptr;    // kMaxRhs x rows
    double* part = nullptr; // slab partials for the graphs
    hipEvent_t done_ev = nullptr;
    hipGraphExec_t exec[kNumBuckets] = {};
    bool busy = false;
    std::vector<uint64_t> batch; // tickets
};

struct MatServe {
    Matrix m{};
    hipStream_t stream = nullptr;
    std::vector<Slot> slots;
    std::deque<uint64_t> pending;
    bool usable = false;
};

} // namespace

struct Server {
    wh_ctx* ctx = nullptr;
    std::mutex mu;
    std::condition_variable cv;
    std::unordered_map<uint64_t, Req> reqs;
    std::map<wh_mat, MatServe> mats;
    uint64_t next_ticket = 1;
    uint64_t arena_used = 0;
    std::thread worker;
    bool stop = false;
    wh_status sticky = WH_OK;
};

namespace {

// The row chunks of one served pass: consecutive ranges of whole block rows
// holding at most `values` matrix values each (at least one block row).
std::vector<std::pair<uint32_t, uint32_t>> serve_chunks(const Matrix& m, uint64_t values)
{
    const uint64_t per = std::max<uint64_t>(4, values / std::max<uint32_t>(1, m.desc.cols) / 4 * 4);
    std::vector<std::pair<uint32_t, uint32_t>> out;
    for (uint64_t r0 = 0; r0 < m.desc.rows; r0 += per)
        out.emplace_back((uint32_t)r0, (uint32_t)std::min<uint64_t>(r0 + per, m.desc.rows));
    return out;
}

// Device memory of one batch slot: U and Y for kMaxRhs vectors, and the FP64
// slab partials the k = 1 or multi-RHS plans of its chunks need (none when
// every plan has one slab; the chunks run in stream order and share them).
// This is what a slot charges against the context's HBM budget.
size_t slot_partials(const Matrix& m, const wh_ctx* ctx)
{
    size_t n = 0;
    for (const auto& c : serve_chunks(m, ctx->serve_chunk_values)) {
        const GemvPlan gp = whz_gemv_plan(m.desc.rows, m.desc.cols, c.first, c.second, ctx->num_cus);
        const MrhsPlan mp = whz_mrhs_plan(m.desc.rows, m.desc.cols, c.first, c.second, ctx->num_cus);
        if (gp.nslab > 1)
            n = std::max(n, (size_t)gp.nslab * gp.part_rows());
        if (mp.nslab > 1)
            n = std::max(n, (size_t)mp.nslab * kMaxRhs * mp.part_rows());
    }
    return n;
}

size_t slot_bytes(const Matrix& m, const wh_ctx* ctx)
{
    return (size_t)kMaxRhs * ((size_t)m.desc.cols + m.desc.rows) * sizeof(float) +
           slot_partials(m, ctx) * sizeof(double);
}

// Capture one graph per k-bucket for a slot: a single fused launch.
wh_status build_slot(Server* sv, MatServe& ms, Slot& sl)
{
    const Matrix& m = ms.m;
    if (hipMalloc(&sl.U, (size_t)kMaxRhs * m.desc.cols * sizeof(float)) != hipSuccess ||
        hipMalloc(&sl.Y, (size_t)kMaxRhs * m.desc.rows * sizeof(float)) != hipSuccess)
        return WH_ERR_NOMEM;
    // the rows the graphs may read before a batch writes them must be finite
    if (hipMemset(sl.U, 0, (size_t)kMaxRhs * m.desc.cols * sizeof(float)) != hipSuccess)
        return WH_ERR_DEVICE;
    const size_t part_n = slot_partials(m, sv->ctx);
    const auto chunks = serve_chunks(m, sv->ctx->serve_chunk_values);
    if (part_n && hipMalloc(&sl.part, part_n * sizeof(double)) != hipSuccess)
        return WH_ERR_NOMEM;
    if (hipEventCreateWithFlags(&sl.done_ev, hipEventDisableTiming) != hipSuccess)
        return WH_ERR_DEVICE;
    for (int b = 0; b < kNumBuckets; ++b) {
        const uint32_t k = kBuckets[b];
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(ms.stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return WH_ERR_DEVICE;
        hipError_t e = hipSuccess;
        for (const auto& c : chunks) {
            if (k == 1) {
                const GemvPlan gp = whz_gemv_plan(m.desc.rows, m.desc.cols, c.first, c.second, sv->ctx->num_cus);
                e = whz_gemv(m.desc.rate, gp, AccMode::Fp64, m.dptr, sl.U, sl.Y + c.first, sl.part, ms.stream);
            } else {
                const MrhsPlan mp = whz_mrhs_plan(m.desc.rows, m.desc.cols, c.first, c.second, sv->ctx->num_cus);
                e = whz_mrhs(m.desc.rate, mp, false, m.dptr, sl.U, m.desc.cols, k, sl.Y + c.first, m.desc.rows,
                             sl.part, ms.stream);
            }
            if (e != hipSuccess)
                break;
        }
        hipError_t e2 = hipStreamEndCapture(ms.stream, &g);
        if (e != hipSuccess || e2 != hipSuccess || !g)
            return WH_ERR_DEVICE;
        e = hipGraphInstantiate(&sl.exec[b], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess)
            return WH_ERR_DEVICE;
    }
    return WH_OK;
}

void free_slot(Slot& sl)
{
    for (int b = 0; b < kNumBuckets; ++b)
        if (sl.exec[b])
            (void)hipGraphExecDestroy(sl.exec[b]);
    if (sl.done_ev)
        (void)hipEventDestroy(sl.done_ev);
    if (sl.U)
        (void)hipFree(sl.U);
    if (sl.Y)
        (void)hipFree(sl.Y);
    if (sl.part)
        (void)hipFree(sl.part);
    sl = Slot{};
}

// Called with sv->mu held (takes ctx->mu).  The first slots still owed to
// the context's resident compressed matrices that have none yet (each one
// that fits the budget on its own).
size_t first_slot_reserve(Server* sv)
{
    size_t r = 0;
    std::lock_guard<std::mutex> lk(sv->ctx->mu);
    for (const auto& kv : sv->ctx->mats) {
        if (kv.second.desc.fmt != WH_FMT_ZFP_FIXED_RATE)
            continue;
        auto it = sv->mats.find(kv.first);
        if (it != sv->mats.end() && !it->second.slots.empty())
            continue;
        const size_t b = slot_bytes(kv.second, sv->ctx);
        if (b <= sv->ctx->budget)
            r += b;
    }
    return r;
}

// Called with sv->mu held.  Adds a slot to a matrix if the budget has room
// for it; the slot's bytes are charged only when it is built.  A second slot
// must leave room for the first slots of the resident matrices that have
// none yet, so a matrix whose first request comes late is not starved.
bool add_slot(Server* sv, MatServe& ms)
{
    const size_t per = slot_bytes(ms.m, sv->ctx);
    const size_t reserve = ms.slots.empty() ? 0 : first_slot_reserve(sv);
    if ((int)ms.slots.size() >= kMaxSlotsPerMatrix || sv->arena_used + per + reserve > sv->ctx->budget)
        return false;
    Slot sl;
    if (build_slot(sv, ms, sl) != WH_OK) {
        free_slot(sl);
        return false;
    }
    sv->arena_used += per;
    ms.slots.push_back(std::move(sl));
    return true;
}

// Called with sv->mu held.  Sets up serving state for a matrix on first use:
// one slot now; a second one later, when a batch of this matrix has to wait
// and the budget has room beyond the first slots owed to the other resident
// matrices.
MatServe* serve_matrix(Server* sv, wh_mat mat, wh_status& st)
{
    auto it = sv->mats.find(mat);
    if (it != sv->mats.end()) {
        st = it->second.usable ? WH_OK : WH_ERR_BUDGET;
        return it->second.usable ? &it->second : nullptr;
    }
    Matrix m;
    {
        std::lock_guard<std::mutex> lk(sv->ctx->mu);
        Matrix* p = find_matrix(sv->ctx, mat);
        if (!p) {
            st = WH_ERR_NOT_FOUND;
            return nullptr;
        }
        m = *p;
    }
    if (m.desc.fmt != WH_FMT_ZFP_FIXED_RATE) {
        st = WH_ERR_FORMAT;
        return nullptr;
    }
    if (slot_bytes(m, sv->ctx) + sv->arena_used > sv->ctx->budget) {
        st = WH_ERR_BUDGET; // cannot hold even one batch of this matrix
        return nullptr;
    }
    MatServe& ms = sv->mats[mat];
    ms.m = m;
    if (hipStreamCreateWithFlags(&ms.stream, hipStreamNonBlocking) != hipSuccess) {
        st = WH_ERR_DEVICE;
        return nullptr;
    }
    if (!add_slot(sv, ms)) {
        st = WH_ERR_NOMEM;
        return nullptr;
    }
    ms.usable = true;
    st = WH_OK;
    return &ms;
}

// Issue one batch on a free slot.  Called with sv->mu held (the HIP calls
// below are asynchronous and short).
wh_status launch_batch(Server* sv, MatServe& ms, Slot& sl)
{
    const Matrix& m = ms.m;
    uint32_t ktot = 0;
    sl.batch.clear();
    while (!ms.pending.empty()) {
        Req& r = sv->reqs[ms.pending.front()];
        if (ktot + r.r.k > kMaxRhs)
            break;
        r.row_off = ktot;
        ktot += r.r.k;
        sl.batch.push_back(ms.pending.front());
        ms.pending.pop_front();
    }
    if (sl.batch.empty())
        return WH_OK;
    const int b = bucket_index(ktot);
    const uint64_t t0 = now_ns();
    const size_t cols = m.desc.cols, rows = m.desc.rows;
    for (uint64_t t : sl.batch) {
        Req& r = sv->reqs[t];
        r.t_start = t0;
        r.batch_size = (uint32_t)sl.batch.size();
        const hipMemcpyKind kind = r.r.u_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        if (hipMemcpyAsync(sl.U + (size_t)r.row_off * cols, r.r.U, (size_t)r.r.k * cols * sizeof(float), kind,
                           ms.stream) != hipSuccess)
            return WH_ERR_DEVICE;
    }
    if (hipGraphLaunch(sl.exec[b], ms.stream) != hipSuccess)
        return WH_ERR_DEVICE;
    for (uint64_t t : sl.batch) {
        Req& r = sv->reqs[t];
        const hipMemcpyKind kind = r.r.y_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        if (hipMemcpyAsync(r.r.Y, sl.Y + (size_t)r.row_off * rows, (size_t)r.r.k * rows * sizeof(float), kind,
                           ms.stream) != hipSuccess)
            return WH_ERR_DEVICE;
    }
    if (hipEventRecord(sl.done_ev, ms.stream) != hipSuccess)
        return WH_ERR_DEVICE;
    sl.busy = true;
    return WH_OK;
}

void fail_all(Server* sv, wh_status st)
{
    sv->sticky = st;
    for (auto& kv : sv->reqs)
        if (kv.second.status == WH_PENDING)
            kv.second.status = st;
    for (auto& mv : sv->mats)
        mv.second.pending.clear();
}

void worker_main(Server* sv)
{
    (void)hipSetDevice(sv->ctx->device);
    std::unique_lock<std::mutex> lk(sv->mu);
    while (!sv->stop) {
        bool busy_any = false;
        // completion
        for (auto& mv : sv->mats) {
            for (Slot& sl : mv.second.slots) {
                if (!sl.busy)
                    continue;
                hipError_t q = hipEventQuery(sl.done_ev);
                if (q == hipErrorNotReady) {
                    busy_any = true;
                    continue;
                }
                const uint64_t t = now_ns();
                const wh_status st = q == hipSuccess ? WH_OK : WH_ERR_DEVICE;
                for (uint64_t tk : sl.batch) {
                    Req& r = sv->reqs[tk];
                    r.t_done = t;
                    r.status = st;
                }
                sl.batch.clear();
                sl.busy = false;
                if (st != WH_OK) {
                    sv->ctx->failed.store(true);
                    fail_all(sv, st);
                }
            }
        }
        // dispatch: every free slot of a matrix with queued requests
        if (sv->sticky == WH_OK) {
            for (auto& mv : sv->mats) {
                MatServe& ms = mv.second;
                bool all_busy = true;
                for (Slot& sl : ms.slots) {
                    if (ms.pending.empty())
                        break;
                    if (sl.busy)
                        continue;
                    all_busy = false;
                    const wh_status st = launch_batch(sv, ms, sl);
                    if (st != WH_OK) {
                        sv->ctx->failed.store(true);
                        fail_all(sv, st);
                        break;
                    }
                    busy_any = true;
                }
                // a batch is waiting on a busy matrix: add a slot if the
                // budget allows, and use it at once
                if (sv->sticky == WH_OK && all_busy && !ms.pending.empty() && add_slot(sv, ms)) {
                    const wh_status st = launch_batch(sv, ms, ms.slots.back());
                    if (st != WH_OK) {
                        sv->ctx->failed.store(true);
                        fail_all(sv, st);
                    }
                    busy_any = true;
                }
            }
        }
        // sleep briefly while batches run; block while idle
        if (busy_any)
            sv->cv.wait_for(lk, std::chrono::microseconds(20));
        else
            sv->cv.wait_for(lk, std::chrono::milliseconds(5));
    }
}

Server* ensure_server(wh_ctx* ctx)
{
    static std::mutex create_mu;
    std::lock_guard<std::mutex> g(create_mu);
    if (!ctx->server) {
        Server* sv = new Server();
        sv->ctx = ctx;
        sv->worker = std::thread(worker_main, sv);
        ctx->server = sv;
    }
    return ctx->server;
}

} // namespace

void serve_shutdown(wh_ctx* ctx)
{
    Server* sv = ctx->server;
    if (!sv)
        return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv.notify_all();
    if (sv->worker.joinable())
        sv->worker.join();
    for (auto& mv : sv->mats) {
        MatServe& ms = mv.second;
        if (ms.stream)
            (void)hipStreamSynchronize(ms.stream);
        for (Slot& sl : ms.slots)
            free_slot(sl);
        if (ms.stream)
            (void)hipStreamDestroy(ms.stream);
    }
    delete sv;
    ctx->server = nullptr;
}

void serve_forget(wh_ctx* ctx, wh_mat m)
{
    Server* sv = ctx->server;
    if (!sv)
        return;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->mats.find(m);
    if (it == sv->mats.end())
        return;
    MatServe& ms = it->second;
    if (ms.stream)
        (void)hipStreamSynchronize(ms.stream); // batches in flight finish
    for (Slot& sl : ms.slots) {
        for (uint64_t tk : sl.batch) { // finished on the device: deliver
            Req& r = sv->reqs[tk];
            r.t_done = now_ns();
            r.status = WH_OK;
        }
        sv->arena_used -= slot_bytes(ms.m, ctx);
        free_slot(sl);
    }
    for (uint64_t tk : ms.pending) // never started
        sv->reqs[tk].status = WH_ERR_NOT_FOUND;
    if (ms.stream)
        (void)hipStreamDestroy(ms.stream);
    sv->mats.erase(it);
}

} // namespace wh

extern "C" wh_status wh_submit(wh_ctx* ctx, const wh_request* req, uint64_t* ticket)
{
    using namespace wh;
    if (!ctx || !req || !ticket)
        return WH_ERR_INVALID;
    if (ctx->failed.load())
        return WH_ERR_DEVICE;
    if (!req->U || !req->Y || req->k == 0)
        return WH_ERR_INVALID;
    if (req->k > kMaxRhs)
        return WH_ERR_BUDGET; // larger than any batch slot
    try {
        const uint64_t t = req->arrival_ns ? req->arrival_ns : now_ns();
        Server* sv = ensure_server(ctx);
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->sticky != WH_OK)
            return sv->sticky;
        if (hipSetDevice(ctx->device) != hipSuccess)
            return WH_ERR_DEVICE;
        wh_status st = WH_OK;
        MatServe* ms = serve_matrix(sv, req->mat, st);
        if (!ms)
            return st;
        // load shedding (off unless WH_SERVE_SHED is set): the matrix's oldest
        // queued request has already waited longer than `serve_shed` of its
        // deadlines, so a new one would wait longer still
        if (ctx->serve_shed && !ms->pending.empty()) {
            const Req& head = sv->reqs[ms->pending.front()];
            const uint64_t now = now_ns();
            if (head.r.deadline_ns && now > head.t_arrive &&
                now - head.t_arrive > (uint64_t)ctx->serve_shed * head.r.deadline_ns)
                return WH_ERR_BUDGET;
        }
        const uint64_t tk = sv->next_ticket++;
        Req& r = sv->reqs[tk];
        r.r = *req;
        r.t_arrive = t;
        ms->pending.push_back(tk);
        *ticket = tk;
        sv->cv.notify_one();
        return WH_OK;
    } catch (const std::bad_alloc&) {
        return WH_ERR_NOMEM;
    } catch (...) {
        return WH_ERR_INVALID;
    }
}

extern "C" wh_status wh_poll(wh_ctx* ctx, uint64_t ticket, wh_result* out)
{
    using namespace wh;
    if (!ctx || !out)
        return WH_ERR_INVALID;
    Server* sv = ctx->server;
    if (!sv)
        return WH_ERR_NOT_FOUND;
    try {
        std::lock_guard<std::mutex> lk(sv->mu);
        auto it = sv->reqs.find(ticket);
        if (it == sv->reqs.end())
            return WH_ERR_NOT_FOUND;
        const Req& r = it->second;
        if (r.status == WH_PENDING)
            return WH_PENDING;
        out->status = r.status;
        out->t_arrive_ns = r.t_arrive;
        out->t_start_ns = r.t_start;
        out->t_done_ns = r.t_done;
        out->missed = r.t_done > r.t_arrive + r.r.deadline_ns ? 1 : 0;
        out->batch_size = r.batch_size;
        const wh_status st = r.status;
        sv->reqs.erase(it);
        return st == WH_OK ? WH_OK : st;
    } catch (...) {
        return WH_ERR_INVALID;
    }
}

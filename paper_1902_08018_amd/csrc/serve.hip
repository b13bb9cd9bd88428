// serve.hip -- the real-time request loop (wh_submit / wh_poll).
//
// The paper's loop evaluates the deformation product every light-stage
// millisecond against resident field matrices, under a firm deadline: a late
// result is still delivered but counts as a miss (Sec. 1, Sec. 2.1, Fig. 2).
// Here many such dose-vector requests, against several resident matrices of
// different sizes, share one GPU:
//
//   submit      any thread; the request is validated (host buffers must be
//               page-locked), stamped and queued.  The first request for a
//               matrix sets up its slot outside the loop's lock
//   slot        per matrix, carved out of the context's HBM budget: U, Y and
//               a staging copy of Y for 64 right-hand-side columns, the FP64
//               slab partials of its plans, and one pre-instantiated hipGraph
//               per (row chunk, k-bucket 1, 2, 4, ..., 64).  A request that
//               can never fit is rejected at submit
//   cyclic scan each matrix's rows are split into chunks of at most
//               ctx->serve_chunk_values values.  The loop launches one chunk
//               at a time, cycling through them, over every column held by a
//               request.  A queued request joins at the next chunk launch: its
//               U is copied into free columns, and it is complete once the
//               scan has gone round once from there.  So a request waits at
//               most one chunk for the pass it joins, not for a whole pass to
//               end, and requests that arrive while others run share the same
//               launches
//   holding     while another matrix's scan is running late (its requests
//               cannot meet their deadlines any more), a matrix with no scan
//               under way holds its queued requests back as long as the most
//               urgent can still wait (its pass, the launches that may be
//               ahead of it and between its chunks, and a margin before the
//               deadline), so that more requests share each of its passes
//   order       every launch goes to one stream of the loop's, at most two in
//               flight, so each runs alone on the device: the loop, not the
//               hardware, decides how the device is shared, and a launch's
//               measured time is what the next one of its chunk and bucket
//               will take.  Requests that can still meet their deadlines go
//               by the latest time their next chunk may start (the earliest
//               first).  A scan running late is paced at one chunk per
//               ctx->serve_pace of its chunk times while that work waits,
//               and takes what is left over
//   copies      vectors in and results out travel on two copy streams, so
//               the transfers overlap the launches: a launch waits only for
//               the copies of the requests that join at it, and results bound
//               for host memory are staged on the device and copied out after
//   completion  the worker polls each launch's events; the requests whose
//               last chunk it was are stamped done once their results are out
//   poll        never blocks: WH_PENDING, or the result once (then retired)
//
// The decisions (columns, chunks, holding, order, pacing, a launch's
// bookkeeping) are serve_policy.hpp's, which makes no device calls; this file
// runs them with HIP.  A matrix's slab partials are shared by its chunks in
// launch order.  Every stream keeps the default priority.
#include <hip/hip_runtime.h>

#include <sys/prctl.h>
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

#include "serve_policy.hpp"
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

using policy::kBuckets;
using policy::kMaxInflight;
using policy::kNumBuckets;
// event sets per matrix: launches whose results are still being copied out
// keep theirs a little longer
constexpr size_t kEventSets = kMaxInflight + 4;
static_assert(kMaxRhs == policy::kSlotCols, "a slot's columns are the bits of a uint64_t");

struct Req {
    wh_request r;
    policy::ReqState ps; // arrival, deadline, k; in the scan: its columns (vector i in the i-th) and chunks left
    uint64_t t_done = 0;
    wh_status status = WH_PENDING;
};

// The events of one chunk launch: t0 and t1 around its graph and the copies
// of its results to the slot's staging columns (launch stream), ty after the
// copies of those results to host memory (copy-out stream), tu after the
// copies in of the requests that joined (copy-in stream).
struct LaunchEvents {
    hipEvent_t t0 = nullptr, t1 = nullptr, ty = nullptr, tu = nullptr;
};

struct Launch {
    LaunchEvents ev;
    bool computed = false;      // t1 has been seen
    bool to_host = false;       // ty was recorded
    uint64_t free = 0;          // columns of the requests it completes, freed when it does
    std::vector<uint64_t> done; // requests whose last chunk this launch is
};

struct MatServe {
    Matrix m{};
    std::vector<std::pair<uint32_t, uint32_t>> chunks;
    float* U = nullptr;      // kMaxRhs x cols
    float* Y = nullptr;      // kMaxRhs x rows
    float* S = nullptr;      // kMaxRhs x rows: results staged for their copy to host
    double* part = nullptr;  // slab partials of the chunk plans
    std::vector<hipGraphExec_t> exec; // [chunk * kNumBuckets + bucket]
    std::vector<LaunchEvents> spare; // event sets not in use
    std::deque<Launch> inflight;
    policy::ScanState st;         // queue, scan, held columns, chunk times, pace
    size_t bytes = 0;             // charged to the budget
    bool building = false, usable = false;
    wh_status build_status = WH_OK;
};

} // namespace

struct Server {
    wh_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;   // every launch of the loop
    hipStream_t copy_in = nullptr;  // requests' vectors into their columns
    hipStream_t copy_out = nullptr; // staged results to host memory
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

// The row chunks of one served pass (policy::chunk_rows).
std::vector<std::pair<uint32_t, uint32_t>> serve_chunks(const Matrix& m, uint64_t values)
{
    return policy::chunk_rows(m.desc.rows, m.desc.cols, values);
}

// Workspace (doubles) the k = 1 or multi-RHS plans of the chunks need: FP64
// slab partials, and B^T U for the multi-RHS kernel (the chunks run in
// stream order and share it).
size_t slot_partials(const Matrix& m, const wh_ctx* ctx)
{
    size_t n = 0;
    for (const auto& c : serve_chunks(m, ctx->serve_chunk_values)) {
        const GemvPlan gp = whz_gemv_plan(m.desc.rate, m.desc.rows, m.desc.cols, c.first, c.second, ctx->num_cus);
        if (gp.nslab > 1)
            n = std::max(n, (size_t)gp.nslab * gp.part_rows());
        for (uint32_t k = 16; k <= kMaxRhs; k += 16) { // the plan and workspace depend on k
            const MrhsPlan mp = whz_mrhs_plan(m.desc.rows, m.desc.cols, c.first, c.second, ctx->num_cus, k, false,
                                              &ctx->gemv_tune);
            n = std::max(n, mrhs_workspace(mp, k).total);
        }
    }
    return n;
}

// What a matrix's slot charges against the context's HBM budget.
size_t slot_bytes(const Matrix& m, const wh_ctx* ctx)
{
    return (size_t)kMaxRhs * ((size_t)m.desc.cols + 2 * (size_t)m.desc.rows) * sizeof(float) +
           slot_partials(m, ctx) * sizeof(double);
}

// A chunk launch's time before any is measured: about a microsecond per
// million matrix values (the fused decoder's rate on a full device).
double model_chunk_ms(const Matrix& m, const std::pair<uint32_t, uint32_t>& c)
{
    return 1e-9 * (double)(c.second - c.first) * (double)m.desc.cols;
}

void free_slot(MatServe& ms)
{
    for (hipGraphExec_t g : ms.exec)
        if (g)
            (void)hipGraphExecDestroy(g);
    ms.exec.clear();
    auto destroy = [](LaunchEvents& e) {
        for (hipEvent_t x : {e.t0, e.t1, e.ty, e.tu})
            if (x)
                (void)hipEventDestroy(x);
        e = LaunchEvents{};
    };
    for (auto& e : ms.spare)
        destroy(e);
    ms.spare.clear();
    for (Launch& l : ms.inflight)
        destroy(l.ev);
    ms.inflight.clear();
    if (ms.U)
        (void)hipFree(ms.U);
    if (ms.Y)
        (void)hipFree(ms.Y);
    if (ms.S)
        (void)hipFree(ms.S);
    if (ms.part)
        (void)hipFree(ms.part);
    ms.U = ms.Y = ms.S = nullptr;
    ms.part = nullptr;
}

// Device memory, events and graphs of a matrix's slot (captured on a stream
// of its own, then launched on the loop's).  Runs without the server lock
// (the worker does not touch a slot being built).
wh_status build_slot(wh_ctx* ctx, MatServe& ms)
{
    struct CaptureStream {
        hipStream_t s = nullptr;
        ~CaptureStream()
        {
            if (s)
                (void)hipStreamDestroy(s);
        }
    } cap;
    const Matrix& m = ms.m;
    if (hipStreamCreateWithFlags(&cap.s, hipStreamNonBlocking) != hipSuccess)
        return WH_ERR_DEVICE;
    hipStream_t st = cap.s;
    if (hipMalloc(&ms.U, (size_t)kMaxRhs * m.desc.cols * sizeof(float)) != hipSuccess ||
        hipMalloc(&ms.Y, (size_t)kMaxRhs * m.desc.rows * sizeof(float)) != hipSuccess ||
        hipMalloc(&ms.S, (size_t)kMaxRhs * m.desc.rows * sizeof(float)) != hipSuccess)
        return WH_ERR_NOMEM;
    // columns the graphs read before a request writes them must be finite
    if (hipMemset(ms.U, 0, (size_t)kMaxRhs * m.desc.cols * sizeof(float)) != hipSuccess)
        return WH_ERR_DEVICE;
    const size_t part_n = slot_partials(m, ctx);
    if (part_n && hipMalloc(&ms.part, part_n * sizeof(double)) != hipSuccess)
        return WH_ERR_NOMEM;
    ms.chunks = serve_chunks(m, ctx->serve_chunk_values);
    for (size_t i = 0; i < kEventSets; ++i) {
        ms.spare.emplace_back();
        LaunchEvents& e = ms.spare.back();
        if (hipEventCreate(&e.t0) != hipSuccess || hipEventCreate(&e.t1) != hipSuccess ||
            hipEventCreateWithFlags(&e.ty, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&e.tu, hipEventDisableTiming) != hipSuccess)
            return WH_ERR_DEVICE;
    }
    ms.exec.assign(ms.chunks.size() * kNumBuckets, nullptr);
    double model = 0.0;
    for (size_t ci = 0; ci < ms.chunks.size(); ++ci) {
        const auto& c = ms.chunks[ci];
        model = std::max(model, model_chunk_ms(m, c));
        for (int b = 0; b < kNumBuckets; ++b) {
            const uint32_t k = kBuckets[b];
            hipGraph_t g = nullptr;
            if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
                return WH_ERR_DEVICE;
            hipError_t e;
            if (k == 1) {
                const GemvPlan gp = whz_gemv_plan(m.desc.rate, m.desc.rows, m.desc.cols, c.first, c.second, ctx->num_cus);
                e = whz_gemv(m.desc.rate, gp, AccMode::Fp64, m.dptr, ms.U, ms.Y + c.first, ms.part, st);
            } else {
                const MrhsPlan mp = whz_mrhs_plan(m.desc.rows, m.desc.cols, c.first, c.second, ctx->num_cus, k, false,
                                                  &ctx->gemv_tune);
                e = whz_mrhs(m.desc.rate, mp, m.dptr, ms.U, m.desc.cols, k, ms.Y + c.first, m.desc.rows,
                             ms.part, st);
            }
            const hipError_t e2 = hipStreamEndCapture(st, &g);
            if (e != hipSuccess || e2 != hipSuccess || !g)
                return WH_ERR_DEVICE;
            e = hipGraphInstantiate(&ms.exec[ci * kNumBuckets + b], g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess || hipGraphUpload(ms.exec[ci * kNumBuckets + b], st) != hipSuccess)
                return WH_ERR_DEVICE;
        }
    }
    // every bucket's graph runs once here (over the zeroed columns), so that
    // the first launch of each in the loop does not set anything up
    for (int b = 0; b < kNumBuckets; ++b)
        for (size_t ci = 0; ci < ms.chunks.size(); ++ci)
            if (hipGraphLaunch(ms.exec[ci * kNumBuckets + b], st) != hipSuccess)
                return WH_ERR_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess)
        return WH_ERR_DEVICE;
    ms.st.nchunks = (uint32_t)ms.chunks.size();
    ms.st.chunk_ms = ms.st.chunk_ms_max = model;
    return WH_OK;
}

// Copies between a request's k contiguous vectors of n floats at `req` and
// its columns of a slot buffer (column c at slot + c * n), one copy per run of
// consecutive columns.  to_slot: request -> slot.
hipError_t copy_cols(float* slot, const float* req_src, float* req_dst, uint64_t mask, size_t n, bool to_slot,
                     hipMemcpyKind kind, hipStream_t st)
{
    size_t i = 0; // vectors of the request done
    while (mask) {
        const uint32_t c0 = (uint32_t)__builtin_ctzll(mask);
        const uint64_t from = mask >> c0;
        const uint32_t len = ~from ? (uint32_t)__builtin_ctzll(~from) : 64u - c0;
        const size_t bytes = (size_t)len * n * sizeof(float);
        const hipError_t e = to_slot ? hipMemcpyAsync(slot + (size_t)c0 * n, req_src + i * n, bytes, kind, st)
                                     : hipMemcpyAsync(req_dst + i * n, slot + (size_t)c0 * n, bytes, kind, st);
        if (e != hipSuccess)
            return e;
        i += len;
        mask &= len >= 64 ? 0ull : ~(((1ull << len) - 1) << c0);
    }
    return hipSuccess;
}

// The columns `mask` of one slot buffer copied to the same columns of another.
hipError_t stage_cols(float* dst, const float* src, uint64_t mask, size_t n, hipStream_t st)
{
    while (mask) {
        const uint32_t c0 = (uint32_t)__builtin_ctzll(mask);
        const uint64_t from = mask >> c0;
        const uint32_t len = ~from ? (uint32_t)__builtin_ctzll(~from) : 64u - c0;
        const hipError_t e = hipMemcpyAsync(dst + (size_t)c0 * n, src + (size_t)c0 * n,
                                            (size_t)len * n * sizeof(float), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess)
            return e;
        mask &= len >= 64 ? 0ull : ~(((1ull << len) - 1) << c0);
    }
    return hipSuccess;
}

// Called with sv->mu held.  Issues the next chunk launch of a matrix: queued
// requests join (FIFO, while columns last) and their vectors are copied into
// their columns on the copy-in stream, which the launch waits for; the
// chunk's graph runs over every held column; the results of the requests
// whose last chunk this was are copied to their device buffers, or staged and
// then copied to host memory on the copy-out stream, so that neither kind of
// host copy holds up the launches.  A column is freed only once the launch
// that completes its request has finished, results copied, so a request that
// takes it over writes its vectors over nothing a launch still needs.  The
// launches issued meanwhile compute the freed column with whatever it holds,
// and the new request's own pass, which begins after its copy in, rewrites
// every row of it.  The HIP calls are asynchronous: copies from and to
// page-locked or device memory only.
wh_status issue_chunk(Server* sv, MatServe& ms)
{
    const Matrix& m = ms.m;
    const size_t cols = m.desc.cols, rows = m.desc.rows;
    const policy::LaunchPlan p =
        policy::plan_launch(ms.st, [sv](uint64_t t) -> policy::ReqState& { return sv->reqs.at(t).ps; }, now_ns());
    for (uint64_t t : p.joined) {
        const Req& r = sv->reqs.at(t);
        const hipMemcpyKind kind = r.r.u_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        if (copy_cols(ms.U, r.r.U, nullptr, r.ps.cols, cols, true, kind, sv->copy_in) != hipSuccess)
            return WH_ERR_DEVICE;
    }
    if (!p.launch)
        return WH_OK;
    Launch l;
    l.ev = ms.spare.back();
    ms.spare.pop_back();
    if (!p.joined.empty() && (hipEventRecord(l.ev.tu, sv->copy_in) != hipSuccess ||
                              hipStreamWaitEvent(sv->stream, l.ev.tu, 0) != hipSuccess))
        return WH_ERR_DEVICE;
    if (hipEventRecord(l.ev.t0, sv->stream) != hipSuccess ||
        hipGraphLaunch(ms.exec[(size_t)p.chunk * kNumBuckets + p.bucket], sv->stream) != hipSuccess)
        return WH_ERR_DEVICE;
    std::vector<const Req*> to_host;
    for (uint64_t t : p.done) {
        const Req& r = sv->reqs.at(t);
        const hipError_t e = r.r.y_on_device
                                 ? copy_cols(ms.Y, nullptr, r.r.Y, r.ps.cols, rows, false, hipMemcpyDeviceToDevice,
                                             sv->stream)
                                 : stage_cols(ms.S, ms.Y, r.ps.cols, rows, sv->stream);
        if (e != hipSuccess)
            return WH_ERR_DEVICE;
        if (!r.r.y_on_device)
            to_host.push_back(&r);
    }
    l.free = p.free;
    l.done = p.done;
    if (hipEventRecord(l.ev.t1, sv->stream) != hipSuccess)
        return WH_ERR_DEVICE;
    if (!to_host.empty()) {
        if (hipStreamWaitEvent(sv->copy_out, l.ev.t1, 0) != hipSuccess)
            return WH_ERR_DEVICE;
        for (const Req* r : to_host)
            if (copy_cols(ms.S, nullptr, r->r.Y, r->ps.cols, rows, false, hipMemcpyDeviceToHost, sv->copy_out) !=
                hipSuccess)
                return WH_ERR_DEVICE;
        if (hipEventRecord(l.ev.ty, sv->copy_out) != hipSuccess)
            return WH_ERR_DEVICE;
        l.to_host = true;
    }
    ms.inflight.push_back(std::move(l));
    return WH_OK;
}

void fail_all(Server* sv, wh_status st)
{
    sv->sticky = st;
    for (auto& kv : sv->reqs)
        if (kv.second.status == WH_PENDING)
            kv.second.status = st;
    for (auto& mv : sv->mats) {
        mv.second.st.pending.clear();
        mv.second.st.active.clear();
    }
}

void worker_main(Server* sv)
{
    (void)hipSetDevice(sv->ctx->device);
    // the loop's short sleeps (20 us while launches run, until a hold ends)
    // should end when due: the default 50 us timer slack would let them run
    // on, so this thread asks for 1 us
    (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
    std::unique_lock<std::mutex> lk(sv->mu);
    while (!sv->stop) {
        // completion, in launch order per matrix: a launch's compute (t1),
        // then the copies of its results to host memory (ty)
        size_t inflight = 0; // launches whose compute has not ended
        wh_status failed = WH_OK;
        for (auto& mv : sv->mats) {
            MatServe& ms = mv.second;
            for (Launch& l : ms.inflight) {
                if (l.computed)
                    continue;
                const hipError_t q = hipEventQuery(l.ev.t1);
                if (q == hipErrorNotReady) {
                    ++inflight;
                    continue;
                }
                if (q != hipSuccess) {
                    failed = WH_ERR_DEVICE;
                    break;
                }
                l.computed = true;
                float ms_el = 0.f;
                if (hipEventElapsedTime(&ms_el, l.ev.t0, l.ev.t1) == hipSuccess && ms_el > 0.f)
                    policy::observe_chunk(ms.st, (double)ms_el);
            }
            while (failed == WH_OK && !ms.inflight.empty() && ms.inflight.front().computed) {
                Launch& l = ms.inflight.front();
                if (l.to_host) {
                    const hipError_t q = hipEventQuery(l.ev.ty);
                    if (q == hipErrorNotReady)
                        break;
                    if (q != hipSuccess) {
                        failed = WH_ERR_DEVICE;
                        break;
                    }
                }
                const uint64_t t = now_ns();
                for (uint64_t tk : l.done) {
                    Req& r = sv->reqs[tk];
                    r.t_done = t;
                    r.status = WH_OK;
                }
                policy::release(ms.st, l.free);
                ms.spare.push_back(l.ev);
                ms.inflight.pop_front();
            }
            if (failed != WH_OK)
                break;
        }
        if (failed != WH_OK) {
            sv->ctx->failed.store(true);
            fail_all(sv, failed);
            for (auto& mv : sv->mats) { // nothing more is launched: take back their events
                for (Launch& l : mv.second.inflight)
                    mv.second.spare.push_back(l.ev);
                mv.second.inflight.clear();
            }
            inflight = 0;
        }
        // dispatch (policy::pick): the earliest latest start among requests
        // that can still meet their deadlines, and the paced chunks of late
        // scans between them; kMaxInflight launches in flight at most
        uint64_t wake = UINT64_MAX; // the earliest end of a hold
        const policy::Tuning tune{sv->ctx->serve_pace, sv->ctx->serve_margin_ns};
        auto get = [sv](uint64_t t) -> const policy::ReqState& { return sv->reqs.at(t).ps; };
        while (sv->sticky == WH_OK && inflight < kMaxInflight) {
            std::vector<policy::ScanState*> scans;
            std::vector<MatServe*> owners;
            for (auto& mv : sv->mats) {
                MatServe& ms = mv.second;
                ms.st.usable = ms.usable;
                ms.st.can_launch = ms.usable && !ms.spare.empty();
                scans.push_back(&ms.st);
                owners.push_back(&ms);
            }
            const int i = policy::pick(scans, get, now_ns(), tune, wake);
            if (i < 0)
                break;
            MatServe* pick = owners[(size_t)i];
            const wh_status st = issue_chunk(sv, *pick);
            if (st != WH_OK) {
                sv->ctx->failed.store(true);
                fail_all(sv, st);
                break;
            }
            ++inflight;
        }
        // sleep briefly while launches or copies run or a hold is about to
        // end; block while idle
        const uint64_t now = now_ns();
        const bool busy = std::any_of(sv->mats.begin(), sv->mats.end(),
                                      [](const std::pair<const wh_mat, MatServe>& mv) {
                                          return !mv.second.inflight.empty();
                                      });
        if (busy || wake <= now + 20000)
            sv->cv.wait_for(lk, std::chrono::microseconds(20));
        else if (wake != UINT64_MAX)
            sv->cv.wait_for(lk, std::chrono::nanoseconds(std::min<uint64_t>(wake - now, 5000000)));
        else
            sv->cv.wait_for(lk, std::chrono::milliseconds(5));
    }
}

// Every launch and copy the loop has issued ends.
void sync_streams(Server* sv)
{
    for (hipStream_t s : {sv->stream, sv->copy_in, sv->copy_out})
        if (s)
            (void)hipStreamSynchronize(s);
}

// The context's serving state, created with its streams and worker on first
// use (nullptr if the stream cannot be created).
Server* ensure_server(wh_ctx* ctx)
{
    static std::mutex create_mu;
    std::lock_guard<std::mutex> g(create_mu);
    if (!ctx->server) {
        hipStream_t st[3] = {nullptr, nullptr, nullptr};
        for (hipStream_t& s : st)
            if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
                for (hipStream_t x : st)
                    if (x)
                        (void)hipStreamDestroy(x);
                return nullptr;
            }
        Server* sv = new Server();
        sv->ctx = ctx;
        sv->stream = st[0];
        sv->copy_in = st[1];
        sv->copy_out = st[2];
        sv->worker = std::thread(worker_main, sv);
        ctx->server = sv;
    }
    return ctx->server;
}

// Host memory given to the loop must be page-locked: its copies are then
// asynchronous, so the loop never waits on one.  Device memory is checked to
// be on the context's device.
bool buffer_ok(const void* p, int on_device, int device)
{
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError(); // pageable host memory: unknown to HIP
        return false;
    }
    if (on_device)
        return a.type == hipMemoryTypeDevice && a.device == device;
    return a.type == hipMemoryTypeHost;
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
    sync_streams(sv);
    for (auto& mv : sv->mats)
        free_slot(mv.second);
    for (hipStream_t s : {sv->stream, sv->copy_in, sv->copy_out})
        if (s)
            (void)hipStreamDestroy(s);
    delete sv;
    ctx->server = nullptr;
}

void serve_forget(wh_ctx* ctx, wh_mat m)
{
    Server* sv = ctx->server;
    if (!sv)
        return;
    std::unique_lock<std::mutex> lk(sv->mu);
    // a slot still being built is finished first (its builder holds no lock)
    sv->cv.wait(lk, [&] {
        auto it = sv->mats.find(m);
        return it == sv->mats.end() || !it->second.building;
    });
    auto it = sv->mats.find(m);
    if (it == sv->mats.end())
        return;
    MatServe& ms = it->second;
    sync_streams(sv); // launches in flight and their copies finish
    for (Launch& l : ms.inflight)
        for (uint64_t tk : l.done) { // their last chunk ran: deliver
            Req& r = sv->reqs[tk];
            r.t_done = now_ns();
            r.status = WH_OK;
        }
    for (uint64_t tk : ms.st.active) // part of the way round the scan
        sv->reqs[tk].status = WH_ERR_NOT_FOUND;
    for (uint64_t tk : ms.st.pending) // never started
        sv->reqs[tk].status = WH_ERR_NOT_FOUND;
    if (ms.usable)
        sv->arena_used -= ms.bytes;
    free_slot(ms);
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
        return WH_ERR_BUDGET; // larger than a slot
    try {
        const uint64_t t = req->arrival_ns ? req->arrival_ns : now_ns();
        if (hipSetDevice(ctx->device) != hipSuccess)
            return WH_ERR_DEVICE;
        if (!buffer_ok(req->U, req->u_on_device, ctx->device) || !buffer_ok(req->Y, req->y_on_device, ctx->device))
            return WH_ERR_INVALID;
        Server* sv = ensure_server(ctx);
        if (!sv)
            return WH_ERR_DEVICE;
        std::unique_lock<std::mutex> lk(sv->mu);
        if (sv->sticky != WH_OK)
            return sv->sticky;
        auto it = sv->mats.find(req->mat);
        if (it == sv->mats.end()) {
            // first request for this matrix: admit its slot, build it unlocked
            Matrix m;
            {
                std::lock_guard<std::mutex> lk2(ctx->mu);
                Matrix* p = find_matrix(ctx, req->mat);
                if (!p)
                    return WH_ERR_NOT_FOUND;
                m = *p;
            }
            if (m.desc.fmt != WH_FMT_ZFP_FIXED_RATE)
                return WH_ERR_FORMAT;
            const size_t bytes = slot_bytes(m, ctx);
            if (bytes + sv->arena_used > ctx->budget)
                return WH_ERR_BUDGET; // cannot hold even one slot of this matrix
            sv->arena_used += bytes;
            MatServe& ms = sv->mats[req->mat];
            ms.m = m;
            ms.bytes = bytes;
            ms.building = true;
            lk.unlock();
            MatServe tmp;
            tmp.m = m;
            wh_status bst = build_slot(ctx, tmp);
            lk.lock();
            MatServe& ms2 = sv->mats[req->mat];
            if (bst == WH_OK) {
                ms2.chunks = std::move(tmp.chunks);
                ms2.U = tmp.U;
                ms2.Y = tmp.Y;
                ms2.S = tmp.S;
                ms2.part = tmp.part;
                ms2.exec = std::move(tmp.exec);
                ms2.spare = std::move(tmp.spare);
                ms2.st.nchunks = tmp.st.nchunks;
                ms2.st.chunk_ms = tmp.st.chunk_ms;
                ms2.st.chunk_ms_max = tmp.st.chunk_ms_max;
                ms2.usable = true;
            } else {
                free_slot(tmp);
                ms2.build_status = bst;
                sv->arena_used -= ms2.bytes;
                for (uint64_t tk : ms2.st.pending) // requests queued meanwhile
                    sv->reqs[tk].status = bst;
                ms2.st.pending.clear();
            }
            ms2.building = false;
            sv->cv.notify_all();
            if (bst != WH_OK) {
                sv->mats.erase(req->mat);
                return bst;
            }
            it = sv->mats.find(req->mat);
        }
        MatServe& ms = it->second;
        if (!ms.usable && !ms.building)
            return ms.build_status != WH_OK ? ms.build_status : WH_ERR_BUDGET;
        // load shedding (off unless WH_SERVE_SHED is set): the matrix's oldest
        // queued request has already waited longer than `serve_shed` of its
        // deadlines, so a new one would wait longer still
        if (ctx->serve_shed && !ms.st.pending.empty()) {
            const Req& head = sv->reqs[ms.st.pending.front()];
            const uint64_t now = now_ns();
            if (head.r.deadline_ns && now > head.ps.t_arrive &&
                now - head.ps.t_arrive > (uint64_t)ctx->serve_shed * head.r.deadline_ns)
                return WH_ERR_BUDGET;
        }
        const uint64_t tk = sv->next_ticket++;
        Req& r = sv->reqs[tk];
        r.r = *req;
        r.ps.t_arrive = t;
        r.ps.deadline_ns = req->deadline_ns;
        r.ps.k = req->k;
        ms.st.pending.push_back(tk);
        *ticket = tk;
        sv->cv.notify_all();
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
        out->t_arrive_ns = r.ps.t_arrive;
        out->t_start_ns = r.ps.t_start;
        out->t_done_ns = r.t_done;
        out->missed = r.t_done > r.ps.t_arrive + r.r.deadline_ns ? 1 : 0;
        out->batch_size = r.ps.batch_size;
        const wh_status st = r.status;
        sv->reqs.erase(it);
        return st == WH_OK ? WH_OK : st;
    } catch (...) {
        return WH_ERR_INVALID;
    }
}

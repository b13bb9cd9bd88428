// serve_policy.hpp -- the serving loop's decisions, with no device calls:
// which columns a joining request takes, how a matrix's rows are cut into
// chunk launches, how long a matrix holds its queued requests, which
// matrix's chunk launches next, and what a chunk launch does to the scan's
// bookkeeping.  serve.hip drives these with HIP graphs, streams and events;
// the host simulation in the tests drives them with modelled launch times.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <deque>
#include <utility>
#include <vector>

namespace wh {
namespace policy {

// right-hand-side buckets of the launch graphs: the multi-RHS kernel's cost
// steps with each group of 16
constexpr uint32_t kBuckets[] = {1, 2, 4, 8, 16, 32, 48, 64};
constexpr int kNumBuckets = sizeof(kBuckets) / sizeof(kBuckets[0]);
// columns of a slot: the bits of a uint64_t
constexpr uint32_t kSlotCols = 64;
// chunk launches in flight on the device (the second keeps the stream busy
// while the worker notices the first one end)
constexpr size_t kMaxInflight = 2;

inline int bucket_index(uint32_t k)
{
    for (int i = 0; i < kNumBuckets; ++i)
        if (k <= kBuckets[i])
            return i;
    return -1;
}

// The k lowest free columns (any, not necessarily consecutive: a request
// never waits for a run of them to come free), or 0 if fewer are free.
inline uint64_t take_cols(uint64_t used, uint32_t k)
{
    uint64_t free = ~used, out = 0;
    for (uint32_t i = 0; i < k; ++i) {
        if (!free)
            return 0;
        const uint64_t low = free & (0 - free);
        out |= low;
        free ^= low;
    }
    return out;
}

// The row chunks of one served pass: consecutive ranges of whole block rows
// holding at most `values` matrix values each (at least one block row).  A
// matrix of at most twice that is one chunk: cutting its pass in two would
// only let other launches in between two halves of a pass short enough to
// meet a deadline.
inline std::vector<std::pair<uint32_t, uint32_t>> chunk_rows(uint32_t rows, uint32_t cols, uint64_t values)
{
    if ((uint64_t)rows * cols <= 2 * values)
        return {{0u, rows}};
    const uint64_t per = std::max<uint64_t>(4, values / std::max<uint32_t>(1, cols) / 4 * 4);
    std::vector<std::pair<uint32_t, uint32_t>> out;
    for (uint64_t r0 = 0; r0 < rows; r0 += per)
        out.emplace_back((uint32_t)r0, (uint32_t)std::min<uint64_t>(r0 + per, rows));
    return out;
}

// What the decisions read of a request.
struct ReqState {
    uint64_t t_arrive = 0;
    uint64_t deadline_ns = 0; // 0: none
    uint32_t k = 0;           // right-hand sides
    uint64_t t_start = 0;     // when it joined the scan
    uint64_t cols = 0;        // its columns of the slot (bit c = column c)
    uint32_t left = 0;        // chunk launches still to issue for it
    uint32_t batch_size = 0;  // requests that joined at the same launch
};

// What the decisions read and update of a matrix's scan.
struct ScanState {
    std::deque<uint64_t> pending; // queued, not yet in the scan
    std::vector<uint64_t> active; // in the scan, chunks left to launch
    uint64_t used = 0;            // columns held (freed when the completing launch is done)
    uint32_t nchunks = 1;
    uint32_t next_chunk = 0;
    double chunk_ms = 0.0;        // running estimate of one chunk launch
    double chunk_ms_max = 0.0;    // the longest recent one (decays)
    double pace_ns = 0.0;         // while its scan runs late: when its next chunk is due
    bool usable = false;          // slot built
    bool can_launch = false;      // usable, and a launch's events are free
};

struct Tuning {
    double pace = 4.0;       // a late scan's chunk times per launch while other work waits
    double margin_ns = 1e6;  // a held request's margin before its deadline
};

// How urgent a matrix's next chunk launch is: the latest start of its
// requests that can still meet their deadlines (deadline less the chunks
// they have left, with `between_ns` for another launch between two of
// them; `late` false), else the pace of a scan running late (`late` true).
// Returns false if it has nothing to launch now; then `hold_until` is when
// its held requests must start (UINT64_MAX: nothing held).  `hold`: another
// matrix's scan is running late, and a matrix with no scan under way holds
// its queued requests while the most urgent can still wait: its pass
// (longest recent chunk times), `ahead_ns` for what may run before its first
// chunk, `between_ns` between its chunks, and the margin.
template <class Get>
bool urgency(const ScanState& ms, Get get, uint64_t now, bool hold, double ahead_ns, double between_ns,
             double margin_ns, double& key, bool& late, uint64_t& hold_until)
{
    hold_until = UINT64_MAX;
    key = 1e300;
    late = false;
    const double chunk_ns = ms.chunk_ms * 1e6;
    if (hold && ms.active.empty() && !ms.pending.empty()) {
        const double nc = (double)ms.nchunks;
        const double pass_ns = ms.chunk_ms_max * 1e6 * nc + between_ns * (nc - 1.0) + ahead_ns;
        double start_by = 1e300;
        uint32_t k = 0;
        for (uint64_t t : ms.pending) {
            const ReqState& r = get(t);
            k += r.k;
            const double due = r.deadline_ns ? (double)(r.t_arrive + r.deadline_ns) : 0.0;
            start_by = std::min(start_by, due - pass_ns - margin_ns);
        }
        if (k < kSlotCols && (double)now < start_by) {
            hold_until = (uint64_t)start_by;
            return false;
        }
    }
    bool any_late = false;
    auto consider = [&](const ReqState& r, uint32_t left) {
        if (!r.deadline_ns) {
            any_late = true;
            return;
        }
        const double due = (double)(r.t_arrive + r.deadline_ns);
        const double rest = left * chunk_ns + (left > 1 ? (left - 1) * between_ns : 0.0);
        if ((double)now + rest + ahead_ns <= due)
            key = std::min(key, due - rest);
        else
            any_late = true;
    };
    for (uint64_t t : ms.active)
        consider(get(t), get(t).left);
    bool joinable = false;
    if (!ms.pending.empty()) {
        const ReqState& head = get(ms.pending.front());
        if (take_cols(ms.used, head.k)) {
            joinable = true;
            consider(head, ms.nchunks);
        }
    }
    if (key == 1e300 && any_late) {
        late = true;
        key = ms.pace_ns > 0.0 ? ms.pace_ns : (double)now;
    }
    return !ms.active.empty() || joinable;
}

// One dispatch decision over the matrices: the index of the one whose chunk
// launches next, or -1; `wake` is the earliest end of a hold.  The earliest
// latest start among requests that can still meet their deadlines goes
// first.  A late scan's paced chunk goes before it when due, if that work
// can still start after it and the launch in flight; a late scan ahead of
// its pace goes only when nothing else waits.  The picked late scan's next
// paced start moves on by `pace` of its chunk times (at most one step either
// side of now).
template <class Get>
int pick(const std::vector<ScanState*>& mats, Get get, uint64_t now, const Tuning& tune, uint64_t& wake)
{
    wake = UINT64_MAX;
    // the scans running late: none of their requests can still meet its deadline
    std::vector<const ScanState*> late_scans;
    for (const ScanState* o : mats) {
        if (!o->usable || o->active.empty())
            continue;
        double key;
        bool late;
        uint64_t h;
        if (urgency(*o, get, now, false, 0.0, 0.0, tune.margin_ns, key, late, h) && late)
            late_scans.push_back(o);
    }
    int feas = -1, late_pick = -1;
    double feas_key = 0.0, late_key = 0.0;
    for (size_t i = 0; i < mats.size(); ++i) {
        const ScanState& ms = *mats[i];
        if (!ms.can_launch)
            continue;
        const bool hold = std::any_of(late_scans.begin(), late_scans.end(),
                                      [&](const ScanState* o) { return o != &ms; });
        // a launch of this matrix may wait for kMaxInflight of the longest
        // recent launches of the others, and each further chunk of its pass
        // for one more
        double between_ns = 0.0;
        for (const ScanState* o : mats)
            if (o != &ms && o->usable)
                between_ns = std::max(between_ns, o->chunk_ms_max * 1e6);
        const double ahead_ns = between_ns * kMaxInflight;
        double key;
        bool late;
        uint64_t h;
        if (!urgency(ms, get, now, hold, ahead_ns, between_ns, tune.margin_ns, key, late, h)) {
            wake = std::min(wake, h);
            continue;
        }
        if (late && (late_pick < 0 || key < late_key)) {
            late_pick = (int)i;
            late_key = key;
        } else if (!late && (feas < 0 || key < feas_key)) {
            feas = (int)i;
            feas_key = key;
        }
    }
    int out = feas;
    if (late_pick >= 0 &&
        (feas < 0 || ((double)now >= late_key &&
                      feas_key - (double)now >= mats[late_pick]->chunk_ms_max * 1e6 * kMaxInflight)))
        out = late_pick;
    if (out >= 0 && out == late_pick) {
        ScanState& ms = *mats[out];
        const double step = tune.pace * ms.chunk_ms * 1e6;
        ms.pace_ns = std::min((double)now + step, std::max((double)now - step, late_key) + step);
    }
    return out;
}

// The bookkeeping of one chunk launch of a matrix.
struct LaunchPlan {
    bool launch = false;          // false: nothing in the scan (no launch)
    uint32_t chunk = 0;           // the chunk it covers
    int bucket = 0;               // the graph's right-hand-side bucket
    std::vector<uint64_t> joined; // requests whose vectors go into their columns first
    std::vector<uint64_t> done;   // requests whose last chunk this is
    uint64_t free = 0;            // their columns, freed when this launch is done
};

// Queued requests join (FIFO, while columns last: each takes its columns,
// all of its chunks still to launch); the launch covers the next chunk of
// the cycle, over the columns up to the highest held; requests that reach
// their last chunk leave the scan (their columns stay held until
// `release`).
template <class GetMut>
LaunchPlan plan_launch(ScanState& ms, GetMut get, uint64_t now)
{
    LaunchPlan p;
    while (!ms.pending.empty()) {
        ReqState& r = get(ms.pending.front());
        const uint64_t mask = take_cols(ms.used, r.k);
        if (!mask)
            break;
        r.cols = mask;
        r.left = ms.nchunks;
        r.t_start = now;
        ms.used |= mask;
        p.joined.push_back(ms.pending.front());
        ms.active.push_back(ms.pending.front());
        ms.pending.pop_front();
    }
    for (uint64_t t : p.joined)
        get(t).batch_size = (uint32_t)p.joined.size();
    if (ms.active.empty())
        return p;
    p.launch = true;
    p.bucket = bucket_index(64u - (uint32_t)__builtin_clzll(ms.used));
    p.chunk = ms.next_chunk;
    ms.next_chunk = (ms.next_chunk + 1) % ms.nchunks;
    size_t keep = 0;
    for (size_t i = 0; i < ms.active.size(); ++i) {
        ReqState& r = get(ms.active[i]);
        if (--r.left > 0) {
            ms.active[keep++] = ms.active[i];
            continue;
        }
        p.free |= r.cols;
        p.done.push_back(ms.active[i]);
    }
    ms.active.resize(keep);
    return p;
}

// A chunk launch's measured time.
inline void observe_chunk(ScanState& ms, double ms_el)
{
    ms.chunk_ms = 0.8 * ms.chunk_ms + 0.2 * ms_el;
    ms.chunk_ms_max = std::max(0.98 * ms.chunk_ms_max, ms_el);
}

// The columns of the requests a launch completed, once its results are out.
inline void release(ScanState& ms, uint64_t free) { ms.used &= ~free; }

} // namespace policy
} // namespace wh

// serve_sim.cpp -- the serving loop's decisions (serve_policy.hpp, the same
// header serve.hip uses) driven by a modelled device, on the host.
//
// The device is one launch queue: a launch starts when the previous one
// ends (or when it is issued, if later) and takes a modelled time that
// depends on its matrix, chunk and right-hand-side bucket.  The loop keeps at
// most kMaxInflight launches whose compute has not ended, decides at every
// arrival, every launch end and every end of a hold, and frees a launch's
// columns when it ends.  Requests arrive as a seeded Poisson process, the
// target matrix uniform over the matrices, k uniform in 1..8.
//
// Checked on every launch and completion (a violation ends the run with exit
// status 3):
//   * a joining request's columns are free: no two requests in a scan, or
//     between a launch and its end, hold a column together;
//   * every request is covered by exactly one launch of each of its
//     matrix's chunks, consecutively in the cycle, between joining and
//     completing;
//   * stamps are ordered: arrival <= start <= done;
//   * every request completes.
// Prints one JSON object: per matrix the requests, p50 / p99 latency and
// service time (ms), the fraction past the deadline and the mean requests
// per joining launch.
//
// usage: serve_sim seed rate_hz n_requests deadline_ms pace margin_us chunk_values
//                  matrix... (each "ROWSxCOLS")
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <cmath>
#include <deque>
#include <vector>

#include "serve_policy.hpp"

using namespace wh::policy;

namespace {

[[noreturn]] void violation(const char* what, uint64_t ticket)
{
    fprintf(stderr, "violation: %s (request %llu)\n", what, (unsigned long long)ticket);
    exit(3);
}

// SplitMix64: the seeded arrivals
struct Rng {
    uint64_t s;
    uint64_t next()
    {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }
};

struct Mat {
    uint32_t rows, cols;
    std::vector<std::pair<uint32_t, uint32_t>> chunks;
    ScanState st;
    uint64_t owned = 0; // columns held by a request between joining and its launch's end
};

struct Req {
    ReqState ps;
    int mat = 0;
    uint64_t t_done = 0;
    bool done = false;
    std::vector<uint32_t> seen; // chunk indices launched while in the scan
};

struct LaunchRec {
    int mat;
    uint64_t end;
    double ms;
    uint64_t free;
    std::vector<uint64_t> done;
};

// Modelled launch time (ms) of `values` matrix values with k held columns:
// the measured cost per 2^28 values of the fused kernel (one column) and of
// the multi-RHS kernel per group of 16 columns, plus a fixed launch cost.
double model_ms(uint64_t values, int bucket)
{
    static const double per228[kNumBuckets] = {0.245, 0.40, 0.40, 0.40, 0.40, 0.44, 0.475, 0.505};
    return 0.03 + per228[bucket] * (double)values / (double)(1ull << 28);
}

double pct(std::vector<double> v, double p)
{
    if (v.empty())
        return 0.0;
    std::sort(v.begin(), v.end());
    const double x = p / 100.0 * (double)(v.size() - 1);
    const size_t i = (size_t)x;
    const double f = x - (double)i;
    return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

} // namespace

int main(int argc, char** argv)
{
    if (argc < 9) {
        fprintf(stderr, "usage: %s seed rate_hz n deadline_ms pace margin_us chunk_values RxC...\n", argv[0]);
        return 2;
    }
    Rng rng{strtoull(argv[1], nullptr, 10)};
    const double rate = atof(argv[2]);
    const size_t n = strtoull(argv[3], nullptr, 10);
    const uint64_t deadline = (uint64_t)(atof(argv[4]) * 1e6);
    const Tuning tune{atof(argv[5]), atof(argv[6]) * 1e3};
    const uint64_t chunk_values = strtoull(argv[7], nullptr, 10);
    std::vector<Mat> mats;
    for (int a = 8; a < argc; ++a) {
        Mat m{};
        if (sscanf(argv[a], "%ux%u", &m.rows, &m.cols) != 2)
            return 2;
        m.chunks = chunk_rows(m.rows, m.cols, chunk_values);
        m.st.nchunks = (uint32_t)m.chunks.size();
        double model = 0.0;
        for (const auto& c : m.chunks)
            model = std::max(model, 1e-9 * (double)(c.second - c.first) * m.cols);
        m.st.chunk_ms = m.st.chunk_ms_max = model;
        m.st.usable = m.st.can_launch = true;
        mats.push_back(std::move(m));
    }
    const int nm = (int)mats.size();

    // arrivals
    std::vector<Req> reqs(n);
    std::vector<uint64_t> arrive(n);
    double t = 0.0;
    for (size_t i = 0; i < n; ++i) {
        t += -std::log1p(-rng.uniform()) / rate;
        arrive[i] = (uint64_t)(t * 1e9) + 1;
        reqs[i].mat = std::min(nm - 1, (int)(rng.uniform() * nm));
        reqs[i].ps.k = 1 + std::min(7u, (uint32_t)(rng.uniform() * 8));
        reqs[i].ps.t_arrive = arrive[i];
        reqs[i].ps.deadline_ns = deadline;
    }
    auto get = [&](uint64_t tk) -> ReqState& { return reqs[tk].ps; };
    auto cget = [&](uint64_t tk) -> const ReqState& { return reqs[tk].ps; };

    std::deque<LaunchRec> inflight; // launches in issue order (one queue)
    uint64_t device_free = 0;        // when the queue's last launch ends
    size_t next_arrival = 0, completed = 0;
    uint64_t now = 0, wake = UINT64_MAX;
    std::vector<double> lat[8], svc[8];
    std::vector<double> batch[8];
    size_t missed[8] = {0};

    while (completed < n) {
        // next event: an arrival, a launch end, or the end of a hold
        uint64_t next = UINT64_MAX;
        if (next_arrival < n)
            next = arrive[next_arrival];
        if (!inflight.empty())
            next = std::min(next, inflight.front().end);
        if (wake != UINT64_MAX && wake > now)
            next = std::min(next, wake);
        if (next == UINT64_MAX)
            violation("requests left with nothing to run them", 0);
        now = std::max(now, next);
        while (next_arrival < n && arrive[next_arrival] <= now) {
            mats[reqs[next_arrival].mat].st.pending.push_back(next_arrival);
            ++next_arrival;
        }
        // launch ends: timing, completions, columns freed
        while (!inflight.empty() && inflight.front().end <= now) {
            LaunchRec& l = inflight.front();
            Mat& m = mats[l.mat];
            observe_chunk(m.st, l.ms);
            for (uint64_t tk : l.done) {
                Req& r = reqs[tk];
                if (r.done)
                    violation("completed twice", tk);
                // exactly one launch of each chunk, consecutive in the cycle
                if (r.seen.size() != m.st.nchunks)
                    violation("not covered by one launch per chunk", tk);
                for (size_t j = 1; j < r.seen.size(); ++j)
                    if (r.seen[j] != (r.seen[j - 1] + 1) % m.st.nchunks)
                        violation("chunks out of cycle order", tk);
                r.done = true;
                r.t_done = l.end;
                if (!(r.ps.t_arrive <= r.ps.t_start && r.ps.t_start <= r.t_done))
                    violation("stamps out of order", tk);
                const double ms = (double)(r.t_done - r.ps.t_arrive) * 1e-6;
                lat[r.mat].push_back(ms);
                svc[r.mat].push_back((double)(r.t_done - r.ps.t_start) * 1e-6);
                if (r.t_done > r.ps.t_arrive + r.ps.deadline_ns)
                    ++missed[r.mat];
                ++completed;
            }
            m.owned &= ~l.free;
            release(m.st, l.free);
            inflight.pop_front();
        }
        // dispatch
        wake = UINT64_MAX;
        for (;;) {
            size_t computing = 0;
            for (const LaunchRec& l : inflight)
                computing += l.end > now;
            if (computing >= kMaxInflight)
                break;
            std::vector<ScanState*> scans;
            for (Mat& m : mats)
                scans.push_back(&m.st);
            uint64_t w;
            const int i = pick(scans, cget, now, tune, w);
            wake = std::min(wake, w);
            if (i < 0)
                break;
            Mat& m = mats[(size_t)i];
            const LaunchPlan p = plan_launch(m.st, get, now);
            for (uint64_t tk : p.joined) {
                const uint64_t c = reqs[tk].ps.cols;
                if ((uint32_t)__builtin_popcountll(c) != reqs[tk].ps.k)
                    violation("wrong number of columns", tk);
                if (c & m.owned)
                    violation("column held twice", tk);
                m.owned |= c;
                batch[i].push_back((double)p.joined.size());
            }
            if (!p.launch)
                break;
            for (uint64_t tk : m.st.active)
                reqs[tk].seen.push_back(p.chunk);
            for (uint64_t tk : p.done)
                reqs[tk].seen.push_back(p.chunk);
            const auto& c = m.chunks[p.chunk];
            const double ms = model_ms((uint64_t)(c.second - c.first) * m.cols, p.bucket);
            const uint64_t start = std::max(now, device_free);
            device_free = start + (uint64_t)(ms * 1e6);
            inflight.push_back(LaunchRec{i, device_free, ms, p.free, p.done});
        }
    }
    for (const Req& r : reqs)
        if (!r.done)
            violation("never completed", 0);

    printf("{\"violations\": 0, \"per_matrix\": [");
    for (int j = 0; j < nm; ++j) {
        double mb = 0.0;
        for (double b : batch[j])
            mb += b;
        printf("%s{\"matrix\": \"%ux%u\", \"chunks\": %u, \"requests\": %zu, \"p50_ms\": %.4f, \"p99_ms\": %.4f, "
               "\"service_p50_ms\": %.4f, \"service_p99_ms\": %.4f, \"miss_rate\": %.5f, \"mean_batch\": %.3f}",
               j ? ", " : "", mats[j].rows, mats[j].cols, mats[j].st.nchunks, lat[j].size(), pct(lat[j], 50),
               pct(lat[j], 99), pct(svc[j], 50), pct(svc[j], 99),
               lat[j].empty() ? 0.0 : (double)missed[j] / (double)lat[j].size(),
               batch[j].empty() ? 0.0 : mb / (double)batch[j].size());
    }
    printf("]}\n");
    return 0;
}

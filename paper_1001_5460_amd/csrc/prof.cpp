// Kernel timing tracer (see prof.hpp) and its C ABI.
#include "prof.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cta.h"
#include "abi_internal.hpp"

namespace cta {

namespace {
struct Rec {
    const char* name;
    hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t take() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

bool prof_enabled() { return g_on; }

int prof_begin(const char* name, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    Rec r{name, take(), take()};
    if (!r.a || !r.b) return -1;
    if (hipEventRecord(r.a, s) != hipSuccess) return -1;
    g_recs.push_back(r);
    return (int)g_recs.size() - 1;
}

void prof_end(int id, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (id >= 0 && id < (int)g_recs.size()) (void)hipEventRecord(g_recs[id].b, s);
}

}  // namespace cta

using namespace cta;

extern "C" cta_status cta_prof_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on != 0;
    return CTA_OK;
}

// While the tracer is on, the events of dropped records go back to a pool for
// the next launches; a reset with the tracer off destroys every event, so the
// library holds no HIP events once tracing is done (none are left for the
// runtime's own teardown at process exit).
extern "C" cta_status cta_prof_reset(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (Rec& r : g_recs) {
        (void)hipEventSynchronize(r.b);
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_recs.clear();
    if (!g_on) {
        for (hipEvent_t e : g_pool) (void)hipEventDestroy(e);
        g_pool.clear();
    }
    return CTA_OK;
}

extern "C" cta_status cta_prof_read(char* host_buf, size_t bytes, size_t* needed) {
    std::lock_guard<std::mutex> lk(g_mu);
    std::map<std::string, std::vector<double>> dur;
    for (Rec& r : g_recs) {
        if (hipEventSynchronize(r.b) != hipSuccess) return fail(CTA_ERR_HIP, "event synchronize failed");
        float ms = 0;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return fail(CTA_ERR_HIP, "event timing failed");
        dur[r.name].push_back(ms);
    }
    std::string out = "{";
    bool first = true;
    for (auto& kv : dur) {
        std::vector<double> d = kv.second;
        std::sort(d.begin(), d.end());
        double total = 0;
        for (double v : d) total += v;
        // active launches: at least a tenth of the 90th-percentile duration
        // (launches gated by a converged solve's flag exit at once)
        const double cut = 0.1 * d[(d.size() - 1) * 9 / 10];
        long nact = 0;
        double tact = 0;
        for (double v : d)
            if (v >= cut) {
                ++nact;
                tact += v;
            }
        char buf[320];
        snprintf(buf, sizeof buf,
                 "%s\"%s\": {\"count\": %ld, \"total_ms\": %.6f, \"min_ms\": %.6f, \"max_ms\": %.6f, "
                 "\"active_count\": %ld, \"active_ms\": %.6f}",
                 first ? "" : ", ", kv.first.c_str(), (long)d.size(), total, d.front(), d.back(), nact, tact);
        out += buf;
        first = false;
    }
    out += "}";
    if (needed) *needed = out.size();
    if (host_buf && bytes > 0) {
        const size_t n = std::min(bytes - 1, out.size());
        std::memcpy(host_buf, out.data(), n);
        host_buf[n] = 0;
    }
    return CTA_OK;
}

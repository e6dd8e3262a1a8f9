// Optional per-kernel timing: when enabled, every launch is bracketed by HIP
// events on its own stream and tagged with its kernel name and the bytes the
// algorithm must move for that launch (inputs read once, outputs written
// once).  Disabled by default; enabling it adds two event records per launch.

#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace prnu {
namespace {

struct Rec {
    const char *name;
    double bytes, flops;
    hipEvent_t a, b;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t get_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void recycle_all() {
    for (auto &r : g_recs) {
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_recs.clear();
}

}  // namespace

KernelTimer::KernelTimer(const char *name, double bytes, hipStream_t s, double flops) : idx_(-1), s_(s) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on) return;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return;
    hipEvent_t a = get_event(), b = get_event();
    if (!a || !b) return;
    if (hipEventRecord(a, s) != hipSuccess) return;
    g_recs.push_back({name, bytes, flops, a, b});
    idx_ = (long)g_recs.size() - 1;
}

KernelTimer::~KernelTimer() {
    if (idx_ < 0) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (idx_ < (long)g_recs.size()) hipEventRecord(g_recs[idx_].b, s_);
}

}  // namespace prnu

extern "C" int prnu_timing_enable(int on) {
    std::lock_guard<std::mutex> lk(prnu::g_mu);
    for (auto &r : prnu::g_recs) {
        hipEventSynchronize(r.b);
    }
    prnu::recycle_all();
    prnu::g_on = on != 0;
    return PRNU_OK;
}

extern "C" int prnu_timing_report(char *buf, size_t len, size_t *needed) {
    std::lock_guard<std::mutex> lk(prnu::g_mu);
    struct Agg {
        long n = 0;
        double ms = 0.0, bytes = 0.0, flops = 0.0;
    };
    std::map<std::string, Agg> agg;
    for (auto &r : prnu::g_recs) {
        if (hipEventSynchronize(r.b) != hipSuccess)
            return prnu::fail(PRNU_E_HIP, "prnu_timing_report: event synchronisation failed");
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
            return prnu::fail(PRNU_E_HIP, "prnu_timing_report: elapsed time failed");
        Agg &g = agg[r.name];
        g.n += 1;
        g.ms += ms;
        g.bytes += r.bytes;
        g.flops += r.flops;
    }
    std::string out;
    char line[256];
    for (auto &kv : agg) {
        snprintf(line, sizeof(line), "%s\t%ld\t%.6f\t%.0f\t%.0f\n", kv.first.c_str(), kv.second.n, kv.second.ms,
                 kv.second.bytes, kv.second.flops);
        out += line;
    }
    if (needed) *needed = out.size() + 1;
    if (buf && len > 0) {
        const size_t k = out.size() < len - 1 ? out.size() : len - 1;
        memcpy(buf, out.data(), k);
        buf[k] = 0;
        if (k < out.size()) return prnu::fail(PRNU_E_INVAL, "prnu_timing_report: buffer too small");
    }
    return PRNU_OK;
}

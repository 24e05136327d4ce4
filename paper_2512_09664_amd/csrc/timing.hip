// Optional per-kernel timing: while enabled, each kernel launch of the library
// is bracketed by two hipEvents recorded on the launch stream; reading the
// timer waits for those events and sums their elapsed times per kernel name.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "launch.hpp"

namespace sp {
namespace {

struct Pending {
    std::string name;
    hipEvent_t start, stop;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;

hipEvent_t take_event()
{
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

TimedScope::TimedScope(const char* name, hipStream_t s) : name_(name), stream_(s), start_(nullptr)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    start_ = take_event();
    if (start_ && hipEventRecord(start_, s) != hipSuccess) {
        g_pool.push_back(start_);
        start_ = nullptr;
    }
}

TimedScope::~TimedScope()
{
    if (!start_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t stop = take_event();
    if (!stop || hipEventRecord(stop, stream_) != hipSuccess) {
        g_pool.push_back(start_);
        if (stop) g_pool.push_back(stop);
        return;
    }
    g_pending.push_back({name_, start_, stop});
}

void timing_enable(bool on)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on;
}

int timing_read(const char* name, double* total_ms, int64_t* launches)
{
    std::lock_guard<std::mutex> lk(g_mu);
    double tot = 0.0;
    int64_t n = 0;
    std::vector<Pending> keep;
    for (const Pending& p : g_pending) {
        if (name && p.name != name) {
            keep.push_back(p);
            continue;
        }
        if (hipEventSynchronize(p.stop) != hipSuccess) return -1;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p.start, p.stop) != hipSuccess) return -1;
        tot += ms;
        ++n;
        g_pool.push_back(p.start);
        g_pool.push_back(p.stop);
    }
    g_pending.swap(keep);
    *total_ms = tot;
    *launches = n;
    return 0;
}

int device_cu_count()
{
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cached[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cached[dev] = n;
    }
    return cached[dev];
}

}  // namespace sp

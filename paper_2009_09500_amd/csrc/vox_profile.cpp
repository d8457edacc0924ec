// Kernel timing for the tracing entry points (vox_profile_* in vox.h): when
// enabled, every kernel launch of the library is bracketed by a pair of HIP
// events recorded on the launch's own stream; durations are collected when
// they are read.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "vox.h"
#include "vox_internal.h"

namespace vox {
namespace {

struct Record {
    std::string name;
    double total_ms = 0.0;
    int64_t launches = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
};

std::atomic<bool> g_enabled{false};
std::mutex g_mu;
std::vector<Record> g_records;
std::vector<hipEvent_t> g_pool;

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

Record& record_for(const char* name) {
    for (auto& r : g_records)
        if (r.name == name) return r;
    g_records.emplace_back();
    g_records.back().name = name;
    return g_records.back();
}

// Resolves every pending pair (synchronising on its end event).
void drain() {
    for (auto& r : g_records) {
        for (auto& p : r.pending) {
            float ms = 0.f;
            if (hipEventSynchronize(p.second) == hipSuccess &&
                hipEventElapsedTime(&ms, p.first, p.second) == hipSuccess) {
                r.total_ms += ms;
                r.launches += 1;
            }
            g_pool.push_back(p.first);
            g_pool.push_back(p.second);
        }
        r.pending.clear();
    }
}

}  // namespace

KernelTimer::KernelTimer(const char* name, hipStream_t stream) : name_(name), stream_(stream) {
    if (!g_enabled.load(std::memory_order_relaxed)) return;
    // Launches being captured into a graph are not timed.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream_, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return;
    std::lock_guard<std::mutex> lk(g_mu);
    start_ = take_event();
    if (start_ && hipEventRecord(start_, stream_) != hipSuccess) {
        g_pool.push_back(start_);
        start_ = nullptr;
    }
}

KernelTimer::~KernelTimer() {
    if (!start_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t end = take_event();
    if (!end || hipEventRecord(end, stream_) != hipSuccess) {
        g_pool.push_back(start_);
        if (end) g_pool.push_back(end);
        return;
    }
    record_for(name_).pending.emplace_back(start_, end);
}

}  // namespace vox

extern "C" {

vox_status vox_profile_enable(int enable) {
    vox::g_enabled.store(enable != 0);
    return VOX_OK;
}

void vox_profile_reset(void) {
    std::lock_guard<std::mutex> lk(vox::g_mu);
    vox::drain();
    vox::g_records.clear();
}

int vox_profile_count(void) {
    std::lock_guard<std::mutex> lk(vox::g_mu);
    return (int)vox::g_records.size();
}

vox_status vox_profile_read(int index, char* name, size_t name_len, double* total_ms,
                            int64_t* launches) {
    std::lock_guard<std::mutex> lk(vox::g_mu);
    vox::drain();
    if (index < 0 || index >= (int)vox::g_records.size()) return VOX_ERR_INVALID_ARGUMENT;
    const auto& r = vox::g_records[index];
    if (name && name_len) {
        std::strncpy(name, r.name.c_str(), name_len - 1);
        name[name_len - 1] = '\0';
    }
    if (total_ms) *total_ms = r.total_ms;
    if (launches) *launches = r.launches;
    return VOX_OK;
}

}  // extern "C"

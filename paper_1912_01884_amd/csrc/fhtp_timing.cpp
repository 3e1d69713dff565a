// Per-kernel timing for benchmarks (fhtp_timing_start / fhtp_timing_stop).
//
// While timing is on, every launch the library makes outside graph capture is
// bracketed by two events recorded on its stream, and each bracket is filed
// under the launch's kernel family.  fhtp_timing_stop waits for the events
// and returns, per family, the number of launches and their summed elapsed
// time.  Off (the default), a launch pays one relaxed atomic load.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fhtp.h"
#include "fhtp_internal.h"

namespace fhtp {
namespace {

struct Bracket {
    const char* family;
    int launches;
    hipEvent_t begin, end;
};

std::atomic<bool> g_on{false};
std::mutex g_mu;
std::vector<Bracket> g_done;
std::vector<hipEvent_t> g_pool;  // events of earlier runs, reused

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

bool capturing(hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return true;  // unknown: do not record
    }
    return cs != hipStreamCaptureStatusNone;
}

}  // namespace

TimedLaunch::TimedLaunch(const char* family, hipStream_t s, int launches)
    : family_(family), stream_(s), launches_(launches) {
    if (!family || launches <= 0 || !g_on.load(std::memory_order_relaxed) || capturing(s)) return;
    std::lock_guard<std::mutex> lock(g_mu);
    begin_ = take_event();
    if (begin_ && hipEventRecord(begin_, s) != hipSuccess) {
        (void)hipGetLastError();
        g_pool.push_back(begin_);
        begin_ = nullptr;
    }
}

void TimedLaunch::close() {
    if (!begin_) return;
    std::lock_guard<std::mutex> lock(g_mu);
    hipEvent_t end = take_event();
    if (!end || hipEventRecord(end, stream_) != hipSuccess) {
        (void)hipGetLastError();
        g_pool.push_back(begin_);
        if (end) g_pool.push_back(end);
    } else {
        g_done.push_back(Bracket{family_, launches_, begin_, end});
    }
    begin_ = nullptr;
}

}  // namespace fhtp

extern "C" {

int fhtp_timing_start(void) {
    std::lock_guard<std::mutex> lock(fhtp::g_mu);
    for (auto& b : fhtp::g_done) {
        fhtp::g_pool.push_back(b.begin);
        fhtp::g_pool.push_back(b.end);
    }
    fhtp::g_done.clear();
    fhtp::g_on.store(true);
    return FHTP_OK;
}

int fhtp_timing_stop(fhtp_kernel_time* out, int cap, int* count) {
    if (!count || (cap > 0 && !out)) return FHTP_ERR_NULL;
    fhtp::g_on.store(false);
    std::lock_guard<std::mutex> lock(fhtp::g_mu);
    std::vector<fhtp_kernel_time> fam;
    int rc = FHTP_OK;
    for (auto& b : fhtp::g_done) {
        float ms = 0.f;
        if (hipEventSynchronize(b.end) != hipSuccess ||
            hipEventElapsedTime(&ms, b.begin, b.end) != hipSuccess) {
            (void)hipGetLastError();
            rc = FHTP_ERR_HIP;
        }
        size_t q = 0;
        while (q < fam.size() && std::strcmp(fam[q].name, b.family) != 0) ++q;
        if (q == fam.size()) {
            fhtp_kernel_time t{};
            std::strncpy(t.name, b.family, sizeof(t.name) - 1);
            fam.push_back(t);
        }
        fam[q].launches += b.launches;
        fam[q].total_ms += ms;
        fhtp::g_pool.push_back(b.begin);
        fhtp::g_pool.push_back(b.end);
    }
    fhtp::g_done.clear();
    *count = (int)fam.size();
    for (int q = 0; q < cap && q < (int)fam.size(); ++q) out[q] = fam[q];
    return rc;
}

}  // extern "C"

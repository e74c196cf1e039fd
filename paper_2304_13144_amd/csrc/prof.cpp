// Event-based timing of library kernels (mtp_profile_enable / mtp_profile_read).
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

namespace mtp {
namespace {
struct Rec {
    std::vector<hipEvent_t> begin, end;
};
std::mutex g_mu;
bool g_on = false;
std::map<std::string, Rec> g_rec;
}  // namespace

void prof_mark(const char *name, bool begin, hipStream_t st) {
    if (!g_on) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    if (hipEventRecord(e, st) != hipSuccess) {
        (void)hipEventDestroy(e);
        return;
    }
    auto &r = g_rec[name];
    (begin ? r.begin : r.end).push_back(e);
}

}  // namespace mtp

extern "C" int mtp_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(mtp::g_mu);
    mtp::g_on = on != 0;
    return MTP_OK;
}

extern "C" int mtp_profile_read(const char *kernel, double *total_ms, int64_t *launches) {
    if (!kernel || !total_ms || !launches) {
        mtp::set_error("NULL argument");
        return MTP_E_INVAL;
    }
    std::lock_guard<std::mutex> lk(mtp::g_mu);
    auto it = mtp::g_rec.find(kernel);
    *total_ms = 0.0;
    *launches = 0;
    if (it == mtp::g_rec.end()) return MTP_OK;
    auto &r = it->second;
    const size_t n = std::min(r.begin.size(), r.end.size());
    double tot = 0.0;
    for (size_t k = 0; k < n; ++k) {
        if (hipEventSynchronize(r.end[k]) != hipSuccess) {
            mtp::set_error("hipEventSynchronize failed");
            return MTP_E_HIP;
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.begin[k], r.end[k]) == hipSuccess) tot += ms;
    }
    for (auto e : r.begin) (void)hipEventDestroy(e);
    for (auto e : r.end) (void)hipEventDestroy(e);
    mtp::g_rec.erase(it);
    *total_ms = tot;
    *launches = (int64_t)n;
    return MTP_OK;
}

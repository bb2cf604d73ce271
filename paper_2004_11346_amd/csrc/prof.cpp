#include "prof.h"

#include <cstdio>
#include <map>

namespace sht {
namespace prof {

namespace {
thread_local Recorder *tl_rec = nullptr;
}

Recorder *current() { return tl_rec; }
void install(Recorder *r) { tl_rec = r; }

Recorder::~Recorder() {
    clear();
    for (hipEvent_t e : pool_) (void)hipEventDestroy(e);
}

hipEvent_t Recorder::get() {
    if (!pool_.empty()) {
        hipEvent_t e = pool_.back();
        pool_.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void Recorder::begin(hipStream_t s, const char *name) {
    Rec r{name, get(), get()};
    if (!r.e0 || !r.e1) return;
    (void)hipEventRecord(r.e0, s);
    recs_.push_back(r);
    open_ = (int)recs_.size() - 1;
}

void Recorder::end(hipStream_t s) {
    if (open_ < 0) return;
    (void)hipEventRecord(recs_[open_].e1, s);
    open_ = -1;
}

std::string Recorder::report() {
    struct Acc {
        int n = 0;
        double ms = 0.0;
    };
    std::map<std::string, Acc> acc;
    for (const Rec &r : recs_) {
        float ms = 0.f;
        if (hipEventSynchronize(r.e1) != hipSuccess) continue;
        if (hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess) continue;
        Acc &a = acc[r.name];
        a.n += 1;
        a.ms += ms;
    }
    std::string out = "{";
    char buf[256];
    bool first = true;
    for (const auto &kv : acc) {
        std::snprintf(buf, sizeof(buf), "%s\"%s\": {\"launches\": %d, \"total_ms\": %.6f, \"avg_ms\": %.6f}",
                      first ? "" : ", ", kv.first.c_str(), kv.second.n, kv.second.ms, kv.second.ms / kv.second.n);
        out += buf;
        first = false;
    }
    return out + "}";
}

void Recorder::clear() {
    for (const Rec &r : recs_) {
        pool_.push_back(r.e0);
        pool_.push_back(r.e1);
    }
    recs_.clear();
    open_ = -1;
}

}  // namespace prof
}  // namespace sht

// Optional per-kernel timing with HIP events recorded on the launch stream.
// A plan with profiling switched on installs its recorder for the duration
// of each API call (thread-local); launchers bracket their kernels with
// Scope objects, which do nothing when no recorder is installed.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

namespace sht {
namespace prof {

class Recorder {
  public:
    ~Recorder();
    void begin(hipStream_t s, const char *name);
    void end(hipStream_t s);
    // waits for the recorded events; returns a JSON object
    // {"<kernel>": {"launches": n, "total_ms": t, "avg_ms": t / n}, ...}
    std::string report();
    void clear();

  private:
    struct Rec {
        const char *name;
        hipEvent_t e0, e1;
    };
    std::vector<Rec> recs_;
    std::vector<hipEvent_t> pool_;
    int open_ = -1;
    hipEvent_t get();
};

Recorder *current();
void install(Recorder *r);

struct Scope {
    Recorder *r;
    hipStream_t s;
    Scope(hipStream_t st, const char *name) : r(current()), s(st) {
        if (r) r->begin(s, name);
    }
    ~Scope() {
        if (r) r->end(s);
    }
};

struct Install {
    Recorder *prev;
    explicit Install(Recorder *r) : prev(current()) { install(r); }
    ~Install() { install(prev); }
};

}  // namespace prof
}  // namespace sht

// Optional per-plan instrumentation: HIP events recorded on the caller's
// stream around kernel groups, read back (with a wait) on request.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

namespace crbm {

struct Profiler {
    struct Rec { int id; hipEvent_t a, b; };
    bool on = false;
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    int open_id = -1;
    hipEvent_t open_ev = nullptr;

    hipEvent_t take() {
        if (used == pool.size()) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
    void begin(int id, hipStream_t s) {
        if (!on) return;
        open_ev = take();
        open_id = id;
        if (open_ev) (void)hipEventRecord(open_ev, s);
    }
    void end(hipStream_t s) {
        if (!on || open_id < 0) return;
        hipEvent_t e = take();
        if (e && open_ev) {
            (void)hipEventRecord(e, s);
            recs.push_back({open_id, open_ev, e});
        }
        open_id = -1;
    }
    void reset() { recs.clear(); used = 0; open_id = -1; }
    ~Profiler() {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

}  // namespace crbm

// Per-stage device timing for diagnostics: when enabled, the entry points
// bracket their kernel launches with HIP events on the call's stream and,
// at the synchronisation point every entry point already has, add the
// elapsed times to process-wide per-stage totals.
#include "kmg_internal.h"

namespace kmg {

namespace {

constexpr int kPairs = 256;

struct TimerState {
    bool enabled = false;
    bool created = false;
    hipEvent_t ev[kPairs][2];
    int stage_of[kPairs];
    int used = 0;
    double ms[kStageCount] = {};
    int64_t launches[kStageCount] = {};
};

TimerState g_timer;

}  // namespace

void timer_begin(int stage, hipStream_t s) {
    TimerState& t = g_timer;
    if (!t.enabled || t.used >= kPairs) return;
    t.stage_of[t.used] = stage;
    (void)hipEventRecord(t.ev[t.used][0], s);
}

void timer_end(int stage, hipStream_t s) {
    TimerState& t = g_timer;
    if (!t.enabled || t.used >= kPairs || t.stage_of[t.used] != stage) return;
    (void)hipEventRecord(t.ev[t.used][1], s);
    ++t.used;
}

void timer_collect() {
    TimerState& t = g_timer;
    if (!t.enabled) return;
    for (int i = 0; i < t.used; ++i) {
        float ms = 0.0f;
        (void)hipEventSynchronize(t.ev[i][1]);
        if (hipEventElapsedTime(&ms, t.ev[i][0], t.ev[i][1]) == hipSuccess) {
            t.ms[t.stage_of[i]] += ms;
            t.launches[t.stage_of[i]] += 1;
        }
    }
    t.used = 0;
}

int timer_enable(int on) {
    TimerState& t = g_timer;
    if (on && !t.created) {
        for (int i = 0; i < kPairs; ++i)
            for (int j = 0; j < 2; ++j)
                if (hipEventCreate(&t.ev[i][j]) != hipSuccess) return -1;
        t.created = true;
    }
    t.enabled = on != 0;
    t.used = 0;
    for (int i = 0; i < kStageCount; ++i) {
        t.ms[i] = 0.0;
        t.launches[i] = 0;
    }
    return 0;
}

int timer_read(double* ms, int64_t* launches, int n) {
    timer_collect();
    const int k = n < kStageCount ? n : kStageCount;
    for (int i = 0; i < k; ++i) {
        if (ms) ms[i] = g_timer.ms[i];
        if (launches) launches[i] = g_timer.launches[i];
    }
    return kStageCount;
}

const char* stage_name(int stage) {
    static const char* names[kStageCount] = {"voxelize", "grid", "search_count", "search_fill", "normals",
                                             "spfh", "fpfh", "j_compact", "match_pack", "match_topk",
                                             "match_rescore", "match_mutual"};
    return (stage >= 0 && stage < kStageCount) ? names[stage] : "unknown";
}

}  // namespace kmg

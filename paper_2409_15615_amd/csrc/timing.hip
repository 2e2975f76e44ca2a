// Per-stage device timing for diagnostics: when enabled, the entry points
// bracket their kernel launches with HIP events on the call's stream and,
// at the synchronisation point every entry point already has, add the
// elapsed times to process-wide per-stage totals.  A stage opened inside
// another one is part of the outer stage.
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
    bool open = false;
    double ms[kStageCount] = {};
    int64_t launches[kStageCount] = {};
    const int64_t* work[kStageCount] = {};  // device counters of the stages' last timed launches
};

TimerState g_timer;

}  // namespace

void timer_begin(int stage, hipStream_t s) {
    TimerState& t = g_timer;
    if (!t.enabled || t.used >= kPairs || t.open) return;
    t.open = true;
    t.stage_of[t.used] = stage;
    (void)hipEventRecord(t.ev[t.used][0], s);
}

void timer_end(int stage, hipStream_t s) {
    TimerState& t = g_timer;
    if (!t.enabled || !t.open || t.stage_of[t.used] != stage) return;
    (void)hipEventRecord(t.ev[t.used][1], s);
    ++t.used;
    t.open = false;
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
    t.open = false;
    for (int i = 0; i < kStageCount; ++i) {
        t.ms[i] = 0.0;
        t.launches[i] = 0;
        t.work[i] = nullptr;
    }
    return 0;
}

void timer_note_work(const int64_t* dev) {
    TimerState& t = g_timer;
    if (!t.enabled || !t.open) return;
    t.work[t.stage_of[t.used]] = dev;
}

int timer_work(int64_t* work, int n) {
    timer_collect();
    const int k = n < kStageCount ? n : kStageCount;
    for (int i = 0; i < k; ++i) {
        int64_t v = 0;
        if (g_timer.work[i] && hipMemcpy(&v, g_timer.work[i], sizeof(v), hipMemcpyDeviceToHost) != hipSuccess) v = -1;
        if (work) work[i] = v;
    }
    return kStageCount;
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
                                             "match_rescore", "match_mutual", "match_image"};
    return (stage >= 0 && stage < kStageCount) ? names[stage] : "unknown";
}

}  // namespace kmg

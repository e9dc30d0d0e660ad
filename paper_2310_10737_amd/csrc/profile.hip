// Kernel timing and work counters for measurement (sogrand_profile_begin / _end).
#include <cstring>

#include "internal.hpp"

namespace sg {

namespace {

const char *kProfNames[PK_COUNT] = {"component", "product_pass", "product_check", "product_init",
                                    "batched", "serve"};

struct EventPair {
    ProfKind kind;
    hipEvent_t start, stop;
};

struct ProfState {
    std::mutex mu;
    bool active = false;
    bool count = false;
    int device = -1;
    ProfCounters *d_counters = nullptr;   // [PK_COUNT][kProfSlots]
    std::vector<EventPair> pairs;
    std::vector<hipEvent_t> pool;
};

ProfState &state() {
    static ProfState s;
    return s;
}

hipEvent_t take_event(ProfState &s) {
    if (!s.pool.empty()) {
        hipEvent_t e = s.pool.back();
        s.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

}  // namespace

ProfCounters *prof_counters(ProfKind kind) {
    ProfState &s = state();
    std::lock_guard<std::mutex> lk(s.mu);
    if (!s.active || !s.count || !s.d_counters) return nullptr;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != s.device) return nullptr;
    return s.d_counters + (size_t)kind * kProfSlots;
}

int prof_start(ProfKind kind, hipStream_t st) {
    ProfState &s = state();
    std::lock_guard<std::mutex> lk(s.mu);
    if (!s.active) return -1;
    EventPair p{kind, take_event(s), take_event(s)};
    if (!p.start || !p.stop) return -1;
    if (hipEventRecord(p.start, st) != hipSuccess) return -1;
    s.pairs.push_back(p);
    return (int)s.pairs.size() - 1;
}

void prof_stop(int token, hipStream_t st) {
    if (token < 0) return;
    ProfState &s = state();
    std::lock_guard<std::mutex> lk(s.mu);
    if (token < (int)s.pairs.size()) (void)hipEventRecord(s.pairs[token].stop, st);
}

}  // namespace sg

extern "C" {

int sogrand_profile_begin(int count_work) {
    using namespace sg;
    ProfState &s = state();
    std::lock_guard<std::mutex> lk(s.mu);
    for (auto &p : s.pairs) {
        s.pool.push_back(p.start);
        s.pool.push_back(p.stop);
    }
    s.pairs.clear();
    SG_HIP(hipGetDevice(&s.device));
    s.count = count_work != 0;
    if (s.count) {
        if (!s.d_counters) SG_HIP(hipMalloc(&s.d_counters, sizeof(ProfCounters) * PK_COUNT * kProfSlots));
        SG_HIP(hipMemset(s.d_counters, 0, sizeof(ProfCounters) * PK_COUNT * kProfSlots));
        SG_HIP(hipDeviceSynchronize());
    }
    s.active = true;
    return SOGRAND_OK;
}

int sogrand_profile_end(sogrand_kernel_stat_t *stats, int max_stats, int *n_stats) {
    using namespace sg;
    if (!n_stats || (max_stats > 0 && !stats)) return fail(SOGRAND_EINVAL, "NULL argument");
    ProfState &s = state();
    std::lock_guard<std::mutex> lk(s.mu);
    s.active = false;
    sogrand_kernel_stat_t acc[PK_COUNT];
    std::memset(acc, 0, sizeof acc);
    for (auto &p : s.pairs) {
        SG_HIP(hipEventSynchronize(p.stop));
        float ms = 0.f;
        SG_HIP(hipEventElapsedTime(&ms, p.start, p.stop));
        acc[p.kind].launches++;
        acc[p.kind].total_ms += ms;
    }
    if (s.count && s.d_counters) {
        std::vector<ProfCounters> h((size_t)PK_COUNT * kProfSlots);
        SG_HIP(hipDeviceSynchronize());
        SG_HIP(hipMemcpy(h.data(), s.d_counters, sizeof(ProfCounters) * h.size(), hipMemcpyDeviceToHost));
        for (int k = 0; k < PK_COUNT; k++)
            for (int j = 0; j < kProfSlots; j++) {
                const ProfCounters &c = h[(size_t)k * kProfSlots + j];
                acc[k].words += c.words;
                acc[k].queries += c.queries;
                acc[k].ranks += c.ranks;
                acc[k].exact_rank += c.exact_rank;
            }
    }
    int n = 0;
    for (int k = 0; k < PK_COUNT; k++) {
        if (!acc[k].launches && !acc[k].words) continue;
        if (n < max_stats) {
            stats[n] = acc[k];
            std::strncpy(stats[n].kernel, kProfNames[k], sizeof(stats[n].kernel) - 1);
        }
        n++;
    }
    *n_stats = n < max_stats ? n : max_stats;
    return SOGRAND_OK;
}

}  // extern "C"

// Process-wide launch statistics for the library's kernels (zolo_stats.h).
#include "stats.hpp"

#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/zolo_stats.h"

namespace zolo {
namespace {

struct Entry {
    std::string name;
    long long launches = 0;
    double ms = 0.0;
    double flops = 0.0;
    double bytes = 0.0;
};

struct Pending {
    int slot;
    int pair;
};

constexpr int kPairs = 8192;

struct Registry {
    std::mutex mu;   // the public entry points and StatScope hold it
    bool on = false;
    std::vector<Entry> entries;
    std::vector<hipEvent_t> ev0, ev1;
    std::vector<Pending> pending;
    int next_pair = 0;

    int slot_for(const char* name) {
        for (size_t i = 0; i < entries.size(); ++i)
            if (entries[i].name == name) return (int)i;
        entries.push_back(Entry{name});
        return (int)entries.size() - 1;
    }
    void collect() {
        for (const Pending& p : pending) {
            float ms = 0.f;
            if (hipEventSynchronize(ev1[p.pair]) == hipSuccess &&
                hipEventElapsedTime(&ms, ev0[p.pair], ev1[p.pair]) == hipSuccess)
                entries[p.slot].ms += ms;
        }
        pending.clear();
        next_pair = 0;
    }
    int take_pair() {
        if (ev0.empty()) {
            ev0.resize(kPairs);
            ev1.resize(kPairs);
            for (int i = 0; i < kPairs; ++i) {
                if (hipEventCreate(&ev0[i]) != hipSuccess || hipEventCreate(&ev1[i]) != hipSuccess) {
                    ev0.clear();
                    ev1.clear();
                    return -1;
                }
            }
        }
        if (next_pair >= kPairs) collect();
        return next_pair++;
    }
};

Registry& reg() {
    static Registry r;
    return r;
}

}  // namespace

bool stats_on() { return reg().on; }

StatScope::StatScope(const char* name, hipStream_t st, double flops, double bytes) {
    Registry& r = reg();
    if (!r.on) return;
    std::lock_guard<std::mutex> lock(r.mu);
    slot_ = r.slot_for(name);
    r.entries[slot_].launches += 1;
    r.entries[slot_].flops += flops;
    r.entries[slot_].bytes += bytes;
    pair_ = r.take_pair();
    st_ = st;
    if (pair_ >= 0 && hipEventRecord(r.ev0[pair_], st) != hipSuccess) pair_ = -1;
}

void StatScope::end() {
    Registry& r = reg();
    if (slot_ < 0 || pair_ < 0) return;
    std::lock_guard<std::mutex> lock(r.mu);
    if (hipEventRecord(r.ev1[pair_], st_) == hipSuccess) r.pending.push_back(Pending{slot_, pair_});
    slot_ = -1;
}

}  // namespace zolo

extern "C" {

int zolo_stats_enable(int on) {
    zolo::reg().on = on != 0;
    return 0;
}

int zolo_stats_reset(void) {
    zolo::Registry& r = zolo::reg();
    std::lock_guard<std::mutex> lock(r.mu);
    r.collect();
    r.entries.clear();
    return 0;
}

int zolo_release_events(void) {
    zolo::Registry& r = zolo::reg();
    {
        std::lock_guard<std::mutex> lock(r.mu);
        r.collect();
        for (size_t i = 0; i < r.ev0.size(); ++i) {
            (void)hipEventDestroy(r.ev0[i]);
            (void)hipEventDestroy(r.ev1[i]);
        }
        r.ev0.clear();
        r.ev1.clear();
    }
    return zolo_autotune_reset();
}

int zolo_stats_count(void) {
    zolo::Registry& r = zolo::reg();
    std::lock_guard<std::mutex> lock(r.mu);
    return (int)r.entries.size();
}

int zolo_stats_get(int index, char* name, int name_len, long long* launches, double* ms, double* flops,
                   double* bytes) {
    zolo::Registry& r = zolo::reg();
    std::lock_guard<std::mutex> lock(r.mu);
    r.collect();
    if (index < 0 || index >= (int)r.entries.size()) return -1;
    const zolo::Entry& e = r.entries[index];
    if (name && name_len > 0) {
        std::strncpy(name, e.name.c_str(), (size_t)name_len - 1);
        name[name_len - 1] = 0;
    }
    if (launches) *launches = e.launches;
    if (ms) *ms = e.ms;
    if (flops) *flops = e.flops;
    if (bytes) *bytes = e.bytes;
    return 0;
}

}  // extern "C"

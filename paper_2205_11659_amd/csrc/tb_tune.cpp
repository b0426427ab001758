// Autotuner for the forward calls' launch variants (tb_tune_* in
// include/treebbox.h).  The paper's measurements show that the best number
// of elements per thread depends on the problem size (section "Performance
// results"); here a variant (elements per thread of the main and of the
// reduce pass, close records per thread of the cross-partition pass) is
// chosen per operation and size class by timing every candidate on the
// caller's own input, and the choice is kept per device kind (architecture
// and compute-unit count) in a process-wide table that can be saved and
// loaded as text.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "tb_forward.h"

namespace tb {
namespace {

std::mutex g_mu;
// (device kind, op, size class) -> variant
std::map<std::tuple<std::string, int, int>, Variant> g_table;
std::map<int, std::string> g_kind;  // device ordinal -> "arch:CUs"

// smallest c with 2^c >= n
int size_class(int64_t n) {
    int c = 0;
    while (c < 62 && ((int64_t)1 << c) < n) ++c;
    return c;
}

// "gfx950:256" for the current device; "none" if HIP cannot say (no device:
// the table still works, for host-side use).  Caller holds g_mu.
std::string device_kind_locked() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return "none";
    auto it = g_kind.find(dev);
    if (it != g_kind.end()) return it->second;
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "none";
    std::string arch(p.gcnArchName);
    const size_t colon = arch.find(':');  // drop feature suffixes such as ":sramecc+:xnack-"
    if (colon != std::string::npos) arch.resize(colon);
    std::string k = arch + ":" + std::to_string(p.multiProcessorCount);
    g_kind[dev] = k;
    return k;
}

}  // namespace

Variant variant_for(int op, int64_t n, bool boxes) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_table.empty()) return default_variant(boxes);
    const std::string k = device_kind_locked();
    auto it = g_table.find(std::make_tuple(k, op, size_class(n)));
    return it == g_table.end() ? default_variant(boxes) : it->second;
}

void variant_set(int op, int64_t n, const Variant *v) {
    std::lock_guard<std::mutex> lk(g_mu);
    const auto key = std::make_tuple(device_kind_locked(), op, size_class(n));
    if (v)
        g_table[key] = *v;
    else
        g_table.erase(key);
}

std::vector<Variant> candidates(bool boxes) {
    std::vector<Variant> c;
    for (int kr : {4, 8})
        for (int kd : {4, 8})
            for (int cu : {2, 4, 8})
                if (boxes || cu == 4) c.push_back(Variant{kr, kd, cu});
    return c;
}

hipError_t tune(int op, int64_t n, bool boxes, int reps, hipStream_t st,
                const std::function<hipError_t(Variant)> &call, Variant *chosen, float *best_ms,
                float *default_ms) {
    if (reps < 1) reps = 1;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    Variant best = default_variant(boxes);
    float best_t = 3.4e38f, def_t = -1.0f;
    for (const Variant &v : candidates(boxes)) {
        if (e != hipSuccess) break;
        if ((e = call(v)) != hipSuccess) break;  // warm-up
        std::vector<float> ts;
        for (int r = 0; r < reps && e == hipSuccess; ++r) {
            if ((e = hipEventRecord(a, st)) != hipSuccess) break;
            if ((e = call(v)) != hipSuccess) break;
            if ((e = hipEventRecord(b, st)) != hipSuccess) break;
            if ((e = hipEventSynchronize(b)) != hipSuccess) break;
            float ms = 0.0f;
            if ((e = hipEventElapsedTime(&ms, a, b)) != hipSuccess) break;
            ts.push_back(ms);
        }
        if (e != hipSuccess) break;
        std::sort(ts.begin(), ts.end());
        const float med = ts[ts.size() / 2];
        const Variant d = default_variant(boxes);
        if (v.kr == d.kr && v.kd == d.kd && v.cu == d.cu) def_t = med;
        if (med < best_t) best_t = med, best = v;
    }
    if (e == hipSuccess) e = call(best);  // the outputs come from the chosen variant
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (e != hipSuccess) return e;
    variant_set(op, n, &best);
    if (chosen) *chosen = best;
    if (best_ms) *best_ms = best_t;
    if (default_ms) *default_ms = def_t;
    return hipSuccess;
}

// Text format: a header line, then one line per entry:
//   <arch:CUs> <op> <size class> <kr> <kd> <cu>
bool tune_save(const char *path) {
    std::lock_guard<std::mutex> lk(g_mu);
    FILE *f = std::fopen(path, "w");
    if (!f) return false;
    bool ok = std::fprintf(f, "treebbox-tune 1\n") > 0;
    for (const auto &kv : g_table) {
        const auto &k = kv.first;
        const Variant &v = kv.second;
        ok = ok && std::fprintf(f, "%s %d %d %d %d %d\n", std::get<0>(k).c_str(), std::get<1>(k),
                                std::get<2>(k), v.kr, v.kd, v.cu) > 0;
    }
    return std::fclose(f) == 0 && ok;
}

// Entries that do not parse or name an invalid variant are skipped; entries
// for other device kinds are kept (they apply when such a device is current).
bool tune_load(const char *path) {
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[256];
    if (!std::fgets(line, sizeof line, f) || std::strncmp(line, "treebbox-tune 1", 15) != 0) {
        std::fclose(f);
        return false;
    }
    std::vector<std::pair<std::tuple<std::string, int, int>, Variant>> got;
    while (std::fgets(line, sizeof line, f)) {
        char kind[128];
        int op, cls;
        Variant v;
        if (std::sscanf(line, "%127s %d %d %d %d %d", kind, &op, &cls, &v.kr, &v.kd, &v.cu) != 6) continue;
        if (!variant_ok(v) || cls < 0 || cls > 62) continue;
        got.emplace_back(std::make_tuple(std::string(kind), op, cls), v);
    }
    std::fclose(f);
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto &kv : got) g_table[kv.first] = kv.second;
    return true;
}

void tune_clear() {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.clear();
}

}  // namespace tb

// Autotuner: times candidate engine settings on the resident graph and keeps
// the fastest.  Settings only change speed, never counts.
//
// Plain path: coordinate descent (two sweeps) over the push->pull threshold
// alpha, the pull->push threshold beta, the lane-serial bottom-up degree, the
// chunked bottom-up degree and the atomic top-down edge limit, timing queries
// at k = 2 and 3 from sample seeds.  Batched path: seeds per launch and the
// heavy-vertex threshold, timing a k = 3 batch.  Results are cached per
// (device architecture, graph content hash, seeds per launch) in memory and in
// a text file ($KHOP_TUNE_CACHE, default ~/.cache/khop/tune.txt).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <sys/stat.h>

#include "khop_impl.h"

namespace {

struct Tuned {
    int alpha, beta, pull_light, pull_heavy, push_atomic_max, batch_seeds, batch_heavy;
};

std::mutex g_cache_mu;
std::map<std::string, Tuned> g_cache;
bool g_cache_loaded = false;

std::string cache_path() {
    if (const char *p = std::getenv("KHOP_TUNE_CACHE")) return p;
    const char *home = std::getenv("HOME");
    return std::string(home ? home : "/tmp") + "/.cache/khop/tune.txt";
}

void load_cache() {
    if (g_cache_loaded) return;
    g_cache_loaded = true;
    FILE *f = std::fopen(cache_path().c_str(), "r");
    if (!f) return;
    char key[256];
    Tuned t;
    while (std::fscanf(f, "%255s %d %d %d %d %d %d %d", key, &t.alpha, &t.beta, &t.pull_light, &t.pull_heavy,
                       &t.push_atomic_max, &t.batch_seeds, &t.batch_heavy) == 8)
        g_cache[key] = t;
    std::fclose(f);
}

void save_cache() {
    const std::string p = cache_path();
    const size_t slash = p.rfind('/');
    if (slash != std::string::npos) {
        std::string dir = p.substr(0, slash);
        for (size_t i = 1; i <= dir.size(); ++i)
            if (i == dir.size() || dir[i] == '/') mkdir(dir.substr(0, i).c_str(), 0755);
    }
    FILE *f = std::fopen(p.c_str(), "w");
    if (!f) return;  // the cache is an optimisation only
    for (auto &kv : g_cache)
        std::fprintf(f, "%s %d %d %d %d %d %d %d\n", kv.first.c_str(), kv.second.alpha, kv.second.beta,
                     kv.second.pull_light, kv.second.pull_heavy, kv.second.push_atomic_max, kv.second.batch_seeds,
                     kv.second.batch_heavy);
    std::fclose(f);
}

Tuned current(const khop::Params &P) {
    return {P.alpha, P.beta, P.pull_light, P.pull_heavy, P.push_atomic_max, P.batch_seeds, P.batch_heavy};
}

void apply(khop::Params &P, const Tuned &t) {
    P.alpha = t.alpha;
    P.beta = t.beta;
    P.pull_light = t.pull_light;
    P.pull_heavy = t.pull_heavy;
    P.push_atomic_max = t.push_atomic_max;
    P.batch_seeds = t.batch_seeds;
    P.batch_heavy = t.batch_heavy;
}

// Deterministic sample of non-isolated vertices, spread over the id range.
std::vector<int32_t> sample_seeds(const khop_graph *g, int count) {
    std::vector<int32_t> cand;
    for (int64_t v = 0; v < g->n; ++v)
        if (g->h_outdeg[v] > 0) cand.push_back((int32_t)v);
    std::vector<int32_t> out;
    if (cand.empty()) return out;
    uint64_t x = 0x9e3779b97f4a7c15ull ^ g->hash;
    for (int i = 0; i < count; ++i) {
        x ^= x << 13;
        x ^= x >> 7;
        x ^= x << 17;
        out.push_back(cand[x % cand.size()]);
    }
    return out;
}

struct Bench {
    khop_graph *g;
    hipStream_t st;
    hipEvent_t e0, e1;
    int32_t *d_seeds;
    int64_t *d_counts, *d_te;
    int64_t n;
    khop::PlainCtx *pc;
};

float time_plain(Bench &b, int n_seeds) {
    KHOP_HIP(hipEventRecord(b.e0, b.st));
    for (int k : {2, 3}) khop::plain_run(b.g, b.pc, b.d_seeds, n_seeds, k, b.d_counts, b.d_te, b.st);
    KHOP_HIP(hipEventRecord(b.e1, b.st));
    KHOP_HIP(hipEventSynchronize(b.e1));
    float ms = 0;
    KHOP_HIP(hipEventElapsedTime(&ms, b.e0, b.e1));
    return ms;
}

float time_batched(Bench &b, const std::vector<int32_t> &ks) {
    KHOP_HIP(hipEventRecord(b.e0, b.st));
    khop::run_batched(b.g, b.d_seeds, ks.data(), (int64_t)ks.size(), b.d_counts, b.st);
    KHOP_HIP(hipEventRecord(b.e1, b.st));
    KHOP_HIP(hipEventSynchronize(b.e1));
    float ms = 0;
    KHOP_HIP(hipEventElapsedTime(&ms, b.e0, b.e1));
    return ms;
}

// Best of `reps` timings for the current parameters.
template <class F>
float best_of(F &&f, int reps) {
    float best = 1e30f;
    for (int r = 0; r < reps; ++r) best = std::min(best, f());
    return best;
}

}  // namespace

extern "C" int khop_autotune(khop_graph *g, int32_t seeds_per_launch) {
    try {
        if (!g) khop::fail(KHOP_EINVAL, "graph is NULL");
        if (seeds_per_launch != 0 && seeds_per_launch != 64 && seeds_per_launch != 128 && seeds_per_launch != 256 &&
            seeds_per_launch != 512 && seeds_per_launch != 1024)
            khop::fail(KHOP_EINVAL, "seeds_per_launch must be 0, 64, 128, 256, 512 or 1024");
        KHOP_HIP(hipSetDevice(g->device));
        hipDeviceProp_t prop;
        KHOP_HIP(hipGetDeviceProperties(&prop, g->device));
        char keybuf[200];
        std::snprintf(keybuf, sizeof(keybuf), "%s:%016llx:%lld:%d", prop.gcnArchName, (unsigned long long)g->hash,
                      (long long)g->n, seeds_per_launch);
        std::string key(keybuf);
        for (char &c : key)
            if (c == ' ') c = '_';
        {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            load_cache();
            auto it = g_cache.find(key);
            if (it != g_cache.end()) {
                apply(g->params, it->second);
                return KHOP_OK;
            }
        }
        const int plain_seeds = 48, batch_seeds = 1024;
        std::vector<int32_t> seeds = sample_seeds(g, batch_seeds);
        if (seeds.empty()) return KHOP_OK;  // no edges: nothing to tune
        Bench b{g, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, g->n, nullptr};
        KHOP_HIP(hipStreamCreateWithFlags(&b.st, hipStreamNonBlocking));
        KHOP_HIP(hipEventCreate(&b.e0));
        KHOP_HIP(hipEventCreate(&b.e1));
        const bool prof_on = g->prof.on;
        g->prof.on = false;
        struct Cleanup {
            Bench &b;
            khop_graph *g;
            bool prof_on;
            ~Cleanup() {
                if (b.st) (void)hipStreamSynchronize(b.st);
                if (b.pc) khop::plain_ctx_destroy(b.pc);
                (void)hipFree(b.d_seeds);
                (void)hipFree(b.d_counts);
                (void)hipFree(b.d_te);
                if (b.e0) (void)hipEventDestroy(b.e0);
                if (b.e1) (void)hipEventDestroy(b.e1);
                if (b.st) (void)hipStreamDestroy(b.st);
                g->prof.on = prof_on;
            }
        } cleanup{b, g, prof_on};
        if (hipMalloc(&b.d_seeds, seeds.size() * 4) != hipSuccess ||
            hipMalloc(&b.d_counts, seeds.size() * 8) != hipSuccess || hipMalloc(&b.d_te, seeds.size() * 8) != hipSuccess) {
            (void)hipGetLastError();
            khop::fail(KHOP_ENOMEM, "device allocation for autotuning failed");
        }
        KHOP_HIP(hipMemcpy(b.d_seeds, seeds.data(), seeds.size() * 4, hipMemcpyHostToDevice));
        b.pc = khop::plain_ctx_create(g);
        khop::Params &P = g->params;
        const int saved_dir = P.dir_mode;
        P.dir_mode = KHOP_DIR_AUTO;

        // ---- plain path: coordinate descent
        auto plain_cost = [&] { return best_of([&] { return time_plain(b, plain_seeds); }, 2); };
        time_plain(b, plain_seeds);  // warm-up (contexts, chunk tables)
        struct Knob {
            int *field;
            std::vector<int> values;
        };
        std::vector<Knob> knobs = {{&P.alpha, {2, 4, 8, 14, 24, 48, 96}},
                                   {&P.beta, {6, 12, 24, 48, 96}},
                                   {&P.pull_light, {8, 16, 32, 64, 128}},
                                   {&P.pull_heavy, {512, 1024, 4096, 16384, 65536}},
                                   {&P.push_atomic_max, {4096, 16384, 65536, 262144, 1048576}}};
        float best = plain_cost();
        for (int sweep = 0; sweep < 2; ++sweep)
            for (auto &kn : knobs) {
                int keep = *kn.field;
                for (int v : kn.values) {
                    if (v == keep) continue;
                    *kn.field = v;
                    float t = plain_cost();
                    if (t < best * 0.98f) {
                        best = t;
                        keep = v;
                    }
                }
                *kn.field = keep;
            }

        // ---- batched path
        std::vector<int32_t> ks(seeds.size(), 3);
        auto batch_cost = [&] { return best_of([&] { return time_batched(b, ks); }, 2); };
        std::vector<int> per = seeds_per_launch ? std::vector<int>{seeds_per_launch}
                                                : std::vector<int>{64, 128, 256, 512, 1024};
        float bbest = 1e30f;
        int best_per = P.batch_seeds, best_heavy = P.batch_heavy;
        for (int ps : per) {
            P.batch_seeds = ps;
            for (int hv : {64, 128, 256, 512, 2048}) {
                P.batch_heavy = hv;
                float t = batch_cost();
                if (t < bbest) {
                    bbest = t;
                    best_per = ps;
                    best_heavy = hv;
                }
            }
        }
        P.batch_seeds = best_per;
        P.batch_heavy = best_heavy;
        P.dir_mode = saved_dir;
        {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            g_cache[key] = current(P);
            save_cache();
        }
        return KHOP_OK;
    } catch (const khop::Error &e) {
        khop::set_last_error(e.msg);
        return e.status;
    } catch (...) {
        khop::set_last_error("internal error in autotuning");
        return KHOP_EINTERNAL;
    }
}

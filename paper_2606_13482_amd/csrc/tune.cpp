// Run-time choice of launch shapes (the library's autotuner).  A tunable
// kernel times its candidate shapes on the device the first time it meets a
// new problem shape (matrix size, column count, precision) and keeps the
// fastest for the process; with BIE_AUTOTUNE_CACHE naming a file, choices are
// also appended there and read back by later processes.  BIE_AUTOTUNE=0 or
// bie_autotune(0) keeps every kernel at its fixed default shape.
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

#include "bie_internal.hpp"

namespace bie {

namespace {
std::mutex g_mu;
std::map<std::string, std::vector<int>> g_choice;
bool g_loaded = false;
int g_enabled = -1;   // -1: not yet read from the environment

void load_locked()
{
    if (g_loaded) return;
    g_loaded = true;
    const char *path = getenv("BIE_AUTOTUNE_CACHE");
    if (!path) return;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string key;
        if (!(is >> key)) continue;
        std::vector<int> v;
        int x;
        while (is >> x) v.push_back(x);
        if (!v.empty()) g_choice[key] = v;
    }
}
}  // namespace

bool tune_enabled()
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_enabled < 0) {
        const char *e = getenv("BIE_AUTOTUNE");
        g_enabled = (e && atoi(e) == 0) ? 0 : 1;
    }
    return g_enabled != 0;
}

void tune_set_enabled(bool on)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_enabled = on ? 1 : 0;
}

bool tune_get(const std::string &key, std::vector<int> &v)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    auto it = g_choice.find(key);
    if (it == g_choice.end()) return false;
    v = it->second;
    return true;
}

void tune_put(const std::string &key, const std::vector<int> &v)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    g_choice[key] = v;
    if (const char *path = getenv("BIE_AUTOTUNE_CACHE")) {
        std::ofstream f(path, std::ios::app);
        f << key;
        for (int x : v) f << " " << x;
        f << "\n";
    }
}

std::string tune_report()
{
    std::lock_guard<std::mutex> lk(g_mu);
    std::string out;
    for (const auto &kv : g_choice) {
        out += kv.first;
        for (int x : kv.second) out += " " + std::to_string(x);
        out += "\n";
    }
    return out;
}

bool stream_capturing(hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) return true;   // unsure: do not time
    return st != hipStreamCaptureStatusNone;
}

// Times fn() with HIP events on s: one untimed launch, then the mean of `reps`.
float time_launches(hipStream_t s, int reps, const std::function<void()> &fn)
{
    hipEvent_t e0, e1;
    BIE_HIP(hipEventCreate(&e0));
    BIE_HIP(hipEventCreate(&e1));
    fn();
    BIE_HIP(hipEventRecord(e0, s));
    for (int i = 0; i < reps; ++i) fn();
    BIE_HIP(hipEventRecord(e1, s));
    const hipError_t es = hipEventSynchronize(e1);
    float ms = 0.f;
    if (es == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    BIE_HIP(es);
    return ms / float(reps);
}

}  // namespace bie

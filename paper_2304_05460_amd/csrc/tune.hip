// Autotuner of launch shapes: the tile-kernel variant of the kernel matvec
// (d = 5..8), the split count of the split-K GEMMs and the split count of
// the GEMVs.  Each tunable has a short list of candidates that compute the
// same result up to the order of the sums; the first call that meets a new
// shape class times every candidate on the caller's own buffers and keeps the
// fastest.  Decisions are kept per process and, if a cache file is set,
// written to it and read back by later processes.
#include <chrono>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "afn_internal.h"
#include "group.h"

namespace afn {
namespace {

struct Decision {
    int choice = 0;
    std::vector<float> ms;       // per-candidate time (empty when read from a file)
};

std::mutex g_mu;
int g_mode = AFN_TUNE_OFF;
int g_force = 0;
std::string g_path;
std::map<std::string, Decision> g_table;

std::string device_tag()
{
    int dev = 0;
    hipDeviceProp_t p{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    char buf[96];
    snprintf(buf, sizeof buf, "%s/%dcu", p.gcnArchName, p.multiProcessorCount);
    for (char *c = buf; *c; ++c)
        if (*c == ' ' || *c == ':') *c = '_';
    return buf;
}

void write_file_locked()
{
    if (g_path.empty()) return;
    FILE *f = fopen(g_path.c_str(), "w");
    if (!f) return;
    for (const auto &kv : g_table) fprintf(f, "%s %d\n", kv.first.c_str(), kv.second.choice);
    fclose(f);
}

afn_status read_file_locked(const std::string &path)
{
    FILE *f = fopen(path.c_str(), "r");
    if (!f) return AFN_OK;       // no cache yet
    char key[512];
    int choice = 0;
    while (fscanf(f, "%511s %d", key, &choice) == 2) {
        Decision d;
        d.choice = choice;
        g_table[key] = d;
    }
    fclose(f);
    return AFN_OK;
}

}  // namespace

int tune_pick(const char *kernel, const std::string &shape, int ncand, int heuristic,
              const std::function<afn_status(int)> &run, hipStream_t s)
{
    if (ncand <= 1) return 0;
    int mode, force;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        mode = g_mode;
        force = g_force;
    }
    if (mode == AFN_TUNE_OFF) return heuristic;
    if (mode == AFN_TUNE_FORCE) return force < ncand ? (force < 0 ? 0 : force) : ncand - 1;
    const std::string key = std::string(kernel) + "|" + shape + "|" + device_tag();
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_table.find(key);
        if (it != g_table.end()) return it->second.choice < ncand ? it->second.choice : heuristic;
    }
    // no timing while the stream records a graph: the heuristic until a
    // later eager call decides
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
        (void)hipGetLastError();
        return heuristic;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipGetLastError();
        if (e0) (void)hipEventDestroy(e0);
        return heuristic;
    }
    Decision d;
    d.ms.assign(ncand, 0.f);
    bool ok = true;
    constexpr int kReps = 3;
    // the timed runs go to the stream at once, also while a unit of work is
    // being recorded for a grouped launch (they write only the launch's own
    // outputs, which the recorded launch writes again)
    RecorderPause pause;
    for (int c = 0; c < ncand && ok; ++c) {
        ok = run(c) == AFN_OK;                     // warm-up
        if (!ok) break;
        ok = hipEventRecord(e0, s) == hipSuccess;
        for (int r = 0; r < kReps && ok; ++r) ok = run(c) == AFN_OK;
        ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
        float t = 0.f;
        ok = ok && hipEventElapsedTime(&t, e0, e1) == hipSuccess;
        d.ms[c] = t / kReps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!ok) {
        (void)hipGetLastError();
        return heuristic;
    }
    d.choice = 0;
    for (int c = 1; c < ncand; ++c)
        if (d.ms[c] < d.ms[d.choice]) d.choice = c;
    std::lock_guard<std::mutex> lk(g_mu);
    g_table[key] = d;
    write_file_locked();
    return d.choice;
}

}  // namespace afn

extern "C" {

afn_status afn_tune_config(int32_t mode, int32_t index, const char *cache_path)
{
    afn::clear_error();
    if (mode < AFN_TUNE_OFF || mode > AFN_TUNE_FORCE || index < 0) {
        afn::set_error("afn_tune_config: invalid argument (mode %d, index %d)", mode, index);
        return AFN_EINVAL;
    }
    std::lock_guard<std::mutex> lk(afn::g_mu);
    afn::g_mode = mode;
    afn::g_force = index;
    afn::g_path = cache_path ? cache_path : "";
    if (!afn::g_path.empty()) return afn::read_file_locked(afn::g_path);
    return AFN_OK;
}

afn_status afn_tune_report(char *buf_host, int64_t cap, int64_t *len)
{
    afn::clear_error();
    if (!len || cap < 0 || (cap > 0 && !buf_host)) {
        afn::set_error("afn_tune_report: invalid argument");
        return AFN_EINVAL;
    }
    std::string out;
    {
        std::lock_guard<std::mutex> lk(afn::g_mu);
        for (const auto &kv : afn::g_table) {
            out += kv.first + " " + std::to_string(kv.second.choice);
            for (float t : kv.second.ms) {
                char b[32];
                snprintf(b, sizeof b, " %.6f", t);
                out += b;
            }
            out += "\n";
        }
    }
    *len = (int64_t)out.size();
    if (cap > 0) {
        const size_t m = (size_t)cap - 1 < out.size() ? (size_t)cap - 1 : out.size();
        memcpy(buf_host, out.data(), m);
        buf_host[m] = 0;
    }
    return AFN_OK;
}

}  // extern "C"

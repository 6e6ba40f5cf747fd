// The autotuner's cache: the schedule chosen for a class of batches, kept in
// a small JSON file so that later plans of the same class skip the trial
// launches (and pick the same schedule every time).
//
// A class is (GPU architecture, field, whether every source row is 4-byte
// aligned, the number of generations, and the byte-madd-weighted means of N,
// K and the packet length, each in half-octave buckets), plus any knobs the
// caller fixed.  The file is GFNC_TUNE_CACHE if that is set ("off" disables
// the cache), else gfnc_tune.json beside the library.
#include <dlfcn.h>
#include <hip/hip_runtime.h>
#include <unistd.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "gf_internal.h"

namespace gfnc {

namespace {

std::mutex g_tune_mu;
bool g_loaded = false;
std::map<std::string, TuneChoice> g_cache;

std::string cache_path()
{
    const char *env = getenv("GFNC_TUNE_CACHE");
    if (env && *env)
        return strcmp(env, "off") == 0 ? std::string() : std::string(env);
    Dl_info info;
    if (dladdr(reinterpret_cast<void *>(&cache_path), &info) && info.dli_fname) {
        std::string so = info.dli_fname;
        const size_t slash = so.rfind('/');
        return (slash == std::string::npos ? std::string(".") : so.substr(0, slash)) + "/gfnc_tune.json";
    }
    return std::string();
}

// Value of "name": after `from` and before `end` in s, as a double.
bool field_num(const std::string &s, size_t from, size_t end, const char *name, double *out)
{
    const std::string pat = std::string("\"") + name + "\":";
    const size_t at = s.find(pat, from);
    if (at == std::string::npos || at >= end)
        return false;
    *out = strtod(s.c_str() + at + pat.size(), nullptr);
    return true;
}

// Reads the entries of a file this code wrote: {"version": 1, "entries": [
// {"key": "...", "form": F, "bytes_per_lane": B, "grid_pct": G, "ms": T}, ...]}.
void load_locked()
{
    g_loaded = true;
    const std::string path = cache_path();
    if (path.empty())
        return;
    FILE *f = fopen(path.c_str(), "rb");
    if (!f)
        return;
    std::string s;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof buf, f)) > 0)
        s.append(buf, n);
    fclose(f);
    size_t pos = 0;
    const std::string kpat = "\"key\": \"";
    while ((pos = s.find(kpat, pos)) != std::string::npos) {
        const size_t k0 = pos + kpat.size();
        const size_t k1 = s.find('"', k0);
        const size_t end = s.find('}', k0);
        if (k1 == std::string::npos || end == std::string::npos)
            break;
        double form = 0, bpl = 0, pct = 0, ms = 0;
        if (field_num(s, k1, end, "form", &form) && field_num(s, k1, end, "bytes_per_lane", &bpl) &&
            field_num(s, k1, end, "grid_pct", &pct) && field_num(s, k1, end, "ms", &ms) && form >= 1 &&
            form <= 5 && (bpl == 0 || bpl == 4 || bpl == 8 || bpl == 16) && pct >= 0 && pct <= 100 && (pct > 0 || form == 1 || form == 3))
            g_cache[s.substr(k0, k1 - k0)] = TuneChoice{(int)form, (int)bpl / 4, (int)pct, ms};
        pos = end;
    }
}

void save_locked()
{
    const std::string path = cache_path();
    if (path.empty())
        return;
    const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
    FILE *f = fopen(tmp.c_str(), "wb");
    if (!f)
        return;
    fprintf(f, "{\"version\": 1, \"entries\": [\n");
    size_t i = 0;
    for (const auto &kv : g_cache) {
        fprintf(f, " {\"key\": \"%s\", \"form\": %d, \"bytes_per_lane\": %d, \"grid_pct\": %d, \"ms\": %.4f}%s\n",
                kv.first.c_str(), kv.second.form, 4 * kv.second.fixed_D, kv.second.grid_pct, kv.second.ms,
                ++i < g_cache.size() ? "," : "");
    }
    fprintf(f, "]}\n");
    const bool ok = fclose(f) == 0;
    if (!ok || rename(tmp.c_str(), path.c_str()) != 0)
        remove(tmp.c_str());
}

int half_octave(double x) { return x > 0 ? (int)std::floor(2.0 * std::log2(x)) : -1; }

}  // namespace

std::string tune_key(int field, const std::vector<DevGen> &g, bool aligned4, int req_form, int req_bpl, int req_grid)
{
    char arch[64] = "unknown";
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        strncpy(arch, prop.gcnArchName, sizeof arch - 1);
        arch[sizeof arch - 1] = 0;
        if (char *colon = strchr(arch, ':'))
            *colon = 0;
    }
    double w = 0, wn = 0, wk = 0, wl = 0;
    for (const DevGen &x : g) {
        const double m = (double)x.K * (double)x.N * (double)x.len;
        w += m;
        wn += m * x.N;
        wk += m * x.K;
        wl += m * (double)x.len;
    }
    char key[256];
    snprintf(key, sizeof key, "%s|f%d|a%d|c%d|n%d|k%d|p%d|t%d.%d.%d", arch, field, aligned4 ? 1 : 0,
             half_octave((double)g.size()), half_octave(w > 0 ? wn / w : 0), half_octave(w > 0 ? wk / w : 0),
             half_octave(w > 0 ? wl / w : 0), req_form, req_bpl, req_grid);
    return key;
}

bool tune_cache_get(const std::string &key, TuneChoice *out)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_loaded)
        load_locked();
    auto it = g_cache.find(key);
    if (it == g_cache.end())
        return false;
    *out = it->second;
    return true;
}

void tune_cache_put(const std::string &key, const TuneChoice &c)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_loaded)
        load_locked();
    g_cache[key] = c;
    save_locked();
}

}  // namespace gfnc

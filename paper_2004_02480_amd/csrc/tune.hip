// tune.hip -- the store of tuned launch choices, shared by the persistent
// solve (grid x lanes per row), the multi-right-hand-side solve (row tiles
// per workgroup) and the batched solve (split plan and queue order).
//
// Entries are keyed by a text key naming the kernel family and the shape
// and dtypes it was measured on, prefixed with the GPU's architecture name,
// so a cache file written on one MI355X is valid on another and ignored on
// other hardware.  A cache file is plain text: a header line carrying the
// library version (files of another version are ignored as a whole), then
// one entry per line, "key<TAB>a<TAB>b<TAB>us".  The store is guarded by a
// mutex.  When the environment variable CSK_TUNE_CACHE names a file, the
// store is read from it on first use and written back after every tuning
// call.
#include "csk_internal.h"
#include "csk_tune.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace csk {
namespace {

std::mutex g_mu;
std::map<std::string, TuneRec> g_store;
bool g_env_loaded = false;

constexpr const char* kHeader = "# csk tune cache, library version ";

// Reads entries of `path` into the store (caller holds the lock).  Returns
// the number of entries read, or -1 when the file is missing, unreadable or
// of another library version.
int load_locked(const char* path)
{
    FILE* f = std::fopen(path, "r");
    if (!f) return -1;
    char line[1024];
    int count = 0;
    bool ok = false;
    if (std::fgets(line, sizeof line, f)) {
        char want[128];
        std::snprintf(want, sizeof want, "%s%d", kHeader, (int)csk_version());
        ok = std::strncmp(line, want, std::strlen(want)) == 0;
    }
    while (ok && std::fgets(line, sizeof line, f)) {
        char* tab1 = std::strchr(line, '\t');
        if (!tab1) continue;
        *tab1 = 0;
        TuneRec r{};
        if (std::sscanf(tab1 + 1, "%d\t%d\t%lf", &r.a, &r.b, &r.us) != 3) continue;
        g_store[std::string(line)] = r;
        ++count;
    }
    std::fclose(f);
    return ok ? count : -1;
}

// Writes the whole store to `path` through a temporary file (caller holds
// the lock).
bool save_locked(const char* path)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return false;
    std::fprintf(f, "%s%d\n", kHeader, (int)csk_version());
    for (const auto& kv : g_store) std::fprintf(f, "%s\t%d\t%d\t%.6f\n", kv.first.c_str(), kv.second.a, kv.second.b, kv.second.us);
    const bool good = std::fflush(f) == 0;
    std::fclose(f);
    return good && std::rename(tmp.c_str(), path) == 0;
}

void env_load_locked()
{
    if (g_env_loaded) return;
    g_env_loaded = true;
    const char* p = std::getenv("CSK_TUNE_CACHE");
    if (p && *p) load_locked(p);
}

}  // namespace

std::string device_arch()
{
    static std::mutex mu;
    static std::vector<std::string> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return "unknown";
    std::lock_guard<std::mutex> lock(mu);
    if ((int)cache.size() <= dev) cache.resize(dev + 1);
    if (cache[dev].empty()) {
        hipDeviceProp_t prop;
        cache[dev] = (hipGetDeviceProperties(&prop, dev) == hipSuccess) ? std::string(prop.gcnArchName) : "unknown";
    }
    return cache[dev];
}

std::string tune_key(const char* fmt, ...)
{
    char body[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(body, sizeof body, fmt, ap);
    va_end(ap);
    return device_arch() + "|" + body;
}

void tune_put(const std::string& key, const TuneRec& r)
{
    std::lock_guard<std::mutex> lock(g_mu);
    env_load_locked();
    g_store[key] = r;
    const char* p = std::getenv("CSK_TUNE_CACHE");
    if (p && *p) save_locked(p);
}

bool tune_get(const std::string& key, TuneRec* out)
{
    std::lock_guard<std::mutex> lock(g_mu);
    env_load_locked();
    const auto it = g_store.find(key);
    if (it == g_store.end()) return false;
    if (out) *out = it->second;
    return true;
}

void tune_reset()
{
    std::lock_guard<std::mutex> lock(g_mu);
    g_store.clear();
    g_env_loaded = true;  // an explicit clear is not undone by the environment's file
}

int tune_load_file(const char* path)
{
    std::lock_guard<std::mutex> lock(g_mu);
    return load_locked(path);
}

bool tune_save_file(const char* path)
{
    std::lock_guard<std::mutex> lock(g_mu);
    return save_locked(path);
}

int tune_count()
{
    std::lock_guard<std::mutex> lock(g_mu);
    return (int)g_store.size();
}

}  // namespace csk

// tune.cpp -- launch-shape tuning and launch logging shared by the kernels'
// launchers: the autotune cache file, the KAPPA_AUTOTUNE policy, the
// single-species tuned shapes, and KAPPA_LOG launch lines.
//
// Environment:
//   KAPPA_AUTOTUNE_CACHE=<path>  a flat JSON object {"key": "block,unroll,grid"}
//                               holding tuned shapes across processes;
//   KAPPA_AUTOTUNE=off|use|refresh  off: the cache is neither read nor written;
//                               use (default): plans and single-species launches
//                               start from the cached shape, and tuning writes it;
//                               refresh: the cache is not read (defaults until
//                               tuned), and tuning writes it;
//   KAPPA_LOG=1                 one line on stderr per kernel launch: kernel,
//                               precision, particles, grid, block, particles per
//                               thread, stream.
// None of these changes any output: every kernel's result is independent of
// its launch shape.
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "kappa_internal.hpp"

namespace kappa {

namespace {

std::mutex g_cache_mutex;

std::map<std::string, std::string> read_cache_file(const char *path)
{
    std::map<std::string, std::string> m;
    FILE *f = std::fopen(path, "r");
    if (!f) return m;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    std::fclose(f);
    // "k": "v" pairs
    size_t pos = 0;
    while (true) {
        const size_t k0 = text.find('"', pos);
        if (k0 == std::string::npos) break;
        const size_t k1 = text.find('"', k0 + 1);
        const size_t v0 = k1 == std::string::npos ? k1 : text.find('"', k1 + 1);
        const size_t v1 = v0 == std::string::npos ? v0 : text.find('"', v0 + 1);
        if (v1 == std::string::npos) break;
        m[text.substr(k0 + 1, k1 - k0 - 1)] = text.substr(v0 + 1, v1 - v0 - 1);
        pos = v1 + 1;
    }
    return m;
}

void write_cache_file(const char *path, const std::map<std::string, std::string> &m)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{\n");
    size_t i = 0;
    for (const auto &kv : m)
        std::fprintf(f, "  \"%s\": \"%s\"%s\n", kv.first.c_str(), kv.second.c_str(), ++i < m.size() ? "," : "");
    std::fprintf(f, "}\n");
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

// single-species shapes of this process, keyed by forward_tune_key: tuned
// here, or looked up once in the cache file (grid 0 marks a key the file
// does not hold), so that a launch reads the file at most once per key
std::mutex g_fwd_mutex;
std::map<std::string, Shape> g_fwd_tuned;

}  // namespace

int autotune_policy()
{
    static const int policy = [] {
        const char *env = std::getenv("KAPPA_AUTOTUNE");
        if (!env || !*env || std::strcmp(env, "use") == 0) return kTuneUse;
        if (std::strcmp(env, "off") == 0) return kTuneOff;
        if (std::strcmp(env, "refresh") == 0) return kTuneRefresh;
        return kTuneUse;
    }();
    return policy;
}

bool cache_lookup(const std::string &key, Shape &shape)
{
    const char *path = std::getenv("KAPPA_AUTOTUNE_CACHE");
    if (!path || autotune_policy() != kTuneUse) return false;
    std::lock_guard<std::mutex> lock(g_cache_mutex);
    const auto m = read_cache_file(path);
    const auto it = m.find(key);
    Shape s{};
    if (it == m.end() || std::sscanf(it->second.c_str(), "%d,%d,%d", &s.block, &s.unroll, &s.grid) != 3) return false;
    shape = s;
    return true;
}

void cache_store(const std::string &key, const Shape &shape)
{
    const char *path = std::getenv("KAPPA_AUTOTUNE_CACHE");
    if (!path || autotune_policy() == kTuneOff) return;
    std::lock_guard<std::mutex> lock(g_cache_mutex);
    auto m = read_cache_file(path);
    char val[64];
    std::snprintf(val, sizeof val, "%d,%d,%d", shape.block, shape.unroll, shape.grid);
    m[key] = val;
    write_cache_file(path, m);
}

int size_bucket(uint64_t n)
{
    int b = 0;
    while ((1ull << b) < n && b < 63) ++b;
    return b;
}

std::string forward_tune_key(int mode, uint64_t n)
{
    char buf[64];
    std::snprintf(buf, sizeof buf, "forward|mode%d|n2^%d", mode, size_bucket(n));
    return buf;
}

bool forward_tuned(int mode, uint64_t n, Shape &shape)
{
    const std::string key = forward_tune_key(mode, n);
    std::lock_guard<std::mutex> lock(g_fwd_mutex);
    auto it = g_fwd_tuned.find(key);
    if (it == g_fwd_tuned.end()) {
        Shape s{0, 0, 0};
        if (!cache_lookup(key, s)) s = Shape{0, 0, 0};
        it = g_fwd_tuned.emplace(key, Shape{s.block, s.unroll, s.block > 0 ? 1 : 0}).first;
    }
    if (it->second.grid == 0) return false;
    shape = it->second;
    return true;
}

void set_forward_tuned(int mode, uint64_t n, const Shape &shape)
{
    const std::string key = forward_tune_key(mode, n);
    {
        std::lock_guard<std::mutex> lock(g_fwd_mutex);
        g_fwd_tuned[key] = Shape{shape.block, shape.unroll, 1};
    }
    cache_store(key, shape);
}

bool log_enabled()
{
    static const bool on = [] {
        const char *env = std::getenv("KAPPA_LOG");
        return env && *env && std::strcmp(env, "0") != 0;
    }();
    return on;
}

void log_launch(const char *kernel, int mode, uint64_t n, const Shape &shape, const void *stream)
{
    if (!log_enabled()) return;
    static const char *names[] = {"FP64", "FP32", "FP32_NOTAIL"};
    std::fprintf(stderr, "[kappa] %s precision=%s n=%llu grid=%d block=%d per_thread=%d stream=%p\n", kernel,
                 mode >= 0 && mode < 3 ? names[mode] : "?", static_cast<unsigned long long>(n), shape.grid,
                 shape.block, shape.unroll, stream);
}

}  // namespace kappa

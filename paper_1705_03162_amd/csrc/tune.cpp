#include "tune.hpp"

#include <dlfcn.h>

#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "plan_core.hpp"

namespace sw {

namespace {

std::once_flag g_once;
std::map<std::pair<int, int>, std::pair<int, int>> g_table;
std::map<std::pair<int, int>, int> g_classic;
std::map<std::pair<int, int>, int> g_batch;

std::string table_path()
{
    if (const char *env = std::getenv("SWEPT_TUNE_FILE")) return env;
    Dl_info info;
    if (dladdr((void *)&tuned_shape, &info) && info.dli_fname) {
        std::string lib = info.dli_fname;
        size_t slash = lib.rfind('/');
        std::string dir = slash == std::string::npos ? "." : lib.substr(0, slash);
        return dir + "/tune_gfx950.txt";
    }
    return "tune_gfx950.txt";
}

void load()
{
    FILE *f = std::fopen(table_path().c_str(), "r");
    if (!f) return;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        int scheme, lg, width, threads;
        if (std::sscanf(line, "classic %d %d %d", &scheme, &lg, &threads) == 3)
            g_classic[{scheme, lg}] = threads;
        else if (std::sscanf(line, "batch %d %d %d", &scheme, &lg, &width) == 3)
            g_batch[{scheme, lg}] = width;   // points per lane
        else if (std::sscanf(line, "%d %d %d %d", &scheme, &lg, &width, &threads) == 4)
            g_table[{scheme, lg}] = {width, threads};
    }
    std::fclose(f);
}

}  // namespace

static int size_class(int64_t n)
{
    int lg = 0;
    while (lg < 62 && ((int64_t)1 << (lg + 1)) <= n) ++lg;
    return lg;
}

bool tuned_classic_threads(const sw_problem &p, int *threads)
{
    std::call_once(g_once, load);
    const int lg = size_class(p.n);
    auto it = g_classic.end();
    for (int c = lg; c >= 0 && it == g_classic.end(); --c) it = g_classic.find({p.scheme, c});
    for (int c = lg + 1; c <= 62 && it == g_classic.end(); ++c) it = g_classic.find({p.scheme, c});
    if (it == g_classic.end() || !legal_threads(it->second)) return false;
    *threads = it->second;
    return true;
}

bool tuned_batch_points(const sw_problem &p, int *points)
{
    std::call_once(g_once, load);
    const int lg = size_class(p.n);
    auto it = g_batch.end();
    for (int c = lg; c >= 0 && it == g_batch.end(); --c) it = g_batch.find({p.scheme, c});
    for (int c = lg + 1; c <= 62 && it == g_batch.end(); ++c) it = g_batch.find({p.scheme, c});
    if (it == g_batch.end()) return false;
    *points = it->second;
    return true;
}

bool tuned_shape(const sw_problem &p, int *width, int *threads)
{
    std::call_once(g_once, load);
    const int lg = size_class(p.n);
    // the measured size class of n, else the nearest smaller one (beyond the largest
    // measured class the device is saturated), else the nearest larger one
    auto it = g_table.end();
    for (int c = lg; c >= 0 && it == g_table.end(); --c) it = g_table.find({p.scheme, c});
    for (int c = lg + 1; c <= 62 && it == g_table.end(); ++c) it = g_table.find({p.scheme, c});
    if (it == g_table.end()) return false;
    const int w = it->second.first, t = it->second.second;
    if (w <= 0 || t <= 0 || p.n % w != 0) return false;
    Geom g;
    std::string err;
    if (make_geom(p, w, t, &g, &err) != 0) return false;
    *width = w;
    *threads = t;
    return true;
}

}  // namespace sw

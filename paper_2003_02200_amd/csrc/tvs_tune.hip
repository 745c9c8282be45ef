// tvs_tune.hip -- launch shapes chosen by timing, remembered per device and library build.
//
// The batched sweep picks its launch shape (waves per workgroup, workgroups per CU or one workgroup
// per item) per bucket of tiles, and the single-grid sweep its waves per workgroup, by timing
// candidates (TVS_FLAG_AUTOTUNE). A choice is keyed by the kind of launch, the decision precision and
// slope form, and the size class of the longest skewed row and of the longest line of sight. Choices
// are kept in memory and appended to a text file (TVS_TUNE_CACHE, else $XDG_CACHE_HOME/libtvs or
// ~/.cache/libtvs) whose lines also name the device and the hash of the library sources the build
// was made from: a later process on the same device and build starts with them, other builds and
// devices ignore them. A cache that cannot be read or written only costs the timing again.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "tvs_host.h"

#ifndef TVS_SOURCE_HASH
#define TVS_SOURCE_HASH "unknown"
#endif

namespace tvs {
namespace host {

namespace {

std::mutex g_mu;
bool g_loaded[64];
std::map<std::tuple<int, int, int, int, int, int>, std::pair<int, int>> g_map;  // (dev, key...) -> (a, b)
std::string g_dev_id[64];

std::string cache_path() {
    if (const char *p = getenv("TVS_TUNE_CACHE")) return p;
    std::string dir;
    if (const char *x = getenv("XDG_CACHE_HOME")) dir = std::string(x) + "/libtvs";
    else if (const char *h = getenv("HOME")) dir = std::string(h) + "/.cache/libtvs";
    else return "";
    return dir + "/tune-v1.txt";
}

void make_parent(const std::string &path) {
    // create the cache's directory (and its parent, the usual ~/.cache) when missing
    const size_t s = path.rfind('/');
    if (s == std::string::npos || s == 0) return;
    const std::string dir = path.substr(0, s);
    const size_t s2 = dir.rfind('/');
    if (s2 != std::string::npos && s2 > 0) (void)mkdir(dir.substr(0, s2).c_str(), 0755);
    (void)mkdir(dir.c_str(), 0755);
}

// Name, architecture and CU count of the device, without blanks.
std::string device_id(int dev) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "dev" + std::to_string(dev);
    std::string s = std::string(p.gcnArchName) + "/" + std::to_string(p.multiProcessorCount) + "/" + p.name;
    for (char &c : s)
        if (c == ' ' || c == '\t' || c == '\n') c = '_';
    return s;
}

// Reads the file's choices for this device and build (caller holds g_mu).
void load(int dev) {
    if (g_loaded[dev]) return;
    g_loaded[dev] = true;
    g_dev_id[dev] = device_id(dev);
    const std::string path = cache_path();
    if (path.empty()) return;
    FILE *f = fopen(path.c_str(), "r");
    if (!f) return;
    char build[128], devid[512];
    int kind, f64, rcp, sb, rb, a, b;
    while (fscanf(f, "%127s %511s %d %d %d %d %d %d %d", build, devid, &kind, &f64, &rcp, &sb, &rb, &a, &b) == 9)
        if (strcmp(build, TVS_SOURCE_HASH) == 0 && g_dev_id[dev] == devid)
            g_map[std::make_tuple(dev, kind, f64, rcp, sb, rb)] = std::make_pair(a, b);
    fclose(f);
}

}  // namespace

const char *source_hash() { return TVS_SOURCE_HASH; }

bool tune_lookup(const TuneKey &k, int &a, int &b) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return false;
    std::lock_guard<std::mutex> g(g_mu);
    load(dev);
    auto it = g_map.find(std::make_tuple(dev, k.kind, k.f64, k.rcp, k.side_b, k.rho_b));
    if (it == g_map.end()) return false;
    a = it->second.first;
    b = it->second.second;
    return true;
}

void tune_store(const TuneKey &k, int a, int b) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return;
    std::lock_guard<std::mutex> g(g_mu);
    load(dev);
    g_map[std::make_tuple(dev, k.kind, k.f64, k.rcp, k.side_b, k.rho_b)] = std::make_pair(a, b);
    const std::string path = cache_path();
    if (path.empty()) return;
    make_parent(path);
    FILE *f = fopen(path.c_str(), "a");
    if (!f) return;
    fprintf(f, "%s %s %d %d %d %d %d %d %d\n", TVS_SOURCE_HASH, g_dev_id[dev].c_str(), k.kind, k.f64, k.rcp, k.side_b,
            k.rho_b, a, b);
    fclose(f);
}

int ceil_log2(int64_t v) {
    int r = 0;
    while (((int64_t)1 << r) < v) ++r;
    return r;
}

}  // namespace host
}  // namespace tvs

// Autotuner result cache: tm_problem_tune's choices keyed by the device
// (architecture name and compute-unit count), the operator's layout and
// precision, the tile count and the batch, kept in a process-wide table and
// written to / merged from a small JSON file:
//   {"tilemag_tune_cache": 1, "entries": [
//    {"arch": "gfx950:sramecc+:xnack-", "cus": 256, "layout": 4, "prec": 0, "n": 2500, "batch": 1,
//     "choice": 1, "ms": 0.0127},
//    ...]}
// (one entry per line; the reader takes exactly this form back).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>

#include "common.h"

namespace tmag {
namespace {

using Key = std::tuple<std::string, int, int, int, int64_t, int64_t>;  // arch, cus, layout, prec, n, batch

std::mutex g_mu;
std::map<Key, TuneResult> g_table;
std::map<int, std::pair<std::string, int>> g_devices;  // ordinal -> (arch, cus)

bool device_id(int device, std::string* arch, int* cus) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_devices.find(device);
    if (it == g_devices.end()) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) != hipSuccess) return false;
        it = g_devices.emplace(device, std::make_pair(std::string(prop.gcnArchName), prop.multiProcessorCount)).first;
    }
    *arch = it->second.first;
    *cus = it->second.second;
    return true;
}

bool make_key(const Problem* p, int64_t B, Key* k) {
    std::string arch;
    int cus = 0;
    if (!device_id(p->ctx->device, &arch, &cus)) return false;
    *k = Key(arch, cus, static_cast<int>(p->T->layout), static_cast<int>(p->T->prec), p->n, B);
    return true;
}

// Value of "key": in one JSON object written by tm_tune_cache_save.
bool field(const std::string& obj, const char* key, std::string* out) {
    const std::string pat = std::string("\"") + key + "\":";
    const size_t at = obj.find(pat);
    if (at == std::string::npos) return false;
    size_t i = at + pat.size();
    while (i < obj.size() && obj[i] == ' ') ++i;
    if (i < obj.size() && obj[i] == '"') {
        const size_t end = obj.find('"', i + 1);
        if (end == std::string::npos) return false;
        *out = obj.substr(i + 1, end - i - 1);
        return true;
    }
    size_t end = i;
    while (end < obj.size() && obj[end] != ',' && obj[end] != '}') ++end;
    *out = obj.substr(i, end - i);
    return !out->empty();
}

}  // namespace

bool tune_lookup(const Problem* p, int64_t B, TuneResult* out) {
    Key k;
    if (!make_key(p, B, &k)) return false;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_table.find(k);
    if (it == g_table.end()) return false;
    *out = it->second;
    return true;
}

void tune_store(const Problem* p, int64_t B, const TuneResult& r) {
    Key k;
    if (!make_key(p, B, &k)) return;
    std::lock_guard<std::mutex> lk(g_mu);
    g_table[k] = r;
}

}  // namespace tmag

using namespace tmag;

extern "C" tm_status tm_tune_cache_save(const char* path) {
    TM_REQUIRE(path, TM_EINVAL, "tm_tune_cache_save: null path");
    std::ostringstream os;
    os << "{\"tilemag_tune_cache\": 1, \"entries\": [\n";
    {
        std::lock_guard<std::mutex> lk(g_mu);
        size_t i = 0;
        for (const auto& kv : g_table) {
            const Key& k = kv.first;
            char num[64];
            std::snprintf(num, sizeof num, "%.6g", kv.second.ms);
            os << " {\"arch\": \"" << std::get<0>(k) << "\", \"cus\": " << std::get<1>(k)
               << ", \"layout\": " << std::get<2>(k) << ", \"prec\": " << std::get<3>(k) << ", \"n\": " << std::get<4>(k)
               << ", \"batch\": " << std::get<5>(k) << ", \"choice\": " << kv.second.choice << ", \"ms\": " << num
               << "}" << (++i < g_table.size() ? "," : "") << "\n";
        }
    }
    os << "]}\n";
    std::ofstream f(path);
    TM_REQUIRE(f.good(), TM_EINVAL, "tm_tune_cache_save: cannot write %s", path);
    f << os.str();
    f.close();
    TM_REQUIRE(f.good(), TM_EINVAL, "tm_tune_cache_save: write to %s failed", path);
    return TM_OK;
}

extern "C" tm_status tm_tune_cache_load(const char* path) {
    TM_REQUIRE(path, TM_EINVAL, "tm_tune_cache_load: null path");
    std::ifstream f(path);
    TM_REQUIRE(f.good(), TM_ENOTFOUND, "tm_tune_cache_load: cannot read %s", path);
    std::string line;
    std::getline(f, line);
    TM_REQUIRE(line.find("\"tilemag_tune_cache\": 1") != std::string::npos, TM_EINVAL,
               "tm_tune_cache_load: %s is not a tilemag tuning cache", path);
    std::map<Key, TuneResult> add;
    while (std::getline(f, line)) {
        if (line.find('{') == std::string::npos) continue;
        std::string arch, cus, layout, prec, n, batch, choice, ms;
        const bool ok = field(line, "arch", &arch) && field(line, "cus", &cus) && field(line, "layout", &layout) &&
                        field(line, "prec", &prec) && field(line, "n", &n) && field(line, "batch", &batch) &&
                        field(line, "choice", &choice) && field(line, "ms", &ms);
        TM_REQUIRE(ok, TM_EINVAL, "tm_tune_cache_load: malformed entry in %s: %s", path, line.c_str());
        TuneResult r;
        r.choice = std::atoi(choice.c_str());
        r.ms = std::atof(ms.c_str());
        add[Key(arch, std::atoi(cus.c_str()), std::atoi(layout.c_str()), std::atoi(prec.c_str()),
                std::atoll(n.c_str()), std::atoll(batch.c_str()))] = r;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto& kv : add) g_table[kv.first] = kv.second;
    return TM_OK;
}

extern "C" tm_status tm_tune_cache_clear(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.clear();
    return TM_OK;
}

extern "C" tm_status tm_tune_cache_size(int64_t* entries) {
    TM_REQUIRE(entries, TM_EINVAL, "tm_tune_cache_size: null argument");
    std::lock_guard<std::mutex> lk(g_mu);
    *entries = static_cast<int64_t>(g_table.size());
    return TM_OK;
}

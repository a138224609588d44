// Autotuner cache: one JSON object per line, {"key": K, "value": V, "ms": T}.  The key names the
// device (architecture and compute-unit count) and the problem; the value is the launch that
// won the timed trials.  Lookups scan the file; a store rewrites it through a temporary file
// and a rename, replacing a line with the same key.

#include <hip/hip_runtime.h>

#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "lbm_internal.h"

namespace pplbm {

namespace {

// The string value of "field": "..." in a line (no escapes: keys and values hold none).
bool field_string(const std::string &line, const char *field, std::string *out) {
    const std::string tag = std::string("\"") + field + "\": \"";
    const size_t a = line.find(tag);
    if (a == std::string::npos) return false;
    const size_t b = line.find('"', a + tag.size());
    if (b == std::string::npos) return false;
    *out = line.substr(a + tag.size(), b - a - tag.size());
    return true;
}

}  // namespace

std::string device_tag() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    std::string arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
    return arch + "/" + std::to_string(prop.multiProcessorCount) + "cu";
}

bool tune_cache_lookup(const char *path, const std::string &key, std::string *value) {
    if (!path || !*path) return false;
    std::ifstream in(path);
    std::string line, k;
    while (std::getline(in, line))
        if (field_string(line, "key", &k) && k == key && field_string(line, "value", value)) return true;
    return false;
}

bool tune_cache_store(const char *path, const std::string &key, const std::string &value, double ms) {
    if (!path || !*path) return false;
    std::vector<std::string> keep;
    {
        std::ifstream in(path);
        std::string line, k;
        while (std::getline(in, line))
            if (!line.empty() && !(field_string(line, "key", &k) && k == key)) keep.push_back(line);
    }
    std::ostringstream rec;
    rec.precision(6);
    rec << "{\"key\": \"" << key << "\", \"value\": \"" << value << "\", \"ms\": " << ms << "}";
    keep.push_back(rec.str());
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream out(tmp, std::ios::trunc);
        if (!out) return false;
        for (const std::string &l : keep) out << l << "\n";
        if (!out) return false;
    }
    return std::rename(tmp.c_str(), path) == 0;
}

}  // namespace pplbm

// tune_cache.cpp -- the autotuner's JSON schedule cache (see tune_cache.h).
#include "tune_cache.h"

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <vector>

namespace sphfilt {

uint64_t fnv1a(uint64_t h, const void *data, size_t n)
{
    const unsigned char *p = (const unsigned char *)data;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ULL;
    }
    return h;
}

std::string hex64(uint64_t v)
{
    char buf[17];
    std::snprintf(buf, sizeof(buf), "%016llx", (unsigned long long)v);
    return buf;
}

namespace {

// Parse one flat object {"k": v, ...} (v a number or a quoted string) out of
// a line; trailing commas and brackets around it are ignored.
bool parse_line(const std::string &line, TuneFields *out)
{
    size_t i = line.find('{');
    if (i == std::string::npos) return false;
    ++i;
    TuneFields f;
    auto skip = [&]() { while (i < line.size() && (line[i] == ' ' || line[i] == '\t')) ++i; };
    for (;;) {
        skip();
        if (i >= line.size()) return false;
        if (line[i] == '}') break;
        if (line[i] != '"') return false;
        const size_t k0 = ++i;
        while (i < line.size() && line[i] != '"') ++i;
        if (i >= line.size()) return false;
        const std::string key = line.substr(k0, i - k0);
        ++i;
        skip();
        if (i >= line.size() || line[i] != ':') return false;
        ++i;
        skip();
        size_t v0 = i;
        if (i < line.size() && line[i] == '"') {
            ++i;
            while (i < line.size() && line[i] != '"') ++i;
            if (i >= line.size()) return false;
            ++i;
        } else {
            while (i < line.size() && line[i] != ',' && line[i] != '}') ++i;
        }
        std::string val = line.substr(v0, i - v0);
        while (!val.empty() && val.back() == ' ') val.pop_back();
        if (val.empty()) return false;
        f[key] = val;
        skip();
        if (i < line.size() && line[i] == ',') { ++i; continue; }
        if (i < line.size() && line[i] == '}') break;
        return false;
    }
    *out = f;
    return true;
}

std::string format_line(const std::string &sig, const TuneFields &fields)
{
    std::ostringstream o;
    o << "{\"sig\": \"" << sig << "\"";
    for (const auto &kv : fields)
        if (kv.first != "sig") o << ", \"" << kv.first << "\": " << kv.second;
    o << "}";
    return o.str();
}

}  // namespace

bool tune_cache_get(const char *path, const std::string &sig, TuneFields *out)
{
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    const std::string key = "\"sig\": \"" + sig + "\"";
    while (std::getline(f, line)) {
        if (line.find(key) == std::string::npos) continue;
        return parse_line(line, out);
    }
    return false;
}

bool tune_cache_put(const char *path, const std::string &sig, const TuneFields &fields)
{
    std::vector<std::string> keep;
    {
        std::ifstream f(path);
        std::string line;
        while (f && std::getline(f, line)) {
            TuneFields g;
            if (line.find("\"sig\": \"") == std::string::npos || !parse_line(line, &g)) continue;
            std::string s;
            if (!tune_string(g, "sig", &s) || s == sig) continue;
            keep.push_back(format_line(s, g));
        }
    }
    keep.push_back(format_line(sig, fields));
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream o(tmp);
        if (!o) return false;
        o << "{\"sphfilt_tune_cache\": 2, \"entries\": [\n";
        for (size_t i = 0; i < keep.size(); ++i) o << "  " << keep[i] << (i + 1 < keep.size() ? ",\n" : "\n");
        o << "]}\n";
        if (!o) return false;
    }
    return std::rename(tmp.c_str(), path) == 0;
}

std::string tune_num(double v)
{
    std::ostringstream o;
    o.precision(10);
    o << v;
    return o.str();
}

std::string tune_str(const std::string &s) { return "\"" + s + "\""; }

bool tune_int(const TuneFields &f, const char *key, int *v)
{
    auto it = f.find(key);
    if (it == f.end()) return false;
    char *end = nullptr;
    const long x = std::strtol(it->second.c_str(), &end, 10);
    if (end == it->second.c_str() || *end) return false;
    *v = (int)x;
    return true;
}

bool tune_double(const TuneFields &f, const char *key, double *v)
{
    auto it = f.find(key);
    if (it == f.end()) return false;
    char *end = nullptr;
    const double x = std::strtod(it->second.c_str(), &end);
    if (end == it->second.c_str() || *end) return false;
    *v = x;
    return true;
}

bool tune_string(const TuneFields &f, const char *key, std::string *v)
{
    auto it = f.find(key);
    if (it == f.end() || it->second.size() < 2 || it->second.front() != '"' || it->second.back() != '"')
        return false;
    *v = it->second.substr(1, it->second.size() - 2);
    return true;
}

const char *tune_cache_default()
{
    const char *e = std::getenv("SPHFILT_TUNE_CACHE");
    return e && *e ? e : nullptr;
}

}  // namespace sphfilt

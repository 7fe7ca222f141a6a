// tune_cache.h -- the autotuner's JSON schedule cache, shared by plans and
// batches (host side).
//
// File format: one JSON object whose "entries" array holds one flat object
// per line,
//   {"sphfilt_tune_cache": 2, "entries": [
//     {"sig": "<16 hex>", "what": "batch", "arch": "gfx950", "split": 1, ...},
//     ...]}
// keyed by "sig" (a hash of the workload and the GPU architecture).  Values
// are numbers or strings without quotes or backslashes inside.
#pragma once
#include <cstdint>
#include <map>
#include <string>

namespace sphfilt {

using TuneFields = std::map<std::string, std::string>;   // key -> raw JSON value

// FNV-1a over bytes, chained through h.
uint64_t fnv1a(uint64_t h, const void *data, size_t n);
constexpr uint64_t kFnvSeed = 1469598103934665603ULL;
std::string hex64(uint64_t v);

// The entry with this signature, or false (missing file or entry, or a
// line that does not parse).
bool tune_cache_get(const char *path, const std::string &sig, TuneFields *out);
// Replace or add the entry (written to a temporary file, then renamed);
// false if the file cannot be written.
bool tune_cache_put(const char *path, const std::string &sig, const TuneFields &fields);

// Field helpers: numbers and strings.
std::string tune_num(double v);
std::string tune_str(const std::string &s);
bool tune_int(const TuneFields &f, const char *key, int *v);
bool tune_double(const TuneFields &f, const char *key, double *v);
bool tune_string(const TuneFields &f, const char *key, std::string *v);

// The cache file to use when a caller passes none: $SPHFILT_TUNE_CACHE, or
// NULL (no tuning).
const char *tune_cache_default();

}  // namespace sphfilt

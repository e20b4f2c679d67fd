// lbm13_tune_cache.h -- host-side cache of autotuned launch configurations
// (see lbm13_tune_cache.cpp for the file format).
#pragma once

#include <string>
#include <vector>

namespace lbm13 {

// Cache key: architecture (the part of the device's gcnArchName before ':'),
// precision, floor(log2(nodes)), floor(log2(domains)), walls or periodic only.
std::string tune_key(const std::string& arch, int precision, long long nodes, int count, bool walls);

// The six integers of a launch configuration stored under key; false if the
// file or the key is missing or damaged.
bool tune_cache_lookup(const char* path, const std::string& key, int cfg[6]);

// Stores (or replaces) key's configuration, keeping the other entries; false
// if the file could not be written.
bool tune_cache_store(const char* path, const std::string& key, const int cfg[6]);

}  // namespace lbm13

// lbm13_tune_cache.cpp -- persistent cache of autotuned launch configurations.
//
// A small JSON file maps a key naming the device architecture, the precision
// and the size class of the work (log2 of the node count, log2 of the domain
// count, walls or none) to the launch configuration the autotuner chose:
//   {"version": 1, "entries": {"gfx950:fp32:n24:d0:periodic": [3, 64, 8, 64, 16, 1], ...}}
// with the six integers of lbm13_launch_config.  Unknown or damaged content is
// ignored (the entry is tuned again and the file rewritten); writes go to a
// temporary file renamed over the cache, so readers never see a partial file.
#include "lbm13_tune_cache.h"

#include <cctype>
#include <cstdio>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <unistd.h>

namespace lbm13 {

namespace {

using Entries = std::map<std::string, std::vector<int>>;

// Parses the "entries" of a cache file: every "key": [i0, ..., i5] pair.
Entries parse(const std::string& text) {
    Entries out;
    size_t p = text.find("\"entries\"");
    if (p == std::string::npos) return out;
    p = text.find('{', p);
    if (p == std::string::npos) return out;
    ++p;
    while (p < text.size()) {
        const size_t k0 = text.find('"', p);
        if (k0 == std::string::npos) break;
        const size_t k1 = text.find('"', k0 + 1);
        if (k1 == std::string::npos) break;
        const std::string key = text.substr(k0 + 1, k1 - k0 - 1);
        size_t q = text.find_first_not_of(" \t\r\n", k1 + 1);
        if (q == std::string::npos || text[q] != ':') break;
        q = text.find_first_not_of(" \t\r\n", q + 1);
        if (q == std::string::npos || text[q] != '[') break;
        const size_t e = text.find(']', q);
        if (e == std::string::npos) break;
        std::vector<int> vals;
        std::istringstream in(text.substr(q + 1, e - q - 1));
        std::string tok;
        bool ok = true;
        while (std::getline(in, tok, ',')) {
            size_t a = tok.find_first_not_of(" \t\r\n"), b = tok.find_last_not_of(" \t\r\n");
            if (a == std::string::npos) { ok = false; break; }
            tok = tok.substr(a, b - a + 1);
            for (size_t i = 0; i < tok.size(); ++i)
                if (!std::isdigit((unsigned char)tok[i]) && !(i == 0 && tok[i] == '-')) ok = false;
            if (!ok || tok.size() > 9) { ok = false; break; }
            vals.push_back(std::stoi(tok));
        }
        if (ok && vals.size() == 6) out[key] = vals;
        p = e + 1;
        const size_t c = text.find_first_not_of(" \t\r\n", p);
        if (c == std::string::npos || text[c] == '}') break;
        if (text[c] != ',') break;
        p = c + 1;
    }
    return out;
}

std::string read_file(const char* path) {
    std::ifstream f(path, std::ios::binary);
    if (!f) return std::string();
    std::ostringstream s;
    s << f.rdbuf();
    return s.str();
}

}  // namespace

std::string tune_key(const std::string& arch, int precision, long long nodes, int count, bool walls) {
    int ln = 0, ld = 0;
    while ((2LL << ln) <= nodes) ++ln;
    while ((2 << ld) <= count) ++ld;
    std::string a = arch.substr(0, arch.find(':'));
    return a + (precision == 0 ? ":fp64" : ":fp32") + ":n" + std::to_string(ln) + ":d" + std::to_string(ld) + ":" +
           (walls ? "walls" : "periodic");
}

bool tune_cache_lookup(const char* path, const std::string& key, int cfg[6]) {
    const Entries e = parse(read_file(path));
    auto it = e.find(key);
    if (it == e.end()) return false;
    for (int i = 0; i < 6; ++i) cfg[i] = it->second[i];
    return true;
}

bool tune_cache_store(const char* path, const std::string& key, const int cfg[6]) {
    Entries e = parse(read_file(path));
    e[key] = std::vector<int>(cfg, cfg + 6);
    std::ostringstream s;
    s << "{\"version\": 1, \"entries\": {";
    bool first = true;
    for (const auto& kv : e) {
        s << (first ? "\n  " : ",\n  ") << '"' << kv.first << "\": [";
        for (int i = 0; i < 6; ++i) s << (i ? ", " : "") << kv.second[i];
        s << ']';
        first = false;
    }
    s << "\n}}\n";
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long long)getpid());
    {
        std::ofstream f(tmp, std::ios::binary | std::ios::trunc);
        if (!f) return false;
        f << s.str();
        if (!f) return false;
    }
    if (std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return false;
    }
    return true;
}

}  // namespace lbm13

// Persisted choices of the batched form's autotuner: one line per size class,
// "<key> <value>", in a text file kept across processes, so a size class is
// timed once per machine instead of once per process.  Header-only host code
// (no HIP), driven directly by the host test-suite.
//
// The file is the environment variable HP_TUNE_CACHE when set (an empty
// value turns persistence off), else $XDG_CACHE_HOME/hipperm/batch_tune.txt,
// else $HOME/.cache/hipperm/batch_tune.txt.  Reading ignores malformed
// lines; a later line for a key overrides an earlier one; writing appends
// one line and never fails the caller.
#pragma once

#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <string>
#include <sys/stat.h>

namespace hp {

inline std::string tune_cache_path() {
    if (const char *p = std::getenv("HP_TUNE_CACHE")) return std::string(p);
    std::string base;
    if (const char *x = std::getenv("XDG_CACHE_HOME"); x && *x) base = x;
    else if (const char *h = std::getenv("HOME"); h && *h) base = std::string(h) + "/.cache";
    else return std::string();
    return base + "/hipperm/batch_tune.txt";
}

// Entries of the cache file at `path` (an empty map when it is missing).
inline std::map<std::string, int> tune_cache_load(const std::string &path) {
    std::map<std::string, int> out;
    if (path.empty()) return out;
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return out;
    char key[256];
    int v = 0;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        if (std::sscanf(line, "%255s %d", key, &v) == 2 && v > 0) out[key] = v;
    }
    std::fclose(f);
    return out;
}

// Appends "key value" to the cache file at `path`, creating its directory
// (one level) when needed.  Returns false when the line could not be written.
inline bool tune_cache_store(const std::string &path, const std::string &key, int value) {
    if (path.empty() || key.empty() || key.find_first_of(" \t\n") != std::string::npos || value <= 0) return false;
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0) {
        const std::string dir = path.substr(0, slash);
        const size_t up = dir.rfind('/');
        if (up != std::string::npos && up > 0) ::mkdir(dir.substr(0, up).c_str(), 0755);
        ::mkdir(dir.c_str(), 0755);
    }
    FILE *f = std::fopen(path.c_str(), "a");
    if (!f) return false;
    const bool ok = std::fprintf(f, "%s %d\n", key.c_str(), value) > 0;
    return std::fclose(f) == 0 && ok;
}

}  // namespace hp

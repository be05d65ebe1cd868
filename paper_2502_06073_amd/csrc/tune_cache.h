// Result cache of the edge-tile tuner: a small JSON object, one entry per
// line, keyed on the device architecture, the model shape and the mean
// number of edges per atom of the tuned workload:
//
//   {
//   "gfx950/w256/c64/l2/L2/d3/tb64-128-256/nb8/bf16/deg72": {"tile": 64, "ms_64": 11.3, "ms_128": 12.9},
//   ...
//   }
//
// Plain C++ (no HIP), so the parsing and update logic is tested on the host.
#pragma once
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <fstream>
#include <map>
#include <sstream>
#include <string>

namespace afm {

struct TuneEntry {
  int tile = 0;
  double ms_64 = 0.0, ms_128 = 0.0;
};

// Parses the entries of a cache file's text; lines that are not entries
// (braces, blank, malformed) are skipped.
inline std::map<std::string, TuneEntry> tune_cache_parse(const std::string& text) {
  std::map<std::string, TuneEntry> out;
  std::istringstream in(text);
  std::string line;
  while (std::getline(in, line)) {
    const size_t q0 = line.find('"');
    if (q0 == std::string::npos) continue;
    const size_t q1 = line.find('"', q0 + 1);
    if (q1 == std::string::npos) continue;
    const std::string key = line.substr(q0 + 1, q1 - q0 - 1);
    auto num = [&](const char* field, double* v) {
      const std::string f = std::string("\"") + field + "\":";
      const size_t p = line.find(f, q1);
      if (p == std::string::npos) return false;
      char* end = nullptr;
      const char* s = line.c_str() + p + f.size();
      *v = strtod(s, &end);
      return end != s;
    };
    double tile = 0.0;
    TuneEntry e;
    if (!num("tile", &tile)) continue;
    e.tile = (int)tile;
    if (e.tile != 64 && e.tile != 128) continue;
    num("ms_64", &e.ms_64);
    num("ms_128", &e.ms_128);
    out[key] = e;
  }
  return out;
}

inline std::string tune_cache_format(const std::map<std::string, TuneEntry>& m) {
  std::string s = "{\n";
  size_t k = 0;
  for (const auto& kv : m) {
    char buf[160];
    snprintf(buf, sizeof buf, "\": {\"tile\": %d, \"ms_64\": %.6g, \"ms_128\": %.6g}", kv.second.tile,
             kv.second.ms_64, kv.second.ms_128);
    s += "\"" + kv.first + buf + (++k < m.size() ? ",\n" : "\n");
  }
  s += "}\n";
  return s;
}

inline bool tune_cache_lookup(const char* path, const std::string& key, TuneEntry* e) {
  if (!path) return false;
  std::ifstream f(path);
  if (!f) return false;
  std::stringstream ss;
  ss << f.rdbuf();
  const auto m = tune_cache_parse(ss.str());
  const auto it = m.find(key);
  if (it == m.end()) return false;
  *e = it->second;
  return true;
}

// Adds or replaces one entry, keeping the others; false if the file cannot
// be written.
inline bool tune_cache_store(const char* path, const std::string& key, const TuneEntry& e) {
  std::map<std::string, TuneEntry> m;
  {
    std::ifstream f(path);
    if (f) {
      std::stringstream ss;
      ss << f.rdbuf();
      m = tune_cache_parse(ss.str());
    }
  }
  m[key] = e;
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream o(tmp, std::ios::trunc);
    if (!o) return false;
    o << tune_cache_format(m);
    if (!o) return false;
  }
  return rename(tmp.c_str(), path) == 0;
}

}  // namespace afm

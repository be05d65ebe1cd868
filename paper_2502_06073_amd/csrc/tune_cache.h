// Result cache of the edge-tile tuner: a small JSON object, one entry per
// line, keyed on the device architecture, the model shape and the mean
// number of edges per atom of the tuned workload:
//
//   {
//   "gfx950/w256/c64/l2/L2/d3/tb64-128-256/nb8/bf16/deg72": {"edges": 64, "waves": 8,
//       "ms_64x8": 11.3, "ms_128x16": 12.9, "ms_128x8": 10.8},   (one line)
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

// the built shapes (edges per tile, wavefronts per workgroup), in the
// order of TuneEntry::ms
constexpr int kTileShapes = 3;
constexpr int kTileEdges[kTileShapes] = {64, 128, 128};
constexpr int kTileWaves[kTileShapes] = {8, 16, 8};
inline const char* tile_shape_name(int s) {
  static const char* names[kTileShapes] = {"64x8", "128x16", "128x8"};
  return names[s];
}
inline int tile_shape_index(int edges, int waves) {
  for (int s = 0; s < kTileShapes; ++s)
    if (kTileEdges[s] == edges && kTileWaves[s] == waves) return s;
  return -1;
}

struct TuneEntry {
  int edges = 0, waves = 0;
  double ms[kTileShapes] = {};
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
    double edges = 0.0, waves = 0.0;
    TuneEntry e;
    if (!num("edges", &edges) || !num("waves", &waves)) continue;
    e.edges = (int)edges;
    e.waves = (int)waves;
    if (tile_shape_index(e.edges, e.waves) < 0) continue;
    for (int s = 0; s < kTileShapes; ++s) num((std::string("ms_") + tile_shape_name(s)).c_str(), &e.ms[s]);
    out[key] = e;
  }
  return out;
}

inline std::string tune_cache_format(const std::map<std::string, TuneEntry>& m) {
  std::string s = "{\n";
  size_t k = 0;
  for (const auto& kv : m) {
    std::string line = "\"" + kv.first + "\": {\"edges\": " + std::to_string(kv.second.edges) +
                       ", \"waves\": " + std::to_string(kv.second.waves);
    for (int q = 0; q < kTileShapes; ++q) {
      char buf[64];
      snprintf(buf, sizeof buf, ", \"ms_%s\": %.6g", tile_shape_name(q), kv.second.ms[q]);
      line += buf;
    }
    s += line + "}" + (++k < m.size() ? ",\n" : "\n");
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

// Tile table: text load/save and lookup by size class.
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <fstream>
#include <sstream>

#include "runtime.hpp"

namespace famlies {

int TileTable::log2c(int64_t x) {
  int l = 0;
  while (((int64_t)1 << l) < x && l < 62) ++l;
  return l;
}

// Nearest tuned class (L1 distance in log2 space, at most 2), if any.
static bool nearest(const std::vector<TileTable::Entry>& entries, int kind, int dtype, int compute, int lm,
                    int ln, int lk, TileCfg* out) {
  int best = 3;
  for (const TileTable::Entry& e : entries) {
    if (e.kind != kind || e.dtype != dtype || e.compute != compute) continue;
    const int d = std::abs(e.lm - lm) + std::abs(e.ln - ln) + std::abs(e.lk - lk);
    if (d < best) {
      best = d;
      *out = e.cfg;
    }
  }
  return best <= 2;
}

bool TileTable::lookup_plain(const Analysis& an, TileCfg* out) const {
  return nearest(entries, 0, an.dtype, an.compute, log2c(an.M), log2c(an.N), log2c(an.K), out);
}

bool TileTable::lookup_batch(int dtype, int64_t m, int64_t n, int64_t k, TileCfg* out) const {
  return nearest(entries, 1, dtype, FAMLIES_NATIVE, log2c(m), log2c(n), log2c(k), out);
}

void TileTable::put(const Entry& e) {
  for (Entry& x : entries)
    if (x.kind == e.kind && x.dtype == e.dtype && x.compute == e.compute && x.lm == e.lm &&
        x.ln == e.ln && x.lk == e.lk) {
      x = e;
      return;
    }
  entries.push_back(e);
}

// Format: '#' comments; one entry per line:
//   <plain|batch> <dtype> <compute> <log2 M> <log2 N> <log2 K> <bm> <bn> <bk> <split> [<index bits> [<split tiles>]]
// where the optional index bits 64 makes plans of that class use 64-bit
// indexing vectors even when 32 bits reach every element, e32 makes them use
// 32-bit element offsets wherever those reach (0 or 32: automatic), and
// split tiles > 0 splits only that many tiles, the last in tile order (0:
// every tile when split > 1).
bool TileTable::load(const std::string& path, std::string* err) {
  std::ifstream f(path);
  if (!f) {
    *err = "cannot open " + path;
    return false;
  }
  std::string line;
  int ln = 0;
  std::vector<Entry> got;
  while (std::getline(f, line)) {
    ++ln;
    if (line.empty() || line[0] == '#') continue;
    std::istringstream is(line);
    std::string kind;
    Entry e;
    if (!(is >> kind >> e.dtype >> e.compute >> e.lm >> e.ln >> e.lk >> e.cfg.bm >> e.cfg.bn >>
          e.cfg.bk >> e.cfg.split) ||
        (kind != "plain" && kind != "batch") || e.cfg.bm <= 0 || e.cfg.bn <= 0 || e.cfg.bk <= 0 ||
        e.cfg.split <= 0) {
      *err = path + ":" + std::to_string(ln) + ": malformed entry";
      return false;
    }
    std::string bits;
    if (is >> bits) {
      if (bits != "0" && bits != "32" && bits != "64" && bits != "e32") {
        *err = path + ":" + std::to_string(ln) + ": index bits must be 0, 32, 64 or e32";
        return false;
      }
      e.cfg.index_bits = bits == "64" ? 64 : bits == "e32" ? kForceElem32 : 0;
      int tail = 0;
      if (is >> tail) {
        if (tail < 0) {
          *err = path + ":" + std::to_string(ln) + ": split tiles must be >= 0";
          return false;
        }
        e.cfg.tail = tail;
      }
    }
    e.kind = kind == "plain" ? 0 : 1;
    got.push_back(e);
  }
  for (const Entry& e : got) put(e);
  return true;
}

bool TileTable::save(const std::string& path, std::string* err) const {
  std::ofstream f(path);
  if (!f) {
    *err = "cannot write " + path;
    return false;
  }
  f << "# famlies tile table: kind dtype compute log2M log2N log2K bm bn bk split [index_bits [split_tiles]]\n";
  for (const Entry& e : entries) {
    f << (e.kind == 0 ? "plain" : "batch") << ' ' << e.dtype << ' ' << e.compute << ' ' << e.lm << ' '
      << e.ln << ' ' << e.lk << ' ' << e.cfg.bm << ' ' << e.cfg.bn << ' ' << e.cfg.bk << ' '
      << e.cfg.split;
    if (e.cfg.index_bits || e.cfg.tail) {
      if (e.cfg.index_bits == kForceElem32)
        f << " e32";
      else
        f << ' ' << e.cfg.index_bits;
    }
    if (e.cfg.tail) f << ' ' << e.cfg.tail;
    f << '\n';
  }
  return (bool)f;
}

}  // namespace famlies

// Autotuner cache: the work-item size and persistent-grid multiplier chosen
// per kernel class, keyed by (device architecture, p, q, r_b bound,
// precision), kept in memory and, when KSTAP_TUNE_CACHE names a file, in a
// small JSON file that later processes read back.
#include <hip/hip_runtime.h>
#include <sys/stat.h>

#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "kstap_tune.h"

namespace kstap {
namespace tune {
namespace {

using Key = std::tuple<std::string, int, int, int, int>;   // arch, p, q, r_b bound, precision

std::mutex g_mu;
std::map<Key, Entry> g_cache;
std::string g_loaded_path;
long long g_loaded_mtime = -1;

const char* cache_path() {
  const char* p = std::getenv("KSTAP_TUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

long long file_mtime(const char* path) {
  struct stat st;
  if (stat(path, &st) != 0) return -1;
  return static_cast<long long>(st.st_mtime) * 1000000000LL + static_cast<long long>(st.st_mtim.tv_nsec);
}

// Minimal reader of the file this module writes: an "entries" array of flat
// objects whose values are strings or numbers.
struct Reader {
  const std::string& s;
  size_t i = 0;
  explicit Reader(const std::string& text) : s(text) {}
  void ws() {
    while (i < s.size() && std::isspace(static_cast<unsigned char>(s[i]))) ++i;
  }
  bool str(std::string* out) {
    ws();
    if (i >= s.size() || s[i] != '"') return false;
    ++i;
    out->clear();
    while (i < s.size() && s[i] != '"') {
      if (s[i] == '\\' && i + 1 < s.size()) ++i;
      out->push_back(s[i++]);
    }
    if (i >= s.size()) return false;
    ++i;
    return true;
  }
  bool num(double* out) {
    ws();
    const char* b = s.c_str() + i;
    char* e = nullptr;
    *out = std::strtod(b, &e);
    if (e == b) return false;
    i += size_t(e - b);
    return true;
  }
  bool lit(char c) {
    ws();
    if (i < s.size() && s[i] == c) {
      ++i;
      return true;
    }
    return false;
  }
};

// Parses the cache file into `out`; false (and `out` untouched) on a malformed file.
bool parse(const std::string& text, std::map<Key, Entry>* out) {
  Reader r(text);
  std::map<Key, Entry> tmp;
  if (!r.lit('{')) return false;
  while (true) {
    std::string key;
    if (!r.str(&key) || !r.lit(':')) return false;
    if (key == "entries") {
      if (!r.lit('[')) return false;
      if (!r.lit(']')) {
        while (true) {
          if (!r.lit('{')) return false;
          std::string arch;
          double p = -1, q = -1, rb = -1, prec = -1, ppb = -1, mult = -1, ms = 0;
          while (true) {
            std::string k;
            if (!r.str(&k) || !r.lit(':')) return false;
            if (k == "arch") {
              if (!r.str(&arch)) return false;
            } else {
              double v;
              if (!r.num(&v)) return false;
              if (k == "p") p = v;
              else if (k == "q") q = v;
              else if (k == "rb_bound") rb = v;
              else if (k == "precision") prec = v;
              else if (k == "pix_per_item") ppb = v;
              else if (k == "grid_mult") mult = v;
              else if (k == "ms") ms = v;
            }
            if (r.lit(',')) continue;
            if (r.lit('}')) break;
            return false;
          }
          if (arch.empty() || p < 0 || q < 0 || rb < 0 || prec < 0 || ppb < 16 || mult < 1) return false;
          Entry e;
          e.ppb = int(ppb);
          e.grid_mult = int(mult);
          e.ms = ms;
          tmp[Key(arch, int(p), int(q), int(rb), int(prec))] = e;
          if (r.lit(',')) continue;
          if (r.lit(']')) break;
          return false;
        }
      }
    } else {
      std::string sv;
      double dv;
      if (!r.str(&sv) && !r.num(&dv)) return false;
    }
    if (r.lit(',')) continue;
    if (r.lit('}')) break;
    return false;
  }
  *out = std::move(tmp);
  return true;
}

// Brings the in-memory cache up to date with the file (entries in the file
// take precedence); caller holds g_mu.
void refresh_locked() {
  const char* path = cache_path();
  if (!path) return;
  const long long mt = file_mtime(path);
  if (mt < 0 || (g_loaded_path == path && mt == g_loaded_mtime)) return;
  FILE* f = std::fopen(path, "rb");
  if (!f) return;
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
  std::fclose(f);
  std::map<Key, Entry> fromfile;
  if (!parse(text, &fromfile)) return;
  for (const auto& kv : fromfile) g_cache[kv.first] = kv.second;
  g_loaded_path = path;
  g_loaded_mtime = mt;
}

bool write_locked(std::string* err) {
  const char* path = cache_path();
  if (!path) return true;
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) {
    *err = std::string("cannot write ") + tmp;
    return false;
  }
  std::fprintf(f, "{\n  \"format\": \"kstap-tune-1\",\n  \"entries\": [");
  bool first = true;
  for (const auto& kv : g_cache) {
    const Key& k = kv.first;
    const Entry& e = kv.second;
    std::fprintf(f,
                 "%s\n    {\"arch\": \"%s\", \"p\": %d, \"q\": %d, \"rb_bound\": %d, \"precision\": %d, "
                 "\"pix_per_item\": %d, \"grid_mult\": %d, \"ms\": %.6g}",
                 first ? "" : ",", std::get<0>(k).c_str(), std::get<1>(k), std::get<2>(k), std::get<3>(k),
                 std::get<4>(k), e.ppb, e.grid_mult, e.ms);
    first = false;
  }
  std::fprintf(f, "\n  ]\n}\n");
  const bool ok = std::fclose(f) == 0;
  if (!ok || std::rename(tmp.c_str(), path) != 0) {
    *err = std::string("cannot replace ") + path;
    return false;
  }
  g_loaded_path = path;
  g_loaded_mtime = file_mtime(path);
  return true;
}

}  // namespace

std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return std::string();
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

bool lookup(const std::string& arch, int p, int q, int rbm, int prec, Entry* out) {
  std::lock_guard<std::mutex> lk(g_mu);
  refresh_locked();
  auto it = g_cache.find(Key(arch, p, q, rbm, prec));
  if (it == g_cache.end()) return false;
  *out = it->second;
  return true;
}

bool record(const std::string& arch, int p, int q, int rbm, int prec, const Entry& e, std::string* err) {
  std::lock_guard<std::mutex> lk(g_mu);
  refresh_locked();
  g_cache[Key(arch, p, q, rbm, prec)] = e;
  return write_locked(err);
}

}  // namespace tune
}  // namespace kstap

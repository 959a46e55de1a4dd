// Persisted pair-kernel tilings: a small JSON file that maps a key
//   <GPU architecture>/<mode>/<work signature>
// to the tiling the autotuner picked (x units per block, y tiles per work
// item) and its time.  The work signature hashes what the pair kernel's
// schedule depends on: the fragment shapes and classes and the oriented pair
// list.  One entry per line, written by this file only:
//   {
//     "gfx950/fp16x2/3f0c2a9e51d7b604": {"xb": 2, "yc": 64, "us": 2233.4},
//     ...
//   }
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include <unistd.h>

#include "fef_internal.h"

namespace {

const char* const kModeName[FEF_NPREC] = {"f64", "f32", "bf16x2", "fp16x2", "bf16x3"};

struct TuneEntry {
  std::string key;
  int32_t xb, yc;
  double us;
};

uint64_t fnv1a(uint64_t h, const void* data, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ULL;
  }
  return h;
}

template <typename T>
uint64_t mix(uint64_t h, T v) {
  return fnv1a(h, &v, sizeof(v));
}

bool tune_key(const fef_plan_s& p, int prec, std::string& key) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, p.device) != hipSuccess) return false;
  std::string arch(prop.gcnArchName);
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch.resize(colon);
  uint64_t h = 1469598103934665603ULL;
  h = mix(h, p.nfrag);
  h = mix(h, p.npair);
  h = mix(h, p.nclass);
  for (const auto& f : p.frag) {
    h = mix(h, f.nbf);
    h = mix(h, f.nocc);
    h = mix(h, f.naux);
    h = mix(h, f.cls);
  }
  for (const auto& q : p.pairs) {
    h = mix(h, q.x);
    h = mix(h, q.y);
  }
  char buf[160];
  snprintf(buf, sizeof(buf), "%s/%s/%016llx", arch.c_str(), kModeName[prec],
           (unsigned long long)h);
  key = buf;
  return true;
}

// Entries of the file; a missing or unreadable file is an empty cache, and
// lines that are not entries are skipped.
std::vector<TuneEntry> read_cache(const char* path) {
  std::vector<TuneEntry> out;
  FILE* f = fopen(path, "r");
  if (!f) return out;
  char line[512];
  while (fgets(line, sizeof(line), f)) {
    char key[256];
    int xb = 0, yc = 0;
    double us = 0.0;
    if (sscanf(line, " \"%255[^\"]\": {\"xb\": %d, \"yc\": %d, \"us\": %lf}", key, &xb, &yc, &us) ==
        4)
      out.push_back({key, xb, yc, us});
  }
  fclose(f);
  return out;
}

// Whole file rewritten through a temporary in the same directory, then
// renamed over the old one, so a reader never sees half a file.
bool write_cache(const char* path, const std::vector<TuneEntry>& entries) {
  const std::string tmp = std::string(path) + ".tmp." + std::to_string((long)getpid());
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return false;
  bool ok = fprintf(f, "{\n") > 0;
  for (size_t i = 0; i < entries.size() && ok; ++i)
    ok = fprintf(f, "  \"%s\": {\"xb\": %d, \"yc\": %d, \"us\": %.1f}%s\n", entries[i].key.c_str(),
                 entries[i].xb, entries[i].yc, entries[i].us,
                 i + 1 < entries.size() ? "," : "") > 0;
  ok = ok && fprintf(f, "}\n") > 0;
  ok = (fclose(f) == 0) && ok;
  if (!ok || rename(tmp.c_str(), path) != 0) {
    remove(tmp.c_str());
    return false;
  }
  return true;
}

}  // namespace

extern "C" {

fef_status fef_autotune_cached(fef_plan p, const void* ops, const double* eps, fef_prec prec,
                               void* ws, size_t ws_bytes, int32_t reps, void* stream,
                               const char* cache_path, int32_t* best_xb, int32_t* best_yc,
                               double* best_us, int32_t* from_cache) {
  if (!p || !cache_path || !best_xb || !best_yc || !best_us || !from_cache) return FEF_E_ARG;
  if (prec < 0 || prec >= FEF_NPREC) return FEF_E_PREC;
  *from_cache = 0;
  std::string key;
  if (!tune_key(*p, prec, key)) return FEF_E_HIP;
  std::vector<TuneEntry> entries = read_cache(cache_path);
  for (const auto& e : entries)
    if (e.key == key && fef_plan_set_tiles(p, prec, e.xb, e.yc) == FEF_OK) {
      *best_xb = e.xb;
      *best_yc = e.yc;
      *best_us = e.us;
      *from_cache = 1;
      return FEF_OK;
    }
  const fef_status st = fef_autotune(p, ops, eps, prec, ws, ws_bytes, reps, stream, best_xb,
                                     best_yc, best_us);
  if (st != FEF_OK) return st;
  bool found = false;
  for (auto& e : entries)
    if (e.key == key) {
      e.xb = *best_xb;
      e.yc = *best_yc;
      e.us = *best_us;
      found = true;
    }
  if (!found) entries.push_back({key, *best_xb, *best_yc, *best_us});
  // the tiling is in place either way; a cache that cannot be written is
  // reported so the caller knows the next process will tune again
  return write_cache(cache_path, entries) ? FEF_OK : FEF_E_IO;
}

}  // extern "C"

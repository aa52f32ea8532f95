// The autotuner's cache: the fastest plan shape found for a (model, mapping,
// plan size, long items, longest item, GPU architecture, compute-unit count)
// bucket, kept in a text file (one line per key: key, reps per wavefront,
// workgroup, wavefronts per long item, milliseconds), so that a process
// need not time every shape again for a plan of the same kind.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <unistd.h>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/mrip.h"

namespace {

int log2_bucket(uint64_t v) {
  int b = 0;
  while (v > 1) {
    v >>= 1;
    ++b;
  }
  return b;
}

bool valid_key(const char *key) {
  if (!key || !*key) return false;
  for (const char *p = key; *p; ++p)
    if (*p == ' ' || *p == '\n' || *p == '\t' || *p == '\r') return false;
  return true;
}

}  // namespace

extern "C" {

mrip_status mrip_tune_key(mrip_model model, mrip_mapping mapping, uint64_t n_items, uint64_t n_long,
                          uint64_t max_customers, const char *arch, uint32_t cus, char *out,
                          uint64_t cap) {
  if (!out || cap == 0 || !arch || !*arch || n_items == 0) return MRIP_E_INVAL;
  std::string a(arch);
  for (char &c : a)  // one token: no blanks, no separators of the file
    if (c == ' ' || c == '\t' || c == '\n' || c == '\r' || c == '/') c = '_';
  char buf[256];
  const int len = std::snprintf(buf, sizeof buf, "m%d/map%d/n2^%d/long2^%d/max2^%d/%s/%ucu",
                                (int)model, (int)mapping, log2_bucket(n_items),
                                log2_bucket(n_long + 1), log2_bucket(max_customers), a.c_str(),
                                cus);
  if (len < 0 || (uint64_t)len + 1 > cap || (size_t)len >= sizeof buf) return MRIP_E_INVAL;
  std::memcpy(out, buf, (size_t)len + 1);
  return MRIP_OK;
}

mrip_status mrip_tune_cache_get(const char *path, const char *key, mrip_tune_entry *out) {
  if (!path || !*path || !valid_key(key) || !out) return MRIP_E_INVAL;
  std::ifstream f(path);
  if (!f) return MRIP_E_STATE;
  std::string line;
  bool found = false;
  mrip_tune_entry e{};
  while (std::getline(f, line)) {  // the last line for a key wins
    std::istringstream is(line);
    std::string k;
    mrip_tune_entry t{};
    if (!(is >> k >> t.reps_per_wave >> t.workgroup >> t.plan_split >> t.ms)) continue;
    if (k == key) {
      e = t;
      found = true;
    }
  }
  if (!found) return MRIP_E_STATE;
  *out = e;
  return MRIP_OK;
}

mrip_status mrip_tune_cache_put(const char *path, const char *key, const mrip_tune_entry *e) {
  if (!path || !*path || !valid_key(key) || !e) return MRIP_E_INVAL;
  std::vector<std::string> keep;
  {
    std::ifstream f(path);
    std::string line;
    while (f && std::getline(f, line)) {
      std::istringstream is(line);
      std::string k;
      if (is >> k && k != key) keep.push_back(line);
    }
  }
  // write a whole new file beside the old one, then rename it into place,
  // so a reader never sees half a file
  const std::string tmp = std::string(path) + ".tmp" + std::to_string((long)getpid());
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) return MRIP_E_INVAL;
    for (const std::string &l : keep) f << l << "\n";
    char ms[64];
    std::snprintf(ms, sizeof ms, "%.9g", (double)e->ms);
    f << key << " " << e->reps_per_wave << " " << e->workgroup << " " << e->plan_split << " " << ms
      << "\n";
    if (!f) return MRIP_E_INVAL;
  }
  if (std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return MRIP_E_INVAL;
  }
  return MRIP_OK;
}

}  // extern "C"

// The GEMM tile table: which tile edge (64 or 32) the launches of each role take in sweeps of a
// given block size.  The INLA autotuners (api_inla.hip) fill it by timing whole evaluations;
// the entry points here set, read, clear, save and load it.  The cache file is JSON:
//   {"tiles": [{"b": 128, "role": "schur_update", "tile": 32}, ...]}
// with the roles named as the profiler names the GEMM groups.  A context created while the
// environment variable ADELIA_TUNE_CACHE names a readable file loads it.
#include "../../include/adelia.h"
#include "common.h"
#include "internal_api.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

namespace adelia {

namespace {

const char* const kRoleNames[GT_COUNT] = {"other", "trailing", "trtri", "panel_rows",
                                          "schur_update", "si_W", "si_ZB", "si_ZD"};

int role_of(const std::string& name) {
  for (int r = 0; r < GT_COUNT; ++r)
    if (name == kRoleNames[r]) return r;
  return -1;
}

// The value after "key": in one object's text (a number or a quoted string); empty if absent.
std::string field(const std::string& obj, const char* key) {
  const std::string k = std::string("\"") + key + "\"";
  size_t p = obj.find(k);
  if (p == std::string::npos) return "";
  p = obj.find(':', p + k.size());
  if (p == std::string::npos) return "";
  ++p;
  while (p < obj.size() && (obj[p] == ' ' || obj[p] == '\n' || obj[p] == '\t')) ++p;
  if (p < obj.size() && obj[p] == '"') {
    const size_t e = obj.find('"', p + 1);
    return e == std::string::npos ? "" : obj.substr(p + 1, e - p - 1);
  }
  size_t e = p;
  while (e < obj.size() && (isdigit((unsigned char)obj[e]) || obj[e] == '-')) ++e;
  return obj.substr(p, e - p);
}

}  // namespace

int tune_load_file(const char* path) {
  FILE* fp = fopen(path, "rb");
  if (!fp) return -1;
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = fread(buf, 1, sizeof(buf), fp)) > 0) text.append(buf, got);
  fclose(fp);
  // each {...} inside the "tiles" array is one entry; entries that do not parse are an error
  const size_t arr = text.find("\"tiles\"");
  if (arr == std::string::npos) return -2;
  size_t p = text.find('[', arr);
  const size_t end = text.find(']', arr);
  if (p == std::string::npos || end == std::string::npos) return -2;
  std::vector<std::array<int, 3>> entries;
  while (true) {
    const size_t o = text.find('{', p);
    if (o == std::string::npos || o > end) break;
    const size_t c = text.find('}', o);
    if (c == std::string::npos || c > end) return -2;
    const std::string obj = text.substr(o, c - o + 1);
    const std::string sb = field(obj, "b"), sr = field(obj, "role"), st = field(obj, "tile");
    const int role = role_of(sr);
    const int b = sb.empty() ? 0 : atoi(sb.c_str()), tile = st.empty() ? 0 : atoi(st.c_str());
    if (role < 1 || role == GT_PROWS || b < 1 || b > kMaxBlock || (tile != 32 && tile != 64))
      return -2;
    entries.push_back({b, role, tile});
    p = c + 1;
  }
  for (const auto& e : entries) set_tuned_tile(e[0], e[1], e[2]);
  return (int)entries.size();
}

int tune_save_file(const char* path) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* fp = fopen(tmp.c_str(), "wb");
  if (!fp) return -1;
  fprintf(fp, "{\"tiles\": [");
  bool first = true;
  for (const auto& e : tuned_tiles()) {
    fprintf(fp, "%s\n  {\"b\": %d, \"role\": \"%s\", \"tile\": %d}", first ? "" : ",", e[0],
            kRoleNames[e[1]], e[2]);
    first = false;
  }
  fprintf(fp, "\n]}\n");
  const bool ok = fclose(fp) == 0;
  if (!ok || rename(tmp.c_str(), path) != 0) return -1;
  return 0;
}

void tune_load_env() {
  const char* path = getenv("ADELIA_TUNE_CACHE");
  if (path && *path) (void)tune_load_file(path);
}

void tune_save_env() {
  const char* path = getenv("ADELIA_TUNE_CACHE");
  if (path && *path) (void)tune_save_file(path);
}

}  // namespace adelia

using namespace adelia;

extern "C" {

int adelia_tune_set(int b, int role, int tile) {
  if (b < 1 || b > kMaxBlock) return -1;
  if (role < 1 || role >= GT_COUNT || role == GT_PROWS) return -2;
  if (tile != 32 && tile != 64) return -3;
  set_tuned_tile(b, role, tile);
  return 0;
}

int adelia_tune_get(int b, int role) {
  if (b < 1 || b > kMaxBlock || role < 0 || role >= GT_COUNT) return 0;
  return tuned_tile(b, role);
}

int adelia_tune_clear(void) {
  clear_tuned_tiles();
  return 0;
}

int adelia_tune_save(const char* path) {
  if (!path || !*path) return -1;
  return tune_save_file(path) ? ADELIA_E_UNSUPPORTED : 0;
}

int adelia_tune_load(const char* path) {
  if (!path || !*path) return -1;
  const int r = tune_load_file(path);
  if (r == -1) return ADELIA_E_UNSUPPORTED;
  if (r < 0) {
    set_last_error("tile cache: malformed entry");
    return ADELIA_E_SHAPE;
  }
  return r;
}

}  // extern "C"

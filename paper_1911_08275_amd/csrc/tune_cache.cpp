// Cache of autotuned launch settings (refine factors, work-chunk target,
// waves per workgroup) keyed by a workload signature: kept in memory and in a
// JSON file, one entry per line,
//   "<key>": {"refine": [rx, ry, rz], "chunk_pct": c, "waves": w, "ms": t},
// at $CP_AUTOTUNE_CACHE, else $HOME/.cache/paper_1911_08275_amd/autotune.json.
// Lines that do not parse are skipped, and a file that cannot be written
// leaves the choice in memory only.  Host code, no device work.
#include "cp_internal.h"

#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <sys/stat.h>
#include <unistd.h>

namespace cp {

namespace {

std::mutex g_mu;
std::map<std::string, TuneChoice> g_mem;
bool g_loaded = false;
std::string g_loaded_path;   // the file g_mem mirrors (CP_AUTOTUNE_CACHE may change)

std::string cache_path() {
  const char *e = getenv("CP_AUTOTUNE_CACHE");
  if (e && e[0]) return e;
  const char *home = getenv("HOME");
  return std::string(home && home[0] ? home : "/tmp") + "/.cache/paper_1911_08275_amd/autotune.json";
}

void mkdirs(const std::string &file) {
  for (size_t i = 1; i < file.size(); i++) {
    if (file[i] != '/') continue;
    const std::string d = file.substr(0, i);
    if (mkdir(d.c_str(), 0755) != 0 && errno != EEXIST) return;
  }
}

// "<key>": {"refine": [a, b, c], "chunk_pct": x, "waves": y, "ms": z}
bool parse_line(const char *s, std::string &key, TuneChoice &t) {
  const char *q0 = strchr(s, '"');
  if (!q0) return false;
  const char *q1 = strchr(q0 + 1, '"');
  if (!q1) return false;
  key.assign(q0 + 1, q1 - q0 - 1);
  const char *r = strstr(q1, "\"refine\"");
  const char *c = strstr(q1, "\"chunk_pct\"");
  const char *w = strstr(q1, "\"waves\"");
  const char *m = strstr(q1, "\"ms\"");
  if (!r || !c || !w || !m) return false;
  if (sscanf(r, "\"refine\": [%d, %d, %d]", &t.refine[0], &t.refine[1], &t.refine[2]) != 3)
    return false;
  if (sscanf(c, "\"chunk_pct\": %d", &t.chunk_pct) != 1) return false;
  if (sscanf(w, "\"waves\": %d", &t.waves) != 1) return false;
  if (sscanf(m, "\"ms\": %lf", &t.ms) != 1) return false;
  for (int a = 0; a < 3; a++)
    if (t.refine[a] < 1 || t.refine[a] > 8) return false;
  return t.chunk_pct >= 10 && t.chunk_pct <= 1000 && t.waves >= 1 && t.waves <= 4;
}

void load_locked() {
  const std::string path = cache_path();
  if (g_loaded && path == g_loaded_path) return;
  if (path != g_loaded_path) g_mem.clear();
  g_loaded = true;
  g_loaded_path = path;
  FILE *f = fopen(path.c_str(), "r");
  if (!f) return;
  char line[1024];
  while (fgets(line, sizeof line, f)) {
    std::string key;
    TuneChoice t;
    if (parse_line(line, key, t)) g_mem[key] = t;
  }
  fclose(f);
}

void save_locked() {
  const std::string path = cache_path();
  mkdirs(path);
  const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
  FILE *f = fopen(tmp.c_str(), "w");
  if (!f) return;
  fprintf(f, "{\n");
  size_t i = 0;
  for (const auto &kv : g_mem) {
    const TuneChoice &t = kv.second;
    fprintf(f, " \"%s\": {\"refine\": [%d, %d, %d], \"chunk_pct\": %d, \"waves\": %d, \"ms\": %.4f}%s\n",
            kv.first.c_str(), t.refine[0], t.refine[1], t.refine[2], t.chunk_pct, t.waves, t.ms,
            ++i < g_mem.size() ? "," : "");
  }
  fprintf(f, "}\n");
  const bool ok = fclose(f) == 0;
  if (!ok || rename(tmp.c_str(), path.c_str()) != 0) unlink(tmp.c_str());
}

} // namespace

bool tune_lookup(const std::string &key, TuneChoice &out) {
  std::lock_guard<std::mutex> lock(g_mu);
  load_locked();
  auto it = g_mem.find(key);
  if (it == g_mem.end()) return false;
  out = it->second;
  return true;
}

void tune_store(const std::string &key, const TuneChoice &t) {
  std::lock_guard<std::mutex> lock(g_mu);
  load_locked();
  g_mem[key] = t;
  // merge entries other processes may have written meanwhile, then rewrite
  g_loaded = false;
  std::map<std::string, TuneChoice> mine = g_mem;
  load_locked();
  for (const auto &kv : mine) g_mem[kv.first] = kv.second;
  save_locked();
}

std::string tune_cache_file() { return cache_path(); }

} // namespace cp

// Autotuning of launch choices that leave every result bit for bit the same:
//   * PCG: eager launches or HIP-graph replay of each chunk, and the chunk
//     length between convergence polls (4 or 8 iterations). Both only change
//     when the host learns that the systems have converged and how the
//     launches reach the GPU; the arithmetic is that of eager launches.
//   * GMRES: how many Krylov vectors one workgroup of the dot-product kernel
//     takes (4, 8 or 16); every partial sum covers the same entries in the
//     same order whatever the grouping.
// The PCG choice is measured over a handle's first solves: one warm-up
// solve, then each candidate twice, ranked by the best time per iteration.
// The GMRES choice is measured directly, three launches per candidate on the
// handle's own basis. Choices are kept in a text file keyed by the device
// and the problem ($TPCG_TUNE_CACHE, else $XDG_CACHE_HOME/tpcg/tune.txt, else
// $HOME/.cache/tpcg/tune.txt); a handle of a known key takes the stored
// choice at its first solve. Nothing is stored when no path is writable.
#include <sys/stat.h>
#include <unistd.h>

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <limits>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

#include "tpcg_internal.h"

namespace tpcg {

namespace {

struct PcgCand {
  int graphs, poll;
};
constexpr PcgCand kPcgCands[4] = {{0, 4}, {0, 8}, {1, 4}, {1, 8}};
constexpr int kNumCands = 4;
constexpr int kRepsPerCand = 2;
constexpr int kGmChunks[3] = {4, 8, 16};

std::mutex g_mu;
std::string g_loaded_path;
std::map<std::string, std::string> g_cache;

std::string cache_path() {
  if (const char* p = std::getenv("TPCG_TUNE_CACHE")) return p;
  if (const char* x = std::getenv("XDG_CACHE_HOME")) return std::string(x) + "/tpcg/tune.txt";
  if (const char* hme = std::getenv("HOME")) return std::string(hme) + "/.cache/tpcg/tune.txt";
  return "";
}

// (re)loads the file when the path differs from the one loaded; g_mu held
void load_locked(const std::string& path) {
  if (path == g_loaded_path) return;
  g_cache.clear();
  g_loaded_path = path;
  if (path.empty()) return;
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    const size_t tab = line.find('\t');
    if (tab == std::string::npos) continue;
    g_cache[line.substr(0, tab)] = line.substr(tab + 1);
  }
}

void mkdirs(const std::string& path) {
  for (size_t i = 1; i < path.size(); ++i)
    if (path[i] == '/') mkdir(path.substr(0, i).c_str(), 0755);
}

bool lookup(const std::string& key, std::string& val) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_locked(cache_path());
  auto it = g_cache.find(key);
  if (it == g_cache.end()) return false;
  val = it->second;
  return true;
}

void store(const std::string& key, const std::string& val) {
  std::lock_guard<std::mutex> lk(g_mu);
  const std::string path = cache_path();
  load_locked(path);
  g_cache[key] = val;
  if (path.empty()) return;
  mkdirs(path);
  const std::string tmp = path + ".tmp." + std::to_string(getpid());
  {
    std::ofstream out(tmp, std::ios::trunc);
    if (!out) return;
    for (const auto& kv : g_cache) out << kv.first << '\t' << kv.second << '\n';
    if (!out) return;
  }
  if (std::rename(tmp.c_str(), path.c_str()) != 0) std::remove(tmp.c_str());
}

int get_int(const std::string& val, const char* name, int dflt) {
  std::istringstream ss(val);
  std::string tok;
  const std::string pre = std::string(name) + "=";
  while (ss >> tok)
    if (tok.compare(0, pre.size(), pre) == 0) return std::atoi(tok.c_str() + pre.size());
  return dflt;
}

std::string key_of(const Handle& h) {
  int dev = 0;
  hipGetDevice(&dev);
  hipDeviceProp_t prop{};
  hipGetDeviceProperties(&prop, dev);
  const Geometry& g = h.g;
  std::ostringstream k;
  k << prop.gcnArchName << "/" << prop.multiProcessorCount << "cu|dim" << g.dim << "|" << g.nelx
    << "x" << g.nely << "x" << g.nelz << "|s" << g.s << "|k" << g.k << "|nsys" << h.nsys_built
    << "|" << (h.mixed ? "mixed" : "fp64") << (h.big ? "|big" : "");
  return k.str();
}

bool cand_allowed(const Handle& h, int c) {
  if (!kPcgCands[c].graphs) return true;
  return h.graphs_ok && h.cpk != nullptr && !h.prof_on;
}

void apply(Handle& h, int c) {
  h.graphs_on = kPcgCands[c].graphs;
  h.poll_every = kPcgCands[c].poll;
}

}  // namespace

void tune_before_solve(Handle& h) {
  h.tune_cand = -1;
  if (!h.tune_on || h.tune_decided) return;
  std::string val;
  if (lookup(key_of(h) + "|pcg", val)) {
    h.graphs_on = get_int(val, "graphs", 0);
    h.poll_every = get_int(val, "poll", 4);
    if (h.poll_every < 1 || h.poll_every > kMaxPoll) h.poll_every = 4;
    h.tune_decided = 1;
    h.tune_from_cache = 1;
    return;
  }
  if (h.tune_seen == 0) return;   // warm-up solve in the current configuration
  int c = (h.tune_seen - 1) % kNumCands;
  while (c < kNumCands && !cand_allowed(h, c)) ++c;
  if (c >= kNumCands) c = 0;
  h.tune_cand = c;
  apply(h, c);
}

void tune_after_solve(Handle& h, double ms, int iters) {
  if (!h.tune_on || h.tune_decided) return;
  if (iters <= 0) return;   // no iteration: nothing measured, nothing counted
  if (h.tune_cand >= 0) {
    const double per = ms / iters;
    double& best = h.tune_ms[h.tune_cand];
    if (best <= 0.0 || per < best) best = per;
  }
  ++h.tune_seen;
  if (h.tune_seen <= kNumCands * kRepsPerCand) return;
  int pick = 0;
  double pick_ms = std::numeric_limits<double>::infinity();
  for (int c = 0; c < kNumCands; ++c)
    if (h.tune_ms[c] > 0.0 && h.tune_ms[c] < pick_ms) {
      pick = c;
      pick_ms = h.tune_ms[c];
    }
  apply(h, pick);
  h.tune_decided = 1;
  std::ostringstream v;
  v << "graphs=" << kPcgCands[pick].graphs << " poll=" << kPcgCands[pick].poll
    << " ms_per_iter=" << pick_ms;
  store(key_of(h) + "|pcg", v.str());
}

void tune_gmres(Handle& h, int nsys, int m) {
  if (!h.tune_on || h.tune_gm_decided) return;
  const std::string key = key_of(h) + "|gmres";
  std::string val;
  if (lookup(key, val)) {
    const int c = get_int(val, "chunk", 8);
    h.gm_chunk = (c == 4 || c == 16) ? c : 8;
    h.tune_gm_decided = 1;
    return;
  }
  const int nv = m < 2 ? 1 : m;
  int pick = 8;
  double best = std::numeric_limits<double>::infinity();
  for (int c : kGmChunks) {
    const double ms = gmres_time_dots(h, nsys, nv, c);
    if (ms > 0.0 && ms < best) {
      best = ms;
      pick = c;
    }
  }
  h.gm_chunk = pick;
  h.tune_gm_decided = 1;
  std::ostringstream v;
  v << "chunk=" << pick << " ms=" << best << " vectors=" << nv;
  store(key, v.str());
}

}  // namespace tpcg

// The autotuner's choices, kept for the whole process and saved to / loaded from a text file,
// so that later grids and later runs take the same kernel variants without timing them again.
//
// An entry is one line "<key> <choice>": the key names the device (architecture and compute
// unit count), the kind of product and every parameter the timing depended on; the choice is
// the variant index the tuner kept.
#include <cstdio>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

#include "api_internal.h"
#include "grid.h"

namespace qflex {
namespace {

std::mutex g_mu;
std::map<std::string, int>& table() {
  static std::map<std::string, int> t;
  return t;
}

}  // namespace

std::string device_signature(int device) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, device) != hipSuccess) return "dev?";
  std::string arch = p.gcnArchName;
  for (char& c : arch)
    if (c == ' ' || c == ':') c = '_';
  return arch + "_cu" + std::to_string(p.multiProcessorCount);
}

bool tune_cache_get(const std::string& key, int* choice) {
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = table().find(key);
  if (it == table().end()) return false;
  *choice = it->second;
  return true;
}

void tune_cache_put(const std::string& key, int choice) {
  std::lock_guard<std::mutex> lock(g_mu);
  table()[key] = choice;
}

}  // namespace qflex

extern "C" {

qflex_status qflex_autotune_cache_save(const char* path) {
  return qflex::run_guarded([&] {
    if (!path) qflex::fail(QFLEX_E_INVALID, "NULL path");
    std::ostringstream o;
    {
      std::lock_guard<std::mutex> lock(qflex::g_mu);
      for (const auto& kv : qflex::table()) o << kv.first << " " << kv.second << "\n";
    }
    std::ofstream f(path, std::ios::trunc);
    if (!f) qflex::fail(QFLEX_E_INVALID, std::string("cannot write ") + path);
    f << o.str();
    if (!f) qflex::fail(QFLEX_E_INVALID, std::string("cannot write ") + path);
  });
}

qflex_status qflex_autotune_cache_load(const char* path, int64_t* n_loaded) {
  return qflex::run_guarded([&] {
    if (!path) qflex::fail(QFLEX_E_INVALID, "NULL path");
    std::ifstream f(path);
    if (!f) qflex::fail(QFLEX_E_INVALID, std::string("cannot read ") + path);
    std::map<std::string, int> got;
    std::string line;
    int64_t lineno = 0;
    while (std::getline(f, line)) {
      ++lineno;
      if (line.empty()) continue;
      std::istringstream in(line);
      std::string key;
      int choice = -1;
      std::string rest;
      if (!(in >> key >> choice) || (in >> rest) || choice < 0)
        qflex::fail(QFLEX_E_INVALID, std::string(path) + ": malformed line " +
                                         std::to_string(lineno));
      got[key] = choice;
    }
    {
      std::lock_guard<std::mutex> lock(qflex::g_mu);
      for (const auto& kv : got) qflex::table()[kv.first] = kv.second;
    }
    if (n_loaded) *n_loaded = (int64_t)got.size();
  });
}

int64_t qflex_autotune_cache_size(void) {
  std::lock_guard<std::mutex> lock(qflex::g_mu);
  return (int64_t)qflex::table().size();
}

void qflex_autotune_cache_clear(void) {
  std::lock_guard<std::mutex> lock(qflex::g_mu);
  qflex::table().clear();
}

}  // extern "C"

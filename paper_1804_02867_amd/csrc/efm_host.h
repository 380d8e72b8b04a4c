// efm_host.h -- host-side internals shared by the single-network and batched
// entry points: the handle structs, device-table building and result assembly.
#pragma once
#include <string>
#include <vector>

#include "../../include/efm.h"
#include "efm_internal.h"

struct efm_network {
  int m = 0, n = 0, mi = 0, W = 0, Wt = 0, MWt = 0;
  std::vector<int32_t> S;
  std::vector<uint8_t> rev, ext;
  std::vector<int> int_row;   // internal metabolite -> row of S
  void *blob = nullptr;
  efm::DevNet dn{};
};

struct efm_result {
  int W = 0, n = 0;
  uint32_t status = 0;
  int64_t count = 0;
  std::vector<efm::u64> keys;
  std::vector<int64_t> flux;
  std::vector<efm_level_stats> levels;
};

// thread-local error text + status code
efm_status fail(efm_status code, const char *fmt, ...);
size_t align256(size_t x);
// smallest instantiated (reaction words, metabolite words) pair covering W, MW
bool choose_shape(int W, int MW, int *Wt, int *MWt);
void build_tables(const efm_network *N, int Wt, int MWt, std::vector<char> &host, std::vector<size_t> &offs);
efm::DevNet bind_tables(const efm_network *N, int Wt, int MWt, char *base, const std::vector<size_t> &offs);
void assemble(efm_result *R, int Wt, const efm::u64 *fk, int64_t cnt, const int64_t *ff, int ffstride);

// Hook into the level loop of the single-network traversal.
struct LevelHook {
  virtual ~LevelHook() = default;
  // true: when the survivors exceed the frontier cap, score() writes one score
  // word per survivor (ascending = kept first) and the truncation ranks by it
  // before the canonical key
  virtual bool orders() const { return false; }
  virtual hipError_t score(const efm_network *, const efm::DevLevel &, int64_t, uint32_t *, hipStream_t) {
    return hipSuccess;
  }
  // called with every new frontier: `count` states, keys SoA [Wt][fcap]
  virtual efm_status frontier(const efm_network *, const efm::u64 *, const efm::u64 *, int64_t, int64_t, int,
                              hipStream_t) {
    return EFM_OK;
  }
};

efm_status enumerate_impl(const efm_network *N, int32_t target, const efm_enum_opts *opts, LevelHook *hook,
                          efm_result **out);

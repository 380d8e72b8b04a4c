// efm_api.hip -- host side of the C ABI (include/efm.h): network tables, the
// workspace layout and the level loop that drives the kernels.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/efm.h"
#include "efm_host.h"

using efm::u64;

namespace {
thread_local std::string g_err;
}  // namespace

efm_status fail(efm_status code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) {                                                               \
      rc = fail(EFM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));              \
      goto done;                                                                          \
    }                                                                                     \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// splitmix64, for the Zobrist keys of the child hash
u64 splitmix64(u64 &state) {
  u64 z = (state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// supported (reaction words, metabolite words) instantiations
static const int kShapes[][2] = {{1, 1}, {1, 2}, {2, 1}, {2, 2}, {2, 4}, {4, 1}, {4, 2}, {4, 4},
                                 {8, 2}, {8, 4}, {8, 8}, {16, 4}, {16, 8}, {16, 16}};

bool choose_shape(int W, int MW, int *Wt, int *MWt) {
  for (auto &sh : kShapes)
    if (sh[0] >= W && sh[1] >= MW) { *Wt = sh[0]; *MWt = sh[1]; return true; }
  return false;
}


// Device tables of one network at the given padded widths, laid out in one host
// buffer (offsets of the parts in `offs`).  Used for single networks and, at a
// common width, for every member of a batch.
void build_tables(const efm_network *N, int Wt, int MWt, std::vector<char> &host, std::vector<size_t> &offs) {
  const int n = N->n, mi = N->mi;

  // host tables
  std::vector<u64> prodM((size_t)n * MWt), consM((size_t)n * MWt), revM((size_t)n * MWt),
      touchM((size_t)n * MWt), oddM((size_t)n * MWt), fwdR((size_t)std::max(mi, 1) * Wt), bwdR((size_t)std::max(mi, 1) * Wt),
      allR((size_t)std::max(mi, 1) * Wt), nbrR((size_t)n * Wt), revb(Wt), zob(n);
  std::vector<int32_t> Sint((size_t)std::max(mi, 1) * n);
  for (int k = 0; k < mi; ++k) {
    const int row = N->int_row[k];
    for (int r = 0; r < n; ++r) {
      const int32_t s = N->S[(size_t)row * n + r];
      Sint[(size_t)k * n + r] = s;
      if (s == 0) continue;
      const u64 mb = 1ull << (k & 63), rb = 1ull << (r & 63);
      const int mq = k >> 6, rw = r >> 6;
      touchM[(size_t)r * MWt + mq] |= mb;
      if (s & 1) oddM[(size_t)r * MWt + mq] |= mb;
      allR[(size_t)k * Wt + rw] |= rb;
      if (N->rev[r]) {
        revM[(size_t)r * MWt + mq] |= mb;
        fwdR[(size_t)k * Wt + rw] |= rb;
        bwdR[(size_t)k * Wt + rw] |= rb;
      } else if (s > 0) {
        prodM[(size_t)r * MWt + mq] |= mb;
        bwdR[(size_t)k * Wt + rw] |= rb;   // a producer balances a consumed metabolite
      } else {
        consM[(size_t)r * MWt + mq] |= mb;
        fwdR[(size_t)k * Wt + rw] |= rb;   // a consumer balances a produced metabolite
      }
    }
  }
  for (int r = 0; r < n; ++r) {
    if (N->rev[r]) revb[r >> 6] |= 1ull << (r & 63);
    for (int q = 0; q < MWt; ++q) {
      u64 bits = touchM[(size_t)r * MWt + q];
      while (bits) {
        const int k = q * 64 + __builtin_ctzll(bits);
        bits &= bits - 1;
        for (int w = 0; w < Wt; ++w) nbrR[(size_t)r * Wt + w] |= allR[(size_t)k * Wt + w];
      }
    }
  }
  // per-reaction column entries for the rank test (internal metabolite, coefficient)
  std::vector<uint32_t> ent((size_t)n * efm::kMaxEnt, 0xFFFF0000u);
  std::vector<int32_t> nnz(n, 0);
  for (int r = 0; r < n; ++r) {
    int c = 0;
    bool fits = true;
    for (int k = 0; k < mi; ++k) {
      const int32_t v = Sint[(size_t)k * n + r];
      if (v == 0) continue;
      if (c >= efm::kMaxEnt || v < -32768 || v > 32767 || k > 0xFFFE) { fits = false; continue; }
      ent[(size_t)r * efm::kMaxEnt + c] = ((uint32_t)k << 16) | ((uint32_t)v & 0xFFFFu);
      c++;
    }
    nnz[r] = fits ? c : -1;
  }
  u64 st = 0x5EEDF00DCAFEull;
  for (int r = 0; r < n; ++r) zob[r] = splitmix64(st);

  struct Part { const void *src; size_t bytes; };
  const Part parts[] = {
      {prodM.data(), prodM.size() * 8}, {consM.data(), consM.size() * 8},
      {revM.data(), revM.size() * 8},   {touchM.data(), touchM.size() * 8},
      {fwdR.data(), fwdR.size() * 8},   {bwdR.data(), bwdR.size() * 8},
      {allR.data(), allR.size() * 8},   {nbrR.data(), nbrR.size() * 8},
      {revb.data(), revb.size() * 8},   {Sint.data(), Sint.size() * 4},
      {zob.data(), zob.size() * 8},     {ent.data(), ent.size() * 4},
      {nnz.data(), nnz.size() * 4},     {oddM.data(), oddM.size() * 8}};
  offs.clear();
  size_t total = 0;
  for (const auto &p : parts) { offs.push_back(total); total += align256(p.bytes); }
  host.assign(total, 0);
  for (size_t i = 0; i < sizeof(parts) / sizeof(parts[0]); ++i) memcpy(host.data() + offs[i], parts[i].src, parts[i].bytes);
}

efm::DevNet bind_tables(const efm_network *N, int Wt, int MWt, char *base, const std::vector<size_t> &offs) {
  auto at = [&](int i) { return (const u64 *)(base + offs[i]); };
  efm::DevNet d{};
  d.n = N->n; d.mi = N->mi; d.Wt = Wt; d.MWt = MWt;
  d.rxn_prodM = at(0); d.rxn_consM = at(1); d.rxn_revM = at(2); d.rxn_touchM = at(3);
  d.met_fwdR = at(4); d.met_bwdR = at(5); d.met_allR = at(6); d.rxn_nbrR = at(7);
  d.rev_bits = at(8);
  d.Sint = (const int32_t *)(base + offs[9]);
  d.zob = at(10);
  d.rxn_ent = (const uint32_t *)(base + offs[11]);
  d.rxn_nnz = (const int32_t *)(base + offs[12]);
  d.rxn_oddM = at(13);
  return d;
}


// Fill a result from found pathways: keys SoA (word w of pathway i at
// fk[w * cnt + i], Wt words) and their nonzero fluxes in key order
// (ff[i * ffstride + j] for the j-th reaction).  Sorted canonically, dense.
void assemble(efm_result *R, int Wt, const u64 *fk, int64_t cnt, const int64_t *ff, int ffstride) {
  const int W = R->W, n = R->n;
  std::vector<int64_t> order(cnt);
  for (int64_t i = 0; i < cnt; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    for (int w = Wt - 1; w >= 0; --w) {
      const u64 x = fk[(size_t)w * cnt + a], y = fk[(size_t)w * cnt + b];
      if (x != y) return x < y;
    }
    return false;
  });
  R->count = cnt;
  R->keys.assign((size_t)cnt * W, 0);
  R->flux.assign((size_t)cnt * n, 0);
  for (int64_t i = 0; i < cnt; ++i) {
    const int64_t src = order[i];
    int j = 0;
    for (int w = 0; w < Wt; ++w) {
      u64 bits = fk[(size_t)w * cnt + src];
      if (w < W) R->keys[(size_t)i * W + w] = bits;
      while (bits) {
        const int r = w * 64 + __builtin_ctzll(bits);
        bits &= bits - 1;
        R->flux[(size_t)i * n + r] = ff[(size_t)src * ffstride + j];
        j++;
      }
    }
  }
}

extern "C" {

const char *efm_last_error(void) { return g_err.c_str(); }

const char *efm_status_string(efm_status s) {
  switch (s) {
    case EFM_OK: return "ok";
    case EFM_EINVAL: return "invalid argument";
    case EFM_ENOMEM: return "workspace or capacity too small";
    case EFM_EDEVICE: return "HIP error";
    case EFM_EOVERFLOW: return "integer overflow";
    default: return "unknown status";
  }
}

efm_status efm_network_create(int32_t n_met, int32_t n_rxn, const int32_t *S, const uint8_t *reversible,
                              const uint8_t *external, efm_network **out) {
  if (!S || !reversible || !external || !out) return fail(EFM_EINVAL, "null pointer");
  if (n_met <= 0 || n_rxn <= 0 || n_rxn > EFM_MAX_RXN)
    return fail(EFM_EINVAL, "bad dimensions %d x %d (reactions must be 1..%d)", n_met, n_rxn, EFM_MAX_RXN);
  efm_network *N = new (std::nothrow) efm_network;
  if (!N) return fail(EFM_ENOMEM, "host allocation failed");
  N->m = n_met;
  N->n = n_rxn;
  N->S.assign(S, S + (size_t)n_met * n_rxn);
  N->rev.assign(reversible, reversible + n_rxn);
  N->ext.assign(external, external + n_met);
  for (int i = 0; i < n_met; ++i)
    if (!N->ext[i]) N->int_row.push_back(i);
  N->mi = (int)N->int_row.size();
  N->W = (n_rxn + 63) / 64;
  const int MW = std::max(1, (N->mi + 63) / 64);
  if (N->mi > 1024) {
    delete N;
    return fail(EFM_EINVAL, "%d internal metabolites (at most 1024)", (int)N->mi);
  }
  choose_shape(N->W, MW, &N->Wt, &N->MWt);
  std::vector<char> host;
  std::vector<size_t> offs;
  build_tables(N, N->Wt, N->MWt, host, offs);
  hipError_t e = hipMalloc(&N->blob, host.size());
  if (e != hipSuccess) {
    delete N;
    return fail(EFM_EDEVICE, "hipMalloc(%zu) failed: %s", host.size(), hipGetErrorString(e));
  }
  e = hipMemcpy(N->blob, host.data(), host.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(N->blob);
    delete N;
    return fail(EFM_EDEVICE, "hipMemcpy failed: %s", hipGetErrorString(e));
  }
  N->dn = bind_tables(N, N->Wt, N->MWt, (char *)N->blob, offs);
  *out = N;
  return EFM_OK;
}

efm_status efm_network_destroy(efm_network *net) {
  if (!net) return EFM_OK;
  if (net->blob) (void)hipFree(net->blob);
  delete net;
  return EFM_OK;
}

}  // extern "C"

namespace {

struct Layout {
  int64_t ucap, fcap, ecap, tcap;
  int xwaves;
  size_t off_counters, off_hist, off_selst, off_root, off_sx, off_fa_keys, off_fa_hash, off_fb_keys, off_fb_hash,
      off_table, off_surv, off_rankq, off_parq, off_parmask, off_exactq, off_sel, off_skey, off_fkeys, off_fflux,
      off_xs, off_sscore, total;
};

int64_t next_pow2(int64_t x) {
  int64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

Layout make_layout(const efm_network *N, const efm_enum_opts *o) {
  Layout L{};
  L.ucap = (o && o->unique_cap > 0) ? o->unique_cap : ((int64_t)1 << 22);
  L.ucap = std::max<int64_t>(L.ucap, 64);
  const int64_t fcapo = (o && o->frontier_cap > 0) ? o->frontier_cap : L.ucap;
  L.fcap = std::max<int64_t>(1, std::min(fcapo, L.ucap));
  L.ecap = (o && o->found_cap > 0) ? o->found_cap : ((int64_t)1 << 18);
  L.tcap = std::max<int64_t>(1024, next_pow2(2 * L.ucap));
  L.xwaves = 512;
  const int Wt = N->Wt;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o2 = off; off += align256(bytes); return o2; };
  L.off_counters = take(efm::kNumCounters * efm::kCounterStride * 8);
  L.off_hist = take(3 * efm::kHistCopies * 256 * 4);
  L.off_selst = take(2 * sizeof(efm::SelState));
  L.off_root = take((size_t)Wt * 8);
  L.off_sx = take((size_t)N->n * 4);
  L.off_fa_keys = take((size_t)Wt * L.fcap * 8);
  L.off_fa_hash = take((size_t)L.fcap * 8);
  L.off_fb_keys = take((size_t)Wt * L.fcap * 8);
  L.off_fb_hash = take((size_t)L.fcap * 8);
  L.off_table = take((size_t)L.tcap * 8);
  L.off_surv = take((size_t)L.ucap * 8);
  L.off_rankq = take((size_t)L.ucap * 8);
  L.off_parq = take((size_t)L.fcap * 8);            // parents with row-closed children
  L.off_parmask = take((size_t)L.fcap * Wt * 8);
  L.off_exactq = take((size_t)L.ucap * 8);
  L.off_sel = take((size_t)efm::sel_stride(L.ucap));   // read four members at a time
  L.off_skey = take((size_t)efm::sel_stride(L.ucap) * 8);
  L.off_fkeys = take((size_t)Wt * L.ecap * 8);
  L.off_fflux = take((size_t)L.ecap * efm::kMaxDepth * 8);
  L.off_xs = take((size_t)L.xwaves * std::max(N->mi, 1) * 64 * sizeof(efm::i128));
  L.off_sscore = (o && (o->flags & EFM_OPT_LEARNED)) ? take((size_t)L.ucap * 4) : 0;
  L.total = off;
  return L;
}

}  // namespace

extern "C" {

efm_status efm_workspace_query(const efm_network *net, const efm_enum_opts *opts, size_t *bytes) {
  if (!net || !bytes) return fail(EFM_EINVAL, "null pointer");
  *bytes = make_layout(net, opts).total;
  return EFM_OK;
}

efm_status efm_enumerate(const efm_network *N, int32_t target, const efm_enum_opts *opts,
                         efm_result **out) {
  if (opts && (opts->flags & EFM_OPT_LEARNED)) {
    efm_enum_opts o = *opts;
    o.flags &= ~EFM_OPT_LEARNED;   // the score array is only used by efm_enumerate_learned
    if (o.workspace && o.workspace_bytes < make_layout(N, opts).total)
      return fail(EFM_ENOMEM, "workspace too small");
    return enumerate_impl(N, target, &o, nullptr, out);
  }
  return enumerate_impl(N, target, opts, nullptr, out);
}

}  // extern "C"

// The level loop shared by the plain traversal, the learned ordering (`hook`
// scores the survivors when they exceed the frontier cap) and trace collection
// (`hook` sees every new frontier).
efm_status enumerate_impl(const efm_network *N, int32_t target, const efm_enum_opts *opts, LevelHook *hook,
                          efm_result **out) {
  if (!N || !out) return fail(EFM_EINVAL, "null pointer");
  if (target < 0 || target >= N->m || !N->ext[target])
    return fail(EFM_EINVAL, "target %d is not an external metabolite", target);
  efm_enum_opts o{};
  if (opts) o = *opts;
  const int n = N->n, Wt = N->Wt;
  std::vector<u64> root(Wt, 0);
  std::vector<int32_t> sx(n);
  int nroot = 0;
  for (int r = 0; r < n; ++r) {
    const int32_t s = N->S[(size_t)target * n + r];
    sx[r] = s;
    if (s > 0 || (s < 0 && N->rev[r])) { root[r >> 6] |= 1ull << (r & 63); nroot++; }
  }
  if (nroot == 0) return fail(EFM_EINVAL, "no reaction can produce target %d", target);
  int D = o.depth_cap > 0 ? o.depth_cap : EFM_MAX_DEPTH;
  D = std::min(D, EFM_MAX_DEPTH);
  D = std::min(D, n);
  const Layout Lo = make_layout(N, &o);
  if (o.workspace && o.workspace_bytes < Lo.total)
    return fail(EFM_ENOMEM, "workspace of %zu bytes, %zu needed", o.workspace_bytes, Lo.total);
  const bool timing = (o.flags & EFM_OPT_TIME_KERNELS) != 0;
  hipStream_t s = (hipStream_t)o.stream;

  efm_status rc = EFM_OK;
  char *ws = (char *)o.workspace;
  bool owned = false;
  efm_result *R = nullptr;
  hipEvent_t ev[12] = {};
  std::vector<u64> hcs((size_t)efm::kNumCounters * efm::kCounterStride), hc(efm::kNumCounters);
  u64 found_host = 0;
  efm::SelState sel_init{};
  int64_t nparents = 1, nfound = 0;
  int level = 0, next_tag = 1;
  double branching = 1.0;
  uint32_t status = 0;
  std::vector<efm_level_stats> stats;
  efm::DevLevel L{};
  u64 *fa_keys, *fa_hash, *fb_keys, *fb_hash;
  bool ordered = false;
  uint32_t *sscore = nullptr;
  std::vector<std::pair<int, int>> passes;   // (byte, refill) of the truncation's radix passes

  if (!ws) {
    HIPCHK(hipMalloc((void **)&ws, Lo.total));
    owned = true;
  }
  if (timing)
    for (auto &e : ev) HIPCHK(hipEventCreate(&e));

  fa_keys = (u64 *)(ws + Lo.off_fa_keys);
  fa_hash = (u64 *)(ws + Lo.off_fa_hash);
  fb_keys = (u64 *)(ws + Lo.off_fb_keys);
  fb_hash = (u64 *)(ws + Lo.off_fb_hash);
  L.counters = (u64 *)(ws + Lo.off_counters);
  L.hist = (uint32_t *)(ws + Lo.off_hist);
  L.selst = (efm::SelState *)(ws + Lo.off_selst);
  L.Sx = (const int32_t *)(ws + Lo.off_sx);
  L.table = (u64 *)(ws + Lo.off_table);
  L.surv = (u64 *)(ws + Lo.off_surv);
  L.rankq = (u64 *)(ws + Lo.off_rankq);
  L.parq = (u64 *)(ws + Lo.off_parq);
  L.parmask = (u64 *)(ws + Lo.off_parmask);
  L.exactq = (u64 *)(ws + Lo.off_exactq);
  L.ucap = Lo.ucap;
  L.fcap = Lo.fcap;
  L.sel = (uint8_t *)(ws + Lo.off_sel);
  L.skey = (uint8_t *)(ws + Lo.off_skey);
  L.fkeys = (u64 *)(ws + Lo.off_fkeys);
  L.fflux = (int64_t *)(ws + Lo.off_fflux);
  L.ecap = Lo.ecap;
  L.xscratch = (efm::i128 *)(ws + Lo.off_xs);
  L.xwaves = Lo.xwaves;
  L.depth_cap = D;
  L.debug_prime = (o.flags & EFM_OPT_EXACT_RANK) ? 1 : 0;
  L.no_gf2 = (o.flags & EFM_OPT_NO_GF2) ? 1 : 0;
  ordered = hook && hook->orders();
  if (ordered && !(o.flags & EFM_OPT_LEARNED)) {
    rc = fail(EFM_EINVAL, "learned ordering needs the EFM_OPT_LEARNED workspace layout");
    goto done;
  }
  sscore = ordered ? (uint32_t *)(ws + Lo.off_sscore) : nullptr;
  L.sscore = sscore;

  HIPCHK(hipMemcpyAsync(ws + Lo.off_root, root.data(), Wt * 8, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ws + Lo.off_sx, sx.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
  HIPCHK(efm::launch_clear(L.table, (size_t)Lo.tcap, s));
  HIPCHK(hipMemsetAsync(L.counters, 0, efm::kNumCounters * efm::kCounterStride * 8, s));
  for (int w = 0; w < Wt; ++w) HIPCHK(hipMemsetAsync(fa_keys + (size_t)w * Lo.fcap, 0, 8, s));
  HIPCHK(hipMemsetAsync(fa_hash, 0, 8, s));

  while (nparents > 0 && level < D) {
    // per-level counters (the found count persists)
    found_host = (u64)nfound;
    HIPCHK(hipMemsetAsync(L.counters, 0, efm::kNumCounters * efm::kCounterStride * 8, s));
    HIPCHK(hipMemcpyAsync(L.counters + efm::cslot(efm::kFound), &found_host, 8, hipMemcpyHostToDevice, s));
    L.keys = fa_keys;
    L.hash = fa_hash;
    L.nkeys = fb_keys;
    L.nhash = fb_hash;
    L.nparents = nparents;
    L.level = level;
    L.root_cand = level == 0 ? (const u64 *)(ws + Lo.off_root) : nullptr;
    L.nfound_prev = nfound;

    // table slots for this level: twice the children the previous level's
    // branching predicts, at least 1024; rerun at full size if that was too few
    {
      int64_t est = level == 0 ? nroot : (int64_t)((double)nparents * branching * 1.5) + 1024;
      int64_t tl = std::max<int64_t>(1024, next_pow2(2 * est));
      tl = std::min<int64_t>(tl, Lo.tcap);
      for (int attempt = 0;; ++attempt) {
        if (next_tag > 127) {
          HIPCHK(efm::launch_clear(L.table, (size_t)Lo.tcap, s));
          next_tag = 1;
        }
        L.tag = next_tag++;
        L.tmask = (u64)tl - 1;
        if (timing) HIPCHK(hipEventRecord(ev[0], s));
        HIPCHK(efm::launch_expand(N->dn, L, s));
        if (timing) HIPCHK(hipEventRecord(ev[1], s));
        HIPCHK(efm::launch_rank_parent(N->dn, L, (o.flags & EFM_OPT_NO_PRUNE) ? 0 : 1, s));
        HIPCHK(efm::launch_rank(N->dn, L, 0, s));
        if (timing) HIPCHK(hipEventRecord(ev[2], s));
        HIPCHK(efm::launch_exact(N->dn, L, s));
        if (timing) HIPCHK(hipEventRecord(ev[3], s));
        HIPCHK(hipMemcpyAsync(hcs.data(), L.counters, hcs.size() * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int c = 0; c < efm::kNumCounters; ++c) hc[c] = hcs[efm::cslot(c)];
        const bool table_full = (hc[efm::kFlags] & efm::kFlagUniqueOverflow) != 0;
        if (!table_full || tl == Lo.tcap) break;
        // discard this attempt: its emissions sit past nfound and are overwritten
        tl = Lo.tcap;
        found_host = (u64)nfound;
        HIPCHK(hipMemsetAsync(L.counters, 0, efm::kNumCounters * efm::kCounterStride * 8, s));
        HIPCHK(hipMemcpyAsync(L.counters + efm::cslot(efm::kFound), &found_host, 8, hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
      }
    }
    {
      const u64 fl = hc[efm::kFlags];
      if (fl & (efm::kFlagUniqueOverflow | efm::kFlagQueueOverflow)) {
        rc = fail(EFM_ENOMEM, "level %d: more than unique_cap=%lld distinct children; raise unique_cap",
                  level + 1, (long long)Lo.ucap);
        goto done;
      }
      if (fl & efm::kFlagFoundOverflow) {
        rc = fail(EFM_ENOMEM, "more than found_cap=%lld pathways; raise found_cap", (long long)Lo.ecap);
        goto done;
      }
      if (fl & efm::kFlagIntOverflow) {
        rc = fail(EFM_EOVERFLOW, "level %d: exact arithmetic exceeded 128-bit headroom", level + 1);
        goto done;
      }
      if ((fl & efm::kFlagDepthCapped) || hc[efm::kCapped] > 0) status |= EFM_DEPTH_CAPPED;
    }
    const int64_t nsurv = (int64_t)hc[efm::kSurv];
    int use_sel = 0;
    float ms_sel = 0.f;
    if (o.frontier_cap > 0 && nsurv > o.frontier_cap) {
      if (timing) HIPCHK(hipEventRecord(ev[4], s));
      use_sel = 1;
      status |= EFM_FRONTIER_TRUNCATED;
      HIPCHK(hipMemsetAsync(L.sel, 2, (size_t)nsurv, s));
      HIPCHK(hipMemsetAsync(L.hist, 0, 3 * efm::kHistCopies * 256 * 4, s));
      sel_init = efm::SelState{};
      sel_init.needed = o.frontier_cap;
      sel_init.nb = nsurv;
      HIPCHK(hipMemcpyAsync(L.selst, &sel_init, sizeof(sel_init), hipMemcpyHostToDevice, s));
      // radix passes from the most significant byte: with a learned ordering the
      // four bytes of the score word come first, then the key's bytes
      passes.clear();
      if (ordered) {
        HIPCHK(hook->score(N, L, nsurv, sscore, s));
        for (int b = 3; b >= 0; --b) passes.push_back({Wt * 8 + b, b == 3});
      }
      {
        const int top = (n - 1) / 8;
        for (int byte = top; byte >= 0; --byte) passes.push_back({byte, byte == top || (byte & 7) == 7});
      }
      // histogram of the first byte; then one sweep per further byte that applies
      // the previous byte's decision and counts the next; the last decision alone
      HIPCHK(efm::launch_select_hist(N->dn, L, passes[0].first, passes[0].second, 0, s));
      for (size_t pass = 1; pass < passes.size(); ++pass)
        HIPCHK(efm::launch_select_step(N->dn, L, passes[pass - 1].first, passes[pass].first, passes[pass].second,
                                       (int)pass, s));
      HIPCHK(efm::launch_select_split(N->dn, L, passes.back().first, (int)passes.size() - 1, s));
      if (timing) HIPCHK(hipEventRecord(ev[5], s));
    }
    if (timing) HIPCHK(hipEventRecord(ev[6], s));
    HIPCHK(efm::launch_materialize(N->dn, L, use_sel, s));
    if (timing) {
      HIPCHK(hipEventRecord(ev[7], s));
      HIPCHK(hipEventSynchronize(ev[7]));
    }
    efm_level_stats st{};
    st.parents = nparents;
    st.children = (int64_t)hc[efm::kChildren];
    st.unique = (int64_t)hc[efm::kUnique];
    st.row_closed = (int64_t)hc[efm::kRowClosed];
    st.pruned = (int64_t)hc[efm::kPruned];
    st.independent = (int64_t)hc[efm::kIndep];
    st.emitted = (int64_t)hc[efm::kEmitted];
    st.kept = use_sel ? o.frontier_cap : nsurv;
    st.rank_rows = (int64_t)hc[efm::kRankRows];
    if (timing) {
      float t;
      HIPCHK(hipEventElapsedTime(&t, ev[0], ev[1])); st.ms_expand = t;
      HIPCHK(hipEventElapsedTime(&t, ev[1], ev[2])); st.ms_rank = t;
      HIPCHK(hipEventElapsedTime(&t, ev[2], ev[3])); st.ms_exact = t;
      if (use_sel) { HIPCHK(hipEventElapsedTime(&t, ev[4], ev[5])); ms_sel = t; }
      st.ms_select = ms_sel;
      HIPCHK(hipEventElapsedTime(&t, ev[6], ev[7])); st.ms_materialize = t;
    }
    stats.push_back(st);
    if (hook) {
      const efm_status hr = hook->frontier(N, L.nkeys, L.nhash, Lo.fcap, st.kept, level, s);
      if (hr != EFM_OK) { rc = hr; goto done; }
    }
    nfound = std::min<int64_t>((int64_t)hc[efm::kFound], Lo.ecap);
    if (level > 0 && nparents > 0) branching = std::max(1.0, (double)st.children / (double)nparents);
    std::swap(fa_keys, fb_keys);
    std::swap(fa_hash, fb_hash);
    nparents = st.kept;
    level++;
  }
  HIPCHK(hipStreamSynchronize(s));

  R = new (std::nothrow) efm_result;
  if (!R) { rc = fail(EFM_ENOMEM, "host allocation failed"); goto done; }
  R->W = N->W;
  R->n = n;
  R->status = status;
  R->levels = stats;
  {
    std::vector<u64> fk((size_t)Wt * std::max<int64_t>(nfound, 1));
    std::vector<int64_t> ff((size_t)std::max<int64_t>(nfound, 1) * efm::kMaxDepth);
    for (int w = 0; w < Wt && nfound > 0; ++w)
      HIPCHK(hipMemcpy(fk.data() + (size_t)w * nfound, L.fkeys + (size_t)w * Lo.ecap, (size_t)nfound * 8,
                       hipMemcpyDeviceToHost));
    if (nfound > 0)
      HIPCHK(hipMemcpy(ff.data(), L.fflux, (size_t)nfound * efm::kMaxDepth * 8, hipMemcpyDeviceToHost));
    assemble(R, Wt, fk.data(), nfound, ff.data(), efm::kMaxDepth);
  }

done:
  if (timing)
    for (auto &e : ev)
      if (e) (void)hipEventDestroy(e);
  if (owned && ws) {
    (void)hipStreamSynchronize(s);
    (void)hipFree(ws);
  }
  if (rc != EFM_OK) {
    delete R;
    return rc;
  }
  *out = R;
  return EFM_OK;
}

extern "C" {

efm_status efm_result_info(const efm_result *res, int64_t *n_pathways, int32_t *words, uint32_t *status_flags,
                           int32_t *n_levels) {
  if (!res) return fail(EFM_EINVAL, "null result");
  if (n_pathways) *n_pathways = res->count;
  if (words) *words = res->W;
  if (status_flags) *status_flags = res->status;
  if (n_levels) *n_levels = (int32_t)res->levels.size();
  return EFM_OK;
}

efm_status efm_result_stats(const efm_result *res, efm_level_stats *stats, int32_t max_levels) {
  if (!res || (!stats && max_levels > 0)) return fail(EFM_EINVAL, "null pointer");
  const int k = std::min<int>(max_levels, (int)res->levels.size());
  for (int i = 0; i < k; ++i) stats[i] = res->levels[i];
  return EFM_OK;
}

efm_status efm_result_bitsets(const efm_result *res, uint64_t *dst, int64_t dst_words) {
  if (!res || (!dst && res->count > 0)) return fail(EFM_EINVAL, "null pointer");
  if (dst_words < res->count * res->W)
    return fail(EFM_EINVAL, "buffer of %lld words, %lld needed", (long long)dst_words,
                (long long)(res->count * res->W));
  if (res->count) memcpy(dst, res->keys.data(), res->keys.size() * 8);
  return EFM_OK;
}

efm_status efm_result_fluxes(const efm_result *res, int64_t *dst, int64_t dst_len) {
  if (!res || (!dst && res->count > 0)) return fail(EFM_EINVAL, "null pointer");
  if (dst_len < res->count * res->n)
    return fail(EFM_EINVAL, "buffer of %lld entries, %lld needed", (long long)dst_len,
                (long long)(res->count * res->n));
  if (res->count) memcpy(dst, res->flux.data(), res->flux.size() * 8);
  return EFM_OK;
}

efm_status efm_result_destroy(efm_result *res) {
  delete res;
  return EFM_OK;
}

}  // extern "C"

// efm_internal.h -- shared declarations of the gfx950 library (host and device).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace efm {

typedef unsigned long long u64;
typedef __int128 i128;

// Modulus of the fast rank test: the Mersenne prime 2^31 - 1.  A "dependent"
// verdict is always confirmed in exact integer arithmetic, and "independent"
// modulo a prime implies independent over the rationals, so the prime only
// decides which children take the exact path.
constexpr uint32_t kPrime = 2147483647u;
constexpr int kMaxDepth = 64;      // support sizes handled (a wave holds one column per lane)
constexpr int kPruneMax = 8192;    // found pathways scanned by the minimality prune
// Longest probe sequence of a table insert.  Tables are kept at most half full,
// where linear probing essentially never runs this long; a longer run is
// reported as a full table instead of scanning it.
constexpr unsigned long long kMaxProbe = 4096;

// Counter slots (u64) in device memory, reset per level except kFound.
enum Counter {
  kSurv = 0,       // survivors (refs) appended this level
  kRankQ,          // row-closed children queued for the rank test
  kExactQ,         // children queued for the exact test
  kFound,          // pathways in the found list (all levels)
  kChildren,       // children generated
  kUnique,         // distinct children
  kPruned,         // row-closed children removed by the found-set prune
  kEmitted,        // pathways found this level
  kNext,           // members written to the next frontier
  kIndep,          // distinct children with independent columns
  kFlags,          // EFM_* flags and overflow bits below
  kBoundary,       // radix-select boundary list length
  kCapped,         // independent children dropped by the depth cap
  kParQ,           // parents queued with their row-closed children
  kRowClosed,      // distinct row-closed children
  kRankRows,       // sum over row-closed unpruned children of the rows their test spans
  kNumCounters
};
// Counters sit 256 bytes apart so that atomics on different counters never share
// a cache line.
constexpr int kCounterStride = 32;
__host__ __device__ inline size_t cslot(int c) { return (size_t)c * kCounterStride; }
// Copies of each selection histogram in device memory: the blocks of a pass add
// into different copies, so that skewed digits (one bin for nearly every key) do
// not put every block's atomic on one address; readers sum the copies.
constexpr int kHistCopies = 16;
constexpr int kMaxEnt = 16;        // column entries kept in registers by the rank test

enum FlagBits : u64 {
  kFlagDepthCapped = 1ull,
  kFlagUniqueOverflow = 1ull << 8,
  kFlagFoundOverflow = 1ull << 9,
  kFlagIntOverflow = 1ull << 10,
  kFlagQueueOverflow = 1ull << 11,
  kFlagFeatOverflow = 1ull << 12,
};

// Device tables of one network.  Masks are padded to the template widths
// Wt (reaction words) and MWt (internal-metabolite words).
struct DevNet {
  int n;            // reactions
  int mi;           // internal metabolites
  int Wt, MWt;      // padded widths
  const u64 *rxn_prodM;   // [n][MWt] internal metabolites an irreversible reaction produces
  const u64 *rxn_consM;   // [n][MWt] ... consumes
  const u64 *rxn_revM;    // [n][MWt] internal metabolites a reversible reaction touches
  const u64 *rxn_touchM;  // [n][MWt] all internal metabolites a reaction touches
  const u64 *met_fwdR;    // [mi][Wt] candidates when only irreversible producers touch i
  const u64 *met_bwdR;    // [mi][Wt] candidates when only irreversible consumers touch i
  const u64 *met_allR;    // [mi][Wt] every reaction touching i
  const u64 *rxn_nbrR;    // [n][Wt] reactions sharing an internal metabolite with r
  const u64 *rev_bits;    // [Wt]
  const int32_t *Sint;    // [mi][n] dense internal rows
  const u64 *zob;         // [n] Zobrist keys
  const uint32_t *rxn_ent;  // [n][kMaxEnt] (internal metabolite << 16) | (coefficient & 0xFFFF)
  const int32_t *rxn_nnz;   // [n] entries, or -1 when they do not fit rxn_ent (use Sint)
  const u64 *rxn_oddM;      // [n][MWt] internal metabolites where the coefficient is odd
};

// Radix-selection state in device memory: the digit decisions are taken on the
// device, so all byte passes are queued without host round trips.
struct SelState {
  int64_t needed;     // members still to select
  int64_t nb;         // members not yet decided
  uint32_t done;
  uint32_t pad;
};

// Per-enumeration device state.
struct DevLevel {
  // frontier being expanded
  const u64 *keys;        // SoA [Wt][fcap]
  const u64 *hash;        // [fcap]
  int64_t nparents;
  int64_t fcap;
  int level;              // members of the frontier have `level` reactions
  int depth_cap;
  // children
  u64 *table;             // [tcap] open addressing, tagged entries
  u64 tmask;              // slots used by this level - 1 (a power of two minus one)
  int tag;                // 1..127, distinct for every expand launch since the last clear
  u64 *surv;              // [ucap] refs of independent children
  u64 *rankq;             // [ucap] refs of row-closed children left undecided per parent
  u64 *parq;              // [fcap] parents with distinct row-closed children
  u64 *parmask;           // [fcap][Wt] those children, as a reaction mask
  u64 *exactq;            // [ucap] refs needing exact arithmetic
  int64_t ucap;
  // next frontier
  u64 *nkeys;             // SoA [Wt][fcap]
  u64 *nhash;
  // found pathways
  u64 *fkeys;             // SoA [Wt][ecap]
  int64_t *fflux;         // [ecap][kMaxDepth], value of the j-th reaction of the key
  int64_t ecap;
  int64_t nfound_prev;    // found pathways from earlier levels (prune scope)
  // target row
  const int32_t *Sx;      // [n]
  // truncation
  uint8_t *sel;           // [ucap] 0 rejected, 1 selected, 2 undecided
  uint8_t *skey;          // [8][sel_stride(ucap)] byte planes of the key word the current selection byte lies in
  uint32_t *hist;         // [3][kHistCopies][256], by pass % 3; block b adds to copy b % kHistCopies
  SelState *selst;        // [2], by pass parity
  const uint32_t *sscore; // [ucap] learned ordering: score word ranked before the key, or null
  u64 *counters;
  i128 *xscratch;         // exact kernel scratch: [xwaves][mi * kMaxDepth]
  int xwaves;
  const u64 *root_cand;   // level 0: candidate reactions of the empty pathway
  int debug_prime;         // every rank test goes to exact arithmetic
  int no_gf2;              // skip the modulo-2 certificate
};

// Row stride of the selection's byte planes: the survivor capacity rounded up to
// 256 bytes, so that every plane is aligned for 32-bit loads of four members.
__host__ __device__ inline int64_t sel_stride(int64_t ucap) { return (ucap + 255) & ~(int64_t)255; }

// kernel launchers (efm_kernels.hip)
hipError_t launch_expand(const DevNet &net, const DevLevel &L, hipStream_t s);
hipError_t launch_rank(const DevNet &net, const DevLevel &L, int prune, hipStream_t s);
hipError_t launch_rank_parent(const DevNet &net, const DevLevel &L, int prune, hipStream_t s);
hipError_t launch_exact(const DevNet &net, const DevLevel &L, hipStream_t s);
hipError_t launch_materialize(const DevNet &net, const DevLevel &L, int use_sel, hipStream_t s);
hipError_t launch_select_hist(const DevNet &net, const DevLevel &L, int byte, int refill, int pass,
                              hipStream_t s);
hipError_t launch_select_split(const DevNet &net, const DevLevel &L, int byte, int pass, hipStream_t s);
// pass-1's split and pass's histogram in one sweep (pass >= 1)
hipError_t launch_select_step(const DevNet &net, const DevLevel &L, int prev_byte, int byte, int refill, int pass,
                              hipStream_t s);
hipError_t launch_clear(u64 *p, size_t n, hipStream_t s);

}  // namespace efm

// efm_batch.hip -- many independent networks, each with one target, traversed in
// one persistent launch.
//
// Each workgroup pops a network from a device work queue (an atomic position in
// a largest-first order) and runs that network's whole level loop itself: the
// same steps as the single-network kernels (expansion with a level-tagged hash
// table, the rank test, exact arithmetic, canonical truncation, the next
// frontier), with workgroup barriers between them and counters in LDS.  The
// network's state lives in the workgroup's slice of one arena.  Device
// timestamps bracket every network.  The launch (queue reset + persistent
// kernel) is captured once in a HIP graph and replayed; the tile shape (waves
// per network, resident networks per CU) is chosen by timing candidates.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "efm_host.h"
#include "efm_wave.h"

namespace efm {

struct BatchNet {
  DevNet net;
  const int32_t *Sx;   // [n] the target row of S
  const u64 *root;     // [Wt] reactions that can produce the target
};

struct BatchRec {
  int64_t off, cnt;    // range of this network's pathways in the output
  int64_t parents;     // frontier members expanded
  int64_t children;    // children generated
  uint32_t status;     // EFM_DEPTH_CAPPED | EFM_FRONTIER_TRUNCATED
  uint32_t err;        // kFlag* overflow bits
  u64 t0, t1;          // device wall clock at start and end
};

struct SliceLayout {
  size_t ka, ha, kb, hb, table, surv, rcq, exq, sel, fkeys, fflux, xs, total;
};

__host__ __device__ inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

__host__ __device__ inline SliceLayout slice_layout(int W, int64_t fcap, int64_t ucap, int64_t tcap, int64_t ecap,
                                                    int dstride, int mi_max, int waves) {
  SliceLayout s{};
  size_t off = 0;
  auto take = [&](size_t b) { size_t o = off; off += al256(b); return o; };
  s.ka = take((size_t)W * fcap * 8);
  s.ha = take((size_t)fcap * 8);
  s.kb = take((size_t)W * fcap * 8);
  s.hb = take((size_t)fcap * 8);
  s.table = take((size_t)tcap * 8);
  s.surv = take((size_t)ucap * 8);
  s.rcq = take((size_t)ucap * 8);
  s.exq = take((size_t)ucap * 8);
  s.sel = take((size_t)ucap);
  s.fkeys = take((size_t)W * ecap * 8);
  s.fflux = take((size_t)ecap * dstride * 8);
  s.xs = take((size_t)waves * (mi_max > 0 ? mi_max : 1) * 64 * sizeof(i128));
  s.total = off;
  return s;
}

struct BatchArgs {
  const BatchNet *nets;
  const int32_t *order;
  int count;
  int depth_cap;
  int64_t fcap;        // frontier buffer (the cap, or ucap without one)
  int64_t trunc;       // frontier cap (0 = none)
  int64_t ucap;        // distinct children per level
  int64_t tcap;        // table slots (power of two)
  int64_t ecap;        // pathways per network
  int prune, no_gf2, exact_only;
  char *arena;
  size_t slice_bytes;
  int mi_max;
  int lds_rows;        // basis rows per wave in LDS: min(depth cap, largest internal-row count)
  u64 *queue;
  u64 *out_keys;       // [out_cap][W]
  int64_t *out_flux;   // [out_cap][dstride]
  int dstride;
  u64 *out_count;
  int64_t out_cap;
  BatchRec *rec;
};

enum { kCS = 0, kCR, kCX, kCF, kCN, kNumLds };

// child P|e_r into a workgroup-private table (same entry format and protocol as
// the single-network table)
template <int W>
DEVI bool slice_insert(u64 *table, u64 tmask, u64 tag, u64 h, u64 p, int r, const u64 *P, const u64 *keys,
                       int64_t fcap, uint32_t *err) {
  const u64 entry = (tag << 57) | (((h >> 50) & 0x3FFFull) << 43) | ((p & 0xFFFFFFFFull) << 11) | (u64)r;
  const u64 fp = (h >> 50) & 0x3FFFull;
  u64 pos = h & tmask;
  const u64 max_probe = tmask < kMaxProbe ? tmask + 1 : kMaxProbe;
  for (u64 probe = 0; probe < max_probe; ++probe) {
    if (*(volatile uint32_t *)err) return false;     // the level already failed
    u64 cur = __hip_atomic_load(&table[pos], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    while ((cur >> 57) != tag) {
      const u64 prev = atomicCAS(&table[pos], cur, entry);
      if (prev == cur) return true;
      cur = prev;
    }
    if (((cur >> 43) & 0x3FFFull) == fp) {
      const u64 p2 = (cur >> 11) & 0xFFFFFFFFull;
      const int r2 = (int)(cur & 0x7FFull);
      bool eq = true;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const u64 a = P[w] | ((r >> 6) == w ? (1ull << (r & 63)) : 0ull);
        const u64 b = keys[(int64_t)w * fcap + p2] | ((r2 >> 6) == w ? (1ull << (r2 & 63)) : 0ull);
        eq = eq && (a == b);
      }
      if (eq) return false;
    }
    pos = (pos + 1) & tmask;
  }
  atomicOr(err, (uint32_t)kFlagUniqueOverflow);
  return false;
}

DEVI void lds_push(int *cnt, u64 *list, int64_t cap, u64 val, uint32_t *err) {
  const int idx = atomicAdd(cnt, 1);
  if (idx < cap) list[idx] = val;
  else atomicOr(err, (uint32_t)kFlagQueueOverflow);
}

template <int W, int MW>
__global__ __launch_bounds__(512) void batch_kernel(BatchArgs A) {
  extern __shared__ uint32_t Bdyn[];    // per wave: depth_cap rows of 64 basis entries
  __shared__ int s_ni;
  __shared__ int s_cnt[kNumLds];
  __shared__ uint32_t s_err, s_status;
  __shared__ unsigned long long s_children;
  __shared__ uint32_t s_hist[256];
  __shared__ int s_digit, s_allsel, s_skip;
  __shared__ int64_t s_needed;

  const int tid = threadIdx.x, bs = blockDim.x, lane = lane_id();
  const int wave = tid >> 6, nwaves = bs >> 6;
  char *base = A.arena + (size_t)blockIdx.x * A.slice_bytes;
  const SliceLayout lay = slice_layout(W, A.fcap, A.ucap, A.tcap, A.ecap, A.dstride, A.mi_max, nwaves);
  u64 *ka = (u64 *)(base + lay.ka), *ha = (u64 *)(base + lay.ha);
  u64 *kb = (u64 *)(base + lay.kb), *hb = (u64 *)(base + lay.hb);
  u64 *table = (u64 *)(base + lay.table);
  u64 *surv = (u64 *)(base + lay.surv), *rcq = (u64 *)(base + lay.rcq), *exq = (u64 *)(base + lay.exq);
  uint8_t *sel = (uint8_t *)(base + lay.sel);
  u64 *fkeys = (u64 *)(base + lay.fkeys);
  int64_t *fflux = (int64_t *)(base + lay.fflux);
  i128 *M = (i128 *)(base + lay.xs) + (size_t)wave * (A.mi_max > 0 ? A.mi_max : 1) * 64;
  const u64 tmask = (u64)A.tcap - 1;

  for (;;) {
    if (tid == 0) {
      const u64 pos = atomicAdd(A.queue, 1ull);
      s_ni = pos < (u64)A.count ? A.order[pos] : -1;
    }
    __syncthreads();
    const int ni = s_ni;
    if (ni < 0) break;
    const u64 t0 = wall_clock64();
    const BatchNet &B = A.nets[ni];
    const DevNet &net = B.net;

    for (int64_t i = tid; i < A.tcap; i += bs) table[i] = 0;
    if (tid < W) ka[(int64_t)tid * A.fcap] = 0;
    if (tid == 0) {
      ha[0] = 0;
      s_err = 0;
      s_status = 0;
      s_children = 0;
      s_cnt[kCF] = 0;
    }
    __syncthreads();
    int64_t nparents = 1, parents_total = 0;

    for (int level = 0; level < A.depth_cap && nparents > 0; ++level) {
      if (tid == 0) {
        s_cnt[kCS] = 0;
        s_cnt[kCR] = 0;
        s_cnt[kCX] = 0;
        s_cnt[kCN] = 0;
      }
      __syncthreads();
      const bool keep = level + 1 < A.depth_cap;
      const u64 tag = (u64)level + 1;
      const int nf_prev = min(s_cnt[kCF], (int)A.ecap);
      parents_total += nparents;

      // ---- expand: one thread per parent
      u64 my_children = 0;
      for (int64_t p = tid; p < nparents; p += bs) {
        if (*(volatile uint32_t *)&s_err) break;        // a capacity overflowed: stop early
        u64 P[W], cand[W], T[MW];
#pragma unroll
        for (int w = 0; w < W; ++w) { P[w] = ka[(int64_t)w * A.fcap + p]; cand[w] = 0; }
#pragma unroll
        for (int q = 0; q < MW; ++q) T[q] = 0;
        const u64 h = ha[p];
        if (level == 0) {
#pragma unroll
          for (int w = 0; w < W; ++w) cand[w] = B.root[w] & ~P[w];
        } else {
          u64 Am[MW], Bm[MW], C[MW], C2[MW];
#pragma unroll
          for (int q = 0; q < MW; ++q) { Am[q] = 0; Bm[q] = 0; C[q] = 0; C2[q] = 0; }
#pragma unroll
          for (int w = 0; w < W; ++w) {
            u64 bits = P[w];
            while (bits) {
              const int r = w * 64 + __builtin_ctzll(bits);
              bits &= bits - 1;
#pragma unroll
              for (int q = 0; q < MW; ++q) {
                const u64 rq = net.rxn_revM[(int64_t)r * MW + q];
                Am[q] |= net.rxn_prodM[(int64_t)r * MW + q];
                Bm[q] |= net.rxn_consM[(int64_t)r * MW + q];
                C2[q] |= C[q] & rq;
                C[q] |= rq;
              }
            }
          }
          int istar = -1;
          u64 Aq = 0, Bq = 0;
#pragma unroll
          for (int q = 0; q < MW; ++q) {
            T[q] = Am[q] | Bm[q] | C[q];
            const u64 U = T[q] & ~((Am[q] & Bm[q]) | (C[q] & (Am[q] | Bm[q])) | C2[q]);
            if (istar < 0 && U) { istar = q * 64 + __builtin_ctzll(U); Aq = Am[q]; Bq = Bm[q]; }
          }
          if (istar >= 0) {
            const u64 bit = 1ull << (istar & 63);
            const u64 *src = (Aq & bit) ? net.met_fwdR : ((Bq & bit) ? net.met_bwdR : net.met_allR);
#pragma unroll
            for (int w = 0; w < W; ++w) cand[w] = src[(int64_t)istar * W + w] & ~P[w];
          } else {
#pragma unroll
            for (int w = 0; w < W; ++w) {
              u64 bits = P[w];
              while (bits) {
                const int r = w * 64 + __builtin_ctzll(bits);
                bits &= bits - 1;
#pragma unroll
                for (int ww = 0; ww < W; ++ww) cand[ww] |= net.rxn_nbrR[(int64_t)r * W + ww];
              }
            }
#pragma unroll
            for (int w = 0; w < W; ++w) cand[w] &= ~P[w];
          }
        }
#pragma unroll
        for (int w = 0; w < W; ++w) {
          u64 bits = cand[w];
          while (bits) {
            const int r = w * 64 + __builtin_ctzll(bits);
            bits &= bits - 1;
            my_children++;
            u64 outside = 0;
#pragma unroll
            for (int q = 0; q < MW; ++q) outside |= net.rxn_touchM[(int64_t)r * MW + q] & ~T[q];
            const bool rc = outside == 0;
            if (!slice_insert<W>(table, tmask, tag, h ^ net.zob[r], (u64)p, r, P, ka, A.fcap, &s_err)) continue;
            const u64 ref = ((u64)p << 12) | ((u64)r << 1) | (rc ? 1ull : 0ull);
            if (rc) lds_push(&s_cnt[kCR], rcq, A.ucap, ref, &s_err);
            else if (keep) lds_push(&s_cnt[kCS], surv, A.ucap, ref, &s_err);
            else atomicOr(&s_status, (uint32_t)EFM_DEPTH_CAPPED);
          }
        }
      }
      if (my_children) atomicAdd(&s_children, (unsigned long long)my_children);
      __syncthreads();

      // ---- rank: one wave per row-closed child
      const int nrc = min(s_cnt[kCR], (int)A.ucap);
      for (int i = wave; i < nrc; i += nwaves) {
        const u64 ref = rcq[i];
        const u64 p = ref >> 12;
        const int r = (int)((ref >> 1) & 0x7FF);
        u64 Q[W];
#pragma unroll
        for (int w = 0; w < W; ++w) Q[w] = ka[(int64_t)w * A.fcap + p] | ((r >> 6) == w ? (1ull << (r & 63)) : 0ull);
        if (A.prune && nf_prev > 0) {
          bool hit = false;
          for (int f0 = 0; f0 < nf_prev && !hit; f0 += 64) {
            const int f = f0 + lane;
            bool sub = f < nf_prev;
            if (sub) {
#pragma unroll
              for (int w = 0; w < W; ++w) sub = sub && ((fkeys[(int64_t)w * A.ecap + f] & ~Q[w]) == 0);
            }
            hit = __ballot(sub) != 0;
          }
          if (hit) continue;
        }
        const bool indep = A.exact_only ? false : wave_rank_child<W, MW>(net, Q, r, A.no_gf2 != 0);
        if (lane == 0) {
          if (!indep) lds_push(&s_cnt[kCX], exq, A.ucap, ref, &s_err);
          else if (keep) lds_push(&s_cnt[kCS], surv, A.ucap, ref, &s_err);
          else atomicOr(&s_status, (uint32_t)EFM_DEPTH_CAPPED);
        }
      }
      __syncthreads();

      // ---- exact arithmetic: one wave per child
      const int nex = min(s_cnt[kCX], (int)A.ucap);
      for (int i = wave; i < nex; i += nwaves) {
        const u64 ref = exq[i];
        const u64 p = ref >> 12;
        const int r = (int)((ref >> 1) & 0x7FF);
        u64 Q[W];
        int kq = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
          Q[w] = ka[(int64_t)w * A.fcap + p] | ((r >> 6) == w ? (1ull << (r & 63)) : 0ull);
          kq += __popcll(Q[w]);
        }
        int64_t vout = 0;
        const int outcome = wave_exact_child<W, MW>(net, Q, B.Sx, M, Bdyn + (size_t)wave * A.lds_rows * 64, vout,
                                                    A.exact_only != 0);
        if (outcome == kExactOverflow) {
          if (lane == 0) atomicOr(&s_err, (uint32_t)kFlagIntOverflow);
        } else if (outcome == kExactIndependent) {
          if (lane == 0) {
            if (keep) lds_push(&s_cnt[kCS], surv, A.ucap, ref, &s_err);
            else atomicOr(&s_status, (uint32_t)EFM_DEPTH_CAPPED);
          }
        } else if (outcome == kExactEmit) {
          int slot = 0;
          if (lane == 0) slot = atomicAdd(&s_cnt[kCF], 1);
          slot = __shfl(slot, 0);
          if (slot < A.ecap) {
#pragma unroll
            for (int w = 0; w < W; ++w)
              if (lane == w) fkeys[(int64_t)w * A.ecap + slot] = Q[w];
            if (lane < kq) fflux[(int64_t)slot * A.dstride + lane] = vout;
          } else if (lane == 0) {
            atomicOr(&s_err, (uint32_t)kFlagFoundOverflow);
          }
        }
      }
      __syncthreads();
      if (s_err) break;

      // ---- canonical truncation: radix selection, one key byte per pass
      const int64_t ns = min((int64_t)s_cnt[kCS], A.ucap);
      const bool trunc = A.trunc > 0 && ns > A.trunc;
      if (trunc) {
        for (int64_t i = tid; i < ns; i += bs) sel[i] = 2;
        if (tid == 0) {
          s_needed = A.trunc;
          s_status |= EFM_FRONTIER_TRUNCATED;
        }
        for (int byte = (net.n - 1) / 8; byte >= 0; --byte) {
          for (int i = tid; i < 256; i += bs) s_hist[i] = 0;
          __syncthreads();
          const int w = byte >> 3, shift = (byte & 7) * 8;
          for (int64_t i = tid; i < ns; i += bs) {
            if (sel[i] != 2) continue;
            const u64 ref = surv[i];
            const u64 p = ref >> 12;
            const int r = (int)((ref >> 1) & 0x7FF);
            const u64 kw = ka[(int64_t)w * A.fcap + p] | ((r >> 6) == w ? (1ull << (r & 63)) : 0ull);
            atomicAdd(&s_hist[(kw >> shift) & 0xFF], 1u);
          }
          __syncthreads();
          if (tid == 0) {
            int64_t cum = 0, und = 0;
            for (int v = 0; v < 256; ++v) und += s_hist[v];
            int v = 0;
            for (v = 0; v < 255; ++v) {
              if (cum + (int64_t)s_hist[v] >= s_needed) break;
              cum += s_hist[v];
            }
            const int64_t hv = s_hist[v];
            s_digit = v;
            s_allsel = hv == s_needed - cum;
            s_skip = !s_allsel && hv == und;
            if (!s_skip && !s_allsel) s_needed -= cum;
          }
          __syncthreads();
          if (!s_skip) {
            const int digit = s_digit, allsel = s_allsel;
            for (int64_t i = tid; i < ns; i += bs) {
              if (sel[i] != 2) continue;
              const u64 ref = surv[i];
              const u64 p = ref >> 12;
              const int r = (int)((ref >> 1) & 0x7FF);
              const u64 kw = ka[(int64_t)w * A.fcap + p] | ((r >> 6) == w ? (1ull << (r & 63)) : 0ull);
              const int d = (int)((kw >> shift) & 0xFF);
              if (d < digit || (d == digit && allsel)) sel[i] = 1;
              else if (d > digit) sel[i] = 0;
            }
          }
          __syncthreads();
          if (s_allsel && !s_skip) break;
        }
      }

      // ---- the next frontier
      for (int64_t i = tid; i < ns; i += bs) {
        if (trunc && sel[i] != 1) continue;
        const u64 ref = surv[i];
        const u64 p = ref >> 12;
        const int r = (int)((ref >> 1) & 0x7FF);
        const int dst = atomicAdd(&s_cnt[kCN], 1);
#pragma unroll
        for (int w = 0; w < W; ++w)
          kb[(int64_t)w * A.fcap + dst] = ka[(int64_t)w * A.fcap + p] | ((r >> 6) == w ? (1ull << (r & 63)) : 0ull);
        hb[dst] = ha[p] ^ net.zob[r];
      }
      __syncthreads();
      nparents = s_cnt[kCN];
      __syncthreads();                  // every thread has read it before the next reset
      u64 *t = ka; ka = kb; kb = t;
      t = ha; ha = hb; hb = t;
    }

    // ---- results of this network
    __shared__ int64_t s_off;
    const int nfound = min(s_cnt[kCF], (int)A.ecap);
    if (tid == 0) {
      int64_t off = (int64_t)atomicAdd(A.out_count, (u64)nfound);
      uint32_t err = s_err;
      if (off + nfound > A.out_cap) { err |= kFlagFoundOverflow; off = -1; }
      s_off = off;
      BatchRec &R = A.rec[ni];
      R.off = off;
      R.cnt = off >= 0 ? nfound : 0;
      R.parents = parents_total;
      R.children = (int64_t)s_children;
      R.status = s_status;
      R.err = err;
      R.t0 = t0;
    }
    __syncthreads();
    if (s_off >= 0) {
      for (int i = tid; i < nfound; i += bs) {
#pragma unroll
        for (int w = 0; w < W; ++w) A.out_keys[(s_off + i) * W + w] = fkeys[(int64_t)w * A.ecap + i];
        for (int j = 0; j < A.dstride; ++j) A.out_flux[(s_off + i) * A.dstride + j] = fflux[(int64_t)i * A.dstride + j];
      }
    }
    __syncthreads();
    if (tid == 0) A.rec[ni].t1 = wall_clock64();
  }
}

__global__ void batch_reset_kernel(u64 *queue, u64 *out_count) {
  if (threadIdx.x == 0) {
    *queue = 0;
    *out_count = 0;
  }
}

template <int W, int MW>
static void do_batch(const BatchArgs &A, int grid, int block, hipStream_t s) {
  const size_t lds = (size_t)(block / 64) * A.lds_rows * 64 * sizeof(uint32_t);
  hipLaunchKernelGGL((batch_kernel<W, MW>), dim3(grid), dim3(block), lds, s, A);
}

static hipError_t launch_batch(int Wt, int MWt, const BatchArgs &A, int grid, int block, hipStream_t s) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, s, A.queue, A.out_count);
  switch (Wt * 100 + MWt) {
    case 101: do_batch<1, 1>(A, grid, block, s); break;
    case 102: do_batch<1, 2>(A, grid, block, s); break;
    case 201: do_batch<2, 1>(A, grid, block, s); break;
    case 202: do_batch<2, 2>(A, grid, block, s); break;
    case 401: do_batch<4, 1>(A, grid, block, s); break;
    case 402: do_batch<4, 2>(A, grid, block, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace efm

using efm::u64;

struct efm_batch {
  int count = 0, Wt = 0, MWt = 0, depth_cap = 0, dstride = 0;
  int nsample = 0;                       // autotuner sample (every 4th network of the order)
  const int32_t *sample_order = nullptr;
  std::vector<int> n_of, W_of;
  efm_batch_config cfg{};
  efm::BatchArgs args{};
  void *blob = nullptr;       // tables, descriptors, order
  void *arena = nullptr;      // per-workgroup slices (sized for the largest tile shape)
  void *io = nullptr;         // queue, output, records
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  double ns_per_tick = 10.0;
  // host mirror of the last run
  std::vector<efm::BatchRec> rec;
  std::vector<u64> out_keys;
  std::vector<int64_t> out_flux;
  bool have_results = false;
};

namespace {

#define BCHK(expr)                                                                        \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) {                                                               \
      rc = fail(EFM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));              \
      goto bad;                                                                           \
    }                                                                                     \
  } while (0)

int64_t next_pow2_b(int64_t x) {
  int64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

// largest waves-per-network whose LDS basis rows fit in 48 KB
int max_waves(const efm_batch *b) {
  int w = 8;
  while (w > 1 && (size_t)w * b->args.lds_rows * 64 * 4 > 48 * 1024) w >>= 1;
  return w;
}

efm_status capture(efm_batch *b) {
  efm_status rc = EFM_OK;
  b->cfg.waves_per_network = std::min(b->cfg.waves_per_network, max_waves(b));
  if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  const int block = 64 * b->cfg.waves_per_network;
  int dev = 0, cus = 256;
  BCHK(hipGetDevice(&dev));
  BCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  {
    const int grid = std::min(b->count, cus * b->cfg.networks_per_cu);
    efm::BatchArgs A = b->args;
    A.slice_bytes = efm::slice_layout(b->Wt, A.fcap, A.ucap, A.tcap, A.ecap, A.dstride, A.mi_max, b->cfg.waves_per_network).total;
    b->args = A;
    BCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    hipError_t le = efm::launch_batch(b->Wt, b->MWt, A, grid, block, b->stream);
    hipGraph_t g = nullptr;
    hipError_t ce = hipStreamEndCapture(b->stream, &g);
    if (le != hipSuccess || ce != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(EFM_EDEVICE, "graph capture failed: %s", hipGetErrorString(le != hipSuccess ? le : ce));
    }
    b->graph = g;
    BCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  }
  return EFM_OK;
bad:
  return rc;
}

efm_status run_once(efm_batch *b, hipStream_t s, float *ms) {
  efm_status rc = EFM_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  BCHK(hipEventCreate(&e0));
  BCHK(hipEventCreate(&e1));
  BCHK(hipEventRecord(e0, s));
  BCHK(hipGraphLaunch(b->exec, s));
  BCHK(hipEventRecord(e1, s));
  BCHK(hipEventSynchronize(e1));
  if (ms) BCHK(hipEventElapsedTime(ms, e0, e1));
bad:
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return rc;
}

}  // namespace

extern "C" {

efm_status efm_batch_create(const efm_network *const *nets, const int32_t *targets, int32_t count,
                            const efm_enum_opts *opts, efm_batch **out) {
  if (!nets || !targets || !out || count <= 0) return fail(EFM_EINVAL, "null pointer or empty batch");
  efm_enum_opts o{};
  if (opts) o = *opts;
  efm_status rc = EFM_OK;
  efm_batch *b = new (std::nothrow) efm_batch;
  if (!b) return fail(EFM_ENOMEM, "host allocation failed");
  b->count = count;
  int maxW = 1, maxMW = 1, mi_max = 1;
  for (int i = 0; i < count; ++i) {
    const efm_network *N = nets[i];
    if (!N) { delete b; return fail(EFM_EINVAL, "network %d is null", i); }
    const int t = targets[i];
    if (t < 0 || t >= N->m || !N->ext[t]) { delete b; return fail(EFM_EINVAL, "network %d: target %d is not external", i, t); }
    bool any = false;
    for (int r = 0; r < N->n; ++r) {
      const int32_t s = N->S[(size_t)t * N->n + r];
      any = any || s > 0 || (s < 0 && N->rev[r]);
    }
    if (!any) { delete b; return fail(EFM_EINVAL, "network %d: no reaction can produce target %d", i, t); }
    maxW = std::max(maxW, N->W);
    maxMW = std::max(maxMW, (N->mi + 63) / 64);
    mi_max = std::max(mi_max, N->mi);
    b->n_of.push_back(N->n);
    b->W_of.push_back(N->W);
  }
  if (!choose_shape(maxW, maxMW, &b->Wt, &b->MWt) || b->Wt > 4 || b->MWt > 2) {
    delete b;
    return fail(EFM_EINVAL, "batched networks must have at most 256 reactions and 128 internal metabolites");
  }
  const int Wt = b->Wt, MWt = b->MWt;
  int D = o.depth_cap > 0 ? std::min(o.depth_cap, EFM_MAX_DEPTH) : EFM_MAX_DEPTH;
  b->depth_cap = D;
  b->dstride = D;

  // tables of every network at the common widths, target rows, root masks, order
  {
    std::vector<char> host;
    std::vector<std::vector<size_t>> offs(count);
    std::vector<size_t> base(count), sx_off(count), root_off(count);
    for (int i = 0; i < count; ++i) {
      std::vector<char> h;
      build_tables(nets[i], Wt, MWt, h, offs[i]);
      base[i] = host.size();
      host.insert(host.end(), h.begin(), h.end());
      const efm_network *N = nets[i];
      sx_off[i] = host.size();
      std::vector<int32_t> sx(N->n);
      for (int r = 0; r < N->n; ++r) sx[r] = N->S[(size_t)targets[i] * N->n + r];
      host.resize(host.size() + align256(sx.size() * 4));
      memcpy(host.data() + sx_off[i], sx.data(), sx.size() * 4);
      root_off[i] = host.size();
      std::vector<u64> root(Wt, 0);
      for (int r = 0; r < N->n; ++r) {
        const int32_t s = sx[r];
        if (s > 0 || (s < 0 && N->rev[r])) root[r >> 6] |= 1ull << (r & 63);
      }
      host.resize(host.size() + align256(Wt * 8));
      memcpy(host.data() + root_off[i], root.data(), Wt * 8);
    }
    const size_t desc_off = host.size();
    host.resize(host.size() + align256(sizeof(efm::BatchNet) * count));
    const size_t order_off = host.size();
    host.resize(host.size() + align256(sizeof(int32_t) * count));
    const size_t sample_off = host.size();   // every 4th network of the order: the autotuner's sample
    host.resize(host.size() + align256(sizeof(int32_t) * count));
    BCHK(hipMalloc(&b->blob, host.size()));
    char *dbase = (char *)b->blob;
    std::vector<efm::BatchNet> desc(count);
    for (int i = 0; i < count; ++i) {
      desc[i].net = bind_tables(nets[i], Wt, MWt, dbase + base[i], offs[i]);
      desc[i].Sx = (const int32_t *)(dbase + sx_off[i]);
      desc[i].root = (const u64 *)(dbase + root_off[i]);
    }
    memcpy(host.data() + desc_off, desc.data(), sizeof(efm::BatchNet) * count);
    // largest networks first: a longest-processing-time order for the queue
    std::vector<int32_t> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
      return (int64_t)nets[a]->n * nets[a]->mi > (int64_t)nets[c]->n * nets[c]->mi;
    });
    memcpy(host.data() + order_off, order.data(), sizeof(int32_t) * count);
    std::vector<int32_t> sample;
    for (int i = 0; i < count; i += (count >= 256 ? 4 : 1)) sample.push_back(order[i]);
    memcpy(host.data() + sample_off, sample.data(), sizeof(int32_t) * sample.size());
    b->nsample = (int)sample.size();
    BCHK(hipMemcpy(b->blob, host.data(), host.size(), hipMemcpyHostToDevice));
    b->args.nets = (const efm::BatchNet *)(dbase + desc_off);
    b->args.order = (const int32_t *)(dbase + order_off);
    b->sample_order = (const int32_t *)(dbase + sample_off);
  }

  {
    efm::BatchArgs &A = b->args;
    A.count = count;
    A.depth_cap = D;
    A.ucap = o.unique_cap > 0 ? o.unique_cap : (1 << 18);
    A.trunc = o.frontier_cap > 0 ? o.frontier_cap : 0;
    A.fcap = A.trunc > 0 ? std::min<int64_t>(A.trunc, A.ucap) : A.ucap;
    A.tcap = std::max<int64_t>(1024, next_pow2_b(2 * A.ucap));
    A.ecap = o.found_cap > 0 ? o.found_cap : 4096;
    A.prune = (o.flags & EFM_OPT_NO_PRUNE) ? 0 : 1;
    A.no_gf2 = (o.flags & EFM_OPT_NO_GF2) ? 1 : 0;
    A.exact_only = (o.flags & EFM_OPT_EXACT_RANK) ? 1 : 0;
    A.mi_max = mi_max;
    A.lds_rows = std::max(1, std::min(D, mi_max));
    A.dstride = b->dstride;
    A.out_cap = std::max<int64_t>(1 << 16, std::min<int64_t>((int64_t)count * A.ecap, (int64_t)1 << 22));
    // arena for the largest tile shape tried: 8 waves, 8 networks per CU
    int dev = 0, cus = 256;
    BCHK(hipGetDevice(&dev));
    BCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int khz = 100000;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) khz = 100000;
    b->ns_per_tick = 1e6 / (double)khz;
    const size_t slice_max = efm::slice_layout(Wt, A.fcap, A.ucap, A.tcap, A.ecap, A.dstride, mi_max, 8).total;
    const int grid_max = std::min(count, cus * 8);
    BCHK(hipMalloc(&b->arena, slice_max * grid_max));
    A.arena = (char *)b->arena;
    const size_t io_bytes = 256 + 256 + align256((size_t)A.out_cap * Wt * 8) +
                            align256((size_t)A.out_cap * A.dstride * 8) + align256(sizeof(efm::BatchRec) * count);
    BCHK(hipMalloc(&b->io, io_bytes));
    char *io = (char *)b->io;
    A.queue = (u64 *)io;
    A.out_count = (u64 *)(io + 256);
    A.out_keys = (u64 *)(io + 512);
    A.out_flux = (int64_t *)(io + 512 + align256((size_t)A.out_cap * Wt * 8));
    A.rec = (efm::BatchRec *)(io + 512 + align256((size_t)A.out_cap * Wt * 8) +
                              align256((size_t)A.out_cap * A.dstride * 8));
  }
  BCHK(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));

  // tile shape: fixed default, or the fastest candidate on this batch
  b->cfg.waves_per_network = 4;
  b->cfg.networks_per_cu = 4;
  if (o.flags & EFM_OPT_AUTOTUNE) {
    // each candidate tile is timed once on a sample of the batch (every 4th
    // network of the largest-first order, so the size mix is kept), after one
    // warm-up launch
    const int cand[][2] = {{1, 8}, {2, 8}, {2, 4}, {4, 4}, {4, 2}, {8, 2}};
    const efm::BatchArgs full = b->args;
    const int full_count = b->count;
    b->args.order = b->sample_order;
    b->args.count = b->nsample;
    b->count = b->nsample;
    float best = 1e30f;
    efm_batch_config best_cfg = b->cfg;
    bool warm = false;
    for (auto &c : cand) {
      if (c[0] > max_waves(b)) continue;
      b->cfg.waves_per_network = c[0];
      b->cfg.networks_per_cu = c[1];
      if ((rc = capture(b)) != EFM_OK) goto bad;
      float ms = 0.f;
      if (!warm && (rc = run_once(b, b->stream, nullptr)) != EFM_OK) goto bad;
      warm = true;
      if ((rc = run_once(b, b->stream, &ms)) != EFM_OK) goto bad;
      if (ms < best) { best = ms; best_cfg = b->cfg; }
    }
    b->args = full;
    b->count = full_count;
    b->cfg = best_cfg;
  }
  if ((rc = capture(b)) != EFM_OK) goto bad;
  *out = b;
  return EFM_OK;
bad:
  efm_batch_destroy(b);
  return rc;
}

efm_status efm_batch_run(efm_batch *b, void *stream) {
  if (!b) return fail(EFM_EINVAL, "null batch");
  efm_status rc = EFM_OK;
  hipStream_t s = stream ? (hipStream_t)stream : b->stream;
  if ((rc = run_once(b, s, nullptr)) != EFM_OK) return rc;
  b->rec.resize(b->count);
  u64 nout = 0;
  BCHK(hipMemcpy(b->rec.data(), b->args.rec, sizeof(efm::BatchRec) * b->count, hipMemcpyDeviceToHost));
  BCHK(hipMemcpy(&nout, b->args.out_count, 8, hipMemcpyDeviceToHost));
  nout = std::min<u64>(nout, (u64)b->args.out_cap);
  b->out_keys.resize((size_t)nout * b->Wt);
  b->out_flux.resize((size_t)nout * b->dstride);
  if (nout) {
    BCHK(hipMemcpy(b->out_keys.data(), b->args.out_keys, b->out_keys.size() * 8, hipMemcpyDeviceToHost));
    BCHK(hipMemcpy(b->out_flux.data(), b->args.out_flux, b->out_flux.size() * 8, hipMemcpyDeviceToHost));
  }
  b->have_results = true;
  // the next run pops the networks in decreasing order of this run's latency
  // (longest processing time first), so the slowest ones start earliest
  {
    std::vector<int32_t> order(b->count);
    for (int i = 0; i < b->count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      return b->rec[x].t1 - b->rec[x].t0 > b->rec[y].t1 - b->rec[y].t0;
    });
    BCHK(hipMemcpy((void *)b->args.order, order.data(), sizeof(int32_t) * b->count, hipMemcpyHostToDevice));
  }
  return EFM_OK;
bad:
  return rc;
}

efm_status efm_batch_config_get(const efm_batch *b, efm_batch_config *cfg) {
  if (!b || !cfg) return fail(EFM_EINVAL, "null pointer");
  *cfg = b->cfg;
  return EFM_OK;
}

efm_status efm_batch_result(const efm_batch *b, int32_t i, efm_result **out) {
  if (!b || !out) return fail(EFM_EINVAL, "null pointer");
  if (!b->have_results) return fail(EFM_EINVAL, "efm_batch_run has not completed");
  if (i < 0 || i >= b->count) return fail(EFM_EINVAL, "network index %d out of range", i);
  const efm::BatchRec &R = b->rec[i];
  if (R.err & (efm::kFlagUniqueOverflow | efm::kFlagQueueOverflow))
    return fail(EFM_ENOMEM, "network %d: more than unique_cap distinct children in a level", i);
  if (R.err & efm::kFlagFoundOverflow) return fail(EFM_ENOMEM, "network %d: more than found_cap pathways", i);
  if (R.err & efm::kFlagIntOverflow) return fail(EFM_EOVERFLOW, "network %d: exact arithmetic overflow", i);
  efm_result *res = new (std::nothrow) efm_result;
  if (!res) return fail(EFM_ENOMEM, "host allocation failed");
  res->W = b->W_of[i];
  res->n = b->n_of[i];
  res->status = R.status;
  efm_level_stats st{};
  st.parents = R.parents;
  st.children = R.children;
  st.emitted = R.cnt;
  res->levels.push_back(st);   // one summary entry for the whole traversal
  const int64_t cnt = R.cnt;
  std::vector<u64> fk((size_t)b->Wt * std::max<int64_t>(cnt, 1));
  for (int64_t k = 0; k < cnt; ++k)
    for (int w = 0; w < b->Wt; ++w) fk[(size_t)w * cnt + k] = b->out_keys[(size_t)(R.off + k) * b->Wt + w];
  const int64_t *ff = cnt ? b->out_flux.data() + (size_t)R.off * b->dstride : nullptr;
  assemble(res, b->Wt, fk.data(), cnt, ff, b->dstride);
  *out = res;
  return EFM_OK;
}

efm_status efm_batch_latency(const efm_batch *b, int64_t *ns) {
  if (!b || !ns) return fail(EFM_EINVAL, "null pointer");
  if (!b->have_results) return fail(EFM_EINVAL, "efm_batch_run has not completed");
  for (int i = 0; i < b->count; ++i)
    ns[i] = (int64_t)((double)(b->rec[i].t1 - b->rec[i].t0) * b->ns_per_tick);
  return EFM_OK;
}

efm_status efm_batch_destroy(efm_batch *b) {
  if (!b) return EFM_OK;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->stream) {
    (void)hipStreamSynchronize(b->stream);
    (void)hipStreamDestroy(b->stream);
  }
  if (b->arena) (void)hipFree(b->arena);
  if (b->io) (void)hipFree(b->io);
  if (b->blob) (void)hipFree(b->blob);
  delete b;
  return EFM_OK;
}

}  // extern "C"

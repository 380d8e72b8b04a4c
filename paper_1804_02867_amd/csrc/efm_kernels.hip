// efm_kernels.hip -- gfx950 kernels of one level of the exhaustive AND/OR traversal.
//
// One level turns the frontier F_k (independent reaction sets of k reactions) into
// the children of level k+1 (paper Section 4.1, Algorithm 3: every metabolite of
// a candidate pathway that is not balanced picks an output/input reaction; here
// every pick is taken):
//   expand       one lane per parent: role masks over the internal metabolites
//                (Definitions 9-10), the lowest unbalanced metabolite (wave-local
//                bit scan), its role-filtered reactions (or every neighbouring
//                reaction when the parent is closed), a Zobrist child hash, an
//                insert into a level-tagged open-addressing table (distinct
//                children), and the row-closure flag that decides whether the
//                child needs a rank test at all;
//   rank         one wave per row-closed child: the found-set minimality prune
//                (Definition 3) and a streaming Gaussian elimination modulo
//                2^31-1 with lanes over the child's columns;
//   exact        one wave per child the modular test called dependent:
//                fraction-free elimination in 128-bit integers, the exact rank,
//                the primitive null vector, the sign and target tests
//                (Definition 2) and the emission of the pathway;
//   select_*     radix selection of the frontier cap's smallest keys;
//   materialize  the next frontier's keys (SoA) and hashes.
#include "efm_internal.h"

namespace efm {

#define DEVI __device__ __forceinline__

// ------------------------------------------------------------------ wave helpers
DEVI int lane_id() { return __lane_id(); }

DEVI u64 lanes_below(int lane) { return lane == 0 ? 0ull : (~0ull >> (64 - lane)); }

// Append `val` to `list` for every lane with pred set; one atomic per wave.
// Must be called by all lanes of the wave (converged control flow).
DEVI void wave_append(bool pred, u64 *list, u64 *counter, u64 val, int64_t cap, u64 *flags) {
  u64 mask = __ballot(pred);
  if (mask == 0) return;
  int lane = lane_id();
  int leader = __ffsll((long long)mask) - 1;
  u64 base = 0;
  if (lane == leader) base = atomicAdd(counter, (u64)__popcll(mask));
  base = __shfl(base, leader);
  if (pred) {
    u64 idx = base + (u64)__popcll(mask & lanes_below(lane));
    if ((int64_t)idx < cap) list[idx] = val;
    else atomicOr(flags, (u64)kFlagQueueOverflow);
  }
}

DEVI void wave_count(bool pred, u64 *counter) {
  u64 mask = __ballot(pred);
  if (mask != 0 && lane_id() == __ffsll((long long)mask) - 1) atomicAdd(counter, (u64)__popcll(mask));
}

// Wave-private staging of list appends in LDS (128 entries): one global atomic per
// flush instead of one per wave and step.  `n` is wave-uniform.
constexpr int kWaveBuf = 128;
struct WaveBuf {
  u64 *lds;
  int n;
};

DEVI void wbuf_flush(WaveBuf &b, u64 *list, u64 *counter, int64_t cap, u64 *flags) {
  if (b.n == 0) return;
  const int lane = lane_id();
  __threadfence_block();
  u64 base = 0;
  if (lane == 0) base = atomicAdd(counter, (u64)b.n);
  base = __shfl(base, 0);
  for (int i = lane; i < b.n; i += 64) {
    const u64 idx = base + (u64)i;
    if ((int64_t)idx < cap) list[idx] = b.lds[i];
    else atomicOr(flags, (u64)kFlagQueueOverflow);
  }
  __threadfence_block();
  b.n = 0;
}

DEVI void wbuf_push(WaveBuf &b, bool pred, u64 val, u64 *list, u64 *counter, int64_t cap, u64 *flags) {
  const u64 mask = __ballot(pred);
  const int cnt = __popcll(mask);
  if (cnt == 0) return;
  if (b.n + cnt > kWaveBuf) wbuf_flush(b, list, counter, cap, flags);
  if (pred) b.lds[b.n + __popcll(mask & lanes_below(lane_id()))] = val;
  b.n += cnt;
}

// Block-wide sum of per-thread counts into global counters (end of kernel; every
// thread of the block must call it).
template <int NC>
DEVI void block_counts(u64 (&v)[NC], u64 *counters, const int (&slot)[NC]) {
  __shared__ u64 acc[NC];
  if (threadIdx.x < NC) acc[threadIdx.x] = 0;
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    u64 t = v[c];
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
    if (lane_id() == 0 && t) atomicAdd(&acc[c], t);
  }
  __syncthreads();
  if (threadIdx.x < NC && acc[threadIdx.x]) atomicAdd(&counters[cslot(slot[threadIdx.x])], acc[threadIdx.x]);
}

DEVI int wave_max_int(int v) {
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
  return v;
}

DEVI u64 wave_or(u64 v) {
  for (int off = 32; off > 0; off >>= 1) v |= __shfl_xor(v, off);
  return v;
}

// 64x64 bit-matrix transpose across the wave: on entry lane j holds row j, on
// exit lane b holds bit b of every lane's entry row (bit j = entry lane j, bit b).
DEVI u64 wave_transpose64(u64 a) {
  const int lane = lane_id();
  const u64 masks[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                        0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
  for (int st = 0; st < 6; ++st) {
    const int j = 32 >> st;
    const u64 m = masks[st];
    const u64 other = __shfl_xor(a, j);
    a = (lane & j) ? ((a & ~m) | ((other & ~m) >> j)) : ((a & m) | ((other & m) << j));
  }
  return a;
}

DEVI i128 shfl_i128(i128 v, int src) {
  unsigned __int128 u = (unsigned __int128)v;
  u64 lo = (u64)u, hi = (u64)(u >> 64);
  lo = __shfl(lo, src);
  hi = __shfl(hi, src);
  return (i128)(((unsigned __int128)hi << 64) | lo);
}

DEVI i128 shfl_xor_i128(i128 v, int off) {
  unsigned __int128 u = (unsigned __int128)v;
  u64 lo = (u64)u, hi = (u64)(u >> 64);
  lo = __shfl_xor(lo, off);
  hi = __shfl_xor(hi, off);
  return (i128)(((unsigned __int128)hi << 64) | lo);
}

// ------------------------------------------------------------- modular arithmetic
DEVI uint32_t mulmod(uint32_t a, uint32_t b) {
  u64 t = (u64)a * b;                       // < 2^62
  t = (t & kPrime) + (t >> 31);             // < 2^32
  t = (t & kPrime) + (t >> 31);             // <= 2^31
  return (uint32_t)(t >= kPrime ? t - kPrime : t);
}
DEVI uint32_t submod(uint32_t a, uint32_t b) { return a >= b ? a - b : a + kPrime - b; }
DEVI uint32_t powmod(uint32_t a, uint32_t e) {
  uint32_t r = 1;
  while (e) {
    if (e & 1) r = mulmod(r, a);
    a = mulmod(a, a);
    e >>= 1;
  }
  return r;
}
DEVI uint32_t tomod(int32_t s) {
  int64_t v = s % (int64_t)kPrime;
  return (uint32_t)(v < 0 ? v + kPrime : v);
}

// ---------------------------------------------------------- exact 128-bit helpers
// Stored matrix entries stay below 2^63 in magnitude, so a product of two fits in
// 126 bits and a difference of two products in 127 bits.  Anything larger raises
// the overflow flag (reported as EFM_EOVERFLOW).
constexpr i128 kSafe = (i128)1 << 63;
DEVI i128 iabs(i128 a) { return a < 0 ? -a : a; }
DEVI bool safe(i128 a) { return a < kSafe && a > -kSafe; }
DEVI i128 gcd_i128(i128 a, i128 b) {
  a = iabs(a);
  b = iabs(b);
  while (b != 0) {
    i128 t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// j-th set bit (0-based) of a W-word key, or -1
template <int W>
DEVI int select_bit(const u64 *Q, int j) {
#pragma unroll
  for (int w = 0; w < W; ++w) {
    int c = __popcll(Q[w]);
    if (j < c) {
      u64 x = Q[w];
      for (int t = 0; t < j; ++t) x &= x - 1;
      return w * 64 + __builtin_ctzll(x);
    }
    j -= c;
  }
  return -1;
}

// ------------------------------------------------------------------------ expand
// Table entry: tag(7) | fingerprint(14) | parent(32) | reaction(11).  A slot whose
// tag differs from the level's tag is free.
DEVI u64 make_entry(u64 tag, u64 h, u64 p, int r) {
  return (tag << 57) | (((h >> 50) & 0x3FFFull) << 43) | ((p & 0xFFFFFFFFull) << 11) | (u64)r;
}

// Insert child P|e_r; returns true when this lane created the entry (first copy).
template <int W>
DEVI bool table_insert(const DevLevel &L, u64 tag, u64 h, u64 p, int r, const u64 *P) {
  const u64 entry = make_entry(tag, h, p, r);
  const u64 fp = (h >> 50) & 0x3FFFull;
  u64 pos = h & L.tmask;
  for (u64 probe = 0; probe <= L.tmask; ++probe) {
    u64 cur = __hip_atomic_load(&L.table[pos], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while ((cur >> 57) != tag) {
      u64 prev = atomicCAS(&L.table[pos], cur, entry);
      if (prev == cur) return true;
      cur = prev;
    }
    if (((cur >> 43) & 0x3FFFull) == fp) {
      const u64 p2 = (cur >> 11) & 0xFFFFFFFFull;
      const int r2 = (int)(cur & 0x7FFull);
      bool eq = true;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        u64 a = P[w] | ((r >> 6) == w ? (1ull << (r & 63)) : 0ull);
        u64 b = L.keys[(int64_t)w * L.fcap + p2] | ((r2 >> 6) == w ? (1ull << (r2 & 63)) : 0ull);
        eq = eq && (a == b);
      }
      if (eq) return false;
    }
    pos = (pos + 1) & L.tmask;
  }
  atomicOr(&L.counters[cslot(kFlags)], (u64)kFlagUniqueOverflow);
  return false;
}

template <int W, int MW>
__global__ __launch_bounds__(256) void expand_kernel(DevNet net, DevLevel L) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = p < L.nparents;
  const u64 tag = (u64)L.tag;
  const bool keep_indep = L.level + 1 < L.depth_cap;
  u64 P[W], cand[W], T[MW];
  u64 h = 0;
  int ncand = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) { P[w] = 0; cand[w] = 0; }
#pragma unroll
  for (int q = 0; q < MW; ++q) T[q] = 0;
  if (live) {
#pragma unroll
    for (int w = 0; w < W; ++w) P[w] = L.keys[(int64_t)w * L.fcap + p];
    h = L.hash[p];
    if (L.root_cand) {
#pragma unroll
      for (int w = 0; w < W; ++w) cand[w] = L.root_cand[w] & ~P[w];
    } else {
      // role masks: A = touched by an irreversible producer, B = by an irreversible
      // consumer, C = by a reversible reaction, C2 = by two or more reversible ones
      u64 A[MW], B[MW], C[MW], C2[MW];
#pragma unroll
      for (int q = 0; q < MW; ++q) { A[q] = 0; B[q] = 0; C[q] = 0; C2[q] = 0; }
#pragma unroll
      for (int w = 0; w < W; ++w) {
        u64 bits = P[w];
        while (bits) {
          const int r = w * 64 + __builtin_ctzll(bits);
          bits &= bits - 1;
          const u64 *pm = net.rxn_prodM + (int64_t)r * MW;
          const u64 *cm = net.rxn_consM + (int64_t)r * MW;
          const u64 *rm = net.rxn_revM + (int64_t)r * MW;
#pragma unroll
          for (int q = 0; q < MW; ++q) {
            const u64 rq = rm[q];
            A[q] |= pm[q];
            B[q] |= cm[q];
            C2[q] |= C[q] & rq;
            C[q] |= rq;
          }
        }
      }
      int istar = -1;
#pragma unroll
      for (int q = 0; q < MW; ++q) {
        T[q] = A[q] | B[q] | C[q];
        const u64 cov = (A[q] & B[q]) | (C[q] & (A[q] | B[q])) | C2[q];
        const u64 U = T[q] & ~cov;
        if (istar < 0 && U) istar = q * 64 + __builtin_ctzll(U);
      }
      if (istar >= 0) {
        const int q = istar >> 6;
        const u64 bit = 1ull << (istar & 63);
        u64 Aq = 0, Bq = 0;
#pragma unroll
        for (int qq = 0; qq < MW; ++qq) if (qq == q) { Aq = A[qq]; Bq = B[qq]; }
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
            const u64 *nb = net.rxn_nbrR + (int64_t)r * W;
#pragma unroll
            for (int ww = 0; ww < W; ++ww) cand[ww] |= nb[ww];
          }
        }
#pragma unroll
        for (int w = 0; w < W; ++w) cand[w] &= ~P[w];
      }
    }
#pragma unroll
    for (int w = 0; w < W; ++w) ncand += __popcll(cand[w]);
  }

  // children: uniform trip count per wave so the ballots stay converged
  __shared__ u64 stage[4][kWaveBuf];
  const int wib = threadIdx.x >> 6;
  WaveBuf bsurv{stage[wib], 0};
  u64 n_unique = 0, n_indep = 0, n_capped = 0, n_rc = 0;
  u64 rcm[W];                  // this parent's distinct row-closed children
#pragma unroll
  for (int w = 0; w < W; ++w) rcm[w] = 0;
  const int maxc = wave_max_int(ncand);
  for (int it = 0; it < maxc; ++it) {
    const bool act = it < ncand;
    bool uniq = false, rc = false;
    int r = 0;
    if (act) {
      bool got = false;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        if (!got && cand[w] != 0) {
          r = w * 64 + __builtin_ctzll(cand[w]);
          cand[w] &= cand[w] - 1;
          got = true;
        }
      }
      const u64 *tm = net.rxn_touchM + (int64_t)r * MW;
      u64 outside = 0;
#pragma unroll
      for (int q = 0; q < MW; ++q) outside |= tm[q] & ~T[q];
      rc = outside == 0;
      uniq = table_insert<W>(L, tag, h ^ net.zob[r], (u64)p, r, P);
    }
    const u64 ref = ((u64)p << 12) | ((u64)r << 1) | (rc ? 1ull : 0ull);
    wbuf_push(bsurv, uniq && !rc && keep_indep, ref, L.surv, &L.counters[cslot(kSurv)], L.ucap,
              &L.counters[cslot(kFlags)]);
    if (uniq && rc) {
#pragma unroll
      for (int w = 0; w < W; ++w) rcm[w] |= (r >> 6) == w ? (1ull << (r & 63)) : 0ull;
    }
    n_rc += (uniq && rc) ? 1 : 0;
    n_unique += uniq ? 1 : 0;
    n_indep += (uniq && !rc) ? 1 : 0;
    n_capped += (uniq && !rc && !keep_indep) ? 1 : 0;
  }
  wbuf_flush(bsurv, L.surv, &L.counters[cslot(kSurv)], L.ucap, &L.counters[cslot(kFlags)]);
  {
    // one rank-queue entry per parent that has row-closed children
    bool any = false;
#pragma unroll
    for (int w = 0; w < W; ++w) any = any || rcm[w] != 0;
    const u64 m = __ballot(any);
    if (m) {
      const int leader = __ffsll((long long)m) - 1;
      u64 b0 = 0;
      if (lane_id() == leader) b0 = atomicAdd(&L.counters[cslot(kParQ)], (u64)__popcll(m));
      b0 = __shfl(b0, leader);
      if (any) {
        const u64 idx = b0 + (u64)__popcll(m & lanes_below(lane_id()));
        if ((int64_t)idx < L.ucap) {
          L.parq[idx] = (u64)p;
#pragma unroll
          for (int w = 0; w < W; ++w) L.parmask[(int64_t)idx * W + w] = rcm[w];
        } else {
          atomicOr(&L.counters[cslot(kFlags)], (u64)kFlagQueueOverflow);
        }
      }
    }
  }
  u64 v[5] = {(u64)ncand, n_unique, n_indep, n_capped, n_rc};
  const int slots[5] = {kChildren, kUnique, kIndep, kCapped, kRowClosed};
  block_counts<5>(v, L.counters, slots);
}

// ------------------------------------------------------------------- rank (parent)
// One wave per parent P with its distinct row-closed children r_1..r_m.  Every
// child's rows lie inside P's rows.  Lane j holds column j of P | {r_1..r_m}.
// The rows are bit masks over those columns (odd coefficients); XOR elimination
// over P's columns only, applied to whole rows, leaves each child's column
// reduced against P modulo 2, so a child is certified independent exactly when
// its reduced column has a 1 in a row P did not use as a pivot.  Independence
// modulo 2 implies independence over the rationals.  Children not certified
// (or pruned by the found set) go on to the per-child test.
template <int W, int MW>
__global__ __launch_bounds__(256) void rank_parent_kernel(DevNet net, DevLevel L, int prune) {
  __shared__ u64 stage[2][4][kWaveBuf];
  const int wib = threadIdx.x >> 6;
  const int lane = lane_id();
  const int wpb = blockDim.x >> 6;
  const int64_t nitems = min((int64_t)L.counters[cslot(kParQ)], L.ucap);
  const bool keep_indep = L.level + 1 < L.depth_cap;
  const int64_t nf = min((int64_t)L.nfound_prev, L.ecap);
  WaveBuf bsurv{stage[0][wib], 0}, bslow{stage[1][wib], 0};
  u64 n_indep = 0, n_pruned = 0, n_capped = 0;

  for (int64_t item = (int64_t)blockIdx.x * wpb + wib; item < nitems; item += (int64_t)gridDim.x * wpb) {
    const u64 p = L.parq[item];
    u64 P[W], M[W], A[W];
    int kall = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      P[w] = L.keys[(int64_t)w * L.fcap + p];
      M[w] = L.parmask[item * W + w];
      A[w] = P[w] | M[w];
      kall += __popcll(A[w]);
    }
    // found-set prune, child by child
    if (prune && nf > 0 && nf <= kPruneMax) {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        u64 bits = M[w];
        while (bits) {
          const int r = w * 64 + __builtin_ctzll(bits);
          bits &= bits - 1;
          bool hit = false;
          for (int64_t f0 = 0; f0 < nf && !hit; f0 += 64) {
            const int64_t f = f0 + lane;
            bool sub = f < nf;
            if (sub) {
#pragma unroll
              for (int ww = 0; ww < W; ++ww) {
                const u64 Qw = P[ww] | ((r >> 6) == ww ? (1ull << (r & 63)) : 0ull);
                sub = sub && ((L.fkeys[(int64_t)ww * L.ecap + f] & ~Qw) == 0);
              }
            }
            hit = __ballot(sub) != 0;
          }
          if (hit) {
            n_pruned += lane == 0 ? 1 : 0;
            M[w] &= ~(1ull << (r & 63));
          }
        }
      }
    }
    kall = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      A[w] = P[w] | M[w];                        // pruned children are gone from M
      kall += __popcll(A[w]);
    }
    bool full = kall <= 64 && !L.debug_prime && !L.no_gf2;
    u64 rowm[MW];
    bool used[MW];
    int col = -1;
    bool child = false;
    if (full) {
      col = lane < kall ? select_bit<W>(A, lane) : -1;
#pragma unroll
      for (int w = 0; w < W; ++w)
        if (col >= 0 && (col >> 6) == w) child = (M[w] >> (col & 63)) & 1ull;
      u64 om[MW], tm[MW];
#pragma unroll
      for (int q = 0; q < MW; ++q) {
        om[q] = col >= 0 ? net.rxn_oddM[(int64_t)col * MW + q] : 0ull;
        tm[q] = (col >= 0 && !child) ? net.rxn_touchM[(int64_t)col * MW + q] : 0ull;
      }
#pragma unroll
      for (int q = 0; q < MW; ++q) {
        // rows P does not touch are dropped (used) so they never serve as pivots
        const u64 T = wave_or(tm[q]);
        rowm[q] = wave_transpose64(om[q]);
        used[q] = !((T >> lane) & 1ull);
      }
      u64 cols = __ballot(col >= 0 && !child);
      while (cols) {
        const int c = __ffsll((long long)cols) - 1;
        cols &= cols - 1;
        int pq = -1, pl = -1;
#pragma unroll
        for (int q = 0; q < MW; ++q) {
          if (pq < 0) {
            const u64 cand = __ballot(!used[q] && ((rowm[q] >> c) & 1ull));
            if (cand) { pq = q; pl = __ffsll((long long)cand) - 1; }
          }
        }
        if (pq < 0) { full = false; break; }
        u64 prow = 0;
#pragma unroll
        for (int q = 0; q < MW; ++q) {
          if (q == pq) {
            const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)rowm[q], pl);
            const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(rowm[q] >> 32), pl);
            prow = ((u64)hi << 32) | lo;
          }
        }
#pragma unroll
        for (int q = 0; q < MW; ++q) {
          const bool me = (q == pq) && (lane == pl);
          if (!me && ((rowm[q] >> c) & 1ull)) rowm[q] ^= prow;
          if (me) used[q] = true;
        }
      }
    }
    // children, in reaction order: certified ones are independent
    u64 ccols = __ballot(child);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      u64 bits = M[w];
      while (bits) {
        const int r = w * 64 + __builtin_ctzll(bits);
        bits &= bits - 1;
        bool cert = false;
        if (full) {
          const int c = __ffsll((long long)ccols) - 1;   // children's columns come in reaction order
          ccols &= ccols - 1;
          bool any = false;
#pragma unroll
          for (int q = 0; q < MW; ++q) any = any || (!used[q] && ((rowm[q] >> c) & 1ull));
          cert = __ballot(any) != 0;
        }
        const u64 ref = (p << 12) | ((u64)r << 1) | 1ull;
        n_indep += (cert && lane == 0) ? 1 : 0;
        n_capped += (cert && !keep_indep && lane == 0) ? 1 : 0;
        wbuf_push(bsurv, cert && keep_indep && lane == 0, ref, L.surv, &L.counters[cslot(kSurv)], L.ucap,
                  &L.counters[cslot(kFlags)]);
        wbuf_push(bslow, !cert && lane == 0, ref, L.rankq, &L.counters[cslot(kRankQ)], L.ucap,
                  &L.counters[cslot(kFlags)]);
      }
    }
  }
  wbuf_flush(bsurv, L.surv, &L.counters[cslot(kSurv)], L.ucap, &L.counters[cslot(kFlags)]);
  wbuf_flush(bslow, L.rankq, &L.counters[cslot(kRankQ)], L.ucap, &L.counters[cslot(kFlags)]);
  u64 v[3] = {n_indep, n_pruned, n_capped};
  const int slots[3] = {kIndep, kPruned, kCapped};
  block_counts<3>(v, L.counters, slots);
}

// -------------------------------------------------------------------------- rank
// One wave per row-closed child Q = P | e_r.  Lane j holds column j (the j-th
// reaction of Q) as its few nonzero entries in registers.  Singleton rows are
// peeled first; the remaining rows then stream through a basis kept in LDS in
// reduced form, and the child is independent once the basis has as many rows as
// there are unpeeled columns.
template <int W, int MW>
__global__ __launch_bounds__(256) void rank_kernel(DevNet net, DevLevel L, int prune, int kq_max) {
  __shared__ u64 stage[2][4][kWaveBuf];
  const int wib = threadIdx.x >> 6;
  const int lane = lane_id();
  const int wpb = blockDim.x >> 6;
  const int64_t nitems = min((int64_t)L.counters[cslot(kRankQ)], L.ucap);
  const bool keep_indep = L.level + 1 < L.depth_cap;
  const int64_t nf = min((int64_t)L.nfound_prev, L.ecap);
  WaveBuf bsurv{stage[0][wib], 0}, bexact{stage[1][wib], 0};
  u64 n_indep = 0, n_pruned = 0, n_capped = 0;

  for (int64_t item = (int64_t)blockIdx.x * wpb + wib; item < nitems; item += (int64_t)gridDim.x * wpb) {
    const u64 ref = L.rankq[item];
    const u64 p = ref >> 12;
    const int r = (int)((ref >> 1) & 0x7FF);
    u64 Q[W];
#pragma unroll
    for (int w = 0; w < W; ++w)
      Q[w] = L.keys[(int64_t)w * L.fcap + p] | ((r >> 6) == w ? (1ull << (r & 63)) : 0ull);

    // minimality prune: a found pathway inside Q makes Q dependent and not elementary
    if (prune && nf > 0 && nf <= kPruneMax) {
      bool hit = false;
      for (int64_t f0 = 0; f0 < nf && !hit; f0 += 64) {
        const int64_t f = f0 + lane;
        bool sub = f < nf;
        if (sub) {
#pragma unroll
          for (int w = 0; w < W; ++w) sub = sub && ((L.fkeys[(int64_t)w * L.ecap + f] & ~Q[w]) == 0);
        }
        hit = __ballot(sub) != 0;
      }
      if (hit) {
        n_pruned += lane == 0 ? 1 : 0;
        continue;
      }
    }

    int kq = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) kq += __popcll(Q[w]);
    const int col = lane < kq ? select_bit<W>(Q, lane) : -1;
    u64 tm[MW];
#pragma unroll
    for (int q = 0; q < MW; ++q) tm[q] = col >= 0 ? net.rxn_touchM[(int64_t)col * MW + q] : 0ull;

    // Singleton peeling: a row that only one live column touches forces that
    // column's flux to zero, so column and row leave the matrix and the rank
    // drops by exactly one.  Q is independent iff what remains is, and it is
    // independent outright once r's column is peeled (P is independent).
    bool alive = col >= 0;
    while (true) {
      u64 once[MW], multi[MW];
#pragma unroll
      for (int q = 0; q < MW; ++q) { once[q] = alive ? tm[q] : 0ull; multi[q] = 0ull; }
      for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int q = 0; q < MW; ++q) {
          const u64 o2 = __shfl_xor(once[q], off), m2 = __shfl_xor(multi[q], off);
          multi[q] = multi[q] | m2 | (once[q] & o2);
          once[q] = (once[q] | o2) & ~multi[q];
        }
      }
      u64 hit = 0;
#pragma unroll
      for (int q = 0; q < MW; ++q) hit |= tm[q] & once[q];
      const bool peel = alive && hit != 0;
      if (__ballot(peel) == 0) break;
      alive = alive && !peel;
    }
    const bool r_alive = __ballot(alive && col == r) != 0;
    const int ncore = __popcll(__ballot(alive));
    u64 T[MW];
#pragma unroll
    for (int q = 0; q < MW; ++q) T[q] = wave_or(alive ? tm[q] : 0ull);
    int nrows = 0;
#pragma unroll
    for (int q = 0; q < MW; ++q) nrows += __popcll(T[q]);

    bool indep = !r_alive;
    if (!L.debug_prime && !L.no_gf2 && r_alive && nrows >= ncore) {
      // GF(2) certificate: columns independent modulo 2 are independent over the
      // rationals.  Lane b holds, for the core row q*64+b, the bit mask of the
      // columns whose coefficient there is odd; XOR elimination over the columns.
      u64 om[MW], rowm[MW];
      bool used[MW];
#pragma unroll
      for (int q = 0; q < MW; ++q) {
        om[q] = alive ? net.rxn_oddM[(int64_t)col * MW + q] : 0ull;
        rowm[q] = wave_transpose64(om[q]);
        used[q] = !((T[q] >> lane) & 1ull);
      }
      u64 cols = __ballot(alive);
      bool ok = true;
      while (cols) {
        const int c = __ffsll((long long)cols) - 1;
        cols &= cols - 1;
        int pq = -1, pl = -1;
#pragma unroll
        for (int q = 0; q < MW; ++q) {
          if (pq < 0) {
            const u64 cand = __ballot(!used[q] && ((rowm[q] >> c) & 1ull));
            if (cand) { pq = q; pl = __ffsll((long long)cand) - 1; }
          }
        }
        if (pq < 0) { ok = false; break; }
        u64 prow = 0;
#pragma unroll
        for (int q = 0; q < MW; ++q) {
          if (q == pq) {
            const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)rowm[q], pl);
            const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(rowm[q] >> 32), pl);
            prow = ((u64)hi << 32) | lo;
          }
        }
#pragma unroll
        for (int q = 0; q < MW; ++q) {
          const bool me = (q == pq) && (lane == pl);
          if (!me && ((rowm[q] >> c) & 1ull)) rowm[q] ^= prow;
          if (me) used[q] = true;
        }
      }
      indep = ok;
    }
    if (!L.debug_prime && r_alive && nrows >= ncore && !indep) {
      // this lane's column entries
      uint32_t ent[kMaxEnt];
      int nnz = alive ? net.rxn_nnz[col] : 0;
      const bool dense = nnz < 0;
#pragma unroll
      for (int e = 0; e < kMaxEnt; ++e) ent[e] = (e < nnz) ? net.rxn_ent[(int64_t)col * kMaxEnt + e] : 0xFFFF0000u;
      // The basis lives in registers (lane j holds column j of every basis row) in
      // reduced row-echelon form without normalisation: row b has a nonzero pivot
      // value d_b in its pivot column and every other row has a 0 there.  A new
      // row x0 is reduced fraction-free, x <- d_b x - (sigma f_b) row_b over the
      // pivots where x0 itself is nonzero (f_b = x0[pc_b], sigma = product of the
      // d_b used so far), which leaves x a nonzero multiple of the exact
      // reduction.  No modular inverse is needed.
      uint32_t B[kMaxDepth];
#pragma unroll
      for (int t = 0; t < kMaxDepth; ++t) B[t] = 0;
      int nb = 0;
      int rowof = -1;              // lane c: the basis row whose pivot column is c
#pragma unroll
      for (int q = 0; q < MW; ++q) {
        u64 bits = T[q];
        while (bits && !indep) {
          const int i = q * 64 + __builtin_ctzll(bits);
          bits &= bits - 1;
          int32_t c = 0;
          if (dense) {
            c = net.Sint[(int64_t)i * net.n + col];
          } else {
#pragma unroll
            for (int e = 0; e < kMaxEnt; ++e)
              if ((int)(ent[e] >> 16) == i) c = (int32_t)(int16_t)(ent[e] & 0xFFFFu);
          }
          const uint32_t x0 = tomod(c);
          uint32_t x = x0, sigma = 1;
          u64 hits = __ballot(x0 != 0 && rowof >= 0);
          while (hits) {
            const int pc = __ffsll((long long)hits) - 1;
            hits &= hits - 1;
            const int bidx = __builtin_amdgcn_readfirstlane(__builtin_amdgcn_readlane(rowof, pc));
            const uint32_t f = (uint32_t)__builtin_amdgcn_readlane((int)x0, pc);
            const uint32_t rb = B[bidx];
            const uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)rb, pc);
            x = submod(mulmod(d, x), mulmod(mulmod(sigma, f), rb));
            sigma = mulmod(sigma, d);
          }
          const u64 nz = __ballot(x != 0);
          if (nz) {
            const int pc = __ffsll((long long)nz) - 1;
            const uint32_t dn = (uint32_t)__builtin_amdgcn_readlane((int)x, pc);
            for (int bb = 0; bb < nb; ++bb) {
              const uint32_t rb = B[bb];
              const uint32_t cb = (uint32_t)__builtin_amdgcn_readlane((int)rb, pc);
              if (cb) B[bb] = submod(mulmod(dn, rb), mulmod(cb, x));
            }
            B[nb] = x;
            if (lane == pc) rowof = nb;
            nb++;
            if (nb == ncore) indep = true;
          }
        }
      }
    }
    if (L.debug_prime) indep = false;
    n_indep += (indep && lane == 0) ? 1 : 0;
    n_capped += (indep && !keep_indep && lane == 0) ? 1 : 0;
    wbuf_push(bsurv, indep && keep_indep && lane == 0, ref, L.surv, &L.counters[cslot(kSurv)], L.ucap,
              &L.counters[cslot(kFlags)]);
    wbuf_push(bexact, !indep && lane == 0, ref, L.exactq, &L.counters[cslot(kExactQ)], L.ucap,
              &L.counters[cslot(kFlags)]);
  }
  wbuf_flush(bsurv, L.surv, &L.counters[cslot(kSurv)], L.ucap, &L.counters[cslot(kFlags)]);
  wbuf_flush(bexact, L.exactq, &L.counters[cslot(kExactQ)], L.ucap, &L.counters[cslot(kFlags)]);
  u64 v[3] = {n_indep, n_pruned, n_capped};
  const int slots[3] = {kIndep, kPruned, kCapped};
  block_counts<3>(v, L.counters, slots);
}

// ------------------------------------------------------------------------- exact
// One wave per child.  Lane j owns column j of the dense matrix S_int[T, Q] kept in
// global scratch (row-major, 64 entries per row); entries of other columns travel
// by lane shuffles only.
template <int W, int MW>
__global__ __launch_bounds__(64) void exact_kernel(DevNet net, DevLevel L) {
  const int lane = lane_id();
  const int64_t nitems = min((int64_t)L.counters[cslot(kExactQ)], L.ucap);
  const bool keep_indep = L.level + 1 < L.depth_cap;
  i128 *M = L.xscratch + (size_t)blockIdx.x * (size_t)net.mi * 64;

  for (int64_t item = blockIdx.x; item < nitems; item += gridDim.x) {
    const u64 ref = L.exactq[item];
    const u64 p = ref >> 12;
    const int r = (int)((ref >> 1) & 0x7FF);
    u64 Q[W];
#pragma unroll
    for (int w = 0; w < W; ++w)
      Q[w] = L.keys[(int64_t)w * L.fcap + p] | ((r >> 6) == w ? (1ull << (r & 63)) : 0ull);
    int kq = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) kq += __popcll(Q[w]);
    const bool mine = lane < kq;
    const int col = mine ? select_bit<W>(Q, lane) : -1;
    u64 T[MW];
#pragma unroll
    for (int q = 0; q < MW; ++q) T[q] = wave_or(col >= 0 ? net.rxn_touchM[(int64_t)col * MW + q] : 0ull);

    // load the column
    int R = 0;
#pragma unroll
    for (int q = 0; q < MW; ++q) {
      u64 bits = T[q];
      while (bits) {
        const int i = q * 64 + __builtin_ctzll(bits);
        bits &= bits - 1;
        M[(size_t)R * 64 + lane] = mine ? (i128)net.Sint[(int64_t)i * net.n + col] : (i128)0;
        R++;
      }
    }

    // fraction-free elimination (Bareiss): after the step on pivot row t every
    // entry below is a (t+2)-minor, so the division by the previous pivot is exact
    bool ovf = false;
    int rank = 0;
    int pivreg = -1;               // lane t holds the pivot column of row t
    i128 prev = 1;
    for (int c = 0; c < kq && rank < R; ++c) {
      int piv = -1;
      if (lane == c)
        for (int i = rank; i < R; ++i)
          if (M[(size_t)i * 64 + lane] != 0) { piv = i; break; }
      piv = __shfl(piv, c);
      if (piv < 0) continue;
      if (piv != rank) {
        const i128 a = M[(size_t)piv * 64 + lane];
        M[(size_t)piv * 64 + lane] = M[(size_t)rank * 64 + lane];
        M[(size_t)rank * 64 + lane] = a;
      }
      const i128 pv = shfl_i128(M[(size_t)rank * 64 + lane], c);
      const i128 top = M[(size_t)rank * 64 + lane];
      for (int i = rank + 1; i < R; ++i) {
        // every row below is updated, also when f = 0: the entries must become minors
        const i128 f = shfl_i128(M[(size_t)i * 64 + lane], c);
        if (lane >= c && mine) {
          const i128 a = M[(size_t)i * 64 + lane];
          if (!safe(a) || !safe(top) || !safe(pv) || !safe(f)) ovf = true;
          else M[(size_t)i * 64 + lane] = (pv * a - f * top) / prev;
        }
      }
      if (lane == rank) pivreg = c;
      prev = pv;
      rank++;
    }
    if (__ballot(ovf)) {
      if (lane == 0) atomicOr(&L.counters[cslot(kFlags)], (u64)kFlagIntOverflow);
      continue;
    }
    if (rank == kq) {                      // the modular test was fooled: independent
      if (lane == 0) {
        atomicAdd(&L.counters[cslot(kIndep)], 1ull);
        if (keep_indep) {
          const u64 idx = atomicAdd(&L.counters[cslot(kSurv)], 1ull);
          if ((int64_t)idx < L.ucap) L.surv[idx] = ref;
          else atomicOr(&L.counters[cslot(kFlags)], (u64)kFlagQueueOverflow);
        } else {
          atomicAdd(&L.counters[cslot(kCapped)], 1ull);
        }
      }
      continue;
    }
    if (rank != kq - 1) continue;          // cannot happen for an independent parent

    // the free column
    bool piv_here = false;
    for (int t = 0; t < rank; ++t) piv_here = piv_here || (__shfl(pivreg, t) == lane);
    const u64 freem = __ballot(mine && !piv_here);
    const int fcol = __ffsll((long long)freem) - 1;

    // integer back substitution, v_f = 1, partial vector kept primitive
    i128 v = lane == fcol ? (i128)1 : (i128)0;
    for (int t = rank - 1; t >= 0 && !ovf; --t) {
      const int pc = __shfl(pivreg, t);
      const i128 a = M[(size_t)t * 64 + lane];
      i128 term = 0;
      if (lane > pc && mine && v != 0 && a != 0) {
        if (!safe(a) || !safe(v)) ovf = true;
        else term = a * v;
      }
      i128 sum = term;
      for (int off = 32; off > 0; off >>= 1) {
        const i128 o = shfl_xor_i128(sum, off);
        if (iabs(sum) >= ((i128)1 << 125) || iabs(o) >= ((i128)1 << 125)) ovf = true;
        sum += o;
      }
      ovf = __ballot(ovf) != 0;
      if (ovf) break;
      const i128 pt = shfl_i128(a, pc);
      const i128 g = gcd_i128(sum, pt);
      const i128 mult = iabs(pt) / g;
      if (lane > pc && mult != 1) {
        if (!safe(v) || !safe(mult)) ovf = true;
        else v *= mult;
      }
      if (lane == pc) v = pt > 0 ? -(sum / g) : (sum / g);
      i128 G = iabs(v);
      for (int off = 32; off > 0; off >>= 1) G = gcd_i128(G, shfl_xor_i128(G, off));
      if (G > 1) v /= G;
      ovf = __ballot(ovf) != 0;
    }
    if (ovf) {
      if (lane == 0) atomicOr(&L.counters[cslot(kFlags)], (u64)kFlagIntOverflow);
      continue;
    }

    // Definition 2 and the target: full support, one sign on irreversible
    // reactions (made positive), S[x,:] v > 0
    if (__ballot(mine && v == 0) != 0) continue;
    const bool irr = mine && !((net.rev_bits[col >> 6] >> (col & 63)) & 1ull);
    const u64 posm = __ballot(irr && v > 0), negm = __ballot(irr && v < 0);
    if (posm && negm) continue;
    i128 prod = mine ? (i128)L.Sx[col] * v : (i128)0;
    for (int off = 32; off > 0; off >>= 1) prod += shfl_xor_i128(prod, off);
    int sgn = posm ? 1 : (negm ? -1 : (prod > 0 ? 1 : -1));
    if (sgn < 0) { v = -v; prod = -prod; }
    if (prod <= 0) continue;
    const i128 lim = (i128)1 << 63;
    if (__ballot(v >= lim || v < -lim) != 0) {
      if (lane == 0) atomicOr(&L.counters[cslot(kFlags)], (u64)kFlagIntOverflow);
      continue;
    }
    u64 slot = 0;
    if (lane == 0) slot = atomicAdd(&L.counters[cslot(kFound)], 1ull);
    slot = __shfl(slot, 0);
    if ((int64_t)slot >= L.ecap) {
      if (lane == 0) atomicOr(&L.counters[cslot(kFlags)], (u64)kFlagFoundOverflow);
      continue;
    }
#pragma unroll
    for (int w = 0; w < W; ++w)
      if (lane == w) L.fkeys[(int64_t)w * L.ecap + slot] = Q[w];
    if (mine) L.fflux[(int64_t)slot * kMaxDepth + lane] = (int64_t)v;
    if (lane == 0) atomicAdd(&L.counters[cslot(kEmitted)], 1ull);
  }
}

// ------------------------------------------------------------- truncation select

// Radix selection of the frontier cap's smallest keys, one key byte per pass from
// the most significant.  sel[i] is 2 while survivor i is undecided, then 1
// (selected) or 0 (rejected).  skey[i] caches the key word the current byte
// lies in; it is refilled when a pass enters a new word.
template <int W>
DEVI u64 key_word(const DevLevel &L, u64 ref, int w) {
  const u64 p = ref >> 12;
  const int r = (int)((ref >> 1) & 0x7FF);
  return L.keys[(int64_t)w * L.fcap + p] | ((r >> 6) == w ? (1ull << (r & 63)) : 0ull);
}

// Histogram of the undecided members' digits for pass `pass` (state and histogram
// are double-buffered by pass parity).  Digits are highly skewed (the top bytes
// of nearly all keys agree), so each wave groups its lanes by digit and adds one
// count per distinct digit.
template <int W>
__global__ __launch_bounds__(256) void select_hist_kernel(DevLevel L, int byte, int refill, int pass) {
  __shared__ uint32_t h[256];
  const SelState *st = L.selst + (pass & 1);
  if (st->done) return;
  uint32_t *hist = L.hist + 256 * (pass & 1);
  const int64_t n = min((int64_t)L.counters[cslot(kSurv)], L.ucap);
  h[threadIdx.x] = 0;
  __syncthreads();
  const int lane = lane_id();
  const int shift = (byte & 7) * 8;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t base = wave * 64; base < n; base += nwaves * 64) {
    const int64_t i = base + lane;
    const bool act = i < n && L.sel[i] == 2;
    if (__ballot(act) == 0) continue;
    uint32_t d = 0;
    if (act) {
      u64 kw;
      if (refill) {
        kw = key_word<W>(L, L.surv[i], byte >> 3);
        L.skey[i] = kw;
      } else {
        kw = L.skey[i];
      }
      d = (uint32_t)((kw >> shift) & 0xFF);
    }
    u64 pending = __ballot(act);
    while (pending) {
      const uint32_t v = (uint32_t)__builtin_amdgcn_readlane((int)d, __ffsll((long long)pending) - 1);
      const u64 m = __ballot(act && d == v) & pending;
      if (lane == __ffsll((long long)m) - 1) atomicAdd(&h[v], (uint32_t)__popcll(m));
      pending &= ~m;
    }
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// Every block derives the pass's decision from the finished histogram: the
// boundary digit v (undecided members below it are selected, above it
// rejected), whether every member with digit v fits, or whether the pass decides
// nothing.  Block 0 writes the next pass's state and clears its histogram.
template <int W>
__global__ __launch_bounds__(256) void select_split_kernel(DevLevel L, int byte, int pass) {
  __shared__ uint32_t dec[3];
  __shared__ int64_t rem;
  const SelState *st = L.selst + (pass & 1);
  SelState *nx = L.selst + ((pass + 1) & 1);
  const uint32_t *hist = L.hist + 256 * (pass & 1);
  const bool lead = blockIdx.x == 0;
  if (lead) L.hist[256 * ((pass + 1) & 1) + threadIdx.x] = 0;
  if (st->done) {
    if (lead && threadIdx.x == 0) *nx = *st;
    return;
  }
  if (threadIdx.x == 0) {
    int64_t cum = 0;
    int v = 0;
    for (v = 0; v < 255; ++v) {
      if (cum + (int64_t)hist[v] >= st->needed) break;
      cum += hist[v];
    }
    const int64_t hv = hist[v];
    const int64_t remaining = st->needed - cum;
    const uint32_t all_sel = hv == remaining ? 1u : 0u;
    dec[0] = (uint32_t)v;
    dec[1] = all_sel;
    dec[2] = (!all_sel && hv == st->nb) ? 1u : 0u;
    rem = remaining;
    if (lead) {
      SelState t = *st;
      if (!dec[2]) {
        t.needed = remaining;
        t.nb = hv;
        t.done = all_sel;
      }
      *nx = t;
    }
  }
  __syncthreads();
  if (dec[2]) return;                       // one digit only: nothing decided here
  const uint32_t digit = dec[0];
  const int all_sel = (int)dec[1];
  const int shift = (byte & 7) * 8;
  const int64_t n = min((int64_t)L.counters[cslot(kSurv)], L.ucap);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    if (L.sel[i] != 2) continue;
    const uint32_t d = (uint32_t)((L.skey[i] >> shift) & 0xFF);
    if (d < digit || (d == digit && all_sel)) L.sel[i] = 1;
    else if (d > digit) L.sel[i] = 0;
  }
}

// Writes the next frontier.  Without a cap the survivor order is kept (position =
// survivor index).  With a cap the selected members are compacted with one global
// atomic per block and per 1024 survivors.
template <int W>
__global__ __launch_bounds__(256) void materialize_kernel(DevNet net, DevLevel L, int use_sel) {
  __shared__ uint32_t wcount[4][4];
  __shared__ u64 bbase;
  const int64_t n = min((int64_t)L.counters[cslot(kSurv)], L.ucap);
  const int lane = lane_id();
  const int wib = threadIdx.x >> 6;
  for (int64_t base = (int64_t)blockIdx.x * 1024; base < n; base += (int64_t)gridDim.x * 1024) {
    bool act[4];
    u64 ref[4], dst[4];
    u64 mask[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t idx = base + t * 256 + threadIdx.x;
      act[t] = idx < n && (!use_sel || L.sel[idx] == 1);
      ref[t] = act[t] ? L.surv[idx] : 0ull;
      dst[t] = (u64)idx;
      mask[t] = __ballot(act[t]);
    }
    if (use_sel) {
      if (lane == 0)
        for (int t = 0; t < 4; ++t) wcount[t][wib] = (uint32_t)__popcll(mask[t]);
      __syncthreads();
      if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (int t = 0; t < 4; ++t)
          for (int w = 0; w < 4; ++w) tot += wcount[t][w];
        bbase = tot ? atomicAdd(&L.counters[cslot(kNext)], (u64)tot) : 0ull;
      }
      __syncthreads();
      u64 off = bbase;
      for (int t = 0; t < 4; ++t) {
        for (int w = 0; w < 4; ++w) {
          if (w == wib) dst[t] = off + (u64)__popcll(mask[t] & lanes_below(lane));
          off += wcount[t][w];
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (!act[t]) continue;
      const u64 p = ref[t] >> 12;
      const int r = (int)((ref[t] >> 1) & 0x7FF);
#pragma unroll
      for (int w = 0; w < W; ++w)
        L.nkeys[(int64_t)w * L.fcap + dst[t]] =
            L.keys[(int64_t)w * L.fcap + p] | ((r >> 6) == w ? (1ull << (r & 63)) : 0ull);
      L.nhash[dst[t]] = L.hash[p] ^ net.zob[r];
    }
  }
}

__global__ void clear_kernel(u64 *p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// -------------------------------------------------------------------- launchers
static int g_cus = 0;
static int num_cus() {
  if (g_cus == 0) {
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&g_cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (g_cus <= 0) g_cus = 256;
  }
  return g_cus;
}

#define EFM_DISPATCH_W(Wv, FN, ...)                        \
  switch (Wv) {                                            \
    case 1: FN<1>(__VA_ARGS__); break;                     \
    case 2: FN<2>(__VA_ARGS__); break;                     \
    case 4: FN<4>(__VA_ARGS__); break;                     \
    case 8: FN<8>(__VA_ARGS__); break;                     \
    default: FN<16>(__VA_ARGS__); break;                   \
  }

#define EFM_DISPATCH_WM(Wv, MWv, FN, ...)                                  \
  switch (Wv * 100 + MWv) {                                                \
    case 101: FN<1, 1>(__VA_ARGS__); break;                                \
    case 102: FN<1, 2>(__VA_ARGS__); break;                                \
    case 201: FN<2, 1>(__VA_ARGS__); break;                                \
    case 202: FN<2, 2>(__VA_ARGS__); break;                                \
    case 204: FN<2, 4>(__VA_ARGS__); break;                                \
    case 401: FN<4, 1>(__VA_ARGS__); break;                                \
    case 402: FN<4, 2>(__VA_ARGS__); break;                                \
    case 404: FN<4, 4>(__VA_ARGS__); break;                                \
    case 802: FN<8, 2>(__VA_ARGS__); break;                                \
    case 804: FN<8, 4>(__VA_ARGS__); break;                                \
    case 808: FN<8, 8>(__VA_ARGS__); break;                                \
    case 1604: FN<16, 4>(__VA_ARGS__); break;                              \
    case 1608: FN<16, 8>(__VA_ARGS__); break;                              \
    default: FN<16, 16>(__VA_ARGS__); break;                               \
  }

template <int W, int MW>
static void do_expand(const DevNet &net, const DevLevel &L, hipStream_t s) {
  const int64_t blocks = (L.nparents + 255) / 256;
  hipLaunchKernelGGL((expand_kernel<W, MW>), dim3((unsigned)blocks), dim3(256), 0, s, net, L);
}
hipError_t launch_expand(const DevNet &net, const DevLevel &L, hipStream_t s) {
  if (L.nparents <= 0) return hipSuccess;
  EFM_DISPATCH_WM(net.Wt, net.MWt, do_expand, net, L, s);
  return hipGetLastError();
}

template <int W, int MW>
static void do_rank_parent(const DevNet &net, const DevLevel &L, int prune, hipStream_t s) {
  hipLaunchKernelGGL((rank_parent_kernel<W, MW>), dim3((unsigned)(num_cus() * 16)), dim3(256), 0, s, net, L, prune);
}
hipError_t launch_rank_parent(const DevNet &net, const DevLevel &L, int prune, hipStream_t s) {
  EFM_DISPATCH_WM(net.Wt, net.MWt, do_rank_parent, net, L, prune, s);
  return hipGetLastError();
}

template <int W, int MW>
static void do_rank(const DevNet &net, const DevLevel &L, int prune, hipStream_t s) {
  const int kq_max = L.level + 1;
  const int wpb = 4;
  const size_t lds = 0;
  hipLaunchKernelGGL((rank_kernel<W, MW>), dim3((unsigned)(num_cus() * 16)), dim3(64 * wpb), lds, s, net, L,
                     prune, kq_max);
}
hipError_t launch_rank(const DevNet &net, const DevLevel &L, int prune, hipStream_t s) {
  EFM_DISPATCH_WM(net.Wt, net.MWt, do_rank, net, L, prune, s);
  return hipGetLastError();
}

template <int W, int MW>
static void do_exact(const DevNet &net, const DevLevel &L, hipStream_t s) {
  hipLaunchKernelGGL((exact_kernel<W, MW>), dim3((unsigned)L.xwaves), dim3(64), 0, s, net, L);
}
hipError_t launch_exact(const DevNet &net, const DevLevel &L, hipStream_t s) {
  EFM_DISPATCH_WM(net.Wt, net.MWt, do_exact, net, L, s);
  return hipGetLastError();
}

template <int W>
static void do_materialize(const DevNet &net, const DevLevel &L, int use_sel, hipStream_t s) {
  hipLaunchKernelGGL((materialize_kernel<W>), dim3((unsigned)(num_cus() * 8)), dim3(256), 0, s, net, L, use_sel);
}
hipError_t launch_materialize(const DevNet &net, const DevLevel &L, int use_sel, hipStream_t s) {
  EFM_DISPATCH_W(net.Wt, do_materialize, net, L, use_sel, s);
  return hipGetLastError();
}

template <int W>
static void do_hist(const DevLevel &L, int byte, int refill, int pass, hipStream_t s) {
  hipLaunchKernelGGL((select_hist_kernel<W>), dim3((unsigned)(num_cus() * 4)), dim3(256), 0, s, L, byte, refill,
                     pass);
}
hipError_t launch_select_hist(const DevNet &net, const DevLevel &L, int byte, int refill, int pass,
                              hipStream_t s) {
  EFM_DISPATCH_W(net.Wt, do_hist, L, byte, refill, pass, s);
  return hipGetLastError();
}

template <int W>
static void do_split(const DevLevel &L, int byte, int pass, hipStream_t s) {
  hipLaunchKernelGGL((select_split_kernel<W>), dim3((unsigned)(num_cus() * 4)), dim3(256), 0, s, L, byte, pass);
}
hipError_t launch_select_split(const DevNet &net, const DevLevel &L, int byte, int pass, hipStream_t s) {
  EFM_DISPATCH_W(net.Wt, do_split, L, byte, pass, s);
  return hipGetLastError();
}

hipError_t launch_clear(u64 *p, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > (size_t)num_cus() * 16) blocks = (size_t)num_cus() * 16;
  hipLaunchKernelGGL(clear_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace efm

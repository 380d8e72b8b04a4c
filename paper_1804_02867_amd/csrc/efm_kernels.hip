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

DEVI int wave_max_int(int v) {
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
  return v;
}

DEVI u64 wave_or(u64 v) {
  for (int off = 32; off > 0; off >>= 1) v |= __shfl_xor(v, off);
  return v;
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
  atomicOr(&L.counters[kFlags], (u64)kFlagUniqueOverflow);
  return false;
}

template <int W, int MW>
__global__ __launch_bounds__(256) void expand_kernel(DevNet net, DevLevel L) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = p < L.nparents;
  const u64 tag = (u64)(L.level % 127) + 1;
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
    wave_append(uniq && !rc && keep_indep, L.surv, &L.counters[kSurv], ref, L.ucap,
                &L.counters[kFlags]);
    wave_append(uniq && rc, L.rankq, &L.counters[kRankQ], ref, L.ucap, &L.counters[kFlags]);
    wave_count(uniq, &L.counters[kUnique]);
    wave_count(uniq && !rc, &L.counters[kIndep]);
    if (__ballot(uniq && !rc && !keep_indep) != 0 && lane_id() == 0)
      atomicOr(&L.counters[kFlags], (u64)kFlagDepthCapped);
  }
  // generated children
  int tot = ncand;
  for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off);
  if (lane_id() == 0 && tot) atomicAdd(&L.counters[kChildren], (u64)tot);
}

// -------------------------------------------------------------------------- rank
// One wave per row-closed child Q = P | e_r.  Lane j holds column j (the j-th
// reaction of Q).  Rows (the internal metabolites P touches) stream through a
// basis kept in LDS in reduced form; the child is independent once the basis has
// |Q| rows.
template <int W, int MW>
__global__ __launch_bounds__(256) void rank_kernel(DevNet net, DevLevel L, int prune, int kq_max) {
  extern __shared__ uint32_t lds[];
  const int wib = threadIdx.x >> 6;
  const int lane = lane_id();
  const int wpb = blockDim.x >> 6;
  uint32_t *basis = lds + (size_t)wib * kq_max * 64;
  const int64_t nitems = min((int64_t)L.counters[kRankQ], L.ucap);
  const bool keep_indep = L.level + 1 < L.depth_cap;
  const int64_t nf = min((int64_t)L.nfound_prev, L.ecap);

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
        if (lane == 0) atomicAdd(&L.counters[kPruned], 1ull);
        continue;
      }
    }

    int kq = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) kq += __popcll(Q[w]);
    const int col = lane < kq ? select_bit<W>(Q, lane) : -1;
    u64 T[MW];
#pragma unroll
    for (int q = 0; q < MW; ++q) T[q] = wave_or(col >= 0 ? net.rxn_touchM[(int64_t)col * MW + q] : 0ull);

    int nb = 0;
    int pcreg = 0;                 // lane b holds the pivot column of basis row b
    bool indep = false;
    if (!L.debug_prime) {
#pragma unroll
      for (int q = 0; q < MW; ++q) {
        u64 bits = T[q];
        while (bits && !indep) {
          const int i = q * 64 + __builtin_ctzll(bits);
          bits &= bits - 1;
          uint32_t x = col >= 0 ? tomod(net.Sint[(int64_t)i * net.n + col]) : 0u;
          for (int b = 0; b < nb; ++b) {
            const uint32_t f = __shfl(x, __shfl(pcreg, b));
            if (f) x = submod(x, mulmod(f, basis[b * 64 + lane]));
          }
          const u64 nz = __ballot(x != 0);
          if (nz) {
            const int pc = __ffsll((long long)nz) - 1;
            const uint32_t inv = powmod(__shfl(x, pc), kPrime - 2);
            basis[nb * 64 + lane] = mulmod(x, inv);
            if (lane == nb) pcreg = pc;
            nb++;
            if (nb == kq) indep = true;
          }
        }
      }
    }
    if (indep) {
      if (lane == 0) {
        atomicAdd(&L.counters[kIndep], 1ull);
        if (keep_indep) {
          const u64 idx = atomicAdd(&L.counters[kSurv], 1ull);
          if ((int64_t)idx < L.ucap) L.surv[idx] = ref;
          else atomicOr(&L.counters[kFlags], (u64)kFlagQueueOverflow);
        } else {
          atomicOr(&L.counters[kFlags], (u64)kFlagDepthCapped);
        }
      }
    } else if (lane == 0) {
      const u64 idx = atomicAdd(&L.counters[kExactQ], 1ull);
      if ((int64_t)idx < L.ucap) L.exactq[idx] = ref;
      else atomicOr(&L.counters[kFlags], (u64)kFlagQueueOverflow);
    }
  }
}

// ------------------------------------------------------------------------- exact
// One wave per child.  Lane j owns column j of the dense matrix S_int[T, Q] kept in
// global scratch (row-major, 64 entries per row); entries of other columns travel
// by lane shuffles only.
template <int W, int MW>
__global__ __launch_bounds__(64) void exact_kernel(DevNet net, DevLevel L) {
  const int lane = lane_id();
  const int64_t nitems = min((int64_t)L.counters[kExactQ], L.ucap);
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
      if (lane == 0) atomicOr(&L.counters[kFlags], (u64)kFlagIntOverflow);
      continue;
    }
    if (rank == kq) {                      // the modular test was fooled: independent
      if (lane == 0) {
        atomicAdd(&L.counters[kIndep], 1ull);
        if (keep_indep) {
          const u64 idx = atomicAdd(&L.counters[kSurv], 1ull);
          if ((int64_t)idx < L.ucap) L.surv[idx] = ref;
          else atomicOr(&L.counters[kFlags], (u64)kFlagQueueOverflow);
        } else {
          atomicOr(&L.counters[kFlags], (u64)kFlagDepthCapped);
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
      if (lane == 0) atomicOr(&L.counters[kFlags], (u64)kFlagIntOverflow);
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
      if (lane == 0) atomicOr(&L.counters[kFlags], (u64)kFlagIntOverflow);
      continue;
    }
    u64 slot = 0;
    if (lane == 0) slot = atomicAdd(&L.counters[kFound], 1ull);
    slot = __shfl(slot, 0);
    if ((int64_t)slot >= L.ecap) {
      if (lane == 0) atomicOr(&L.counters[kFlags], (u64)kFlagFoundOverflow);
      continue;
    }
#pragma unroll
    for (int w = 0; w < W; ++w)
      if (lane == w) L.fkeys[(int64_t)w * L.ecap + slot] = Q[w];
    if (mine) L.fflux[(int64_t)slot * kMaxDepth + lane] = (int64_t)v;
    if (lane == 0) atomicAdd(&L.counters[kEmitted], 1ull);
  }
}

// ------------------------------------------------------------- truncation select
template <int W>
DEVI uint32_t key_byte(const DevLevel &L, u64 ref, int byte) {
  const u64 p = ref >> 12;
  const int r = (int)((ref >> 1) & 0x7FF);
  const int w = byte >> 3;
  u64 kw = L.keys[(int64_t)w * L.fcap + p] | ((r >> 6) == w ? (1ull << (r & 63)) : 0ull);
  return (uint32_t)((kw >> ((byte & 7) * 8)) & 0xFF);
}

template <int W>
__global__ __launch_bounds__(256) void select_hist_kernel(DevLevel L, int byte, int first, int64_t nb) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t idx = first ? i : (int64_t)L.blist[i];
    atomicAdd(&h[key_byte<W>(L, L.surv[idx], byte)], 1u);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&L.hist[threadIdx.x], h[threadIdx.x]);
}

template <int W>
__global__ __launch_bounds__(256) void select_split_kernel(DevLevel L, int byte, int first, int64_t nb,
                                                           uint32_t digit, int all_sel) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t idx = first ? i : (int64_t)L.blist[i];
    const uint32_t d = key_byte<W>(L, L.surv[idx], byte);
    if (d < digit || (d == digit && all_sel)) {
      L.sel[idx] = 1;
    } else if (d == digit) {
      const u64 k = atomicAdd(&L.counters[kBoundary], 1ull);
      L.blist2[k] = (uint32_t)idx;
    }
  }
}

// ------------------------------------------------------------------ materialize
template <int W>
__global__ __launch_bounds__(256) void materialize_kernel(DevNet net, DevLevel L, int use_sel) {
  const int64_t n = min((int64_t)L.counters[kSurv], L.ucap);
  const int lane = lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t base = wave * 64; base < n; base += nwaves * 64) {
    const int64_t idx = base + lane;
    const bool act = idx < n && (!use_sel || L.sel[idx] == 1);
    u64 ref = act ? L.surv[idx] : 0ull;
    const u64 mask = __ballot(act);
    if (mask == 0) continue;
    const int leader = __ffsll((long long)mask) - 1;
    u64 dst = 0;
    if (lane == leader) dst = atomicAdd(&L.counters[kNext], (u64)__popcll(mask));
    dst = __shfl(dst, leader) + (u64)__popcll(mask & lanes_below(lane));
    if (act) {
      const u64 p = ref >> 12;
      const int r = (int)((ref >> 1) & 0x7FF);
#pragma unroll
      for (int w = 0; w < W; ++w)
        L.nkeys[(int64_t)w * L.fcap + dst] =
            L.keys[(int64_t)w * L.fcap + p] | ((r >> 6) == w ? (1ull << (r & 63)) : 0ull);
      L.nhash[dst] = L.hash[p] ^ net.zob[r];
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
static void do_rank(const DevNet &net, const DevLevel &L, int prune, hipStream_t s) {
  const int kq_max = L.level + 1;
  const int wpb = 4;
  const size_t lds = (size_t)wpb * kq_max * 64 * sizeof(uint32_t);
  hipLaunchKernelGGL((rank_kernel<W, MW>), dim3((unsigned)(num_cus() * 8)), dim3(64 * wpb), lds, s, net, L,
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
static void do_hist(const DevLevel &L, int byte, int first, int64_t nb, hipStream_t s) {
  hipLaunchKernelGGL((select_hist_kernel<W>), dim3((unsigned)(num_cus() * 4)), dim3(256), 0, s, L, byte, first, nb);
}
hipError_t launch_select_hist(const DevNet &net, const DevLevel &L, int byte, int first, int64_t nb,
                              hipStream_t s) {
  EFM_DISPATCH_W(net.Wt, do_hist, L, byte, first, nb, s);
  return hipGetLastError();
}

template <int W>
static void do_split(const DevLevel &L, int byte, int first, int64_t nb, uint32_t digit, int all_sel,
                     hipStream_t s) {
  hipLaunchKernelGGL((select_split_kernel<W>), dim3((unsigned)(num_cus() * 4)), dim3(256), 0, s, L, byte, first,
                     nb, digit, all_sel);
}
hipError_t launch_select_split(const DevNet &net, const DevLevel &L, int byte, int first, int64_t nb,
                               uint32_t digit, int all_sel, hipStream_t s) {
  EFM_DISPATCH_W(net.Wt, do_split, L, byte, first, nb, digit, all_sel, s);
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

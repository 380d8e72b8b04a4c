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
#include "efm_wave.h"

namespace efm {

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
  const u64 max_probe = L.tmask < kMaxProbe ? L.tmask + 1 : kMaxProbe;
  for (u64 probe = 0; probe < max_probe; ++probe) {
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
  constexpr int kExpandBuf = 512;      // most waves flush once, at the end
  __shared__ u64 stage[4][kExpandBuf];
  const int wib = threadIdx.x >> 6;
  WaveBuf bsurv{stage[wib], 0, kExpandBuf};
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
  wbuf_flush_block(bsurv, L.surv, &L.counters[cslot(kSurv)], L.ucap, &L.counters[cslot(kFlags)]);
  {
    // one rank-queue entry per parent that has row-closed children
    bool any = false;
#pragma unroll
    for (int w = 0; w < W; ++w) any = any || rcm[w] != 0;
    const u64 idx = block_append_index(any, &L.counters[cslot(kParQ)]);
    if (any) {
      if ((int64_t)idx < L.fcap) {             // one entry per parent: at most the frontier capacity
        L.parq[idx] = (u64)p;
#pragma unroll
        for (int w = 0; w < W; ++w) L.parmask[(int64_t)idx * W + w] = rcm[w];
      } else {
        atomicOr(&L.counters[cslot(kFlags)], (u64)kFlagQueueOverflow);
      }
    }
  }
  u64 v[5] = {(u64)ncand, n_unique, n_indep, n_capped, n_rc};
  const int slots[5] = {kChildren, kUnique, kIndep, kCapped, kRowClosed};
  block_counts<5>(v, L.counters, slots);
}

// ------------------------------------------------------------------- rank (parent)
// One wave per parent P with its distinct row-closed children r_1..r_m.  Every
// child's rows lie inside P's rows.  Lane j holds column j of P | {r_1..r_m} (in
// reaction order) as the mask of its odd coefficients over the internal
// metabolites; column elimination modulo 2 by P's columns leaves each child's
// column reduced against P, so a child is certified independent exactly when its
// reduced column is nonzero.  Independence modulo 2 implies independence over the
// rationals.  Children not certified (or pruned by the found set) go on to the
// per-child test.  Two parents of at most 32 columns each share one wave, one per
// half.
struct RankCounts {
  u64 indep = 0, pruned = 0, capped = 0, rows = 0;
};

template <int W, int MW>
DEVI void rank_parent_one(const DevNet &net, const DevLevel &L, int64_t item, int prune, int64_t nf,
                          bool keep_indep, uint16_t *colx, WaveBuf &bsurv, WaveBuf &bslow, RankCounts &cnt) {
  const int lane = lane_id();
  u64 &n_indep = cnt.indep, &n_pruned = cnt.pruned, &n_capped = cnt.capped, &n_rows = cnt.rows;
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
    int kp = 0, nch = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      A[w] = P[w] | M[w];                        // pruned children are gone from M
      kall += __popcll(A[w]);
      kp += __popcll(P[w]);
      nch += __popcll(M[w]);
    }
    const bool full = kall <= 64 && !L.debug_prime && !L.no_gf2;
    int rows = 0;            // rows the children's tests span: the parent's touched metabolites
    if (full) {
      // one column per lane, in reaction order: lane j holds the j-th reaction of
      // P | children (compacted through LDS), as its odd-coefficient mask over the
      // internal metabolites (S mod 2)
      {
        int base = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
          if ((A[w] >> lane) & 1ull) colx[base + __popcll(A[w] & lanes_below(lane))] = (uint16_t)(w * 64 + lane);
          base += __popcll(A[w]);
        }
      }
      __threadfence_block();
      const int col = lane < kall ? (int)colx[lane] : -1;
      bool child = false;
#pragma unroll
      for (int w = 0; w < W; ++w)
        if (col >= 0 && (col >> 6) == w) child = (M[w] >> (col & 63)) & 1ull;
      u64 v[MW];
#pragma unroll
      for (int q = 0; q < MW; ++q) {
        v[q] = col >= 0 ? net.rxn_oddM[(int64_t)col * MW + q] : 0ull;
        rows += __popcll(wave_or((col >= 0 && !child) ? net.rxn_touchM[(int64_t)col * MW + q] : 0ull));
      }
      // column elimination modulo 2 by the parent's columns, in order: each reduced
      // parent column gives a pivot row (its lowest set bit) that is cleared from
      // every other column; pivots of later columns never set an earlier pivot row
      u64 pcols = __ballot(col >= 0 && !child);
      bool ok = true;
      while (pcols) {
        const int j = __ffsll((long long)pcols) - 1;
        pcols &= pcols - 1;
        u64 pv[MW];
        int pq = -1;
#pragma unroll
        for (int q = 0; q < MW; ++q) {
          pv[q] = readlane64(v[q], j);
          if (pq < 0 && pv[q] != 0) pq = q;
        }
        if (pq < 0) { ok = false; break; }    // the parent is dependent modulo 2: no certificate
        int b = 0;
        u64 vq = 0;
#pragma unroll
        for (int q = 0; q < MW; ++q)
          if (q == pq) { b = __builtin_ctzll(pv[q]); vq = v[q]; }
        if (lane != j && ((vq >> b) & 1ull)) {
#pragma unroll
          for (int q = 0; q < MW; ++q) v[q] ^= pv[q];
        }
      }
      // a child whose reduced column is nonzero is outside the parent's span
      // modulo 2, hence independent over the rationals
      bool nz = false;
#pragma unroll
      for (int q = 0; q < MW; ++q) nz = nz || v[q] != 0;
      const bool cert = ok && child && nz;
      const u64 ref = ((u64)p << 12) | ((u64)(col < 0 ? 0 : col) << 1) | 1ull;
      const u64 cm = __ballot(cert);
      if (lane == 0) {
        n_indep += __popcll(cm);
        n_capped += keep_indep ? 0 : __popcll(cm);
      }
      wbuf_push(bsurv, cert && keep_indep, ref, L.surv, &L.counters[cslot(kSurv)], L.ucap,
                &L.counters[cslot(kFlags)]);
      wbuf_push(bslow, child && !cert, ref, L.rankq, &L.counters[cslot(kRankQ)], L.ucap,
                &L.counters[cslot(kFlags)]);
      __threadfence_block();
    } else {
      // no certificate (too many columns, or disabled): every child is tested
      for (int c0 = 0; c0 < kp; c0 += 64) {
        const int pc = c0 + lane < kp ? select_bit<W>(P, c0 + lane) : -1;
#pragma unroll
        for (int q = 0; q < MW; ++q) rows += __popcll(wave_or(pc >= 0 ? net.rxn_touchM[(int64_t)pc * MW + q] : 0ull));
      }
#pragma unroll
      for (int w = 0; w < W; ++w) {
        u64 bits = M[w];
        while (bits) {
          const int r = w * 64 + __builtin_ctzll(bits);
          bits &= bits - 1;
          const u64 ref = (p << 12) | ((u64)r << 1) | 1ull;
          wbuf_push(bslow, lane == 0, ref, L.rankq, &L.counters[cslot(kRankQ)], L.ucap,
                    &L.counters[cslot(kFlags)]);
        }
      }
    }
    n_rows += lane == 0 ? (u64)rows * (u64)nch : 0ull;
}

// two parents, one per half-wave (both of at most 32 columns, no found-set prune)
template <int W, int MW>
DEVI void rank_parent_two(const DevNet &net, const DevLevel &L, int64_t i0, int64_t i1, bool keep_indep,
                          uint16_t *colx, WaveBuf &bsurv, WaveBuf &bslow, RankCounts &cnt) {
  const int lane = lane_id();
  const int h = lane >> 5, hl = lane & 31;
  const int64_t item = h ? i1 : i0;
  const u64 p = L.parq[item];
  u64 P[W], M[W], A[W];
  int kall = 0, nch = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    P[w] = L.keys[(int64_t)w * L.fcap + p];
    M[w] = L.parmask[item * W + w];
    A[w] = P[w] | M[w];
    kall += __popcll(A[w]);
    nch += __popcll(M[w]);
  }
  // columns of this half's parent, in reaction order, into colx[32h ..]
  {
    int base = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
#pragma unroll
      for (int sub = 0; sub < 2; ++sub) {
        const int b = hl + 32 * sub;
        if ((A[w] >> b) & 1ull) colx[32 * h + base + __popcll(A[w] & ((1ull << b) - 1ull))] = (uint16_t)(w * 64 + b);
      }
      base += __popcll(A[w]);
    }
  }
  __threadfence_block();
  const int col = hl < kall ? (int)colx[32 * h + hl] : -1;
  bool child = false;
#pragma unroll
  for (int w = 0; w < W; ++w)
    if (col >= 0 && (col >> 6) == w) child = (M[w] >> (col & 63)) & 1ull;
  u64 v[MW];
  int rows = 0;
#pragma unroll
  for (int q = 0; q < MW; ++q) {
    v[q] = col >= 0 ? net.rxn_oddM[(int64_t)col * MW + q] : 0ull;
    u64 t = (col >= 0 && !child) ? net.rxn_touchM[(int64_t)col * MW + q] : 0ull;
    for (int off = 16; off > 0; off >>= 1) t |= __shfl_xor(t, off);     // OR within the half
    rows += __popcll(t);
  }
  const u64 pc = __ballot(col >= 0 && !child);
  u64 pa = pc & 0xFFFFFFFFull, pb = pc >> 32;
  bool ok = true;
  while (pa | pb) {
    const int ja = pa ? __ffsll((long long)pa) - 1 : -1;
    const int jb = pb ? 32 + __ffsll((long long)pb) - 1 : -1;
    if (pa) pa &= pa - 1;
    if (pb) pb &= pb - 1;
    const int j = h ? jb : ja;
    const int src = j >= 0 ? j : lane;
    u64 pv[MW];
    int pq = -1;
#pragma unroll
    for (int q = 0; q < MW; ++q) {
      const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v[q], src);
      const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v[q] >> 32), src);
      pv[q] = ((u64)hi << 32) | lo;
      if (pq < 0 && pv[q] != 0) pq = q;
    }
    if (j < 0 || !ok) continue;               // this half is done (or has no certificate)
    if (pq < 0) { ok = false; continue; }     // its parent is dependent modulo 2
    int b = 0;
    u64 vq = 0;
#pragma unroll
    for (int q = 0; q < MW; ++q)
      if (q == pq) { b = __builtin_ctzll(pv[q]); vq = v[q]; }
    if (lane != j && ((vq >> b) & 1ull)) {
#pragma unroll
      for (int q = 0; q < MW; ++q) v[q] ^= pv[q];
    }
  }
  bool nz = false;
#pragma unroll
  for (int q = 0; q < MW; ++q) nz = nz || v[q] != 0;
  const bool cert = ok && child && nz;
  const u64 ref = (p << 12) | ((u64)(col < 0 ? 0 : col) << 1) | 1ull;
  const u64 cm = __ballot(cert);
  if (lane == 0) {
    cnt.indep += __popcll(cm);
    cnt.capped += keep_indep ? 0 : __popcll(cm);
  }
  if (hl == 0) cnt.rows += (u64)rows * (u64)nch;
  wbuf_push(bsurv, cert && keep_indep, ref, L.surv, &L.counters[cslot(kSurv)], L.ucap, &L.counters[cslot(kFlags)]);
  wbuf_push(bslow, child && !cert, ref, L.rankq, &L.counters[cslot(kRankQ)], L.ucap, &L.counters[cslot(kFlags)]);
  __threadfence_block();
}

template <int W, int MW>
__global__ __launch_bounds__(256) void rank_parent_kernel(DevNet net, DevLevel L, int prune) {
  constexpr int kRankBuf = 256;
  __shared__ u64 stage[2][4][kRankBuf];
  __shared__ uint16_t colx[4][64];
  const int wib = threadIdx.x >> 6;
  const int wpb = blockDim.x >> 6;
  const int64_t nitems = min((int64_t)L.counters[cslot(kParQ)], L.fcap);
  const bool keep_indep = L.level + 1 < L.depth_cap;
  const int64_t nf = min((int64_t)L.nfound_prev, L.ecap);
  const bool pairs_ok = !(prune && nf > 0) && !L.debug_prime && !L.no_gf2;
  WaveBuf bsurv{stage[0][wib], 0, kRankBuf}, bslow{stage[1][wib], 0, kRankBuf};
  RankCounts cnt;

  // items in pairs: two narrow parents share the wave, otherwise one at a time
  for (int64_t pr = (int64_t)blockIdx.x * wpb + wib; 2 * pr < nitems; pr += (int64_t)gridDim.x * wpb) {
    const int64_t i0 = 2 * pr, i1 = i0 + 1;
    bool two = pairs_ok && i1 < nitems;
    if (two) {
      int k0 = 0, k1 = 0;
      const u64 p0 = L.parq[i0], p1 = L.parq[i1];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        k0 += __popcll(L.keys[(int64_t)w * L.fcap + p0] | L.parmask[i0 * W + w]);
        k1 += __popcll(L.keys[(int64_t)w * L.fcap + p1] | L.parmask[i1 * W + w]);
      }
      two = k0 <= 32 && k1 <= 32;
    }
    if (two) {
      rank_parent_two<W, MW>(net, L, i0, i1, keep_indep, colx[wib], bsurv, bslow, cnt);
    } else {
      rank_parent_one<W, MW>(net, L, i0, prune, nf, keep_indep, colx[wib], bsurv, bslow, cnt);
      if (i1 < nitems) rank_parent_one<W, MW>(net, L, i1, prune, nf, keep_indep, colx[wib], bsurv, bslow, cnt);
    }
  }
  wbuf_flush_block(bsurv, L.surv, &L.counters[cslot(kSurv)], L.ucap, &L.counters[cslot(kFlags)]);
  wbuf_flush_block(bslow, L.rankq, &L.counters[cslot(kRankQ)], L.ucap, &L.counters[cslot(kFlags)]);
  u64 v[4] = {cnt.indep, cnt.pruned, cnt.capped, cnt.rows};
  const int slots[4] = {kIndep, kPruned, kCapped, kRankRows};
  block_counts<4>(v, L.counters, slots);
}

// -------------------------------------------------------------------------- rank
// One wave per row-closed child Q = P | e_r.  Lane j holds column j (the j-th
// reaction of Q) as its few nonzero entries in registers.  Singleton rows are
// peeled first; the remaining rows then stream through a basis kept in LDS in
// reduced form, and the child is independent once the basis has as many rows as
// there are unpeeled columns.
template <int W, int MW>
__global__ __launch_bounds__(256) void rank_kernel(DevNet net, DevLevel L, int prune, int kq_max) {
  constexpr int kRankBuf = 256;
  __shared__ u64 stage[2][4][kRankBuf];
  const int wib = threadIdx.x >> 6;
  const int lane = lane_id();
  const int wpb = blockDim.x >> 6;
  const int64_t nitems = min((int64_t)L.counters[cslot(kRankQ)], L.ucap);
  const bool keep_indep = L.level + 1 < L.depth_cap;
  const int64_t nf = min((int64_t)L.nfound_prev, L.ecap);
  WaveBuf bsurv{stage[0][wib], 0, kRankBuf}, bexact{stage[1][wib], 0, kRankBuf};
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

    const bool indep = L.debug_prime ? false : wave_rank_child<W, MW>(net, Q, r, L.no_gf2 != 0);
    n_indep += (indep && lane == 0) ? 1 : 0;
    n_capped += (indep && !keep_indep && lane == 0) ? 1 : 0;
    wbuf_push(bsurv, indep && keep_indep && lane == 0, ref, L.surv, &L.counters[cslot(kSurv)], L.ucap,
              &L.counters[cslot(kFlags)]);
    wbuf_push(bexact, !indep && lane == 0, ref, L.exactq, &L.counters[cslot(kExactQ)], L.ucap,
              &L.counters[cslot(kFlags)]);
  }
  wbuf_flush_block(bsurv, L.surv, &L.counters[cslot(kSurv)], L.ucap, &L.counters[cslot(kFlags)]);
  wbuf_flush_block(bexact, L.exactq, &L.counters[cslot(kExactQ)], L.ucap, &L.counters[cslot(kFlags)]);
  u64 v[3] = {n_indep, n_pruned, n_capped};
  const int slots[3] = {kIndep, kPruned, kCapped};
  block_counts<3>(v, L.counters, slots);
}

// ------------------------------------------------------------------------- exact
template <int W, int MW>
__global__ __launch_bounds__(64) void exact_kernel(DevNet net, DevLevel L) {
  __shared__ uint32_t Bl[kMaxDepth * 64];
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
    int64_t vout = 0;
    const int outcome = wave_exact_child<W, MW>(net, Q, L.Sx, M, Bl, vout, L.debug_prime != 0);
    if (outcome == kExactOverflow) {
      if (lane == 0) atomicOr(&L.counters[cslot(kFlags)], (u64)kFlagIntOverflow);
      continue;
    }
    if (outcome == kExactIndependent) {
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
    if (outcome != kExactEmit) continue;
    int kq = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) kq += __popcll(Q[w]);
    const bool mine = lane < kq;
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
    if (mine) L.fflux[(int64_t)slot * kMaxDepth + lane] = vout;
    if (lane == 0) atomicAdd(&L.counters[cslot(kEmitted)], 1ull);
  }
}

// ------------------------------------------------------------- truncation select

// Radix selection of the frontier cap's smallest keys, one key byte per pass from
// the most significant.  sel[i] is 2 while survivor i is undecided, then 1
// (selected) or 0 (rejected).  skey caches the key word the current byte lies in
// as eight byte planes (plane b, member i at b * sel_stride + i), refilled when a
// pass enters a new word, so that a pass reads only the bytes it compares.  Each
// lane takes four consecutive members with 32-bit loads of sel and the planes.
template <int W>
DEVI u64 key_word(const DevLevel &L, u64 ref, int w) {
  const u64 p = ref >> 12;
  const int r = (int)((ref >> 1) & 0x7FF);
  return L.keys[(int64_t)w * L.fcap + p] | ((r >> 6) == w ? (1ull << (r & 63)) : 0ull);
}

DEVI uint32_t ld32(const uint8_t *p) { return *(const uint32_t *)p; }
DEVI void st32(uint8_t *p, uint32_t v) { *(uint32_t *)p = v; }
DEVI uint32_t byte_of(uint32_t v, int k) { return (v >> (8 * k)) & 0xFFu; }

// Members i0..i0+3 flagged in act4 (bit k): load the key word of `byte` (or the
// learned score word), store its eight byte planes and return the digits of `byte`.
template <int W>
DEVI void refill4(const DevLevel &L, int64_t i0, uint32_t act4, int byte, uint32_t (&d)[4]) {
  const int64_t ps = sel_stride(L.ucap);
  const int shift = (byte & 7) * 8;
  uint32_t pw[8];
#pragma unroll
  for (int b = 0; b < 8; ++b) pw[b] = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if ((act4 >> k) & 1u) {
      const int64_t i = i0 + k;
      const u64 kw = (byte >> 3) >= W ? (u64)L.sscore[i] : key_word<W>(L, L.surv[i], byte >> 3);
#pragma unroll
      for (int b = 0; b < 8; ++b) pw[b] |= (uint32_t)((kw >> (8 * b)) & 0xFF) << (8 * k);
      d[k] = (uint32_t)((kw >> shift) & 0xFF);
    }
  }
  if (act4) {
#pragma unroll
    for (int b = 0; b < 8; ++b) st32(L.skey + b * ps + i0, pw[b]);
  }
}

// bit k set when member i0+k exists and is undecided
DEVI uint32_t undecided4(uint32_t s4, int64_t i0, int64_t n) {
  uint32_t a = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) a |= (i0 + k < n && byte_of(s4, k) == 2u) ? (1u << k) : 0u;
  return a;
}

// Histogram of the undecided members' digits for pass `pass` (state and histogram
// are double-buffered by pass parity).  Digits are highly skewed (the top bytes
// of nearly all keys agree), so each wave adds its lanes in groups of equal
// digits (wave_hist_add).
// Adds the wave's active digits to an LDS histogram: lanes that share a digit
// with the first or second pending lane add as one group (the common case, since
// most keys agree on most bytes); any other lane adds its own count.
DEVI void wave_hist_add(uint32_t *h, bool act, uint32_t d) {
  u64 pending = __ballot(act);
  const int lane = lane_id();
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    if (!pending) return;
    const uint32_t v = (uint32_t)__builtin_amdgcn_readlane((int)d, __ffsll((long long)pending) - 1);
    const u64 m = __ballot(act && d == v) & pending;
    if (lane == __ffsll((long long)m) - 1) atomicAdd(&h[v], (uint32_t)__popcll(m));
    pending &= ~m;
  }
  if ((pending >> lane) & 1ull) atomicAdd(&h[d], 1u);
}

// Boundary digit of a finished 256-bin histogram: the first v (at most 255)
// whose inclusive prefix sum reaches `needed`, the count below it and its own
// count.  Every thread of the 256-thread block calls it (block-wide scan in LDS).
DEVI void hist_boundary(const uint32_t *hist, int64_t needed, int &v, int64_t &cum, int64_t &hv) {
  __shared__ int64_t sc[256];
  __shared__ int64_t bin[256];
  __shared__ int vsel;
  const int t = threadIdx.x;
  int64_t c = 0;
#pragma unroll
  for (int k = 0; k < kHistCopies; ++k) c += hist[k * 256 + t];
  sc[t] = c;
  bin[t] = c;
  if (t == 0) vsel = 255;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int64_t add = t >= off ? sc[t - off] : 0;
    __syncthreads();
    sc[t] += add;
    __syncthreads();
  }
  if (t < 255 && sc[t] >= needed) atomicMin(&vsel, t);
  __syncthreads();
  v = vsel;
  hv = bin[v];
  cum = sc[v] - hv;
}

template <int W>
__global__ __launch_bounds__(256) void select_hist_kernel(DevLevel L, int byte, int refill, int pass) {
  __shared__ uint32_t h[256];
  const SelState *st = L.selst + (pass & 1);
  if (st->done) return;
  uint32_t *hist = L.hist + kHistCopies * 256 * (pass % 3);
  const int64_t n = min((int64_t)L.counters[cslot(kSurv)], L.ucap);
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t ps = sel_stride(L.ucap);
  const int lane = lane_id();
  const int64_t ng = (n + 3) >> 2;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t base = wave * 64; base < ng; base += nwaves * 64) {
    const int64_t g = base + lane;
    const int64_t i0 = g * 4;
    uint32_t s4 = 0, c4 = 0;
    if (g < ng) {
      s4 = ld32(L.sel + i0);
      if (!refill) c4 = ld32(L.skey + (byte & 7) * ps + i0);
    }
    const uint32_t act4 = g < ng ? undecided4(s4, i0, n) : 0u;
    if (__ballot(act4 != 0) == 0) continue;
    uint32_t d[4] = {byte_of(c4, 0), byte_of(c4, 1), byte_of(c4, 2), byte_of(c4, 3)};
    if (refill) refill4<W>(L, i0, act4, byte, d);
#pragma unroll
    for (int k = 0; k < 4; ++k) wave_hist_add(h, (act4 >> k) & 1u, d[k]);
  }
  (void)lane;
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&hist[(blockIdx.x % kHistCopies) * 256 + threadIdx.x], h[threadIdx.x]);
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
  const uint32_t *hist = L.hist + kHistCopies * 256 * (pass % 3);
  const bool lead = blockIdx.x == 0;
  if (lead)
    for (int k = 0; k < kHistCopies; ++k) L.hist[kHistCopies * 256 * ((pass + 1) % 3) + k * 256 + threadIdx.x] = 0;
  if (st->done) {
    if (lead && threadIdx.x == 0) *nx = *st;
    return;
  }
  int v;
  int64_t cum, hv;
  hist_boundary(hist, st->needed, v, cum, hv);
  if (threadIdx.x == 0) {
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
  const bool all_sel = dec[1] != 0;
  const int64_t ps = sel_stride(L.ucap);
  const int64_t n = min((int64_t)L.counters[cslot(kSurv)], L.ucap);
  const int64_t ng = (n + 3) >> 2;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ng; g += stride) {
    const int64_t i0 = g * 4;
    const uint32_t s4 = ld32(L.sel + i0);
    const uint32_t c4 = ld32(L.skey + (byte & 7) * ps + i0);
    const uint32_t act4 = undecided4(s4, i0, n);
    if (!act4) continue;
    uint32_t o4 = s4;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (!((act4 >> k) & 1u)) continue;
      const uint32_t d = byte_of(c4, k);
      const uint32_t v = (d < digit || (d == digit && all_sel)) ? 1u : (d > digit ? 0u : 2u);
      o4 = (o4 & ~(0xFFu << (8 * k))) | (v << (8 * k));
    }
    if (o4 != s4) st32(L.sel + i0, o4);
  }
}

// One pass of the selection in one sweep: applies pass-1's decision (from its
// finished histogram, derived by every block as in select_split_kernel) and adds
// the digits of `byte` of the members still undecided to pass's histogram.
// Histograms are triple-buffered (pass % 3): block 0 clears the one for pass+1,
// which nobody reads or writes during this launch.
template <int W>
__global__ __launch_bounds__(256) void select_step_kernel(DevLevel L, int prev_byte, int byte, int refill, int pass) {
  __shared__ uint32_t dec[3];
  __shared__ int64_t rem;
  __shared__ uint32_t h[256];
  const SelState *st = L.selst + ((pass - 1) & 1);
  SelState *nx = L.selst + (pass & 1);
  const uint32_t *hprev = L.hist + kHistCopies * 256 * ((pass - 1) % 3);
  uint32_t *hcur = L.hist + kHistCopies * 256 * (pass % 3);
  const bool lead = blockIdx.x == 0;
  if (lead)
    for (int k = 0; k < kHistCopies; ++k) L.hist[kHistCopies * 256 * ((pass + 1) % 3) + k * 256 + threadIdx.x] = 0;
  if (st->done) {
    if (lead && threadIdx.x == 0) *nx = *st;
    return;
  }
  h[threadIdx.x] = 0;
  int v;
  int64_t cum, hv;
  hist_boundary(hprev, st->needed, v, cum, hv);
  if (threadIdx.x == 0) {
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
  const bool decides = !dec[2];
  const uint32_t digit = dec[0];
  const bool all_sel = dec[1] != 0;
  const int64_t ps = sel_stride(L.ucap);
  const int lane = lane_id();
  const int64_t n = min((int64_t)L.counters[cslot(kSurv)], L.ucap);
  const int64_t ng = (n + 3) >> 2;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t base = wave * 64; base < ng; base += nwaves * 64) {
    const int64_t g = base + lane;
    const int64_t i0 = g * 4;
    uint32_t s4 = 0, p4 = 0, c4 = 0;
    if (g < ng) {
      s4 = ld32(L.sel + i0);
      if (decides) p4 = ld32(L.skey + (prev_byte & 7) * ps + i0);
      if (!refill) c4 = ld32(L.skey + (byte & 7) * ps + i0);
    }
    uint32_t act4 = g < ng ? undecided4(s4, i0, n) : 0u;
    if (__ballot(act4 != 0) == 0) continue;
    if (decides && act4) {
      uint32_t o4 = s4;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (!((act4 >> k) & 1u)) continue;
        const uint32_t dp = byte_of(p4, k);
        if (dp < digit || (dp == digit && all_sel)) {
          o4 = (o4 & ~(0xFFu << (8 * k))) | (1u << (8 * k));
          act4 &= ~(1u << k);
        } else if (dp > digit) {
          o4 &= ~(0xFFu << (8 * k));
          act4 &= ~(1u << k);
        }
      }
      if (o4 != s4) st32(L.sel + i0, o4);
    }
    uint32_t d[4] = {byte_of(c4, 0), byte_of(c4, 1), byte_of(c4, 2), byte_of(c4, 3)};
    if (refill) refill4<W>(L, i0, act4, byte, d);
#pragma unroll
    for (int k = 0; k < 4; ++k) wave_hist_add(h, (act4 >> k) & 1u, d[k]);
  }
  (void)lane;
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&hcur[(blockIdx.x % kHistCopies) * 256 + threadIdx.x], h[threadIdx.x]);
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

template <int W>
static void do_step(const DevLevel &L, int prev_byte, int byte, int refill, int pass, hipStream_t s) {
  hipLaunchKernelGGL((select_step_kernel<W>), dim3((unsigned)(num_cus() * 4)), dim3(256), 0, s, L, prev_byte, byte,
                     refill, pass);
}
hipError_t launch_select_step(const DevNet &net, const DevLevel &L, int prev_byte, int byte, int refill, int pass,
                              hipStream_t s) {
  EFM_DISPATCH_W(net.Wt, do_step, L, prev_byte, byte, refill, pass, s);
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

// efm_wave.h -- wave-level decisions on one child pathway, shared by the level
// kernels and the batched engine: the rank test (peeling, GF(2) certificate,
// elimination modulo 2^31-1) and the exact 128-bit null-vector computation.
#pragma once
#include "efm_device.h"

namespace efm {

// Rank test of one child Q = P | e_r (P independent), by the whole wave: singleton
// peeling, the GF(2) certificate on the core, then elimination modulo 2^31-1.
// Returns true when Q is independent; false sends Q to exact arithmetic.
template <int W, int MW>
DEVI bool wave_rank_child(const DevNet &net, const u64 *Q, int r, bool no_gf2) {
  const int lane = lane_id();
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
    if (!false && !no_gf2 && r_alive && nrows >= ncore) {
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
    if (!false && r_alive && nrows >= ncore && !indep) {
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
  return indep;
}

// Exact decision for a child Q that the modular test called dependent, by the
// whole wave.  The modular lift above is tried first (unless bareiss_only); the
// 128-bit elimination below decides what it cannot.  Lane j owns column j of the dense matrix S_int[rows of Q, Q] kept in
// scratch M (row-major, 64 entries per row); entries of other columns travel by
// lane shuffles only.  On kExactEmit, vout holds (in lane j) the primitive flux of
// the j-th reaction of Q, signed as Definition 2 and the target require.
enum ExactOutcome { kExactDrop = 0, kExactIndependent = 1, kExactEmit = 2, kExactOverflow = 3 };

// ---- modular null vector with rational reconstruction (the common, cheap case)
DEVI int64_t wave_sum_i64(int64_t v) {
  for (int off = 32; off > 0; off >>= 1) v += (int64_t)__shfl_xor((long long)v, off);
  return v;
}
DEVI int64_t gcd_i64(int64_t a, int64_t b) {
  a = a < 0 ? -a : a;
  b = b < 0 ? -b : b;
  while (b) { const int64_t t = a % b; a = b; b = t; }
  return a;
}

// The smallest fraction a/b (|a| <= 32767, 0 < b <= 32767) congruent to w modulo
// 2^31-1, by the extended Euclidean algorithm stopped at the half-size remainder
// (Wang's rational reconstruction).  Returns false when none exists.
DEVI bool rational_reconstruct(uint32_t w, int64_t &a, int64_t &b) {
  constexpr int64_t N = 32767;
  int64_t r0 = kPrime, r1 = w, t0 = 0, t1 = 1;
  while (r1 > N) {
    const int64_t q = r0 / r1;
    const int64_t r2 = r0 - q * r1, t2 = t0 - q * t1;
    r0 = r1; r1 = r2; t0 = t1; t1 = t2;
  }
  if (t1 == 0 || t1 > N || t1 < -N) return false;
  a = t1 < 0 ? -r1 : r1;
  b = t1 < 0 ? -t1 : t1;
  return gcd_i64(a, b) == 1;
}

// Definition 2 and the target on an exact null vector v (lane j: entry of the
// j-th reaction): full support, one sign on the irreversible reactions (made
// positive), S[x,:] v > 0.  |v| < 2^55.
DEVI int wave_sign_target(const DevNet &net, const int32_t *Sx, bool mine, int col, int64_t v, int64_t &vout) {
  if (__ballot(mine && v == 0) != 0) return kExactDrop;
  const bool irr = mine && !((net.rev_bits[col >> 6] >> (col & 63)) & 1ull);
  const u64 posm = __ballot(irr && v > 0), negm = __ballot(irr && v < 0);
  if (posm && negm) return kExactDrop;
  int64_t prod = wave_sum_i64(mine ? (int64_t)Sx[col] * v : 0);
  const int sgn = posm ? 1 : (negm ? -1 : (prod > 0 ? 1 : -1));
  if (sgn < 0) { v = -v; prod = -prod; }
  if (prod <= 0) return kExactDrop;
  vout = v;
  return kExactEmit;
}

// Exact decision through arithmetic modulo 2^31-1: the null vector modulo p of
// S_int[rows of Q, Q], lifted entry by entry by rational reconstruction, scaled
// to a primitive integer vector and checked against S_int v = 0 in exact 64-bit
// arithmetic.  A vector that passes is the exact null vector (the parent is
// independent, so the null space has dimension one); anything else returns -1
// and the caller falls back to 128-bit elimination.
template <int W, int MW>
DEVI int wave_exact_modp(const DevNet &net, const u64 *Q, const int32_t *Sx, uint32_t *Bl, int64_t &vout) {
  const int lane = lane_id();
  int kq = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) kq += __popcll(Q[w]);
  const bool mine = lane < kq;
  const int col = mine ? select_bit<W>(Q, lane) : -1;
  u64 T[MW];
#pragma unroll
  for (int q = 0; q < MW; ++q) T[q] = wave_or(col >= 0 ? net.rxn_touchM[(int64_t)col * MW + q] : 0ull);
  uint32_t ent[kMaxEnt];
  const int nnz = mine ? net.rxn_nnz[col] : 0;
  const bool dense = nnz < 0;
#pragma unroll
  for (int e = 0; e < kMaxEnt; ++e) ent[e] = (e < nnz) ? net.rxn_ent[(int64_t)col * kMaxEnt + e] : 0xFFFF0000u;
  auto coef = [&](int i) -> int32_t {
    int32_t c = 0;
    if (!mine) return 0;
    if (dense) return net.Sint[(int64_t)i * net.n + col];
#pragma unroll
    for (int e = 0; e < kMaxEnt; ++e)
      if ((int)(ent[e] >> 16) == i) c = (int32_t)(int16_t)(ent[e] & 0xFFFFu);
    return c;
  };

  // reduced row-echelon basis modulo p, unnormalised (as in the rank test); basis
  // row b lives in Bl[b * 64 + lane], each lane touching only its own column
  int nb = 0, rowof = -1;
#pragma unroll
  for (int q = 0; q < MW; ++q) {
    u64 bits = T[q];
    while (bits) {
      const int i = q * 64 + __builtin_ctzll(bits);
      bits &= bits - 1;
      const uint32_t x0 = tomod(coef(i));
      uint32_t x = x0, sigma = 1;
      u64 hits = __ballot(x0 != 0 && rowof >= 0);
      while (hits) {
        const int pc = __ffsll((long long)hits) - 1;
        hits &= hits - 1;
        const int bidx = __builtin_amdgcn_readfirstlane(__builtin_amdgcn_readlane(rowof, pc));
        const uint32_t f = (uint32_t)__builtin_amdgcn_readlane((int)x0, pc);
        const uint32_t rb = Bl[bidx * 64 + lane];
        const uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)rb, pc);
        x = submod(mulmod(d, x), mulmod(mulmod(sigma, f), rb));
        sigma = mulmod(sigma, d);
      }
      const u64 nz = __ballot(x != 0);
      if (nz) {
        if (nb >= kq) return -1;                 // cannot happen: rank <= columns
        const int pc = __ffsll((long long)nz) - 1;
        const uint32_t dn = (uint32_t)__builtin_amdgcn_readlane((int)x, pc);
        for (int bb = 0; bb < nb; ++bb) {
          const uint32_t rb = Bl[bb * 64 + lane];
          const uint32_t cb = (uint32_t)__builtin_amdgcn_readlane((int)rb, pc);
          if (cb) Bl[bb * 64 + lane] = submod(mulmod(dn, rb), mulmod(cb, x));
        }
        Bl[nb * 64 + lane] = x;
        if (lane == pc) rowof = nb;
        nb++;
      }
    }
  }
  if (nb == kq) return kExactIndependent;     // independent modulo p, hence over the rationals
  if (nb != kq - 1) return -1;
  const int f = __ffsll((long long)__ballot(mine && rowof < 0)) - 1;
  // Null vector modulo p without per-pivot inverses: with pivot values d_b and
  // free-column entries e_b, v_f = prod d_b and v_pc(b) = -e_b prod_{b' != b} d_b'.
  uint32_t dreg = 1, ereg = 0;     // lane b: d_b, e_b
  for (int b = 0; b < nb; ++b) {
    const uint32_t rb = Bl[b * 64 + lane];
    const int pc = __ffsll((long long)__ballot(rowof == b)) - 1;
    const uint32_t e = (uint32_t)__builtin_amdgcn_readlane((int)rb, f);
    const uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)rb, pc);
    if (lane == b) { dreg = d; ereg = e; }
  }
  uint32_t pre = 1, Dall = 1;      // lane b: product of d_b' for b' < b
  for (int b = 0; b < nb; ++b) {
    if (lane == b) pre = Dall;
    Dall = mulmod(Dall, (uint32_t)__builtin_amdgcn_readlane((int)dreg, b));
  }
  uint32_t suf = 1, acc = 1;       // lane b: product of d_b' for b' > b
  for (int b = nb - 1; b >= 0; --b) {
    if (lane == b) suf = acc;
    acc = mulmod(acc, (uint32_t)__builtin_amdgcn_readlane((int)dreg, b));
  }
  const uint32_t cb_ = mulmod(mulmod(pre, suf), ereg);   // lane b: e_b prod_{b' != b} d_b'
  const uint32_t Dinv = powmod(Dall, kPrime - 2);
  uint32_t vp = lane == f ? 1u : 0u;                      // entries divided by v_f = prod d_b
  for (int b = 0; b < nb; ++b) {
    const int pc = __ffsll((long long)__ballot(rowof == b)) - 1;
    const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)cb_, b);
    if (lane == pc) vp = c ? mulmod(kPrime - c, Dinv) : 0u;
  }
  // lift: v_j / v_f = a_j / b_j, then clear denominators
  int64_t a = 0, den = 1;
  bool ok = !mine || rational_reconstruct(vp, a, den);
  if (__ballot(!ok) != 0) return -1;
  int64_t L = mine ? den : 1;
  for (int off = 32; off > 0; off >>= 1) {
    const int64_t o = (int64_t)__shfl_xor((long long)L, off);
    const int64_t lg = L / gcd_i64(L, o);
    if (lg > (((int64_t)1 << 40) / o)) { ok = false; L = 1; }
    else L = lg * o;
  }
  if (__ballot(!ok) != 0) return -1;
  int64_t v = mine ? a * (L / den) : 0;
  int64_t g = v < 0 ? -v : v;
  for (int off = 32; off > 0; off >>= 1) g = gcd_i64(g, (int64_t)__shfl_xor((long long)g, off));
  if (g > 1) v /= g;
  // exact check S_int v = 0 on every row of Q (|coef| < 2^15, |v| < 2^55)
#pragma unroll
  for (int q = 0; q < MW; ++q) {
    u64 bits = T[q];
    while (bits) {
      const int i = q * 64 + __builtin_ctzll(bits);
      bits &= bits - 1;
      if (wave_sum_i64((int64_t)coef(i) * v) != 0) return -1;
    }
  }
  return wave_sign_target(net, Sx, mine, col, v, vout);
}

template <int W, int MW>
DEVI int wave_exact_child(const DevNet &net, const u64 *Q, const int32_t *Sx, i128 *M, uint32_t *Bl,
                          int64_t &vout, bool bareiss_only = false) {
  const int lane = lane_id();
  if (!bareiss_only) {
    const int fast = wave_exact_modp<W, MW>(net, Q, Sx, Bl, vout);
    if (fast >= 0) return fast;
  }
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
    if (__ballot(ovf)) return kExactOverflow;
    if (rank == kq) return kExactIndependent;   // the modular test was fooled
    if (rank != kq - 1) return kExactDrop;      // cannot happen for an independent parent

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
    if (ovf) return kExactOverflow;

    // Definition 2 and the target: full support, one sign on irreversible
    // reactions (made positive), S[x,:] v > 0
    if (__ballot(mine && v == 0) != 0) return kExactDrop;
    const bool irr = mine && !((net.rev_bits[col >> 6] >> (col & 63)) & 1ull);
    const u64 posm = __ballot(irr && v > 0), negm = __ballot(irr && v < 0);
    if (posm && negm) return kExactDrop;
    i128 prod = mine ? (i128)Sx[col] * v : (i128)0;
    for (int off = 32; off > 0; off >>= 1) prod += shfl_xor_i128(prod, off);
    int sgn = posm ? 1 : (negm ? -1 : (prod > 0 ? 1 : -1));
    if (sgn < 0) { v = -v; prod = -prod; }
    if (prod <= 0) return kExactDrop;
    const i128 lim = (i128)1 << 63;
    if (__ballot(v >= lim || v < -lim) != 0) return kExactOverflow;
    vout = (int64_t)v;
    return kExactEmit;
}


// One wave per child.  Lane j owns column j of the dense matrix S_int[T, Q] kept in
// global scratch (row-major, 64 entries per row); entries of other columns travel
// by lane shuffles only.
}  // namespace efm

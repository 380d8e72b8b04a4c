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
// whole wave.  Lane j owns column j of the dense matrix S_int[rows of Q, Q] kept in
// scratch M (row-major, 64 entries per row); entries of other columns travel by
// lane shuffles only.  On kExactEmit, vout holds (in lane j) the primitive flux of
// the j-th reaction of Q, signed as Definition 2 and the target require.
enum ExactOutcome { kExactDrop = 0, kExactIndependent = 1, kExactEmit = 2, kExactOverflow = 3 };

template <int W, int MW>
DEVI int wave_exact_child(const DevNet &net, const u64 *Q, const int32_t *Sx, i128 *M, int64_t &vout) {
  const int lane = lane_id();
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

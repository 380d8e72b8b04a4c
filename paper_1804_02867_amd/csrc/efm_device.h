// efm_device.h -- device helpers shared by the level kernels and the batched
// engine: wave-level reductions and appends, a lane-shuffle bit transpose,
// arithmetic modulo 2^31-1 and checked 128-bit integer helpers.
#pragma once
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

// Wave-private staging of list appends in LDS (`cap` entries, kWaveBuf unless the
// kernel gives more): one global atomic per flush instead of one per wave and
// step.  `n` is wave-uniform.
constexpr int kWaveBuf = 128;
struct WaveBuf {
  u64 *lds;
  int n;
  int cap = kWaveBuf;     // entries the LDS buffer holds
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
  if (b.n + cnt > b.cap) wbuf_flush(b, list, counter, cap, flags);
  if (pred) b.lds[b.n + __popcll(mask & lanes_below(lane_id()))] = val;
  b.n += cnt;
}

// Final flush of every wave's buffer in the block with one global atomic for the
// block (a list counter is shared by every block, so its atomics serialize).
// Every thread of the block (at most 4 waves) must call it.
DEVI void wbuf_flush_block(WaveBuf &b, u64 *list, u64 *counter, int64_t cap, u64 *flags) {
  __shared__ u64 wcnt[4], wbase[4];
  const int wib = threadIdx.x >> 6, lane = lane_id();
  __threadfence_block();
  if (lane == 0) wcnt[wib] = (u64)b.n;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (int)(blockDim.x >> 6);
    u64 tot = 0;
    for (int w = 0; w < nw; ++w) tot += wcnt[w];
    u64 base = tot ? atomicAdd(counter, tot) : 0ull;
    for (int w = 0; w < nw; ++w) { wbase[w] = base; base += wcnt[w]; }
  }
  __syncthreads();
  const u64 base = wbase[wib];
  for (int i = lane; i < b.n; i += 64) {
    const u64 idx = base + (u64)i;
    if ((int64_t)idx < cap) list[idx] = b.lds[i];
    else atomicOr(flags, (u64)kFlagQueueOverflow);
  }
  b.n = 0;
}

// Slot of this lane in a list that every lane with pred appends one entry to, with
// one global atomic for the block.  Every thread of the block (at most 4 waves)
// must call it; the result is meaningful where pred is set.
DEVI u64 block_append_index(bool pred, u64 *counter) {
  __shared__ u64 acnt[4], abase[4];
  const int wib = threadIdx.x >> 6, lane = lane_id();
  const u64 m = __ballot(pred);
  if (lane == 0) acnt[wib] = (u64)__popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (int)(blockDim.x >> 6);
    u64 tot = 0;
    for (int w = 0; w < nw; ++w) tot += acnt[w];
    u64 base = tot ? atomicAdd(counter, tot) : 0ull;
    for (int w = 0; w < nw; ++w) { abase[w] = base; base += acnt[w]; }
  }
  __syncthreads();
  return abase[wib] + (u64)__popcll(m & lanes_below(lane));
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

// 64-bit value of lane src, broadcast to the wave
DEVI u64 readlane64(u64 v, int src) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), src);
  return ((u64)hi << 32) | lo;
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

}  // namespace efm

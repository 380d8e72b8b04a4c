// efm_learn.hip -- the learned frontier ordering: model inputs of partial
// pathways, the perceptron's inference and training kernels (sparse gather for
// the input layer, bf16 MFMA for the dense layers, fp32 accumulation), trace
// collection from the plain traversal, and the C ABI of traces and models.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <new>
#include <vector>

#include "../../include/efm.h"
#include "efm_device.h"
#include "efm_host.h"

using efm::u64;

namespace efm {

constexpr int kFeatMax = EFM_FEAT_MAX;
constexpr int kH = 256;                 // hidden units
constexpr int kTraceW = EFM_TRACE_WORDS;
constexpr int kTile = 16;               // items per wave tile (the MFMA M dimension)
constexpr int kMaxCounts = 1024;
constexpr int kMaxBatch = 65536;

typedef short s4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

struct ModelDev {
  const uint16_t *W1b;    // [F][kH] bf16
  const uint16_t *W2Tb;   // [kH out][kH in] bf16 (forward B operand)
  const uint16_t *W2b;    // [kH in][kH out] bf16 (backward B operand)
  const uint16_t *w3b;    // [kH] bf16
  const float *b1, *b2, *b3;
};

struct FeatDev {
  const uint16_t *rpos;   // [n] relabelled reaction positions
  const uint16_t *mpos;   // [mi] relabelled internal-metabolite positions
  int in_bits, mi;
};

struct TraceDev {
  uint16_t *ent;          // [cap][kFeatMax]
  uint16_t *len;          // [cap]
  uint8_t *lab;           // [cap]
  u64 *keys;              // [cap][kTraceW]
  u64 *ctr;               // [0] records written, [1] overflow flags, [2] positive records
  int64_t cap;
};

// where the score kernel takes its items from
struct ScoreSrc {
  int mode;               // 0 the level's survivors, 1 bitsets, 2 trace records
  const u64 *keys;        // mode 1: [n][kw]
  int kw;
  TraceDev tr;            // mode 2: records first ..
  int64_t first;
};

DEVI float bf2f(uint32_t b) { return __uint_as_float((b & 0xFFFFu) << 16); }
DEVI uint32_t f2bf(float f) {        // round to nearest even (finite inputs)
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}
DEVI void wave_sync() {
  __threadfence_block();
  __builtin_amdgcn_wave_barrier();
}
DEVI float entry_value(uint32_t code) { return code == 0 ? 1.f : (float)code * 0.125f; }

// Score word of a logit: ascending word order = descending score.
DEVI uint32_t score_word(float s) {
  const uint32_t u = __float_as_uint(s);
  const uint32_t ord = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  return ~ord;
}

DEVI u64 mix64(u64 x) {
  x ^= x >> 30;
  x *= 0xBF58476D1CE4E5B9ull;
  x ^= x >> 27;
  x *= 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// Model input of the partial pathway K (the same in every lane) as entry words in
// lst (wave-private LDS): its reactions in increasing index (wave ballot over
// the bits of each key word), then the internal metabolites with a non-zero
// clamped imbalance count in increasing index, as the magnitude on the
// metabolite's surplus or deficit row.  cnt is wave-private LDS of mi
// ints, zero on entry and on return.  Returns the entry count (above kFeatMax
// the list is cut).
template <int W>
DEVI int wave_featurize(const DevNet &net, const FeatDev &ft, const u64 (&K)[W], uint16_t *lst, int *cnt) {
  const int lane = lane_id();
  const u64 below = lanes_below(lane);
  int base = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const u64 word = K[w];
    if ((word >> lane) & 1ull) {
      const int idx = base + __popcll(word & below);
      if (idx < kFeatMax) lst[idx] = (uint16_t)(ft.rpos[w * 64 + lane] << 4);
    }
    base += __popcll(word);
  }
#pragma unroll
  for (int w = 0; w < W; ++w) {
    u64 word = K[w];
    while (word) {
      const int r = w * 64 + __builtin_ctzll(word);
      word &= word - 1;
      if (lane < net.rxn_nnz[r]) {
        const uint32_t e = net.rxn_ent[(size_t)r * kMaxEnt + lane];
        atomicAdd(&cnt[e >> 16], (int16_t)(e & 0xFFFFu) > 0 ? 1 : -1);
      }
    }
  }
  wave_sync();
  for (int q = 0; q < ft.mi; q += 64) {
    const int k = q + lane;
    int u = 0;
    if (k < ft.mi) {
      u = cnt[k];
      cnt[k] = 0;
    }
    u = u < -7 ? -7 : (u > 7 ? 7 : u);
    const u64 nz = __ballot(u != 0);
    if (u != 0) {
      const int idx = base + __popcll(nz & below);
      const int row = ft.in_bits + 2 * ft.mpos[k] + (u < 0 ? 1 : 0);
      if (idx < kFeatMax) lst[idx] = (uint16_t)((row << 4) | (u < 0 ? -u : u));
    }
    base += __popcll(nz);
  }
  wave_sync();
  return base;
}

// First layer, sparse: this lane's units 4*lane .. 4*lane+3 of
// b1 + sum over the entries of value * W1[row] (rows are 512-byte bf16 lines, read
// whole by the wave), four rows in flight at a time.
DEVI void wave_layer1(const ModelDev &md, const uint16_t *lst, int n, float (&h)[4]) {
  const int lane = lane_id();
  const float4 b = *(const float4 *)(md.b1 + lane * 4);
  h[0] = b.x;
  h[1] = b.y;
  h[2] = b.z;
  h[3] = b.w;
  int e = 0;
  for (; e + 4 <= n; e += 4) {
    uint32_t v[4];
    uint2 w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = lst[e + q];
#pragma unroll
    for (int q = 0; q < 4; ++q) w[q] = *(const uint2 *)(md.W1b + (size_t)(v[q] >> 4) * kH + lane * 4);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float x = entry_value(v[q] & 15u);
      h[0] = fmaf(x, bf2f(w[q].x), h[0]);
      h[1] = fmaf(x, bf2f(w[q].x >> 16), h[1]);
      h[2] = fmaf(x, bf2f(w[q].y), h[2]);
      h[3] = fmaf(x, bf2f(w[q].y >> 16), h[3]);
    }
  }
  for (; e < n; ++e) {
    const uint32_t v = lst[e];
    const uint2 w = *(const uint2 *)(md.W1b + (size_t)(v >> 4) * kH + lane * 4);
    const float x = entry_value(v & 15u);
    h[0] = fmaf(x, bf2f(w.x), h[0]);
    h[1] = fmaf(x, bf2f(w.x >> 16), h[1]);
    h[2] = fmaf(x, bf2f(w.y), h[2]);
    h[3] = fmaf(x, bf2f(w.y >> 16), h[3]);
  }
}

// rectified first-layer units of one item, rounded to bf16, into row t of H1s
DEVI void store_h1(uint16_t *H1s, int t, const float (&h)[4]) {
  const int lane = lane_id();
  uint2 pk;
  pk.x = f2bf(fmaxf(h[0], 0.f)) | (f2bf(fmaxf(h[1], 0.f)) << 16);
  pk.y = f2bf(fmaxf(h[2], 0.f)) | (f2bf(fmaxf(h[3], 0.f)) << 16);
  *(uint2 *)(H1s + t * kH + lane * 4) = pk;
}

// Layers 2 and 3 of the 16 items whose bf16 first-layer activations are the rows
// of H1s (wave-private LDS [16][kH]).  v_mfma_f32_16x16x16_bf16 lane layout: lane
// l holds A[l%16][4(l/16)+v], B[4(l/16)+v][l%16] and D[4(l/16)+v][l%16], v = 0..3.
// s[v] receives the logit of item 4(l/16)+v in every lane of that 16-lane group;
// z2s (LDS [16][kH] fp32, may be null) the second layer's pre-activations.
DEVI void wave_layer23(const ModelDev &md, const uint16_t *H1s, float (&s)[4], float *z2s) {
  const int lane = lane_id();
  const int col = lane & 15, grp = lane >> 4;
  s4_t A[16];
#pragma unroll
  for (int kb = 0; kb < 16; ++kb) A[kb] = *(const s4_t *)(H1s + col * kH + kb * 16 + grp * 4);
  float part[4] = {0.f, 0.f, 0.f, 0.f};
  for (int nb = 0; nb < 16; ++nb) {
    f4_t acc = {0.f, 0.f, 0.f, 0.f};
    const uint16_t *brow = md.W2Tb + (size_t)(nb * 16 + col) * kH + grp * 4;
#pragma unroll
    for (int kb = 0; kb < 16; ++kb) {
      const s4_t b = *(const s4_t *)(brow + kb * 16);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A[kb], b, acc, 0, 0, 0);
    }
    const int j = nb * 16 + col;
    const float bj = md.b2[j], wj = bf2f(md.w3b[j]);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float z = acc[v] + bj;
      if (z2s) z2s[(grp * 4 + v) * kH + j] = z;
      part[v] = fmaf(fmaxf(z, 0.f), wj, part[v]);
    }
  }
  const float b3 = md.b3[0];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    float t = part[v];
    t += __shfl_xor(t, 8);
    t += __shfl_xor(t, 4);
    t += __shfl_xor(t, 2);
    t += __shfl_xor(t, 1);
    s[v] = t + b3;
  }
}

// copy of trace record `rec` into lst (wave-private LDS); returns its length
DEVI int wave_load_record(const TraceDev &tr, int64_t rec, uint16_t *lst) {
  const int lane = lane_id();
  const int n = tr.len[rec];
  for (int e = lane; e < n; e += 64) lst[e] = tr.ent[rec * kFeatMax + e];
  wave_sync();
  return n;
}

__host__ __device__ inline size_t score_lds_per_wave(int mi) {
  return (size_t)kTile * kH * 2 + kFeatMax * 2 + (size_t)((mi + 63) & ~63) * 4;
}

// Scores tiles of 16 items per wave: each item's input is built (from a key) or
// loaded (from a record) into LDS, its first layer gathered, then layers 2-3 run
// on the tile with MFMA.  Writes score words (mode 0) or logits.
template <int W>
__global__ __launch_bounds__(256) void score_kernel(DevNet net, DevLevel L, FeatDev ft, ModelDev md, ScoreSrc src,
                                                    int64_t n, uint32_t *words, float *logits, u64 *flags) {
  extern __shared__ __align__(16) char smem[];
  const int wib = threadIdx.x >> 6, lane = lane_id();
  const int mi_pad = (ft.mi + 63) & ~63;
  char *mine = smem + (size_t)wib * score_lds_per_wave(ft.mi);
  uint16_t *H1s = (uint16_t *)mine;
  uint16_t *lst = H1s + kTile * kH;
  int *cnt = (int *)(lst + kFeatMax);
  for (int k = lane; k < mi_pad; k += 64) cnt[k] = 0;
  wave_sync();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  bool over = false;
  for (int64_t tile = wave; tile * kTile < n; tile += nwaves) {
    for (int t = 0; t < kTile; ++t) {
      const int64_t i = tile * kTile + t;
      float h[4] = {0.f, 0.f, 0.f, 0.f};
      if (i < n) {
        int ne;
        if (src.mode == 2) {
          ne = wave_load_record(src.tr, src.first + i, lst);
        } else {
          u64 K[W];
          if (src.mode == 1) {
#pragma unroll
            for (int w = 0; w < W; ++w) K[w] = w < src.kw ? src.keys[i * src.kw + w] : 0ull;
          } else {
            const u64 ref = L.surv[i];
            const int64_t p = (int64_t)(ref >> 12);
            const int r = (int)((ref >> 1) & 0x7FF);
#pragma unroll
            for (int w = 0; w < W; ++w)
              K[w] = L.keys[(int64_t)w * L.fcap + p] | ((r >> 6) == w ? (1ull << (r & 63)) : 0ull);
          }
          ne = wave_featurize<W>(net, ft, K, lst, cnt);
          if (ne > kFeatMax) {
            over = true;
            ne = kFeatMax;
          }
        }
        wave_layer1(md, lst, ne, h);
      }
      store_h1(H1s, t, h);
      wave_sync();
    }
    float s[4];
    wave_layer23(md, H1s, s, nullptr);
    if ((lane & 15) == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = tile * kTile + (lane >> 4) * 4 + v;
        if (i < n) {
          if (words) words[i] = score_word(s[v]);
          else logits[i] = s[v];
        }
      }
    }
    wave_sync();
  }
  if (over && lane == 0) atomicOr((unsigned long long *)flags, (unsigned long long)kFlagFeatOverflow);
}

// ------------------------------------------------------------------ training
// A minibatch of B records (indices idx[0..B)), padded to Bp = 16k items.
// Forward with the loss gradient per item, g = (pw*y*(sigmoid(s)-1) +
// (1-y)*sigmoid(s)) / B; writes the bf16 activations a1 and second-layer
// gradients dz2 item-major and transposed (MFMA operands of the backward
// kernels) and accumulates the gradients of w3, b2, b3 and the loss sum.
__global__ __launch_bounds__(128) void train_fwd_kernel(ModelDev md, TraceDev tr, const int32_t *idx, int B, int Bp,
                                                        float pw, float invB, uint16_t *A1, uint16_t *A1T,
                                                        uint16_t *DZ2, uint16_t *DZ2T, float *gw3, float *gb2,
                                                        float *gb3, float *loss) {
  extern __shared__ __align__(16) char smem[];
  const int wib = threadIdx.x >> 6, lane = lane_id();
  const int col = lane & 15, grp = lane >> 4;
  char *mine = smem + (size_t)wib * (kTile * kH * 2 + kFeatMax * 2 + kTile * kH * 4);
  uint16_t *H1s = (uint16_t *)mine;
  uint16_t *lst = H1s + kTile * kH;
  float *z2s = (float *)(lst + kFeatMax);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int ntiles = Bp / kTile;
  for (int64_t tile = wave; tile < ntiles; tile += nwaves) {
    for (int t = 0; t < kTile; ++t) {
      const int item = (int)tile * kTile + t;
      float h[4] = {0.f, 0.f, 0.f, 0.f};
      if (item < B) {
        const int ne = wave_load_record(tr, idx[item], lst);
        wave_layer1(md, lst, ne, h);
      }
      store_h1(H1s, t, h);
      wave_sync();
      const uint2 pk = *(const uint2 *)(H1s + t * kH + lane * 4);
      *(uint2 *)(A1 + (size_t)item * kH + lane * 4) = pk;
      A1T[(size_t)(lane * 4 + 0) * Bp + item] = (uint16_t)(pk.x & 0xFFFF);
      A1T[(size_t)(lane * 4 + 1) * Bp + item] = (uint16_t)(pk.x >> 16);
      A1T[(size_t)(lane * 4 + 2) * Bp + item] = (uint16_t)(pk.y & 0xFFFF);
      A1T[(size_t)(lane * 4 + 3) * Bp + item] = (uint16_t)(pk.y >> 16);
    }
    float s[4];
    wave_layer23(md, H1s, s, z2s);
    wave_sync();
    float g[4], lsum = 0.f, gsum = 0.f;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int item = (int)tile * kTile + grp * 4 + v;
      g[v] = 0.f;
      if (item < B) {
        const float y = tr.lab[idx[item]] ? 1.f : 0.f;
        const float sv = s[v];
        const float sig = 1.f / (1.f + expf(-sv));
        g[v] = (pw * y * (sig - 1.f) + (1.f - y) * sig) * invB;
        // softplus(t) = max(t, 0) + log1p(exp(-|t|))
        const float sp_pos = fmaxf(sv, 0.f) + log1pf(expf(-fabsf(sv)));   // softplus(s)
        const float sp_neg = sp_pos - sv;                                  // softplus(-s)
        if (col == 0) {
          lsum += pw * y * sp_neg + (1.f - y) * sp_pos;
          gsum += g[v];
        }
      }
    }
    for (int nb = 0; nb < 16; ++nb) {
      const int j = nb * 16 + col;
      const float wj = bf2f(md.w3b[j]);
      float dw = 0.f, db = 0.f;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int item = (int)tile * kTile + grp * 4 + v;
        const float z = z2s[(grp * 4 + v) * kH + j];
        const float dz = z > 0.f ? g[v] * wj : 0.f;
        dw = fmaf(g[v], fmaxf(z, 0.f), dw);
        db += dz;
        const uint16_t b16 = (uint16_t)f2bf(dz);
        DZ2[(size_t)item * kH + j] = b16;
        DZ2T[(size_t)j * Bp + item] = b16;
      }
      dw += __shfl_xor(dw, 16);
      dw += __shfl_xor(dw, 32);
      db += __shfl_xor(db, 16);
      db += __shfl_xor(db, 32);
      if (grp == 0) {
        atomicAdd(&gw3[j], dw);
        atomicAdd(&gb2[j], db);
      }
    }
    lsum += __shfl_xor(lsum, 16);
    lsum += __shfl_xor(lsum, 32);
    gsum += __shfl_xor(gsum, 16);
    gsum += __shfl_xor(gsum, 32);
    if (lane == 0) {
      atomicAdd(loss, lsum);
      atomicAdd(gb3, gsum);
    }
    wave_sync();
  }
}

// dW2 = A1^T dZ2 over the minibatch: one wave per 16x16 output tile, MFMA over
// the items (operands read from the transposed copies, 8 contiguous bytes per
// lane).  Each tile has one owner, so the gradient is added without atomics.
__global__ __launch_bounds__(256) void dw2_kernel(const uint16_t *A1T, const uint16_t *DZ2T, int Bp, float *gW2) {
  const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (wave >= 256) return;
  const int lane = lane_id();
  const int col = lane & 15, grp = lane >> 4;
  const int mb = wave >> 4, nb = wave & 15;
  const uint16_t *arow = A1T + (size_t)(mb * 16 + col) * Bp + grp * 4;
  const uint16_t *brow = DZ2T + (size_t)(nb * 16 + col) * Bp + grp * 4;
  f4_t acc = {0.f, 0.f, 0.f, 0.f};
  for (int ib = 0; ib < Bp; ib += 16)
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(*(const s4_t *)(arow + ib), *(const s4_t *)(brow + ib), acc, 0,
                                                     0, 0);
#pragma unroll
  for (int v = 0; v < 4; ++v) gW2[(size_t)(mb * 16 + grp * 4 + v) * kH + nb * 16 + col] += acc[v];
}

// dZ1 = (dZ2 W2^T) masked by a1 > 0 (MFMA per 16-item tile), then the sparse
// first layer: dW1[row] += value * dz1 for every input entry (fp32 atomics) and
// db1 += dz1.
__global__ __launch_bounds__(128) void bwd1_kernel(ModelDev md, TraceDev tr, const int32_t *idx, int B, int Bp,
                                                   const uint16_t *A1, const uint16_t *DZ2, float *gW1, float *gb1) {
  extern __shared__ __align__(16) char smem[];
  const int wib = threadIdx.x >> 6, lane = lane_id();
  const int col = lane & 15, grp = lane >> 4;
  char *mine = smem + (size_t)wib * (kTile * kH * 4 + kFeatMax * 2);
  float *dz1s = (float *)mine;
  uint16_t *lst = (uint16_t *)(dz1s + kTile * kH);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int ntiles = Bp / kTile;
  float db[4] = {0.f, 0.f, 0.f, 0.f};
  for (int64_t tile = wave; tile < ntiles; tile += nwaves) {
    s4_t A[16];
#pragma unroll
    for (int kb = 0; kb < 16; ++kb)
      A[kb] = *(const s4_t *)(DZ2 + (size_t)(tile * kTile + col) * kH + kb * 16 + grp * 4);
    for (int nb = 0; nb < 16; ++nb) {
      f4_t acc = {0.f, 0.f, 0.f, 0.f};
      const uint16_t *brow = md.W2b + (size_t)(nb * 16 + col) * kH + grp * 4;
#pragma unroll
      for (int kb = 0; kb < 16; ++kb)
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A[kb], *(const s4_t *)(brow + kb * 16), acc, 0, 0, 0);
      const int k = nb * 16 + col;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t item = tile * kTile + grp * 4 + v;
        const bool on = (A1[(size_t)item * kH + k] & 0x7FFFu) != 0;   // a1 > 0 (a signed zero is off)
        dz1s[(grp * 4 + v) * kH + k] = on ? acc[v] : 0.f;
      }
    }
    wave_sync();
    for (int t = 0; t < kTile; ++t) {
      const int item = (int)tile * kTile + t;
      if (item >= B) break;
      const float4 d = *(const float4 *)(dz1s + t * kH + lane * 4);
      db[0] += d.x;
      db[1] += d.y;
      db[2] += d.z;
      db[3] += d.w;
      const int ne = wave_load_record(tr, idx[item], lst);
      for (int e = 0; e < ne; ++e) {
        const uint32_t v = lst[e];
        const float x = entry_value(v & 15u);
        float *g = gW1 + (size_t)(v >> 4) * kH + lane * 4;
        atomicAdd(g + 0, x * d.x);
        atomicAdd(g + 1, x * d.y);
        atomicAdd(g + 2, x * d.z);
        atomicAdd(g + 3, x * d.w);
      }
      wave_sync();
    }
    wave_sync();
  }
#pragma unroll
  for (int c = 0; c < 4; ++c)
    if (db[c] != 0.f) atomicAdd(&gb1[lane * 4 + c], db[c]);
}

struct ParamMap {
  int64_t n, oW1, nW1, oW2, ow3;
  uint16_t *W1b, *W2b, *W2Tb, *w3b;
};

DEVI void store_copy(const ParamMap &pm, int64_t p, float w) {
  const uint16_t b = (uint16_t)f2bf(w);
  if (p >= pm.oW1 && p < pm.oW1 + pm.nW1) {
    pm.W1b[p - pm.oW1] = b;
  } else if (p >= pm.oW2 && p < pm.oW2 + kH * kH) {
    const int64_t q = p - pm.oW2;
    pm.W2b[q] = b;
    pm.W2Tb[(q % kH) * kH + q / kH] = b;
  } else if (p >= pm.ow3 && p < pm.ow3 + kH) {
    pm.w3b[p - pm.ow3] = b;
  }
}

// One Adam step with bias corrections c1 = 1/(1-beta1^t), c2 = 1/(1-beta2^t);
// clears the gradient and refreshes the bf16 copies.
__global__ __launch_bounds__(256) void adam_kernel(float *P, float *G, float *M, float *V, ParamMap pm, float lr,
                                                   float beta1, float beta2, float eps, float c1, float c2) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < pm.n; p += stride) {
    const float g = G[p];
    G[p] = 0.f;
    const float m = beta1 * M[p] + (1.f - beta1) * g;
    const float v = beta2 * V[p] + (1.f - beta2) * g * g;
    M[p] = m;
    V[p] = v;
    const float w = P[p] - lr * (m * c1) / (sqrtf(v * c2) + eps);
    P[p] = w;
    store_copy(pm, p, w);
  }
}

__global__ __launch_bounds__(256) void copies_kernel(const float *P, ParamMap pm) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < pm.n; p += stride) store_copy(pm, p, P[p]);
}

// ------------------------------------------------------------------- traces
// lab[i] = 1 when frontier state i is a subset of one of the nf found pathways
// (AoS [nf][W]); npos counts them.
template <int W>
__global__ __launch_bounds__(256) void label_kernel(const u64 *keys, int64_t fcap, int64_t n, const u64 *found,
                                                    int64_t nf, uint8_t *lab, u64 *npos) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    u64 K[W];
#pragma unroll
    for (int w = 0; w < W; ++w) K[w] = keys[(int64_t)w * fcap + i];
    bool hit = false;
    for (int64_t f = 0; f < nf && !hit; ++f) {
      bool sub = true;
#pragma unroll
      for (int w = 0; w < W; ++w) sub = sub && (K[w] & ~found[f * W + w]) == 0;
      hit = sub;
    }
    lab[i] = hit ? 1 : 0;
    const u64 m = __ballot(hit);
    if (lane_id() == __ffsll((long long)__ballot(1)) - 1 && m) atomicAdd((unsigned long long *)npos, (unsigned long long)__popcll(m));
  }
}

// Appends as records the positive states whose mixed hash is <= thr_pos and the
// negative ones whose mixed hash is <= thr (one wave builds one record).
template <int W>
__global__ __launch_bounds__(256) void record_kernel(DevNet net, FeatDev ft, const u64 *keys, const u64 *hash,
                                                     int64_t fcap, int64_t n, const uint8_t *lab, u64 thr,
                                                     u64 thr_pos, u64 salt, TraceDev tr) {
  extern __shared__ __align__(16) char smem[];
  const int wib = threadIdx.x >> 6, lane = lane_id();
  const int mi_pad = (ft.mi + 63) & ~63;
  char *mine = smem + (size_t)wib * ((size_t)kFeatMax * 2 + (size_t)mi_pad * 4);
  uint16_t *lst = (uint16_t *)mine;
  int *cnt = (int *)(lst + kFeatMax);
  for (int k = lane; k < mi_pad; k += 64) cnt[k] = 0;
  wave_sync();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t base = wave * 64; base < n; base += nwaves * 64) {
    const int64_t i = base + lane;
    bool take = false;
    if (i < n) {
      const u64 hm = mix64(hash[i] ^ salt);
      take = lab[i] != 0 ? hm <= thr_pos : hm <= thr;
    }
    u64 m = __ballot(take);
    while (m) {
      const int src = __ffsll((long long)m) - 1;
      m &= m - 1;
      const int64_t st = base + src;
      u64 slot = 0;
      if (lane == 0) slot = atomicAdd((unsigned long long *)tr.ctr, 1ull);
      slot = readlane64(slot, 0);
      if ((int64_t)slot >= tr.cap) {
        if (lane == 0) atomicOr((unsigned long long *)(tr.ctr + 1), (unsigned long long)kFlagQueueOverflow);
        continue;
      }
      u64 K[W];
#pragma unroll
      for (int w = 0; w < W; ++w) K[w] = keys[(int64_t)w * fcap + st];
      int ne = wave_featurize<W>(net, ft, K, lst, cnt);
      if (ne > kFeatMax) {
        if (lane == 0) atomicOr((unsigned long long *)(tr.ctr + 1), (unsigned long long)kFlagFeatOverflow);
        ne = kFeatMax;
      }
      for (int e = lane; e < ne; e += 64) tr.ent[(int64_t)slot * kFeatMax + e] = lst[e];
      if (lane == 0) {
        tr.len[slot] = (uint16_t)ne;
        tr.lab[slot] = lab[st];
        if (lab[st]) atomicAdd((unsigned long long *)(tr.ctr + 2), 1ull);
      }
      u64 kv = 0;
#pragma unroll
      for (int w = 0; w < W; ++w)
        if (lane == w) kv = K[w];
      if (lane < kTraceW) tr.keys[(int64_t)slot * kTraceW + lane] = kv;
      wave_sync();
    }
  }
}

// ------------------------------------------------------------------ launchers

static int g_cus = 0;
static int num_cus_l() {
  if (g_cus == 0) {
    int dev = 0, c = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) ==
                                                hipSuccess && c > 0)
      g_cus = c;
    else
      g_cus = 256;
  }
  return g_cus;
}

// waves per block whose LDS fits 64 KB
static int waves_for(size_t per_wave) {
  for (int w = 4; w >= 1; w >>= 1)
    if (per_wave * (size_t)w <= 65536) return w;
  return 1;
}

template <int W>
static hipError_t do_score(const DevNet &net, const DevLevel &L, const FeatDev &ft, const ModelDev &md,
                           const ScoreSrc &src, int64_t n, uint32_t *words, float *logits, u64 *flags,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const size_t per = score_lds_per_wave(ft.mi);
  const int wpb = waves_for(per);
  const int64_t tiles = (n + kTile - 1) / kTile;
  const int64_t blocks = std::min<int64_t>((tiles + wpb - 1) / wpb, (int64_t)num_cus_l() * 16);
  hipLaunchKernelGGL((score_kernel<W>), dim3((unsigned)blocks), dim3(64 * wpb), per * wpb, s, net, L, ft, md, src, n,
                     words, logits, flags);
  return hipGetLastError();
}

static hipError_t launch_score(int Wt, const DevNet &net, const DevLevel &L, const FeatDev &ft, const ModelDev &md,
                               const ScoreSrc &src, int64_t n, uint32_t *words, float *logits, u64 *flags,
                               hipStream_t s) {
  switch (Wt) {
    case 1: return do_score<1>(net, L, ft, md, src, n, words, logits, flags, s);
    case 2: return do_score<2>(net, L, ft, md, src, n, words, logits, flags, s);
    case 4: return do_score<4>(net, L, ft, md, src, n, words, logits, flags, s);
    case 8: return do_score<8>(net, L, ft, md, src, n, words, logits, flags, s);
    default: return do_score<16>(net, L, ft, md, src, n, words, logits, flags, s);
  }
}

template <int W>
static hipError_t do_trace(const DevNet &net, const FeatDev &ft, const u64 *keys, const u64 *hash, int64_t fcap,
                           int64_t n, const u64 *found, int64_t nf, uint8_t *lab, u64 *npos, int phase, u64 thr,
                           u64 thr_pos, u64 salt, const TraceDev &tr, hipStream_t s) {
  if (phase == 0) {
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, (int64_t)num_cus_l() * 16);
    hipLaunchKernelGGL((label_kernel<W>), dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, s, keys, fcap,
                       n, found, nf, lab, npos);
  } else {
    const size_t per = (size_t)kFeatMax * 2 + (size_t)((ft.mi + 63) & ~63) * 4;
    const int wpb = waves_for(per);
    const int64_t blocks = std::min<int64_t>((n + 64 * wpb - 1) / (64 * wpb), (int64_t)num_cus_l() * 16);
    hipLaunchKernelGGL((record_kernel<W>), dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(64 * wpb), per * wpb, s,
                       net, ft, keys, hash, fcap, n, lab, thr, thr_pos, salt, tr);
  }
  return hipGetLastError();
}

static hipError_t launch_trace(int Wt, const DevNet &net, const FeatDev &ft, const u64 *keys, const u64 *hash,
                               int64_t fcap, int64_t n, const u64 *found, int64_t nf, uint8_t *lab, u64 *npos,
                               int phase, u64 thr, u64 thr_pos, u64 salt, const TraceDev &tr, hipStream_t s) {
  switch (Wt) {
    case 1: return do_trace<1>(net, ft, keys, hash, fcap, n, found, nf, lab, npos, phase, thr, thr_pos, salt, tr, s);
    case 2: return do_trace<2>(net, ft, keys, hash, fcap, n, found, nf, lab, npos, phase, thr, thr_pos, salt, tr, s);
    case 4: return do_trace<4>(net, ft, keys, hash, fcap, n, found, nf, lab, npos, phase, thr, thr_pos, salt, tr, s);
    case 8: return do_trace<8>(net, ft, keys, hash, fcap, n, found, nf, lab, npos, phase, thr, thr_pos, salt, tr, s);
    default:
      return do_trace<16>(net, ft, keys, hash, fcap, n, found, nf, lab, npos, phase, thr, thr_pos, salt, tr, s);
  }
}

}  // namespace efm

// ------------------------------------------------------------------ host side

struct efm_model {
  int in_bits = 0, in_counts = 0, F = 0;
  int64_t nparam = 0, oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, ow3 = 0, ob3 = 0;
  float *P = nullptr, *G = nullptr, *M = nullptr, *V = nullptr;
  uint16_t *W1b = nullptr, *W2b = nullptr, *W2Tb = nullptr, *w3b = nullptr;
  int64_t step = 0;
  void *mem = nullptr;

  efm::ModelDev dev() const {
    return efm::ModelDev{W1b, W2Tb, W2b, w3b, P + ob1, P + ob2, P + ob3};
  }
  efm::ParamMap map() const {
    return efm::ParamMap{nparam, oW1, (int64_t)F * efm::kH, oW2, ow3, W1b, W2b, W2Tb, w3b};
  }
};

struct efm_traces {
  int in_bits = 0, in_counts = 0;
  int64_t cap = 0, count = 0, positives = 0;
  efm::TraceDev d{};
  void *mem = nullptr;
};

namespace {

#define LCHK(expr)                                                                        \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) {                                                               \
      rc = fail(EFM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));              \
      goto done;                                                                          \
    }                                                                                     \
  } while (0)

u64 sm64(u64 &state) {
  u64 z = (state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Relabelled positions of reactions and internal metabolites around target x:
// breadth-first distance from the reactions touching x over the bipartite graph
// of internal metabolites and reactions, then decreasing degree, then index.
efm_status relabel(const efm_network *N, int x, int in_bits, int in_counts, std::vector<uint16_t> &rpos,
                   std::vector<uint16_t> &mpos) {
  const int n = N->n, mi = N->mi;
  if (n > in_bits) return fail(EFM_EINVAL, "network has %d reactions, model input has %d", n, in_bits);
  if (mi > in_counts)
    return fail(EFM_EINVAL, "network has %d internal metabolites, model input has %d", mi, in_counts);
  std::vector<std::vector<int>> r_m(n), m_r(mi);
  for (int k = 0; k < mi; ++k) {
    const int row = N->int_row[k];
    for (int r = 0; r < n; ++r) {
      const int32_t v = N->S[(size_t)row * n + r];
      if (v == 0) continue;
      r_m[r].push_back(k);
      m_r[k].push_back(r);
      if (v < -32768 || v > 32767)
        return fail(EFM_EINVAL, "coefficient of reaction %d outside the 16-bit range of the model input", r);
    }
  }
  for (int r = 0; r < n; ++r)
    if ((int)r_m[r].size() > efm::kMaxEnt)
      return fail(EFM_EINVAL, "reaction %d touches more than %d internal metabolites", r, efm::kMaxEnt);
  const int kUn = 1 << 30;
  std::vector<int> rd(n, kUn), md(mi, kUn);
  std::deque<std::pair<int, int>> q;   // (kind 0 = reaction, 1 = metabolite, index)
  for (int r = 0; r < n; ++r)
    if (N->S[(size_t)x * n + r] != 0) {
      rd[r] = 0;
      q.push_back({0, r});
    }
  while (!q.empty()) {
    auto [kind, v] = q.front();
    q.pop_front();
    if (kind == 0) {
      for (int k : r_m[v])
        if (md[k] == kUn) { md[k] = rd[v] + 1; q.push_back({1, k}); }
    } else {
      for (int r : m_r[v])
        if (rd[r] == kUn) { rd[r] = md[v] + 1; q.push_back({0, r}); }
    }
  }
  std::vector<int> ro(n), mo(mi);
  for (int i = 0; i < n; ++i) ro[i] = i;
  for (int i = 0; i < mi; ++i) mo[i] = i;
  std::sort(ro.begin(), ro.end(), [&](int a, int b) {
    if (rd[a] != rd[b]) return rd[a] < rd[b];
    if (r_m[a].size() != r_m[b].size()) return r_m[a].size() > r_m[b].size();
    return a < b;
  });
  std::sort(mo.begin(), mo.end(), [&](int a, int b) {
    if (md[a] != md[b]) return md[a] < md[b];
    if (m_r[a].size() != m_r[b].size()) return m_r[a].size() > m_r[b].size();
    return a < b;
  });
  rpos.assign(n, 0);
  mpos.assign(std::max(mi, 1), 0);
  for (int p = 0; p < n; ++p) rpos[ro[p]] = (uint16_t)p;
  for (int p = 0; p < mi; ++p) mpos[mo[p]] = (uint16_t)p;
  return EFM_OK;
}

// device copy of the relabelling (owned by the caller: free `mem`)
struct FeatTables {
  efm::FeatDev d{};
  void *mem = nullptr;
  ~FeatTables() {
    if (mem) (void)hipFree(mem);
  }
};

efm_status upload_feat(const efm_network *N, int x, int in_bits, int in_counts, FeatTables &ft) {
  if (x < 0 || x >= N->m || !N->ext[x]) return fail(EFM_EINVAL, "target %d is not an external metabolite", x);
  std::vector<uint16_t> rpos, mpos;
  efm_status rc = relabel(N, x, in_bits, in_counts, rpos, mpos);
  if (rc != EFM_OK) return rc;
  const size_t rb = align256(rpos.size() * 2), mb = align256(mpos.size() * 2);
  char *p = nullptr;
  LCHK(hipMalloc((void **)&p, rb + mb + 256));
  ft.mem = p;
  LCHK(hipMemcpy(p, rpos.data(), rpos.size() * 2, hipMemcpyHostToDevice));
  LCHK(hipMemcpy(p + rb, mpos.data(), mpos.size() * 2, hipMemcpyHostToDevice));
  ft.d = efm::FeatDev{(const uint16_t *)p, (const uint16_t *)(p + rb), in_bits, N->mi};
done:
  return rc;
}

// Training scratch of one minibatch size.
struct TrainBufs {
  int Bp = 0;
  uint16_t *A1 = nullptr, *A1T = nullptr, *DZ2 = nullptr, *DZ2T = nullptr;
  float *loss = nullptr;
  int32_t *idx = nullptr;
  void *mem = nullptr;
  ~TrainBufs() {
    if (mem) (void)hipFree(mem);
  }
  hipError_t alloc(int bp, int64_t nidx) {
    Bp = bp;
    const size_t act = align256((size_t)bp * efm::kH * 2);
    const size_t total = 4 * act + 256 + align256((size_t)nidx * 4);
    char *p = nullptr;
    hipError_t e = hipMalloc((void **)&p, total);
    if (e != hipSuccess) return e;
    mem = p;
    A1 = (uint16_t *)p;
    A1T = (uint16_t *)(p + act);
    DZ2 = (uint16_t *)(p + 2 * act);
    DZ2T = (uint16_t *)(p + 3 * act);
    loss = (float *)(p + 4 * act);
    idx = (int32_t *)(p + 4 * act + 256);
    return hipSuccess;
  }
};

// Forward + backward of one minibatch (gradients accumulate into model->G).
hipError_t run_grad(const efm_model *M, const efm_traces *T, const int32_t *idx, int B, float pw, TrainBufs &tb,
                    hipStream_t s) {
  const int Bp = (B + efm::kTile - 1) / efm::kTile * efm::kTile;
  const efm::ModelDev md = M->dev();
  const int tiles = Bp / efm::kTile;
  const size_t lds_f = 2 * (size_t)(efm::kTile * efm::kH * 2 + efm::kFeatMax * 2 + efm::kTile * efm::kH * 4);
  const size_t lds_b = 2 * (size_t)(efm::kTile * efm::kH * 4 + efm::kFeatMax * 2);
  const unsigned blocks = (unsigned)std::min<int64_t>((tiles + 1) / 2, (int64_t)efm::num_cus_l() * 8);
  hipLaunchKernelGGL(efm::train_fwd_kernel, dim3(blocks), dim3(128), lds_f, s, md, T->d, idx, B, Bp, pw,
                     1.f / (float)B, tb.A1, tb.A1T, tb.DZ2, tb.DZ2T, M->G + M->ow3, M->G + M->ob2, M->G + M->ob3,
                     tb.loss);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(efm::dw2_kernel, dim3(64), dim3(256), 0, s, tb.A1T, tb.DZ2T, Bp, M->G + M->oW2);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(efm::bwd1_kernel, dim3(blocks), dim3(128), lds_b, s, md, T->d, idx, B, Bp, tb.A1, tb.DZ2,
                     M->G + M->oW1, M->G + M->ob1);
  return hipGetLastError();
}

hipError_t refresh_copies(const efm_model *M, hipStream_t s) {
  hipLaunchKernelGGL(efm::copies_kernel, dim3(512), dim3(256), 0, s, M->P, M->map());
  return hipGetLastError();
}

efm_status model_alloc(int in_bits, int in_counts, efm_model **out) {
  efm_status rc = EFM_OK;
  efm_model *M = new (std::nothrow) efm_model;
  if (!M) return fail(EFM_ENOMEM, "host allocation failed");
  M->in_bits = in_bits;
  M->in_counts = in_counts;
  M->F = in_bits + 2 * in_counts;
  const int64_t H = efm::kH;
  M->oW1 = 0;
  M->ob1 = M->oW1 + (int64_t)M->F * H;
  M->oW2 = M->ob1 + H;
  M->ob2 = M->oW2 + H * H;
  M->ow3 = M->ob2 + H;
  M->ob3 = M->ow3 + H;
  M->nparam = M->ob3 + 1;
  {
    const size_t pv = align256((size_t)M->nparam * 4);
    const size_t w1 = align256((size_t)M->F * H * 2), w2 = align256((size_t)H * H * 2), w3 = align256((size_t)H * 2);
    char *p = nullptr;
    LCHK(hipMalloc((void **)&p, 4 * pv + w1 + 2 * w2 + w3));
    M->mem = p;
    M->P = (float *)p;
    M->G = (float *)(p + pv);
    M->M = (float *)(p + 2 * pv);
    M->V = (float *)(p + 3 * pv);
    M->W1b = (uint16_t *)(p + 4 * pv);
    M->W2b = (uint16_t *)(p + 4 * pv + w1);
    M->W2Tb = (uint16_t *)(p + 4 * pv + w1 + w2);
    M->w3b = (uint16_t *)(p + 4 * pv + w1 + 2 * w2);
    LCHK(hipMemset(M->G, 0, pv * 3));
  }
  *out = M;
  return EFM_OK;
done:
  if (M->mem) (void)hipFree(M->mem);
  delete M;
  return rc;
}

// Level hook of the learned ordering: scores the survivors when they exceed the
// budget.
struct LearnHook : LevelHook {
  const efm_model *M = nullptr;
  efm::FeatDev ft{};
  u64 *flag = nullptr;
  bool orders() const override { return true; }
  hipError_t score(const efm_network *N, const efm::DevLevel &L, int64_t nsurv, uint32_t *sscore,
                   hipStream_t s) override {
    efm::ScoreSrc src{};
    return efm::launch_score(N->Wt, N->dn, L, ft, M->dev(), src, nsurv, sscore, nullptr, flag, s);
  }
};

// Level hook of trace collection: labels and samples every new frontier.
struct TraceHook : LevelHook {
  efm_traces *T = nullptr;
  efm::FeatDev ft{};
  const u64 *found = nullptr;
  int64_t nf = 0;
  uint8_t *lab = nullptr;
  int64_t lab_cap = 0;
  u64 *npos_d = nullptr;
  double neg_per_pos = 4.0;
  int64_t neg_min = 64;
  int64_t pos_max = 0;
  u64 seed = 0;
  efm_trace_info info{};
  ~TraceHook() override {
    if (lab) (void)hipFree(lab);
  }
  efm_status frontier(const efm_network *N, const u64 *keys, const u64 *hash, int64_t fcap, int64_t count, int level,
                      hipStream_t s) override {
    efm_status rc = EFM_OK;
    u64 npos = 0;
    if (count <= 0) return EFM_OK;
    if (count > lab_cap) {
      if (lab) (void)hipFree(lab);
      lab = nullptr;
      LCHK(hipMalloc((void **)&lab, (size_t)count));
      lab_cap = count;
    }
    LCHK(hipMemsetAsync(npos_d, 0, 8, s));
    LCHK(efm::launch_trace(N->Wt, N->dn, ft, keys, hash, fcap, count, found, nf, lab, npos_d, 0, 0, 0, 0, T->d, s));
    LCHK(hipMemcpyAsync(&npos, npos_d, 8, hipMemcpyDeviceToHost, s));
    LCHK(hipStreamSynchronize(s));
    {
      auto threshold = [](double p) -> u64 {
        if (p >= 1.0) return ~0ull;
        return p > 0.0 ? (u64)(p * 18446744073709551616.0) : 0ull;
      };
      const double kept_pos = pos_max > 0 ? std::min<double>((double)npos, (double)pos_max) : (double)npos;
      const double p_pos = npos > 0 ? kept_pos / (double)npos : 0.0;
      const int64_t nneg = count - (int64_t)npos;
      const double want = std::max((double)neg_min, neg_per_pos * kept_pos);
      const double p = nneg > 0 ? std::min(1.0, want / (double)nneg) : 0.0;
      const u64 thr = threshold(p), thr_pos = threshold(p_pos);
      const u64 salt = seed ^ ((u64)(level + 1) * 0x9E3779B97F4A7C15ull);
      if (thr_pos > 0 || thr > 0)
        LCHK(efm::launch_trace(N->Wt, N->dn, ft, keys, hash, fcap, count, found, nf, lab, npos_d, 1, thr, thr_pos,
                               salt, T->d, s));
    }
    info.states += count;
    info.positives += (int64_t)npos;
  done:
    return rc;
  }
};

}  // namespace

extern "C" {

// ------------------------------------------------------------------- traces

efm_status efm_traces_create(int32_t in_bits, int32_t in_counts, int64_t capacity, efm_traces **out) {
  if (!out) return fail(EFM_EINVAL, "null pointer");
  if (in_bits <= 0 || in_bits > EFM_MAX_RXN || in_counts <= 0 || in_counts > efm::kMaxCounts || capacity <= 0)
    return fail(EFM_EINVAL, "bad trace dimensions");
  efm_status rc = EFM_OK;
  efm_traces *T = new (std::nothrow) efm_traces;
  if (!T) return fail(EFM_ENOMEM, "host allocation failed");
  T->in_bits = in_bits;
  T->in_counts = in_counts;
  T->cap = capacity;
  {
    const size_t e = align256((size_t)capacity * efm::kFeatMax * 2), l = align256((size_t)capacity * 2),
                 b = align256((size_t)capacity), k = align256((size_t)capacity * efm::kTraceW * 8);
    char *p = nullptr;
    LCHK(hipMalloc((void **)&p, e + l + b + k + 256));
    T->mem = p;
    T->d.ent = (uint16_t *)p;
    T->d.len = (uint16_t *)(p + e);
    T->d.lab = (uint8_t *)(p + e + l);
    T->d.keys = (u64 *)(p + e + l + b);
    T->d.ctr = (u64 *)(p + e + l + b + k);
    T->d.cap = capacity;
    LCHK(hipMemset(T->d.ctr, 0, 256));
  }
  *out = T;
  return EFM_OK;
done:
  if (T->mem) (void)hipFree(T->mem);
  delete T;
  return rc;
}

efm_status efm_traces_destroy(efm_traces *T) {
  if (!T) return EFM_OK;
  if (T->mem) (void)hipFree(T->mem);
  delete T;
  return EFM_OK;
}

efm_status efm_traces_info(const efm_traces *T, int64_t *count, int64_t *positives) {
  if (!T) return fail(EFM_EINVAL, "null traces");
  if (count) *count = T->count;
  if (positives) *positives = T->positives;
  return EFM_OK;
}

efm_status efm_traces_append(efm_traces *T, const uint16_t *entries, const uint16_t *lengths, const uint8_t *labels,
                             int64_t count) {
  if (!T || (count > 0 && (!entries || !lengths || !labels))) return fail(EFM_EINVAL, "null pointer");
  if (count < 0) return fail(EFM_EINVAL, "negative count");
  if (T->count + count > T->cap) return fail(EFM_ENOMEM, "traces full (%lld records)", (long long)T->cap);
  const int F = T->in_bits + 2 * T->in_counts;
  int64_t pos = 0;
  for (int64_t i = 0; i < count; ++i) {
    if (lengths[i] > efm::kFeatMax) return fail(EFM_EINVAL, "record %lld longer than EFM_FEAT_MAX", (long long)i);
    for (int e = 0; e < lengths[i]; ++e) {
      const uint16_t v = entries[i * efm::kFeatMax + e];
      if ((int)(v >> 4) >= F) return fail(EFM_EINVAL, "record %lld has an entry beyond the model input", (long long)i);
      if ((v & 15u) > 7u) return fail(EFM_EINVAL, "record %lld has an entry code above 7", (long long)i);
    }
    pos += labels[i] ? 1 : 0;
  }
  efm_status rc = EFM_OK;
  {
    const int64_t c0 = T->count;
    const u64 pos_total = (u64)(T->positives + pos);
    std::vector<uint8_t> lab(labels, labels + count);
    for (auto &v : lab) v = v ? 1 : 0;
    LCHK(hipMemcpy(T->d.ent + c0 * efm::kFeatMax, entries, (size_t)count * efm::kFeatMax * 2, hipMemcpyHostToDevice));
    LCHK(hipMemcpy(T->d.len + c0, lengths, (size_t)count * 2, hipMemcpyHostToDevice));
    LCHK(hipMemcpy(T->d.lab + c0, lab.data(), (size_t)count, hipMemcpyHostToDevice));
    LCHK(hipMemset(T->d.keys + c0 * efm::kTraceW, 0, (size_t)count * efm::kTraceW * 8));
    const u64 c1 = (u64)(c0 + count);
    LCHK(hipMemcpy(T->d.ctr, &c1, 8, hipMemcpyHostToDevice));
    LCHK(hipMemcpy(T->d.ctr + 2, &pos_total, 8, hipMemcpyHostToDevice));
    T->count = c0 + count;
    T->positives += pos;
  }
done:
  return rc;
}

efm_status efm_traces_fetch(const efm_traces *T, int64_t first, int64_t count, uint16_t *entries, uint16_t *lengths,
                            uint8_t *labels, uint64_t *keys) {
  if (!T) return fail(EFM_EINVAL, "null traces");
  if (first < 0 || count < 0 || first + count > T->count) return fail(EFM_EINVAL, "record range out of bounds");
  efm_status rc = EFM_OK;
  if (entries)
    LCHK(hipMemcpy(entries, T->d.ent + first * efm::kFeatMax, (size_t)count * efm::kFeatMax * 2,
                   hipMemcpyDeviceToHost));
  if (lengths) LCHK(hipMemcpy(lengths, T->d.len + first, (size_t)count * 2, hipMemcpyDeviceToHost));
  if (labels) LCHK(hipMemcpy(labels, T->d.lab + first, (size_t)count, hipMemcpyDeviceToHost));
  if (keys)
    LCHK(hipMemcpy(keys, T->d.keys + first * efm::kTraceW, (size_t)count * efm::kTraceW * 8, hipMemcpyDeviceToHost));
done:
  return rc;
}

efm_status efm_trace_collect(efm_traces *T, const efm_network *N, int32_t target, const efm_enum_opts *opts,
                             const efm_trace_opts *topts, efm_trace_info *info) {
  if (!T || !N) return fail(EFM_EINVAL, "null pointer");
  efm_status rc = EFM_OK;
  FeatTables ft;
  efm_result *R1 = nullptr, *R2 = nullptr;
  u64 *dev = nullptr;
  TraceHook hook;
  u64 ctr[3] = {0, 0, 0};
  rc = upload_feat(N, target, T->in_bits, T->in_counts, ft);
  if (rc != EFM_OK) return rc;
  rc = enumerate_impl(N, target, opts, nullptr, &R1);
  if (rc != EFM_OK) return rc;
  {
    const int Wt = N->Wt, W = R1->W;
    const int64_t nf = R1->count;
    std::vector<u64> fk((size_t)std::max<int64_t>(nf, 1) * Wt, 0);
    for (int64_t f = 0; f < nf; ++f)
      for (int w = 0; w < W; ++w) fk[(size_t)f * Wt + w] = R1->keys[(size_t)f * W + w];
    LCHK(hipMalloc((void **)&dev, fk.size() * 8 + 256));
    LCHK(hipMemcpy(dev, fk.data(), fk.size() * 8, hipMemcpyHostToDevice));
    hook.T = T;
    hook.ft = ft.d;
    hook.found = dev;
    hook.nf = nf;
    hook.npos_d = dev + fk.size();
    if (topts) {
      if (topts->neg_per_pos > 0) hook.neg_per_pos = topts->neg_per_pos;
      if (topts->neg_min > 0) hook.neg_min = topts->neg_min;
      if (topts->pos_max > 0) hook.pos_max = topts->pos_max;
      hook.seed = topts->seed;
    }
    rc = enumerate_impl(N, target, opts, &hook, &R2);
    if (rc != EFM_OK) goto done;
    LCHK(hipMemcpy(ctr, T->d.ctr, 24, hipMemcpyDeviceToHost));
    const int64_t before = T->count;
    T->count = std::min<int64_t>((int64_t)ctr[0], T->cap);
    T->positives = (int64_t)ctr[2];
    hook.info.recorded = T->count - before;
    hook.info.pathways = nf;
    hook.info.status = R1->status;
    if (info) *info = hook.info;
    if (ctr[1] & efm::kFlagFeatOverflow) {
      rc = fail(EFM_EINVAL, "a partial pathway has more than EFM_FEAT_MAX input entries");
      goto done;
    }
    if (ctr[1] & efm::kFlagQueueOverflow) {
      const u64 c = (u64)T->count;
      (void)hipMemcpy(T->d.ctr, &c, 8, hipMemcpyHostToDevice);
      rc = fail(EFM_ENOMEM, "traces full (%lld records)", (long long)T->cap);
      goto done;
    }
  }
done:
  if (dev) (void)hipFree(dev);
  if (R1) efm_result_destroy(R1);
  if (R2) efm_result_destroy(R2);
  return rc;
}

// -------------------------------------------------------------------- model

efm_status efm_model_create(int32_t in_bits, int32_t in_counts, int32_t hidden, uint64_t seed, efm_model **out) {
  if (!out) return fail(EFM_EINVAL, "null pointer");
  if (hidden != efm::kH) return fail(EFM_EINVAL, "hidden must be %d", efm::kH);
  if (in_bits <= 0 || in_bits > EFM_MAX_RXN || in_counts <= 0 || in_counts > efm::kMaxCounts)
    return fail(EFM_EINVAL, "bad model input dimensions");
  efm_model *M = nullptr;
  efm_status rc = model_alloc(in_bits, in_counts, &M);
  if (rc != EFM_OK) return rc;
  {
    std::vector<float> P((size_t)M->nparam, 0.f);
    u64 st = seed;
    auto uni = [&](double a) { return (float)(a * (2.0 * ((double)(sm64(st) >> 11) * 0x1.0p-53) - 1.0)); };
    const double a1 = std::sqrt(6.0 / 32.0), a2 = std::sqrt(6.0 / efm::kH);
    for (int64_t i = 0; i < (int64_t)M->F * efm::kH; ++i) P[M->oW1 + i] = uni(a1);
    for (int64_t i = 0; i < (int64_t)efm::kH * efm::kH; ++i) P[M->oW2 + i] = uni(a2);
    for (int64_t i = 0; i < efm::kH; ++i) P[M->ow3 + i] = uni(a2);
    LCHK(hipMemcpy(M->P, P.data(), P.size() * 4, hipMemcpyHostToDevice));
    LCHK(refresh_copies(M, nullptr));
    LCHK(hipDeviceSynchronize());
  }
  *out = M;
  return EFM_OK;
done:
  efm_model_destroy(M);
  return rc;
}

efm_status efm_model_destroy(efm_model *M) {
  if (!M) return EFM_OK;
  if (M->mem) (void)hipFree(M->mem);
  delete M;
  return EFM_OK;
}

efm_status efm_model_info(const efm_model *M, int64_t *n_params, int32_t *in_bits, int32_t *in_counts,
                          int32_t *hidden) {
  if (!M) return fail(EFM_EINVAL, "null model");
  if (n_params) *n_params = M->nparam;
  if (in_bits) *in_bits = M->in_bits;
  if (in_counts) *in_counts = M->in_counts;
  if (hidden) *hidden = efm::kH;
  return EFM_OK;
}

efm_status efm_model_get_params(const efm_model *M, float *dst, int64_t len) {
  if (!M || !dst) return fail(EFM_EINVAL, "null pointer");
  if (len < M->nparam) return fail(EFM_EINVAL, "buffer of %lld floats, %lld needed", (long long)len,
                                   (long long)M->nparam);
  efm_status rc = EFM_OK;
  LCHK(hipMemcpy(dst, M->P, (size_t)M->nparam * 4, hipMemcpyDeviceToHost));
done:
  return rc;
}

efm_status efm_model_set_params(efm_model *M, const float *src, int64_t len) {
  if (!M || !src) return fail(EFM_EINVAL, "null pointer");
  if (len != M->nparam) return fail(EFM_EINVAL, "%lld floats given, %lld expected", (long long)len,
                                    (long long)M->nparam);
  efm_status rc = EFM_OK;
  for (int64_t i = 0; i < len; ++i)
    if (!std::isfinite(src[i])) return fail(EFM_EINVAL, "parameter %lld is not finite", (long long)i);
  LCHK(hipMemcpy(M->P, src, (size_t)len * 4, hipMemcpyHostToDevice));
  LCHK(hipMemset(M->G, 0, (size_t)len * 4));
  LCHK(hipMemset(M->M, 0, (size_t)len * 4));
  LCHK(hipMemset(M->V, 0, (size_t)len * 4));
  M->step = 0;
  LCHK(refresh_copies(M, nullptr));
  LCHK(hipDeviceSynchronize());
done:
  return rc;
}

static const char kMagic[8] = {'E', 'F', 'M', 'M', 'L', 'P', '0', '1'};

efm_status efm_model_save(const efm_model *M, const char *path) {
  if (!M || !path) return fail(EFM_EINVAL, "null pointer");
  efm_status rc = EFM_OK;
  std::vector<float> buf((size_t)M->nparam * 3);
  FILE *f = nullptr;
  LCHK(hipMemcpy(buf.data(), M->P, (size_t)M->nparam * 4, hipMemcpyDeviceToHost));
  LCHK(hipMemcpy(buf.data() + M->nparam, M->M, (size_t)M->nparam * 4, hipMemcpyDeviceToHost));
  LCHK(hipMemcpy(buf.data() + 2 * M->nparam, M->V, (size_t)M->nparam * 4, hipMemcpyDeviceToHost));
  f = fopen(path, "wb");
  if (!f) return fail(EFM_EINVAL, "cannot open %s for writing", path);
  {
    const int32_t hdr[4] = {M->in_bits, M->in_counts, efm::kH, 0};
    const int64_t h2[2] = {M->step, M->nparam};
    bool ok = fwrite(kMagic, 1, 8, f) == 8 && fwrite(hdr, 4, 4, f) == 4 && fwrite(h2, 8, 2, f) == 2 &&
              fwrite(buf.data(), 4, buf.size(), f) == buf.size();
    ok = (fclose(f) == 0) && ok;
    if (!ok) rc = fail(EFM_EINVAL, "write to %s failed", path);
  }
done:
  return rc;
}

efm_status efm_model_load(const char *path, efm_model **out) {
  if (!path || !out) return fail(EFM_EINVAL, "null pointer");
  FILE *f = fopen(path, "rb");
  if (!f) return fail(EFM_EINVAL, "cannot open %s", path);
  char mg[8];
  int32_t hdr[4];
  int64_t h2[2];
  const bool ok = fread(mg, 1, 8, f) == 8 && memcmp(mg, kMagic, 8) == 0 && fread(hdr, 4, 4, f) == 4 &&
                  fread(h2, 8, 2, f) == 2;
  if (!ok || hdr[2] != efm::kH || hdr[0] <= 0 || hdr[0] > EFM_MAX_RXN || hdr[1] <= 0 || hdr[1] > efm::kMaxCounts) {
    fclose(f);
    return fail(EFM_EINVAL, "%s is not a model file", path);
  }
  efm_model *M = nullptr;
  efm_status rc = model_alloc(hdr[0], hdr[1], &M);
  if (rc != EFM_OK) {
    fclose(f);
    return rc;
  }
  std::vector<float> buf((size_t)M->nparam * 3);
  if (h2[1] != M->nparam || fread(buf.data(), 4, buf.size(), f) != buf.size()) {
    fclose(f);
    efm_model_destroy(M);
    return fail(EFM_EINVAL, "%s is truncated", path);
  }
  fclose(f);
  M->step = h2[0];
  LCHK(hipMemcpy(M->P, buf.data(), (size_t)M->nparam * 4, hipMemcpyHostToDevice));
  LCHK(hipMemcpy(M->M, buf.data() + M->nparam, (size_t)M->nparam * 4, hipMemcpyHostToDevice));
  LCHK(hipMemcpy(M->V, buf.data() + 2 * M->nparam, (size_t)M->nparam * 4, hipMemcpyHostToDevice));
  LCHK(refresh_copies(M, nullptr));
  LCHK(hipDeviceSynchronize());
  *out = M;
  return EFM_OK;
done:
  efm_model_destroy(M);
  return rc;
}

efm_status efm_model_score(const efm_model *M, const efm_traces *T, int64_t first, int64_t count, float *scores) {
  if (!M || !T || (count > 0 && !scores)) return fail(EFM_EINVAL, "null pointer");
  if (T->in_bits != M->in_bits || T->in_counts != M->in_counts)
    return fail(EFM_EINVAL, "trace and model inputs differ");
  if (first < 0 || count < 0 || first + count > T->count) return fail(EFM_EINVAL, "record range out of bounds");
  if (count == 0) return EFM_OK;
  efm_status rc = EFM_OK;
  float *d = nullptr;
  LCHK(hipMalloc((void **)&d, (size_t)count * 4 + 256));
  {
    efm::ScoreSrc src{};
    src.mode = 2;
    src.tr = T->d;
    src.first = first;
    efm::FeatDev ft{};
    efm::DevNet dn{};
    efm::DevLevel L{};
    LCHK(efm::launch_score(1, dn, L, ft, M->dev(), src, count, nullptr, d, nullptr, nullptr));
    LCHK(hipMemcpy(scores, d, (size_t)count * 4, hipMemcpyDeviceToHost));
  }
done:
  if (d) (void)hipFree(d);
  return rc;
}

efm_status efm_model_score_keys(const efm_model *M, const efm_network *N, int32_t target, const uint64_t *keys,
                                int64_t count, float *scores) {
  if (!M || !N || (count > 0 && (!keys || !scores))) return fail(EFM_EINVAL, "null pointer");
  if (count < 0) return fail(EFM_EINVAL, "negative count");
  FeatTables ft;
  efm_status rc = upload_feat(N, target, M->in_bits, M->in_counts, ft);
  if (rc != EFM_OK) return rc;
  if (count == 0) return EFM_OK;
  char *d = nullptr;
  u64 flag = 0;
  const size_t kb = align256((size_t)count * N->W * 8), sb = align256((size_t)count * 4);
  LCHK(hipMalloc((void **)&d, kb + sb + 256));
  LCHK(hipMemcpy(d, keys, (size_t)count * N->W * 8, hipMemcpyHostToDevice));
  LCHK(hipMemset(d + kb + sb, 0, 8));
  {
    efm::ScoreSrc src{};
    src.mode = 1;
    src.keys = (const u64 *)d;
    src.kw = N->W;
    efm::DevLevel L{};
    LCHK(efm::launch_score(N->Wt, N->dn, L, ft.d, M->dev(), src, count, nullptr, (float *)(d + kb),
                           (u64 *)(d + kb + sb), nullptr));
    LCHK(hipMemcpy(scores, d + kb, (size_t)count * 4, hipMemcpyDeviceToHost));
    LCHK(hipMemcpy(&flag, d + kb + sb, 8, hipMemcpyDeviceToHost));
    if (flag & efm::kFlagFeatOverflow) rc = fail(EFM_EINVAL, "a partial pathway has more than EFM_FEAT_MAX entries");
  }
done:
  if (d) (void)hipFree(d);
  return rc;
}

efm_status efm_model_grad(const efm_model *M, const efm_traces *T, int64_t first, int64_t count, float pos_weight,
                          float *grad, double *loss) {
  if (!M || !T || !grad) return fail(EFM_EINVAL, "null pointer");
  if (T->in_bits != M->in_bits || T->in_counts != M->in_counts)
    return fail(EFM_EINVAL, "trace and model inputs differ");
  if (first < 0 || count <= 0 || count > efm::kMaxBatch || first + count > T->count)
    return fail(EFM_EINVAL, "record range out of bounds (1..%d records)", efm::kMaxBatch);
  efm_status rc = EFM_OK;
  TrainBufs tb;
  float ls = 0.f;
  std::vector<int32_t> idx((size_t)count);
  for (int64_t i = 0; i < count; ++i) idx[i] = (int32_t)(first + i);
  LCHK(tb.alloc((int)((count + efm::kTile - 1) / efm::kTile * efm::kTile), count));
  LCHK(hipMemcpy(tb.idx, idx.data(), (size_t)count * 4, hipMemcpyHostToDevice));
  LCHK(hipMemset(M->G, 0, (size_t)M->nparam * 4));
  LCHK(hipMemset(tb.loss, 0, 4));
  LCHK(run_grad(M, T, tb.idx, (int)count, pos_weight, tb, nullptr));
  LCHK(hipMemcpy(grad, M->G, (size_t)M->nparam * 4, hipMemcpyDeviceToHost));
  LCHK(hipMemcpy(&ls, tb.loss, 4, hipMemcpyDeviceToHost));
  LCHK(hipMemset(M->G, 0, (size_t)M->nparam * 4));
  if (loss) *loss = (double)ls / (double)count;
done:
  return rc;
}

efm_status efm_model_train(efm_model *M, const efm_traces *T, const efm_train_opts *opts, efm_train_stats *stats) {
  if (!M || !T) return fail(EFM_EINVAL, "null pointer");
  if (T->in_bits != M->in_bits || T->in_counts != M->in_counts)
    return fail(EFM_EINVAL, "trace and model inputs differ");
  if (T->count <= 0) return fail(EFM_EINVAL, "no trace records");
  efm_train_opts o{};
  if (opts) o = *opts;
  const int epochs = o.epochs > 0 ? o.epochs : 1;
  const int batch = (int)std::min<int64_t>(o.batch > 0 ? o.batch : 1024, efm::kMaxBatch);
  const float lr = o.lr > 0 ? o.lr : 1e-3f, b1 = o.beta1 > 0 ? o.beta1 : 0.9f, b2 = o.beta2 > 0 ? o.beta2 : 0.999f,
              eps = o.eps > 0 ? o.eps : 1e-8f;
  float pw = o.pos_weight;
  if (pw <= 0) {
    const int64_t np = std::max<int64_t>(T->positives, 1), nn = std::max<int64_t>(T->count - T->positives, 1);
    pw = (float)std::min(1e4, std::max(1.0, (double)nn / (double)np));
  }
  hipStream_t s = (hipStream_t)o.stream;
  efm_status rc = EFM_OK;
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t n = T->count;
  TrainBufs tb;
  std::vector<int32_t> perm((size_t)n);
  efm_train_stats st{};
  u64 rs = o.seed;
  LCHK(tb.alloc((batch + efm::kTile - 1) / efm::kTile * efm::kTile, n));
  for (int ep = 0; ep < epochs; ++ep) {
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; --i) {      // Fisher-Yates
      const int64_t j = (int64_t)(sm64(rs) % (u64)(i + 1));
      std::swap(perm[i], perm[j]);
    }
    LCHK(hipMemcpyAsync(tb.idx, perm.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
    LCHK(hipMemsetAsync(tb.loss, 0, 4, s));
    for (int64_t b0 = 0; b0 < n; b0 += batch) {
      const int B = (int)std::min<int64_t>(batch, n - b0);
      LCHK(run_grad(M, T, tb.idx + b0, B, pw, tb, s));
      M->step++;
      st.steps++;
      const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, (double)M->step)));
      const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, (double)M->step)));
      const unsigned blocks = (unsigned)std::min<int64_t>((M->nparam + 255) / 256, (int64_t)efm::num_cus_l() * 8);
      hipLaunchKernelGGL(efm::adam_kernel, dim3(blocks), dim3(256), 0, s, M->P, M->G, M->M, M->V, M->map(), lr, b1,
                         b2, eps, c1, c2);
      LCHK(hipGetLastError());
    }
    float ls = 0.f;
    LCHK(hipMemcpyAsync(&ls, tb.loss, 4, hipMemcpyDeviceToHost, s));
    LCHK(hipStreamSynchronize(s));
    if (ep == 0) st.loss_first = (double)ls / (double)n;
    st.loss_last = (double)ls / (double)n;
  }
  st.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (stats) *stats = st;
done:
  return rc;
}

efm_status efm_enumerate_learned(const efm_network *N, int32_t target, int64_t budget, const efm_model *M,
                                 const efm_enum_opts *opts, efm_result **out) {
  if (!N || !M || !out) return fail(EFM_EINVAL, "null pointer");
  if (budget <= 0) return fail(EFM_EINVAL, "budget must be positive");
  FeatTables ft;
  efm_status rc = upload_feat(N, target, M->in_bits, M->in_counts, ft);
  if (rc != EFM_OK) return rc;
  efm_enum_opts o{};
  if (opts) o = *opts;
  o.frontier_cap = budget;
  o.flags |= EFM_OPT_LEARNED;
  u64 *flag = nullptr;
  u64 fl = 0;
  efm_result *R = nullptr;
  LearnHook hook;
  LCHK(hipMalloc((void **)&flag, 256));
  LCHK(hipMemsetAsync(flag, 0, 8, (hipStream_t)o.stream));
  hook.M = M;
  hook.ft = ft.d;
  hook.flag = flag;
  rc = enumerate_impl(N, target, &o, &hook, &R);
  if (rc != EFM_OK) goto done;
  LCHK(hipMemcpy(&fl, flag, 8, hipMemcpyDeviceToHost));
  if (fl & efm::kFlagFeatOverflow) {
    rc = fail(EFM_EINVAL, "a partial pathway has more than EFM_FEAT_MAX model input entries");
    goto done;
  }
  *out = R;
  R = nullptr;
done:
  if (R) efm_result_destroy(R);
  if (flag) (void)hipFree(flag);
  return rc;
}

}  // extern "C"

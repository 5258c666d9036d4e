// Kernels of the sweep-correction network: periodic width-5 convolutions over space as
// implicit GEMMs on the matrix cores, its training (loss, backward passes, weight gradients,
// Adam) and its in-place application to an Lhat^{-T} sweep output.
//
// Convolution (64 output channels): one workgroup of 4 waves takes a tile of 64 grid points of
// one sample, stages the 68 input rows it reads (periodic wrap inside the sample) in LDS, and
// wave w produces output channels 16w..16w+15 for all 64 points: its 16 x (5 CIN) slice of the
// weights stays in registers for the whole launch, the input fragments come from LDS.  The
// contraction index is k = t * CIN + ci (tap t, input channel ci), so every lane's operand is
// a run of consecutive channels of one staged row.  float32 uses v_mfma_f32_16x16x4f32 (one
// value per lane), bfloat16 v_mfma_f32_16x16x16bf16_1k (four per lane); both accumulate in
// float32 and return element e of lane group q as row 4 q + e of the 16 x 16 tile.
//
// Weight gradients (float32): rows = output channel, columns = k, contraction over the grid
// points of the workgroup's tiles; partial sums per workgroup are reduced in a fixed order.
#include <hip/hip_runtime.h>

#include "lanes.h"
#include "net.h"

namespace svar {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

static constexpr int GRID_CAP = 1024;
int net_grid_cap() { return GRID_CAP; }
static_assert(NET_CIN1 == 16 || NET_CIN1 == 32, "layer-1 kernels are instantiated for 16 or 32 channels");

__device__ __forceinline__ uint16_t f2bf(float f) {  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

template <typename E> __device__ __forceinline__ E to_e(float v);
template <> __device__ __forceinline__ float to_e<float>(float v) { return v; }
template <> __device__ __forceinline__ uint16_t to_e<uint16_t>(float v) { return f2bf(v); }
template <typename E> __device__ __forceinline__ float to_f(E v);
template <> __device__ __forceinline__ float to_f<float>(float v) { return v; }
template <> __device__ __forceinline__ float to_f<uint16_t>(uint16_t v) { return bf2f(v); }

__device__ __forceinline__ int wrap(int p, int s) {
  p %= s;
  return p < 0 ? p + s : p;
}

// ------------------------------------------------------------------ MFMA traits
template <typename E> struct NetMma;
template <> struct NetMma<float> {
  static constexpr int KS = 4;  // contraction length of one instruction
  typedef float frag;
  static __device__ __forceinline__ v4f mma(frag a, frag b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ frag ld(const float* p) { return *p; }
};
template <> struct NetMma<uint16_t> {
  static constexpr int KS = 16;
  typedef v4s frag;
  static __device__ __forceinline__ v4f mma(frag a, frag b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ frag ld(const uint16_t* p) { return *(const v4s*)p; }
};

// bfloat16 with a 32-long contraction per instruction (v_mfma_f32_16x16x32_bf16: lane l holds
// A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16], j < 8; result row 4 (l / 16) + e, as
// checked on the device against a host product); used where the contraction length is a
// multiple of 32 (64 input channels)
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
struct NetMma32 {
  static constexpr int KS = 32;
  typedef bf8 frag;
  static __device__ __forceinline__ v4f mma(frag a, frag b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ frag ld(const uint16_t* p) { return *(const bf8*)p; }
};
template <typename E, int CIN> struct ConvMma { typedef NetMma<E> type; };
template <> struct ConvMma<uint16_t, 64> { typedef NetMma32 type; };

// LDS row strides (elements), chosen so that the 16 rows read by one lane group fall in
// distinct banks and every row starts on an 8-byte (16-byte for 16-byte reads) boundary
template <typename E, int CIN> struct ConvStride;
template <> struct ConvStride<float, 16> { static constexpr int v = 18; };
template <> struct ConvStride<float, 32> { static constexpr int v = 34; };
template <> struct ConvStride<float, 64> { static constexpr int v = 66; };
template <> struct ConvStride<uint16_t, 16> { static constexpr int v = 20; };
template <> struct ConvStride<uint16_t, 32> { static constexpr int v = 36; };
template <> struct ConvStride<uint16_t, 64> { static constexpr int v = 72; };

// ------------------------------------------------------------------ parameters
__global__ void k_net_pack(const float* __restrict__ th, NetLayout L, NetWeights W) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // layers 1..3, kernel layout [co][t * CIN + ci]
  for (int l = 0; l < 3; ++l) {
    const int CIN = l == 0 ? NET_CIN1 : NET_C;
    const int cin = l == 0 ? L.cin : NET_C;
    if (e < (int64_t)NET_C * NET_W * CIN) {
      const int co = (int)(e / (NET_W * CIN)), kk = (int)(e % (NET_W * CIN));
      const int t = kk / CIN, ci = kk % CIN;
      const float v = ci < cin ? th[L.w[l] + ((int64_t)co * cin + ci) * NET_W + t] : 0.0f;
      W.wf[l][e] = v;
      W.wb[l][e] = f2bf(v);
    }
  }
  // layers 2, 3 transposed and tap-reversed for the backward pass: [ci][t' * 64 + co]
  for (int l = 1; l < 3; ++l) {
    if (e < (int64_t)NET_C * NET_W * NET_C) {
      const int ci = (int)(e / (NET_W * NET_C)), kk = (int)(e % (NET_W * NET_C));
      const int tp = kk / NET_C, co = kk % NET_C;
      W.wflip[l - 1][e] = th[L.w[l] + ((int64_t)co * NET_C + ci) * NET_W + (NET_W - 1 - tp)];
    }
  }
  if (e < NET_W * NET_C) {
    const int t = (int)(e / NET_C), c = (int)(e % NET_C);
    W.w4[e] = th[L.w[3] + (int64_t)c * NET_W + t];
  }
}

// ------------------------------------------------------------------ per-system scale
__global__ __launch_bounds__(256) void k_net_sumsq(const double* __restrict__ v,
                                                   const NetChunk* __restrict__ ch,
                                                   double* __restrict__ part,
                                                   const int* __restrict__ skip) {
  __shared__ double red[4];
  if (skip && *skip) return;
  const NetChunk c = ch[blockIdx.x];
  double acc = 0.0;
  for (int64_t e = c.e0 + threadIdx.x; e < c.e1; e += 256) {
    const double x = v[e];
    acc += x * x;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// sigma = rms over the system (chunk0[sys] .. chunk0[sys + 1] hold its chunks, whose element
// counts sum to the system length stored in chunk0's companion: the last chunk's e1 - first e0)
__global__ void k_net_sigma(const double* __restrict__ part, const int32_t* __restrict__ chunk0,
                            const NetChunk* __restrict__ ch, int nsys, double* __restrict__ sigma,
                            double* __restrict__ inv_sigma, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsys) return;
  const int c0 = chunk0[i], c1 = chunk0[i + 1];
  double acc = 0.0;
  for (int c = c0; c < c1; ++c) acc += part[c];
  const double len = c1 > c0 ? (double)(ch[c1 - 1].e1 - ch[c0].e0) : 1.0;
  const double sg = sqrt(acc / len);
  sigma[i] = sg;
  inv_sigma[i] = sg > 0.0 ? 1.0 / sg : 0.0;
}

__global__ void k_net_norm_pairs(const double* __restrict__ chat, const double* __restrict__ cex,
                                 const double* __restrict__ inv, int64_t len, int npair,
                                 float* __restrict__ x, float* __restrict__ y) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len * npair) return;
  const double is = inv[e / len];
  const double a = chat[e];
  x[e] = (float)(a * is);
  y[e] = (float)((cex[e] - a) * is);
}

// ------------------------------------------------------------------ layer-1 features
// channel 0: own block; 1..S: block e + 1 + m k (zero past the last block); 1+S+(e-blk): 1
template <typename E, typename SRC>
__global__ __launch_bounds__(64) void k_net_feat(const SRC* __restrict__ src,
                                                 const double* __restrict__ inv_sigma,
                                                 const NetSample* __restrict__ smp,
                                                 const NetTile* __restrict__ tiles,
                                                 int64_t row_base, int k, int S,
                                                 E* __restrict__ X0,
                                                 const int* __restrict__ skip,
                                                 const int* __restrict__ off) {
  if (skip && *skip) return;
  const NetTile T = tiles[blockIdx.x];
  const NetSample P = smp[T.sample];
  if (off && off[P.sys]) return;  // switched off: the correction is not applied
  const int pos = T.pos0 + threadIdx.x;
  if (pos >= P.s) return;
  const double isg = inv_sigma ? inv_sigma[P.sys] : 1.0;
  const int e = min((P.blk / k) * k + k - 1, P.nb - 1);
  const int hot = 1 + S + (e - P.blk);
  alignas(16) E vals[NET_CIN1];
#pragma unroll
  for (int c = 0; c < NET_CIN1; ++c) {
    float v = 0.0f;
    if (c == 0) {
      v = (float)((double)src[P.src + (int64_t)P.blk * P.s + pos] * isg);
    } else if (c <= S) {
      const int b = e + 1 + (c - 1) * k;
      if (b < P.nb) v = (float)((double)src[P.src + (int64_t)b * P.s + pos] * isg);
    } else if (c == hot) {
      v = 1.0f;
    }
    vals[c] = to_e<E>(v);
  }
  // the row (16 channels) is written as 16-byte pieces
  uint4* o = (uint4*)(X0 + (P.row0 - row_base + pos) * NET_CIN1);
  const uint4* vv = (const uint4*)vals;
#pragma unroll
  for (int i = 0; i < NET_CIN1 * (int)sizeof(E) / 16; ++i) o[i] = vv[i];
}

// ------------------------------------------------------------------ convolution, 64 outputs
template <typename E, int CIN, int BWD>
__global__ __launch_bounds__(256) void k_net_conv(const E* __restrict__ in, E* __restrict__ out,
                                                  const E* __restrict__ W,
                                                  const float* __restrict__ bias,
                                                  const float* __restrict__ mask,
                                                  const NetSample* __restrict__ smp,
                                                  const NetTile* __restrict__ tiles, int ntiles,
                                                  int64_t row_base,
                                                  const int* __restrict__ skip,
                                                  const int* __restrict__ off) {
  typedef typename ConvMma<E, CIN>::type MM;
  constexpr int EPL = MM::KS / 4;            // operand elements per lane
  constexpr int NKS = NET_W * CIN / MM::KS;  // contraction steps
  constexpr int STR = ConvStride<E, CIN>::v;
  constexpr int CPR = CIN * (int)sizeof(E) / 8;  // 8-byte pieces per row
  __shared__ __align__(16) E tile[NET_ROWS * STR];
  if (skip && *skip) return;
  const int lane = threadIdx.x & 63, q = lane >> 4, r16 = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int co = wave * 16 + r16;
  typename MM::frag bw[NKS];
#pragma unroll
  for (int ks = 0; ks < NKS; ++ks)
    bw[ks] = MM::ld(W + (int64_t)co * (NET_W * CIN) + ks * MM::KS + q * EPL);
  const float bco = BWD ? 0.0f : bias[co];
  // the input rows of the next tile are loaded into registers while the current tile's
  // MFMAs run (PF pieces of 8 bytes per thread), then moved to LDS between two barriers
  constexpr int NPC = NET_ROWS * CPR;             // 8-byte pieces per tile
  constexpr int PF = (NPC + 255) / 256;
  uint2 pre[PF];
  auto fetch = [&](int ti, bool& act) {
    const NetTile T = tiles[ti];
    const NetSample P = smp[T.sample];
    act = !(off && off[P.sys]);  // uniform over the workgroup
    if (!act) return;
    const int64_t rb = P.row0 - row_base;
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int c = threadIdx.x + 256 * i;
      if (c < NPC) {
        const int rr = c / CPR, cc = c - rr * CPR;
        const int p = wrap(T.pos0 - NET_HALO + rr, P.s);
        pre[i] = *(const uint2*)((const char*)(in + (rb + p) * CIN) + cc * 8);
      }
    }
  };
  auto park = [&]() {
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int c = threadIdx.x + 256 * i;
      if (c < NPC) {
        const int rr = c / CPR, cc = c - rr * CPR;
        *(uint2*)((char*)(tile + rr * STR) + cc * 8) = pre[i];
      }
    }
  };
  bool act_cur = false;
  if ((int)blockIdx.x < ntiles) {
    fetch(blockIdx.x, act_cur);
    if (act_cur) park();
  }
  __syncthreads();
  for (int ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
    const int tn = ti + gridDim.x;
    bool act_next = false;
    if (tn < ntiles) fetch(tn, act_next);
    const NetTile T = tiles[ti];
    const NetSample P = smp[T.sample];
    const int64_t rb = P.row0 - row_base;
    if (act_cur) {
    v4f acc[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) acc[rt] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const int kl = ks * MM::KS + q * EPL;
      const int t = kl / CIN, ci = kl - t * CIN;
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
        acc[rt] = MM::mma(MM::ld(tile + (rt * 16 + r16 + t) * STR + ci), bw[ks], acc[rt]);
    }
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int pos = T.pos0 + rt * 16 + 4 * q + e;
        if (pos >= P.s) continue;
        const int64_t o = (rb + pos) * NET_C + co;
        float v = acc[rt][e];
        if (BWD)
          v = mask[o] > 0.0f ? v : 0.0f;
        else
          v = fmaxf(v + bco, 0.0f);
        out[o] = to_e<E>(v);
      }
    }
    __syncthreads();  // every wave is done with this tile's rows
    if (tn < ntiles && act_next) park();
    __syncthreads();
    act_cur = act_next;
  }
}

// bfloat16 inference variant: the 4 waves form a 2 x 2 grid over (grid points, output
// channels): wave w takes points 32 (w & 1) .. +31 and channels 32 (w >> 1) .. +31, i.e. 2 x 2
// accumulator tiles, with its two 16-channel weight slices in registers.  Each staged input
// fragment is read from LDS by two waves (four in the float32 kernel above) and feeds two
// MFMAs, and each workgroup loads every weight twice (once per channel half).
template <int CIN>
__global__ __launch_bounds__(256) void k_net_conv_bf(const uint16_t* __restrict__ in,
                                                     uint16_t* __restrict__ out,
                                                     const uint16_t* __restrict__ W,
                                                     const float* __restrict__ bias,
                                                     const NetSample* __restrict__ smp,
                                                     const NetTile* __restrict__ tiles,
                                                     int ntiles, int64_t row_base,
                                                     const int* __restrict__ skip,
                                                     const int* __restrict__ off) {
  typedef NetMma<uint16_t> MM;
  constexpr int NKS = NET_W * CIN / 16;
  constexpr int STR = ConvStride<uint16_t, CIN>::v;
  constexpr int CPR = CIN * 2 / 8;
  __shared__ __align__(16) uint16_t tile[NET_ROWS * STR];
  if (skip && *skip) return;
  const int lane = threadIdx.x & 63, q = lane >> 4, r16 = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rh = wave & 1, chh = wave >> 1;
  v4s bw[2][NKS];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks)
      bw[c][ks] =
          MM::ld(W + (int64_t)((chh * 2 + c) * 16 + r16) * (NET_W * CIN) + ks * 16 + q * 4);
  float bco[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) bco[c] = bias[(chh * 2 + c) * 16 + r16];
  constexpr int NPC = NET_ROWS * CPR;
  constexpr int PF = (NPC + 255) / 256;
  uint2 pre[PF];
  auto fetch = [&](int ti, bool& act) {
    const NetTile T = tiles[ti];
    const NetSample P = smp[T.sample];
    act = !(off && off[P.sys]);
    if (!act) return;
    const int64_t rb = P.row0 - row_base;
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int c = threadIdx.x + 256 * i;
      if (c < NPC) {
        const int rr = c / CPR, cc = c - rr * CPR;
        const int p = wrap(T.pos0 - NET_HALO + rr, P.s);
        pre[i] = *(const uint2*)((const char*)(in + (rb + p) * CIN) + cc * 8);
      }
    }
  };
  auto park = [&]() {
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int c = threadIdx.x + 256 * i;
      if (c < NPC) {
        const int rr = c / CPR, cc = c - rr * CPR;
        *(uint2*)((char*)(tile + rr * STR) + cc * 8) = pre[i];
      }
    }
  };
  bool act_cur = false;
  if ((int)blockIdx.x < ntiles) {
    fetch(blockIdx.x, act_cur);
    if (act_cur) park();
  }
  __syncthreads();
  for (int ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
    const int tn = ti + gridDim.x;
    bool act_next = false;
    if (tn < ntiles) fetch(tn, act_next);
    if (act_cur) {
      const NetTile T = tiles[ti];
      const NetSample P = smp[T.sample];
      const int64_t rb = P.row0 - row_base;
      v4f acc[2][2];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[rt][c] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
        const int kl = ks * 16 + q * 4;
        const int tp = kl / CIN, ci = kl - tp * CIN;
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
          const v4s a = MM::ld(tile + (rh * 32 + rt * 16 + r16 + tp) * STR + ci);
#pragma unroll
          for (int c = 0; c < 2; ++c) acc[rt][c] = MM::mma(a, bw[c][ks], acc[rt][c]);
        }
      }
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int pos = T.pos0 + rh * 32 + rt * 16 + 4 * q + e;
          if (pos >= P.s) continue;
          uint16_t* o = out + (rb + pos) * NET_C + chh * 32 + r16;
#pragma unroll
          for (int c = 0; c < 2; ++c) o[c * 16] = f2bf(fmaxf(acc[rt][c][e] + bco[c], 0.0f));
        }
    }
    __syncthreads();
    if (tn < ntiles && act_next) park();
    __syncthreads();
    act_cur = act_next;
  }
}

// ------------------------------------------------------------------ last layer (64 -> 1)
template <typename E, int APPLY>
__global__ __launch_bounds__(64) void k_net_out(const E* __restrict__ a3,
                                                const float* __restrict__ w4,
                                                const float* __restrict__ b4,
                                                const NetSample* __restrict__ smp,
                                                const NetTile* __restrict__ tiles,
                                                int64_t row_base, float* __restrict__ outv,
                                                double* __restrict__ dst,
                                                const double* __restrict__ sigma,
                                                const int* __restrict__ off,
                                                const int* __restrict__ skip) {
  // the tile's 68 input rows are staged in LDS (16-byte pieces, coalesced) and each thread
  // contracts its 5 x 64 window from there
  constexpr int VE = 16 / (int)sizeof(E);        // elements per 16-byte piece
  constexpr int OSTR = NET_C + VE;               // row stride (elements), 16-byte aligned
  constexpr int PPR = NET_C / VE;                // pieces per row
  __shared__ float w[NET_W * NET_C];
  __shared__ __align__(16) E tile[NET_ROWS * OSTR];
  if (skip && *skip) return;
  const NetTile T = tiles[blockIdx.x];
  const NetSample P = smp[T.sample];
  if (off && off[P.sys]) return;
  const int64_t rb = P.row0 - row_base;
  for (int i = threadIdx.x; i < NET_W * NET_C; i += 64) w[i] = w4[i];
  for (int c = threadIdx.x; c < NET_ROWS * PPR; c += 64) {
    const int rr = c / PPR, cc = c - rr * PPR;
    const int p = wrap(T.pos0 - NET_HALO + rr, P.s);
    *(uint4*)(tile + rr * OSTR + cc * VE) = *(const uint4*)(a3 + (rb + p) * NET_C + cc * VE);
  }
  __syncthreads();
  const int pos = T.pos0 + threadIdx.x;
  if (pos >= P.s) return;
  float acc = b4[0];
#pragma unroll
  for (int t = 0; t < NET_W; ++t) {
    const E* row = tile + (threadIdx.x + t) * OSTR;
    const float* wt = w + t * NET_C;
#pragma unroll
    for (int c16 = 0; c16 < PPR; ++c16) {
      const uint4 v = *(const uint4*)(row + c16 * VE);
      const E* e = (const E*)&v;
#pragma unroll
      for (int i = 0; i < VE; ++i) acc += wt[c16 * VE + i] * to_f<E>(e[i]);
    }
  }
  if (APPLY) {
    dst[P.src + (int64_t)P.blk * P.s + pos] += sigma[P.sys] * (double)acc;
  } else {
    outv[rb + pos] = acc;
  }
}

// ------------------------------------------------------------------ fused inference (bfloat16)
// The whole network on one tile of NET_FTILE output points of one sample, every intermediate
// activation in LDS: the features of NET_FTILE + 16 staged rows (8 halo rows per side, 2 per
// width-5 layer), three MFMA convolutions and the output layer.  Every layer is computed on all
// staged rows; an output row depends on input rows r-2..r+2 only, so the valid rows shrink by 2
// per side and layer and the last layer's rows 8 .. 8 + NET_FTILE - 1 are exact.  The staged
// rows are the periodic extension of the sample (positions mod s), which makes this the same
// as applying each periodic layer to the whole sample, for any s.  Wave w keeps the weights of
// output channels 16w..16w+15 of the three convolutions in registers for the whole launch
// (persistent workgroups, three per CU, loop over the tiles); hidden activations are rounded to
// bfloat16 as in the layer-by-layer kernels, accumulation is float32; the 64 -> 1 output layer
// runs on the MFMA too, with its float32 weights split into two bfloat16 parts.  The feature
// rows share LDS with the second hidden layer's buffer.  The output (the normalised correction,
// float32) goes to a workspace row per grid point and k_net_apply adds sigma times it to the
// sweep output afterwards: adding it in place here would race with tiles that still read the
// vector (halo rows, later segment starts).
namespace fz {
constexpr int ROWS = NET_FTILE + 16;    // computed rows per layer
constexpr int PADR = NET_HALO;          // zero rows above and below (taps past both ends)
constexpr int LROWS = ROWS + 2 * PADR;  // LDS rows per buffer
// Row strides (elements).  A 16-byte LDS read serves 32 lanes at a time and is free of bank
// conflicts when their 16-byte slots differ modulo 32.  An MFMA operand read puts rows
// r16 = 0..15 and two consecutive slots (q = 0, 1 or 2, 3) in each half-wave: a stride of
// 2 x odd slots makes stride * r16 run over the 16 even residues and the +1 over the odd ones.
constexpr int SX = NET_CIN1 + 16;       // 6 slots
constexpr int SA = NET_C + 16;          // 10 slots
constexpr int RT = ROWS / 16;           // MFMA row tiles per layer
constexpr int FRG = 3;                  // row tiles accumulated together
}  // namespace fz
static_assert(fz::ROWS % 16 == 0 && NET_FTILE == 8 * 16, "two output row tiles per wave");
static_assert(NET_CIN1 % 32 == 0, "the fused layer 1 contracts 32 channels per instruction");
static_assert((fz::SX / 8) % 4 == 2 && (fz::SA / 8) % 4 == 2, "row strides of 2 x odd slots");

// two floats to bfloat16 (round to nearest even) in one dword, a in the low half
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
  const bf2 v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(uint32_t, v);
}

// ReLU of two packed bfloat16 values: as 16-bit integers every negative value (sign bit set,
// -0 included) is below 0 and the non-negative ones keep their order (v_pk_max_i16)
__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t u) {
  typedef short s2 __attribute__((ext_vector_type(2)));
  const s2 z = {0, 0};
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s2, u), z));
}

// one convolution of the fused kernel: out rows PADR.. = relu(conv(in) + bias) for this
// lane's output channel co; the RT row tiles in groups of RG independent accumulation chains
template <int CIN, int STR, int RG>
__device__ __forceinline__ void fused_layer(const uint16_t* __restrict__ in,
                                            uint16_t* __restrict__ out,
                                            const bf8 (&bw)[NET_W * CIN / 32], float bias, int q,
                                            int r16, int co) {
  constexpr int NKS = NET_W * CIN / 32;
  static_assert(fz::RT % RG == 0, "row tile groups");
#pragma unroll
  for (int g = 0; g < fz::RT; g += RG) {
    v4f acc[RG];
#pragma unroll
    for (int j = 0; j < RG; ++j) acc[j] = v4f{bias, bias, bias, bias};  // bias summed first
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const int kl = ks * 32 + q * 8;
      const int t = kl / CIN, ci = kl - t * CIN;
      // output row m, tap t reads input row m + t - 2, stored at LDS row m + t
#pragma unroll
      for (int j = 0; j < RG; ++j)
        acc[j] = NetMma32::mma(*(const bf8*)(in + ((g + j) * 16 + r16 + t) * STR + ci), bw[ks],
                               acc[j]);
    }
    // lane (q, r16) holds rows 4q..4q+3 of channel co.  Neighbouring lanes trade one packed
    // pair so that the even lane writes rows 4q, 4q+1 and the odd lane rows 4q+2, 4q+3, each
    // as channel pairs (co & ~1, co | 1) in one dword: one write instruction covers the rows
    // 0, 2, .., 14 of the tile (or 1, 3, .., 15), 8 dwords each, which the 40-dword row
    // stride puts in distinct banks.  Round to nearest even (v_cvt_pk_bf16_f32), then ReLU on
    // the packed pair.
    const bool odd = r16 & 1;
#pragma unroll
    for (int j = 0; j < RG; ++j) {
      const uint32_t u01 = relu_bf16x2(pack_bf16(acc[j][0], acc[j][1]));
      const uint32_t u23 = relu_bf16x2(pack_bf16(acc[j][2], acc[j][3]));
      const uint32_t own = odd ? u23 : u01;
      const uint32_t oth = (uint32_t)__builtin_amdgcn_update_dpp(
          0, (int)(odd ? u01 : u23), lanes::DPP_XOR1, 0xf, 0xf, false);
      const uint32_t lo = odd ? oth : own, hi = odd ? own : oth;  // channels co & ~1, co | 1
      uint32_t* o = (uint32_t*)(out + ((g + j) * 16 + 4 * q + (odd ? 2 : 0) + fz::PADR) * fz::SA +
                                (co & ~1));
      o[0] = __builtin_amdgcn_perm(hi, lo, 0x05040100u);          // low halves: first row
      o[fz::SA / 2] = __builtin_amdgcn_perm(hi, lo, 0x07060302u);  // high halves: second row
    }
  }
}

__global__ __launch_bounds__(256, 3) void k_net_fused(
    const double* __restrict__ src, const double* __restrict__ inv_sigma,
    const NetSample* __restrict__ smp, const NetTile* __restrict__ tiles, int ntiles,
    int64_t row_base, int k, int S, const uint16_t* __restrict__ W1,
    const uint16_t* __restrict__ W2, const uint16_t* __restrict__ W3,
    const float* __restrict__ b1, const float* __restrict__ b2, const float* __restrict__ b3,
    const float* __restrict__ w4, const float* __restrict__ b4, float* __restrict__ corr,
    const int* __restrict__ skip, const int* __restrict__ off) {
  using namespace fz;
  __shared__ __align__(16) uint16_t A1[LROWS * SA];
  __shared__ __align__(16) uint16_t A2[LROWS * SA];
  // output-layer weights split into bfloat16 high and low parts (w = hi + lo to 2^-16
  // relative), the two nonzero columns of the output layer's MFMA operand
  __shared__ __align__(16) uint16_t w4hl[2][NET_W * NET_C];
  // the features live inside A2's computed rows: layer 1 reads them before layer 2 writes A2,
  // and A2's zero pad rows stay clear of them.  Layer 2 overwrites X's pad rows, so every tile
  // clears them again.
  uint16_t* const X = A2 + PADR * SA;
  static_assert(LROWS * SX <= ROWS * SA, "features fit in A2's computed rows");
  if (skip && *skip) return;
  const int lane = threadIdx.x & 63, q = lane >> 4, r16 = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int co = wave * 16 + r16;
  bf8 bw1[NET_W * NET_CIN1 / 32], bw2[NET_W * NET_C / 32], bw3[NET_W * NET_C / 32];
#pragma unroll
  for (int ks = 0; ks < NET_W * NET_CIN1 / 32; ++ks)
    bw1[ks] = *(const bf8*)(W1 + (int64_t)co * (NET_W * NET_CIN1) + ks * 32 + q * 8);
#pragma unroll
  for (int ks = 0; ks < NET_W * NET_C / 32; ++ks) {
    bw2[ks] = *(const bf8*)(W2 + (int64_t)co * (NET_W * NET_C) + ks * 32 + q * 8);
    bw3[ks] = *(const bf8*)(W3 + (int64_t)co * (NET_W * NET_C) + ks * 32 + q * 8);
  }
  const float c1 = b1[co], c2 = b2[co], c3 = b3[co], c4 = b4[0];
  // zero the buffers once: the pad rows are never written again
  const uint4 z4 = {0u, 0u, 0u, 0u};
  for (int i = threadIdx.x; i < LROWS * SA / 8; i += 256) {
    ((uint4*)A1)[i] = z4;
    ((uint4*)A2)[i] = z4;
  }
  for (int i = threadIdx.x; i < NET_W * NET_C; i += 256) {
    const float w = w4[i];
    const __bf16 hi = (__bf16)w;
    w4hl[0][i] = __builtin_bit_cast(uint16_t, hi);
    w4hl[1][i] = __builtin_bit_cast(uint16_t, (__bf16)(w - (float)hi));
  }
  __syncthreads();
  for (int ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
    const NetTile T = tiles[ti];
    const NetSample P = smp[T.sample];
    if (off && off[P.sys]) continue;  // uniform over the workgroup
    const double isg = inv_sigma[P.sys];
    const int e = min((P.blk / k) * k + k - 1, P.nb - 1);
    const int hot = 1 + S + (e - P.blk);
    // features, channel 0: own block, 1..S: later segment starts (zero past the last block),
    // then the one-hot of e - blk.  The block values are loaded with consecutive threads on
    // consecutive grid points (coalesced), in batches of FB loads issued before the first is
    // used (more would exceed the 168 registers of three workgroups per CU), and the constant
    // channels are written in a second pass.
    constexpr int FB = 2;
    constexpr int JM = ((NET_CIN1 * ROWS + 255) / 256 + FB - 1) / FB * FB;
    const int nval = (1 + S) * ROWS;
#pragma unroll
    for (int j0 = 0; j0 < JM; j0 += FB) {
      if (j0 * 256 >= nval) break;  // uniform
      double v[FB];
#pragma unroll
      for (int j = 0; j < FB; ++j) {
        const int it = threadIdx.x + 256 * (j0 + j);
        const int m = it / ROWS, r = it - m * ROWS;
        const int b = m == 0 ? P.blk : e + 1 + (m - 1) * k;
        // T.pos0 - 8 + r lies in [-8, s + 136): one correction when s >= 144 (uniform)
        int pos = T.pos0 - 4 * NET_HALO + r;
        if (P.s >= ROWS) {
          pos = pos < 0 ? pos + P.s : (pos >= P.s ? pos - P.s : pos);
        } else {
          pos = wrap(pos, P.s);
        }
        v[j] = (it < nval && b < P.nb) ? src[P.src + (int64_t)b * P.s + pos] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < FB; ++j) {
        const int it = threadIdx.x + 256 * (j0 + j);
        const int m = it / ROWS, r = it - m * ROWS;
        if (it < nval) X[(r + PADR) * SX + m] = (uint16_t)pack_bf16((float)(v[j] * isg), 0.0f);
      }
    }
    // channels S+1..31 (zeros and the one-hot) are the same in every row: thread r < ROWS
    // writes the 8-channel pieces of row r that hold no block value whole and the constant
    // channels of the piece that holds both one by one (the value stores above write its other
    // channels; the two sets of bytes are disjoint)
    if (threadIdx.x < ROWS) {
      uint16_t* xr = X + (threadIdx.x + PADR) * SX;
      const int gm = (S + 1) / 8;  // the first piece with a constant channel (uniform)
#pragma unroll
      for (int g = 0; g < NET_CIN1 / 8; ++g) {
        if (g < gm) continue;
        if (8 * g > S) {
          uint32_t wv[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int c = 8 * g + 2 * i;
            wv[i] = (c == hot ? 0x3f80u : 0u) | (c + 1 == hot ? 0x3f800000u : 0u);
          }
          *(uint4*)(xr + 8 * g) = uint4{wv[0], wv[1], wv[2], wv[3]};
        } else {
          for (int c = S + 1; c < 8 * g + 8; ++c) xr[c] = c == hot ? (uint16_t)0x3f80u : 0;
        }
      }
    }
    if (threadIdx.x < 2 * PADR * (NET_CIN1 / 8)) {  // pad rows 0, 1, LROWS - 2, LROWS - 1
      const int pr = threadIdx.x / (NET_CIN1 / 8), pc = threadIdx.x - pr * (NET_CIN1 / 8);
      const int row = pr < PADR ? pr : LROWS - 2 * PADR + pr;
      *(uint4*)(X + row * SX + pc * 8) = z4;
    }
    __syncthreads();
    fused_layer<NET_CIN1, SX, FRG>(X, A1, bw1, c1, q, r16, co);
    __syncthreads();
    fused_layer<NET_C, SA, FRG>(A1, A2, bw2, c2, q, r16, co);
    __syncthreads();
    fused_layer<NET_C, SA, FRG>(A2, A1, bw3, c3, q, r16, co);
    __syncthreads();
    // output layer (64 -> 1) on the MFMA: points 16 g .. 16 g + 15 (output row tiles 2w, 2w + 1
    // of wave w) against a 320 x 16 weight operand whose columns 0 and 1 hold the high and
    // low bfloat16 parts of the float32 weights (the other columns zero); their sum is the
    // output.  Point p sits at row 8 + p.  A1 is next written by the following tile's layer 1,
    // after the barrier that follows its features.
    {
      v4f oacc[2];
#pragma unroll
      for (int j = 0; j < 2; ++j) oacc[j] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int ks = 0; ks < NET_W * NET_C / 32; ++ks) {
        const int kl = ks * 32 + q * 8;
        const int t = kl / NET_C, ci = kl - t * NET_C;
        bf8 b = {};
        if (r16 < 2) b = *(const bf8*)(&w4hl[r16][kl]);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int g = 2 * wave + j;
          const bf8 a = *(const bf8*)(A1 + (4 * NET_HALO + g * 16 + r16 + t) * SA + ci);
          oacc[j] = NetMma32::mma(a, b, oacc[j]);
        }
      }
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          // column 0 (lane r16 = 0) plus column 1 (lane r16 = 1)
          const float tot = oacc[j][e] + __int_as_float(__builtin_amdgcn_update_dpp(
                                             0, __float_as_int(oacc[j][e]), lanes::DPP_XOR1,
                                             0xf, 0xf, false));
          const int pos = T.pos0 + (2 * wave + j) * 16 + 4 * q + e;
          if (r16 == 0 && pos < P.s) corr[P.row0 - row_base + pos] = tot + c4;
        }
    }
  }
}

// dst += sigma * corr for every point of the tiles (the fused kernel's output)
__global__ __launch_bounds__(64) void k_net_apply(const float* __restrict__ corr,
                                                  const NetSample* __restrict__ smp,
                                                  const NetTile* __restrict__ tiles,
                                                  int64_t row_base, double* __restrict__ dst,
                                                  const double* __restrict__ sigma,
                                                  const int* __restrict__ off,
                                                  const int* __restrict__ skip) {
  if (skip && *skip) return;
  const NetTile T = tiles[blockIdx.x];
  const NetSample P = smp[T.sample];
  if (off && off[P.sys]) return;
  const int pos = T.pos0 + threadIdx.x;
  if (pos >= P.s) return;
  dst[P.src + (int64_t)P.blk * P.s + pos] +=
      sigma[P.sys] * (double)corr[P.row0 - row_base + pos];
}

// ------------------------------------------------------------------ training
__global__ __launch_bounds__(64) void k_net_loss(const float* __restrict__ outv,
                                                 const float* __restrict__ y,
                                                 const NetSample* __restrict__ smp,
                                                 const NetTile* __restrict__ tiles, float scale,
                                                 float* __restrict__ g4,
                                                 double* __restrict__ lpart) {
  const NetTile T = tiles[blockIdx.x];
  const NetSample P = smp[T.sample];
  const int pos = T.pos0 + threadIdx.x;
  double d2 = 0.0;
  if (pos < P.s) {
    const int64_t r = P.row0 + pos;
    const float d = outv[r] - y[P.src + (int64_t)P.blk * P.s + pos];
    g4[r] = scale * d;
    d2 = (double)d * (double)d;
  }
  for (int o = 32; o > 0; o >>= 1) d2 += __shfl_xor(d2, o);
  if (threadIdx.x == 0) lpart[blockIdx.x] = d2;
}

// g3[row][c] = relu'(a3) * sum_t W4[t][c] g4[pos - t + 2]
__global__ __launch_bounds__(256) void k_net_out_bwd(const float* __restrict__ g4,
                                                     const float* __restrict__ w4,
                                                     const float* __restrict__ a3,
                                                     float* __restrict__ g3,
                                                     const NetSample* __restrict__ smp,
                                                     const NetTile* __restrict__ tiles) {
  const NetTile T = tiles[blockIdx.x];
  const NetSample P = smp[T.sample];
  const int c = threadIdx.x & 63;
  for (int p = threadIdx.x >> 6; p < NET_TILE; p += 4) {
    const int pos = T.pos0 + p;
    if (pos >= P.s) break;
    const int64_t r = P.row0 + pos;
    float acc = 0.0f;
#pragma unroll
    for (int t = 0; t < NET_W; ++t)
      acc += w4[t * NET_C + c] * g4[P.row0 + wrap(pos - t + NET_HALO, P.s)];
    g3[r * NET_C + c] = a3[r * NET_C + c] > 0.0f ? acc : 0.0f;
  }
}

// dW4[t][c] = sum_pos g4[pos] a3[pos + t - 2][c], db4 = sum g4: partials per workgroup
__global__ __launch_bounds__(256) void k_net_wgrad4(const float* __restrict__ g4,
                                                    const float* __restrict__ a3,
                                                    const NetSample* __restrict__ smp,
                                                    const NetTile* __restrict__ tiles,
                                                    int ntiles, float* __restrict__ part) {
  __shared__ float gt[NET_TILE];
  constexpr int NE = NET_W * NET_C + 1;
  float acc0 = 0.0f, acc1 = 0.0f;  // elements threadIdx.x and threadIdx.x + 256
  const int e0 = threadIdx.x, e1 = threadIdx.x + 256;
  for (int ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
    const NetTile T = tiles[ti];
    const NetSample P = smp[T.sample];
    __syncthreads();
    if (threadIdx.x < NET_TILE) {
      const int pos = T.pos0 + threadIdx.x;
      gt[threadIdx.x] = pos < P.s ? g4[P.row0 + pos] : 0.0f;
    }
    __syncthreads();
    const int np = min(NET_TILE, P.s - T.pos0);
    {
      const int t = e0 / NET_C, c = e0 % NET_C;
      for (int p = 0; p < np; ++p)
        acc0 += gt[p] * a3[(P.row0 + wrap(T.pos0 + p + t - NET_HALO, P.s)) * NET_C + c];
    }
    if (e1 < NE - 1) {
      const int t = e1 / NET_C, c = e1 % NET_C;
      for (int p = 0; p < np; ++p)
        acc1 += gt[p] * a3[(P.row0 + wrap(T.pos0 + p + t - NET_HALO, P.s)) * NET_C + c];
    } else if (e1 == NE - 1) {
      for (int p = 0; p < np; ++p) acc1 += gt[p];
    }
  }
  part[(int64_t)blockIdx.x * NE + e0] = acc0;
  if (e1 < NE) part[(int64_t)blockIdx.x * NE + e1] = acc1;
}

// dW[co][t * CIN + ci] = sum_pos g[pos][co] a[pos + t - 2][ci], db[co] = sum_pos g[pos][co]
template <int CIN>
__global__ __launch_bounds__(256) void k_net_wgrad(const float* __restrict__ g,
                                                   const float* __restrict__ a,
                                                   const NetSample* __restrict__ smp,
                                                   const NetTile* __restrict__ tiles,
                                                   int ntiles, float* __restrict__ part) {
  constexpr int GS = 80;                     // = 16 mod 32
  constexpr int AS = CIN == 64 ? 80 : 48;    // = 16 mod 32 (CIN = 16 or 32 fit in 48)
  constexpr int NCT = NET_W * CIN / 16;      // column tiles
  constexpr int CTW = (NCT + 3) / 4;         // column tiles per wave
  constexpr int NE = NET_C * NET_W * CIN + NET_C;
  __shared__ __align__(16) float gt[NET_TILE * GS];
  __shared__ __align__(16) float at[NET_ROWS * AS];
  const int lane = threadIdx.x & 63, q = lane >> 4, r16 = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  v4f acc[4][CTW];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int c = 0; c < CTW; ++c) acc[rt][c] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
  float bacc = 0.0f;
  for (int ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
    const NetTile T = tiles[ti];
    const NetSample P = smp[T.sample];
    __syncthreads();
    for (int e = threadIdx.x; e < NET_TILE * NET_C; e += 256) {
      const int p = e / NET_C, c = e % NET_C;
      const int pos = T.pos0 + p;
      gt[p * GS + c] = pos < P.s ? g[(P.row0 + pos) * NET_C + c] : 0.0f;
    }
    for (int e = threadIdx.x; e < NET_ROWS * CIN; e += 256) {
      const int rr = e / CIN, c = e % CIN;
      at[rr * AS + c] = a[(P.row0 + wrap(T.pos0 - NET_HALO + rr, P.s)) * CIN + c];
    }
    __syncthreads();
    if (threadIdx.x < NET_C)
      for (int p = 0; p < NET_TILE; ++p) bacc += gt[p * GS + threadIdx.x];
#pragma unroll 4
    for (int ks = 0; ks < NET_TILE / 4; ++ks) {
      const int p = ks * 4 + q;
      float af[4];
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) af[rt] = gt[p * GS + rt * 16 + r16];
#pragma unroll
      for (int c = 0; c < CTW; ++c) {
        const int ct = wave + 4 * c;
        if (ct >= NCT) continue;
        const int kidx = ct * 16 + r16;
        const int t = kidx / CIN, ci = kidx - t * CIN;
        const float bf = at[(p + t) * AS + ci];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
          acc[rt][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[rt], bf, acc[rt][c], 0, 0, 0);
      }
    }
  }
  float* pp = part + (int64_t)blockIdx.x * NE;
#pragma unroll
  for (int c = 0; c < CTW; ++c) {
    const int ct = wave + 4 * c;
    if (ct >= NCT) continue;
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int co = rt * 16 + 4 * q + e;
        pp[(int64_t)co * (NET_W * CIN) + ct * 16 + r16] = acc[rt][c][e];
      }
  }
  if (threadIdx.x < NET_C) pp[NET_C * NET_W * CIN + threadIdx.x] = bacc;
}

// sum the workgroup partials (fixed order: groups of WR_G partials, then the groups) and
// scatter into the flat gradient
#define WR_G 16
__global__ void k_net_wreduce1(const float* __restrict__ part, int grid, int NE,
                               float* __restrict__ part2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NE) return;
  const int g0 = blockIdx.y * WR_G, g1 = min(grid, g0 + WR_G);
  float acc = 0.0f;
  for (int g = g0; g < g1; ++g) acc += part[(int64_t)g * NE + e];
  part2[(int64_t)blockIdx.y * NE + e] = acc;
}
__global__ void k_net_wreduce(const float* __restrict__ part, int grid, int layer, NetLayout L,
                              float* __restrict__ grad) {
  const int CIN = layer == 0 ? NET_CIN1 : NET_C;
  const int cin = layer == 0 ? L.cin : NET_C;
  const int NE = layer == 3 ? NET_W * NET_C + 1 : NET_C * NET_W * CIN + NET_C;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NE) return;
  float acc = 0.0f;
  for (int g = 0; g < grid; ++g) acc += part[(int64_t)g * NE + e];
  if (layer == 3) {
    if (e == NE - 1) {
      grad[L.b[3]] = acc;
    } else {
      const int t = e / NET_C, c = e % NET_C;
      grad[L.w[3] + (int64_t)c * NET_W + t] = acc;
    }
    return;
  }
  const int nw = NET_C * NET_W * CIN;
  if (e >= nw) {
    grad[L.b[layer] + (e - nw)] = acc;
    return;
  }
  const int co = e / (NET_W * CIN), kk = e % (NET_W * CIN);
  const int t = kk / CIN, ci = kk % CIN;
  if (ci < cin) grad[L.w[layer] + ((int64_t)co * cin + ci) * NET_W + t] = acc;
}

__global__ void k_net_adam(float* __restrict__ th, const float* __restrict__ g,
                           float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                           float b1, float b2, float eps, float bc1, float bc2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

__global__ void k_net_fill_int(int* __restrict__ p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ launchers
static unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

void net_fill_int(int* p, int n, int v, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_net_fill_int, dim3(nblk(n, 256)), dim3(256), 0, st, p, n, v);
}
void net_pack(const float* theta, const NetLayout& L, const NetWeights& W, hipStream_t st) {
  const int64_t n = (int64_t)NET_C * NET_W * NET_C;
  hipLaunchKernelGGL(k_net_pack, dim3(nblk(n, 256)), dim3(256), 0, st, theta, L, W);
}
void net_sumsq(const double* v, const NetChunk* chunks, int nchunk, double* part,
               const int* skip, hipStream_t st) {
  if (nchunk > 0)
    hipLaunchKernelGGL(k_net_sumsq, dim3(nchunk), dim3(256), 0, st, v, chunks, part, skip);
}
void net_sigma_impl(const double* part, const int32_t* chunk0, const NetChunk* ch, int nsys,
                    double* sigma, double* inv_sigma, const int* skip, hipStream_t st) {
  hipLaunchKernelGGL(k_net_sigma, dim3(nblk(nsys, 64)), dim3(64), 0, st, part, chunk0, ch, nsys,
                     sigma, inv_sigma, skip);
}
void net_norm_pairs(const double* chat, const double* cex, const double* inv_sigma,
                    int64_t len, int npair, float* x, float* y, hipStream_t st) {
  hipLaunchKernelGGL(k_net_norm_pairs, dim3(nblk(len * npair, 256)), dim3(256), 0, st, chat,
                     cex, inv_sigma, len, npair, x, y);
}
void net_feat_f(const float* src, const NetSample* smp, const NetTile* tiles, int ntiles,
                int64_t row_base, int k, int S, int bf16, void* X0, hipStream_t st) {
  if (ntiles <= 0) return;
  if (bf16)
    hipLaunchKernelGGL((k_net_feat<uint16_t, float>), dim3(ntiles), dim3(64), 0, st, src,
                       (const double*)nullptr, smp, tiles, row_base, k, S, (uint16_t*)X0,
                       (const int*)nullptr, (const int*)nullptr);
  else
    hipLaunchKernelGGL((k_net_feat<float, float>), dim3(ntiles), dim3(64), 0, st, src,
                       (const double*)nullptr, smp, tiles, row_base, k, S, (float*)X0,
                       (const int*)nullptr, (const int*)nullptr);
}
void net_feat_d(const double* src, const double* inv_sigma, const NetSample* smp,
                const NetTile* tiles, int ntiles, int64_t row_base, int k, int S, int bf16,
                void* X0, const int* skip, const int* off, hipStream_t st) {
  if (ntiles <= 0) return;
  if (bf16)
    hipLaunchKernelGGL((k_net_feat<uint16_t, double>), dim3(ntiles), dim3(64), 0, st, src,
                       inv_sigma, smp, tiles, row_base, k, S, (uint16_t*)X0, skip, off);
  else
    hipLaunchKernelGGL((k_net_feat<float, double>), dim3(ntiles), dim3(64), 0, st, src,
                       inv_sigma, smp, tiles, row_base, k, S, (float*)X0, skip, off);
}
void net_conv(int bf16, int cin16, int bwd, const void* in, void* out, const void* W,
              const float* bias, const float* mask, const NetSample* smp, const NetTile* tiles,
              int ntiles, int64_t row_base, const int* skip, const int* off, hipStream_t st) {
  if (ntiles <= 0) return;
  const dim3 g((unsigned)std::min(ntiles, GRID_CAP)), b(256);
#define NET_CONV(E, CIN, BWD)                                                               \
  hipLaunchKernelGGL((k_net_conv<E, CIN, BWD>), g, b, 0, st, (const E*)in, (E*)out,         \
                     (const E*)W, bias, mask, smp, tiles, ntiles, row_base, skip, off)
  if (bf16) {
    if (cin16)
      hipLaunchKernelGGL(k_net_conv_bf<NET_CIN1>, g, b, 0, st, (const uint16_t*)in, (uint16_t*)out,
                         (const uint16_t*)W, bias, smp, tiles, ntiles, row_base, skip, off);
    else  // measured faster for 64 input channels than the 2 x 2 variant
      NET_CONV(uint16_t, 64, 0);
  } else if (bwd) {
    NET_CONV(float, 64, 1);
  } else if (cin16) {
    NET_CONV(float, NET_CIN1, 0);
  } else {
    NET_CONV(float, 64, 0);
  }
#undef NET_CONV
}
void net_out(int bf16, const void* a3, const float* w4, const float* b4, const NetSample* smp,
             const NetTile* tiles, int ntiles, int64_t row_base, float* outv, double* dst,
             const double* sigma, const int* off, const int* skip, hipStream_t st) {
  if (ntiles <= 0) return;
  const dim3 g(ntiles), b(64);
  if (dst) {
    if (bf16)
      hipLaunchKernelGGL((k_net_out<uint16_t, 1>), g, b, 0, st, (const uint16_t*)a3, w4, b4, smp,
                         tiles, row_base, outv, dst, sigma, off, skip);
    else
      hipLaunchKernelGGL((k_net_out<float, 1>), g, b, 0, st, (const float*)a3, w4, b4, smp,
                         tiles, row_base, outv, dst, sigma, off, skip);
  } else {
    if (bf16)
      hipLaunchKernelGGL((k_net_out<uint16_t, 0>), g, b, 0, st, (const uint16_t*)a3, w4, b4, smp,
                         tiles, row_base, outv, dst, sigma, off, skip);
    else
      hipLaunchKernelGGL((k_net_out<float, 0>), g, b, 0, st, (const float*)a3, w4, b4, smp,
                         tiles, row_base, outv, dst, sigma, off, skip);
  }
}
void net_fused(const double* src, const double* inv_sigma, const NetSample* smp,
               const NetTile* ftiles, int nftiles, int64_t row_base, int k, int S,
               const NetWeights& W, const float* theta, const NetLayout& L, float* corr,
               const int* skip, const int* off, hipStream_t st) {
  if (nftiles <= 0) return;
  static int resident = 0;  // workgroups resident on the device at once (3 per CU by design)
  if (resident == 0) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_net_fused, 256, 0) == hipSuccess &&
        per > 0)
      resident = cus * per;
    else
      resident = GRID_CAP;
  }
  hipLaunchKernelGGL(k_net_fused, dim3((unsigned)std::min(nftiles, resident)), dim3(256), 0, st,
                     src, inv_sigma, smp, ftiles, nftiles, row_base, k, S, W.wb[0], W.wb[1],
                     W.wb[2], theta + L.b[0], theta + L.b[1], theta + L.b[2], W.w4,
                     theta + L.b[3], corr, skip, off);
}
void net_apply(const float* corr, const NetSample* smp, const NetTile* tiles, int ntiles,
               int64_t row_base, double* dst, const double* sigma, const int* off,
               const int* skip, hipStream_t st) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(k_net_apply, dim3(ntiles), dim3(64), 0, st, corr, smp, tiles, row_base, dst,
                     sigma, off, skip);
}
void net_loss(const float* outv, const float* y, const NetSample* smp, const NetTile* tiles,
              int ntiles, float scale, float* g4, double* lpart, hipStream_t st) {
  hipLaunchKernelGGL(k_net_loss, dim3(ntiles), dim3(64), 0, st, outv, y, smp, tiles, scale, g4,
                     lpart);
}
void net_out_bwd(const float* g4, const float* w4, const float* a3, float* g3,
                 const NetSample* smp, const NetTile* tiles, int ntiles, hipStream_t st) {
  hipLaunchKernelGGL(k_net_out_bwd, dim3(ntiles), dim3(256), 0, st, g4, w4, a3, g3, smp, tiles);
}
void net_wgrad4(const float* g4, const float* a3, const NetSample* smp, const NetTile* tiles,
                int ntiles, int grid, float* part, hipStream_t st) {
  hipLaunchKernelGGL(k_net_wgrad4, dim3(grid), dim3(256), 0, st, g4, a3, smp, tiles, ntiles,
                     part);
}
void net_wgrad(int cin16, const float* g, const float* a, const NetSample* smp,
               const NetTile* tiles, int ntiles, int grid, float* part, hipStream_t st) {
  if (cin16)
    hipLaunchKernelGGL(k_net_wgrad<NET_CIN1>, dim3(grid), dim3(256), 0, st, g, a, smp, tiles,
                       ntiles, part);
  else
    hipLaunchKernelGGL(k_net_wgrad<NET_C>, dim3(grid), dim3(256), 0, st, g, a, smp, tiles,
                       ntiles, part);
}
void net_wreduce(const float* part, float* part2, int grid, int layer, const NetLayout& L,
                 float* grad, hipStream_t st) {
  const int CIN = layer == 0 ? NET_CIN1 : NET_C;
  const int NE = layer == 3 ? NET_W * NET_C + 1 : NET_C * NET_W * CIN + NET_C;
  const int ng = (grid + WR_G - 1) / WR_G;
  hipLaunchKernelGGL(k_net_wreduce1, dim3(nblk(NE, 256), ng), dim3(256), 0, st, part, grid, NE,
                     part2);
  hipLaunchKernelGGL(k_net_wreduce, dim3(nblk(NE, 256)), dim3(256), 0, st, part2, ng, layer, L,
                     grad);
}
void net_adam(float* theta, const float* grad, float* m, float* v, int64_t n, float lr,
              float b1, float b2, float eps, float bc1, float bc2, hipStream_t st) {
  hipLaunchKernelGGL(k_net_adam, dim3(nblk(n, 256)), dim3(256), 0, st, theta, grad, m, v, n, lr,
                     b1, b2, eps, bc1, bc2);
}

}  // namespace svar

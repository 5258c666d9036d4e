// Cross-lane sums over a wave64 that stay in the VALU: v_permlane32_swap / v_permlane16_swap
// (gfx950) exchange the two halves of the wave and neighbouring rows of 16 lanes, and DPP row
// rotations / mirrors / quad permutations work inside a row.  __shfl_xor compiles to
// ds_bpermute, which goes through the LDS crossbar: in the Gram-Schmidt dot kernels its 136
// exchanges per basis slot cost more than the slot's global loads.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace svar {
namespace lanes {

__device__ __forceinline__ uint32_t lo32(double x) {
  return (uint32_t)(uint64_t)__double_as_longlong(x);
}
__device__ __forceinline__ uint32_t hi32(double x) {
  return (uint32_t)((uint64_t)__double_as_longlong(x) >> 32);
}
__device__ __forceinline__ double mk(uint32_t l, uint32_t h) {
  return __longlong_as_double((long long)(((uint64_t)h << 32) | (uint64_t)l));
}

// O = 32: lanes 32..63 of a trade places with lanes 0..31 of b; O = 16: the odd rows of 16
// lanes of a with the even rows of b.  Afterwards a + b holds, in every lane, its own value
// plus its partner's (lane ^ O): of a where lane & O is clear, of b where it is set.
template <int O>
__device__ __forceinline__ void swap_pair(double& a, double& b) {
  static_assert(O == 32 || O == 16, "permlane swaps exist for 32 and 16");
  const uint32_t al = lo32(a), ah = hi32(a), bl = lo32(b), bh = hi32(b);
  if constexpr (O == 32) {
    const auto rl = __builtin_amdgcn_permlane32_swap(al, bl, false, false);
    const auto rh = __builtin_amdgcn_permlane32_swap(ah, bh, false, false);
    a = mk(rl[0], rh[0]);
    b = mk(rl[1], rh[1]);
  } else {
    const auto rl = __builtin_amdgcn_permlane16_swap(al, bl, false, false);
    const auto rh = __builtin_amdgcn_permlane16_swap(ah, bh, false, false);
    a = mk(rl[0], rh[0]);
    b = mk(rl[1], rh[1]);
  }
}

// DPP controls (within rows of 16 lanes): rotate by 8 (= lane ^ 8), mirror inside groups of
// 8 (lane ^ 7), quad permutations lane ^ 2 and lane ^ 1
constexpr int DPP_ROR8 = 0x128, DPP_MIRROR8 = 0x141, DPP_XOR2 = 0x4E, DPP_XOR1 = 0xB1;
template <int CTRL>
__device__ __forceinline__ double dpp(double x) {
  const int l = __builtin_amdgcn_update_dpp(0, (int)lo32(x), CTRL, 0xf, 0xf, false);
  const int h = __builtin_amdgcn_update_dpp(0, (int)hi32(x), CTRL, 0xf, 0xf, false);
  return mk((uint32_t)l, (uint32_t)h);
}

// sum over the 64 lanes; every lane gets the total
__device__ __forceinline__ double wave_sum(double v) {
  double w = v;
  swap_pair<32>(v, w);
  v += w;
  w = v;
  swap_pair<16>(v, w);
  v += w;
  v += dpp<DPP_ROR8>(v);
  v += dpp<DPP_MIRROR8>(v);
  v += dpp<DPP_XOR2>(v);
  v += dpp<DPP_XOR1>(v);
  return v;
}

// 16 values per lane summed over the wave by a halving exchange: at each of four steps a lane
// keeps half of its values and adds its partner's copy of that half (partners lane ^ 32,
// lane ^ 16, lane ^ 8, lane ^ 7), then two quad steps finish.  Lane l ends with the wave total
// of value (l >> 2) & 15.
__device__ __forceinline__ double wave_sum16(double (&v)[16]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    swap_pair<32>(v[i], v[i + 8]);
    v[i] += v[i + 8];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    swap_pair<16>(v[i], v[i + 4]);
    v[i] += v[i + 4];
  }
  {
    const bool up = (lane & 8) != 0;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const double send = up ? v[i] : v[i + 2];
      const double keep = up ? v[i + 2] : v[i];
      v[i] = keep + dpp<DPP_ROR8>(send);
    }
  }
  {
    const bool up = (lane & 4) != 0;
    const double send = up ? v[0] : v[1];
    const double keep = up ? v[1] : v[0];
    v[0] = keep + dpp<DPP_MIRROR8>(send);
  }
  double r = v[0];
  r += dpp<DPP_XOR2>(r);
  r += dpp<DPP_XOR1>(r);
  return r;
}

}  // namespace lanes
}  // namespace svar

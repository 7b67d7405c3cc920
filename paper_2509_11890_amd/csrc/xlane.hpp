// Cross-lane exchanges of a 64-lane wavefront on the VALU (DPP row moves and
// the gfx950 permlane swaps) instead of __shfl_xor, which goes through the LDS
// crossbar (ds_bpermute) and costs a round trip per step.  Each xorK(v)
// returns the value v holds in lane (lane ^ K) exactly, so a butterfly built
// from them adds the same operands in the same order as the __shfl_xor
// butterfly and gives bit-identical sums.  All lanes taking part must be
// active (the callers reduce in wavefront-uniform or row-uniform control
// flow).
#pragma once

#include <hip/hip_runtime.h>

namespace ttipm {
namespace xlane {

// 32-bit DPP move with every row and bank enabled
template <int CTRL>
__device__ __forceinline__ int dpp(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp<CTRL>((int)b), hi = dpp<CTRL>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

constexpr int kQuadXor1 = 0xB1;    // quad_perm [1, 0, 3, 2]
constexpr int kQuadXor2 = 0x4E;    // quad_perm [2, 3, 0, 1]
constexpr int kRowShl4 = 0x104;    // lane i reads lane i + 4 of its row of 16
constexpr int kRowShr4 = 0x114;    // lane i reads lane i - 4 of its row of 16
constexpr int kRowRor8 = 0x128;    // rotate the row of 16 by 8: lane i reads lane i ^ 8

__device__ __forceinline__ double xor1(double v) { return dpp<kQuadXor1>(v); }
__device__ __forceinline__ double xor2(double v) { return dpp<kQuadXor2>(v); }
__device__ __forceinline__ double xor4(double v) {
  const double up = dpp<kRowShl4>(v), down = dpp<kRowShr4>(v);
  return (__lane_id() & 4) ? down : up;
}
__device__ __forceinline__ double xor8(double v) { return dpp<kRowRor8>(v); }

// permlane16_swap (permlane32_swap) of v with itself returns, in each lane,
// its own value and that of lane ^ 16 (^ 32), in an order that depends on the
// lane's half; the select keeps the partner's.
__device__ __forceinline__ double xor16(double v) {
  const long long b = __double_as_longlong(v);
  const auto lo = __builtin_amdgcn_permlane16_swap((int)b, (int)b, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((int)(b >> 32), (int)(b >> 32), false, false);
  const bool odd = __lane_id() & 16;
  const int l = odd ? lo[0] : lo[1], h = odd ? hi[0] : hi[1];
  return __longlong_as_double(((long long)h << 32) | (unsigned int)l);
}
__device__ __forceinline__ double xor32(double v) {
  const long long b = __double_as_longlong(v);
  const auto lo = __builtin_amdgcn_permlane32_swap((int)b, (int)b, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((int)(b >> 32), (int)(b >> 32), false, false);
  const bool up = __lane_id() & 32;
  const int l = up ? lo[0] : lo[1], h = up ? hi[0] : hi[1];
  return __longlong_as_double(((long long)h << 32) | (unsigned int)l);
}

// Sum over the 64 lanes (every lane receives it), partners 32, 16, ..., 1.
__device__ __forceinline__ double wave_sum(double v) {
  v += xor32(v);
  v += xor16(v);
  v += xor8(v);
  v += xor4(v);
  v += xor2(v);
  v += xor1(v);
  return v;
}

// Sum over each row of 16 lanes (every lane of the row receives it), partners
// 8, 4, 2, 1.
__device__ __forceinline__ double row16_sum(double v) {
  v += xor8(v);
  v += xor4(v);
  v += xor2(v);
  v += xor1(v);
  return v;
}

}  // namespace xlane
}  // namespace ttipm

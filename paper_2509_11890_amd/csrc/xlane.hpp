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

__device__ __forceinline__ int xor1(int v) { return dpp<kQuadXor1>(v); }
__device__ __forceinline__ int xor2(int v) { return dpp<kQuadXor2>(v); }
__device__ __forceinline__ int xor4(int v) {
  const int up = dpp<kRowShl4>(v), down = dpp<kRowShr4>(v);
  return (__lane_id() & 4) ? down : up;
}
__device__ __forceinline__ int xor8(int v) { return dpp<kRowRor8>(v); }

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
__device__ __forceinline__ int xor16(int v) {
  const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  return (__lane_id() & 16) ? r[0] : r[1];
}
__device__ __forceinline__ int xor32(int v) {
  const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  return (__lane_id() & 32) ? r[0] : r[1];
}
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

// Partial pivoting's choice: the largest v, ties to the smallest idx (a total
// order for non-NaN v, so every reduction order gives the same winner).
__device__ __forceinline__ bool pivot_better(double b, int ib, double a, int ia) {
  return b > a || (b == a && ib < ia);
}

template <int K>
__device__ __forceinline__ void argmax_step(double& v, int& idx) {
  double b;
  int ib;
  if constexpr (K == 32) { b = xor32(v); ib = xor32(idx); }
  else if constexpr (K == 16) { b = xor16(v); ib = xor16(idx); }
  else if constexpr (K == 8) { b = xor8(v); ib = xor8(idx); }
  else if constexpr (K == 4) { b = xor4(v); ib = xor4(idx); }
  else if constexpr (K == 2) { b = xor2(v); ib = xor2(idx); }
  else { b = xor1(v); ib = xor1(idx); }
  if (pivot_better(b, ib, v, idx)) {
    v = b;
    idx = ib;
  }
}

// Pivot choice over the 64 lanes (every lane receives it).
__device__ __forceinline__ void wave_argmax(double& v, int& idx) {
  argmax_step<32>(v, idx);
  argmax_step<16>(v, idx);
  argmax_step<8>(v, idx);
  argmax_step<4>(v, idx);
  argmax_step<2>(v, idx);
  argmax_step<1>(v, idx);
}

// Pivot choice over a workgroup of NWAVE wavefronts (every thread receives
// it), when only the first nwr wavefronts (a uniform count) hold candidates:
// those reduce on the VALU and publish their winners through red_v / red_i,
// and every thread combines the nwr winners.  The other wavefronts do no
// reduction work (they share the SIMDs with the ones that do).  One barrier;
// the caller must not rewrite red_v / red_i before a later barrier.
template <int NWAVE>
__device__ __forceinline__ void block_argmax(double& v, int& idx, int nwr, double* red_v, int* red_i) {
  if ((int)(threadIdx.x >> 6) < nwr) {
    wave_argmax(v, idx);
    if ((threadIdx.x & 63) == 0) {
      red_v[threadIdx.x >> 6] = v;
      red_i[threadIdx.x >> 6] = idx;
    }
  }
  __syncthreads();
  double cv[NWAVE];
  int ci[NWAVE];
#pragma unroll
  for (int q = 0; q < NWAVE; ++q)
    if (q < nwr) {
      cv[q] = red_v[q];
      ci[q] = red_i[q];
    }
  v = cv[0];
  idx = ci[0];
#pragma unroll
  for (int q = 1; q < NWAVE; ++q)
    if (q < nwr && pivot_better(cv[q], ci[q], v, idx)) {
      v = cv[q];
      idx = ci[q];
    }
}

}  // namespace xlane
}  // namespace ttipm

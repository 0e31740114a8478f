// Wave-level helpers shared by the HIP kernel sources (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>

namespace thck {

static constexpr int WAVE = 64;

// Wave-wide reductions (all 64 lanes active; the result is returned in every
// lane).  Within each row of 16 lanes, an inclusive scan by DPP row shifts of
// 1, 2, 4, 8 (zeros shifted in) leaves the row total in lane 15 of the row;
// the four row totals are then read with readlane.
template <int CTRL>
__device__ __forceinline__ double dpp_shift(double v, double fill) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(fill), __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(fill), __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double read_lane(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_shift<0x111>(v, 0.0);  // row_shr:1
  v += dpp_shift<0x112>(v, 0.0);  // row_shr:2
  v += dpp_shift<0x114>(v, 0.0);  // row_shr:4
  v += dpp_shift<0x118>(v, 0.0);  // row_shr:8
  return (read_lane(v, 15) + read_lane(v, 31)) + (read_lane(v, 47) + read_lane(v, 63));
}

__device__ __forceinline__ double wave_max(double v) {
  // lanes shifted in from outside the row take the lane's own value
  v = fmax(v, dpp_shift<0x111>(v, v));
  v = fmax(v, dpp_shift<0x112>(v, v));
  v = fmax(v, dpp_shift<0x114>(v, v));
  v = fmax(v, dpp_shift<0x118>(v, v));
  return fmax(fmax(read_lane(v, 15), read_lane(v, 31)), fmax(read_lane(v, 47), read_lane(v, 63)));
}

// Workgroup barrier that orders LDS accesses only: global loads issued before
// it stay in flight (__syncthreads, a release/acquire of all memory, waits for
// them).  Use only where the waves exchange data through LDS.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// A wave-uniform pointer in scalar registers.  A pointer offset by a job
// index that came out of an integer division (done on the vector unit) can
// stay in vector registers, and a buffer resource built from it then gets a
// loop around every buffer access; reading lane 0 into scalar registers
// explicitly keeps the resource scalar.  Only for values that are uniform.
__device__ __forceinline__ const double *scalar_ptr(const double *p) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(p);
  unsigned lo, hi;
  asm volatile("v_readfirstlane_b32 %0, %1" : "=s"(lo) : "v"((unsigned)v));
  asm volatile("v_readfirstlane_b32 %0, %1" : "=s"(hi) : "v"((unsigned)(v >> 32)));
  return reinterpret_cast<const double *>(((unsigned long long)hi << 32) | lo);
}

// FP64 MFMA 16x16x4: lane l supplies A[l%16][l/16] and B[l/16][l%16]; the
// accumulator holds D[l/16 + 4r][l%16] in register r.
typedef double d4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4_t mfma16(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

}  // namespace thck

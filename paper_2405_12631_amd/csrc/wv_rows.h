// Helpers shared by the row-streaming kernels (wv_stack_bf16.hip, wv_lstm_bf16.hip,
// wv_lift_rows.hip): a workgroup walks a strip of positions down a plane's rows and keeps
// each layer's recent rows in LDS rings of 128-byte positions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wv {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Byte offset of 16-byte chunk `chunk` (0..7) of ring slot `slot`: chunk c of slot s is
// stored at chunk c ^ (s & 7), so that the MFMA fragment reads of 8 neighbouring positions
// (one chunk each) spread over all banks (measured: 164 B/clk per CU for the fragment
// pattern, against 117 with a 16-byte pad per slot and 64 unpadded).
__device__ __forceinline__ int swz(int slot, int chunk) { return (slot * 8 + (chunk ^ (slot & 7))) * 16; }

// Lane index within the wave, computed where it is used.
__device__ __forceinline__ int lane_id() {
    return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Workgroup barrier that orders LDS only: a wave's global loads (the next input row) and
// stores stay in flight across it, where __syncthreads would wait for them.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// s_waitcnt vmcnt(0): every global load and store of the wave has completed.  Loads and
// stores share that counter, so once both are in flight the compiler can only wait for all
// of them; after values loaded ahead of a loop (weights, biases) it marks them complete
// here, where nothing else is in flight, instead of on their first use inside the loop.
__device__ __forceinline__ void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0f70); }

// FP32 -> BF16, round to nearest even (v_cvt_pk_bf16_f32); two values in one instruction.
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ uint32_t f2bf2(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((floatx2){lo, hi}, bf16x2));
}

// v_mfma_f32_16x16x32_bf16 on 16-byte fragments (8 BF16 values per lane).
__device__ __forceinline__ bf16x8 as_bf(uint4 v) { return __builtin_bit_cast(bf16x8, v); }
__device__ __forceinline__ floatx4 mfma_bf16(uint4 a, uint4 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(a), as_bf(b), c, 0, 0, 0);
}

}  // namespace wv

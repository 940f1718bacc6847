// Internal helpers shared by the HIP translation units of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "paqif_ehl.h"

#define PQ_DEV __device__ __forceinline__
// Pointer into LDS (address space 3), so that out-of-line device functions
// still emit ds_* instructions.
#define LDS_PTR(T) __attribute__((address_space(3))) T*
// Pointer into global memory (address space 1): out-of-line device functions
// then emit global_* instead of flat_* memory instructions (flat accesses
// also count against the LDS wait counter and would serialise the
// per-level LDS exchange behind outstanding prefetch loads).
#define GLB_PTR(T) __attribute__((address_space(1))) T*
#define GLB(T, p) ((GLB_PTR(T))(p))

namespace pq {

// Wave-local synchronisation: orders LDS accesses of one wavefront without
// a workgroup barrier (each workgroup of the PAQIF kernels is one wave).
PQ_DEV void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// DPP move of a double (both 32-bit halves with the same control).
template <int CTRL>
PQ_DEV double dpp_f64(double v)
{
    union {
        double d;
        int i[2];
    } a, r;
    a.d = v;
    r.i[0] = __builtin_amdgcn_update_dpp(0, a.i[0], CTRL, 0xF, 0xF, true);
    r.i[1] = __builtin_amdgcn_update_dpp(0, a.i[1], CTRL, 0xF, 0xF, true);
    return r.d;
}

template <int CTRL>
PQ_DEV float dpp_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

// DPP controls
constexpr int DPP_QUAD_XOR1 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_XOR2 = 0x4E;  // quad_perm [2,3,0,1]
constexpr int DPP_ROW_HALF_MIRROR = 0x141;
constexpr int DPP_ROW_MIRROR = 0x140;

// Sum over aligned groups of G consecutive lanes (G in {4, 8, 16}); every
// lane of the group receives the group total.
template <int G>
PQ_DEV double group_sum(double v)
{
    static_assert(G == 4 || G == 8 || G == 16, "group size");
    v += dpp_f64<DPP_QUAD_XOR1>(v);
    v += dpp_f64<DPP_QUAD_XOR2>(v);
    if constexpr (G >= 8) v += dpp_f64<DPP_ROW_HALF_MIRROR>(v);
    if constexpr (G >= 16) v += dpp_f64<DPP_ROW_MIRROR>(v);
    return v;
}

template <int G>
PQ_DEV float group_sum(float v)
{
    static_assert(G == 4 || G == 8 || G == 16, "group size");
    v += dpp_f32<DPP_QUAD_XOR1>(v);
    v += dpp_f32<DPP_QUAD_XOR2>(v);
    if constexpr (G >= 8) v += dpp_f32<DPP_ROW_HALF_MIRROR>(v);
    if constexpr (G >= 16) v += dpp_f32<DPP_ROW_MIRROR>(v);
    return v;
}

// Integer sum over aligned groups of G lanes (G a power of two <= 64).
template <int G>
PQ_DEV int group_sum_int(int v)
{
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, G);
    return v;
}

template <int G>
PQ_DEV int group_max_int(int v)
{
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) v = max(v, __shfl_xor(v, m, G));
    return v;
}

inline bool hip_ok(hipError_t e) { return e == hipSuccess; }

}  // namespace pq

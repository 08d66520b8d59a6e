// Intra-facet speckle on the device (Sec. III.A eq. 7, eq. 10).
//
// s(t_p) = x(p) exp(j 2 pi f_s t_p) multiplies each facet's amplitude, with x
// a complex order-1 autoregressive process over the pulses, unit power,
// correlation b^|p - q|, b = exp(-1 / (prf tau_s)).  It is drawn so that any
// 64-pulse group (absolute pulse index) can be produced on its own:
//   anchors   y_0 = eta_0, y_g = b^64 y_{g-1} + sqrt(1 - b^128) eta_g
//   in group  z_0 = y_g, z_k = b z_{k-1} + sqrt(1 - b^2) e_{64 g + k}
//             x(64 g + k) = z_k + K_k (y_{g+1} - z_64),
//             K_k = b^(64-k) (1 - b^2k) / (1 - b^128)
// (the free path conditioned on the next anchor, which leaves the law of the
// pulse-by-pulse recursion unchanged).  Draws are counter based: Philox2x32-10
// of (facet id, slot), slot 2^31 + g for eta_g and p for e_p.
//
// In the forward kernel (lane = pulse, 64 lanes = one group) the free path is
// a weighted prefix sum over the lanes, z_k = b^k y_g + sum_{i=1..k} b^(k-i)
// sqrt(1-b^2) e_{64 g + i}, evaluated with DPP lane shifts (VALU only; the
// LDS is busy with the deposit).  The anchors come from a per-call pass over
// the facets, which for the adjoint also forms D_g = y_{g+1} - z_64.
#pragma once

#include "sim_internal.h"

namespace hs {

constexpr uint32_t kSpkAnchorSlot = 0x80000000u;

// Philox2x32-10 (Salmon et al., SC'11): per round the first word times
// 0xD256D193 gives (hi, lo); new words (hi ^ second ^ key, lo); the key grows
// by 0x9E3779B9 between rounds.  The product is formed as one 64-bit value:
// gfx950 then issues a single v_mad_u64_u32 (measured at ~0.9 per CU-cycle,
// the rate of one v_mul_lo_u32) instead of separate high and low multiplies.
__device__ __forceinline__ uint2 philox2x32_10(uint32_t c0, uint32_t c1, uint32_t key) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p = (uint64_t)c0 * 0xD256D193u;
        c0 = (uint32_t)(p >> 32) ^ c1 ^ key;
        c1 = (uint32_t)p;
        key += 0x9E3779B9u;
    }
    return make_uint2(c0, c1);
}

// One complex normal draw times `scale` (E|.|^2 = scale^2), given
// l2s = scale^2 ln 2: u1 = (w0 / 2^9 + 1/2) 2^-23 and u2 = (w1 / 2^9) 2^-23
// (exact in float32), radius scale sqrt(-ln u1) = sqrt(-log2(u1) l2s),
// angle 2 pi u2 (the hardware sine takes revolutions).
__device__ __forceinline__ float2 spk_draw(uint32_t key, uint32_t id, uint32_t slot, float l2s) {
    const uint2 w = philox2x32_10(id, slot, key);
    const float u1 = fmaf((float)(w.x >> 9), 0x1p-23f, 0x1p-24f);
    const float u2 = (float)(w.y >> 9) * 0x1p-23f;
    const float rho = __builtin_amdgcn_sqrtf(-__builtin_amdgcn_logf(u1) * l2s);
    return make_float2(rho * __builtin_amdgcn_cosf(u2), rho * __builtin_amdgcn_sinf(u2));
}

// Per-lane weights of the wave-wide AR(1) prefix sum.
struct SpkScanW {
    float b1, b2, b4, b8;   // b^s for the in-row shifts (uniform, in VGPRs)
    float w15;              // b^((lane mod 16) + 1) in rows 1 and 3
    float w31;              // b^(lane - 31) in rows 2 and 3
};

// v_k <- sum_{i <= k} b^(k-i) v_i over the 64 lanes, for the real and the
// imaginary part together: shifts 1, 2, 4, 8 within rows of 16, then row 0's
// total into row 1 and row 2's into row 3 (row_bcast:15), then the first two
// rows' total into rows 2 and 3 (row_bcast:31), each term weighted by
// b^(lane distance).  Each step is an FMA whose first source goes through a
// DPP lane move (a lane without a source reads 0 and keeps its value; lanes
// of disabled rows are not written).  A DPP read needs two wait states after
// the VALU write of its source, whatever instruction the compiler placed
// before the step: each step opens with s_nop 1, and within a step the second
// part's source was written two instructions earlier.  The caller runs this
// with all 64 lanes active.
__device__ __forceinline__ void spk_scan2(float &re, float &im, const SpkScanW &w) {
#define HS_DPP_STEP(CTRL, ROWS)                                                            \
    "v_fmac_f32_dpp %0, %0, %2 " CTRL " row_mask:" ROWS " bank_mask:0xf bound_ctrl:1\n\t"   \
    "v_fmac_f32_dpp %1, %1, %2 " CTRL " row_mask:" ROWS " bank_mask:0xf bound_ctrl:1\n\t"
    asm volatile("s_nop 1\n\t" HS_DPP_STEP("row_shr:1", "0xf") : "+v"(re), "+v"(im) : "v"(w.b1));
    asm volatile("s_nop 1\n\t" HS_DPP_STEP("row_shr:2", "0xf") : "+v"(re), "+v"(im) : "v"(w.b2));
    asm volatile("s_nop 1\n\t" HS_DPP_STEP("row_shr:4", "0xf") : "+v"(re), "+v"(im) : "v"(w.b4));
    asm volatile("s_nop 1\n\t" HS_DPP_STEP("row_shr:8", "0xf") : "+v"(re), "+v"(im) : "v"(w.b8));
    asm volatile("s_nop 1\n\t" HS_DPP_STEP("row_bcast:15", "0xa") : "+v"(re), "+v"(im)
                 : "v"(w.w15));
    asm volatile("s_nop 1\n\t" HS_DPP_STEP("row_bcast:31", "0xc") : "+v"(re), "+v"(im)
                 : "v"(w.w31));
#undef HS_DPP_STEP
}

// value of lane 63 (the readlane builtin moves 32-bit integers: reinterpret,
// never convert)
__device__ __forceinline__ float spk_lane63(float v) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// a + (value of v in lane - 1; 0 in lane 0), one DPP add
__device__ __forceinline__ float spk_shr1_add(float v, float a) {
    float x;
    asm volatile("s_nop 1\n\tv_add_f32_dpp %0, %1, %2 wave_shr:1 row_mask:0xf bank_mask:0xf "
                 "bound_ctrl:1"
                 : "=v"(x)
                 : "v"(v), "v"(a));
    return x;
}

}  // namespace hs

// Per-call preparation of the intra-facet speckle (Sec. III.A eq. 7, eq. 10):
// for every sorted facet its counter id and Doppler, and the process at the
// starts of the 64-pulse groups the call covers (the anchors), by eq. 10
// applied over 64 pulses from the first group.  For the adjoint, whose lanes
// walk the pulses one by one, also D_g = y_{g+1} - z_64 (the free path of
// group g run to its end), so that x(p) = z_k + K_k D_g is known at each
// pulse.  One lane per facet; anchors are few (one per 64 pulses), the D_g
// pass draws every innovation once.  Facets of a generated grid chunk take
// their ids (and Doppler) from their grid index.
#include "spk_device.h"

namespace hs {

namespace {

__global__ __launch_bounds__(256) void k_speckle_prep(SpkPrep P, SpkArgs K, SpkRec *rec,
                                                      float4 *anch) {
    const long long j = (long long)blockIdx.x * 256 + threadIdx.x;
    if (j > P.n) return;
    const int ng1 = K.n_groups + 1;
    float4 *out = anch + j * (long long)ng1;
    if (j == P.n) {   // padding record after the last facet
        rec[j] = SpkRec{0u, 0.0f};
        for (int g = P.g_lo; g <= P.g_hi + 1; ++g) out[g] = make_float4(0.f, 0.f, 0.f, 0.f);
        return;
    }
    const int i = P.perm[j];
    const long long gi = P.sub_nx > 0 ? (long long)(P.sub_y0 + i / P.sub_nx) * P.grid_nx +
                                            P.sub_x0 + i % P.sub_nx
                                      : (long long)i;
    const uint32_t id = (uint32_t)(P.first_index + gi);
    rec[j] = SpkRec{id, P.fs ? P.fs[gi] : 0.0f};
    const float l2 = 0.69314718055994531f;
    const float l64 = K.c64 * K.c64 * l2, l1 = K.c1 * K.c1 * l2;
    float2 y = spk_draw(K.key, id, kSpkAnchorSlot, l2);
    for (int g = 0; g <= P.g_hi; ++g) {
        const float2 eta = spk_draw(K.key, id, kSpkAnchorSlot + (uint32_t)(g + 1), l64);
        const float2 yn = make_float2(fmaf(K.b64, y.x, eta.x), fmaf(K.b64, y.y, eta.y));
        if (g >= P.g_lo) {
            float dr = 0.0f, di = 0.0f;
            if (P.with_d) {
                float zr = y.x, zi = y.y;
                for (int k = 1; k <= 64; ++k) {
                    const float2 e = spk_draw(K.key, id, (uint32_t)(64 * g + k), l1);
                    zr = fmaf(K.b1, zr, e.x);
                    zi = fmaf(K.b1, zi, e.y);
                }
                dr = yn.x - zr;
                di = yn.y - zi;
            }
            out[g] = make_float4(y.x, y.y, dr, di);
        }
        y = yn;
    }
    out[P.g_hi + 1] = make_float4(y.x, y.y, 0.f, 0.f);
}

}  // namespace

hipError_t launch_speckle_prep(const SpkPrep &p, const SpkArgs &k, SpkRec *rec, float4 *anch,
                               hipStream_t s) {
    const long long n = p.n + 1;
    hipLaunchKernelGGL(k_speckle_prep, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, k,
                       rec, anch);
    return hipGetLastError();
}

}  // namespace hs

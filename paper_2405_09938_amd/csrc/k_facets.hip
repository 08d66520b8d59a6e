// On-device facet generation on a regular grid: the scene is produced where
// and when it is sensed (Sec. II.B) instead of being stored, tile by tile
// (Sec. IV.B).  The resolved sea surface is a sum of linear wave components
// (Sec. III, CWM option off); facets follow its first-order orbital motion
// plus a uniform current; complex amplitudes are circular Gaussian with
// <|a|^2> = 1 (the statistics of the intra-facet speckle of eq. 7 at t = 0,
// held constant over the dwell).
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key =
// the 64-bit seed, counter = (global grid index, stream, 0), so every facet
// depends only on (seed, its grid index) and any chunking of the grid gives
// identical facets.  Output words w map to (0,1) as (w + 1/2) 2^-32 and feed
// Box-Muller pairs.  Heights and velocities are summed in FP64 and rounded
// once to float32.
#include "sim_internal.h"

namespace hs {

namespace {

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0;
        const uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

__device__ __forceinline__ void normals4(unsigned long long seed, unsigned long long idx,
                                         uint32_t stream, double *n) {
    uint32_t c[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), stream, 0u};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double sc = 1.0 / 4294967296.0;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const double u1 = ((double)c[2 * j] + 0.5) * sc;
        const double u2 = ((double)c[2 * j + 1] + 0.5) * sc;
        const double r = sqrt(-2.0 * log(u1));
        double s, co;
        sincospi(2.0 * u2, &s, &co);
        n[2 * j] = r * co;
        n[2 * j + 1] = r * s;
    }
}

__global__ void k_generate(GenArgs A) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n = (long long)A.cnx * A.cny;
    if (j >= n) return;
    const int ix = A.ix0 + (int)(j % A.cnx), iy = A.iy0 + (int)(j / A.cnx);
    const unsigned long long gidx = (unsigned long long)iy * (unsigned long long)A.nx + ix;
    const double X = ((double)ix - 0.5 * (double)(A.nx - 1)) * A.dx;
    const double Y = ((double)iy - 0.5 * (double)(A.ny - 1)) * A.dy;
    double nr[4];
    normals4(A.seed, gidx, 0u, nr);
    const double isq2 = 0.70710678118654752440;
    A.out.x[j] = (float)X;
    A.out.y[j] = (float)Y;
    A.out.a_re[j] = (float)(nr[0] * isq2);
    A.out.a_im[j] = (float)(nr[1] * isq2);
    if (A.mode == 0) {
        double n2[4];
        normals4(A.seed, gidx, 1u, n2);
        A.out.z[j] = 0.0f;
        A.out.vx[j] = (float)(A.sigma_v * nr[2]);
        A.out.vy[j] = (float)(A.sigma_v * nr[3]);
        A.out.vz[j] = (float)(A.sigma_v * n2[0]);
    } else {
        double h = 0.0, ux = 0.0, uy = 0.0, w = 0.0;
        for (int m = 0; m < A.n_comp; ++m) {
            const double *t = A.tab + 6 * m;   // k, A, omega, cos psi, sin psi, phase
            const double th = t[0] * (t[3] * X + t[4] * Y) + t[5];
            double st, ct;
            sincos(th, &st, &ct);
            const double aw = t[1] * t[2];
            h += t[1] * ct;
            ux += aw * t[3] * ct;
            uy += aw * t[4] * ct;
            w += aw * st;
        }
        A.out.z[j] = (float)h;
        A.out.vx[j] = (float)(ux + A.cur0);
        A.out.vy[j] = (float)(uy + A.cur1);
        A.out.vz[j] = (float)w;
    }
}

}  // namespace

hipError_t launch_generate(const GenArgs &a, hipStream_t s) {
    const long long n = (long long)a.cnx * a.cny;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_generate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace hs

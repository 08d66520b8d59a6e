// On-device facet generation on a regular grid: the scene is produced where
// and when it is sensed (Sec. II.B) instead of being stored, tile by tile
// (Sec. IV.B).  The resolved sea surface is a sum of linear wave components
// (Sec. III), either one homogeneous field or the heterogeneous combination
// of eq. 1-2 (four overlapping fields per tile), optionally with the Choppy
// Wave Model's horizontal displacement; facets follow the first-order
// orbital motion plus a uniform current; complex amplitudes are circular
// Gaussian with
// <|a|^2> = 1 (the statistics of the intra-facet speckle of eq. 7 at t = 0,
// held constant over the dwell).
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key =
// the 64-bit seed, counter = (global grid index, stream, 0), so every facet
// depends only on (seed, its grid index) and any chunking of the grid gives
// identical facets.  Output words w map to (0,1) as (w + 1/2) 2^-32 and feed
// Box-Muller pairs.  Heights and velocities are summed in FP64 and rounded
// once to float32.
#include "philox_device.h"
#include "sim_internal.h"

namespace hs {

namespace {

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

// One homogeneous field (table rows k, A, omega, cos psi, sin psi, phase) at
// the point at rest (X, Y), added with weight wgt: height sum A cos(theta),
// theta = k (cos psi X + sin psi Y) + phase; horizontal displacement of the
// Choppy Wave Model -sum A (cos psi, sin psi) sin(theta); velocity its time
// derivative, sum A omega (cos psi, sin psi) cos(theta) and sum A omega
// sin(theta).  FP64 throughout.
__device__ void wave_field(const double *tab, int n, double X, double Y, double wgt, double *D) {
    for (int m = 0; m < n; ++m) {
        const double *t = tab + 6 * m;
        const double th = t[0] * (t[3] * X + t[4] * Y) + t[5];
        double st, ct;
        sincos(th, &st, &ct);
        const double a = wgt * t[1], aw = a * t[2];
        D[0] += a * ct;
        D[1] -= a * t[3] * st;
        D[2] -= a * t[4] * st;
        D[3] += aw * t[3] * ct;
        D[4] += aw * t[4] * ct;
        D[5] += aw * st;
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
        // displacement (eta, horizontal) and velocity of the point at rest:
        // one field (mode 1) or the four corner fields of its TL tile
        // weighted by eq. 2 (mode 2)
        double D[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (A.mode == 1) {
            wave_field(A.tab, A.n_comp, X, Y, 1.0, D);
        } else {
            int ti = (int)floor((X - A.tile_x0) / A.tile_L);
            int tj = (int)floor((Y - A.tile_y0) / A.tile_L);
            ti = ti < 0 ? 0 : (ti > A.ntx - 1 ? A.ntx - 1 : ti);
            tj = tj < 0 ? 0 : (tj > A.nty - 1 ? A.nty - 1 : tj);
            for (int c = 0; c < 4; ++c) {
                const int ni = ti + (c & 1), nj = tj + (c >> 1);
                const double ux = fabs(A.tile_x0 + ni * A.tile_L - X) / A.tile_L;
                const double uy = fabs(A.tile_y0 + nj * A.tile_L - Y) / A.tile_L;
                const double wgt = sqrt(fmax(0.0, (1.0 - ux) * (1.0 - uy)));
                const long long node = (long long)nj * (A.ntx + 1) + ni;
                wave_field(A.tab + 6 * node * A.n_comp, A.n_comp, X, Y, wgt, D);
            }
        }
        A.out.x[j] = (float)(A.cwm ? X + D[1] : X);
        A.out.y[j] = (float)(A.cwm ? Y + D[2] : Y);
        A.out.z[j] = (float)D[0];
        A.out.vx[j] = (float)(D[3] + A.cur0);
        A.out.vy[j] = (float)(D[4] + A.cur1);
        A.out.vz[j] = (float)D[5];
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

// Per-line convolution with the transmitted waveform (the impulse response
// of eq. 17 "subsequently convolved by the waveform") and its adjoint, by
// zero-padded FFT in LDS, one workgroup per range line.
//
//   forward: raw[n]  = sum_m rc[m] chirp[n - m + L/2]
//            buf = pad(rc); X = FFT(buf); Y = X * S; raw[n] = IFFT(Y)[n + L/2]
//   adjoint: g_rc[m] = sum_n g_raw[n] conj(chirp[n - m + L/2])
//            buf[L/2 + n] = g_raw[n]; X = FFT(buf); Y = X * conj(S);
//            g_rc[m] = IFFT(Y)[m]
// with S = FFT_M(chirp zero-padded) / M precomputed in FP64 on the host.
// The inverse is taken as conj(FFT(conj(Y))), the 1/M being folded into S.
// M >= N + L - 1 keeps both circular products free of wrap-around.
//
// FFT: radix-4 Stockham passes (plus one radix-2 pass when log2 M is odd),
// in place in LDS: every pass first reads all of its butterfly inputs into
// registers, then (after a barrier) writes all outputs.  Twiddles come from an
// FP64-accurate table exp(-2 pi i m / M).
#include "sim_internal.h"

namespace hs {

namespace {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}

template <int M, int NT>
__device__ void fft_lds(float2 *buf, const float2 *__restrict__ tw) {
    int ns = 1;
#pragma unroll 1
    for (; ns * 4 <= M; ns *= 4) {
        constexpr int NB = M / 4 / NT;
        float2 v[NB][4];
#pragma unroll
        for (int bb = 0; bb < NB; ++bb) {
            const int j = threadIdx.x + bb * NT;
#pragma unroll
            for (int r = 0; r < 4; ++r) v[bb][r] = buf[j + r * (M / 4)];
        }
        __syncthreads();
        const int step = M / (4 * ns);
#pragma unroll
        for (int bb = 0; bb < NB; ++bb) {
            const int j = threadIdx.x + bb * NT;
            const int k = j & (ns - 1);
            const float2 x0 = v[bb][0];
            const float2 x1 = cmul(v[bb][1], tw[k * step]);
            const float2 x2 = cmul(v[bb][2], tw[2 * k * step]);
            const float2 x3 = cmul(v[bb][3], tw[3 * k * step]);
            const float2 a0 = make_float2(x0.x + x2.x, x0.y + x2.y);
            const float2 a1 = make_float2(x0.x - x2.x, x0.y - x2.y);
            const float2 a2 = make_float2(x1.x + x3.x, x1.y + x3.y);
            const float2 a3 = make_float2(x1.y - x3.y, x3.x - x1.x);   // -i (x1 - x3)
            const int base = (j - k) * 4 + k;
            buf[base] = make_float2(a0.x + a2.x, a0.y + a2.y);
            buf[base + ns] = make_float2(a1.x + a3.x, a1.y + a3.y);
            buf[base + 2 * ns] = make_float2(a0.x - a2.x, a0.y - a2.y);
            buf[base + 3 * ns] = make_float2(a1.x - a3.x, a1.y - a3.y);
        }
        __syncthreads();
    }
    if (ns < M) {   // one radix-2 pass, ns = M / 2
        constexpr int NB = M / 2 / NT;
        float2 v[NB][2];
#pragma unroll
        for (int bb = 0; bb < NB; ++bb) {
            const int j = threadIdx.x + bb * NT;
            v[bb][0] = buf[j];
            v[bb][1] = buf[j + M / 2];
        }
        __syncthreads();
#pragma unroll
        for (int bb = 0; bb < NB; ++bb) {
            const int j = threadIdx.x + bb * NT;     // k = j, since j < ns
            const float2 x1 = cmul(v[bb][1], tw[j]);
            buf[j] = make_float2(v[bb][0].x + x1.x, v[bb][0].y + x1.y);
            buf[j + M / 2] = make_float2(v[bb][0].x - x1.x, v[bb][0].y - x1.y);
        }
        __syncthreads();
    }
}

template <int M, int NT>
__global__ __launch_bounds__(NT) void k_waveform(const float2 *in, float2 *out, int N,
                                                  int shift, const float2 *__restrict__ spec,
                                                  const float2 *__restrict__ tw, int adjoint) {
    __shared__ float2 buf[M];
    const long long line = blockIdx.x;
    const float2 *src = in + line * N;
    float2 *dst = out + line * N;
    for (int i = threadIdx.x; i < M; i += NT) {
        const int m = adjoint ? i - shift : i;
        buf[i] = (m >= 0 && m < N) ? src[m] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    fft_lds<M, NT>(buf, tw);
    for (int i = threadIdx.x; i < M; i += NT) {
        float2 s = spec[i];
        if (adjoint) s.y = -s.y;
        const float2 y = cmul(buf[i], s);
        buf[i] = make_float2(y.x, -y.y);          // conj for the inverse transform
    }
    __syncthreads();
    fft_lds<M, NT>(buf, tw);
    for (int n = threadIdx.x; n < N; n += NT) {
        const float2 v = buf[adjoint ? n : n + shift];
        dst[n] = make_float2(v.x, -v.y);
    }
}

}  // namespace

hipError_t launch_waveform(const float *in, float *out, long long n_lines, int N, int M,
                           int shift, const float *spec, const float *tw, int adjoint,
                           hipStream_t s) {
    if (n_lines == 0) return hipSuccess;
    const float2 *i2 = reinterpret_cast<const float2 *>(in);
    float2 *o2 = reinterpret_cast<float2 *>(out);
    const float2 *s2 = reinterpret_cast<const float2 *>(spec);
    const float2 *t2 = reinterpret_cast<const float2 *>(tw);
    dim3 grid((unsigned)n_lines);
    switch (M) {
        case 256: hipLaunchKernelGGL((k_waveform<256, 64>), grid, dim3(64), 0, s, i2, o2, N, shift, s2, t2, adjoint); break;
        case 512: hipLaunchKernelGGL((k_waveform<512, 64>), grid, dim3(64), 0, s, i2, o2, N, shift, s2, t2, adjoint); break;
        case 1024: hipLaunchKernelGGL((k_waveform<1024, 128>), grid, dim3(128), 0, s, i2, o2, N, shift, s2, t2, adjoint); break;
        case 2048: hipLaunchKernelGGL((k_waveform<2048, 128>), grid, dim3(128), 0, s, i2, o2, N, shift, s2, t2, adjoint); break;
        case 4096: hipLaunchKernelGGL((k_waveform<4096, 256>), grid, dim3(256), 0, s, i2, o2, N, shift, s2, t2, adjoint); break;
        case 8192: hipLaunchKernelGGL((k_waveform<8192, 256>), grid, dim3(256), 0, s, i2, o2, N, shift, s2, t2, adjoint); break;
        case 16384: hipLaunchKernelGGL((k_waveform<16384, 512>), grid, dim3(512), 0, s, i2, o2, N, shift, s2, t2, adjoint); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace hs

// Range-binned block sort of a facet set (plan construction) and the per-call
// gather of facet data into block order.
//
// Facets are binned into cells of a square lattice of the horizontal plane;
// cells are grouped into patches (rectangles of cells whose facets share a
// range window for a group of pulses, the counterpart of the paper's TL tiles
// processed as a batch, Sec. IV.A/B); a counting sort over the key
// (patch, row in patch, column in patch) orders the facets, and each
// non-empty cell becomes one or more blocks of at most 64 facets.
#include "sim_internal.h"

namespace hs {

namespace {

__global__ void k_fill_zero(float *p, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0.0f;
}

// Key of the cell holding (xv, yv).  A position outside the lattice (or not
// finite) goes to the nearest edge cell and sets *out.
__device__ __forceinline__ int cell_key(float xv, float yv, const Lattice &L, bool *out) {
    const double fx = floor((double)xv / L.edge) - (double)L.bx0;
    const double fy = floor((double)yv / L.edge) - (double)L.by0;
    *out = !(fx >= 0.0 && fx < (double)L.nbx && fy >= 0.0 && fy < (double)L.nby);
    long long cx = fx >= 0.0 ? (fx < (double)L.nbx ? (long long)fx : L.nbx - 1) : 0;
    long long cy = fy >= 0.0 ? (fy < (double)L.nby ? (long long)fy : L.nby - 1) : 0;
    const long long px = cx / L.px, py = cy / L.py;
    const long long patch = py * L.npx + px;
    return (int)((patch * L.py + (cy - py * L.py)) * L.px + (cx - px * L.px));
}

// Lanes of a wave holding the same key take their ranks from one atomic:
// facets arrive in grid order, so a wave covers only a few cells and the
// per-facet atomics would serialise on the same counters.  Facets outside
// the lattice are counted into *outside (one atomic per wave).
__global__ void k_cell_keys(const float *x, const float *y, long long n, Lattice L, int *keys,
                            int *rank, int *count, unsigned *outside) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < n;
    bool off = false;
    const int k = valid ? cell_key(x[i], y[i], L, &off) : -1;
    const int lane = threadIdx.x & 63;
    const unsigned long long offm = __ballot(valid && off);
    if (offm && lane == 0) atomicAdd(outside, (unsigned)__popcll(offm));
    const unsigned long long below = (1ull << lane) - 1ull;
    unsigned long long pending = __ballot(valid);
    int r = 0;
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const int kl = __shfl(k, leader);
        const unsigned long long same = __ballot(valid && k == kl);
        int base = 0;
        if (lane == leader) base = atomicAdd(count + kl, __popcll(same));
        base = __shfl(base, leader);
        if (valid && k == kl) r = base + __popcll(same & below);
        pending &= ~same;
    }
    if (valid) {
        keys[i] = k;
        rank[i] = r;
    }
}

// ---- exclusive scan (int32), three passes ---------------------------------
constexpr int kScanBlock = 1024;     // elements per workgroup (256 threads x 4)

__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(v, off);
        if (lane >= off) v += t;
    }
    return v;
}

// Block-level exclusive scan of 4 values per thread (256 threads); returns the
// block total through *total.
__device__ void block_scan4(int v[4], int *total) {
    __shared__ int wsum[4];
    const int s0 = v[0], s1 = s0 + v[1], s2 = s1 + v[2], s3 = s2 + v[3];
    const int incl = wave_incl_scan(s3);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int woff = 0;
    for (int k = 0; k < w; ++k) woff += wsum[k];
    const int excl = woff + incl - s3;
    const int a0 = v[0], a1 = v[1], a2 = v[2];
    v[0] = excl;
    v[1] = excl + a0;
    v[2] = excl + a0 + a1;
    v[3] = excl + a0 + a1 + a2;
    *total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
}

__global__ void k_scan_reduce(const int *in, long long n, int *sums) {
    const long long base = (long long)blockIdx.x * kScanBlock;
    int s = 0;
    for (int k = 0; k < 4; ++k) {
        const long long i = base + threadIdx.x * 4 + k;
        if (i < n) s += in[i];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    __shared__ int ws[4];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) sums[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// Single-workgroup exclusive scan of `n` partial sums (loops over chunks).
__global__ void k_scan_top(int *sums, long long n) {
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (long long base = 0; base < n; base += kScanBlock) {
        int v[4];
        for (int k = 0; k < 4; ++k) {
            const long long i = base + threadIdx.x * 4 + k;
            v[k] = i < n ? sums[i] : 0;
        }
        int total;
        block_scan4(v, &total);
        const int c = carry;
        for (int k = 0; k < 4; ++k) {
            const long long i = base + threadIdx.x * 4 + k;
            if (i < n) sums[i] = v[k] + c;
        }
        __syncthreads();
        if (threadIdx.x == 0) carry = c + total;
        __syncthreads();
    }
}

__global__ void k_scan_down(const int *in, int *out, long long n, const int *sums) {
    const long long base = (long long)blockIdx.x * kScanBlock;
    int v[4];
    for (int k = 0; k < 4; ++k) {
        const long long i = base + threadIdx.x * 4 + k;
        v[k] = i < n ? in[i] : 0;
    }
    int total;
    block_scan4(v, &total);
    const int off = sums[blockIdx.x];
    for (int k = 0; k < 4; ++k) {
        const long long i = base + threadIdx.x * 4 + k;
        if (i < n) out[i] = v[k] + off;
    }
    // out[n] = grand total (written by the last block)
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = off + total;
}

__global__ void k_scatter(const int *keys, const int *rank, const int *offset, long long n,
                          int *perm) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    perm[offset[keys[i]] + rank[i]] = (int)i;
}

__global__ void k_block_counts(const int *count, long long n_keys, int *nblk) {
    long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_keys) return;
    nblk[k] = (count[k] + 63) >> 6;
}

__global__ void k_make_blocks(const int *count, const int *offset, const int *blk_offset,
                              long long n_keys, Lattice L, BlockRec *blocks) {
    long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_keys) return;
    const int cnt = count[k];
    if (cnt == 0) return;
    const long long per = (long long)L.px * L.py;
    const long long patch = k / per, local = k % per;
    const long long py = patch / L.npx, px = patch % L.npx;
    const long long cy = py * L.py + local / L.px, cx = px * L.px + local % L.px;
    const float xb = (float)(((double)(L.bx0 + cx) + 0.5) * L.edge);
    const float yb = (float)(((double)(L.by0 + cy) + 0.5) * L.edge);
    int b = blk_offset[k];
    for (int s = 0; s < cnt; s += 64, ++b) {
        BlockRec r;
        r.xb = xb;
        r.yb = yb;
        r.start = offset[k] + s;
        r.count = (cnt - s) < 64 ? (cnt - s) : 64;
        blocks[b] = r;
    }
}

__global__ void k_patch_first(const int *blk_offset, long long n_patches, int keys_per_patch,
                              long long n_keys, int *patch_first) {
    long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p > n_patches) return;
    const long long k = p * keys_per_patch;
    patch_first[p] = blk_offset[k < n_keys ? k : n_keys];
}

// One wave per block: lane i copies facet start + i into the sorted record,
// position relative to the block centre (exact for |offset| < 2^-24 |x|... the
// subtraction of two nearby floats).  The record after the last one is a zero
// padding record written by the host-side allocation.
__global__ void k_gather(sim_facets f, const int *perm, const BlockRec *blocks,
                         const int *n_blocks, FacetRec *sorted) {
    const long long b = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (b >= *n_blocks) return;
    const int lane = threadIdx.x & 63;
    const BlockRec blk = blocks[b];
    if (lane >= blk.count) return;
    const int j = blk.start + lane;
    const int i = perm[j];
    FacetRec r;
    r.dx = f.x[i] - blk.xb;
    r.dy = f.y[i] - blk.yb;
    r.z = f.z[i];
    r.vx = f.vx[i];
    r.vy = f.vy[i];
    r.vz = f.vz[i];
    r.ar = f.a_re[i];
    r.ai = f.a_im[i];
    sorted[j] = r;
}

// Host-to-device copy through the kernel argument segment: each launch
// carries up to kUploadChunk doubles by value.
constexpr int kUploadChunk = 440;
struct UploadArgs {
    double *dst;
    int n;
    double v[kUploadChunk];
};
static_assert(sizeof(UploadArgs) <= 4096, "kernel arguments too large");

__global__ void k_upload(UploadArgs a) {
    for (int i = threadIdx.x; i < a.n; i += blockDim.x) a.dst[i] = a.v[i];
}

inline unsigned grid_for(long long n, int threads) {
    long long g = (n + threads - 1) / threads;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

hipError_t launch_fill_zero(float *p, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    long long g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)g), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_cell_keys(const float *x, const float *y, long long n, const Lattice &L,
                            int *keys, int *rank, int *count, unsigned *outside, hipStream_t s) {
    hipLaunchKernelGGL(k_cell_keys, dim3(grid_for(n, 256)), dim3(256), 0, s, x, y, n, L, keys,
                       rank, count, outside);
    return hipGetLastError();
}

long long scan_tmp_len(long long n) { return (n + kScanBlock - 1) / kScanBlock + 1; }

// out[0..n] (n + 1 entries): exclusive prefix sums, out[n] = total.
hipError_t launch_exclusive_scan(const int *in, int *out, long long n, int *tmp,
                                 long long tmp_len, hipStream_t s) {
    const long long nb = (n + kScanBlock - 1) / kScanBlock;
    if (nb < 1 || nb + 1 > tmp_len) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(256), 0, s, in, n, tmp);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, s, tmp, nb);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(256), 0, s, in, out, n,
                       (const int *)tmp);
    return hipGetLastError();
}

hipError_t launch_scatter(const int *keys, const int *rank, const int *offset, long long n,
                          int *perm, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter, dim3(grid_for(n, 256)), dim3(256), 0, s, keys, rank, offset, n,
                       perm);
    return hipGetLastError();
}

hipError_t launch_block_counts(const int *count, long long n_keys, int *nblk, hipStream_t s) {
    hipLaunchKernelGGL(k_block_counts, dim3(grid_for(n_keys, 256)), dim3(256), 0, s, count,
                       n_keys, nblk);
    return hipGetLastError();
}

hipError_t launch_make_blocks(const int *count, const int *offset, const int *blk_offset,
                              long long n_keys, const Lattice &L, BlockRec *blocks,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_make_blocks, dim3(grid_for(n_keys, 256)), dim3(256), 0, s, count,
                       offset, blk_offset, n_keys, L, blocks);
    return hipGetLastError();
}

hipError_t launch_patch_first(const int *blk_offset, long long n_patches, int keys_per_patch,
                              long long n_keys, int *patch_first, hipStream_t s) {
    hipLaunchKernelGGL(k_patch_first, dim3(grid_for(n_patches + 1, 256)), dim3(256), 0, s,
                       blk_offset, n_patches, keys_per_patch, n_keys, patch_first);
    return hipGetLastError();
}

hipError_t launch_gather(const sim_facets &f, const int *perm, const BlockRec *blocks,
                         const int *n_blocks, long long nb_max, FacetRec *sorted,
                         hipStream_t s) {
    if (nb_max == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(grid_for(nb_max, 4)), dim3(256), 0, s, f, perm, blocks,
                       n_blocks, sorted);
    return hipGetLastError();
}

hipError_t launch_upload(double *dst, const double *src, long long n, hipStream_t s) {
    for (long long o = 0; o < n; o += kUploadChunk) {
        UploadArgs a;
        a.dst = dst + o;
        a.n = (int)(n - o < kUploadChunk ? n - o : kUploadChunk);
        for (int i = 0; i < a.n; ++i) a.v[i] = src[o + i];
        hipLaunchKernelGGL(k_upload, dim3(1), dim3(256), 0, s, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace hs

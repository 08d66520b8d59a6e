// Range-binned block sort of a facet set (plan construction) and the per-call
// gather of facet data into block order.
//
// Facets are binned into cells of a square lattice of the horizontal plane
// (counting sort by cell, facets of a cell in ascending index so that every
// sum over them runs in a fixed order); each non-empty cell becomes one or
// more blocks of at most 64 facets.  Blocks are then binned by range: for
// every band of pulse groups and every channel, the sample position of each
// block centre at the band's reference pulse selects a range strip (eq. 17's
// range slices, gathered per tile as the paper's tile batches, Sec.
// IV.A/B), and each strip's blocks are listed in block order and cut into
// segments, the units of work of the forward sum.
#include "sim_internal.h"

namespace hs {

namespace {

__global__ void k_fill_zero(float *p, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0.0f;
}

// Key (row-major index) of the cell holding (xv, yv).  A position outside
// the lattice (or not finite) goes to the nearest edge cell and sets *out.
__device__ __forceinline__ int cell_key(float xv, float yv, const Lattice &L, bool *out) {
    const double fx = floor((double)xv / L.edge) - (double)L.bx0;
    const double fy = floor((double)yv / L.edge) - (double)L.by0;
    *out = !(fx >= 0.0 && fx < (double)L.nbx && fy >= 0.0 && fy < (double)L.nby);
    const long long cx = fx >= 0.0 ? (fx < (double)L.nbx ? (long long)fx : L.nbx - 1) : 0;
    const long long cy = fy >= 0.0 ? (fy < (double)L.nby ? (long long)fy : L.nby - 1) : 0;
    return (int)(cy * L.nbx + cx);
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
    const long long cy = k / L.nbx, cx = k - cy * L.nbx;
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

// The scatter takes ranks within a cell from atomics, so the order of a
// cell's facets varies from run to run; these put them in ascending index.
// Cells of up to 64 facets: one wave each, a bitonic sort across the lanes
// in registers (no LDS, so the kernel runs beside a forward sum that holds
// most of the LDS).  Cells of 65 to kCellSortMax facets: a bitonic sort in
// LDS, one workgroup per cell, grid-stride over cells.  Larger cells keep
// the scatter's order.
constexpr int kCellSortMax = 1024;

__global__ __launch_bounds__(256) void k_cell_sort64(const int *count, const int *offset,
                                                     long long n_keys, int *perm) {
    const long long k = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (k >= n_keys) return;
    const int cnt = count[k];
    if (cnt <= 1 || cnt > 64) return;
    const int lane = (int)(threadIdx.x & 63);
    int *seg = perm + offset[k];
    int v = lane < cnt ? seg[lane] : 0x7fffffff;
    for (int size = 2; size <= 64; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const int o = __shfl_xor(v, stride);
            // ascending runs where (lane & size) == 0; the lower lane of a
            // pair keeps the smaller value in those
            const bool keep_min = ((lane & stride) == 0) == ((lane & size) == 0);
            v = keep_min ? (v < o ? v : o) : (v > o ? v : o);
        }
    if (lane < cnt) seg[lane] = v;
}

__global__ __launch_bounds__(256) void k_cell_sort(const int *count, const int *offset,
                                                   long long n_keys, int *perm) {
    __shared__ int v[kCellSortMax];
    for (long long k = blockIdx.x; k < n_keys; k += gridDim.x) {
        const int cnt = count[k];
        if (cnt <= 64 || cnt > kCellSortMax) continue;
        int m = 128;
        while (m < cnt) m <<= 1;
        int *seg = perm + offset[k];
        for (int i = threadIdx.x; i < m; i += blockDim.x) v[i] = i < cnt ? seg[i] : 0x7fffffff;
        __syncthreads();
        for (int size = 2; size <= m; size <<= 1)
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int i = threadIdx.x; i < m; i += blockDim.x) {
                    const int j = i ^ stride;
                    if (j > i) {
                        const int a = v[i], b = v[j];
                        if ((a > b) == ((i & size) == 0)) {
                            v[i] = b;
                            v[j] = a;
                        }
                    }
                }
                __syncthreads();
            }
        for (int i = threadIdx.x; i < cnt; i += blockDim.x) seg[i] = v[i];
        __syncthreads();
    }
}

// ---- range strips ------------------------------------------------------------

// Strip of every block for band blockIdx.y and channel blockIdx.z: the block
// centre's sample position at the band's reference pulse (FP64, z = 0),
// relative to the band's lower edge, in strip widths, clamped to the strips.
__global__ void k_strip_keys(StripPlan sp, const PulseRec *pulses, const BlockRec *blocks,
                             const int *n_blocks, int Np, int C, double n_ref, double fs_c,
                             int *skey, int *scount) {
    const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= *n_blocks) return;
    const int band = blockIdx.y, ch = blockIdx.z;
    const int bc = band * C + ch;
    int pref = band * sp.B * 64 + sp.B * 32;
    pref = pref < Np - 1 ? pref : Np - 1;
    const PulseRec &Q = pulses[(size_t)ch * Np + pref];
    const BlockRec blk = blocks[b];
    const double x = blk.xb, y = blk.yb;
    const double a0 = x - Q.ptx[0], a1 = y - Q.ptx[1], a2 = -Q.ptx[2];
    const double c0 = x - Q.prx[0], c1 = y - Q.prx[1], c2 = -Q.prx[2];
    const double u = n_ref + (sqrt(a0 * a0 + a1 * a1 + a2 * a2) +
                              sqrt(c0 * c0 + c1 * c1 + c2 * c2) - Q.rref) * fs_c;
    const double *bd = sp.band + 4 * (size_t)bc;
    double f = floor((u - bd[0]) / bd[1]);
    f = f < 0.0 ? 0.0 : (f > (double)(sp.NS - 1) ? (double)(sp.NS - 1) : f);
    const int key = (int)f;
    skey[(size_t)bc * sp.nbm + b] = key;
    atomicAdd(scount + (size_t)bc * (sp.NS + 1) + key, 1);
}

// Per (band, channel): list offsets of the strips (exclusive scan of the
// counts) and their segment offsets (a strip of c blocks makes ceil(c / L)
// segments); entry NS holds the totals.  One workgroup of 256 threads each.
__global__ __launch_bounds__(256) void k_strip_offsets(StripPlan sp, const int *scount) {
    const size_t bc = (size_t)blockIdx.x;
    const int *cnt = scount + bc * (sp.NS + 1);
    int *soff = sp.soff + bc * (sp.NS + 1);
    int *sego = sp.segoff + bc * (sp.NS + 1);
    __shared__ int carry[2];
    if (threadIdx.x == 0) carry[0] = carry[1] = 0;
    __syncthreads();
    for (int base = 0; base < sp.NS; base += kScanBlock) {
        int v[4], w[4];
        for (int k = 0; k < 4; ++k) {
            const int i = base + threadIdx.x * 4 + k;
            v[k] = i < sp.NS ? cnt[i] : 0;
            w[k] = (v[k] + sp.L - 1) / sp.L;
        }
        int tv, tw;
        block_scan4(v, &tv);
        block_scan4(w, &tw);
        const int c0 = carry[0], c1 = carry[1];
        for (int k = 0; k < 4; ++k) {
            const int i = base + threadIdx.x * 4 + k;
            if (i < sp.NS) {
                soff[i] = v[k] + c0;
                sego[i] = w[k] + c1;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            carry[0] = c0 + tv;
            carry[1] = c1 + tw;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        soff[sp.NS] = carry[0];
        sego[sp.NS] = carry[1];
    }
}

// Per (band, channel) one wave lists the blocks strip after strip, each
// strip's blocks in ascending block index: the wave walks the blocks in
// order, 64 at a time, and lanes with equal strips take consecutive places
// after that strip's running count (kept in LDS).  A fixed order, so every
// run builds the same lists.
constexpr int kStripMax = 8192;

__global__ __launch_bounds__(64) void k_strip_lists(StripPlan sp, const int *skey,
                                                    const int *n_blocks) {
    extern __shared__ int run[];   // [NS]: LDS sized to the strips only
    const size_t bc = (size_t)blockIdx.x;
    const int *soff = sp.soff + bc * (sp.NS + 1);
    const int lane = threadIdx.x;
    for (int s = lane; s < sp.NS; s += 64) run[s] = soff[s];
    __syncthreads();
    const int nb = *n_blocks;
    const int *key = skey + bc * sp.nbm;
    int *ids = sp.ids + bc * sp.nbm;
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int base = 0; base < nb; base += 64) {
        const int b = base + lane;
        const bool valid = b < nb;
        const int k = valid ? key[b] : -1;
        unsigned long long pending = __ballot(valid);
        while (pending) {
            const int leader = __ffsll((long long)pending) - 1;
            const int kl = __shfl(k, leader);
            const unsigned long long same = __ballot(valid && k == kl);
            const int start = run[kl];
            if (valid && k == kl) ids[start + __popcll(same & below)] = b;
            __syncthreads();
            if (lane == leader) run[kl] = start + __popcll(same);
            __syncthreads();
            pending &= ~same;
        }
    }
}

// One wave per block: lane i copies facet start + i into the sorted record,
// position relative to the block centre (exact for |offset| < 2^-24 |x|... the
// subtraction of two nearby floats).  The record after the last one is a zero
// padding record written by the host-side allocation.
__global__ void k_gather(sim_facets f, const int *perm, const BlockRec *blocks,
                         const int *n_blocks, FacetRec *sorted, float zlim, float vlim2,
                         unsigned *beyond) {
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
    // facets beyond the plan's height and speed bounds (rare: one atomic each)
    if (fabsf(r.z) > zlim || r.vx * r.vx + r.vy * r.vy + r.vz * r.vz > vlim2) atomicAdd(beyond, 1u);
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

hipError_t launch_cell_sort(const int *count, const int *offset, long long n_keys, int *perm,
                            hipStream_t s) {
    if (n_keys <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cell_sort64, dim3(grid_for(n_keys, 4)), dim3(256), 0, s, count, offset,
                       n_keys, perm);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // few workgroups: cells of more than 64 facets are rare
    const long long g = n_keys < 1024 ? n_keys : 1024;
    hipLaunchKernelGGL(k_cell_sort, dim3((unsigned)g), dim3(256), 0, s, count, offset, n_keys,
                       perm);
    return hipGetLastError();
}

hipError_t launch_strips(const StripPlan &sp, const PulseRec *pulses, const BlockRec *blocks,
                         const int *n_blocks, int Np, int C, double n_ref, double fs_c, int *skey,
                         int *scount, hipStream_t s) {
    if (sp.NS > kStripMax) return hipErrorInvalidValue;
    hipError_t e = launch_fill_zero((float *)scount, (long long)sp.NB * C * (sp.NS + 1), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_strip_keys, dim3(grid_for(sp.nbm, 256), (unsigned)sp.NB, (unsigned)C),
                       dim3(256), 0, s, sp, pulses, blocks, n_blocks, Np, C, n_ref, fs_c, skey,
                       scount);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_strip_offsets, dim3((unsigned)(sp.NB * C)), dim3(256), 0, s, sp,
                       (const int *)scount);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_strip_lists, dim3((unsigned)(sp.NB * C)), dim3(64),
                       sizeof(int) * (size_t)sp.NS, s, sp, (const int *)skey, n_blocks);
    return hipGetLastError();
}

hipError_t launch_gather(const sim_facets &f, const int *perm, const BlockRec *blocks,
                         const int *n_blocks, long long nb_max, FacetRec *sorted, float zlim,
                         float vlim, unsigned *beyond, hipStream_t s) {
    hipError_t e = launch_fill_zero((float *)beyond, 1, s);
    if (e != hipSuccess || nb_max == 0) return e;
    hipLaunchKernelGGL(k_gather, dim3(grid_for(nb_max, 4)), dim3(256), 0, s, f, perm, blocks,
                       n_blocks, sorted, zlim, vlim * vlim, beyond);
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

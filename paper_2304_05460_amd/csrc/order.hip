// Spatially coherent, deterministic order of a point set.
//
// The points are binned into a grid of at most 2^18 cells over their bounding
// box (B bits per coordinate on the first D' coordinates, B * D' <= 18), the
// cells are visited along a Hilbert curve (consecutive cells are neighbours,
// so runs of consecutive points stay compact), and the points of one cell in
// ascending index.  The Hilbert index comes from Skilling's transpose
// algorithm ("Programming the Hilbert curve", AIP Conf. Proc. 707, 2004).
// Counting sort: cell counts, exclusive scan, an atomic scatter into the cell
// segments, then one wavefront per cell ranks its entries by index, so the
// result does not depend on scheduling.
//
// Uses: the tile kernels of the kernel matvec read the points in this order
// (nearby points share tiles, so tile pairs that are far apart can be
// skipped), and the FSAI rows are computed in it (concurrent rows share
// pattern columns in cache).
#include "afn_internal.h"

namespace afn {
namespace {

constexpr int kCellBits = 18;

void cell_shape(int d, int &bits, int &dims)
{
    bits = kCellBits / d > 0 ? kCellBits / d : 1;
    if (bits > 16) bits = 16;
    dims = kCellBits / bits < d ? kCellBits / bits : d;
}

__global__ __launch_bounds__(256) void bbox_partial(const double *X, int64_t n, int d, int dims, double *part)
{
    __shared__ double lo[256], hi[256];
    for (int t = 0; t < dims; ++t) {
        double a = __builtin_inf(), b = -__builtin_inf();
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
            const double x = X[i * d + t];
            a = x < a ? x : a;
            b = x > b ? x : b;
        }
        lo[threadIdx.x] = a;
        hi[threadIdx.x] = b;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (threadIdx.x < h) {
                lo[threadIdx.x] = lo[threadIdx.x + h] < lo[threadIdx.x] ? lo[threadIdx.x + h] : lo[threadIdx.x];
                hi[threadIdx.x] = hi[threadIdx.x + h] > hi[threadIdx.x] ? hi[threadIdx.x + h] : hi[threadIdx.x];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            part[(blockIdx.x * dims + t) * 2] = lo[0];
            part[(blockIdx.x * dims + t) * 2 + 1] = hi[0];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(64) void bbox_final(const double *part, int nb, int dims, double *box)
{
    const int t = threadIdx.x;
    if (t >= dims) return;
    double a = __builtin_inf(), b = -__builtin_inf();
    for (int g = 0; g < nb; ++g) {
        const double x = part[(g * dims + t) * 2], y = part[(g * dims + t) * 2 + 1];
        a = x < a ? x : a;
        b = y > b ? y : b;
    }
    box[2 * t] = a;
    box[2 * t + 1] = b;
}

// Hilbert index of the cell with coordinates x[0..dims) (each < 2^bits):
// undo the excess work of the curve's reflections and rotations, Gray-encode,
// then interleave the transposed bits (most significant axis first).
__device__ uint32_t hilbert_index(uint32_t *x, int bits, int dims)
{
    const uint32_t M = 1u << (bits - 1);
    for (uint32_t Q = M; Q > 1; Q >>= 1) {
        const uint32_t P = Q - 1;
        for (int i = 0; i < dims; ++i) {
            if (x[i] & Q) {
                x[0] ^= P;
            } else {
                const uint32_t t = (x[0] ^ x[i]) & P;
                x[0] ^= t;
                x[i] ^= t;
            }
        }
    }
    for (int i = 1; i < dims; ++i) x[i] ^= x[i - 1];
    uint32_t t = 0;
    for (uint32_t Q = M; Q > 1; Q >>= 1)
        if (x[dims - 1] & Q) t ^= Q - 1;
    for (int i = 0; i < dims; ++i) x[i] ^= t;
    uint32_t h = 0;
    for (int b = 0; b < bits; ++b)
        for (int i = 0; i < dims; ++i) h |= ((x[i] >> b) & 1u) << (b * dims + (dims - 1 - i));
    return h;
}

__global__ __launch_bounds__(256) void cell_keys(const double *X, int64_t n, int d, int bits, int dims,
                                                 const double *box, int32_t *key, unsigned long long *cnt)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int cells1 = 1 << bits;
    uint32_t x[kCellBits];
    for (int t = 0; t < dims; ++t) {
        const double lo = box[2 * t], span = box[2 * t + 1] - lo;
        int q = span > 0.0 ? (int)((X[i * d + t] - lo) / span * cells1) : 0;
        x[t] = (uint32_t)(q < 0 ? 0 : (q >= cells1 ? cells1 - 1 : q));
    }
    const uint32_t kk = dims == 1 ? x[0] : hilbert_index(x, bits, dims);
    key[i] = (int32_t)kk;
    atomicAdd(&cnt[kk], 1ULL);
}

// Exclusive scan of `count` counters into start[0..count], in three passes:
// the sum of each 1024-counter block, the exclusive scan of the block sums
// (one workgroup), then each block's own scan plus its offset.
__device__ int64_t block_scan_1024(int64_t v, int64_t *part)
{
    // inclusive scan over the 1024 threads of the workgroup (Hillis-Steele)
    part[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    return part[threadIdx.x];
}

__global__ __launch_bounds__(1024) void scan_block_sums(const unsigned long long *cnt, int64_t count,
                                                        int64_t *bsum)
{
    __shared__ int64_t part[1024];
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    const int64_t v = i < count ? (int64_t)cnt[i] : 0;
    const int64_t inc = block_scan_1024(v, part);
    if (threadIdx.x == 1023) bsum[blockIdx.x] = inc;
}

__global__ __launch_bounds__(1024) void scan_block_offsets(int64_t *bsum, int64_t nblk, int64_t count,
                                                           int64_t *start)
{
    __shared__ int64_t part[1024];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nblk; base += 1024) {
        const int64_t b = base + threadIdx.x;
        const int64_t v = b < nblk ? bsum[b] : 0;
        const int64_t inc = block_scan_1024(v, part);
        if (b < nblk) bsum[b] = carry + inc - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += inc;
        __syncthreads();
    }
    if (threadIdx.x == 0) start[count] = carry;
}

__global__ __launch_bounds__(1024) void scan_block_apply(const unsigned long long *cnt, int64_t count,
                                                         const int64_t *boff, int64_t *start)
{
    __shared__ int64_t part[1024];
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    const int64_t v = i < count ? (int64_t)cnt[i] : 0;
    const int64_t inc = block_scan_1024(v, part);
    if (i < count) start[i] = boff[blockIdx.x] + inc - v;
}

__global__ __launch_bounds__(256) void cell_scatter(const int32_t *key, int64_t n, const int64_t *start,
                                                    unsigned long long *cursor, int32_t *tmp)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int32_t kk = key[i];
    const unsigned long long pos = atomicAdd(&cursor[kk], 1ULL);
    tmp[start[kk] + (int64_t)pos] = (int32_t)i;
}

// Within each cell segment, entry e goes to start + #{entries with a smaller
// index} (indices in a cell are distinct); one wavefront per cell.
__global__ __launch_bounds__(256) void cell_rank(const int64_t *__restrict__ start, int64_t cells,
                                                 const int32_t *__restrict__ tmp, int32_t *__restrict__ order)
{
    const int lane = threadIdx.x & 63;
    const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= cells) return;
    const int64_t b = start[c], len = start[c + 1] - b;
    for (int64_t e = lane; e < len; e += 64) {
        const int32_t r = tmp[b + e];
        int64_t rank = 0;
        for (int64_t j = 0; j < len; ++j) rank += tmp[b + j] < r ? 1 : 0;
        order[b + rank] = r;
    }
}

}  // namespace

size_t spatial_order_work_bytes(int64_t n, int d)
{
    int bits, dims;
    cell_shape(d, bits, dims);
    const int64_t cells = (int64_t)1 << (bits * dims);
    const int64_t nn = n > 0 ? n : 1;
    return (size_t)(round_up(8 * 256 * 2 * dims, 256) + round_up(8 * 2 * dims, 256) + round_up(4 * nn, 256) +
                    round_up(8 * cells, 256) + round_up(8 * (cells + 1), 256) + round_up(4 * nn, 256) +
                    round_up(8 * ceil_div(cells, 1024), 256));
}

afn_status spatial_order(const double *X, int64_t n, int d, int32_t *order, void *work, hipStream_t s)
{
    if (n <= 0) return AFN_OK;
    int bits, dims;
    cell_shape(d, bits, dims);
    const int64_t cells = (int64_t)1 << (bits * dims);
    char *q = (char *)work;
    auto take = [&](int64_t bytes) {
        char *r = q;
        q += round_up(bytes, 256);
        return r;
    };
    double *part = (double *)take(8 * 256 * 2 * dims);
    double *box = (double *)take(8 * 2 * dims);
    int32_t *key = (int32_t *)take(4 * n);
    unsigned long long *cnt = (unsigned long long *)take(8 * cells);
    int64_t *start = (int64_t *)take(8 * (cells + 1));
    int32_t *tmp = (int32_t *)take(4 * n);
    const int64_t nblk = ceil_div(cells, 1024);
    int64_t *bsum = (int64_t *)take(8 * nblk);
    const int nb = (int)(ceil_div(n, 256) < 256 ? ceil_div(n, 256) : 256);
    const unsigned g = (unsigned)ceil_div(n, 256);
    hipLaunchKernelGGL(bbox_partial, dim3(nb), dim3(256), 0, s, X, n, d, dims, part);
    hipLaunchKernelGGL(bbox_final, dim3(1), dim3(64), 0, s, part, nb, dims, box);
    AFN_HIP(hipMemsetAsync(cnt, 0, sizeof(unsigned long long) * (size_t)cells, s));
    hipLaunchKernelGGL(cell_keys, dim3(g), dim3(256), 0, s, X, n, d, bits, dims, box, key, cnt);
    hipLaunchKernelGGL(scan_block_sums, dim3((unsigned)nblk), dim3(1024), 0, s, cnt, cells, bsum);
    hipLaunchKernelGGL(scan_block_offsets, dim3(1), dim3(1024), 0, s, bsum, nblk, cells, start);
    hipLaunchKernelGGL(scan_block_apply, dim3((unsigned)nblk), dim3(1024), 0, s, cnt, cells, bsum, start);
    AFN_HIP(hipMemsetAsync(cnt, 0, sizeof(unsigned long long) * (size_t)cells, s));
    hipLaunchKernelGGL(cell_scatter, dim3(g), dim3(256), 0, s, key, n, start, cnt, tmp);
    hipLaunchKernelGGL(cell_rank, dim3((unsigned)ceil_div(cells, 4)), dim3(256), 0, s, start, cells, tmp,
                       order);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

}  // namespace afn

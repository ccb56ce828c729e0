// Exclusive prefix sum of int64 counts (three passes: block sums, scan of the
// block sums, block-local scan plus offset).
#include <algorithm>

#include "nlfem_internal.h"

namespace nlfem {
namespace {

constexpr int kBlock = 256;
constexpr int kItems = 4;                 // per thread
constexpr int kTile = kBlock * kItems;    // per block

__device__ int64_t block_exclusive(int64_t v, int64_t *sh, int64_t *total)
{
    // Hillis-Steele over 256 threads in shared memory
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {
        int64_t add = t >= o ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    int64_t incl = sh[t];
    *total = sh[kBlock - 1];
    __syncthreads();
    return incl - v;
}

// Segments k = 0..nseg-1 of `stride` slots each; the first n slots of a
// segment are scanned.  Block b covers tile b % bps of segment b / bps.

__global__ void __launch_bounds__(kBlock) k_block_sums(const int64_t *in, int64_t n, int64_t stride, int64_t bps,
                                                       int64_t *sums, int64_t *bmax)
{
    __shared__ int64_t sh[kBlock];
    const int64_t seg = blockIdx.x / bps, lb = blockIdx.x % bps;
    const int64_t *x = in + seg * stride;
    const int64_t base = lb * kTile + threadIdx.x * kItems;
    int64_t s = 0, mx = 0;
    for (int i = 0; i < kItems; ++i)
        if (base + i < n) {
            s += x[base + i];
            mx = max(mx, x[base + i]);
        }
    int64_t tot;
    block_exclusive(s, sh, &tot);
    if (threadIdx.x == 0) sums[seg * (bps + 1) + lb] = tot;
    if (bmax) {
        // block maximum (inputs are counts, >= 0)
        for (int o = 32; o > 0; o >>= 1) mx = max(mx, (int64_t)__shfl_xor((long long)mx, o));
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t m = sh[0];
            for (int w = 1; w < kBlock / 64; ++w) m = max(m, sh[w]);
            bmax[seg * (bps + 1) + lb] = m;
        }
    }
}

// one block per segment: exclusive scan of its bps block sums in place,
// total in sums[bps] and, if given, in totals[seg]; the largest input in
// maxes[seg] when bmax is given
__global__ void __launch_bounds__(kBlock) k_scan_sums(int64_t *sums, int64_t bps, int64_t *totals,
                                                      const int64_t *bmax, int64_t *maxes)
{
    __shared__ int64_t sh[kBlock];
    int64_t *x = sums + blockIdx.x * (bps + 1);
    int64_t carry = 0, mx = 0;
    for (int64_t base = 0; base < bps; base += kBlock) {
        const int64_t i = base + threadIdx.x;
        const int64_t v = i < bps ? x[i] : 0;
        if (bmax && i < bps) mx = max(mx, bmax[blockIdx.x * (bps + 1) + i]);
        int64_t tot;
        const int64_t ex = block_exclusive(v, sh, &tot);
        if (i < bps) x[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        x[bps] = carry;
        if (totals) totals[blockIdx.x] = carry;
    }
    if (bmax) {
        __syncthreads();
        for (int o = 32; o > 0; o >>= 1) mx = max(mx, (int64_t)__shfl_xor((long long)mx, o));
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t m = sh[0];
            for (int w = 1; w < kBlock / 64; ++w) m = max(m, sh[w]);
            maxes[blockIdx.x] = m;
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_scan_apply(const int64_t *in, int64_t *out, int64_t n, int64_t stride,
                                                       int64_t bps, const int64_t *sums)
{
    __shared__ int64_t sh[kBlock];
    const int64_t seg = blockIdx.x / bps, lb = blockIdx.x % bps;
    const int64_t *x = in + seg * stride;
    int64_t *y = out + seg * stride;
    const int64_t *sm = sums + seg * (bps + 1);
    const int64_t base = lb * kTile + threadIdx.x * kItems;
    int64_t v[kItems];
    int64_t s = 0;
    for (int i = 0; i < kItems; ++i) {
        v[i] = base + i < n ? x[base + i] : 0;
        s += v[i];
    }
    int64_t tot;
    int64_t ex = block_exclusive(s, sh, &tot) + sm[lb];
    for (int i = 0; i < kItems; ++i) {
        if (base + i < n) y[base + i] = ex;
        ex += v[i];
    }
    if (lb == bps - 1 && threadIdx.x == 0) y[n] = sm[bps];
}

}  // namespace

int64_t scan_tmp_size(int64_t n, int nseg)
{
    return 2 * (int64_t)nseg * (std::max<int64_t>((n + kTile - 1) / kTile, 1) + 1) + 1;
}

int exclusive_scan_segments(const int64_t *in, int64_t *out, int64_t n, int nseg, int64_t stride, int64_t *tmp,
                            int64_t tmp_cap, int64_t *totals, hipStream_t s, int64_t *maxes)
{
    const int64_t bps = std::max<int64_t>((n + kTile - 1) / kTile, 1);
    if (2 * nseg * (bps + 1) > tmp_cap) return set_error(NLFEM_E_OVERFLOW, "scan workspace too small");
    int64_t *bmax = maxes ? tmp + nseg * (bps + 1) : nullptr;
    hipLaunchKernelGGL(k_block_sums, dim3((unsigned)(nseg * bps)), dim3(kBlock), 0, s, in, n, stride, bps, tmp,
                       bmax);
    hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nseg), dim3(kBlock), 0, s, tmp, bps, totals,
                       (const int64_t *)bmax, maxes);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)(nseg * bps)), dim3(kBlock), 0, s, in, out, n, stride, bps,
                       (const int64_t *)tmp);
    NLFEM_HIP(hipGetLastError());
    return NLFEM_OK;
}

int exclusive_scan(const int64_t *in, int64_t *out, int64_t n, int64_t *tmp, int64_t tmp_cap, hipStream_t s,
                   int64_t *total, int64_t *maxval)
{
    return exclusive_scan_segments(in, out, n, 1, n + 1, tmp, tmp_cap, total, s, maxval);
}

}  // namespace nlfem

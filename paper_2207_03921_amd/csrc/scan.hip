// Exclusive prefix sum of int64 counts (three passes: block sums, scan of the
// block sums, block-local scan plus offset).
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

__global__ void __launch_bounds__(kBlock) k_block_sums(const int64_t *in, int64_t n, int64_t *sums)
{
    __shared__ int64_t sh[kBlock];
    int64_t base = (int64_t)blockIdx.x * kTile + threadIdx.x * kItems;
    int64_t s = 0;
    for (int i = 0; i < kItems; ++i)
        if (base + i < n) s += in[base + i];
    int64_t tot;
    block_exclusive(s, sh, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// single block: exclusive scan of nb block sums in place, total in sums[nb]
__global__ void __launch_bounds__(kBlock) k_scan_sums(int64_t *sums, int64_t nb)
{
    __shared__ int64_t sh[kBlock];
    int64_t carry = 0;
    for (int64_t base = 0; base < nb; base += kBlock) {
        int64_t i = base + threadIdx.x;
        int64_t v = i < nb ? sums[i] : 0;
        int64_t tot;
        int64_t ex = block_exclusive(v, sh, &tot);
        if (i < nb) sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) sums[nb] = carry;
}

__global__ void __launch_bounds__(kBlock) k_scan_apply(const int64_t *in, int64_t *out, int64_t n,
                                                       const int64_t *sums, int64_t nb)
{
    __shared__ int64_t sh[kBlock];
    int64_t base = (int64_t)blockIdx.x * kTile + threadIdx.x * kItems;
    int64_t v[kItems];
    int64_t s = 0;
    for (int i = 0; i < kItems; ++i) {
        v[i] = base + i < n ? in[base + i] : 0;
        s += v[i];
    }
    int64_t tot;
    int64_t ex = block_exclusive(s, sh, &tot) + sums[blockIdx.x];
    for (int i = 0; i < kItems; ++i) {
        if (base + i < n) out[base + i] = ex;
        ex += v[i];
    }
    if (blockIdx.x == nb - 1 && threadIdx.x == 0) out[n] = sums[nb];
}

}  // namespace

int64_t scan_tmp_size(int64_t n) { return (n + kTile - 1) / kTile + 1; }

int exclusive_scan(const int64_t *in, int64_t *out, int64_t n, int64_t *tmp, int64_t tmp_cap,
                   hipStream_t s)
{
    if (n <= 0) {
        NLFEM_HIP(hipMemsetAsync(out, 0, sizeof(int64_t), s));
        return NLFEM_OK;
    }
    int64_t nb = (n + kTile - 1) / kTile;
    if (nb + 1 > tmp_cap) return set_error(NLFEM_E_OVERFLOW, "scan workspace too small");
    hipLaunchKernelGGL(k_block_sums, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, tmp);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBlock), 0, s, tmp, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kBlock), 0, s, in, out, n, tmp, nb);
    NLFEM_HIP(hipGetLastError());
    return NLFEM_OK;
}

}  // namespace nlfem

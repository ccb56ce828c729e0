// Exclusive prefix sums of int64 counts in two launches: tile sums, then
// every tile adds the sums of the tiles before it (read directly: the number
// of tiles is small) to its own block-local scan.  One call scans up to
// kScanParts independent arrays.
#include <algorithm>

#include "nlfem_internal.h"

namespace nlfem {
namespace {

constexpr int kBlock = 256;
constexpr int kItems = 4;                 // per thread
constexpr int kTile = kBlock * kItems;    // per block

struct ScanList {
    ScanPart p[kScanParts];
    int64_t first[kScanParts + 1];        // first tile of each part
    int32_t cnt;
    int64_t *sums, *bmax;                 // [tiles]
    SpecGate gate;
};

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

// sum (MAX = false) or maximum over the block, returned to every thread
template <bool MAX>
__device__ int64_t block_reduce(int64_t v, int64_t *sh)
{
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t y = __shfl_xor((long long)v, o);
        v = MAX ? max(v, y) : v + y;
    }
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    int64_t r = sh[0];
    for (int w = 1; w < kBlock / 64; ++w) r = MAX ? max(r, sh[w]) : r + sh[w];
    __syncthreads();
    return r;
}

__device__ inline int part_of(const ScanList &L, int64_t b)
{
    int k = 0;
    while (k + 1 < L.cnt && L.first[k + 1] <= b) ++k;
    return k;
}

__global__ void __launch_bounds__(kBlock) k_scan_tiles(ScanList L)
{
    __shared__ int64_t sh[kBlock / 64];
    if (gated(L.gate)) return;
    const int64_t b = blockIdx.x;
    const ScanPart &P = L.p[part_of(L, b)];
    const int64_t lb = b - L.first[part_of(L, b)];
    const int64_t base = lb * kTile + threadIdx.x * kItems;
    int64_t s = 0, mx = 0;
    for (int i = 0; i < kItems; ++i)
        if (base + i < P.n) {
            const int64_t x = P.in[base + i];
            s += x;
            mx = max(mx, x);
        }
    s = block_reduce<false>(s, sh);
    if (threadIdx.x == 0) L.sums[b] = s;
    if (P.maxv) {   // inputs are counts (>= 0)
        mx = block_reduce<true>(mx, sh);
        if (threadIdx.x == 0) L.bmax[b] = mx;
    }
}

__global__ void __launch_bounds__(kBlock) k_scan_apply(ScanList L)
{
    __shared__ int64_t sh[kBlock];
    if (gated(L.gate)) return;
    const int64_t b = blockIdx.x;
    const int k = part_of(L, b);
    const ScanPart &P = L.p[k];
    const int64_t t0 = L.first[k], lb = b - t0, last = L.first[k + 1] - 1;
    // offset of this tile: the sums of the part's tiles before it
    int64_t part = 0;
    for (int64_t i = t0 + threadIdx.x; i < b; i += kBlock) part += L.sums[i];
    const int64_t off = block_reduce<false>(part, sh);
    const int64_t base = lb * kTile + threadIdx.x * kItems;
    int64_t v[kItems];
    int64_t s = 0;
    for (int i = 0; i < kItems; ++i) {
        v[i] = base + i < P.n ? P.in[base + i] : 0;
        s += v[i];
    }
    int64_t tot;
    int64_t ex = block_exclusive(s, sh, &tot) + off;
    for (int i = 0; i < kItems; ++i) {
        if (base + i < P.n) P.out[base + i] = ex;
        ex += v[i];
    }
    if (b == last) {
        // last tile of the part: total and largest input
        if (threadIdx.x == 0) {
            P.out[P.n] = off + tot;
            if (P.total) *P.total = off + tot;
        }
        if (P.maxv) {
            int64_t mx = 0;
            for (int64_t i = t0 + threadIdx.x; i <= last; i += kBlock) mx = max(mx, L.bmax[i]);
            mx = block_reduce<true>(mx, sh);
            if (threadIdx.x == 0) *P.maxv = mx;
        }
    }
}

int64_t tiles_of(int64_t n) { return std::max<int64_t>((n + kTile - 1) / kTile, 1); }

}  // namespace

int64_t scan_tmp_size(int64_t n, int nseg)
{
    return 2 * (int64_t)nseg * tiles_of(n) + 1;
}

int exclusive_scan_multi(const ScanPart *parts, int cnt, int64_t *tmp, int64_t tmp_cap, hipStream_t s,
                         const SpecGate &gate)
{
    if (cnt < 1 || cnt > kScanParts) return set_error(NLFEM_E_INVALID, "scan: 1..8 arrays per call");
    ScanList L{};
    L.cnt = cnt;
    int64_t tiles = 0;
    for (int k = 0; k < cnt; ++k) {
        L.p[k] = parts[k];
        L.first[k] = tiles;
        tiles += tiles_of(parts[k].n);
    }
    L.first[cnt] = tiles;
    if (2 * tiles > tmp_cap) return set_error(NLFEM_E_OVERFLOW, "scan workspace too small");
    L.sums = tmp;
    L.bmax = tmp + tiles;
    L.gate = gate;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(kBlock), 0, s, L);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)tiles), dim3(kBlock), 0, s, L);
    NLFEM_HIP(hipGetLastError());
    return NLFEM_OK;
}

int exclusive_scan_segments(const int64_t *in, int64_t *out, int64_t n, int nseg, int64_t stride, int64_t *tmp,
                            int64_t tmp_cap, int64_t *totals, hipStream_t s, int64_t *maxes,
                            const SpecGate &gate)
{
    ScanPart parts[kScanParts];
    if (nseg < 1 || nseg > kScanParts) return set_error(NLFEM_E_INVALID, "scan: 1..8 segments per call");
    for (int k = 0; k < nseg; ++k)
        parts[k] = ScanPart{in + k * stride, out + k * stride, n, totals ? totals + k : nullptr,
                            maxes ? maxes + k : nullptr};
    return exclusive_scan_multi(parts, nseg, tmp, tmp_cap, s, gate);
}

int exclusive_scan(const int64_t *in, int64_t *out, int64_t n, int64_t *tmp, int64_t tmp_cap, hipStream_t s,
                   int64_t *total, int64_t *maxval, const SpecGate &gate)
{
    const ScanPart p{in, out, n, total, maxval};
    return exclusive_scan_multi(&p, 1, tmp, tmp_cap, s, gate);
}

}  // namespace nlfem

// Exclusive prefix sums of int64 counts in one launch (chained scan).  Every
// workgroup takes a ticket, scans its tile of 1024 counts, publishes the
// tile's sum, then adds the published words of the tiles before it: their
// sums back to the nearest tile that has already published its inclusive
// prefix.  Maxima go to their slots by atomic maximum.  Tickets are taken in the order workgroups start, so every tile a
// workgroup waits for belongs to a workgroup that is running and waits only
// for earlier tickets itself.  The wait is bounded: past the limit the
// workgroup sums the inputs before its tile directly, which needs no other
// workgroup.  One call scans up to kScanParts independent arrays.
#include <algorithm>
#include <cstdlib>

#include "nlfem_internal.h"

namespace nlfem {
namespace {

constexpr int kBlock = 256;
constexpr int kItems = 4;                 // per thread
constexpr int kTile = kBlock * kItems;    // per block
constexpr int kSpinDefault = 1 << 14;     // polls of the look-back before the direct sum

// a tile's published word: status in the top two bits, a sum below
enum : unsigned { kNone = 0, kAgg = 1, kInc = 2 };   // nothing, the tile's sum, its inclusive prefix
constexpr unsigned long long kSumMask = (1ull << 62) - 1;

struct ScanList {
    ScanPart p[kScanParts];
    int64_t first[kScanParts + 1];        // first tile of each part
    int32_t cnt;
    int32_t spin;                         // poll limit; < 0: always the direct sum
    unsigned long long *ticket;           // [1], zero at launch
    unsigned long long *word;             // [tiles], zero at launch
    SpecGate gate;
};

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

// Words are read and written by workgroups on other dies: device-scope
// atomics.  Each word carries its own value, so no ordering with other
// memory is needed.
__device__ inline unsigned long long load_word(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void store_word(unsigned long long *p, unsigned status, int64_t sum)
{
    __hip_atomic_store(p, ((unsigned long long)status << 62) | (unsigned long long)sum, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// Sum of the tiles t0 .. b-1 from their words, by one wave; false when the
// wait ran past the limit.
__device__ bool look_back(const ScanList &L, int64_t t0, int64_t b, int64_t *sum)
{
    if (L.spin < 0) return false;
    const int lane = threadIdx.x & 63;
    int64_t s = 0;
    int64_t j = b - 1;   // nearest tile not yet added
    int polls = 0;
    while (true) {
        const int64_t t = j - lane;
        const unsigned long long w = t >= t0 ? load_word(&L.word[t]) : 0ull;
        const unsigned st = (unsigned)(w >> 62);
        if (!__all(t < t0 || st != kNone)) {
            if (++polls > L.spin) return false;
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        // the first tile of a part publishes its inclusive prefix at once, so
        // a window that reaches it always holds one
        const unsigned long long incl = __ballot(t >= t0 && st == kInc);
        const int stop = incl ? __ffsll((long long)incl) - 1 : 64;
        if (lane <= stop && t >= t0) s += (int64_t)(w & kSumMask);
        if (incl) break;
        j -= 64;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor((long long)s, o);
    *sum = s;
    return true;
}

__global__ void __launch_bounds__(kBlock) k_scan(ScanList L)
{
    __shared__ int64_t wsum[kBlock / 64], wmax[kBlock / 64];
    __shared__ int64_t s_b, s_pre;
    __shared__ int s_ok;
    if (gated(L.gate)) return;
    if (threadIdx.x == 0) s_b = (int64_t)atomicAdd(L.ticket, 1ull);
    __syncthreads();
    const int64_t b = s_b;
    if (b >= L.first[L.cnt]) return;   // a ticket counter not cleared: leave everything untouched
    const int k = part_of(L, b);
    const ScanPart &P = L.p[k];
    const int64_t t0 = L.first[k], lb = b - t0, last = L.first[k + 1] - 1;
    const int64_t base = lb * kTile + threadIdx.x * kItems;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int64_t v[kItems];
    int64_t s = 0, mx = 0;
    for (int i = 0; i < kItems; ++i) {
        v[i] = base + i < P.n ? P.in[base + i] : 0;   // counts: >= 0
        s += v[i];
        mx = max(mx, v[i]);
    }
    // tile scan: waves by shuffles, then the wave totals
    int64_t incl = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up((long long)incl, o);
        if (lane >= o) incl += y;
    }
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, (int64_t)__shfl_xor((long long)mx, o));
    if (lane == 63) wsum[wv] = incl;
    if (lane == 0) wmax[wv] = mx;
    __syncthreads();
    int64_t before = 0, tot = 0, tmax = 0;
    for (int i = 0; i < kBlock / 64; ++i) {
        before += i < wv ? wsum[i] : 0;
        tot += wsum[i];
        tmax = max(tmax, wmax[i]);
    }
    if (threadIdx.x < 64) {
        int64_t pre = 0;
        bool ok = true;
        if (lb == 0) {
            if (threadIdx.x == 0) store_word(&L.word[b], kInc, tot);
        } else {
            if (threadIdx.x == 0) store_word(&L.word[b], kAgg, tot);
            ok = look_back(L, t0, b, &pre);
        }
        if (threadIdx.x == 0) {
            s_pre = pre;
            s_ok = ok;
        }
    }
    __syncthreads();
    if (!s_ok) {
        // the direct sum of the inputs before this tile
        int64_t ds = 0;
        for (int64_t i = threadIdx.x; i < lb * kTile; i += kBlock) ds += P.in[i];
        ds = block_reduce<false>(ds, wsum);
        if (threadIdx.x == 0) s_pre = ds;
        __syncthreads();
    }
    const int64_t pre = s_pre;
    if (threadIdx.x == 0) {
        if (lb > 0) store_word(&L.word[b], kInc, pre + tot);
        // the part's largest input (the slot starts at zero)
        if (P.maxv && tmax > 0) atomicMax((unsigned long long *)P.maxv, (unsigned long long)tmax);
    }
    int64_t ex = pre + before + incl - s;
    for (int i = 0; i < kItems; ++i) {
        if (base + i < P.n) P.out[base + i] = ex;
        ex += v[i];
    }
    if (b == last && threadIdx.x == 0) {
        // last tile of the part: the total
        P.out[P.n] = pre + tot;
        if (P.total) *P.total = pre + tot;
    }
}

int64_t tiles_of(int64_t n) { return std::max<int64_t>((n + kTile - 1) / kTile, 1); }

// poll limit of the look-back; NLFEM_SCAN_SPIN=-1 makes every tile take the
// direct sum (a test of that path)
int spin_limit()
{
    const char *e = std::getenv("NLFEM_SCAN_SPIN");
    return e ? std::atoi(e) : kSpinDefault;
}

}  // namespace

int64_t scan_tiles(int64_t n, int nseg) { return (int64_t)nseg * tiles_of(n); }

int exclusive_scan_multi(const ScanPart *parts, int cnt, const ScanWork &w, hipStream_t s, const SpecGate &gate)
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
    if (tiles > w.tiles) return set_error(NLFEM_E_OVERFLOW, "scan workspace too small");
    L.spin = spin_limit();
    L.ticket = (unsigned long long *)w.hdr;
    L.word = (unsigned long long *)w.hdr + 1;
    L.gate = gate;
    hipLaunchKernelGGL(k_scan, dim3((unsigned)tiles), dim3(kBlock), 0, s, L);
    NLFEM_HIP(hipGetLastError());
    return NLFEM_OK;
}

int exclusive_scan_segments(const int64_t *in, int64_t *out, int64_t n, int nseg, int64_t stride,
                            const ScanWork &w, int64_t *totals, hipStream_t s, int64_t *maxes,
                            const SpecGate &gate)
{
    ScanPart parts[kScanParts];
    if (nseg < 1 || nseg > kScanParts) return set_error(NLFEM_E_INVALID, "scan: 1..8 segments per call");
    for (int k = 0; k < nseg; ++k)
        parts[k] = ScanPart{in + k * stride, out + k * stride, n, totals ? totals + k : nullptr,
                            maxes ? maxes + k : nullptr};
    return exclusive_scan_multi(parts, nseg, w, s, gate);
}

int exclusive_scan(const int64_t *in, int64_t *out, int64_t n, const ScanWork &w, hipStream_t s, int64_t *total,
                   int64_t *maxval, const SpecGate &gate)
{
    const ScanPart p{in, out, n, total, maxval};
    return exclusive_scan_multi(&p, 1, w, s, gate);
}

}  // namespace nlfem

// Batched assembly of many independent problems (meshes of uneven size and
// kernel) in a few persistent launches over a global work queue.
//
// The items of one phase (non-touching pairs, touching pairs of one class,
// element diagonals, matrix rows) of all problems that share a kernel
// specialisation form one queue: problem p owns the global items
// [pre[p], pre[p+1]).  Workgroups of a persistent grid take `chunk`
// consecutive items at a time from an atomic counter, find the problem by
// binary search in the prefix table (in LDS) and run the same per-item
// function as the single-problem kernels, so the results are bit-identical
// to assembling the problems one by one.  Every workgroup leaves once the
// counter has passed the end of the queue.
//
// A batch is fixed at creation (problems, configurations, output arrays), so
// its launches can be captured once into a HIP graph and replayed.  Counters
// are cleared by a small kernel (no memset node in the graph).  The chunk
// sizes and workgroups per CU of each phase are chosen by timing a few
// candidates on the device and can be cached in a text file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "assemble_items.h"
#include "batch.h"

using namespace nlfem;
using namespace nlfem::items;

namespace {

struct QueueArgs {
    int32_t nprob;
    const int64_t *pre;               // [nprob + 1]
    unsigned long long *counter;
    int32_t chunk;
};

// The lanes of a wave hold consecutive items, so the items of one problem
// sit in a run of consecutive lanes.  A wave takes its problems one run at a
// time: `next_run` returns the problem of the first pending lane as a
// wave-uniform value (the per-problem tables are then read with scalar
// loads), its first lane and its lane mask, and removes the run from `todo`.
struct Run {
    int p, lane0;
    unsigned long long mask;
};

__device__ inline Run next_run(int p, unsigned long long *todo)
{
    Run r;
    r.lane0 = (int)__builtin_ctzll(*todo);
    r.p = __builtin_amdgcn_readlane(p, r.lane0);
    r.mask = __ballot(p == r.p);
    *todo &= ~r.mask;
    return r;
}

__device__ inline int find_prob(const int64_t *pre, int n, int64_t it)
{
    int lo = 0, hi = n;   // pre[lo] <= it < pre[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= it) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Loads the prefix table into LDS; returns the number of items.
__device__ inline int64_t load_prefix(const QueueArgs &q, int64_t *pre)
{
    for (int t = threadIdx.x; t <= q.nprob; t += blockDim.x) pre[t] = q.pre[t];
    __syncthreads();
    return pre[q.nprob];
}

// Next chunk of the queue for the whole workgroup.
__device__ inline int64_t grab(const QueueArgs &q, unsigned long long *slot)
{
    if (threadIdx.x == 0) *slot = atomicAdd(q.counter, (unsigned long long)q.chunk);
    __syncthreads();
    const int64_t b0 = (int64_t)*slot;
    __syncthreads();
    return b0;
}

template <int KER, typename T>
constexpr bool batch_far_staged() { return !(Ker<KER>::NK == 3 && sizeof(T) == 8); }

// records staged through LDS as in the single-problem kernel where it fits
template <int KER, typename T, int PM, bool POLY>
__global__ void __launch_bounds__(256) kb_far(QueueArgs q, const FarArgs *__restrict__ fa, const RoleArgs *__restrict__ r1,
                                                const RoleArgs *__restrict__ r2)
{
    constexpr bool STAGED = batch_far_staged<KER, T>() && !POLY;
    constexpr int NV = kFarStage<Ker<KER>::NK>;
    extern __shared__ __align__(16) unsigned char dyn[];
    __shared__ unsigned long long slot;
    __shared__ T slots[STAGED ? 4 * 64 * NV : 1];
    __shared__ double sdir[POLY ? 4 : 1][POLY ? 2 * kMaxPoly : 1];   // the wave's problem's polygon
    int64_t *pre = (int64_t *)dyn;
    const int64_t total = load_prefix(q, pre);
    const int lane = threadIdx.x & 63;
    int staged = -1;   // problem whose polygon the wave's sdir holds
    for (;;) {
        const int64_t b0 = grab(q, &slot);
        if (b0 >= total) break;
        const int64_t b1 = min(b0 + (int64_t)q.chunk, total);
        for (int64_t it0 = b0; it0 < b1; it0 += blockDim.x) {
            const int64_t it = it0 + threadIdx.x;
            const bool act = it < b1;
            const int p = act ? find_prob(pre, q.nprob, it) : -1;
            unsigned long long todo = __ballot(act);
            while (todo) {
                const Run r = next_run(p, &todo);
                const bool mine = p == r.p;
                const int64_t base = pre[r.p];
                if (STAGED) {
                    const FarArgs &a = fa[r.p];
                    FarAcc<KER, T> acc;
                    bool self = false;
                    if (mine) {
                        const int64_t idx = it - base;
                        const int32_t e = a.ue[idx], f = a.uf[idx];
                        self = e == f;
                        const uint2 mm = a.m[idx];
                        far_whole<KER, T, PM>(a, r1[r.p], r2[r.p], e, f, mm.x, mm.y, acc);
                    }
                    far_store_wave<KER, T>(a, it - lane + r.lane0 - base, __popcll(r.mask), self, acc,
                                           slots + (threadIdx.x >> 6) * 64 * NV, r.lane0);
                } else if (POLY) {
                    double *sd = sdir[POLY ? threadIdx.x >> 6 : 0];
                    if (r.p != staged) {
                        wave_sync();
                        for (int t = lane; t < 2 * fa[r.p].N; t += 64) sd[t] = fa[r.p].dir[t];
                        wave_sync();
                        staged = r.p;
                    }
                    if (mine) {
                        FarArgs al = fa[r.p];
                        al.dir = sd;
                        far_item<KER, T, PM, POLY>(al, r1[r.p], r2[r.p], it - base);
                    }
                } else if (mine) {
                    far_item<KER, T, PM, POLY>(fa[r.p], r1[r.p], r2[r.p], it - base);
                }
            }
        }
    }
}

template <int KER, int CLS, int G>
__global__ void __launch_bounds__(256) kb_touch(QueueArgs q, const TouchArgs *__restrict__ ta, const GaussArgs *__restrict__ ga)
{
    extern __shared__ __align__(16) unsigned char dyn[];
    __shared__ unsigned long long slot;
    __shared__ double gst[4][2 * kMaxGauss];   // the rule of the wave's problem
    int64_t *pre = (int64_t *)dyn;
    const int64_t total = load_prefix(q, pre);
    const int group = threadIdx.x / G, sub = threadIdx.x % G, groups = blockDim.x / G;
    const int lane = threadIdx.x & 63;
    double *gw = gst[threadIdx.x >> 6];
    int staged = -1;   // problem whose rule gw holds (uniform in the wave)
    for (;;) {
        const int64_t b0 = grab(q, &slot);
        if (b0 >= total) break;
        const int64_t b1 = min(b0 + (int64_t)q.chunk, total);
        for (int64_t it0 = b0; it0 < b1; it0 += groups) {
            const int64_t it = it0 + group;   // uniform within a lane group
            const bool act = it < b1;
            const int p = act ? find_prob(pre, q.nprob, it) : -1;
            unsigned long long todo = __ballot(act);
            while (todo) {
                const Run r = next_run(p, &todo);   // whole lane groups
                if (r.p != staged) {
                    wave_sync();
                    gw[lane] = lane < kMaxGauss ? ga[r.p].x[lane] : ga[r.p].w[lane - kMaxGauss];
                    wave_sync();
                    staged = r.p;
                }
                if (p == r.p)
                    touch_item<KER, CLS, G>(ta[r.p], GaussView{gw, gw + kMaxGauss, ga[r.p].n}, it - pre[r.p], sub);
            }
        }
    }
}

template <int NK, typename TR, bool MOM = false>
__global__ void __launch_bounds__(256) kb_diag(QueueArgs q, const DiagArgs *__restrict__ da)
{
    extern __shared__ __align__(16) unsigned char dyn[];
    __shared__ unsigned long long slot;
    int64_t *pre = (int64_t *)dyn;
    const int64_t total = load_prefix(q, pre);
    constexpr int G = diag_group<MOM>();
    const int group = threadIdx.x / G, sub = threadIdx.x % G, groups = blockDim.x / G;
    for (;;) {
        const int64_t b0 = grab(q, &slot);
        if (b0 >= total) break;
        const int64_t b1 = min(b0 + (int64_t)q.chunk, total);
        for (int64_t it0 = b0; it0 < b1; it0 += groups) {
            const int64_t it = it0 + group;   // one element per lane group
            const int p = it < b1 ? find_prob(pre, q.nprob, it) : -1;
            unsigned long long todo = __ballot(it < b1);
            while (todo) {
                const Run r = next_run(p, &todo);   // whole lane groups
                if (p == r.p) diag_item<NK, TR, MOM>(da[r.p], it - pre[r.p], sub);
            }
        }
    }
}

// Rows cost about the same each, so they are spread statically, one per
// workgroup of one wave, with the XCD-aware order of the single-problem
// kernel over the rows of all problems of the group (no queue).
template <int NC, typename TR, bool MOM = false>
__global__ void __launch_bounds__(64) kb_rows(QueueArgs q, const RowArgs *__restrict__ ra, size_t pre_bytes)
{
    extern __shared__ __align__(16) unsigned char dyn[];
    __shared__ RowShared sh;
    __shared__ double mq[MOM ? kRowMom : 1];
    int64_t *pre = (int64_t *)dyn;
    unsigned char *rowmem = dyn + pre_bytes;
    const int64_t total = load_prefix(q, pre);
    for (int64_t b = blockIdx.x; b < xcd_span(total); b += gridDim.x) {
        const int64_t it = xcd_item(b, total);
        if (it >= total) continue;
        // one row per workgroup of one wave: the problem is uniform
        const int p = __builtin_amdgcn_readfirstlane(find_prob(pre, q.nprob, it));
        const RowArgs &a = ra[p];
        row_item<NC, TR, MOM>(a, a.rows[it - pre[p]], rowmem, sh, mq);
    }
}

__global__ void k_zero_u64(unsigned long long *c, int n)
{
    for (int t = threadIdx.x; t < n; t += blockDim.x) c[t] = 0ull;
}

// ------------------------------------------------------------ host side

enum Phase { kFar = 0, kTouch, kDiag, kRows, kPhases };

struct Shape {
    int chunk, per_cu;   // items per grab, workgroups per CU
};

struct Group {
    Phase phase;
    int kernel = 0, cls = 0, nc = 1;
    bool fp32 = false, poly = false, seven = false;
    bool mom = false;           // kDiag, kRows: moment form (no far records)
    std::vector<int> probs;
    std::vector<int64_t> pre;   // host copy
    size_t off_pre = 0, off_args = 0, off_r1 = 0, off_r2 = 0;
    size_t row_lds = 0;         // kRows: largest row buffer of the group
    int counter = 0;
};

}  // namespace

struct nlfem_batch {
    int n = 0;
    int cus = 0;
    std::vector<AssemblePlan> plans;
    std::vector<Group> groups;
    void *dev = nullptr;              // all tables and counters (in mem)
    DevBlock mem;
    size_t dev_bytes = 0;
    unsigned long long *counters = nullptr;
    Shape shape[kPhases] = {{1024, 4}, {256, 4}, {64, 4}, {4, 16}};
    hipStream_t capture = nullptr;
    // per-problem phases: launches spread round-robin over the caller's
    // stream and these (forked and joined by events, also under capture)
    hipStream_t side[3] = {nullptr, nullptr, nullptr};
    hipEvent_t fork = nullptr, join[3] = {nullptr, nullptr, nullptr};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<nlfem_pairs *> handles;
    std::vector<uint64_t> generation;   // of each handle at creation
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

template <class T>
const T *dptr(const nlfem_batch *b, size_t off)
{
    return (const T *)((const char *)b->dev + off);
}

// ---- launching one group

template <int KER, typename T, bool POLY>
void far_group(const nlfem_batch *b, const Group &g, const QueueArgs &q, const Shape &sh, hipStream_t s)
{
    const size_t lds = sizeof(int64_t) * (g.probs.size() + 1);
    const dim3 grid((unsigned)(b->cus * sh.per_cu)), block(256);
    const FarArgs *fa = dptr<FarArgs>(b, g.off_args);
    const RoleArgs *r1 = dptr<RoleArgs>(b, g.off_r1), *r2 = dptr<RoleArgs>(b, g.off_r2);
    if (g.seven) hipLaunchKernelGGL((kb_far<KER, T, 7, POLY>), grid, block, lds, s, q, fa, r1, r2);
    else hipLaunchKernelGGL((kb_far<KER, T, 0, POLY>), grid, block, lds, s, q, fa, r1, r2);
}

template <int KER>
void far_group_k(const nlfem_batch *b, const Group &g, const QueueArgs &q, const Shape &sh, hipStream_t s)
{
    if (g.poly) {
        if (g.fp32) far_group<KER, float, true>(b, g, q, sh, s);
        else far_group<KER, double, true>(b, g, q, sh, s);
    } else {
        if (g.fp32) far_group<KER, float, false>(b, g, q, sh, s);
        else far_group<KER, double, false>(b, g, q, sh, s);
    }
}

template <int KER>
void touch_group(const nlfem_batch *b, const Group &g, const QueueArgs &q, const Shape &sh, hipStream_t s)
{
    const size_t lds = sizeof(int64_t) * (g.probs.size() + 1);
    const dim3 grid((unsigned)(b->cus * sh.per_cu)), block(256);
    const TouchArgs *ta = dptr<TouchArgs>(b, g.off_args);
    const GaussArgs *ga = dptr<GaussArgs>(b, g.off_r1);
    if (g.cls == 3) hipLaunchKernelGGL((kb_touch<KER, 3, touch_lanes(3)>), grid, block, lds, s, q, ta, ga);
    else if (g.cls == 2) hipLaunchKernelGGL((kb_touch<KER, 2, touch_lanes(2)>), grid, block, lds, s, q, ta, ga);
    else hipLaunchKernelGGL((kb_touch<KER, 1, touch_lanes(1)>), grid, block, lds, s, q, ta, ga);
}

void launch_group(const nlfem_batch *b, const Group &g, const Shape &sh, hipStream_t s)
{
    QueueArgs q{(int32_t)g.probs.size(), dptr<int64_t>(b, g.off_pre), b->counters + g.counter, sh.chunk};
    const size_t pre_lds = align256(sizeof(int64_t) * (g.probs.size() + 1));
    switch (g.phase) {
    case kFar:
        if (g.kernel == NLFEM_K_CONSTANT) far_group_k<NLFEM_K_CONSTANT>(b, g, q, sh, s);
        else if (g.kernel == NLFEM_K_INV_DIST) far_group_k<NLFEM_K_INV_DIST>(b, g, q, sh, s);
        else if (g.kernel == NLFEM_K_FRAC_HALF) far_group_k<NLFEM_K_FRAC_HALF>(b, g, q, sh, s);
        else far_group_k<NLFEM_K_PERIDYNAMIC>(b, g, q, sh, s);
        break;
    case kTouch:
        if (g.kernel == NLFEM_K_CONSTANT) touch_group<NLFEM_K_CONSTANT>(b, g, q, sh, s);
        else if (g.kernel == NLFEM_K_INV_DIST) touch_group<NLFEM_K_INV_DIST>(b, g, q, sh, s);
        else if (g.kernel == NLFEM_K_FRAC_HALF) touch_group<NLFEM_K_FRAC_HALF>(b, g, q, sh, s);
        else touch_group<NLFEM_K_PERIDYNAMIC>(b, g, q, sh, s);
        break;
    case kDiag: {
        const dim3 grid((unsigned)(b->cus * sh.per_cu)), block(256);
        const DiagArgs *da = dptr<DiagArgs>(b, g.off_args);
        if (g.nc == 1 && g.mom) {
            if (g.fp32) hipLaunchKernelGGL((kb_diag<1, float, true>), grid, block, pre_lds, s, q, da);
            else hipLaunchKernelGGL((kb_diag<1, double, true>), grid, block, pre_lds, s, q, da);
        } else if (g.nc == 1) {
            if (g.fp32) hipLaunchKernelGGL((kb_diag<1, float>), grid, block, pre_lds, s, q, da);
            else hipLaunchKernelGGL((kb_diag<1, double>), grid, block, pre_lds, s, q, da);
        } else {
            if (g.fp32) hipLaunchKernelGGL((kb_diag<3, float>), grid, block, pre_lds, s, q, da);
            else hipLaunchKernelGGL((kb_diag<3, double>), grid, block, pre_lds, s, q, da);
        }
        break;
    }
    default: {
        const dim3 grid(xcd_grid(g.pre.back())), block(64);
        const RowArgs *ra = dptr<RowArgs>(b, g.off_args);
        const size_t lds = pre_lds + g.row_lds;
        if (g.nc == 1 && g.mom) {
            if (g.fp32) hipLaunchKernelGGL((kb_rows<1, float, true>), grid, block, lds, s, q, ra, pre_lds);
            else hipLaunchKernelGGL((kb_rows<1, double, true>), grid, block, lds, s, q, ra, pre_lds);
        } else if (g.nc == 1) {
            if (g.fp32) hipLaunchKernelGGL((kb_rows<1, float>), grid, block, lds, s, q, ra, pre_lds);
            else hipLaunchKernelGGL((kb_rows<1, double>), grid, block, lds, s, q, ra, pre_lds);
        } else {
            if (g.fp32) hipLaunchKernelGGL((kb_rows<2, float>), grid, block, lds, s, q, ra, pre_lds);
            else hipLaunchKernelGGL((kb_rows<2, double>), grid, block, lds, s, q, ra, pre_lds);
        }
    }
    }
}

// Shape {0, 0}: the phase as the single-problem launches of each problem
// in turn (the same per-item functions, so the same values); the tuner
// takes it where it is faster than the shared queue.
int run_phase(const nlfem_batch *b, Phase ph, const Shape &sh, hipStream_t s)
{
    if (sh.chunk == 0) {
        constexpr int NS = 4;   // the caller's stream and the three side streams
        const bool fan = b->side[0] != nullptr;
        if (fan) {
            NLFEM_HIP(hipEventRecord(b->fork, s));
            for (int k = 0; k < NS - 1; ++k) NLFEM_HIP(hipStreamWaitEvent(b->side[k], b->fork, 0));
        }
        for (size_t i = 0; i < b->plans.size(); ++i) {
            const int k = fan ? (int)(i % NS) : 0;
            launch_phase(b->plans[i], (int)ph, k == 0 ? s : b->side[k - 1]);
        }
        if (fan)
            for (int k = 0; k < NS - 1; ++k) {
                NLFEM_HIP(hipEventRecord(b->join[k], b->side[k]));
                NLFEM_HIP(hipStreamWaitEvent(s, b->join[k], 0));
            }
        NLFEM_HIP(hipGetLastError());
        return NLFEM_OK;
    }
    for (const Group &g : b->groups)
        if (g.phase == ph) launch_group(b, g, sh, s);
    NLFEM_HIP(hipGetLastError());
    return NLFEM_OK;
}

// touching pairs, far pairs, element diagonals, rows, in that order on s.
// `timed`: HIP events of the per-phase timing around each phase (not while
// capturing)
int run_all(const nlfem_batch *b, hipStream_t s, bool timed)
{
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(256), 0, s, b->counters, (int)b->groups.size());
    // touching records, then the far records, on one stream: run side by
    // side the far launch (2 waves per SIMD by registers) left the touching
    // waves no room and both took longer than one after the other
    if (timed) timing_begin(kPhTouch, s);
    NLFEM_TRY(run_phase(b, kTouch, b->shape[kTouch], s));
    if (timed) timing_end(kPhTouch, s);
    if (timed) timing_begin(kPhFar, s);
    NLFEM_TRY(run_phase(b, kFar, b->shape[kFar], s));
    if (timed) timing_end(kPhFar, s);
    if (timed) timing_begin(kPhDiag, s);
    NLFEM_TRY(run_phase(b, kDiag, b->shape[kDiag], s));
    if (timed) timing_end(kPhDiag, s);
    if (timed) timing_begin(kPhRows, s);
    NLFEM_TRY(run_phase(b, kRows, b->shape[kRows], s));
    if (timed) timing_end(kPhRows, s);
    return NLFEM_OK;
}

// ---- grouping and device tables

int64_t items_of(const AssemblePlan &p, Phase ph, int cls)
{
    switch (ph) {
    case kFar: return p.mom ? 0 : p.far.n;
    case kTouch: return p.touch[cls == 3 ? 0 : cls == 2 ? 1 : 2].n;
    case kDiag: return p.rows.nrows > 0 ? p.diag.K : 0;
    default: return p.rows.nrows;
    }
}

void make_groups(nlfem_batch *b)
{
    std::map<std::string, int> index;
    for (int i = 0; i < b->n; ++i) {
        const AssemblePlan &p = b->plans[i];
        for (int ph = 0; ph < kPhases; ++ph) {
            const int ncls = ph == kTouch ? 3 : 1;
            for (int c = 0; c < ncls; ++c) {
                const int cls = ph == kTouch ? 3 - c : 0;
                if (items_of(p, (Phase)ph, cls) == 0) continue;
                Group g;
                g.phase = (Phase)ph;
                g.fp32 = p.fp32;
                g.nc = p.nc;
                if (ph == kFar) {
                    g.kernel = p.kernel;
                    g.poly = p.poly;
                    g.seven = p.seven;
                } else if (ph == kTouch) {
                    g.kernel = p.kernel;
                    g.cls = cls;
                } else if (ph == kRows) {
                    // rows grouped by their LDS need in steps of 1.2x: each
                    // launch reserves its own problems' size (the largest of a
                    // single group would cap the resident waves of the others)
                    const size_t need = row_lds_bytes(p.rows.maxlen, p.nc, p.rows.hcap);
                    int c2 = 0;
                    for (double lim = 1024.0; lim < (double)need; lim *= 1.2) ++c2;
                    g.cls = c2;
                    g.mom = p.mom;
                } else if (ph == kDiag) {
                    g.mom = p.mom;
                }
                char key[96];
                std::snprintf(key, sizeof key, "%d/%d/%d/%d/%d/%d/%d/%d", ph, g.kernel, g.cls, g.nc, (int)g.fp32,
                              (int)g.poly, (int)g.seven, (int)g.mom);
                auto it = index.find(key);
                if (it == index.end()) {
                    it = index.emplace(key, (int)b->groups.size()).first;
                    b->groups.push_back(g);
                }
                b->groups[it->second].probs.push_back(i);
            }
        }
    }
    for (size_t k = 0; k < b->groups.size(); ++k) {
        Group &g = b->groups[k];
        g.counter = (int)k;
        g.pre.assign(1, 0);
        for (int i : g.probs) {
            const AssemblePlan &p = b->plans[i];
            g.pre.push_back(g.pre.back() + items_of(p, g.phase, g.cls));
            if (g.phase == kRows)
                g.row_lds = std::max(g.row_lds, row_lds_bytes(p.rows.maxlen, p.nc, p.rows.hcap));
        }
    }
}

// offsets of the groups' tables in one block; returns its size
size_t table_layout(nlfem_batch *b)
{
    size_t off = align256(sizeof(unsigned long long) * std::max<size_t>(b->groups.size(), 1));
    for (Group &g : b->groups) {
        const size_t np = g.probs.size();
        g.off_pre = off;
        off = align256(off + sizeof(int64_t) * (np + 1));
        g.off_args = off;
        size_t one = g.phase == kFar ? sizeof(FarArgs) : g.phase == kTouch ? sizeof(TouchArgs)
                   : g.phase == kDiag ? sizeof(DiagArgs) : sizeof(RowArgs);
        off = align256(off + one * np);
        if (g.phase == kFar) {
            g.off_r1 = off;
            off = align256(off + sizeof(RoleArgs) * np);
            g.off_r2 = off;
            off = align256(off + sizeof(RoleArgs) * np);
        } else if (g.phase == kTouch) {
            g.off_r1 = off;   // Gauss rules
            off = align256(off + sizeof(GaussArgs) * np);
        }
    }
    return off;
}

// the host image of the tables (counters zero)
std::vector<unsigned char> table_image(const nlfem_batch *b, size_t bytes)
{
    std::vector<unsigned char> host(bytes, 0);
    for (const Group &g : b->groups) {
        std::memcpy(&host[g.off_pre], g.pre.data(), sizeof(int64_t) * g.pre.size());
        for (size_t j = 0; j < g.probs.size(); ++j) {
            const AssemblePlan &p = b->plans[g.probs[j]];
            switch (g.phase) {
            case kFar:
                std::memcpy(&host[g.off_args + j * sizeof(FarArgs)], &p.far, sizeof(FarArgs));
                std::memcpy(&host[g.off_r1 + j * sizeof(RoleArgs)], &p.r1, sizeof(RoleArgs));
                std::memcpy(&host[g.off_r2 + j * sizeof(RoleArgs)], &p.r2, sizeof(RoleArgs));
                break;
            case kTouch: {
                const TouchArgs &t = p.touch[g.cls == 3 ? 0 : g.cls == 2 ? 1 : 2];
                std::memcpy(&host[g.off_args + j * sizeof(TouchArgs)], &t, sizeof(TouchArgs));
                std::memcpy(&host[g.off_r1 + j * sizeof(GaussArgs)], &p.gauss, sizeof(GaussArgs));
                break;
            }
            case kDiag:
                std::memcpy(&host[g.off_args + j * sizeof(DiagArgs)], &p.diag, sizeof(DiagArgs));
                break;
            default:
                std::memcpy(&host[g.off_args + j * sizeof(RowArgs)], &p.rows, sizeof(RowArgs));
            }
        }
    }
    return host;
}

int upload_tables(nlfem_batch *b, hipStream_t s)
{
    const size_t off = table_layout(b);
    const std::vector<unsigned char> host = table_image(b, off);
    NLFEM_TRY(dev_alloc(b->mem, off, s));
    b->dev = b->mem.p;
    b->dev_bytes = off;
    b->counters = (unsigned long long *)b->dev;
    NLFEM_HIP(hipMemcpyAsync(b->dev, host.data(), off, hipMemcpyHostToDevice, s));
    NLFEM_HIP(hipStreamSynchronize(s));   // the host table is freed on return
    return NLFEM_OK;
}

// ---- tuning

const Shape kCandidates[kPhases][6] = {
    {{256, 2}, {1024, 2}, {1024, 4}, {4096, 4}, {256, 8}, {1024, 8}},
    {{64, 2}, {256, 2}, {256, 4}, {1024, 4}, {64, 8}, {256, 8}},
    {{16, 4}, {64, 4}, {256, 4}, {64, 8}, {16, 8}, {256, 8}},
    {{1, 16}, {4, 16}, {16, 16}, {1, 32}, {4, 32}, {4, 8}},
};

std::string tune_key(const nlfem_batch *b)
{
    // device, then the group structure and item counts (rounded to 1/8 powers of two)
    hipDeviceProp_t prop{};
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipGetDeviceProperties(&prop, dev);
    std::string k = std::string(prop.gcnArchName) + "-cu" + std::to_string(b->cus);
    for (const Group &g : b->groups) {
        int64_t n = g.pre.back(), r = 1;
        while (r * 2 <= n) r *= 2;
        const int64_t q = n / std::max<int64_t>(r / 8, 1);
        char buf[64];
        std::snprintf(buf, sizeof buf, "|%d.%d.%d.%d.%lldx%lld", (int)g.phase, g.kernel, g.cls, (int)g.fp32,
                      (long long)q, (long long)std::max<int64_t>(r / 8, 1));
        k += buf;
    }
    return k;
}

// cache file: one line per key, "key chunk0 per_cu0 chunk1 per_cu1 ..."
bool cache_read(const char *path, const std::string &key, Shape *out)
{
    if (!path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[8192];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        const size_t kl = key.size();
        if (std::strncmp(line, key.c_str(), kl) != 0 || line[kl] != ' ') continue;
        Shape s[kPhases];
        int nread = std::sscanf(line + kl, " %d %d %d %d %d %d %d %d", &s[0].chunk, &s[0].per_cu, &s[1].chunk,
                                &s[1].per_cu, &s[2].chunk, &s[2].per_cu, &s[3].chunk, &s[3].per_cu);
        if (nread == 2 * kPhases) {
            bool ok = true;
            for (int p = 0; p < kPhases; ++p)
                ok &= (s[p].chunk == 0 && s[p].per_cu == 0) || (s[p].chunk > 0 && s[p].per_cu > 0 && s[p].per_cu <= 64);
            if (ok) {
                std::memcpy(out, s, sizeof s);
                found = true;
            }
        }
    }
    std::fclose(f);
    return found;
}

void cache_write(const char *path, const std::string &key, const Shape *s)
{
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s", key.c_str());
    for (int p = 0; p < kPhases; ++p) std::fprintf(f, " %d %d", s[p].chunk, s[p].per_cu);
    std::fprintf(f, "\n");
    std::fclose(f);
}

// Times every candidate shape of every phase (the phases before it have
// run, so each phase sees its real inputs) and keeps the fastest.
int tune(nlfem_batch *b, hipStream_t s)
{
    hipEvent_t e0, e1;
    NLFEM_HIP(hipEventCreate(&e0));
    NLFEM_HIP(hipEventCreate(&e1));
    int rc = NLFEM_OK;
    for (int ph = 0; ph < kPhases && rc == NLFEM_OK; ++ph) {
        bool any = false;
        for (const Group &g : b->groups) any |= g.phase == ph;
        if (!any) continue;
        // the queue shapes (rows: the static mapping only), then the
        // per-problem launches
        std::vector<Shape> cands;
        if (ph == kRows) cands.push_back(b->shape[ph]);
        else cands.assign(kCandidates[ph], kCandidates[ph] + 6);
        cands.push_back(Shape{0, 0});
        float best = 1e30f;
        for (const Shape &cand : cands) {
            float total = 0.f;
            for (int rep = 0; rep < 3 && rc == NLFEM_OK; ++rep) {
                hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(256), 0, s, b->counters, (int)b->groups.size());
                if (hipEventRecord(e0, s) != hipSuccess) rc = set_error(NLFEM_E_HIP, "hipEventRecord");
                if (rc == NLFEM_OK) rc = run_phase(b, (Phase)ph, cand, s);
                if (rc == NLFEM_OK && hipEventRecord(e1, s) != hipSuccess) rc = set_error(NLFEM_E_HIP, "hipEventRecord");
                if (rc == NLFEM_OK && hipEventSynchronize(e1) != hipSuccess) rc = set_error(NLFEM_E_HIP, "hipEventSynchronize");
                float ms = 0.f;
                if (rc == NLFEM_OK) (void)hipEventElapsedTime(&ms, e0, e1);
                if (rep > 0) total += ms;   // first run warms up
            }
            if (rc == NLFEM_OK && total < best) {
                best = total;
                b->shape[ph] = cand;
            }
        }
        // leave this phase's results in place for the next phase
        if (rc == NLFEM_OK) {
            hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(256), 0, s, b->counters, (int)b->groups.size());
            rc = run_phase(b, (Phase)ph, b->shape[ph], s);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

}  // namespace

namespace nlfem {

int batch_create(const std::vector<AssemblePlan> &plans, const std::vector<nlfem_pairs *> &handles,
                 const char *tune_cache, int tune_mode, nlfem_batch **out, hipStream_t s)
{
    nlfem_batch *b = new (std::nothrow) nlfem_batch();
    if (!b) return set_error(NLFEM_E_NOMEM, "host allocation failed");
    b->n = (int)plans.size();
    b->plans = plans;
    // the queue kernels take no speculative-rebuild gate (the handles are
    // checked on the host at each run); the per-problem launches alike
    for (AssemblePlan &p : b->plans) p.far.gate = p.diag.gate = p.rows.gate = SpecGate{};
    b->handles = handles;
    for (const nlfem_pairs *h : handles) b->generation.push_back(h->generation);
    int dev = 0;
    int rc = NLFEM_OK;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || b->cus < 1)
        rc = set_error(NLFEM_E_HIP, "cannot query the compute-unit count");
    if (rc == NLFEM_OK) {
        make_groups(b);
        rc = upload_tables(b, s);
    }
    for (int k = 0; k < 3 && rc == NLFEM_OK; ++k)
        if (hipStreamCreateWithFlags(&b->side[k], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming) != hipSuccess)
            rc = set_error(NLFEM_E_HIP, "cannot create the batch's side streams");
    if (rc == NLFEM_OK && hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess)
        rc = set_error(NLFEM_E_HIP, "cannot create the batch's events");
    if (rc == NLFEM_OK && tune_mode != 0) {
        const std::string key = tune_key(b);
        if (tune_mode == 2 || !cache_read(tune_cache, key, b->shape)) {
            rc = tune(b, s);
            if (rc == NLFEM_OK) cache_write(tune_cache, key, b->shape);
        }
    }
    if (rc == NLFEM_OK && hipStreamSynchronize(s) != hipSuccess) rc = set_error(NLFEM_E_HIP, "hipStreamSynchronize");
    if (rc != NLFEM_OK) {
        batch_free(b);
        return rc;
    }
    *out = b;
    return NLFEM_OK;
}

namespace {

// finishes unchecked rebuilds of the batch's handles; a handle built plainly
// since the batch was created may have other sizes and buffers
int check_handles(nlfem_batch *b)
{
    for (size_t i = 0; i < b->handles.size(); ++i) {
        NLFEM_TRY(resolve(b->handles[i]));
        if (b->handles[i]->generation != b->generation[i])
            return set_error(NLFEM_E_MISMATCH, "pairs handle " + std::to_string(i) +
                                                   " was rebuilt since the batch was created");
    }
    return NLFEM_OK;
}

}  // namespace

int batch_run(nlfem_batch *b, hipStream_t s)
{
    NLFEM_TRY(check_handles(b));
    return run_all(b, s, true);
}

int batch_graph_launch(nlfem_batch *b, hipStream_t s)
{
    NLFEM_TRY(check_handles(b));
    if (!b->exec) {
        if (!b->capture) NLFEM_HIP(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
        NLFEM_HIP(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
        const int rc = run_all(b, b->capture, false);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->capture, &g);
        if (rc != NLFEM_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_error(e, "hipStreamEndCapture");
        b->graph = g;
        NLFEM_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    NLFEM_HIP(hipGraphLaunch(b->exec, s));
    return NLFEM_OK;
}

void batch_free(nlfem_batch *b)
{
    if (!b) return;
    (void)hipDeviceSynchronize();   // no launch of the batch may still be running
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    for (int k = 0; k < 3; ++k) {
        if (b->side[k]) (void)hipStreamDestroy(b->side[k]);
        if (b->join[k]) (void)hipEventDestroy(b->join[k]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    dev_release(b->mem);
    delete b;
}

int batch_info(const nlfem_batch *b, int32_t *groups, int32_t *shape)
{
    *groups = (int32_t)b->groups.size();
    for (int p = 0; p < kPhases; ++p) {
        shape[2 * p] = b->shape[p].chunk;
        shape[2 * p + 1] = b->shape[p].per_cu;
    }
    return NLFEM_OK;
}

// ---- the allocation-free one-shot batch

namespace {

// Tables and queue counters of nlfem_assemble_batched_noalloc: one array per
// device, held until the process ends.  Host code never passes `scratch`
// itself (a host-side stand-in): it uses the device address taken by
// hipGetSymbolAddress on each device.
constexpr size_t kScratchBytes = NLFEM_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices];

int scratch_address(void **out)
{
    int dev = -1;
    NLFEM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return set_error(NLFEM_E_INVALID, "device ordinal above 63");
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_error(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return NLFEM_OK;
}

}  // namespace

size_t batch_scratch_bytes() { return kScratchBytes; }

int batch_assemble_noalloc(const std::vector<AssemblePlan> &plans, hipStream_t s)
{
    void *ptr = nullptr;
    NLFEM_TRY(scratch_address(&ptr));
    nlfem_batch b;   // host bookkeeping only: no streams, events or device memory
    b.n = (int)plans.size();
    b.plans = plans;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&b.cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || b.cus < 1)
        return set_error(NLFEM_E_HIP, "cannot query the compute-unit count");
    make_groups(&b);
    const size_t bytes = table_layout(&b);
    if (bytes > kScratchBytes)
        return set_error(NLFEM_E_OVERFLOW, "batch tables of " + std::to_string(bytes) +
                                               " bytes exceed the static workspace of " +
                                               std::to_string(kScratchBytes) + " bytes");
    const std::vector<unsigned char> host = table_image(&b, bytes);
    b.dev = ptr;
    b.dev_bytes = bytes;
    b.counters = (unsigned long long *)ptr;
    NLFEM_HIP(hipMemcpyAsync(ptr, host.data(), bytes, hipMemcpyHostToDevice, s));
    // the host image is freed on return; the copy reads it before then
    NLFEM_HIP(hipStreamSynchronize(s));
    // the counters start at zero (a fill kernel, as in the graph path); all
    // phases on the caller's stream: touching, non-touching, diagonals, rows
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(256), 0, s, b.counters, (int)b.groups.size());
    NLFEM_TRY(run_phase(&b, kTouch, b.shape[kTouch], s));
    NLFEM_TRY(run_phase(&b, kFar, b.shape[kFar], s));
    NLFEM_TRY(run_phase(&b, kDiag, b.shape[kDiag], s));
    NLFEM_TRY(run_phase(&b, kRows, b.shape[kRows], s));
    return NLFEM_OK;
}

}  // namespace nlfem

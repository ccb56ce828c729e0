// Post-processing of the interaction lists.
//
// 1. Every segment S(e) is sorted by neighbour id (in LDS, one wave per
//    element: by ranks up to kRankMax entries, else a bitonic network), so
//    that the pair (f, e) can be found in S(f) by binary search.
// 2. The entries with f >= e are the unordered pairs.  The same wave, with
//    the sorted list in LDS, compacts them into work lists: non-touching
//    pairs with their point status, touching pairs grouped by class
//    (identical, edge, vertex).  Each upper entry records the index of its
//    work item; each lower entry (f < e) takes the index of its mirror
//    (f, e) later, in the last workgroups of the CSR rows launch.  The
//    assembly computes one result per work item and every matrix row finds
//    the results of all its pairs through these indices.
#include "nlfem_internal.h"

namespace nlfem {
namespace {

constexpr int kRankMax = 256;   // longest list sorted by ranks

struct ListArgs {
    int64_t K, K1;
    const int64_t *sptr;
    const int64_t *loff;       // [kLsLast][K1] per-element offsets of the upper classes
    int32_t cap;               // power of two >= longest segment
    int32_t singular;
    int64_t baseE, baseV;
    const int64_t *scr;        // [K + 1] scratch segments of the pair search
    const int32_t *snbr_tmp;
    const uint8_t *sflag_tmp;
    const uint2 *smask_tmp;
    int32_t *snbr;
    uint8_t *sflag;
    int32_t *srec;
    int4 *snode;
    const int32_t *E;
    const int32_t *lab;
    const int64_t *ne_ptr;     // node -> element incidence
    const int32_t *ne_list;
    int32_t *ue, *uf;
    uint2 *um;
    int32_t *te, *tf;
    int32_t *err;
    SpecGate gate;
};

__global__ void __launch_bounds__(64) k_sort_lists(ListArgs a)
{
    extern __shared__ unsigned long long key[];
    if (gated(a.gate)) return;
    const int lane = threadIdx.x;
    for (int64_t b = blockIdx.x; b < xcd_span(a.K); b += gridDim.x) {
        const int64_t e = xcd_item(b, a.K);
        if (e >= a.K) continue;
        // conforming mesh (Sec. 2.2, Assumption 2): lane v counts the labelled
        // elements holding edge v of e (vertex indices are valid by now: the
        // build stops at an index error before this launch)
        if (lane < 3) {
            const int32_t le = a.lab[e];
            if (le == 1 || le == 2) {
                const int32_t va = a.E[3 * e + lane], vb = a.E[3 * e + (lane + 1) % 3];
                int cnt = 0;
                for (int64_t i = a.ne_ptr[va]; i < a.ne_ptr[va + 1]; ++i) {
                    const int32_t g = a.ne_list[i];
                    const int32_t lg = a.lab[g];
                    if (lg != 1 && lg != 2) continue;
                    cnt += (a.E[3 * (int64_t)g] == vb) | (a.E[3 * (int64_t)g + 1] == vb) |
                           (a.E[3 * (int64_t)g + 2] == vb);
                }
                if (cnt > 2) atomicOr(a.err, kErrEdge);
            }
        }
        const int64_t s0 = a.sptr[e], r0 = a.scr[e];   // final list, scratch segment
        const int n = (int)(a.sptr[e + 1] - s0);
        if (n == 0) continue;
        if (n <= kRankMax) {
            // rank sort: the place of a key is the number of smaller keys (the
            // keys differ); every lane reads every key by LDS broadcast, which
            // costs far less LDS bandwidth than the passes of a sorting network
            unsigned long long kv[kRankMax / 64];
            int rk[kRankMax / 64];
#pragma unroll
            for (int u = 0; u < kRankMax / 64; ++u) {
                const int t = lane + 64 * u;
                kv[u] = t < n ? (((unsigned long long)(uint32_t)a.snbr_tmp[r0 + t]) << 32) | (uint32_t)t : ~0ull;
                rk[u] = 0;
                if (t < n) key[t] = kv[u];
            }
            if (lane == 0 && (n & 1)) key[n] = ~0ull;   // n < cap when odd: pads the last pair
            __syncthreads();
            for (int j = 0; j < n; j += 2) {
                const unsigned long long x = key[j], y = key[j + 1];
#pragma unroll
                for (int u = 0; u < kRankMax / 64; ++u)
                    if (64 * u < n) rk[u] += (int)(x < kv[u]) + (int)(y < kv[u]);
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kRankMax / 64; ++u)
                if (lane + 64 * u < n) key[rk[u]] = kv[u];
            __syncthreads();
        } else {
            // bitonic sort of the keys padded to a power of two
            int n2 = 1;
            while (n2 < n) n2 <<= 1;
            for (int t = lane; t < n2; t += 64)
                key[t] = t < n ? (((unsigned long long)(uint32_t)a.snbr_tmp[r0 + t]) << 32) | (uint32_t)t : ~0ull;
            __syncthreads();
            for (int k = 2; k <= n2; k <<= 1)
                for (int j = k >> 1; j > 0; j >>= 1) {
                    for (int t = lane; t < n2; t += 64) {
                        const int ixj = t ^ j;
                        if (ixj > t) {
                            const unsigned long long x = key[t], y = key[ixj];
                            if ((x > y) == ((t & k) == 0)) {
                                key[t] = y;
                                key[ixj] = x;
                            }
                        }
                    }
                    __syncthreads();
                }
        }
        // the sorted list, and the upper entries (f >= e) appended to the work
        // lists of their class in list order; lower entries get their record
        // from the mirror (link_element, in the CSR rows launch)
        const unsigned long long lt = (1ull << lane) - 1ull;
        int64_t oF = a.loff[kLsUF * a.K1 + e];
        int64_t oI = a.loff[kLsUI * a.K1 + e];
        int64_t oE = a.baseE + a.loff[kLsUE * a.K1 + e];
        int64_t oV = a.baseV + a.loff[kLsUV * a.K1 + e];
        for (int t0 = 0; t0 < n; t0 += 64) {
            const int t = t0 + lane;
            bool isF = false, isI = false, isE = false, isV = false;
            int32_t f = 0;
            int src = 0;
            if (t < n) {
                const unsigned long long kk = key[t];
                src = (int)(kk & 0xffffffffull);
                f = (int32_t)(kk >> 32);
                const uint8_t fl = a.sflag_tmp[r0 + src];
                a.snbr[s0 + t] = f;
                a.sflag[s0 + t] = fl;
                a.snode[s0 + t] = make_int4(f, a.E[3 * (int64_t)f], a.E[3 * (int64_t)f + 1], a.E[3 * (int64_t)f + 2]);
                const int cls = (fl >> 2) & 3;
                const bool upper = f >= e;
                isF = upper && cls == 0;
                isI = upper && cls == 3;
                isE = upper && cls == 2;
                isV = upper && cls == 1;
            }
            const unsigned long long bF = __ballot(isF), bI = __ballot(isI);
            const unsigned long long bE = __ballot(isE), bV = __ballot(isV);
            int32_t rec = -1;
            if (isF) {
                // the point status travels with the non-touching work item only
                const uint2 m = a.smask_tmp[r0 + src];
                const int64_t u = oF + __popcll(bF & lt);
                a.ue[u] = (int32_t)e;
                a.uf[u] = f;
                a.um[u] = make_uint2(m.x, f == e ? 0u : m.y);
                rec = (int32_t)u;
            }
            if (isI || isE || isV) {
                const int64_t u = isI ? oI + __popcll(bI & lt) : isE ? oE + __popcll(bE & lt)
                                                                      : oV + __popcll(bV & lt);
                a.te[u] = (int32_t)e;
                a.tf[u] = f;
                rec = (int32_t)u;
            }
            if (t < n) a.srec[s0 + t] = rec;
            oF += __popcll(bF);
            oI += __popcll(bI);
            oE += __popcll(bE);
            oV += __popcll(bV);
        }
        __syncthreads();
    }
}

ListArgs list_args(nlfem_pairs *h)
{
    ListArgs a{};
    a.K = h->K;
    a.K1 = h->K + 1;
    a.sptr = h->loff + (int64_t)kLsS * (h->K + 1);
    a.loff = h->loff;
    int cap = 64;
    while (cap < h->max_S) cap <<= 1;
    a.cap = cap;
    a.singular = h->singular;
    a.baseE = h->nUTc[0];
    a.baseV = h->nUTc[0] + h->nUTc[1];
    a.scr = h->scr_off;
    a.snbr_tmp = h->snbr_tmp;
    a.sflag_tmp = h->sflag_tmp;
    a.smask_tmp = h->smask_tmp;
    a.snbr = h->snbr;
    a.sflag = h->sflag;
    a.srec = h->srec;
    a.snode = h->snode;
    a.E = h->mesh_elements;
    a.lab = h->mesh_labels;
    a.ne_ptr = h->ne_ptr;
    a.ne_list = h->ne_list;
    a.ue = h->ue;
    a.uf = h->uf;
    a.um = h->um;
    a.te = h->te;
    a.tf = h->tf;
    a.err = h->err;
    a.gate = h->gate;
    return a;
}

}  // namespace

int launch_sort_lists(nlfem_pairs *h, hipStream_t s)
{
    ListArgs a = list_args(h);
    if (a.cap > 8192) return set_error(NLFEM_E_OVERFLOW, "neighbour list longer than 8192 entries");
    const unsigned grid = xcd_grid(h->K);
    hipLaunchKernelGGL(k_sort_lists, dim3(grid), dim3(64), sizeof(unsigned long long) * a.cap, s, a);
    NLFEM_HIP(hipGetLastError());
    return NLFEM_OK;
}


}  // namespace nlfem

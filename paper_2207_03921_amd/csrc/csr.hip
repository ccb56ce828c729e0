// CSR pattern of the stiffness matrix and export of the pair list.
//
// Row i (a degree of freedom) holds the union of the vertex sets of all
// interacting pairs that have i as a vertex.  With the symmetric neighbour
// list S(e) this is the union over the elements e containing i (those with
// S(e) non-empty) of nodes(e) and of nodes(f) for f in S(e).  One wave per
// row inserts these ids into an open-addressing hash set in LDS, compacts and
// sorts the unique ids and writes them to a row slot of a staging
// buffer; after the scan of the row lengths a copy kernel packs the slots.
// A neighbour f met again through another element of the row adds nothing
// new: a second hash set of element ids lets only the first meeting insert
// the vertices of f.
// The entries of all the row's elements are handled as one flat range: each
// lane loads kCsrU neighbour ids and their vertices before it inserts any,
// so the dependent loads of a step overlap.
#include "nlfem_internal.h"

namespace nlfem {
namespace {

constexpr int kEmpty = -1;
constexpr int kCsrQ = 64;    // elements around a node per batch
constexpr int kCsrU = 4;     // entries per lane per step
constexpr int kRankMax = 256;   // longest row sorted by ranks

struct CsrArgs {
    const int32_t *E;
    const int32_t *rows;                   // dof nodes
    const unsigned long long *nrows;       // [1] their number
    const int64_t *ne_ptr;
    const int32_t *ne_list;
    const int64_t *sptr;     // [K + 1]
    const int4 *snode;       // (f, vertices of f) per neighbour-list entry
    int32_t hcap;            // power of two
    int32_t cap;             // slot length of the staging buffer (3/4 hcap)
    int32_t *stage;          // [n_dof][cap]
    int64_t *nlen;
    int32_t *err;
    SpecGate gate;
    // mirror links, run by the link_blocks workgroups after the row_blocks
    // workgroups of the rows
    int64_t K, link_blocks, row_blocks;
    int32_t wpb;             // waves (rows) per workgroup: fewer when the hash tables are large
    const int32_t *snbr;     // sorted neighbour lists
    int32_t *srec;
};

// Lower entries (f < e) of S(e) take the record of their mirror (f, e) in
// S(f), found by binary search (the lists are sorted); one wave per element.
__device__ void link_element(const CsrArgs &a, int64_t e, int lane)
{
    const int64_t s0 = a.sptr[e], s1 = a.sptr[e + 1];
    for (int64_t t = s0 + lane; t < s1; t += 64) {
        const int32_t f = a.snbr[t];
        if (f >= e) continue;
        int64_t lo = a.sptr[f], hi = a.sptr[f + 1];
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (a.snbr[mid] < e) lo = mid + 1;
            else hi = mid;
        }
        if (lo < a.sptr[f + 1] && a.snbr[lo] == (int32_t)e) a.srec[t] = a.srec[lo];
        else atomicOr(a.err, kErrSlot);
    }
}

__device__ inline bool hash_insert(int32_t *tab, int32_t mask, int32_t key, bool *overflow)
{
    uint32_t h = ((uint32_t)key * 2654435761u) & (uint32_t)mask;
    for (int probe = 0; probe <= mask; ++probe) {
        const int32_t old = atomicCAS(&tab[h], kEmpty, key);
        if (old == kEmpty) return true;
        if (old == key) return false;
        h = (h + 1) & (uint32_t)mask;
    }
    *overflow = true;
    return false;
}

// true when key was in the table already; inserts it otherwise (a full table
// answers false, so the caller treats the key as new)
__device__ inline bool hash_seen(int32_t *tab, int32_t mask, int32_t key)
{
    uint32_t h = ((uint32_t)key * 2654435761u) & (uint32_t)mask;
    for (int probe = 0; probe <= mask; ++probe) {
        const int32_t old = atomicCAS(&tab[h], kEmpty, key);
        if (old == kEmpty) return false;
        if (old == key) return true;
        h = (h + 1) & (uint32_t)mask;
    }
    return false;
}

__device__ inline int wave_sum(int v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Each wave of a workgroup owns one row and its LDS; the waves never wait
// for each other.
__global__ void __launch_bounds__(64 * kWavesPerRowBlock) k_csr_rows(CsrArgs a)
{
    extern __shared__ int32_t dyn[];
    if (gated(a.gate)) return;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if ((int64_t)blockIdx.x >= a.row_blocks) {
        // the links share the launch: both are latency-bound and independent,
        // and the shorter link items fill the tail of the rows
        const int64_t ng = (a.K + a.wpb - 1) / a.wpb;
        for (int64_t b = blockIdx.x - a.row_blocks; b < xcd_span(ng); b += a.link_blocks) {
            const int64_t e = xcd_item(b, ng) * a.wpb + w;
            if (e < a.K) link_element(a, e, lane);
        }
        return;
    }
    // [hcap] node hash table, then [hcap] element hash table, which becomes
    // the sort buffer once the row's ids are in
    int32_t *tab = dyn + (size_t)w * 2 * a.hcap;
    int32_t *etab = tab + a.hcap, *buf = etab;
    __shared__ int64_t qs_w[kWavesPerRowBlock][kCsrQ];
    __shared__ int32_t pre_w[kWavesPerRowBlock][kCsrQ + 1];
    int64_t *qs = qs_w[w];
    int32_t *pre = pre_w[w];
    const int32_t mask = a.hcap - 1;
    const int64_t nrows = (int64_t)*a.nrows;
    const int64_t ngroups = (nrows + a.wpb - 1) / a.wpb;
    for (int64_t b = blockIdx.x; b < xcd_span(ngroups); b += a.row_blocks) {
        const int64_t item = xcd_item(b, ngroups) * a.wpb + w;
        if (item >= nrows) continue;
        const int64_t i = a.rows[item];
        for (int t = lane; t < a.hcap; t += 64) {
            tab[t] = kEmpty;
            etab[t] = kEmpty;
        }
        wave_sync();
        bool overflow = false;
        int added = 0;
        const int64_t q0 = a.ne_ptr[i], q1 = a.ne_ptr[i + 1];
        for (int64_t qb = q0; qb < q1; qb += kCsrQ) {
            const int nq = (int)min((int64_t)kCsrQ, q1 - qb);
            int cnt = 0;
            if (lane < nq) {
                const int32_t e = a.ne_list[qb + lane];
                const int64_t s0 = a.sptr[e];
                cnt = (int)(a.sptr[e + 1] - s0);
                qs[lane] = s0;
                if (cnt > 0) {   // elements of interacting pairs contribute their own nodes
                    const int32_t v0 = a.E[3 * (int64_t)e], v1 = a.E[3 * (int64_t)e + 1], v2 = a.E[3 * (int64_t)e + 2];
                    added += hash_insert(tab, mask, v0, &overflow);
                    added += hash_insert(tab, mask, v1, &overflow);
                    added += hash_insert(tab, mask, v2, &overflow);
                }
            }
            int incl = cnt;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(incl, o);
                if (lane >= o) incl += y;
            }
            if (lane < nq) pre[lane + 1] = incl;
            if (lane == 0) pre[0] = 0;
            const int total = __shfl(incl, nq - 1);
            wave_sync();
            for (int base = 0; base < total; base += 64 * kCsrU) {
                int4 sn[kCsrU];
#pragma unroll
                for (int k = 0; k < kCsrU; ++k) {
                    const int flat = base + k * 64 + lane;
                    sn[k] = make_int4(-1, -1, -1, -1);
                    if (flat < total) {
                        int lo = 0, hi = nq;   // pre[lo] <= flat < pre[hi]
                        while (hi - lo > 1) {
                            const int mid = (lo + hi) >> 1;
                            if (pre[mid] <= flat) lo = mid;
                            else hi = mid;
                        }
                        sn[k] = a.snode[qs[lo] + (flat - pre[lo])];
                    }
                }
                bool fresh[kCsrU];
#pragma unroll
                for (int k = 0; k < kCsrU; ++k) fresh[k] = sn[k].x >= 0 && !hash_seen(etab, mask, sn[k].x);
#pragma unroll
                for (int k = 0; k < kCsrU; ++k) {
                    if (!fresh[k]) continue;
                    added += hash_insert(tab, mask, sn[k].y, &overflow);
                    added += hash_insert(tab, mask, sn[k].z, &overflow);
                    added += hash_insert(tab, mask, sn[k].w, &overflow);
                }
            }
            wave_sync();
        }
        const int n = wave_sum(added);
        const bool full = __any(overflow) || n > a.cap;
        if (full) {
            if (lane == 0) {
                atomicOr(a.err, kErrRowCap);
                a.nlen[i] = 0;
            }
            wave_sync();
            continue;
        }
        // compact in slot order, then sort
        int basec = 0;
        for (int t0 = 0; t0 < a.hcap; t0 += 64) {
            const int32_t v = tab[t0 + lane];
            const unsigned long long bb = __ballot(v != kEmpty);
            if (v != kEmpty) buf[basec + __popcll(bb & ((1ull << lane) - 1ull))] = v;
            basec += __popcll(bb);
        }
        wave_sync();
        int32_t *out = a.stage + item * (int64_t)a.cap;
        if (n <= kRankMax) {
            // rank sort: the place of an id is the number of smaller ids (the
            // ids differ), read by LDS broadcast; each id goes straight to
            // its place in the slot
            int32_t kv[kRankMax / 64];
            int rk[kRankMax / 64];
#pragma unroll
            for (int u = 0; u < kRankMax / 64; ++u) {
                const int t = lane + 64 * u;
                kv[u] = t < n ? buf[t] : 0x7fffffff;
                rk[u] = 0;
            }
            for (int j = 0; j < n; ++j) {
                const int32_t x = buf[j];
#pragma unroll
                for (int u = 0; u < kRankMax / 64; ++u)
                    if (64 * u < n) rk[u] += (int)(x < kv[u]);
            }
#pragma unroll
            for (int u = 0; u < kRankMax / 64; ++u)
                if (lane + 64 * u < n) out[rk[u]] = kv[u];
        } else {
            // bitonic sort of the ids padded to a power of two
            int n2 = 1;
            while (n2 < n) n2 <<= 1;
            for (int t = n + lane; t < n2; t += 64) buf[t] = 0x7fffffff;
            wave_sync();
            for (int k = 2; k <= n2; k <<= 1) {
                for (int j = k >> 1; j > 0; j >>= 1) {
                    for (int t = lane; t < n2; t += 64) {
                        const int ixj = t ^ j;
                        if (ixj > t) {
                            const int32_t x = buf[t], y = buf[ixj];
                            const bool up = (t & k) == 0;
                            if ((x > y) == up) {
                                buf[t] = y;
                                buf[ixj] = x;
                            }
                        }
                    }
                    wave_sync();
                }
            }
            for (int t = lane; t < n; t += 64) out[t] = buf[t];
        }
        if (lane == 0) a.nlen[i] = n;   // the longest row comes from the scan of nlen
        wave_sync();
    }
}

// packs the staged rows: ncol[nptr[i] ...] = stage[item][0 .. nlen[i])
// With slots_out (pinned host memory), the first workgroup also copies the
// reduction slots there before anything else (every slot is final by this
// launch), so a rebuild needs no separate read-back copy.
__global__ void __launch_bounds__(256) k_csr_pack(const int32_t *rows, const unsigned long long *nrows,
                                                  const int64_t *nptr, const int32_t *stage, int32_t cap,
                                                  int32_t *ncol, SpecGate gate, const unsigned long long *slots,
                                                  unsigned long long *slots_out)
{
    if (slots_out && blockIdx.x == 0 && threadIdx.x < kRedSlots) slots_out[threadIdx.x] = slots[threadIdx.x];
    if (gated(gate)) return;
    const int64_t nr = (int64_t)*nrows;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int64_t item = (int64_t)blockIdx.x * 4 + w; item < nr; item += (int64_t)gridDim.x * 4) {
        const int64_t i = rows[item];
        const int64_t o = nptr[i], len = nptr[i + 1] - o;
        const int32_t *src = stage + item * (int64_t)cap;
        for (int64_t t = lane; t < len; t += 64) ncol[o + t] = src[t];
    }
}

// scalar CSR (n components per node, interleaved) from the node-level pattern
__global__ void __launch_bounds__(256) k_pattern_rows(int64_t M, int ncomp, const int64_t *nptr,
                                                      int64_t *row_ptr)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > M) return;
    if (i == M) {
        row_ptr[(int64_t)ncomp * M] = (int64_t)ncomp * ncomp * nptr[M];
        return;
    }
    const int64_t len = nptr[i + 1] - nptr[i];
    for (int c = 0; c < ncomp; ++c)
        row_ptr[(int64_t)ncomp * i + c] = (int64_t)ncomp * ncomp * nptr[i] + (int64_t)c * ncomp * len;
}

__global__ void __launch_bounds__(256) k_pattern_cols(int64_t M, int ncomp, const int64_t *nptr,
                                                      const int32_t *ncol, int32_t *col)
{
    const int64_t i = blockIdx.x;   // node row
    if (i >= M) return;
    const int64_t s = nptr[i], len = nptr[i + 1] - s;
    for (int64_t t = threadIdx.x; t < len; t += blockDim.x) {
        const int32_t j = ncol[s + t];
        for (int c = 0; c < ncomp; ++c)
            for (int d = 0; d < ncomp; ++d)
                col[(int64_t)ncomp * ncomp * s + (int64_t)c * ncomp * len + (int64_t)ncomp * t + d] =
                    ncomp * j + d;
    }
}

// ordered pairs (k = e, l = f) with bit0 of the flags, sorted by f per e
__global__ void __launch_bounds__(64) k_export(int64_t K, const int64_t *sptr, const int32_t *snbr,
                                               const uint8_t *sflag, const int64_t *pptr, int cap,
                                               int32_t *ko, int32_t *lo, int8_t *co)
{
    extern __shared__ int32_t sh[];   // [cap] keys (f << 2 | cls)
    const int lane = threadIdx.x;
    for (int64_t e = blockIdx.x; e < K; e += gridDim.x) {
        const int64_t s0 = sptr[e], s1 = sptr[e + 1];
        int base = 0;
        for (int64_t t0 = s0; t0 < s1; t0 += 64) {
            const int64_t t = t0 + lane;
            bool take = false;
            int32_t key = 0;
            if (t < s1) {
                const uint8_t fl = sflag[t];
                take = (fl & 1u) != 0;
                key = (snbr[t] << 2) | ((fl >> 2) & 3);
            }
            const unsigned long long b = __ballot(take);
            if (take) sh[base + __popcll(b & ((1ull << lane) - 1ull))] = key;
            base += __popcll(b);
        }
        const int n = base;
        int n2 = 1;
        while (n2 < n) n2 <<= 1;
        for (int t = n + lane; t < n2; t += 64) sh[t] = 0x7fffffff;
        __syncthreads();
        for (int k = 2; k <= n2; k <<= 1)
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int t = lane; t < n2; t += 64) {
                    const int ixj = t ^ j;
                    if (ixj > t) {
                        const int32_t x = sh[t], y = sh[ixj];
                        if ((x > y) == ((t & k) == 0)) {
                            sh[t] = y;
                            sh[ixj] = x;
                        }
                    }
                }
                __syncthreads();
            }
        const int64_t o = pptr[e];
        for (int t = lane; t < n; t += 64) {
            ko[o + t] = (int32_t)e;
            lo[o + t] = sh[t] >> 2;
            co[o + t] = (int8_t)(sh[t] & 3);
        }
        __syncthreads();
    }
}

}  // namespace

int launch_csr_rows(nlfem_pairs *h, const nlfem_mesh *m, hipStream_t s, bool links, bool rows)
{
    CsrArgs a{m->elements, h->dof_list, h->red + kRedDofs, h->ne_ptr, h->ne_list,
              h->loff + (int64_t)kLsS * (h->K + 1), h->snode, h->hcap, csr_slot(h->hcap), h->csr_stage, h->nlen,
              h->err, h->gate};
    // with links: the last workgroups set the mirror records (once per build)
    a.K = h->K;
    // each wave holds two hash tables of hcap ids; at most 128 KB of LDS per
    // workgroup (gfx950 has 160 KB per CU): fewer rows per workgroup for
    // long rows (horizons of many mesh sizes)
    const size_t per_wave = sizeof(int32_t) * 2 * (size_t)h->hcap;
    a.wpb = kWavesPerRowBlock;
    while (a.wpb > 1 && per_wave * a.wpb > ((size_t)128 << 10)) a.wpb >>= 1;
    a.link_blocks = links && h->nS > 0 ? xcd_grid((h->K + a.wpb - 1) / a.wpb) : 0;
    a.row_blocks = rows ? xcd_grid((h->M + a.wpb - 1) / a.wpb) : 0;   // links only: rows of the
                                                                        // discontinuous ansatz come from dg.hip
    if (a.row_blocks + a.link_blocks == 0) return NLFEM_OK;
    a.snbr = h->snbr;
    a.srec = h->srec;
    const size_t lds = per_wave * a.wpb;
    hipLaunchKernelGGL(k_csr_rows, dim3((unsigned)(a.row_blocks + a.link_blocks)), dim3(64 * a.wpb), lds, s, a);
    NLFEM_HIP(hipGetLastError());
    return NLFEM_OK;
}

int launch_csr_pack(nlfem_pairs *h, hipStream_t s, unsigned long long *slots_out)
{
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(grid_for(h->n_dof, 4), 1 << 16));
    hipLaunchKernelGGL(k_csr_pack, dim3(grid), dim3(256), 0, s, h->dof_list, h->red + kRedDofs, h->nptr,
                       h->csr_stage, csr_slot(h->hcap), h->ncol, h->gate, h->red, slots_out);
    NLFEM_HIP(hipGetLastError());
    return NLFEM_OK;
}

int launch_pattern(const nlfem_pairs *h, int64_t *row_ptr, int32_t *col, hipStream_t s)
{
    hipLaunchKernelGGL(k_pattern_rows, dim3(grid_for(h->M + 1, 256)), dim3(256), 0, s, h->M, h->ncomp,
                       h->nptr, row_ptr);
    if (h->nnz_node > 0)
        hipLaunchKernelGGL(k_pattern_cols, dim3((unsigned)h->M), dim3(256), 0, s, h->M, h->ncomp, h->nptr,
                           h->ncol, col);
    NLFEM_HIP(hipGetLastError());
    return NLFEM_OK;
}

int launch_export(const nlfem_pairs *h, int32_t *k, int32_t *l, int8_t *cls, hipStream_t s)
{
    if (h->nP == 0) return NLFEM_OK;
    int cap = 64;
    while (cap < h->max_S) cap <<= 1;
    if (cap > 16384) return set_error(NLFEM_E_OVERFLOW, "neighbour list too long for export");
    const unsigned grid = (unsigned)std::min<int64_t>(h->K, 1 << 20);
    hipLaunchKernelGGL(k_export, dim3(grid), dim3(64), sizeof(int32_t) * cap, s, h->K,
                       h->loff + (int64_t)kLsS * (h->K + 1), h->snbr, h->sflag,
                       h->loff + (int64_t)kLsP * (h->K + 1), cap, k, l, cls);
    NLFEM_HIP(hipGetLastError());
    return NLFEM_OK;
}

}  // namespace nlfem

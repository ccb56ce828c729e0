// CSR pattern of the stiffness matrix and export of the pair list.
//
// Row i (a degree of freedom) holds the union of the vertex sets of all
// interacting pairs that have i as a vertex.  With the symmetric neighbour
// list S(e) this is the union over the elements e containing i (those with
// S(e) non-empty) of nodes(e) and of nodes(f) for f in S(e).  One wave per
// row inserts these ids into an open-addressing hash set in LDS, then
// compacts and bitonic-sorts the unique ids.
#include "nlfem_internal.h"

namespace nlfem {
namespace {

constexpr int kEmpty = -1;

struct CsrArgs {
    int64_t K1, M;
    const int32_t *E;
    const int32_t *rows;                   // dof nodes
    const unsigned long long *nrows;       // [1] their number
    const int64_t *ne_ptr;
    const int32_t *ne_list;
    const int64_t *sptr;     // [K + 1]
    const int32_t *snbr;
    int32_t hcap;            // power of two
    int64_t *nlen;           // count pass
    unsigned long long *max_row;
    const int64_t *nptr;     // fill pass
    int32_t *ncol;
    int32_t *err;
};

__device__ inline bool hash_insert(int32_t *tab, int32_t mask, int32_t key, bool *overflow)
{
    uint32_t h = ((uint32_t)key * 2654435761u) & (uint32_t)mask;
    for (int probe = 0; probe <= mask; ++probe) {
        int32_t old = atomicCAS(&tab[h], kEmpty, key);
        if (old == kEmpty) return true;
        if (old == key) return false;
        h = (h + 1) & (uint32_t)mask;
    }
    *overflow = true;
    return false;
}

__device__ inline int wave_sum(int v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <bool FILL>
__global__ void __launch_bounds__(64) k_csr(CsrArgs a)
{
    extern __shared__ int32_t tab[];   // [hcap] hash table, then [hcap] sort buffer
    int32_t *buf = tab + a.hcap;
    const int lane = threadIdx.x;
    const int64_t nrows = (int64_t)*a.nrows;
    for (int64_t b = blockIdx.x; b < xcd_span(nrows); b += gridDim.x) {
        const int64_t item = xcd_item(b, nrows);
        if (item >= nrows) continue;
        const int64_t i = a.rows[item];
        for (int t = lane; t < a.hcap; t += 64) tab[t] = kEmpty;
        __syncthreads();
        const int32_t mask = a.hcap - 1;
        bool overflow = false;
        int added = 0;
        for (int64_t q = a.ne_ptr[i]; q < a.ne_ptr[i + 1]; ++q) {
            const int32_t e = a.ne_list[q];
            const int64_t s0 = a.sptr[e], s1 = a.sptr[e + 1];
            if (s1 == s0) continue;
            if (lane < 3) added += hash_insert(tab, mask, a.E[3 * (int64_t)e + lane], &overflow);
            for (int64_t t = s0 + lane; t < s1; t += 64) {
                const int32_t f = a.snbr[t];
                added += hash_insert(tab, mask, a.E[3 * (int64_t)f], &overflow);
                added += hash_insert(tab, mask, a.E[3 * (int64_t)f + 1], &overflow);
                added += hash_insert(tab, mask, a.E[3 * (int64_t)f + 2], &overflow);
            }
        }
        const int n = wave_sum(added);
        const bool full = __any(overflow) || 4 * n > 3 * a.hcap;
        if (full) {
            if (lane == 0) atomicOr(a.err, kErrRowCap);
            if (!FILL && lane == 0) a.nlen[i] = 0;
            __syncthreads();
            continue;
        }
        if (!FILL) {
            if (lane == 0) {
                a.nlen[i] = n;
                atomicMax(a.max_row, (unsigned long long)n);
            }
            __syncthreads();
            continue;
        }
        __syncthreads();
        // compact in slot order
        int base = 0;
        for (int t0 = 0; t0 < a.hcap; t0 += 64) {
            const int32_t v = tab[t0 + lane];
            const unsigned long long b = __ballot(v != kEmpty);
            if (v != kEmpty) buf[base + __popcll(b & ((1ull << lane) - 1ull))] = v;
            base += __popcll(b);
        }
        int n2 = 1;
        while (n2 < n) n2 <<= 1;
        for (int t = n + lane; t < n2; t += 64) buf[t] = 0x7fffffff;
        __syncthreads();
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
                __syncthreads();
            }
        }
        const int64_t o = a.nptr[i];
        for (int t = lane; t < n; t += 64) a.ncol[o + t] = buf[t];
        __syncthreads();
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

int launch_csr(nlfem_pairs *h, const nlfem_mesh *m, bool fill, hipStream_t s)
{
    CsrArgs a{h->K + 1, h->M, m->elements, h->dof_list, h->red + 8, h->ne_ptr, h->ne_list,
              h->loff + (int64_t)kLsS * (h->K + 1), h->snbr, h->hcap, h->nlen, h->red + 9, h->nptr, h->ncol,
              h->err};
    const size_t lds = sizeof(int32_t) * 2 * (size_t)h->hcap;
    const unsigned grid = xcd_grid(h->M);
    if (fill) hipLaunchKernelGGL(k_csr<true>, dim3(grid), dim3(64), lds, s, a);
    else hipLaunchKernelGGL(k_csr<false>, dim3(grid), dim3(64), lds, s, a);
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

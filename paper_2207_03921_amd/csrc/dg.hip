// Discontinuous P1 ansatz (Sec. 1 and 2.3: the ansatz space may be
// continuous or discontinuous).  Every element carries its own three basis
// functions, unknown n (3k + a) + c for vertex a of element k (stored order)
// and component c; rows exist for the elements of Omega.  The matrix row
// block of element e holds, for every element f of S+(e) (the sorted
// neighbour list S(e), with e inserted when missing), the 3n x 3n block of
// the pairs (e, f) and (f, e): far pairs give the cross block X of their
// record (transposed when f < e) and e's own block the summed diagonal
// blocks; touching pairs of a singular kernel give their local matrix over
// the six (identical: three) unknowns, whose (e, e) part also lands in e's
// own block.
//
// Touching pairs: identical pairs have the continuous basis differences and
// use the reduced transforms of the continuous path; edge and vertex pairs
// use the 4D tensor form of the regularising transforms (the basis values no
// longer vanish at the shared vertices, so the radial direction is not
// integrated in closed form): edge pairs
//   v = rho w, w on the faces (p, 1-p, q), (p, (1-p)q, 1), (-p, 1, (1-p)q),
//   (-p, q, 1-p), xi_1 = max(0, v_1) + (1 - rho) tau, xi_2 = v_2,
//   eta = (xi_1 - v_1, v_3), weight rho^2 (1 - rho) (1 - p on the collapsed
//   faces),
// vertex pairs xi = s (1 - a, a), eta = t (1 - b, b) with t = s w (weight
// s^3 w) or s = t w (weight t^3 w), in the frames of the continuous path.
#include "assemble_items.h"

namespace nlfem {
using namespace items;
namespace {

// the row of element e in S+(e): start and length of S(e), e's position and
// whether e is listed
struct DgRow {
    int64_t s0;
    int n, cnt, pe;
    bool ein;
};

__device__ inline DgRow dg_row(const int64_t *sptr, const int32_t *snbr, int64_t e)
{
    DgRow r;
    r.s0 = sptr[e];
    r.n = (int)(sptr[e + 1] - r.s0);
    int lo = 0, hi = r.n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (snbr[r.s0 + mid] < (int32_t)e) lo = mid + 1;
        else hi = mid;
    }
    r.pe = lo;
    r.ein = lo < r.n && snbr[r.s0 + lo] == (int32_t)e;
    r.cnt = r.n == 0 ? 0 : r.n + (r.ein ? 0 : 1);
    return r;
}

// element at position j of S+(e) and its list index (-1: e inserted)
__device__ inline int32_t dg_entry(const DgRow &r, const int32_t *snbr, int64_t e, int j, int64_t *t)
{
    if (r.ein || j < r.pe) {
        *t = r.s0 + j;
        return snbr[*t];
    }
    if (j == r.pe) {
        *t = -1;
        return (int32_t)e;
    }
    *t = r.s0 + j - 1;
    return snbr[*t];
}

struct DgCountArgs {
    int64_t K;
    const int32_t *lab;
    const int64_t *sptr;
    const int32_t *snbr;
    int64_t *cnt;
    unsigned long long *ndof;   // Omega elements (x 3 unknowns per component)
};

__global__ void __launch_bounds__(256) k_dg_counts(DgCountArgs a)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool om = e < a.K && a.lab[e] == 1;
    if (e < a.K) a.cnt[e] = om ? dg_row(a.sptr, a.snbr, e).cnt : 0;
    const unsigned long long b = __ballot(om);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(a.ndof, (unsigned long long)__popcll(b));
}

struct DgPatternArgs {
    int64_t K;
    int32_t nc;
    const int64_t *dptr;     // [K + 1] element blocks before each element
    const int64_t *sptr;
    const int32_t *snbr;
    const int32_t *lab;
    int64_t *row_ptr;        // [nc 3K + 1]
    int32_t *col;
};

__global__ void __launch_bounds__(256) k_dg_row_ptr(DgPatternArgs a)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nrow = 3 * a.nc * a.K;
    if (r > nrow) return;
    const int bw = 3 * a.nc;   // unknowns per element block
    if (r == nrow) {
        a.row_ptr[r] = (int64_t)bw * bw * a.dptr[a.K];
        return;
    }
    const int64_t e = r / bw;
    const int64_t cnt = a.dptr[e + 1] - a.dptr[e];
    a.row_ptr[r] = (int64_t)bw * bw * a.dptr[e] + (r - e * bw) * bw * cnt;
}

__global__ void __launch_bounds__(64) k_dg_cols(DgPatternArgs a)
{
    const int lane = threadIdx.x;
    const int bw = 3 * a.nc;
    for (int64_t e = blockIdx.x; e < a.K; e += gridDim.x) {
        const int64_t cnt = a.dptr[e + 1] - a.dptr[e];
        if (cnt == 0) continue;
        const DgRow rr = dg_row(a.sptr, a.snbr, e);
        const int64_t base = (int64_t)bw * bw * a.dptr[e];
        for (int j = lane; j < (int)cnt; j += 64) {
            int64_t t;
            const int32_t f = dg_entry(rr, a.snbr, e, j, &t);
            for (int row = 0; row < bw; ++row)
                for (int u = 0; u < bw; ++u)
                    a.col[base + (int64_t)row * bw * cnt + (int64_t)j * bw + u] = bw * f + u;
        }
    }
}

// values of the row block of every Omega element
struct DgRowArgs {
    int64_t K;
    const int64_t *dptr;
    const int64_t *sptr;
    const int32_t *snbr;
    const uint8_t *sflag;
    const int32_t *srec;
    const void *far_rec;
    int64_t n_far;     // records (Rec layout)
    const double *dsum;      // [K][6 NK]
    const double *touch_rec;
    int32_t touch_stride;
    double *val;
    SpecGate gate;
    // label-dependent kernel: the columns of the element holding x are scaled
    // by c[m(x's element)][m(y's element)] (far blocks (e, f): c[m(f)][m(e)];
    // e's own block: the diagonal sums carry c[m(e)][m(f)] already)
    MatArgs mat;
};

template <int NC, typename TR>
__global__ void __launch_bounds__(64) k_dg_rows(DgRowArgs a)
{
    constexpr int NK = NC == 1 ? 1 : 3;
    constexpr int BW = 3 * NC;
    if (gated(a.gate)) return;
    const int lane = threadIdx.x;
    for (int64_t b = blockIdx.x; b < xcd_span(a.K); b += gridDim.x) {
        const int64_t e = xcd_item(b, a.K);
        if (e >= a.K) continue;
        const int64_t cnt = a.dptr[e + 1] - a.dptr[e];
        if (cnt == 0) continue;
        const DgRow rr = dg_row(a.sptr, a.snbr, e);
        const int64_t base = (int64_t)BW * BW * a.dptr[e];
        // e's own block also takes the (e, e) part of every edge and vertex
        // touching pair: summed over the wave, added by the lane owning e
        double self[BW][BW];
#pragma unroll
        for (int r = 0; r < BW; ++r)
#pragma unroll
            for (int s = 0; s < BW; ++s) self[r][s] = 0.0;
        for (int64_t t = rr.s0 + lane; t < rr.s0 + rr.n; t += 64) {
            const int cls = (a.sflag[t] >> 2) & 3;
            const int32_t u = a.srec[t];
            if (cls == 0 || cls == 3 || u < 0) continue;
            const double *L = a.touch_rec + (int64_t)u * a.touch_stride;
            const int oe = (int32_t)e < a.snbr[t] ? 0 : BW;
            const double w = a.mat.n == 0 ? 2.0 : 2.0 * a.mat.coef((int32_t)e, a.snbr[t]);
#pragma unroll
            for (int r = 0; r < BW; ++r)
#pragma unroll
                for (int s = 0; s < BW; ++s) self[r][s] += w * L[sym_index(oe + r, oe + s, 2 * BW)];
        }
#pragma unroll
        for (int r = 0; r < BW; ++r)
#pragma unroll
            for (int s = 0; s < BW; ++s) {
                double v = self[r][s];
                for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
                self[r][s] = v;
            }
        for (int j = lane; j < (int)cnt; j += 64) {
            int64_t t;
            const int32_t f = dg_entry(rr, a.snbr, e, j, &t);
            double blk[BW][BW];
#pragma unroll
            for (int r = 0; r < BW; ++r)
#pragma unroll
                for (int s = 0; s < BW; ++s) blk[r][s] = 0.0;
            const int cls = t >= 0 ? (a.sflag[t] >> 2) & 3 : 0;
            const int32_t u = t >= 0 ? a.srec[t] : -1;
            if (f == (int32_t)e) {
#pragma unroll
                for (int r = 0; r < BW; ++r)
#pragma unroll
                    for (int s = 0; s < BW; ++s) blk[r][s] = self[r][s];
                // summed diagonal blocks of the far pairs
                const double *ds = a.dsum + e * 6 * NK;
#pragma unroll
                for (int p = 0; p < 3; ++p)
#pragma unroll
                    for (int q = 0; q < 3; ++q)
#pragma unroll
                        for (int c = 0; c < NC; ++c)
#pragma unroll
                            for (int d = 0; d < NC; ++d)
                                blk[NC * p + c][NC * q + d] += ds[sym_index(p, q, 3) * NK + (NC == 1 ? 0 : c + d)];
            }
            // coefficient of the columns of f (f holds x): c[m(f)][m(e)]
            const double cfe = a.mat.n == 0 ? 1.0 : a.mat.coef(f, (int32_t)e);
            if (u >= 0 && cls == 0) {
                // far record: rows of e are the rows of X (e first) or its
                // columns (f first); the self pair stores X + X^T
#pragma unroll
                for (int p = 0; p < 3; ++p) {
                    const TR *rec = (const TR *)a.far_rec + (f >= (int32_t)e ? Rec<NK>::r(p, u, a.n_far)
                                                                               : Rec<NK>::c(p, u, a.n_far));
#pragma unroll
                    for (int q = 0; q < 3; ++q)
#pragma unroll
                        for (int c = 0; c < NC; ++c)
#pragma unroll
                            for (int d = 0; d < NC; ++d)
                                blk[NC * p + c][NC * q + d] += cfe * (double)rec[q * NK + (NC == 1 ? 0 : c + d)];
                }
            } else if (u >= 0) {
                const double *L = a.touch_rec + (int64_t)u * a.touch_stride;
                if (cls == 3) {
                    // identical: the local matrix over e's unknowns, once
#pragma unroll
                    for (int r = 0; r < BW; ++r)
#pragma unroll
                        for (int s = 0; s < BW; ++s) blk[r][s] += cfe * L[sym_index(r, s, BW)];
                } else {
                    // edge / vertex: [first element | second element] unknowns;
                    // both ordered pairs give the same matrix
                    const int oe = (int32_t)e < f ? 0 : BW, of = (int32_t)e < f ? BW : 0;
#pragma unroll
                    for (int r = 0; r < BW; ++r)
#pragma unroll
                        for (int s = 0; s < BW; ++s) blk[r][s] += 2.0 * cfe * L[sym_index(oe + r, of + s, 2 * BW)];
                }
            }
#pragma unroll
            for (int r = 0; r < BW; ++r)
#pragma unroll
                for (int s = 0; s < BW; ++s) a.val[base + (int64_t)r * BW * cnt + (int64_t)j * BW + s] = blk[r][s];
        }
    }
}

// 4D regularising transforms of edge (CLS 2) and vertex (CLS 1) pairs with
// discontinuous basis functions: one wave per unordered pair e < f
struct DgTouchArgs {
    int64_t n;
    const int32_t *te, *tf;
    const int32_t *E;
    const double *V;
    double *rec;
    int32_t stride;
    double c;
    SpecGate gate;
};

// frame of element k for the pair (the continuous path's vertex orders) and
// the stored position of each frame vertex
__device__ inline void dg_frame(int cls, const int32_t *ek, const int32_t *el, int32_t fr[3], int slot[3])
{
    if (cls == 2) {
        int32_t sh0 = -1, sh1 = -1, third = -1;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const bool in = ek[a] == el[0] || ek[a] == el[1] || ek[a] == el[2];
            if (!in) third = ek[a];
            else if (sh0 < 0) sh0 = ek[a];
            else sh1 = ek[a];
        }
        fr[0] = min(sh0, sh1);
        fr[1] = max(sh0, sh1);
        fr[2] = third;
    } else {
        int ia = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (ek[a] == el[0] || ek[a] == el[1] || ek[a] == el[2]) ia = a;
        fr[0] = ek[ia];
        fr[1] = ek[ia == 2 ? 0 : ia + 1];
        fr[2] = ek[ia == 0 ? 2 : ia - 1];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) slot[a] = ek[0] == fr[a] ? 0 : ek[1] == fr[a] ? 1 : 2;
}

template <int KER, int CLS>
__global__ void __launch_bounds__(64) k_touch_dg(DgTouchArgs a, GaussArgs g)
{
    constexpr int NC = Ker<KER>::NC;
    constexpr int D = 6 * NC;
    constexpr int NL = D * (D + 1) / 2;
    if (gated(a.gate)) return;
    const int lane = threadIdx.x;
    const int n = g.n;
    const int n4 = n * n * n * n;
    for (int64_t pr = blockIdx.x; pr < a.n; pr += gridDim.x) {
        const int32_t e = a.te[pr], f = a.tf[pr];
        const int32_t ek[3] = {a.E[3 * (int64_t)e], a.E[3 * (int64_t)e + 1], a.E[3 * (int64_t)e + 2]};
        const int32_t el[3] = {a.E[3 * (int64_t)f], a.E[3 * (int64_t)f + 1], a.E[3 * (int64_t)f + 2]};
        int32_t fk[3], fl[3];
        int sk[3], sl[3];
        dg_frame(CLS, ek, el, fk, sk);
        dg_frame(CLS, el, ek, fl, sl);
        const double2 k0 = vtx(a.V, fk[0]), k1 = vtx(a.V, fk[1]), k2 = vtx(a.V, fk[2]);
        const double2 l0 = vtx(a.V, fl[0]), l1 = vtx(a.V, fl[1]), l2 = vtx(a.V, fl[2]);
        const double Jk00 = k1.x - k0.x, Jk01 = k2.x - k0.x, Jk10 = k1.y - k0.y, Jk11 = k2.y - k0.y;
        const double Jl00 = l1.x - l0.x, Jl01 = l2.x - l0.x, Jl10 = l1.y - l0.y, Jl11 = l2.y - l0.y;
        const double dk = fabs(Jk00 * Jk11 - Jk01 * Jk10), dl = fabs(Jl00 * Jl11 - Jl01 * Jl10);
        double L[NL];
#pragma unroll
        for (int i = 0; i < NL; ++i) L[i] = 0.0;
        // the piece (edge face, vertex region) is a compile-time index and
        // the lanes share the n^4 points of each piece; the frame and the
        // face selection avoid lane-dependent indexing, which gave wrong
        // values here
#pragma unroll
        for (int piece = 0; piece < (CLS == 2 ? 4 : 2); ++piece) {
            for (int sidx = lane; sidx < n4; sidx += 64) {
                const int i3 = sidx % n, i2 = (sidx / n) % n, i1 = (sidx / (n * n)) % n, i0 = sidx / (n * n * n);
                const double t0 = g.x[i0], t1 = g.x[i1], t2 = g.x[i2], t3 = g.x[i3];
                double xi0, xi1, et0, et1, jac;
                if (CLS == 2) {
                    const double rho = t0, p = t1, q = t2, tau = t3;
                    const double u = 1.0 - p;
                    const double w0 = piece < 2 ? p : -p;
                    const double w1 = piece == 0 ? u : piece == 1 ? u * q : piece == 2 ? 1.0 : q;
                    const double w2 = piece == 0 ? q : piece == 1 ? 1.0 : piece == 2 ? u * q : u;
                    const double jf = piece == 1 || piece == 2 ? u : 1.0;
                    const double v0 = rho * w0, v1 = rho * w1, v2 = rho * w2;
                    xi0 = (piece < 2 ? v0 : 0.0) + (1.0 - rho) * tau;
                    xi1 = v1;
                    et0 = xi0 - v0;
                    et1 = v2;
                    jac = rho * rho * (1.0 - rho) * jf;
                } else {
                    const double gg = t0, w = t1, al = t2, be = t3;
                    const double s = piece == 0 ? gg : gg * w, tt = piece == 0 ? gg * w : gg;
                    xi0 = s * (1.0 - al);
                    xi1 = s * al;
                    et0 = tt * (1.0 - be);
                    et1 = tt * be;
                    jac = gg * gg * gg * w;
                }
                const double wt = g.w[i0] * g.w[i1] * g.w[i2] * g.w[i3] * jac * dk * dl;
                const double xx = k0.x + (Jk00 * xi0 + Jk01 * xi1), xy = k0.y + (Jk10 * xi0 + Jk11 * xi1);
                const double yx = l0.x + (Jl00 * et0 + Jl01 * et1), yy = l0.y + (Jl10 * et0 + Jl11 * et1);
                double kv[3];
                kernel_eval<KER, double>(xx - yx, xy - yy, a.c, kv);
                // basis differences over [e's stored unknowns | f's stored unknowns]
                double av[6];
                const double pk[3] = {1.0 - xi0 - xi1, xi0, xi1}, pl[3] = {1.0 - et0 - et1, et0, et1};
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    av[sk[q]] = pk[q];
                    av[3 + sl[q]] = -pl[q];
                }
#pragma unroll
                for (int r2 = 0; r2 < D; ++r2)
#pragma unroll
                    for (int s2 = r2; s2 < D; ++s2) {
                        const int c = r2 % NC, d = s2 % NC;
                        const double kk = NC == 1 ? kv[0] : kv[c + d];
                        L[sym_index(r2, s2, D)] += wt * kk * av[r2 / NC] * av[s2 / NC];
                    }
            }
        }
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            double v = L[i];
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
            L[i] = v;
        }
        if (lane == 0)
            for (int i = 0; i < NL; ++i) a.rec[pr * a.stride + i] = L[i];
    }
}

template <int KER>
void touch_dg_launch(const DgTouchArgs &ae, const DgTouchArgs &av, const GaussArgs &g, hipStream_t s)
{
    if (ae.n > 0)
        hipLaunchKernelGGL((k_touch_dg<KER, 2>), dim3((unsigned)std::min<int64_t>(ae.n, 1 << 20)), dim3(64), 0, s,
                           ae, g);
    if (av.n > 0)
        hipLaunchKernelGGL((k_touch_dg<KER, 1>), dim3((unsigned)std::min<int64_t>(av.n, 1 << 20)), dim3(64), 0, s,
                           av, g);
}

}  // namespace

int launch_dg_counts(nlfem_pairs *h, hipStream_t s)
{
    DgCountArgs a{h->K, h->mesh_labels, h->loff + (int64_t)kLsS * (h->K + 1), h->snbr, h->dg_cnt,
                  h->red + kRedDgDofs};
    hipLaunchKernelGGL(k_dg_counts, dim3(grid_for(h->K, 256)), dim3(256), 0, s, a);
    NLFEM_HIP(hipGetLastError());
    return NLFEM_OK;
}

int launch_dg_pattern(const nlfem_pairs *h, int64_t *row_ptr, int32_t *col, hipStream_t s)
{
    DgPatternArgs a{h->K, h->ncomp, h->dg_ptr, h->loff + (int64_t)kLsS * (h->K + 1), h->snbr, h->mesh_labels,
                    row_ptr, col};
    const int64_t nrow = 3 * (int64_t)h->ncomp * h->K;
    hipLaunchKernelGGL(k_dg_row_ptr, dim3(grid_for(nrow + 1, 256)), dim3(256), 0, s, a);
    if (h->nnz_node > 0)
        hipLaunchKernelGGL(k_dg_cols, dim3((unsigned)std::min<int64_t>(h->K, 1 << 20)), dim3(64), 0, s, a);
    NLFEM_HIP(hipGetLastError());
    return NLFEM_OK;
}

int launch_dg_assemble_rest(const nlfem_pairs *h, const nlfem_mesh *m, const nlfem_config *cfg, const GaussArgs &g,
                            double *val, hipStream_t s)
{
    // edge and vertex touching records (the identical ones come from the
    // continuous path's launch)
    const int64_t nI = h->nUTc[0], nE = h->nUTc[1], nV = h->nUTc[2];
    DgTouchArgs ae{nE, h->te + nI, h->tf + nI, m->elements, m->vertices, h->touch_rec + nI * h->touch_stride,
                   h->touch_stride, cfg->c, h->asm_gate};
    DgTouchArgs av{nV, h->te + nI + nE, h->tf + nI + nE, m->elements, m->vertices,
                   h->touch_rec + (nI + nE) * h->touch_stride, h->touch_stride, cfg->c, h->asm_gate};
    if (nE + nV > 0) {
        timing_begin(kPhTouch, s);
        switch (h->kernel) {
        case NLFEM_K_CONSTANT: touch_dg_launch<NLFEM_K_CONSTANT>(ae, av, g, s); break;
        case NLFEM_K_INV_DIST: touch_dg_launch<NLFEM_K_INV_DIST>(ae, av, g, s); break;
        case NLFEM_K_FRAC_HALF: touch_dg_launch<NLFEM_K_FRAC_HALF>(ae, av, g, s); break;
        default: touch_dg_launch<NLFEM_K_PERIDYNAMIC>(ae, av, g, s); break;
        }
        timing_end(kPhTouch, s);
    }
    return NLFEM_OK;
}

int launch_dg_rows(const nlfem_pairs *h, const nlfem_mesh *m, const nlfem_config *cfg, double *val, hipStream_t s)
{
    if (h->nnz_node == 0) return NLFEM_OK;
    DgRowArgs a{h->K,           h->dg_ptr,        h->loff + (int64_t)kLsS * (h->K + 1), h->snbr, h->sflag,
                h->srec,        h->far_rec,       h->nUF, h->dsum, h->touch_rec, h->touch_stride, val,
                h->asm_gate,    material_args(m->materials, cfg)};
    const unsigned grid = xcd_grid(h->K);
    const bool fp32 = cfg->precision == NLFEM_P_MIXED;
    timing_begin(kPhRows, s);
    if (h->ncomp == 1) {
        if (fp32) hipLaunchKernelGGL((k_dg_rows<1, float>), dim3(grid), dim3(64), 0, s, a);
        else hipLaunchKernelGGL((k_dg_rows<1, double>), dim3(grid), dim3(64), 0, s, a);
    } else {
        if (fp32) hipLaunchKernelGGL((k_dg_rows<2, float>), dim3(grid), dim3(64), 0, s, a);
        else hipLaunchKernelGGL((k_dg_rows<2, double>), dim3(grid), dim3(64), 0, s, a);
    }
    timing_end(kPhRows, s);
    NLFEM_HIP(hipGetLastError());
    return NLFEM_OK;
}

}  // namespace nlfem

// Stiffness-matrix values of one problem: the per-item functions of
// assemble_items.h launched over the handle's work lists.
#include "assemble_items.h"

namespace nlfem {
using namespace items;
namespace {

// record staging through LDS (coalesced stores) where it fits: all but the
// two-component FP64 records (28 KB per wave)
template <int KER, typename T>
constexpr bool far_staged() { return !(Ker<KER>::NK == 3 && sizeof(T) == 8); }

// thread per record; consecutive lanes hold consecutive records
template <int KER, typename T, int PM, bool POLY>
__global__ void __launch_bounds__(256) k_far_rec(FarArgs a, RoleArgs r1, RoleArgs r2)
{
    if (gated(a.gate)) return;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!far_staged<KER, T>() || POLY) {
        if (idx >= a.n) return;
        far_item<KER, T, PM, POLY>(a, r1, r2, idx);
        return;
    }
    constexpr int NV = kFarStage<Ker<KER>::NK>;
    __shared__ T slots[far_staged<KER, T>() ? 4 * 64 * NV : 1];
    const int64_t idx0 = idx - (threadIdx.x & 63);
    if (idx0 >= a.n) return;   // whole waves leave together
    const int nvalid = (int)min((int64_t)64, a.n - idx0);
    FarAcc<KER, T> acc;
    bool self = false;
    if (idx < a.n) {
        const int32_t e = a.ue[idx], f = a.uf[idx];
        self = e == f;
        const uint2 mm = a.m[idx];
        far_whole<KER, T, PM>(a, r1, r2, e, f, mm.x, mm.y, acc);
    }
    far_store_wave<KER, T>(a, idx0, nvalid, self, acc, slots + (threadIdx.x >> 6) * 64 * NV);
}

// polygon ball: one wave per workgroup shares the straddling points of its pairs
template <int KER, typename T, int PM>
__global__ void __launch_bounds__(64) k_far_rec_poly(FarArgs a, RoleArgs r1, RoleArgs r2)
{
    constexpr int NV = 21 * Ker<KER>::NK;
    __shared__ int32_t queue[64 * 2 * kMaxRule];
    __shared__ int32_t pe[64], pf[64];
    __shared__ T slots[64 * NV];
    __shared__ double sdir[2 * kMaxPoly];
    if (gated(a.gate)) return;
    // the polygon directions in LDS: every clip pass reads them
    for (int t = threadIdx.x; t < 2 * a.N; t += 64) sdir[t] = a.dir[t];
    wave_sync();
    FarArgs al = a;
    al.dir = sdir;
    const int64_t idx = (int64_t)blockIdx.x * 64 + threadIdx.x;
    far_wave_poly<KER, T, PM>(al, r1, r2, idx, idx < a.n, queue, pe, pf, slots);
}

// the three classes in one launch: blocks [0, nb[0]) take the vertex class
// (the longest items first), then edge, then identical
struct TouchLaunch {
    TouchArgs t[3];   // identical, edge, vertex
    int64_t nb[3];    // blocks of the vertex, edge and identical classes
    SpecGate gate;
};

template <int KER, int CLS>
__device__ __forceinline__ void touch_block(const TouchArgs &a, const GaussView &g, int64_t b)
{
    constexpr int G = touch_lanes(CLS);
    const int64_t gid = b * 256 + threadIdx.x;
    const int64_t pair = gid / G;
    if (pair >= a.n) return;   // whole groups leave together
    touch_item<KER, CLS, G>(a, g, pair, (int)(gid % G));
}

template <int KER>
__global__ void __launch_bounds__(256) k_touch_rec(TouchLaunch L, GaussArgs g)
{
    if (gated(L.gate)) return;
    // the rule in LDS: the point loops read it at every step
    __shared__ double gs[2 * kMaxGauss];
    if (threadIdx.x < 2 * kMaxGauss)
        gs[threadIdx.x] = threadIdx.x < kMaxGauss ? g.x[threadIdx.x] : g.w[threadIdx.x - kMaxGauss];
    __syncthreads();
    const GaussView gv{gs, gs + kMaxGauss, g.n};
    int64_t b = blockIdx.x;
    if (b < L.nb[0]) {
        touch_block<KER, 1>(L.t[2], gv, b);
        return;
    }
    b -= L.nb[0];
    if (b < L.nb[1]) {
        touch_block<KER, 2>(L.t[1], gv, b);
        return;
    }
    touch_block<KER, 3>(L.t[0], gv, b - L.nb[1]);
}

template <int NK, typename TR, bool MOM = false>
__global__ void __launch_bounds__(256) k_elem_diag(DiagArgs a)
{
    if (gated(a.gate)) return;
    constexpr int G = diag_group<MOM>();
    constexpr int per = 256 / G;   // elements per workgroup
    const int64_t e = xcd_item(blockIdx.x, (a.K + per - 1) / per) * per + threadIdx.x / G;
    if (e >= a.K) return;   // whole lane groups leave together
    diag_item<NK, TR, MOM>(a, e, threadIdx.x % G);
}

template <int NC, typename TR, bool MOM = false>
__global__ void __launch_bounds__(64) k_rows(RowArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ RowShared sh;
    __shared__ double mq[MOM ? kRowMom : 1];
    if (gated(a.gate)) return;
    for (int64_t b = blockIdx.x; b < xcd_span(a.nrows); b += gridDim.x) {
        const int64_t item = xcd_item(b, a.nrows);
        if (item >= a.nrows) continue;
        row_item<NC, TR, MOM>(a, a.rows[item], smem, sh, mq);
    }
}

// ------------------------------------------------------------ launching

template <int KER, typename T, bool POLY>
void far_launch(const FarArgs &a, const RoleArgs &r1, const RoleArgs &r2, bool seven, hipStream_t s)
{
    if (POLY) {
        const unsigned grid = grid_for(a.n, 64);
        if (seven) hipLaunchKernelGGL((k_far_rec_poly<KER, T, 7>), dim3(grid), dim3(64), 0, s, a, r1, r2);
        else hipLaunchKernelGGL((k_far_rec_poly<KER, T, 0>), dim3(grid), dim3(64), 0, s, a, r1, r2);
        return;
    }
    const unsigned grid = grid_for(a.n, 256);
    if (seven) hipLaunchKernelGGL((k_far_rec<KER, T, 7, POLY>), dim3(grid), dim3(256), 0, s, a, r1, r2);
    else hipLaunchKernelGGL((k_far_rec<KER, T, 0, POLY>), dim3(grid), dim3(256), 0, s, a, r1, r2);
}

template <int KER>
void far_dispatch(const AssemblePlan &p, hipStream_t s)
{
    if (p.poly) {
        if (p.fp32) far_launch<KER, float, true>(p.far, p.r1, p.r2, p.seven, s);
        else far_launch<KER, double, true>(p.far, p.r1, p.r2, p.seven, s);
    } else {
        if (p.fp32) far_launch<KER, float, false>(p.far, p.r1, p.r2, p.seven, s);
        else far_launch<KER, double, false>(p.far, p.r1, p.r2, p.seven, s);
    }
}

template <int KER>
void touch_dispatch(const AssemblePlan &p, hipStream_t s)
{
    TouchLaunch L{};
    for (int c = 0; c < 3; ++c) L.t[c] = p.touch[c];
    L.gate = p.far.gate;
    L.nb[0] = (p.touch[2].n * touch_lanes(1) + 255) / 256;
    L.nb[1] = (p.touch[1].n * touch_lanes(2) + 255) / 256;
    L.nb[2] = (p.touch[0].n * touch_lanes(3) + 255) / 256;
    const int64_t blocks = L.nb[0] + L.nb[1] + L.nb[2];
    if (blocks > 0) hipLaunchKernelGGL((k_touch_rec<KER>), dim3((unsigned)blocks), dim3(256), 0, s, L, p.gauss);
}

}  // namespace

namespace items {

RoleArgs roles(const RuleArgs &r, bool a_outer, bool b_outer)
{
    RoleArgs o{};
    o.PA = a_outer ? r.P : r.Q;
    o.PB = b_outer ? r.P : r.Q;
    for (int p = 0; p < kMaxRule; ++p) {
        for (int c = 0; c < 2; ++c) {
            o.xa[p][c] = a_outer ? r.pxi[p][c] : r.qxi[p][c];
            o.xb[p][c] = b_outer ? r.pxi[p][c] : r.qxi[p][c];
        }
        o.wa[p] = a_outer ? r.pw[p] : r.qw[p];
        o.wb[p] = b_outer ? r.pw[p] : r.qw[p];
        for (int c = 0; c < 3; ++c) {
            o.pa[p][c] = a_outer ? r.pphi[p][c] : r.qphi[p][c];
            o.pb[p][c] = b_outer ? r.pphi[p][c] : r.qphi[p][c];
        }
    }
    return o;
}

MomArgs moment_args(const nlfem_pairs *h, const nlfem_config *cfg)
{
    MomArgs m;
    if (cfg->kernel != NLFEM_K_CONSTANT || h->approach != NLFEM_A_NOCAPS_BARY || h->ncomp != 1 || h->dg ||
        h->rules.P > kMomP)
        return m;
    const RuleArgs &r = h->rules;
    m.on = 1;
    m.P = r.P;
    m.m = h->um;
    m.det = h->det;
    m.c = cfg->c;
    for (int p = 0; p < r.P; ++p) {
        m.wo[p] = r.pw[p];
        for (int a = 0; a < 3; ++a) {
            m.mo[p][a] = r.pw[p] * r.pphi[p][a];
            for (int b = a; b < 3; ++b) m.qo[p][sym_index(a, b, 3)] = r.pw[p] * r.pphi[p][a] * r.pphi[p][b];
        }
    }
    for (int q = 0; q < r.Q; ++q) {
        m.wi += r.qw[q];
        for (int a = 0; a < 3; ++a) {
            m.mi[a] += r.qw[q] * r.qphi[q][a];
            for (int b = a; b < 3; ++b) m.qi[sym_index(a, b, 3)] += r.qw[q] * r.qphi[q][a] * r.qphi[q][b];
        }
    }
    return m;
}

AssemblePlan make_plan(const nlfem_pairs *h, const nlfem_mesh *m, const nlfem_config *cfg, const GaussArgs &g,
                       double *val)
{
    AssemblePlan p{};
    p.kernel = kernel_variant(cfg);
    p.nc = h->ncomp;
    p.fp32 = cfg->precision == NLFEM_P_MIXED;
    p.poly = clipped_ball(h->approach);
    p.gauss = g;
    // far records
    FarArgs &a = p.far;
    a.n = h->nUF;
    a.ue = h->ue;
    a.uf = h->uf;
    a.m = h->um;
    a.v0 = h->v0;
    a.J = h->J;
    a.det = h->det;
    a.rec = h->far_rec;
    a.stride = h->far_stride;
    a.c = cfg->c;
    a.same = h->rules.same;
    a.xp = h->xp;
    a.P = h->rules.P;
    a.E = m->elements;
    a.V = m->vertices;
    a.dir = h->poly_dir;
    a.N = h->poly.N;
    a.caps = caps_mode(h->approach);
    a.delta = h->delta;
    a.cap = kMaxPoly + 4;
    a.err = h->err;
    a.gate = h->asm_gate;
    // same rules: one pass, A and B both the outer rule.  Otherwise pass 1
    // (outer on e, inner on f) and pass 2 (inner on e, outer on f).
    p.r1 = roles(h->rules, true, h->rules.same ? true : false);
    p.r2 = roles(h->rules, false, true);
    p.seven = p.r1.PA == 7 && p.r1.PB == 7 && (a.same || (p.r2.PA == 7 && p.r2.PB == 7));
    // touching records by class: [ident | edge | vertex]
    int64_t off = 0;
    for (int c = 0; c < 3; ++c) {
        TouchArgs &t = p.touch[c];
        t.n = h->nUTc[c];
        t.te = h->te + off;
        t.tf = h->tf + off;
        t.E = m->elements;
        t.V = m->vertices;
        t.rec = h->touch_rec + off * h->touch_stride;
        t.stride = h->touch_stride;
        t.c = cfg->c;
        off += h->nUTc[c];
    }
    // rows
    RowArgs &r = p.rows;
    r.nrows = h->nnz_node > 0 ? h->n_dof : 0;
    r.rows = h->dof_list;
    r.nptr = h->nptr;
    r.ncol = h->ncol;
    r.ne_ptr = h->ne_ptr;
    r.ne_list = h->ne_list;
    r.E = m->elements;
    r.sptr = h->loff + (int64_t)kLsS * (h->K + 1);
    r.snode = h->snode;
    r.sflag = h->sflag;
    r.srec = h->srec;
    r.far_rec = h->far_rec;
    r.far_stride = h->far_stride;
    r.n_far = h->nUF;
    r.dsum = h->dsum;
    r.touch_rec = h->touch_rec;
    r.touch_stride = h->touch_stride;
    r.n_touch = h->nUT;
    int hc = 64;
    while (hc < 2 * h->max_row) hc <<= 1;
    r.hcap = hc;
    r.maxlen = (int32_t)h->max_row;
    r.val = val;
    r.err = h->err;
    r.gate = h->asm_gate;
    r.mat = material_args(m->materials, cfg);
    r.nonsym = h->nonsym;
    r.mom = moment_args(h, cfg);
    p.diag = DiagArgs{h->K,        r.sptr,   h->snbr, h->sflag, h->srec, h->far_rec, h->far_stride,
                      h->nUF,      h->dsum,  h->err,  h->asm_gate, r.mat, r.mom};
    // the moment form needs no far records
    p.mom = r.mom.on != 0;
    return p;
}

}  // namespace items

namespace items {

void launch_phase(const AssemblePlan &p, int phase, hipStream_t s)
{
    switch (phase) {
    case 0:   // non-touching pairs
        if (p.far.n == 0 || p.mom) return;
        switch (p.kernel) {
        case NLFEM_K_CONSTANT: far_dispatch<NLFEM_K_CONSTANT>(p, s); break;
        case NLFEM_K_INV_DIST: far_dispatch<NLFEM_K_INV_DIST>(p, s); break;
        case NLFEM_K_FRAC_HALF: far_dispatch<NLFEM_K_FRAC_HALF>(p, s); break;
        case NLFEM_K_INV_DIST | kKerNoZeroDiv: far_dispatch<NLFEM_K_INV_DIST | kKerNoZeroDiv>(p, s); break;
        case NLFEM_K_PERIDYNAMIC | kKerNoZeroDiv:
            far_dispatch<NLFEM_K_PERIDYNAMIC | kKerNoZeroDiv>(p, s);
            break;
        default: far_dispatch<NLFEM_K_PERIDYNAMIC>(p, s); break;
        }
        return;
    case 1:   // touching pairs (all classes present in the plan)
        switch (p.kernel) {
        case NLFEM_K_CONSTANT: touch_dispatch<NLFEM_K_CONSTANT>(p, s); break;
        case NLFEM_K_INV_DIST: touch_dispatch<NLFEM_K_INV_DIST>(p, s); break;
        case NLFEM_K_FRAC_HALF: touch_dispatch<NLFEM_K_FRAC_HALF>(p, s); break;
        default: touch_dispatch<NLFEM_K_PERIDYNAMIC>(p, s); break;
        }
        return;
    case 2: {   // element-diagonal sums
        if (p.rows.nrows == 0) return;
        const int per = 256 / (p.mom ? diag_group<true>() : diag_group<false>());
        const unsigned dg = xcd_grid((p.diag.K + per - 1) / per, INT32_MAX);
        if (p.nc == 1 && p.mom) {
            if (p.fp32) hipLaunchKernelGGL((k_elem_diag<1, float, true>), dim3(dg), dim3(256), 0, s, p.diag);
            else hipLaunchKernelGGL((k_elem_diag<1, double, true>), dim3(dg), dim3(256), 0, s, p.diag);
        } else if (p.nc == 1) {
            if (p.fp32) hipLaunchKernelGGL((k_elem_diag<1, float>), dim3(dg), dim3(256), 0, s, p.diag);
            else hipLaunchKernelGGL((k_elem_diag<1, double>), dim3(dg), dim3(256), 0, s, p.diag);
        } else {
            if (p.fp32) hipLaunchKernelGGL((k_elem_diag<3, float>), dim3(dg), dim3(256), 0, s, p.diag);
            else hipLaunchKernelGGL((k_elem_diag<3, double>), dim3(dg), dim3(256), 0, s, p.diag);
        }
        return;
    }
    default: {   // row gather (continuous ansatz)
        if (p.rows.nrows == 0) return;
        const size_t lds = row_lds_bytes(p.rows.maxlen, p.nc, p.rows.hcap);
        const unsigned grid = xcd_grid(p.rows.nrows);
        if (p.nc == 1 && p.mom) {
            if (p.fp32) hipLaunchKernelGGL((k_rows<1, float, true>), dim3(grid), dim3(64), lds, s, p.rows);
            else hipLaunchKernelGGL((k_rows<1, double, true>), dim3(grid), dim3(64), lds, s, p.rows);
        } else if (p.nc == 1) {
            if (p.fp32) hipLaunchKernelGGL((k_rows<1, float>), dim3(grid), dim3(64), lds, s, p.rows);
            else hipLaunchKernelGGL((k_rows<1, double>), dim3(grid), dim3(64), lds, s, p.rows);
        } else {
            if (p.fp32) hipLaunchKernelGGL((k_rows<2, float>), dim3(grid), dim3(64), lds, s, p.rows);
            else hipLaunchKernelGGL((k_rows<2, double>), dim3(grid), dim3(64), lds, s, p.rows);
        }
    }
    }
}

}  // namespace items

int far_record_stride(int ncomp) { return ncomp == 1 ? Rec<1>::kValues : Rec<3>::kValues; }
// packed symmetric local matrices over the union of the pair's unknowns:
// at most 5 nodes (continuous) or 6 unknowns (discontinuous) per component
int touch_record_stride(int ncomp, bool dg)
{
    const int d = (dg ? 6 : 5) * ncomp;
    return d * (d + 1) / 2;
}

int launch_assemble(const nlfem_pairs *h, const nlfem_mesh *m, const nlfem_config *cfg, const GaussArgs &g,
                    double *val, hipStream_t s)
{
    AssemblePlan p = make_plan(h, m, cfg, g, val);
    if (h->dg || h->nonsym) {
        // discontinuous ansatz or non-symmetric material table: the identical
        // pairs by the reduced transforms here, edge and vertex pairs by the
        // 4D transforms of dg.hip
        p.touch[1].n = 0;
        p.touch[2].n = 0;
        NLFEM_TRY(launch_dg_assemble_rest(h, m, cfg, g, val, s));
    }
    const bool has_touch = p.touch[0].n + p.touch[1].n + p.touch[2].n > 0;
    // one stream: a second stream for the touching pairs costs more in the
    // two cross-queue waits than their overlap with the far records gains
    if (has_touch) {
        timing_begin(kPhTouch, s);
        items::launch_phase(p, 1, s);
        timing_end(kPhTouch, s);
    }
    if (p.far.n > 0 && !p.mom) {
        timing_begin(kPhFar, s);
        items::launch_phase(p, 0, s);
        timing_end(kPhFar, s);
    }
    if (p.rows.nrows > 0) {
        timing_begin(kPhDiag, s);
        items::launch_phase(p, 2, s);
        timing_end(kPhDiag, s);
        if (h->dg) return launch_dg_rows(h, m, cfg, val, s);
        timing_begin(kPhRows, s);
        items::launch_phase(p, 3, s);
        timing_end(kPhRows, s);
    }
    NLFEM_HIP(hipGetLastError());
    return NLFEM_OK;
}

}  // namespace nlfem

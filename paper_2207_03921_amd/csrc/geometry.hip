// Element geometry (pull-back to the reference triangle, Sec. 2.4), node
// labels and node->element incidence.
//
// Every quantity that takes part in an inclusion decision (barycentres and
// outer quadrature points) is computed in FP64 without contraction, in the
// fixed order x_p = v0 + (J00 xi_1 + J01 xi_2, J10 xi_1 + J11 xi_2),
// bary = ((v0 + v1) + v2) / 3, so that the decisions are reproducible
// bit for bit by any plain FP64 implementation.
#include <cstring>

#include "nlfem_internal.h"

#pragma clang fp contract(off)

namespace nlfem {
namespace {

// order-preserving map of a double onto unsigned keys (for atomic min/max)
__device__ inline unsigned long long dkey(double v)
{
    unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}

__device__ inline double wave_min(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
__device__ inline double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

struct GeoArgs {
    int64_t K, M;
    const double *V;
    const int32_t *E;
    const int32_t *lab;
    double2 *v0;
    double4 *J;
    double *det;
    double2 *bary;
    double2 *xp;
    uint32_t *node_flags;
    int32_t *err;
    unsigned long long *red;
    const int32_t *mat;   // material ids, checked against nmat when a table is given
    int32_t nmat;
};

__global__ void __launch_bounds__(256) k_geometry(GeoArgs a, RuleArgs r)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double bx = 1e300, by = 1e300, Bx = -1e300, By = -1e300, rq = 0.0, rv = 0.0;
    if (k < a.K) {
        int32_t n0 = a.E[3 * k], n1 = a.E[3 * k + 1], n2 = a.E[3 * k + 2];
        int32_t lab = a.lab[k];
        bool ok = n0 >= 0 && n1 >= 0 && n2 >= 0 && n0 < a.M && n1 < a.M && n2 < a.M;
        if (!ok) {
            atomicOr(a.err, kErrIndex);
            n0 = n1 = n2 = 0;
        }
        const double v0x = a.V[2 * (int64_t)n0], v0y = a.V[2 * (int64_t)n0 + 1];
        const double v1x = a.V[2 * (int64_t)n1], v1y = a.V[2 * (int64_t)n1 + 1];
        const double v2x = a.V[2 * (int64_t)n2], v2y = a.V[2 * (int64_t)n2 + 1];
        const double J00 = v1x - v0x, J01 = v2x - v0x, J10 = v1y - v0y, J11 = v2y - v0y;
        const double d = fabs(J00 * J11 - J01 * J10);
        const bool active = lab == 1 || lab == 2;
        if (ok && active && !(d > 0.0)) atomicOr(a.err, kErrArea);
        if (active && a.nmat > 0 && (unsigned)a.mat[k] >= (unsigned)a.nmat) atomicOr(a.err, kErrMaterial);
        a.v0[k] = make_double2(v0x, v0y);
        a.J[k] = make_double4(J00, J01, J10, J11);
        a.det[k] = d;
        const double cx = ((v0x + v1x) + v2x) / 3.0;
        const double cy = ((v0y + v1y) + v2y) / 3.0;
        a.bary[k] = make_double2(cx, cy);
        for (int p = 0; p < r.P; ++p) {
            const double xx = v0x + (J00 * r.pxi[p][0] + J01 * r.pxi[p][1]);
            const double yy = v0y + (J10 * r.pxi[p][0] + J11 * r.pxi[p][1]);
            a.xp[k * r.P + p] = make_double2(xx, yy);
            if (active) rq = fmax(rq, sqrt((xx - cx) * (xx - cx) + (yy - cy) * (yy - cy)));
        }
        if (active) {
            bx = Bx = cx;
            by = By = cy;
            rv = fmax(rv, sqrt((v0x - cx) * (v0x - cx) + (v0y - cy) * (v0y - cy)));
            rv = fmax(rv, sqrt((v1x - cx) * (v1x - cx) + (v1y - cy) * (v1y - cy)));
            rv = fmax(rv, sqrt((v2x - cx) * (v2x - cx) + (v2y - cy) * (v2y - cy)));
            if (ok) {
                uint32_t fl = lab == 1 ? 1u : 2u;
                atomicOr(&a.node_flags[n0], fl);
                atomicOr(&a.node_flags[n1], fl);
                atomicOr(&a.node_flags[n2], fl);
            }
        }
    }
    // one set of atomics per workgroup (same-address atomics from every
    // wave would serialise)
    __shared__ double part[4][6];
    bx = wave_min(bx);
    by = wave_min(by);
    Bx = wave_max(Bx);
    By = wave_max(By);
    rq = wave_max(rq);
    rv = wave_max(rv);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        part[w][0] = bx;
        part[w][1] = by;
        part[w][2] = Bx;
        part[w][3] = By;
        part[w][4] = rq;
        part[w][5] = rv;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < (int)(blockDim.x >> 6); ++v) {
            bx = fmin(bx, part[v][0]);
            by = fmin(by, part[v][1]);
            Bx = fmax(Bx, part[v][2]);
            By = fmax(By, part[v][3]);
            rq = fmax(rq, part[v][4]);
            rv = fmax(rv, part[v][5]);
        }
        if (Bx >= bx) {
            atomicMin(&a.red[0], dkey(bx));
            atomicMin(&a.red[1], dkey(by));
            atomicMax(&a.red[2], dkey(Bx));
            atomicMax(&a.red[3], dkey(By));
            atomicMax(&a.red[4], dkey(rq));
            atomicMax(&a.red[5], dkey(rv));
        }
    }
}

// Clears up to kZeroMax ranges of 32-bit words in one launch; with init_red
// also starts the reduction slots (min slots at the +inf key, the rest 0).
__global__ void __launch_bounds__(256) k_zero(ZeroList z, unsigned long long *red)
{
    if (red && blockIdx.x == 0 && threadIdx.x < kRedSlots) red[threadIdx.x] = threadIdx.x < 2 ? ~0ull : 0ull;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int r = 0; r < z.cnt; ++r)
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < z.n[r]; i += stride) z.p[r][i] = 0u;
}

}  // namespace

int launch_zero(const ZeroList &z, unsigned long long *init_red, hipStream_t s)
{
    int64_t most = 1;
    for (int r = 0; r < z.cnt; ++r) most = std::max<int64_t>(most, z.n[r]);
    const unsigned grid = (unsigned)std::min<int64_t>(grid_for(most, 256), 2048);
    hipLaunchKernelGGL(k_zero, dim3(grid), dim3(256), 0, s, z, init_red);
    NLFEM_HIP(hipGetLastError());
    return NLFEM_OK;
}

double key_to_double(unsigned long long key)
{
    unsigned long long b = (key & 0x8000000000000000ull) ? (key & ~0x8000000000000000ull) : ~key;
    double v;
    memcpy(&v, &b, sizeof v);
    return v;
}

int launch_geometry(nlfem_pairs *h, const nlfem_mesh *m, hipStream_t s, const ZeroList &later)
{
    GeoArgs a{h->K,        h->M,     m->vertices, m->elements, m->labels,
              h->v0,       h->J,     h->det,      h->bary,     h->xp,
              h->node_flags, h->err, h->red,      h->materials > 0 ? m->materials : nullptr, h->materials};
    ZeroList z = later;
    z.add(h->node_flags, h->M);
    NLFEM_TRY(launch_zero(z, h->red, s));   // also clears err (a reduction slot)
    hipLaunchKernelGGL(k_geometry, dim3(grid_for(h->K, 256)), dim3(256), 0, s, a, h->rules);
    NLFEM_HIP(hipGetLastError());
    return NLFEM_OK;
}


}  // namespace nlfem

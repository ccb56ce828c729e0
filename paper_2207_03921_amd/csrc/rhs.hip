// Load vector (f, phi_i) over the Omega elements with the outer rule:
//   b_(n i + c) += |J_T| sum_p d_p f_c(x_p) phi^_(i)(xi_p).
#include "nlfem_internal.h"

namespace nlfem {
namespace {

struct RhsArgs {
    int64_t K, M;
    const double *V;
    const int32_t *E;
    const int32_t *lab;
    const double *fqp;      // [K][P][n] or null
    double aff[2][3];       // affine f when fqp is null
    int32_t ncomp;
    double *b;
};

__global__ void __launch_bounds__(256) k_rhs(RhsArgs a, RuleArgs r)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.K || a.lab[k] != 1) return;
    const int32_t n0 = a.E[3 * k], n1 = a.E[3 * k + 1], n2 = a.E[3 * k + 2];
    // an element with an index outside [0, M) is skipped (the pair build
    // reports it; this call validates no device data)
    if ((uint64_t)n0 >= (uint64_t)a.M || (uint64_t)n1 >= (uint64_t)a.M || (uint64_t)n2 >= (uint64_t)a.M) return;
    const double v0x = a.V[2 * (int64_t)n0], v0y = a.V[2 * (int64_t)n0 + 1];
    const double J00 = a.V[2 * (int64_t)n1] - v0x, J10 = a.V[2 * (int64_t)n1 + 1] - v0y;
    const double J01 = a.V[2 * (int64_t)n2] - v0x, J11 = a.V[2 * (int64_t)n2 + 1] - v0y;
    const double det = fabs(J00 * J11 - J01 * J10);
    double acc[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    for (int p = 0; p < r.P; ++p) {
        const double x = v0x + J00 * r.pxi[p][0] + J01 * r.pxi[p][1];
        const double y = v0y + J10 * r.pxi[p][0] + J11 * r.pxi[p][1];
        for (int c = 0; c < a.ncomp; ++c) {
            const double fv = a.fqp ? a.fqp[(k * r.P + p) * a.ncomp + c]
                                    : a.aff[c][0] + a.aff[c][1] * x + a.aff[c][2] * y;
            for (int i = 0; i < 3; ++i) acc[i][c] += r.pw[p] * fv * r.pphi[p][i];
        }
    }
    const int32_t nd[3] = {n0, n1, n2};
    for (int i = 0; i < 3; ++i)
        for (int c = 0; c < a.ncomp; ++c) atomicAdd(&a.b[(int64_t)a.ncomp * nd[i] + c], det * acc[i][c]);
}

// discontinuous ansatz: every element owns its entries (zero outside Omega)
__global__ void __launch_bounds__(256) k_rhs_dg(RhsArgs a, RuleArgs r)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.K) return;
    double acc[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    const int32_t n0 = a.E[3 * k], n1 = a.E[3 * k + 1], n2 = a.E[3 * k + 2];
    const bool ok = a.lab[k] == 1 && (uint64_t)n0 < (uint64_t)a.M && (uint64_t)n1 < (uint64_t)a.M &&
                    (uint64_t)n2 < (uint64_t)a.M;
    if (ok) {
        const double v0x = a.V[2 * (int64_t)n0], v0y = a.V[2 * (int64_t)n0 + 1];
        const double J00 = a.V[2 * (int64_t)n1] - v0x, J10 = a.V[2 * (int64_t)n1 + 1] - v0y;
        const double J01 = a.V[2 * (int64_t)n2] - v0x, J11 = a.V[2 * (int64_t)n2 + 1] - v0y;
        const double det = fabs(J00 * J11 - J01 * J10);
        for (int p = 0; p < r.P; ++p) {
            const double x = v0x + J00 * r.pxi[p][0] + J01 * r.pxi[p][1];
            const double y = v0y + J10 * r.pxi[p][0] + J11 * r.pxi[p][1];
            for (int c = 0; c < a.ncomp; ++c) {
                const double fv = a.fqp ? a.fqp[(k * r.P + p) * a.ncomp + c]
                                        : a.aff[c][0] + a.aff[c][1] * x + a.aff[c][2] * y;
                for (int i = 0; i < 3; ++i) acc[i][c] += r.pw[p] * fv * r.pphi[p][i];
            }
        }
        for (int i = 0; i < 3; ++i)
            for (int c = 0; c < a.ncomp; ++c) acc[i][c] *= det;
    }
    for (int i = 0; i < 3; ++i)
        for (int c = 0; c < a.ncomp; ++c) a.b[(int64_t)a.ncomp * (3 * k + i) + c] = acc[i][c];
}

__global__ void __launch_bounds__(256) k_fill0(double *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

}  // namespace

int launch_rhs(const nlfem_mesh *m, const RuleArgs &r, int ncomp, const double *f_qp, const double *f_affine,
               double *b, hipStream_t s, bool dg)
{
    RhsArgs a{};
    a.K = m->n_elements;
    a.M = m->n_vertices;
    a.V = m->vertices;
    a.E = m->elements;
    a.lab = m->labels;
    a.fqp = f_qp;
    if (!f_qp)
        for (int c = 0; c < ncomp; ++c)
            for (int t = 0; t < 3; ++t) a.aff[c][t] = f_affine[3 * c + t];
    a.ncomp = ncomp;
    a.b = b;
    if (dg) {
        hipLaunchKernelGGL(k_rhs_dg, dim3(grid_for(a.K, 256)), dim3(256), 0, s, a, r);
        NLFEM_HIP(hipGetLastError());
        return NLFEM_OK;
    }
    const int64_t nb = (int64_t)ncomp * m->n_vertices;
    hipLaunchKernelGGL(k_fill0, dim3((unsigned)std::min<int64_t>(grid_for(nb, 256), 4096)), dim3(256), 0, s, b, nb);
    hipLaunchKernelGGL(k_rhs, dim3(grid_for(a.K, 256)), dim3(256), 0, s, a, r);
    NLFEM_HIP(hipGetLastError());
    return NLFEM_OK;
}

}  // namespace nlfem

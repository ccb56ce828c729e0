// Stiffness-matrix values: local contributions (eq. def:localStiffness) of all
// interacting pairs, summed into the CSR pattern (eq. biFormApprox).
//
// Non-touching pairs (truncation quadrature, Sec. 2.4.1).  An unordered pair
// {e, f} is processed once for both ordered pairs (e,f) and (f,e).  With the
// same outer and inner rule both directions share the kernel values
//   G_pq = w_p |J_e| w_q |J_f| Psi(x_p(e) - x_q(f)),
// and with the inclusion indicators s_p (x_p(e) sees T_f) and t_q (x_q(f)
// sees T_e) the four terms of eq. case-one-factoredOut of both directions add
// up to
//   rows e, cols e:  sum_p alpha_p phi_p phi_p^T,   alpha_p = sum_q H_pq
//   rows f, cols f:  sum_q beta_q  phi_q phi_q^T,   beta_q  = sum_p H_pq
//   rows e, cols f:  X = -Phi_e^T H Phi_f,  rows f, cols e: X^T
// with H_pq = G_pq (s_p + t_q).  alpha and beta are summed per element in a
// small accumulator (7 values per element instead of 9 matrix entries per
// pair); a last pass turns them into the element-diagonal blocks.  The self
// pair (e, e) is the single ordered pair with t = 0.
//
// Touching pairs of a singular configuration (Sec. 2.4.2, Alg. 1) use the
// regularising transforms to (0,1)^4 with the radial direction integrated in
// closed form: the integrand is homogeneous of degree d = 2 + deg(Psi) in
// the radial variable, so the Gauss rule in that direction (exact for the
// polynomial it meets) can be replaced by its exact value.  What remains:
//   identical: 6 hexagon sectors x n points,   factor 1/((d+2)(d+3)(d+4))
//   edge:      4 faces x n^2 points,           factor 1/((d+3)(d+4))
//   vertex:    2 regions x n^3 points,          factor 1/(d+4)
// For a symmetric kernel the rules give L_fe = L_ef, so each unordered
// touching pair adds 2 L_ef (L_ee for the identical pair).
#include "nlfem_internal.h"

namespace nlfem {
namespace {

struct FarArgs {
    int64_t n;
    const int32_t *ue, *uf;
    const uint32_t *m_ef, *m_fe;
    const int32_t *E;
    const double2 *v0;
    const double4 *J;
    const double *det;
    const uint32_t *node_flags;
    const int64_t *nptr;
    const int32_t *ncol;
    double *val;
    double *daccA;     // accumulator of the A-role points (on e)
    double *daccB;     // accumulator of the B-role points (on f)
    int64_t dstride;   // doubles per element
    double c;
    int32_t use_s, use_t;
    int32_t *err;
};

// rule points of the two roles (A on e, B on f)
struct RoleArgs {
    int32_t PA, PB;
    double xa[kMaxRule][2], wa[kMaxRule], pa[kMaxRule][3];
    double xb[kMaxRule][2], wb[kMaxRule], pb[kMaxRule][3];
};

__device__ inline double rsqrt64(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    for (int it = 0; it < 2; ++it) {
        const double t = x * y;
        const double e = fma(-t, y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}
__device__ inline float rsqrt32(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline double rsq(double x) { return rsqrt64(x); }
__device__ inline float rsq(float x) { return rsqrt32(x); }

// position of column j in node row i, -1 if absent
__device__ inline int64_t find_col(const int64_t *nptr, const int32_t *ncol, int32_t i, int32_t j)
{
    int64_t lo = nptr[i], hi = nptr[i + 1];
    const int64_t base = lo;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (ncol[mid] < j) lo = mid + 1;
        else hi = mid;
    }
    if (lo < nptr[i + 1] && ncol[lo] == j) return lo - base;
    return -1;
}

// add an n x n block v[c][d] at node row i, node column j
template <int NC>
__device__ inline void add_block(const int64_t *nptr, const int32_t *ncol, double *val, int32_t *err,
                                 int32_t i, int32_t j, const double *v)
{
    const int64_t pos = find_col(nptr, ncol, i, j);
    if (pos < 0) {
        atomicOr(err, kErrSlot);
        return;
    }
    if (NC == 1) {
        atomicAdd(&val[nptr[i] + pos], v[0]);
    } else {
        const int64_t len = nptr[i + 1] - nptr[i];
        const int64_t b = (int64_t)NC * NC * nptr[i];
        for (int c = 0; c < NC; ++c)
            for (int d = 0; d < NC; ++d)
                atomicAdd(&val[b + (int64_t)c * NC * len + (int64_t)NC * pos + d], v[c * NC + d]);
    }
}

// kernel values; for NC == 2 the symmetric 2x2 block (k00, k01, k11)
template <int KER, typename T>
__device__ inline void kernel_eval(T zx, T zy, T c, T *k)
{
    if (KER == NLFEM_K_CONSTANT) {
        k[0] = c;
    } else if (KER == NLFEM_K_INV_DIST) {
        k[0] = c * rsq(zx * zx + zy * zy);
    } else {
        const T r = rsq(zx * zx + zy * zy);
        const T s = c * r * r * r;
        k[0] = s * zx * zx;
        k[1] = s * zx * zy;
        k[2] = s * zy * zy;
    }
}

// ---------------------------------------------------------------------------
// non-touching pairs, barycentre ball (every point status is out or whole)

template <int KER, typename T, int PM>
__global__ void __launch_bounds__(256) k_far_bary(FarArgs a, RoleArgs r)
{
    constexpr int NC = KER == NLFEM_K_PERIDYNAMIC ? 2 : 1;
    constexpr int NK = NC == 1 ? 1 : 3;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.n) return;
    const int PA = PM > 0 ? PM : r.PA;
    const int PB = PM > 0 ? PM : r.PB;
    const int32_t e = a.ue[idx], f = a.uf[idx];
    const uint32_t ms = a.use_s ? a.m_ef[idx] : 0u;
    const uint32_t mt = a.use_t ? a.m_fe[idx] : 0u;
    const double2 v0e = a.v0[e], v0f = a.v0[f];
    const double4 Je = a.J[e], Jf = a.J[f];
    const T dx = (T)(v0e.x - v0f.x), dy = (T)(v0e.y - v0f.y);
    const T cc = (T)a.c;
    constexpr int PMAX = PM > 0 ? PM : kMaxRule;
    T ox[PMAX], oy[PMAX], we0[PMAX], we[PMAX];
    T fx[PMAX], fy[PMAX], wf[PMAX];
    const double dete = a.det[e], detf = a.det[f];
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
        if (p < PA) {
            ox[p] = (T)(Je.x * r.xa[p][0] + Je.y * r.xa[p][1]) + dx;
            oy[p] = (T)(Je.z * r.xa[p][0] + Je.w * r.xa[p][1]) + dy;
            we0[p] = (T)(r.wa[p] * dete);
            we[p] = we0[p] * (T)((ms >> (2 * p)) & 1u);
        }
        if (p < PB) {
            fx[p] = (T)(Jf.x * r.xb[p][0] + Jf.y * r.xb[p][1]);
            fy[p] = (T)(Jf.z * r.xb[p][0] + Jf.w * r.xb[p][1]);
            wf[p] = (T)(r.wb[p] * detf);
        }
    }
    T alpha[PMAX][NK], beta[PMAX][NK], tm[PMAX][3][NK];
#pragma unroll
    for (int p = 0; p < PMAX; ++p)
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            alpha[p][k] = 0;
            beta[p][k] = 0;
            tm[p][0][k] = tm[p][1][k] = tm[p][2][k] = 0;
        }
#pragma unroll
    for (int q = 0; q < PMAX; ++q) {
        if (q >= PB) continue;
        const T tq = (T)((mt >> (2 * q)) & 1u) * wf[q];
        const T wq = wf[q];
#pragma unroll
        for (int p = 0; p < PMAX; ++p) {
            if (p >= PA) continue;
            const T zx = ox[p] - fx[q], zy = oy[p] - fy[q];
            T kv[NK];
            kernel_eval<KER, T>(zx, zy, cc, kv);
            // H = G (s_p + t_q), G = w_p|J_e| w_q|J_f| Psi
            const T wgt = we[p] * wq + we0[p] * tq;
#pragma unroll
            for (int k = 0; k < NK; ++k) {
                const T hv = wgt * kv[k];
                alpha[p][k] += hv;
                beta[q][k] += hv;
                tm[p][0][k] += hv * (T)r.pb[q][0];
                tm[p][1][k] += hv * (T)r.pb[q][1];
                tm[p][2][k] += hv * (T)r.pb[q][2];
            }
        }
    }
    // X_ab = -sum_p phi_pa tm[p][b]
    double X[3][3][NK];
#pragma unroll
    for (int ia = 0; ia < 3; ++ia)
#pragma unroll
        for (int ib = 0; ib < 3; ++ib)
#pragma unroll
            for (int k = 0; k < NK; ++k) {
                T s = 0;
#pragma unroll
                for (int p = 0; p < PMAX; ++p)
                    if (p < PA) s += (T)r.pa[p][ia] * tm[p][ib][k];
                X[ia][ib][k] = -(double)s;
            }
    const int32_t ne[3] = {a.E[3 * (int64_t)e], a.E[3 * (int64_t)e + 1], a.E[3 * (int64_t)e + 2]};
    const int32_t nf[3] = {a.E[3 * (int64_t)f], a.E[3 * (int64_t)f + 1], a.E[3 * (int64_t)f + 2]};
    bool dof_e[3], dof_f[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        dof_e[i] = a.node_flags[ne[i]] == 1u;
        dof_f[i] = a.node_flags[nf[i]] == 1u;
    }
#pragma unroll
    for (int ia = 0; ia < 3; ++ia)
#pragma unroll
        for (int ib = 0; ib < 3; ++ib) {
            double blk[NC * NC], blkT[NC * NC];
            if (NC == 1) {
                blk[0] = blkT[0] = X[ia][ib][0];
            } else {
                blk[0] = X[ia][ib][0];
                blk[1] = X[ia][ib][1];
                blk[2] = X[ia][ib][1];
                blk[3] = X[ia][ib][2];
                for (int t = 0; t < 4; ++t) blkT[t] = blk[t];   // symmetric 2x2
            }
            if (dof_e[ia]) add_block<NC>(a.nptr, a.ncol, a.val, a.err, ne[ia], nf[ib], blk);
            if (dof_f[ib]) add_block<NC>(a.nptr, a.ncol, a.val, a.err, nf[ib], ne[ia], blkT);
        }
    const bool any_e = dof_e[0] || dof_e[1] || dof_e[2];
    const bool any_f = dof_f[0] || dof_f[1] || dof_f[2];
    constexpr int NN = NC * NC;
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
        if (any_e && p < PA)
#pragma unroll
            for (int k = 0; k < NK; ++k) atomicAdd(&a.daccA[(int64_t)e * a.dstride + p * NN + k], (double)alpha[p][k]);
        if (any_f && p < PB)
#pragma unroll
            for (int k = 0; k < NK; ++k) atomicAdd(&a.daccB[(int64_t)f * a.dstride + p * NN + k], (double)beta[p][k]);
    }
}

// element-diagonal blocks from the per-element accumulators
struct DiagArgs {
    int64_t K;
    const int64_t *sptr;     // [K + 1] offsets of the neighbour lists
    const int32_t *E;
    const uint32_t *node_flags;
    const int64_t *nptr;
    const int32_t *ncol;
    double *val;
    const double *dacc;
    int64_t dstride;
    int32_t P, Q, same;
    int32_t *err;
};

template <int NC>
__global__ void __launch_bounds__(256) k_diag(DiagArgs a, RuleArgs r)
{
    constexpr int NK = NC == 1 ? 1 : 3;
    constexpr int NN = NC * NC;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.K) return;
    if (a.sptr[e + 1] == a.sptr[e]) return;   // no interacting pair: nothing to add
    const int32_t nd[3] = {a.E[3 * e], a.E[3 * e + 1], a.E[3 * e + 2]};
    bool dof[3];
    for (int i = 0; i < 3; ++i) dof[i] = a.node_flags[nd[i]] == 1u;
    if (!(dof[0] || dof[1] || dof[2])) return;
    double D[3][3][NK];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < NK; ++k) D[i][j][k] = 0.0;
    const double *acc = a.dacc + e * a.dstride;
    for (int p = 0; p < a.P; ++p)
        for (int k = 0; k < NK; ++k) {
            const double v = acc[p * NN + k];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) D[i][j][k] += v * r.pphi[p][i] * r.pphi[p][j];
        }
    if (!a.same) {
        const double *acc2 = acc + (int64_t)a.P * NN;
        for (int q = 0; q < a.Q; ++q)
            for (int k = 0; k < NK; ++k) {
                const double v = acc2[q * NN + k];
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) D[i][j][k] += v * r.qphi[q][i] * r.qphi[q][j];
            }
    }
    for (int i = 0; i < 3; ++i) {
        if (!dof[i]) continue;
        for (int j = 0; j < 3; ++j) {
            double blk[NN];
            if (NC == 1) {
                blk[0] = D[i][j][0];
            } else {
                blk[0] = D[i][j][0];
                blk[1] = blk[2] = D[i][j][1];
                blk[3] = D[i][j][2];
            }
            add_block<NC>(a.nptr, a.ncol, a.val, a.err, nd[i], nd[j], blk);
        }
    }
}

// ---------------------------------------------------------------------------
// touching pairs

struct TouchArgs {
    int64_t n;
    const int32_t *te, *tf;
    const int32_t *E;
    const double *V;
    const uint32_t *node_flags;
    const int64_t *nptr;
    const int32_t *ncol;
    double *val;
    double c;
    int32_t *err;
};

__device__ inline double2 vtx(const double *V, int32_t n) { return make_double2(V[2 * (int64_t)n], V[2 * (int64_t)n + 1]); }

// accumulate w * Psi(z) (g g^T) into the packed upper triangle of L (nu nodes)
template <int KER, int NU>
__device__ inline void acc_sample(double (&L)[(NU * (KER == NLFEM_K_PERIDYNAMIC ? 2 : 1)) *
                                              (NU * (KER == NLFEM_K_PERIDYNAMIC ? 2 : 1) + 1) / 2],
                                  double w, double zx, double zy, const double (&g)[NU], double c)
{
    constexpr int NC = KER == NLFEM_K_PERIDYNAMIC ? 2 : 1;
    constexpr int D = NU * NC;
    double k[3];
    kernel_eval<KER, double>(zx, zy, c, k);
    double kk[NC][NC];
    if (NC == 1) {
        kk[0][0] = k[0];
    } else {
        kk[0][0] = k[0];
        kk[0][1] = kk[1][0] = k[1];
        kk[1][1] = k[2];
    }
    int idx = 0;
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
        for (int s = r; s < D; ++s) {
            L[idx++] += w * kk[r % NC][s % NC] * g[r / NC] * g[s / NC];
        }
}

template <int KER, int NU>
__device__ inline void scatter_touch(const TouchArgs &a, const int32_t (&nodes)[NU],
                                     const double (&L)[(NU * (KER == NLFEM_K_PERIDYNAMIC ? 2 : 1)) *
                                                       (NU * (KER == NLFEM_K_PERIDYNAMIC ? 2 : 1) + 1) / 2],
                                     double scale)
{
    constexpr int NC = KER == NLFEM_K_PERIDYNAMIC ? 2 : 1;
    constexpr int D = NU * NC;
    for (int i = 0; i < NU; ++i) {
        if (a.node_flags[nodes[i]] != 1u) continue;
        for (int j = 0; j < NU; ++j) {
            double blk[NC * NC];
            for (int c = 0; c < NC; ++c)
                for (int d = 0; d < NC; ++d) {
                    int r = i * NC + c, s = j * NC + d;
                    if (r > s) {
                        int t = r;
                        r = s;
                        s = t;
                    }
                    // packed upper index of (r, s)
                    const int idx = r * D - r * (r - 1) / 2 + (s - r);
                    blk[c * NC + d] = scale * L[idx];
                }
            add_block<NC>(a.nptr, a.ncol, a.val, a.err, nodes[i], nodes[j], blk);
        }
    }
}

template <int KER>
constexpr int homog_degree() { return KER == NLFEM_K_CONSTANT ? 2 : 1; }

template <int KER>
__global__ void __launch_bounds__(256) k_touch_ident(TouchArgs a, GaussArgs g)
{
    constexpr int NC = KER == NLFEM_K_PERIDYNAMIC ? 2 : 1;
    constexpr int D = 3 * NC;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.n) return;
    const int32_t e = a.te[idx];
    const int32_t nodes[3] = {a.E[3 * (int64_t)e], a.E[3 * (int64_t)e + 1], a.E[3 * (int64_t)e + 2]};
    const double2 p0 = vtx(a.V, nodes[0]), p1 = vtx(a.V, nodes[1]), p2 = vtx(a.V, nodes[2]);
    const double J00 = p1.x - p0.x, J01 = p2.x - p0.x, J10 = p1.y - p0.y, J11 = p2.y - p0.y;
    const double det = fabs(J00 * J11 - J01 * J10);
    double L[D * (D + 1) / 2];
    for (int t = 0; t < D * (D + 1) / 2; ++t) L[t] = 0.0;
    const double hx[6] = {1, 0, -1, -1, 0, 1}, hy[6] = {0, 1, 1, 0, -1, -1};
    for (int j = 0; j < 6; ++j) {
        const int j1 = j == 5 ? 0 : j + 1;
        for (int iu = 0; iu < g.n; ++iu) {
            const double u = g.x[iu];
            const double wx = (1.0 - u) * hx[j] + u * hx[j1];
            const double wy = (1.0 - u) * hy[j] + u * hy[j1];
            // a = phi(x^) - phi(x^ + z) = -grad phi . z ; z = rho w
            const double gg[3] = {wx + wy, -wx, -wy};
            const double zx = J00 * wx + J01 * wy, zy = J10 * wx + J11 * wy;
            acc_sample<KER, 3>(L, g.w[iu], zx, zy, gg, a.c);
        }
    }
    constexpr int d = homog_degree<KER>();
    const double scale = det * det / (double)((d + 2) * (d + 3) * (d + 4));
    scatter_touch<KER, 3>(a, nodes, L, scale);
}

template <int KER>
__global__ void __launch_bounds__(256) k_touch_edge(TouchArgs a, GaussArgs g)
{
    constexpr int NC = KER == NLFEM_K_PERIDYNAMIC ? 2 : 1;
    constexpr int D = 4 * NC;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.n) return;
    const int32_t e = a.te[idx], f = a.tf[idx];
    const int32_t ek[3] = {a.E[3 * (int64_t)e], a.E[3 * (int64_t)e + 1], a.E[3 * (int64_t)e + 2]};
    const int32_t el[3] = {a.E[3 * (int64_t)f], a.E[3 * (int64_t)f + 1], a.E[3 * (int64_t)f + 2]};
    // frames (P0, P1, A) and (P0, P1, B), P0 the smaller shared node id
    int32_t sh0 = -1, sh1 = -1, A = -1, B = -1;
    for (int i = 0; i < 3; ++i) {
        const bool in = ek[i] == el[0] || ek[i] == el[1] || ek[i] == el[2];
        if (in) {
            if (sh0 < 0) sh0 = ek[i];
            else sh1 = ek[i];
        } else {
            A = ek[i];
        }
        const bool inl = el[i] == ek[0] || el[i] == ek[1] || el[i] == ek[2];
        if (!inl) B = el[i];
    }
    const int32_t P0 = min(sh0, sh1), P1 = max(sh0, sh1);
    const int32_t nodes[4] = {P0, P1, A, B};
    const double2 q0 = vtx(a.V, P0), q1 = vtx(a.V, P1), qa = vtx(a.V, A), qb = vtx(a.V, B);
    // x - y = E v, E = [P1 - P0, A - P0, -(B - P0)]
    const double E0x = q1.x - q0.x, E0y = q1.y - q0.y;
    const double E1x = qa.x - q0.x, E1y = qa.y - q0.y;
    const double E2x = -(qb.x - q0.x), E2y = -(qb.y - q0.y);
    const double detk = fabs(E0x * E1y - E1x * E0y);
    const double detl = fabs(E0x * E2y - E2x * E0y);
    double L[D * (D + 1) / 2];
    for (int t = 0; t < D * (D + 1) / 2; ++t) L[t] = 0.0;
    for (int face = 0; face < 4; ++face)
        for (int ip = 0; ip < g.n; ++ip)
            for (int iq = 0; iq < g.n; ++iq) {
                const double p = g.x[ip], q = g.x[iq];
                double w0, w1, w2, jf;
                if (face == 0) { w0 = p; w1 = 1.0 - p; w2 = q; jf = 1.0; }
                else if (face == 1) { w0 = p; w1 = (1.0 - p) * q; w2 = 1.0; jf = 1.0 - p; }
                else if (face == 2) { w0 = -p; w1 = 1.0; w2 = (1.0 - p) * q; jf = 1.0 - p; }
                else { w0 = -p; w1 = q; w2 = 1.0 - p; jf = 1.0; }
                const double gg[4] = {-w0 - w1 + w2, w0, w1, -w2};
                const double zx = E0x * w0 + E1x * w1 + E2x * w2;
                const double zy = E0y * w0 + E1y * w1 + E2y * w2;
                acc_sample<KER, 4>(L, g.w[ip] * g.w[iq] * jf, zx, zy, gg, a.c);
            }
    constexpr int d = homog_degree<KER>();
    const double scale = 2.0 * detk * detl / (double)((d + 3) * (d + 4));
    scatter_touch<KER, 4>(a, nodes, L, scale);
}

template <int KER>
__global__ void __launch_bounds__(256) k_touch_vertex(TouchArgs a, GaussArgs g)
{
    constexpr int NC = KER == NLFEM_K_PERIDYNAMIC ? 2 : 1;
    constexpr int D = 5 * NC;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.n) return;
    const int32_t e = a.te[idx], f = a.tf[idx];
    const int32_t ek[3] = {a.E[3 * (int64_t)e], a.E[3 * (int64_t)e + 1], a.E[3 * (int64_t)e + 2]};
    const int32_t el[3] = {a.E[3 * (int64_t)f], a.E[3 * (int64_t)f + 1], a.E[3 * (int64_t)f + 2]};
    int ia = 0, ib = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            if (ek[i] == el[j]) {
                ia = i;
                ib = j;
            }
    const int32_t nodes[5] = {ek[ia], ek[(ia + 1) % 3], ek[(ia + 2) % 3], el[(ib + 1) % 3], el[(ib + 2) % 3]};
    const double2 q0 = vtx(a.V, nodes[0]), a1 = vtx(a.V, nodes[1]), a2 = vtx(a.V, nodes[2]);
    const double2 b1 = vtx(a.V, nodes[3]), b2 = vtx(a.V, nodes[4]);
    const double A1x = a1.x - q0.x, A1y = a1.y - q0.y, A2x = a2.x - q0.x, A2y = a2.y - q0.y;
    const double B1x = b1.x - q0.x, B1y = b1.y - q0.y, B2x = b2.x - q0.x, B2y = b2.y - q0.y;
    const double detk = fabs(A1x * A2y - A2x * A1y);
    const double detl = fabs(B1x * B2y - B2x * B1y);
    double L[D * (D + 1) / 2];
    for (int t = 0; t < D * (D + 1) / 2; ++t) L[t] = 0.0;
    for (int iw = 0; iw < g.n; ++iw) {
        const double w = g.x[iw];
        for (int iaa = 0; iaa < g.n; ++iaa) {
            const double al = g.x[iaa];
            const double ex = (1.0 - al) * A1x + al * A2x, ey = (1.0 - al) * A1y + al * A2y;
            for (int ibb = 0; ibb < g.n; ++ibb) {
                const double be = g.x[ibb];
                const double fx = (1.0 - be) * B1x + be * B2x, fy = (1.0 - be) * B1y + be * B2y;
                const double wt = g.w[iw] * g.w[iaa] * g.w[ibb] * w;
                {   // region t <= s: t = s w
                    const double gg[5] = {w - 1.0, 1.0 - al, al, -w * (1.0 - be), -w * be};
                    acc_sample<KER, 5>(L, wt, ex - w * fx, ey - w * fy, gg, a.c);
                }
                {   // region s <= t: s = t w
                    const double gg[5] = {1.0 - w, w * (1.0 - al), w * al, -(1.0 - be), -be};
                    acc_sample<KER, 5>(L, wt, w * ex - fx, w * ey - fy, gg, a.c);
                }
            }
        }
    }
    constexpr int d = homog_degree<KER>();
    const double scale = 2.0 * detk * detl / (double)(d + 4);
    scatter_touch<KER, 5>(a, nodes, L, scale);
}

__global__ void __launch_bounds__(256) k_zero(double *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

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

template <int KER, typename T>
void far_launch(const FarArgs &a, const RoleArgs &r, hipStream_t s)
{
    const unsigned grid = grid_for(a.n, 256);
    if (r.PA == 7 && r.PB == 7) hipLaunchKernelGGL((k_far_bary<KER, T, 7>), dim3(grid), dim3(256), 0, s, a, r);
    else hipLaunchKernelGGL((k_far_bary<KER, T, 0>), dim3(grid), dim3(256), 0, s, a, r);
}

template <int KER>
void far_dispatch(const FarArgs &a, const RoleArgs &r, bool fp32, hipStream_t s)
{
    if (fp32) far_launch<KER, float>(a, r, s);
    else far_launch<KER, double>(a, r, s);
}

template <int KER>
void touch_launch(const nlfem_pairs *h, TouchArgs t, const GaussArgs &g, hipStream_t s)
{
    const int64_t nI = h->nUTc[0], nE = h->nUTc[1], nV = h->nUTc[2];
    if (nI > 0) {
        t.n = nI;
        t.te = h->te;
        t.tf = h->tf;
        hipLaunchKernelGGL(k_touch_ident<KER>, dim3(grid_for(nI, 256)), dim3(256), 0, s, t, g);
    }
    if (nE > 0) {
        t.n = nE;
        t.te = h->te + nI;
        t.tf = h->tf + nI;
        hipLaunchKernelGGL(k_touch_edge<KER>, dim3(grid_for(nE, 256)), dim3(256), 0, s, t, g);
    }
    if (nV > 0) {
        t.n = nV;
        t.te = h->te + nI + nE;
        t.tf = h->tf + nI + nE;
        hipLaunchKernelGGL(k_touch_vertex<KER>, dim3(grid_for(nV, 256)), dim3(256), 0, s, t, g);
    }
}

}  // namespace

int launch_assemble(const nlfem_pairs *h, const nlfem_mesh *m, const nlfem_config *cfg, const GaussArgs &g,
                    double *val, hipStream_t s)
{
    const int nc = h->ncomp;
    const int64_t nnz = h->nnz_node * nc * nc;
    const int64_t ndacc = h->K * h->dacc_stride;
    if (nnz > 0)
        hipLaunchKernelGGL(k_zero, dim3((unsigned)std::min<int64_t>(grid_for(nnz, 256), 8192)), dim3(256), 0, s, val, nnz);
    if (ndacc > 0)
        hipLaunchKernelGGL(k_zero, dim3((unsigned)std::min<int64_t>(grid_for(ndacc, 256), 8192)), dim3(256), 0, s,
                           h->dacc, ndacc);
    const bool fp32 = cfg->precision == NLFEM_P_MIXED;
    if (h->nUF > 0) {
        FarArgs a{};
        a.n = h->nUF;
        a.ue = h->ue;
        a.uf = h->uf;
        a.m_ef = h->um_ef;
        a.m_fe = h->um_fe;
        a.E = m->elements;
        a.v0 = h->v0;
        a.J = h->J;
        a.det = h->det;
        a.node_flags = h->node_flags;
        a.nptr = h->nptr;
        a.ncol = h->ncol;
        a.val = val;
        a.dstride = h->dacc_stride;
        a.c = cfg->c;
        a.err = h->err;
        const int NN = nc * nc;
        auto run = [&](const RoleArgs &r) {
            switch (h->kernel) {
            case NLFEM_K_CONSTANT: far_dispatch<NLFEM_K_CONSTANT>(a, r, fp32, s); break;
            case NLFEM_K_INV_DIST: far_dispatch<NLFEM_K_INV_DIST>(a, r, fp32, s); break;
            default: far_dispatch<NLFEM_K_PERIDYNAMIC>(a, r, fp32, s); break;
            }
        };
        if (h->rules.same) {
            a.use_s = a.use_t = 1;
            a.daccA = a.daccB = h->dacc;
            run(roles(h->rules, true, true));
        } else {
            // direction e -> f: outer points on e, inner points on f
            a.use_s = 1;
            a.use_t = 0;
            a.daccA = h->dacc;
            a.daccB = h->dacc + (int64_t)h->rules.P * NN;
            run(roles(h->rules, true, false));
            // direction f -> e: outer points on f, inner points on e
            a.use_s = 0;
            a.use_t = 1;
            a.daccA = h->dacc + (int64_t)h->rules.P * NN;
            a.daccB = h->dacc;
            run(roles(h->rules, false, true));
        }
    }
    if (h->nUT > 0) {
        TouchArgs t{};
        t.E = m->elements;
        t.V = m->vertices;
        t.node_flags = h->node_flags;
        t.nptr = h->nptr;
        t.ncol = h->ncol;
        t.val = val;
        t.c = cfg->c;
        t.err = h->err;
        switch (h->kernel) {
        case NLFEM_K_CONSTANT: touch_launch<NLFEM_K_CONSTANT>(h, t, g, s); break;
        case NLFEM_K_INV_DIST: touch_launch<NLFEM_K_INV_DIST>(h, t, g, s); break;
        default: touch_launch<NLFEM_K_PERIDYNAMIC>(h, t, g, s); break;
        }
    }
    if (h->K > 0) {
        DiagArgs d{h->K, h->loff + (int64_t)kLsS * (h->K + 1), m->elements, h->node_flags, h->nptr, h->ncol, val, h->dacc, h->dacc_stride,
                   h->rules.P, h->rules.Q, h->rules.same, h->err};
        if (nc == 1) hipLaunchKernelGGL(k_diag<1>, dim3(grid_for(h->K, 256)), dim3(256), 0, s, d, h->rules);
        else hipLaunchKernelGGL(k_diag<2>, dim3(grid_for(h->K, 256)), dim3(256), 0, s, d, h->rules);
    }
    NLFEM_HIP(hipGetLastError());
    return NLFEM_OK;
}

}  // namespace nlfem

// Per-item device code of the assembly (Sec. 2.3-2.4): arguments and the
// work of one non-touching pair, one touching pair, one element diagonal and
// one matrix row.  The single-problem kernels (assemble.hip) and the
// persistent batched kernels (batch.hip) run the same functions, so both give
// bit-identical results.
//
// The local contributions (eq. def:localStiffness) of all interacting pairs
// are summed into the CSR pattern (eq. biFormApprox).
//
// Phase 1 computes one result per unordered pair; phase 2 owns the matrix
// rows and gathers.  No global atomics, no zero fill: every stored entry is
// written exactly once by the wave that owns its row.
//
// Non-touching pairs (truncation quadrature, Sec. 2.4.1).  For {e, f} both
// ordered pairs (e,f) and (f,e) are evaluated together.  With the same rule
// on both sides they share the kernel values
//   G_pq = w_p |J_e| w_q |J_f| Psi(x_p(e) - x_q(f)),
// and with the point indicators s_p (x_p(e) sees T_f) and t_q (x_q(f) sees
// T_e) the four terms of eq. case-one-factoredOut of both directions become
//   rows e, cols f:  X  = -Phi_e^T H Phi_f,        H_pq = G_pq (s_p + t_q)
//   rows e, cols e:  De = sum_p (sum_q H_pq) phi_p phi_p^T
//   rows f, cols f:  Df = sum_q (sum_p H_pq) phi_q phi_q^T
//   rows f, cols e:  X^T.
// The record of the pair holds X, De and Df (FP32 in the mixed form: FP32
// quadrature with FP32 accumulation per pair).  The self pair (e, e) is the
// single ordered pair with t = 0 and stores X + X^T and De + Df.
//
// Touching pairs of a singular configuration (Sec. 2.4.2, Alg. 1): the
// regularising transforms to (0,1)^4 with the radial direction integrated in
// closed form.  The integrand is homogeneous of degree d = 2 + deg(Psi) in
// the radial variable and the Gauss rule integrates that direction exactly,
// so it is replaced by its exact value.  What remains:
//   identical: 6 hexagon sectors x n points,   factor 1/((d+2)(d+3)(d+4))
//   edge:      4 faces x n^2 points,           factor 1/((d+3)(d+4))
//   vertex:    2 regions x n^3 points,          factor 1/(d+4)
// A group of lanes shares one pair and reduces through cross-lane shuffles.
// For a symmetric kernel the rules give L_fe = L_ef, so a row that meets the
// pair only through one of its elements adds 2 L, a row of a shared vertex
// meets it twice and adds L each time.
#pragma once

#include "caps.h"
#include "nlfem_internal.h"

namespace nlfem {
namespace items {

// ------------------------------------------------------------------ helpers

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
__device__ inline double rsq(double x) { return rsqrt64(x); }
__device__ inline float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

template <int KER>
struct Ker {
    static constexpr int BASE = KER & (kKerNoZeroDiv - 1);
    static constexpr bool NZD = (KER & kKerNoZeroDiv) != 0;
    static constexpr int NC = BASE == NLFEM_K_PERIDYNAMIC ? 2 : 1;
    static constexpr int NK = NC == 1 ? 1 : 3;   // stored values of a symmetric NC x NC block
    // homogeneity degree of the integrand: 2 + the degree of Psi
    static constexpr int D = BASE == NLFEM_K_CONSTANT ? 2 : BASE == NLFEM_K_FRAC_HALF ? -1 : 1;
};

// kernel values; for two components the symmetric block (k00, k01, k11).
// With the no-zero-division variant the values are 0 for |z|^2 <= z2min.
template <int KER, typename T>
__device__ inline void kernel_eval(T zx, T zy, T c, T *k, T z2min = 0)
{
    constexpr int B = Ker<KER>::BASE;
    const T r2 = zx * zx + zy * zy;
    if (B == NLFEM_K_CONSTANT) {
        k[0] = c;
    } else if (B == NLFEM_K_INV_DIST) {
        k[0] = c * rsq(r2);
    } else if (B == NLFEM_K_FRAC_HALF) {
        const T r = rsq(r2);
        k[0] = c * r * r * r;
    } else {
        const T r = rsq(r2);
        const T s = c * r * r * r;
        k[0] = s * zx * zx;
        k[1] = s * zx * zy;
        k[2] = s * zy * zy;
    }
    if constexpr (Ker<KER>::NZD) {
#pragma unroll
        for (int i = 0; i < Ker<KER>::NK; ++i) k[i] = r2 <= z2min ? (T)0 : k[i];
    }
}

__host__ __device__ constexpr int sym_index(int r, int s, int D)
{
    if (r > s) {
        const int t = r;
        r = s;
        s = t;
    }
    return r * D - r * (r - 1) / 2 + (s - r);
}

// Vertex order of the transforms.  identical: the stored order; edge:
// (P0, P1, A, B) with P0 < P1 the shared nodes, A and B the third vertices
// of the first and second element; vertex: (P0, A1, A2, B1, B2) with P0 the
// shared node and each element's other vertices in cyclic order after P0.
__device__ inline int touch_frame(int cls, const int32_t *ek, const int32_t *el, int32_t *n)
{
    if (cls == 3) {
        n[0] = ek[0];
        n[1] = ek[1];
        n[2] = ek[2];
        return 3;
    }
    if (cls == 2) {
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
        n[0] = min(sh0, sh1);
        n[1] = max(sh0, sh1);
        n[2] = A;
        n[3] = B;
        return 4;
    }
    int ia = 0, ib = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            if (ek[i] == el[j]) {
                ia = i;
                ib = j;
            }
    // selects instead of indexing, so the triples stay in registers
    const int a1 = ia == 2 ? 0 : ia + 1, a2 = ia == 0 ? 2 : ia - 1;
    const int b1 = ib == 2 ? 0 : ib + 1, b2 = ib == 0 ? 2 : ib - 1;
    n[0] = ia == 0 ? ek[0] : ia == 1 ? ek[1] : ek[2];
    n[1] = a1 == 0 ? ek[0] : a1 == 1 ? ek[1] : ek[2];
    n[2] = a2 == 0 ? ek[0] : a2 == 1 ? ek[1] : ek[2];
    n[3] = b1 == 0 ? el[0] : b1 == 1 ? el[1] : el[2];
    n[4] = b2 == 0 ? el[0] : b2 == 1 ? el[1] : el[2];
    return 5;
}

__device__ inline double2 vtx(const double *V, int32_t n) { return make_double2(V[2 * (int64_t)n], V[2 * (int64_t)n + 1]); }

// ------------------------------------------------------ phase 1: far pairs

struct FarArgs {
    int64_t n;
    const int32_t *ue, *uf;
    const uint2 *m;          // status masks (e's outer points vs f, f's vs e)
    const double2 *v0;
    const double4 *J;
    const double *det;
    void *rec;
    int32_t stride;
    double c;
    int32_t same;
    // polygon ball only
    const double2 *xp;       // [K][P] outer points (FP64)
    int32_t P;
    const int32_t *E;
    const double *V;
    const double *dir;       // [N][2]
    int32_t N;
    int32_t caps;            // 1 nocaps, 2 approximate caps (caps.h): polygons from the circle's crossings
    double delta;
    int32_t cap;             // clip buffer length per lane
    int32_t *err;
    SpecGate gate;           // single-problem launches after an unchecked rebuild
};

// Non-touching pair records (n records, NK values per block entry), stored
// by use: the row chunks R_loc (row loc of X: e's vertex loc against the
// vertices of f), the column chunks C_loc (column loc of X: f's vertex loc
// against the vertices of e), then the element-diagonal blocks De and Df.
// Each array is contiguous over the record index, so the rows of e's
// vertices read the R chunks of e's upper list entries and those of f's
// vertices the C chunks, each chunk once and only the values used; the
// diagonal sums read De of the upper entries and Df of the lower ones.
template <int NK>
struct Rec {
    static constexpr int kValues = 30 * NK;   // per record
    __host__ __device__ static int64_t r(int loc, int64_t u, int64_t n) { return ((int64_t)loc * n + u) * 3 * NK; }
    __host__ __device__ static int64_t c(int loc, int64_t u, int64_t n)
    {
        return ((int64_t)(3 + loc) * n + u) * 3 * NK;
    }
    // De (second = false) or Df (second = true) of record u: 6 NK values
    __host__ __device__ static int64_t d(int64_t u, int64_t n, bool second)
    {
        return (second ? 24 : 18) * NK * n + u * 6 * NK;
    }
};

// Constant kernel under the barycentre ball (scalar, continuous ansatz): a
// point pair of a non-touching pair counts iff the status bit of its outer
// point says so, and the kernel value does not depend on the points, so the
// double sums behind X, De and Df (Sec. 2.3, the four terms of the bilinear
// form; Sec. 2.4.1) factor into sums over one element's rule.  With, for a
// status mask m, M_O(m)_a = sum over the outer points p set in m of
// w_p phi_a(x_p), T_O(m) = sum of their w_p, Q_O(m)_ab = sum of their
// w_p phi_a phi_b, the same sums over every inner point M_I, W_I, Q_I, and
// me / mf the masks of e's / f's outer points against the other element:
//   row a of e against vertex b of f:  -c |J_e| |J_f| (M_O(me)_a M_I,b + M_I,a M_O(mf)_b)
//   e's element-diagonal block:         c |J_e| |J_f| (Q_O(me) W_I + Q_I T_O(mf))
// (both directions of the pair; the self pair takes me = mf, which gives
// X + X^T and De + Df).  The row gather and the diagonal sums evaluate these
// from the masks and determinants, so such problems form no far records.
constexpr int kMomP = 8;   // outer points of the moment form (two nibbles of status bits)
struct MomArgs {
    int32_t on = 0;
    int32_t P = 0;                                     // outer points: status fields per mask
    const uint2 *m = nullptr;                          // masks of the unordered pairs (first, second element)
    const double *det = nullptr;                       // |det J| per element
    double c = 0.0;
    double mo[kMomP][3] = {};                          // w_p phi_a(x_p), outer rule
    double mi[3] = {};                                 // M_I
    double wo[kMomP] = {};                             // w_p, outer rule
    double qo[kMomP][6] = {};                          // w_p phi_a phi_b (a <= b, packed), outer rule
    double qi[6] = {};                                 // Q_I
    double wi = 0.0;                                   // W_I
};

// status bit "whole" of outer point p as 0.0 / 1.0
__device__ __forceinline__ double whole_bit(uint32_t m, int p) { return (double)((m >> (2 * p)) & 1u); }

// the "whole" bits of outer points 4n .. 4n+3 as a 4-bit index
__device__ __forceinline__ uint32_t whole_nibble(uint32_t m, int n)
{
    uint32_t x = (m >> (8 * n)) & 0x55u;
    x = (x | (x >> 1)) & 0x33u;
    return (x | (x >> 2)) & 0x0fu;
}

// masks of the entry f in e's list (record u): e's outer points, then f's
__device__ __forceinline__ void entry_masks(const MomArgs &m, int64_t u, int32_t e, int32_t f, uint32_t &me,
                                            uint32_t &mf)
{
    const uint2 x = m.m[u];
    const uint32_t x0 = x.x, x1 = x.y;
    me = f >= e ? x0 : x1;
    mf = f > e ? x1 : x0;
}

// rule points of the two roles (A on e, B on f)
struct RoleArgs {
    int32_t PA, PB;
    double xa[kMaxRule][2], wa[kMaxRule], pa[kMaxRule][3];
    double xb[kMaxRule][2], wb[kMaxRule], pb[kMaxRule][3];
};

template <int KER, typename T, int PM>
__device__ inline void far_direction(const RoleArgs &r, T dx, T dy, const double4 &Je, const double4 &Jf,
                                     double dete, double detf, uint32_t ms, uint32_t mt, T cc,
                                     T (&X)[3][3][Ker<KER>::NK], T (&De)[6][Ker<KER>::NK],
                                     T (&Df)[6][Ker<KER>::NK])
{
    constexpr int NK = Ker<KER>::NK;
    constexpr int PMAX = PM > 0 ? PM : kMaxRule;
    const int PA = PM > 0 ? PM : r.PA;
    const int PB = PM > 0 ? PM : r.PB;
    T fx[PMAX], fy[PMAX], wf[PMAX], tf[PMAX];
    T beta[PMAX][NK];
    const T z2min = Ker<KER>::NZD ? (T)(1e-12 * fmin(dete, detf)) : (T)0;
#pragma unroll
    for (int q = 0; q < PMAX; ++q) {
        if (q < PB) {
            fx[q] = (T)(Jf.x * r.xb[q][0] + Jf.y * r.xb[q][1]);
            fy[q] = (T)(Jf.z * r.xb[q][0] + Jf.w * r.xb[q][1]);
            wf[q] = (T)(r.wb[q] * detf);
            tf[q] = wf[q] * (T)((mt >> (2 * q)) & 1u);
        }
#pragma unroll
        for (int k = 0; k < NK; ++k) beta[q][k] = 0;
    }
    auto outer = [&](int p) {
        const T ox = (T)(Je.x * r.xa[p][0] + Je.y * r.xa[p][1]) + dx;
        const T oy = (T)(Je.z * r.xa[p][0] + Je.w * r.xa[p][1]) + dy;
        const T we0 = (T)(r.wa[p] * dete);
        const T we = we0 * (T)((ms >> (2 * p)) & 1u);
        T alpha[NK], tm[3][NK];
#pragma unroll
        for (int k = 0; k < NK; ++k) alpha[k] = tm[0][k] = tm[1][k] = tm[2][k] = 0;
#pragma unroll
        for (int q = 0; q < PMAX; ++q) {
            if (q >= PB) continue;
            const T zx = ox - fx[q], zy = oy - fy[q];
            T kv[NK];
            kernel_eval<KER, T>(zx, zy, cc, kv, z2min);
            const T wgt = we * wf[q] + we0 * tf[q];   // w_p|J_e| w_q|J_f| (s_p + t_q)
#pragma unroll
            for (int k = 0; k < NK; ++k) {
                const T hv = wgt * kv[k];
                alpha[k] += hv;
                beta[q][k] += hv;
                tm[0][k] += hv * (T)r.pb[q][0];
                tm[1][k] += hv * (T)r.pb[q][1];
                tm[2][k] += hv * (T)r.pb[q][2];
            }
        }
        const T pp[3] = {(T)r.pa[p][0], (T)r.pa[p][1], (T)r.pa[p][2]};
#pragma unroll
        for (int k = 0; k < NK; ++k) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) X[a][b][k] -= pp[a] * tm[b][k];
            De[0][k] += alpha[k] * pp[0] * pp[0];
            De[1][k] += alpha[k] * pp[0] * pp[1];
            De[2][k] += alpha[k] * pp[0] * pp[2];
            De[3][k] += alpha[k] * pp[1] * pp[1];
            De[4][k] += alpha[k] * pp[1] * pp[2];
            De[5][k] += alpha[k] * pp[2] * pp[2];
        }
    };
    if constexpr (PM > 0 && sizeof(T) == 4 && NK == 1) {
        // a fixed rule in FP32, scalar kernel: the outer points in a loop
        // (uniform index into the rule tables), the inner ones unrolled; this
        // halves the register count (4 waves per SIMD instead of 2).  The
        // other cases keep their occupancy either way and run faster
        // unrolled.
#pragma unroll 1
        for (int p = 0; p < PM; ++p) outer(p);
    } else {
#pragma unroll
        for (int p = 0; p < PMAX; ++p)
            if (p < PA) outer(p);
    }
#pragma unroll
    for (int q = 0; q < PMAX; ++q) {
        if (q >= PB) continue;
        const T b0 = (T)r.pb[q][0], b1 = (T)r.pb[q][1], b2 = (T)r.pb[q][2];
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            Df[0][k] += beta[q][k] * b0 * b0;
            Df[1][k] += beta[q][k] * b0 * b1;
            Df[2][k] += beta[q][k] * b0 * b2;
            Df[3][k] += beta[q][k] * b1 * b1;
            Df[4][k] += beta[q][k] * b1 * b2;
            Df[5][k] += beta[q][k] * b2 * b2;
        }
    }
}

// ---- polygon ball: outer points whose polygon straddles the inner element
//
// Sutherland-Hodgman clip of the inner triangle by the regular N-gon around
// the outer point, in the operation order of the pair search (no
// contraction), so the polygon is the one whose status the search recorded;
// then the fan from the first vertex of the clipped polygon with the inner
// rule on every sub-triangle and the basis functions of the inner element at
// the mapped points (Sec. 2.4.1, eq. discrete-inner).  The clip buffers are
// per-lane arrays, [2 buffers][2 coordinates][cap]; passes that cut nothing
// do not touch them, so only the 1-3 cutting passes of a typical straddling
// point read and write them.

__device__ inline double &cb(double *buf, int cap, int lane, int b, int c, int i)
{
    return buf[((b * 2 + c) * cap + i) + lane];
}

// returns the vertex count; the polygon is left in buffer *which
// Edges of the polygon around (x, y) whose pass can change a polygon derived
// from the triangle (bit j): an edge with every triangle vertex inside by
// 1e-9 C |e| (C bounds the coordinates) cannot, since every point a pass
// produces is a convex combination of the vertices up to rounding many
// orders below that margin, so the plain clip returns its input unchanged
// there.  Skipping those passes gives the same polygon, bit for bit.
__device__ inline uint64_t clip_active(double x, double y, const double vx[3], const double vy[3], const double *dir,
                                       int N, double delta)
{
#pragma clang fp contract(off)
    const double C = fmax(fmax(fmax(fabs(x), fabs(y)), fmax(fabs(vx[0]), fabs(vy[0]))),
                          fmax(fmax(fabs(vx[1]), fabs(vy[1])), fmax(fabs(vx[2]), fabs(vy[2])))) +
                     delta;
    uint64_t act = 0;
    // vertex j + 1 of one edge is vertex j of the next (the same values)
    double qa0 = x + delta * dir[0], qa1 = y + delta * dir[1];
    for (int j = 0; j < N; ++j) {
        const int j1 = j + 1 == N ? 0 : j + 1;
        const double qb0 = x + delta * dir[2 * j1], qb1 = y + delta * dir[2 * j1 + 1];
        const double e0 = qb0 - qa0, e1 = qb1 - qa1;
        const double tol = 1e-9 * C * (fabs(e0) + fabs(e1));
        const double d0 = e0 * (vy[0] - qa1) - e1 * (vx[0] - qa0);
        const double d1 = e0 * (vy[1] - qa1) - e1 * (vx[1] - qa0);
        const double d2 = e0 * (vy[2] - qa1) - e1 * (vx[2] - qa0);
        if (!(d0 > tol && d1 > tol && d2 > tol)) act |= 1ull << j;
        qa0 = qb0;
        qa1 = qb1;
    }
    return act;
}

__device__ inline int clip_polygon(double x, double y, const double vx[3], const double vy[3], const double *dir, int N,
                            double delta, double *buf, int cap, int lane, int *which, bool *ovf)
{
#pragma clang fp contract(off)
    for (int k = 0; k < 3; ++k) {
        cb(buf, cap, lane, 0, 0, k) = vx[k];
        cb(buf, cap, lane, 0, 1, k) = vy[k];
    }
    const uint64_t act = clip_active(x, y, vx, vy, dir, N, delta);
    int cnt = 3, cur = 0;
    for (uint64_t rest = act; rest && cnt > 0; rest &= rest - 1) {
        const int j = __ffsll((unsigned long long)rest) - 1;
        const int j1 = j + 1 == N ? 0 : j + 1;
        const double qa0 = x + delta * dir[2 * j], qa1 = y + delta * dir[2 * j + 1];
        const double qb0 = x + delta * dir[2 * j1], qb1 = y + delta * dir[2 * j1 + 1];
        const double e0 = qb0 - qa0, e1 = qb1 - qa1;
        // a pass that finds every vertex inside returns the list unchanged
        bool cuts = false;
        for (int i = 0; i < cnt; ++i)
            cuts |= !(e0 * (cb(buf, cap, lane, cur, 1, i) - qa1) - e1 * (cb(buf, cap, lane, cur, 0, i) - qa0) >= 0.0);
        if (!cuts) continue;
        const int nxt = 1 - cur;
        int m = 0;
        for (int i = 0; i < cnt; ++i) {
            const int i1 = i + 1 == cnt ? 0 : i + 1;
            const double p0 = cb(buf, cap, lane, cur, 0, i), p1 = cb(buf, cap, lane, cur, 1, i);
            const double q0 = cb(buf, cap, lane, cur, 0, i1), q1 = cb(buf, cap, lane, cur, 1, i1);
            const double dp = e0 * (p1 - qa1) - e1 * (p0 - qa0);
            const double dq = e0 * (q1 - qa1) - e1 * (q0 - qa0);
            const bool pin = dp >= 0.0, qin = dq >= 0.0;
            if (m + (pin ? 1 : 0) + (pin != qin ? 1 : 0) > cap) {
                *ovf = true;
                return 0;
            }
            if (pin) {
                cb(buf, cap, lane, nxt, 0, m) = p0;
                cb(buf, cap, lane, nxt, 1, m) = p1;
                ++m;
            }
            if (pin != qin) {
                const double t = dp / (dp - dq);
                cb(buf, cap, lane, nxt, 0, m) = p0 + t * (q0 - p0);
                cb(buf, cap, lane, nxt, 1, m) = p1 + t * (q1 - p1);
                ++m;
            }
        }
        cnt = m;
        cur = nxt;
    }
    *which = cur;
    return cnt;
}

// Samples of one straddling outer point xo (weight wo = w_p |J_outer|, basis
// values po) against the inner element; the inner rule is role B of r when
// inner_b, else role A.  outer_e: the outer element is e (rows of X).
template <int KER, typename T>
__device__ __forceinline__ void straddle_point(const FarArgs &a, double xo_x, double xo_y, double wo, const double (&po)[3],
                               int32_t inner, const double2 &v0i, const double4 &Ji, const RoleArgs &r,
                               bool inner_b, bool outer_e, double *buf, int lane, T cc, T z2min,
                               T (&X)[3][3][Ker<KER>::NK], T (&De)[6][Ker<KER>::NK], T (&Df)[6][Ker<KER>::NK],
                               bool *ovf)
{
    constexpr int NK = Ker<KER>::NK;
    double vx[3], vy[3];
    for (int k = 0; k < 3; ++k) {
        const int32_t n = a.E[3 * (int64_t)inner + k];
        vx[k] = a.V[2 * (int64_t)n];
        vy[k] = a.V[2 * (int64_t)n + 1];
    }
    int cur = 0;
    int cnt;
    if (a.caps) {
        double px[kMaxCaps], py[kMaxCaps];
        cnt = caps_polygon(xo_x, xo_y, vx, vy, a.delta, a.caps == 2, px, py);
        for (int i = 0; i < cnt; ++i) {
            cb(buf, a.cap, lane, 0, 0, i) = px[i];
            cb(buf, a.cap, lane, 0, 1, i) = py[i];
        }
    } else {
        cnt = clip_polygon(xo_x, xo_y, vx, vy, a.dir, a.N, a.delta, buf, a.cap, lane, &cur, ovf);
    }
    if (cnt < 3) return;
    const double deti = Ji.x * Ji.w - Ji.y * Ji.z;
    const double rdet = 1.0 / deti;
    const int Q = inner_b ? r.PB : r.PA;
    const double s0x = cb(buf, a.cap, lane, cur, 0, 0), s0y = cb(buf, a.cap, lane, cur, 1, 0);
    const T pe[3] = {(T)po[0], (T)po[1], (T)po[2]};
    for (int s = 1; s + 1 < cnt; ++s) {
        const double s1x = cb(buf, a.cap, lane, cur, 0, s), s1y = cb(buf, a.cap, lane, cur, 1, s);
        const double s2x = cb(buf, a.cap, lane, cur, 0, s + 1), s2y = cb(buf, a.cap, lane, cur, 1, s + 1);
        const double S00 = s1x - s0x, S01 = s2x - s0x, S10 = s1y - s0y, S11 = s2y - s0y;
        const double adet = fabs(S00 * S11 - S01 * S10);
        for (int q = 0; q < Q; ++q) {
            const double x1 = inner_b ? r.xb[q][0] : r.xa[q][0];
            const double x2 = inner_b ? r.xb[q][1] : r.xa[q][1];
            const double wq = inner_b ? r.wb[q] : r.wa[q];
            const double yx = s0x + (S00 * x1 + S01 * x2), yy = s0y + (S10 * x1 + S11 * x2);
            const double dx = yx - v0i.x, dy = yy - v0i.y;
            const double h1 = (Ji.w * dx - Ji.y * dy) * rdet;
            const double h2 = (-Ji.z * dx + Ji.x * dy) * rdet;
            const T pi[3] = {(T)(1.0 - h1 - h2), (T)h1, (T)h2};
            T kv[NK];
            kernel_eval<KER, T>((T)(xo_x - yx), (T)(xo_y - yy), cc, kv, z2min);
            const T w = (T)(wo * wq * adet);
            const T *pr = outer_e ? pe : pi;   // basis of e at its point
            const T *pc = outer_e ? pi : pe;   // basis of f at its point
#pragma unroll
            for (int k = 0; k < NK; ++k) {
                const T hv = w * kv[k];
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) X[i][j][k] -= hv * pr[i] * pc[j];
                De[0][k] += hv * pr[0] * pr[0];
                De[1][k] += hv * pr[0] * pr[1];
                De[2][k] += hv * pr[0] * pr[2];
                De[3][k] += hv * pr[1] * pr[1];
                De[4][k] += hv * pr[1] * pr[2];
                De[5][k] += hv * pr[2] * pr[2];
                Df[0][k] += hv * pc[0] * pc[0];
                Df[1][k] += hv * pc[0] * pc[1];
                Df[2][k] += hv * pc[0] * pc[2];
                Df[3][k] += hv * pc[1] * pc[1];
                Df[4][k] += hv * pc[1] * pc[2];
                Df[5][k] += hv * pc[2] * pc[2];
            }
        }
    }
}

// record of unordered non-touching pair idx
// Record values of one unordered non-touching pair.
template <int KER, typename T>
struct FarAcc {
    static constexpr int NK = Ker<KER>::NK;
    T X[3][3][NK], De[6][NK], Df[6][NK];
    __device__ inline void zero()
    {
#pragma unroll
        for (int k = 0; k < NK; ++k) {
#pragma unroll
            for (int i = 0; i < 9; ++i) X[i / 3][i % 3][k] = 0;
#pragma unroll
            for (int i = 0; i < 6; ++i) De[i][k] = Df[i][k] = 0;
        }
    }
    __device__ inline void add(const FarAcc &o)
    {
#pragma unroll
        for (int k = 0; k < NK; ++k) {
#pragma unroll
            for (int i = 0; i < 9; ++i) X[i / 3][i % 3][k] += o.X[i / 3][i % 3][k];
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                De[i][k] += o.De[i][k];
                Df[i][k] += o.Df[i][k];
            }
        }
    }
};

// points whose ball covers the other element wholly (status 1)
template <int KER, typename T, int PM>
__device__ __forceinline__ void far_whole(const FarArgs &a, const RoleArgs &r1, const RoleArgs &r2, int32_t e,
                                          int32_t f, uint32_t ms, uint32_t mt, FarAcc<KER, T> &acc)
{
    const double2 v0e = a.v0[e], v0f = a.v0[f];
    const double4 Je = a.J[e], Jf = a.J[f];
    const double dete = a.det[e], detf = a.det[f];
    const T dx = (T)(v0e.x - v0f.x), dy = (T)(v0e.y - v0f.y);
    const T cc = (T)a.c;
    acc.zero();
    if (a.same) {
        far_direction<KER, T, PM>(r1, dx, dy, Je, Jf, dete, detf, ms, mt, cc, acc.X, acc.De, acc.Df);
    } else {
        // (e, f): outer rule on e, inner rule on f
        far_direction<KER, T, PM>(r1, dx, dy, Je, Jf, dete, detf, ms, 0u, cc, acc.X, acc.De, acc.Df);
        // (f, e): inner rule on e, outer rule on f
        if (e != f) far_direction<KER, T, PM>(r2, dx, dy, Je, Jf, dete, detf, 0u, mt, cc, acc.X, acc.De, acc.Df);
    }
}

// Contribution of one straddling point (status 2), computed from zero:
// side 0 is outer point p of e against f, side 1 outer point p of f
// against e.  Every path adds these contributions to the pair's values one
// by one in the order (side 0, p ascending), (side 1, p ascending).
template <int KER, typename T>
__device__ __forceinline__ void straddle_item(const FarArgs &a, const RoleArgs &r1, const RoleArgs &r2, int side,
                                              int p, int32_t e, int32_t f, FarAcc<KER, T> &c, bool *ovf)
{
    double clipbuf[2 * 2 * (kMaxPoly + 4)];
    const T cc = (T)a.c;
    const T z2min = Ker<KER>::NZD ? (T)(1e-12 * fmin(a.det[e], a.det[f])) : (T)0;
    c.zero();
    if (side == 0) {
        const double2 xo = a.xp[(int64_t)e * a.P + p];
        const double po[3] = {r1.pa[p][0], r1.pa[p][1], r1.pa[p][2]};
        straddle_point<KER, T>(a, xo.x, xo.y, r1.wa[p] * a.det[e], po, f, a.v0[f], a.J[f], r1, true, true, clipbuf,
                               0, cc, z2min, c.X, c.De, c.Df, ovf);
    } else if (a.same) {   // one rule: both directions use r1
        const double2 xo = a.xp[(int64_t)f * a.P + p];
        const double po[3] = {r1.pb[p][0], r1.pb[p][1], r1.pb[p][2]};
        straddle_point<KER, T>(a, xo.x, xo.y, r1.wb[p] * a.det[f], po, e, a.v0[e], a.J[e], r1, false, false,
                               clipbuf, 0, cc, z2min, c.X, c.De, c.Df, ovf);
    } else {               // the outer rule on f is role B of r2
        const double2 xo = a.xp[(int64_t)f * a.P + p];
        const double po[3] = {r2.pb[p][0], r2.pb[p][1], r2.pb[p][2]};
        straddle_point<KER, T>(a, xo.x, xo.y, r2.wb[p] * a.det[f], po, e, a.v0[e], a.J[e], r2, false, false,
                               clipbuf, 0, cc, z2min, c.X, c.De, c.Df, ovf);
    }
}

// straddling points of a pair: bits p of the two status masks
__device__ inline uint32_t straddle_bits(uint32_t m, int P)
{
    uint32_t b = 0;
    for (int p = 0; p < P; ++p)
        if (((m >> (2 * p)) & 3u) == kStraddle) b |= 1u << p;
    return b;
}

// Record idx (Rec layout over a.n records).  Consecutive lanes hold
// consecutive records, so each chunk store of a wave covers a contiguous
// range.  The self pair (e, e) stores X + X^T in its R chunks and De + Df.
template <int KER, typename T>
__device__ __forceinline__ void far_store(const FarArgs &a, int64_t idx, bool self, const FarAcc<KER, T> &acc)
{
    constexpr int NK = Ker<KER>::NK;
    using L = Rec<NK>;
    T *base = (T *)a.rec;
    const int64_t n = a.n;
#pragma unroll
    for (int loc = 0; loc < 3; ++loc) {
        T *r = base + L::r(loc, idx, n);
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int k = 0; k < NK; ++k) r[b * NK + k] = self ? acc.X[loc][b][k] + acc.X[b][loc][k] : acc.X[loc][b][k];
    }
    if (!self) {
#pragma unroll
        for (int loc = 0; loc < 3; ++loc) {
            T *c = base + L::c(loc, idx, n);
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int k = 0; k < NK; ++k) c[b * NK + k] = acc.X[b][loc][k];
        }
    }
    T *de = base + L::d(idx, n, false), *df = base + L::d(idx, n, true);
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            de[i * NK + k] = self ? acc.De[i][k] + acc.Df[i][k] : acc.De[i][k];
            df[i * NK + k] = self ? (T)0 : acc.Df[i][k];
        }
}

// Records idx0 .. idx0 + nvalid - 1 of one wave (lane lane0 + l holds record
// idx0 + l), through LDS: the wave then stores its block of each record
// array with consecutive lanes at consecutive addresses.  All lanes of the
// wave call it.  slots: kFarStage<NK> values per lane; the six chunk arrays
// and the diagonal blocks pass through it one after the other (a smaller
// buffer leaves LDS for more resident waves).
template <int NK>
constexpr int kFarStage = 18 * NK;
template <int KER, typename T>
__device__ __forceinline__ void far_store_wave(const FarArgs &a, int64_t idx0, int nvalid, bool self,
                                               const FarAcc<KER, T> &acc, T *slots, int lane0 = 0)
{
    constexpr int NK = Ker<KER>::NK, NS = kFarStage<NK>, W = 3 * NK;
    const int hw = threadIdx.x & 63;
    const int lane = hw - lane0;   // position of this lane's record in the run
    const bool mine = lane >= 0 && lane < nvalid;
    T *sl = slots + lane * NS;
    T *base = (T *)a.rec;
    const int64_t n = a.n;
    if (mine) {
        // [R_0 R_1 R_2 C_0 C_1 C_2], the order of the record arrays
#pragma unroll
        for (int loc = 0; loc < 3; ++loc)
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int k = 0; k < NK; ++k) {
                    sl[loc * W + b * NK + k] = self ? acc.X[loc][b][k] + acc.X[b][loc][k] : acc.X[loc][b][k];
                    sl[(3 + loc) * W + b * NK + k] = self ? (T)0 : acc.X[b][loc][k];
                }
    }
    wave_sync();
    for (int p = 0; p < 6; ++p) {
        T *out = base + ((int64_t)p * n + idx0) * W;
        for (int t = hw; t < nvalid * W; t += 64) out[t] = slots[(t / W) * NS + p * W + t % W];
    }
    wave_sync();
    if (mine) {
        // [De | Df]
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int k = 0; k < NK; ++k) {
                sl[i * NK + k] = self ? acc.De[i][k] + acc.Df[i][k] : acc.De[i][k];
                sl[(6 + i) * NK + k] = self ? (T)0 : acc.Df[i][k];
            }
    }
    wave_sync();
    for (int h = 0; h < 2; ++h) {
        T *out = base + Rec<NK>::d(idx0, n, h == 1);
        for (int t = hw; t < nvalid * 2 * W; t += 64) out[t] = slots[(t / (2 * W)) * NS + h * 2 * W + t % (2 * W)];
    }
    wave_sync();
}

// record of unordered non-touching pair idx, one lane alone
template <int KER, typename T, int PM, bool POLY>
__device__ __forceinline__ void far_item(const FarArgs &a, const RoleArgs &r1, const RoleArgs &r2, int64_t idx)
{
    const int32_t e = a.ue[idx], f = a.uf[idx];
    const uint2 mm = a.m[idx];
    const uint32_t ms = mm.x, mt = mm.y;   // mt == 0 for the self pair
    FarAcc<KER, T> acc;
    far_whole<KER, T, PM>(a, r1, r2, e, f, ms, mt, acc);
    if (POLY) {
        bool ovf = false;
        FarAcc<KER, T> c;
        // both masks cover the outer points (a.P) of their element
        const uint32_t b0 = straddle_bits(ms, a.P), b1 = e == f ? 0u : straddle_bits(mt, a.P);
        for (int p = 0; p < kMaxRule; ++p)
            if ((b0 >> p) & 1u) {
                straddle_item<KER, T>(a, r1, r2, 0, p, e, f, c, &ovf);
                acc.add(c);
            }
        for (int p = 0; p < kMaxRule; ++p)
            if ((b1 >> p) & 1u) {
                straddle_item<KER, T>(a, r1, r2, 1, p, e, f, c, &ovf);
                acc.add(c);
            }
        if (ovf) atomicOr(a.err, kErrClip);
    }
    far_store<KER, T>(a, idx, e == f, acc);
}

// The same for the 64 pairs of a one-wave workgroup (polygon ball): the
// straddling points of all pairs are queued in pair order and computed by
// all lanes; each pair then adds its own contributions in queue order, so
// the values are those of far_item.
template <int KER, typename T, int PM>
__device__ __forceinline__ void far_wave_poly(const FarArgs &a, const RoleArgs &r1, const RoleArgs &r2, int64_t idx,
                                              bool active, int32_t *queue, int32_t *pe, int32_t *pf, T *slots)
{
    constexpr int NV = 21 * Ker<KER>::NK;   // values of one record
    const int lane = threadIdx.x & 63;
    int32_t e = 0, f = 0;
    uint32_t ms = 0, mt = 0;
    FarAcc<KER, T> acc;
    acc.zero();
    if (active) {
        e = a.ue[idx];
        f = a.uf[idx];
        const uint2 mm = a.m[idx];
        ms = mm.x;
        mt = mm.y;
        far_whole<KER, T, PM>(a, r1, r2, e, f, ms, mt, acc);
    }
    const uint32_t b0 = active ? straddle_bits(ms, a.P) : 0u;
    const uint32_t b1 = active && e != f ? straddle_bits(mt, a.P) : 0u;
    const int cnt = __popc(b0) + __popc(b1);
    int incl = cnt;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    const int off = incl - cnt, total = __shfl(incl, 63);
    {   // this pair's items: side 0 in point order, then side 1
        int k = off;
        for (int p = 0; p < kMaxRule; ++p)
            if ((b0 >> p) & 1u) queue[k++] = (lane << 5) | p;
        for (int p = 0; p < kMaxRule; ++p)
            if ((b1 >> p) & 1u) queue[k++] = (lane << 5) | 16 | p;
    }
    pe[lane] = e;
    pf[lane] = f;
    wave_sync();
    bool ovf = false;
    for (int r0 = 0; r0 < total; r0 += 64) {
        const int it = r0 + lane;
        if (it < total) {
            const int code = queue[it];
            const int ol = code >> 5;
            FarAcc<KER, T> c;
            straddle_item<KER, T>(a, r1, r2, (code >> 4) & 1, code & 15, pe[ol], pf[ol], c, &ovf);
            T *sl = slots + lane * NV;
#pragma unroll
            for (int k = 0; k < Ker<KER>::NK; ++k) {
#pragma unroll
                for (int i = 0; i < 9; ++i) sl[i * Ker<KER>::NK + k] = c.X[i / 3][i % 3][k];
#pragma unroll
                for (int i = 0; i < 6; ++i) {
                    sl[(9 + i) * Ker<KER>::NK + k] = c.De[i][k];
                    sl[(15 + i) * Ker<KER>::NK + k] = c.Df[i][k];
                }
            }
        }
        wave_sync();
        // the pair's items that fell into this round, in order
        const int lo = max(off, r0), hi = min(off + cnt, r0 + 64);
        for (int it2 = lo; it2 < hi; ++it2) {
            const T *sl = slots + (it2 - r0) * NV;
            FarAcc<KER, T> c;
#pragma unroll
            for (int k = 0; k < Ker<KER>::NK; ++k) {
#pragma unroll
                for (int i = 0; i < 9; ++i) c.X[i / 3][i % 3][k] = sl[i * Ker<KER>::NK + k];
#pragma unroll
                for (int i = 0; i < 6; ++i) {
                    c.De[i][k] = sl[(9 + i) * Ker<KER>::NK + k];
                    c.Df[i][k] = sl[(15 + i) * Ker<KER>::NK + k];
                }
            }
            acc.add(c);
        }
        wave_sync();
    }
    if (ovf) atomicOr(a.err, kErrClip);
    if (active) far_store<KER, T>(a, idx, e == f, acc);
}

// ------------------------------------------------- phase 1: touching pairs

struct TouchArgs {
    int64_t n;
    const int32_t *te, *tf;
    const int32_t *E;
    const double *V;
    double *rec;
    int32_t stride;
    double c;
};

// 1-D Gauss rule on [0, 1] as the touching-pair loops read it (in LDS
// where the caller staged it)
struct GaussView {
    const double *x, *w;
    int n;
};

// accumulate w * Psi(z) (g g^T) into the packed upper triangle of L, but
// only the rows and columns of the first NU - 1 nodes: the basis
// differences g of every sample sum to zero over the nodes, so the last
// node's rows follow from the others (touch_last_node)
template <int KER, int NU>
__device__ inline void acc_sample(double *L, double w, double zx, double zy, const double *g, double c)
{
    constexpr int NC = Ker<KER>::NC;
    constexpr int D = NU * NC;
    constexpr int DC = D - NC;
    double k[3];
    kernel_eval<KER, double>(zx, zy, c, k);
    double wk[2][2];
    if (NC == 1) {
        wk[0][0] = w * k[0];
    } else {
        wk[0][0] = w * k[0];
        wk[0][1] = wk[1][0] = w * k[1];
        wk[1][1] = w * k[2];
    }
#pragma unroll
    for (int r = 0; r < DC; ++r) {
        const double gr = g[r / NC];
#pragma unroll
        for (int s = r; s < DC; ++s) L[sym_index(r, s, D)] += (gr * wk[r % NC][s % NC]) * g[s / NC];
    }
}

// the rows of the last node from the zero sums over the nodes:
// L[(last, c), (v, d)] = -sum over u < last of L[(u, c), (v, d)]
template <int NC, int NU>
__device__ inline void touch_last_node(double *L)
{
    constexpr int D = NU * NC;
    constexpr int DC = D - NC;
#pragma unroll
    for (int r = 0; r < DC; ++r)
#pragma unroll
        for (int d = 0; d < NC; ++d) {
            double v = 0.0;
#pragma unroll
            for (int u = 0; u < NU - 1; ++u) v -= L[sym_index(r, u * NC + d, D)];
            L[sym_index(r, DC + d, D)] = v;
        }
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int d = c; d < NC; ++d) {
            double v = 0.0;
#pragma unroll
            for (int u = 0; u < NU - 1; ++u) v -= L[sym_index(u * NC + c, DC + d, D)];
            L[sym_index(DC + c, DC + d, D)] = v;
        }
}

// lanes per touching pair: the vertex class (2n^3 points) runs in groups of
// 8, so a launch holds fewer, longer waves and the gathers that start each
// wave are paid less often; the others in groups of 16.  The grouping fixes
// the order of the sums, so every path uses this one.
__host__ __device__ constexpr int touch_lanes(int cls) { return cls == 1 ? 8 : 16; }

// record of touching pair `pair` of class CLS, computed by the G lanes
// sub = 0..G-1 of an aligned lane group (all of them must call)
template <int KER, int CLS, int G>
__device__ __forceinline__ void touch_item(const TouchArgs &a, const GaussView &g, int64_t pair, int sub)
{
    constexpr int NC = Ker<KER>::NC;
    constexpr int NU = CLS == 3 ? 3 : CLS == 2 ? 4 : 5;
    constexpr int D = NU * NC;
    constexpr int NP = D * (D + 1) / 2;
    const int32_t e = a.te[pair], f = a.tf[pair];
    const int32_t ek[3] = {a.E[3 * (int64_t)e], a.E[3 * (int64_t)e + 1], a.E[3 * (int64_t)e + 2]};
    const int32_t el[3] = {a.E[3 * (int64_t)f], a.E[3 * (int64_t)f + 1], a.E[3 * (int64_t)f + 2]};
    int32_t nd[5];
    touch_frame(CLS, ek, el, nd);
    double L[NP];
#pragma unroll
    for (int t = 0; t < NP; ++t) L[t] = 0.0;
    const int n = g.n;
    double scale;
    if (CLS == 3) {
        const double2 p0 = vtx(a.V, nd[0]), p1 = vtx(a.V, nd[1]), p2 = vtx(a.V, nd[2]);
        const double J00 = p1.x - p0.x, J01 = p2.x - p0.x, J10 = p1.y - p0.y, J11 = p2.y - p0.y;
        const double det = fabs(J00 * J11 - J01 * J10);
        // point ev = j n + iu; the indices advance by G without divisions
        int j = sub / n, iu = sub - (sub / n) * n;
        for (int ev = sub; ev < 6 * n; ev += G) {
            // hexagon corners (1,0),(0,1),(-1,1),(-1,0),(0,-1),(1,-1)
            const int j1 = j == 5 ? 0 : j + 1;
            const double cx0 = j == 0 || j == 5 ? 1.0 : (j == 2 || j == 3 ? -1.0 : 0.0);
            const double cy0 = j == 1 || j == 2 ? 1.0 : (j == 4 || j == 5 ? -1.0 : 0.0);
            const double cx1 = j1 == 0 || j1 == 5 ? 1.0 : (j1 == 2 || j1 == 3 ? -1.0 : 0.0);
            const double cy1 = j1 == 1 || j1 == 2 ? 1.0 : (j1 == 4 || j1 == 5 ? -1.0 : 0.0);
            const double u = g.x[iu];
            const double wx = (1.0 - u) * cx0 + u * cx1;
            const double wy = (1.0 - u) * cy0 + u * cy1;
            // phi(x^) - phi(x^ + z) = -grad phi . z, z = rho w
            const double gg[3] = {wx + wy, -wx, -wy};
            acc_sample<KER, 3>(L, g.w[iu], J00 * wx + J01 * wy, J10 * wx + J11 * wy, gg, a.c);
            iu += G;
            while (iu >= n) {
                iu -= n;
                ++j;
            }
        }
        constexpr int d = Ker<KER>::D;
        scale = det * det / (double)((d + 2) * (d + 3) * (d + 4));
    } else if (CLS == 2) {
        const double2 q0 = vtx(a.V, nd[0]), q1 = vtx(a.V, nd[1]), qa = vtx(a.V, nd[2]), qb = vtx(a.V, nd[3]);
        // x - y = E v,  E = [P1 - P0, A - P0, -(B - P0)]
        const double E0x = q1.x - q0.x, E0y = q1.y - q0.y;
        const double E1x = qa.x - q0.x, E1y = qa.y - q0.y;
        const double E2x = -(qb.x - q0.x), E2y = -(qb.y - q0.y);
        // faces of the cone {max(v2 + v1+, v3 + v1-) <= 1} are unrolled at
        // compile time; the lanes of the group share the n^2 points of each
        // face (a data-dependent face index miscompiled here once: keep it
        // out of divergent control flow)
#pragma unroll
        for (int face = 0; face < 4; ++face) {
            int ip = sub / n, iq = sub - (sub / n) * n;
            for (int ev = sub; ev < n * n; ev += G) {
                const double p = g.x[ip], q = g.x[iq];
                const double u = 1.0 - p, t = u * q;
                const double w0 = face < 2 ? p : -p;
                const double w1 = face == 0 ? u : face == 1 ? t : face == 2 ? 1.0 : q;
                const double w2 = face == 0 ? q : face == 1 ? 1.0 : face == 2 ? t : u;
                const double jf = (face == 1 || face == 2) ? u : 1.0;
                const double gg[4] = {-w0 - w1 + w2, w0, w1, -w2};
                acc_sample<KER, 4>(L, g.w[ip] * g.w[iq] * jf, E0x * w0 + E1x * w1 + E2x * w2,
                                   E0y * w0 + E1y * w1 + E2y * w2, gg, a.c);
                iq += G;
                while (iq >= n) {
                    iq -= n;
                    ++ip;
                }
            }
        }
        const double detk = fabs(E0x * E1y - E1x * E0y), detl = fabs(E0x * E2y - E2x * E0y);
        constexpr int d = Ker<KER>::D;
        scale = detk * detl / (double)((d + 3) * (d + 4));
    } else {
        const double2 q0 = vtx(a.V, nd[0]), a1 = vtx(a.V, nd[1]), a2 = vtx(a.V, nd[2]);
        const double2 b1 = vtx(a.V, nd[3]), b2 = vtx(a.V, nd[4]);
        const double A1x = a1.x - q0.x, A1y = a1.y - q0.y, A2x = a2.x - q0.x, A2y = a2.y - q0.y;
        const double B1x = b1.x - q0.x, B1y = b1.y - q0.y, B2x = b2.x - q0.x, B2y = b2.y - q0.y;
        int iw = sub / (n * n), ia = (sub - iw * n * n) / n, ib = sub - iw * n * n - ia * n;
        for (int ev = sub; ev < n * n * n; ev += G) {
            const double w = g.x[iw], al = g.x[ia], be = g.x[ib];
            const double ex = (1.0 - al) * A1x + al * A2x, ey = (1.0 - al) * A1y + al * A2y;
            const double fx = (1.0 - be) * B1x + be * B2x, fy = (1.0 - be) * B1y + be * B2y;
            const double wt = g.w[iw] * g.w[ia] * g.w[ib] * w;
            {   // region t <= s: t = s w
                const double gg[5] = {w - 1.0, 1.0 - al, al, -w * (1.0 - be), -w * be};
                acc_sample<KER, 5>(L, wt, ex - w * fx, ey - w * fy, gg, a.c);
            }
            {   // region s <= t: s = t w
                const double gg[5] = {1.0 - w, w * (1.0 - al), w * al, -(1.0 - be), -be};
                acc_sample<KER, 5>(L, wt, w * ex - fx, w * ey - fy, gg, a.c);
            }
            ib += G;
            while (ib >= n) {
                ib -= n;
                ++ia;
            }
            while (ia >= n) {
                ia -= n;
                ++iw;
            }
        }
        const double detk = fabs(A1x * A2y - A2x * A1y), detl = fabs(B1x * B2y - B2x * B1y);
        constexpr int d = Ker<KER>::D;
        scale = detk * detl / (double)(d + 4);
    }
    constexpr int DC = D - NC;
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1)
#pragma unroll
        for (int r = 0; r < DC; ++r)
#pragma unroll
            for (int s = r; s < DC; ++s) {
                const int t = sym_index(r, s, D);
                L[t] += __shfl_xor(L[t], off, G);
            }
    touch_last_node<NC, NU>(L);
    double *out = a.rec + pair * a.stride;
#pragma unroll
    for (int t = 0; t < NP; ++t)
        if (t % G == sub) out[t] = scale * L[t];
}

// ------------------------------------------ phase 1b: element diagonals
// D_e = sum over the non-touching pairs of e of the element-diagonal part of
// their records (De when e is the first element, Df when it is the second).
// One wave per element; the rows then add D_e once per element.

struct DiagArgs {
    int64_t K;
    const int64_t *sptr;
    const int32_t *snbr;
    const uint8_t *sflag;
    const int32_t *srec;
    const void *far_rec;
    int32_t far_stride;
    int64_t n_far;
    double *dsum;
    int32_t *err;
    SpecGate gate;
    MatArgs mat;   // label-dependent kernel: e's block of pair (e, f) scaled by c[m(e)][m(f)]
    MomArgs mom;   // mom.on: the blocks from the masks, no records
};

// D_e of element e by the kDiagG lanes sub = 0..kDiagG-1 of an aligned lane
// group (all of them call).  Lane sub adds the entries sub, sub + kDiagG, ...
// of S(e) in that order, kDiagU of them with their loads in flight at once,
// then the group sums by shuffles; the grouping fixes the order of the sums,
// so every path uses these constants.
constexpr int kDiagG = 32;
constexpr int kDiagU = 4;
// the moment form reads 16 bytes per entry and reduces more values: groups
// of 16 lanes, each with more entries (8: 1.52 ms, 4: 1.74 ms, 16: 1.47 ms
// for the diagonal sums of the 64-problem batch)
constexpr int kDiagGMom = 16;
template <bool MOM>
constexpr int diag_group() { return MOM ? kDiagGMom : kDiagG; }

// The same from the masks (a.mom.on, scalar): per outer point p the lanes sum
// A_p = coef(e, f) |J_f| over the entries whose me has p set, and
// B = coef(e, f) |J_f| T_O(mf); the group reduces them, and
// D_e = c |J_e| (W_I sum_p A_p w_p phi(x_p) phi(x_p)^T + Q_I B).
__device__ __forceinline__ void diag_item_mom(const DiagArgs &a, int64_t e, int sub)
{
    constexpr int G = kDiagGMom;
    const MomArgs &m = a.mom;
    double A[kMomP], B = 0.0;
#pragma unroll
    for (int p = 0; p < kMomP; ++p) A[p] = 0.0;
    bool bad = false;
    const int64_t s0 = a.sptr[e], s1 = a.sptr[e + 1];
    for (int64_t t0 = s0 + sub; t0 < s1; t0 += G * kDiagU) {
        int32_t u[kDiagU], f[kDiagU];
        bool use[kDiagU];
#pragma unroll
        for (int k = 0; k < kDiagU; ++k) {
            const int64_t t = t0 + (int64_t)k * G;
            use[k] = t < s1 && ((a.sflag[t] >> 2) & 3) == 0;
            u[k] = use[k] ? a.srec[t] : 0;
            f[k] = use[k] ? a.snbr[t] : 0;
        }
        uint32_t me[kDiagU], mf[kDiagU];
        double w[kDiagU];
#pragma unroll
        for (int k = 0; k < kDiagU; ++k) {
            me[k] = mf[k] = 0u;
            w[k] = 0.0;
            if (!use[k]) continue;
            if (u[k] < 0 || u[k] >= a.n_far) {
                bad = true;
                continue;
            }
            entry_masks(m, u[k], (int32_t)e, f[k], me[k], mf[k]);
            w[k] = m.det[f[k]];
            if (a.mat.n) w[k] *= a.mat.coef((int32_t)e, f[k]);
        }
#pragma unroll
        for (int k = 0; k < kDiagU; ++k) {
            double to = 0.0;
#pragma unroll
            for (int p = 0; p < kMomP; ++p) {
                if (p < m.P) {
                    A[p] = fma(w[k], whole_bit(me[k], p), A[p]);
                    to = fma(whole_bit(mf[k], p), m.wo[p], to);
                }
            }
            B = fma(w[k], to, B);
        }
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
#pragma unroll
        for (int p = 0; p < kMomP; ++p)
            if (p < m.P) A[p] += __shfl_xor(A[p], o, G);
        B += __shfl_xor(B, o, G);
    }
    if (bad) atomicOr(a.err, kErrSlot);
    const double ce = m.c * m.det[e];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double q = 0.0;
#pragma unroll
        for (int p = 0; p < kMomP; ++p)
            if (p < m.P) q = fma(A[p], m.qo[p][i], q);
        if (i % G == sub) a.dsum[e * 6 + i] = ce * (m.wi * q + m.qi[i] * B);
    }
}

template <int NK, typename TR, bool MOM = false>
__device__ __forceinline__ void diag_item(const DiagArgs &a, int64_t e, int sub)
{
    static_assert(!MOM || NK == 1, "the moment form is scalar");
    if constexpr (MOM) {
        diag_item_mom(a, e, sub);
        return;
    }
    constexpr int G = kDiagG;
    double acc[6 * NK];
#pragma unroll
    for (int i = 0; i < 6 * NK; ++i) acc[i] = 0.0;
    bool bad = false;
    const int64_t s0 = a.sptr[e], s1 = a.sptr[e + 1];
    for (int64_t t0 = s0 + sub; t0 < s1; t0 += G * kDiagU) {
        int32_t u[kDiagU], f[kDiagU];
        bool use[kDiagU];
#pragma unroll
        for (int k = 0; k < kDiagU; ++k) {
            const int64_t t = t0 + (int64_t)k * G;
            use[k] = t < s1 && ((a.sflag[t] >> 2) & 3) == 0;
            u[k] = use[k] ? a.srec[t] : 0;
            f[k] = use[k] ? a.snbr[t] : 0;
        }
#pragma unroll
        for (int k = 0; k < kDiagU; ++k) {
            if (!use[k]) continue;
            if (u[k] < 0 || u[k] >= a.n_far) {
                bad = true;
                continue;
            }
            const TR *r = (const TR *)a.far_rec + Rec<NK>::d(u[k], a.n_far, f[k] < e);
            if (a.mat.n == 0) {
#pragma unroll
                for (int i = 0; i < 6 * NK; ++i) acc[i] += (double)r[i];
            } else {
                const double cf = a.mat.coef((int32_t)e, f[k]);
#pragma unroll
                for (int i = 0; i < 6 * NK; ++i) acc[i] += cf * (double)r[i];
            }
        }
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1)
#pragma unroll
        for (int i = 0; i < 6 * NK; ++i) acc[i] += __shfl_xor(acc[i], o, G);
    if (bad) atomicOr(a.err, kErrSlot);
#pragma unroll
    for (int i = 0; i < 6 * NK; ++i)
        if (i % G == sub) a.dsum[e * 6 * NK + i] = acc[i];
}

// ------------------------------------------------- phase 2: row gather
//
// One wave per degree-of-freedom node.  The wave maps the row's column ids to
// positions through an LDS hash table, accumulates the row in LDS and writes
// it once.  The work items are the entries (e, f) of the neighbour lists S(e)
// of the elements e around the node.  Each lane takes kRowU entries per step
// and issues all their loads (list entry, then vertices of f and record
// values) before it adds any of them, so the dependent global loads of a
// step overlap instead of forming one chain per entry.

struct RowArgs {
    int64_t nrows;
    const int32_t *rows;     // dof nodes
    const int64_t *nptr;
    const int32_t *ncol;
    const int64_t *ne_ptr;
    const int32_t *ne_list;
    const int32_t *E;
    const int64_t *sptr;
    const int4 *snode;       // (f, vertices of f) per neighbour-list entry
    const uint8_t *sflag;
    const int32_t *srec;
    const void *far_rec;
    int32_t far_stride;
    int64_t n_far;
    const double *dsum;
    const double *touch_rec;
    int32_t touch_stride;
    int64_t n_touch;
    int32_t hcap;        // power of two, >= 2 * longest row
    int32_t maxlen;
    double *val;
    int32_t *err;
    SpecGate gate;
    // label-dependent kernel: the block (rows e, columns f) of a
    // non-touching pair scaled by c[m(f)][m(e)]; touching records by
    // c[m(e)][m(f)] (a symmetric table), or, with a non-symmetric table, edge
    // and vertex records in the discontinuous form folded per column
    MatArgs mat;
    int32_t nonsym;
    MomArgs mom;   // mom.on: far entries from the masks (row_item<1, TR, true>), no records
};

constexpr int kRowQ = 64;   // elements around a node per batch (one per lane)
constexpr int kRowU = 4;    // neighbour-list entries per lane per step

__device__ inline int hpos(const int32_t *hk, const int32_t *hv, int32_t mask, int32_t key)
{
    uint32_t h = ((uint32_t)key * 2654435761u) & (uint32_t)mask;
    for (int probe = 0; probe <= mask; ++probe) {
        const int32_t k = hk[h];
        if (k == key) return hv[h];
        if (k < 0) return -1;
        h = (h + 1) & (uint32_t)mask;
    }
    return -1;
}

template <int NC>
__device__ inline void add_sym_block(double *acc, int pos, const double *v)
{
    if (NC == 1) {
        atomicAdd(&acc[pos], v[0]);
    } else {
        atomicAdd(&acc[pos * 4 + 0], v[0]);
        atomicAdd(&acc[pos * 4 + 1], v[1]);
        atomicAdd(&acc[pos * 4 + 2], v[1]);
        atomicAdd(&acc[pos * 4 + 3], v[2]);
    }
}

__device__ inline int32_t pick3(int i, int32_t x0, int32_t x1, int32_t x2)
{
    return i == 0 ? x0 : (i == 1 ? x1 : x2);
}

// The vertex order of touch_frame, on scalars (a: first element of the
// ordered pair, b: second); unused slots are -1.
struct Frame {
    int32_t n0, n1, n2, n3, n4;
    int nu;
};

__device__ inline Frame frame_of(int cls, int32_t a0, int32_t a1, int32_t a2, int32_t b0, int32_t b1,
                                 int32_t b2)
{
    if (cls == 3) return Frame{a0, a1, a2, -1, -1, 3};
    if (cls == 2) {
        const bool i0 = a0 == b0 || a0 == b1 || a0 == b2;
        const bool i1 = a1 == b0 || a1 == b1 || a1 == b2;
        const int32_t s0 = !i0 ? a1 : a0;
        const int32_t s1 = (!i0 || !i1) ? a2 : a1;
        const int32_t A = !i0 ? a0 : (!i1 ? a1 : a2);
        const bool j0 = b0 == a0 || b0 == a1 || b0 == a2;
        const bool j1 = b1 == a0 || b1 == a1 || b1 == a2;
        const int32_t B = !j0 ? b0 : (!j1 ? b1 : b2);
        return Frame{min(s0, s1), max(s0, s1), A, B, -1, 4};
    }
    const int32_t av[3] = {a0, a1, a2}, bv[3] = {b0, b1, b2};
    int ia = 0, ib = 0;
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int y = 0; y < 3; ++y)
            if (av[x] == bv[y]) {
                ia = x;
                ib = y;
            }
    const int ia1 = ia == 2 ? 0 : ia + 1, ia2 = ia == 0 ? 2 : ia - 1;
    const int ib1 = ib == 2 ? 0 : ib + 1, ib2 = ib == 0 ? 2 : ib - 1;
    return Frame{pick3(ia, a0, a1, a2), pick3(ia1, a0, a1, a2), pick3(ia2, a0, a1, a2),
                 pick3(ib1, b0, b1, b2), pick3(ib2, b0, b1, b2), 5};
}

// Row i's share of a touching pair: factor * (row rr of L) over the frame
// nodes, rr the frame slot of i.
template <int NC>
__device__ inline bool add_touch(double *acc, const int32_t *hk, const int32_t *hv, int32_t mask, int32_t i,
                                 int cls, int32_t e, int32_t f, int32_t e0, int32_t e1, int32_t e2,
                                 int32_t f0, int32_t f1, int32_t f2, const double *L, double scale)
{
    constexpr int NN = NC * NC;
    const bool first = e <= f;
    const Frame fr = first ? frame_of(cls, e0, e1, e2, f0, f1, f2) : frame_of(cls, f0, f1, f2, e0, e1, e2);
    const int32_t nodes[5] = {fr.n0, fr.n1, fr.n2, fr.n3, fr.n4};
    int rr = 0;
#pragma unroll
    for (int c = 0; c < 5; ++c)
        if (nodes[c] == i) rr = c;
    const bool ine = e0 == i || e1 == i || e2 == i;
    const bool inf = f0 == i || f1 == i || f2 == i;
    const double factor = ((cls == 3 || (ine && inf)) ? 1.0 : 2.0) * scale;
    const int D = fr.nu * NC;
    bool ok = true;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        if (c >= fr.nu) break;
        const int pc = hpos(hk, hv, mask, nodes[c]);
        if (pc < 0) {
            ok = false;
            continue;
        }
#pragma unroll
        for (int cc = 0; cc < NC; ++cc)
#pragma unroll
            for (int dd = 0; dd < NC; ++dd)
                atomicAdd(&acc[pc * NN + cc * NC + dd], factor * L[sym_index(rr * NC + cc, c * NC + dd, D)]);
    }
    return ok;
}

// Row i's share of an edge or vertex touching pair in the discontinuous form
// (non-symmetric material table): L is the packed symmetric 6n x 6n matrix
// over [stored vertices of the smaller element p | of the larger q] with the
// plain kernel; the pair's continuous matrix is P^T L S P with P folding the
// six slots onto their nodes and S scaling the columns of p by c[m(p)][m(q)]
// and those of q by c[m(q)][m(p)] (the element holding x first).  Row i is the
// sum of the rows of its slots; factor as in add_touch.
template <int NC>
__device__ inline bool add_touch_dg(double *acc, const int32_t *hk, const int32_t *hv, int32_t mask, int32_t i,
                                    int32_t e, int32_t f, int32_t e0, int32_t e1, int32_t e2, int32_t f0,
                                    int32_t f1, int32_t f2, const double *L, double cpq, double cqp)
{
    constexpr int NN = NC * NC;
    constexpr int D = 6 * NC;
    const bool first = e < f;
    const int32_t nd[6] = {first ? e0 : f0, first ? e1 : f1, first ? e2 : f2,
                           first ? f0 : e0, first ? f1 : e1, first ? f2 : e2};
    int rp = -1, rq = -1;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (nd[c] == i) rp = c;
        if (nd[3 + c] == i) rq = 3 + c;
    }
    const double factor = rp >= 0 && rq >= 0 ? 1.0 : 2.0;
    bool ok = true;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const int pc = hpos(hk, hv, mask, nd[c]);
        if (pc < 0) {
            ok = false;
            continue;
        }
        const double sc = factor * (c < 3 ? cpq : cqp);
#pragma unroll
        for (int cc = 0; cc < NC; ++cc)
#pragma unroll
            for (int dd = 0; dd < NC; ++dd) {
                double v = 0.0;
                if (rp >= 0) v += L[sym_index(rp * NC + cc, c * NC + dd, D)];
                if (rq >= 0) v += L[sym_index(rq * NC + cc, c * NC + dd, D)];
                atomicAdd(&acc[pc * NN + cc * NC + dd], sc * v);
            }
    }
    return ok;
}

// LDS of one row gather besides the dynamic part (accumulator, hash table)
// touching entries of a row are queued and then handled by all lanes at once
// (they take a longer path than the non-touching ones)
constexpr int kRowTouchCap = 320;

struct RowShared {
    int64_t qs[kRowQ];
    int32_t pre[kRowQ + 1], qe[kRowQ], qloc[kRowQ], qn[kRowQ][3], qp[kRowQ][3];
    int32_t tt[kRowTouchCap];   // queued touching entries: list index and element slot
    uint8_t tq[kRowTouchCap];
};
// moment form, LDS of kRowMom doubles beside RowShared: the sums M_O over
// the set bits of each 4-bit index of the two nibbles of a mask,
// [nibble][index][a], then M_I
constexpr int kRowMomLut = 2 * 16 * 3;
constexpr int kRowMom = kRowMomLut + 3;

// adds the queued touching entries of row i (element slots of the current batch)
template <int NC>
__device__ inline bool flush_touch(const RowArgs &a, RowShared &sh, int ntouch, int64_t i, double *acc,
                                   const int32_t *hk, const int32_t *hv, int32_t mask, int lane)
{
    bool ok = true;
    for (int j = lane; j < ntouch; j += 64) {
        const int32_t t = sh.tt[j];
        const int q = sh.tq[j];
        const int4 sn = a.snode[t];
        const int cls = (a.sflag[t] >> 2) & 3;
        const int32_t u = a.srec[t];
        if (u < 0 || u >= a.n_touch) {
            ok = false;
            continue;
        }
        const double *L = a.touch_rec + (int64_t)u * a.touch_stride;
        const int32_t e = sh.qe[q], f = sn.x;
        if (a.nonsym && cls != 3) {
            const int32_t p = min(e, f), r = max(e, f);
            if (!add_touch_dg<NC>(acc, hk, hv, mask, (int32_t)i, e, f, sh.qn[q][0], sh.qn[q][1], sh.qn[q][2], sn.y,
                                  sn.z, sn.w, L, a.mat.coef(p, r), a.mat.coef(r, p)))
                ok = false;
        } else {
            // identical pairs and symmetric tables: one coefficient per pair
            const double scale = a.mat.n == 0 ? 1.0 : a.mat.coef(e, f);
            if (!add_touch<NC>(acc, hk, hv, mask, (int32_t)i, cls, e, f, sh.qn[q][0], sh.qn[q][1], sh.qn[q][2],
                               sn.y, sn.z, sn.w, L, scale))
                ok = false;
        }
    }
    return ok;
}

// dynamic LDS bytes of one row gather
inline size_t row_lds_bytes(int64_t maxlen, int nc, int hcap)
{
    return sizeof(double) * (size_t)maxlen * nc * nc + sizeof(int32_t) * 2 * (size_t)hcap;
}

// row of dof node i by the 64 lanes of a one-wave workgroup; smem holds
// row_lds_bytes(a.maxlen, NC, a.hcap) bytes
template <int NC, typename TR, bool MOM = false>
__device__ __forceinline__ void row_item(const RowArgs &a, int64_t i, unsigned char *smem, RowShared &sh,
                                         double *mq = nullptr)
{
    static_assert(!MOM || NC == 1, "the moment form is scalar");
    constexpr int NN = NC * NC;
    constexpr int NK = NC == 1 ? 1 : 3;
    double *acc = (double *)smem;                              // [maxlen * NN]
    int32_t *hk = (int32_t *)(acc + (size_t)a.maxlen * NN);    // [hcap]
    int32_t *hv = hk + a.hcap;                                 // [hcap]
    int64_t *qs = sh.qs;
    int32_t *pre = sh.pre, *qe = sh.qe, *qloc = sh.qloc;
    int32_t (*qn)[3] = sh.qn;
    int32_t (*qp)[3] = sh.qp;
    const int lane = threadIdx.x;
    const int32_t mask = a.hcap - 1;
    {
        const int64_t s = a.nptr[i];
        const int len = (int)(a.nptr[i + 1] - s);
        if (len == 0) return;
        if constexpr (MOM) {
            for (int t = lane; t < kRowMom; t += 64) {
                const int n = t / 48, idx = (t / 3) % 16, b = t % 3;
                double v = 0.0;
                if (t >= kRowMomLut) {
                    v = a.mom.mi[t - kRowMomLut];
                } else {
                    for (int j = 0; j < 4; ++j)
                        if (((idx >> j) & 1) && 4 * n + j < a.mom.P) v += a.mom.mo[4 * n + j][b];
                }
                mq[t] = v;
            }
        }
        for (int t = lane; t < a.hcap; t += 64) hk[t] = -1;
        for (int t = lane; t < len * NN; t += 64) acc[t] = 0.0;
        __syncthreads();
        for (int t = lane; t < len; t += 64) {
            const int32_t key = a.ncol[s + t];
            uint32_t h = ((uint32_t)key * 2654435761u) & (uint32_t)mask;
            for (int probe = 0; probe <= mask; ++probe) {
                if (atomicCAS(&hk[h], -1, key) == -1) {
                    hv[h] = t;
                    break;
                }
                h = (h + 1) & (uint32_t)mask;
            }
        }
        __syncthreads();
        bool bad = false;
        const int64_t q0 = a.ne_ptr[i], q1 = a.ne_ptr[i + 1];
        for (int64_t qb = q0; qb < q1; qb += kRowQ) {
            const int nq = (int)min((int64_t)kRowQ, q1 - qb);
            int cnt = 0;
            if (lane < nq) {
                // the elements around the node: id, local index of the node,
                // vertex ids and their column positions
                const int32_t e = a.ne_list[qb + lane];
                const int32_t v0 = a.E[3 * (int64_t)e], v1 = a.E[3 * (int64_t)e + 1], v2 = a.E[3 * (int64_t)e + 2];
                const int64_t se0 = a.sptr[e], se1 = a.sptr[e + 1];
                qe[lane] = e;
                qs[lane] = se0;
                qn[lane][0] = v0;
                qn[lane][1] = v1;
                qn[lane][2] = v2;
                const int p0 = hpos(hk, hv, mask, v0), p1 = hpos(hk, hv, mask, v1), p2 = hpos(hk, hv, mask, v2);
                qp[lane][0] = p0;
                qp[lane][1] = p1;
                qp[lane][2] = p2;
                const int loc = v0 == (int32_t)i ? 0 : v1 == (int32_t)i ? 1 : 2;
                qloc[lane] = loc;
                cnt = (int)(se1 - se0);
                if (cnt > 0) {
                    // summed element-diagonal block of e's non-touching pairs, row loc
                    const double *dv = a.dsum + (int64_t)e * 6 * NK;
                    const int pb[3] = {p0, p1, p2};
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        if (pb[b] < 0) {
                            bad = true;
                            continue;
                        }
                        double ds[NK];
#pragma unroll
                        for (int k = 0; k < NK; ++k) ds[k] = dv[sym_index(loc, b, 3) * NK + k];
                        add_sym_block<NC>(acc, pb[b], ds);
                    }
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
            __syncthreads();
            int ntouch = 0;
            // the element q with pre[q] <= flat < pre[q + 1]: a lane's flat
            // index only grows, so q advances from where it stopped
            int qcur = 0;
            for (int base = 0; base < total; base += 64 * kRowU) {
                int32_t fe[kRowU], uu[kRowU], qq[kRowU], cl[kRowU], nf0[kRowU], nf1[kRowU], nf2[kRowU], tt[kRowU];
                bool act[kRowU];
                TR xv[MOM ? 1 : kRowU][3][NK];
                uint32_t me[MOM ? kRowU : 1], mf[MOM ? kRowU : 1];
                double dv[MOM ? kRowU : 1];
#pragma unroll
                for (int k = 0; k < kRowU; ++k) {
                    const int flat = base + k * 64 + lane;
                    act[k] = flat < total;
                    fe[k] = 0;
                    nf0[k] = nf1[k] = nf2[k] = -1;
                    uu[k] = -1;
                    cl[k] = 0;
                    qq[k] = 0;
                    if (act[k]) {
                        while (qcur + 1 < nq && pre[qcur + 1] <= flat) ++qcur;
                        const int lo = qcur;
                        qq[k] = lo;
                        const int64_t t = qs[lo] + (flat - pre[lo]);
                        tt[k] = (int32_t)t;
                        const int4 sn = a.snode[t];
                        fe[k] = sn.x;
                        nf0[k] = sn.y;
                        nf1[k] = sn.z;
                        nf2[k] = sn.w;
                        cl[k] = (a.sflag[t] >> 2) & 3;
                        uu[k] = a.srec[t];
                    }
                }
#pragma unroll
                for (int k = 0; k < kRowU; ++k) {
                    if (!act[k]) continue;
                    if (uu[k] < 0 || uu[k] >= (cl[k] == 0 ? a.n_far : a.n_touch)) {
                        bad = true;
                        act[k] = false;
                        continue;
                    }
                    const int32_t f = fe[k];
                    if (cl[k] == 0) {
                        const int32_t e = qe[qq[k]];
                        if constexpr (MOM) {
                            entry_masks(a.mom, uu[k], e, f, me[k], mf[k]);
                            dv[k] = a.mom.det[f] * a.mom.det[e];
                        } else {
                            // row loc of X (e first) or column loc (e second);
                            // the self pair stores X + X^T
                            const int loc = qloc[qq[k]];
                            const TR *r = (const TR *)a.far_rec + (f >= e ? Rec<NK>::r(loc, uu[k], a.n_far)
                                                                           : Rec<NK>::c(loc, uu[k], a.n_far));
#pragma unroll
                            for (int b = 0; b < 3; ++b)
#pragma unroll
                                for (int kk = 0; kk < NK; ++kk) xv[k][b][kk] = r[b * NK + kk];
                        }
                    }
                }
#pragma unroll
                for (int k = 0; k < kRowU; ++k) {
                    if (!act[k]) continue;
                    const int q = qq[k];
                    const int32_t e = qe[q], f = fe[k];
                    if (cl[k] == 0) {
                        const int32_t nb[3] = {nf0[k], nf1[k], nf2[k]};
                        double xm[3];
                        if constexpr (MOM) {
                            // -c |J_e| |J_f| (M_O(me)_loc M_I + M_I,loc M_O(mf))
                            const int loc = qloc[q];
                            // M_O of each mask from the two nibble sums
                            const double *lut = mq;
                            const int e0 = (int)whole_nibble(me[k], 0) * 3, e1 = 48 + (int)whole_nibble(me[k], 1) * 3;
                            const int f0 = (int)whole_nibble(mf[k], 0) * 3, f1 = 48 + (int)whole_nibble(mf[k], 1) * 3;
                            const double ol = lut[e0 + loc] + lut[e1 + loc];
                            double ob[3];
#pragma unroll
                            for (int b = 0; b < 3; ++b) ob[b] = lut[f0 + b] + lut[f1 + b];
                            const double il = mq[kRowMomLut + loc];
                            const double sc = -a.mom.c * dv[k];
#pragma unroll
                            for (int b = 0; b < 3; ++b) xm[b] = sc * (ol * a.mom.mi[b] + il * ob[b]);
                        }
#pragma unroll
                        for (int b = 0; b < 3; ++b) {
                            const int px = f == e ? qp[q][b] : hpos(hk, hv, mask, nb[b]);
                            if (px < 0) {
                                bad = true;
                                continue;
                            }
                            double xs[NK];
#pragma unroll
                            for (int kk = 0; kk < NK; ++kk) xs[kk] = MOM ? xm[b] : (double)xv[MOM ? 0 : k][b][kk];
                            if (a.mat.n) {
                                // rows e, columns f: the element of the column holds x
                                const double cf = a.mat.coef(f, e);
#pragma unroll
                                for (int kk = 0; kk < NK; ++kk) xs[kk] *= cf;
                            }
                            add_sym_block<NC>(acc, px, xs);
                        }
                    }
                }
                // queue the touching entries of this step
#pragma unroll
                for (int k = 0; k < kRowU; ++k) {
                    const bool tk = act[k] && cl[k] != 0;
                    const unsigned long long bl = __ballot(tk);
                    if (tk) {
                        const int pos = ntouch + __popcll(bl & ((1ull << lane) - 1ull));
                        sh.tt[pos] = tt[k];
                        sh.tq[pos] = (uint8_t)qq[k];
                    }
                    ntouch += __popcll(bl);
                }
                if (ntouch > kRowTouchCap - 64 * kRowU) {
                    __syncthreads();
                    if (!flush_touch<NC>(a, sh, ntouch, i, acc, hk, hv, mask, lane)) bad = true;
                    ntouch = 0;
                    __syncthreads();
                }
            }
            if (ntouch > 0) {   // before the element slots of this batch are reused
                __syncthreads();
                if (!flush_touch<NC>(a, sh, ntouch, i, acc, hk, hv, mask, lane)) bad = true;
            }
            __syncthreads();
        }
        if (bad) atomicOr(a.err, kErrSlot);
        if (NC == 1) {
            for (int t = lane; t < len; t += 64) a.val[s + t] = acc[t];
        } else {
            for (int t = lane; t < len * 4; t += 64) {
                const int pos = t >> 2, c = (t >> 1) & 1, d = t & 1;
                a.val[4 * s + (int64_t)c * 2 * len + 2 * pos + d] = acc[t];
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- plans

// Everything one assembly of one problem launches with (host side).
struct AssemblePlan {
    int kernel, nc;
    bool fp32, poly, seven;          // seven: both rules have 7 points
    bool mom;                        // moment form (MomArgs): no far-record launch
    FarArgs far;                     // far.n == 0: no non-touching pairs
    RoleArgs r1, r2;
    TouchArgs touch[3];              // identical, edge, vertex classes
    GaussArgs gauss;
    DiagArgs diag;
    RowArgs rows;                    // rows.nrows == 0: empty pattern
};

RoleArgs roles(const RuleArgs &r, bool a_outer, bool b_outer);
MomArgs moment_args(const nlfem_pairs *h, const nlfem_config *cfg);
// the single-problem launches of one phase of a plan (0 non-touching pairs,
// 1 touching pairs, 2 element diagonals, 3 rows; continuous ansatz), on s
void launch_phase(const AssemblePlan &p, int phase, hipStream_t s);
AssemblePlan make_plan(const nlfem_pairs *h, const nlfem_mesh *m, const nlfem_config *cfg, const GaussArgs &g,
                       double *val);

}  // namespace items
}  // namespace nlfem

/*
 * oracle.c - plain, slow FP64 CPU reference for nonlocal P1 stiffness
 * assembly (Klar, Vollmann, Schulz: "nlfem", arXiv 2207.03921).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this file.  It shares no code with
 * the GPU library: every formula is written out again here from the paper.
 *
 * What it computes (all FP64, compiled with -ffp-contract=off):
 *   - element pairs by brute force over all K^2 ordered pairs (Sec. 2.5
 *     defines the interaction graph; we enumerate it directly), and the
 *     breadth-first traversal of Alg. 2 as a cross-check;
 *   - each local contribution A_kl (eq. def:localStiffness) as a weighted
 *     sum of the integrand Phi_ij (eq. def:integrand) over quadrature
 *     samples (x, y): product rules with the approximate ball for disjoint
 *     pairs (Sec. 2.4.1, eq. discrete-inner) and regularising transforms to
 *     (0,1)^4 with a tensor Gauss rule for touching pairs (Sec. 2.4.2);
 *   - the sum over all ordered pairs (eq. biFormApprox) into a given CSR
 *     pattern, rows restricted to degrees of freedom;
 *   - the load vector (f, phi_i).
 *
 * Parity status: see the pins in tests/test_oracle_pins.py.  The absolute
 * values of the far-field 1/|z| and peridynamic quadrature on jittered
 * meshes and of 32-gon sub-triangle sums have no closed form; they are
 * pinned only through the invariants and the independent integrals there.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_K_CONSTANT = 0, ORC_K_INV_DIST = 1, ORC_K_PERIDYNAMIC = 2, ORC_K_FRAC_HALF = 3 };
enum { ORC_A_BARY = 0, ORC_A_POLY = 1, ORC_A_INF = 2, ORC_A_NOCAPS = 3, ORC_A_APPROXCAPS = 4 };
enum { ORC_FAR = 0, ORC_VERTEX = 1, ORC_EDGE = 2, ORC_IDENT = 3 };

typedef struct {
    int64_t n_vertices, n_elements;
    const double *vertices;   /* [M][2] */
    const int32_t *elements;  /* [K][3] */
    const int32_t *labels;    /* [K]    1 = Omega, 2 = Omega_D, else ignored */
    const int32_t *materials; /* [K]    material ids (NULL: all 0) */
} orc_mesh;

typedef struct {
    int32_t kernel;           /* ORC_K_* */
    int32_t ncomp;            /* 1 scalar, 2 peridynamic */
    double c, delta;
    int32_t approach;         /* ORC_A_* */
    int32_t polygon_n;
    const double *polygon_dirs; /* [N][2] unit directions, CCW */
    int32_t P; const double *pxi; const double *pw;   /* outer rule */
    int32_t Q; const double *qxi; const double *qw;   /* inner rule */
    int32_t singular_n;       /* 0 = product rule on touching pairs too */
    const double *gl_x;       /* [singular_n] Gauss-Legendre nodes on [0,1] */
    const double *gl_w;       /* [singular_n] weights on [0,1] */
    int32_t dg;               /* 1: discontinuous P1 (three unknowns per element,
                                 numbered 3k + local vertex), 0: continuous */
    int32_t n_materials;      /* 0: no table */
    const double *material_c; /* [n][n]: Psi(x, y) = material_c[m(x)][m(y)] Psi0(x, y),
                                 m(x) the material of the element holding x
                                 (Sec. 1 and 2.1: label-dependent, possibly
                                 non-symmetric kernels) */
} orc_cfg;

/* ------------------------------------------------------------------ */
/* element geometry: chi_k(xi) = v0 + J xi, J = [v1 - v0, v2 - v0]     */

typedef struct {
    int32_t node[3];
    double v[3][2];
    double J[2][2];
    double absdet;
    int32_t mat;   /* material id (0 without a table) */
} elem_t;

static int32_t material_of(const orc_mesh *m, int64_t k)
{
    return m->materials ? m->materials[k] : 0;
}

static void load_elem(const orc_mesh *m, int64_t k, elem_t *e)
{
    for (int a = 0; a < 3; ++a) {
        e->node[a] = m->elements[3 * k + a];
        e->v[a][0] = m->vertices[2 * (int64_t)e->node[a] + 0];
        e->v[a][1] = m->vertices[2 * (int64_t)e->node[a] + 1];
    }
    e->J[0][0] = e->v[1][0] - e->v[0][0];
    e->J[0][1] = e->v[2][0] - e->v[0][0];
    e->J[1][0] = e->v[1][1] - e->v[0][1];
    e->J[1][1] = e->v[2][1] - e->v[0][1];
    e->absdet = fabs(e->J[0][0] * e->J[1][1] - e->J[0][1] * e->J[1][0]);
}

/* element with its vertices listed in a prescribed order */
static void load_elem_ordered(const orc_mesh *m, const int32_t order[3], elem_t *e)
{
    for (int a = 0; a < 3; ++a) {
        e->node[a] = order[a];
        e->v[a][0] = m->vertices[2 * (int64_t)order[a] + 0];
        e->v[a][1] = m->vertices[2 * (int64_t)order[a] + 1];
    }
    e->J[0][0] = e->v[1][0] - e->v[0][0];
    e->J[0][1] = e->v[2][0] - e->v[0][0];
    e->J[1][0] = e->v[1][1] - e->v[0][1];
    e->J[1][1] = e->v[2][1] - e->v[0][1];
    e->absdet = fabs(e->J[0][0] * e->J[1][1] - e->J[0][1] * e->J[1][0]);
}

/* Discontinuous ansatz (Sec. 1 and 2.3: nlfem assembles CG or DG spaces):
 * every element carries its own three basis functions, so the union of a
 * pair's unknowns never merges vertices of different elements.  The node
 * ids of a loaded element become 3 kk + (stored position of the vertex). */
static void dg_ids(const orc_mesh *m, int64_t kk, elem_t *e)
{
    for (int a = 0; a < 3; ++a) {
        int slot = 0;
        for (int s = 0; s < 3; ++s)
            if (m->elements[3 * kk + s] == e->node[a]) slot = s;
        e->node[a] = (int32_t)(3 * kk + slot);
    }
}

static void to_phys(const elem_t *e, const double xi[2], double x[2])
{
    x[0] = e->v[0][0] + (e->J[0][0] * xi[0] + e->J[0][1] * xi[1]);
    x[1] = e->v[0][1] + (e->J[1][0] * xi[0] + e->J[1][1] * xi[1]);
}

static void barycentre(const elem_t *e, double b[2])
{
    b[0] = ((e->v[0][0] + e->v[1][0]) + e->v[2][0]) / 3.0;
    b[1] = ((e->v[0][1] + e->v[1][1]) + e->v[2][1]) / 3.0;
}

/* inverse of chi_e: reference coordinates of a physical point */
static void to_ref(const elem_t *e, const double x[2], double xi[2])
{
    double det = e->J[0][0] * e->J[1][1] - e->J[0][1] * e->J[1][0];
    double dx = x[0] - e->v[0][0], dy = x[1] - e->v[0][1];
    xi[0] = (e->J[1][1] * dx - e->J[0][1] * dy) / det;
    xi[1] = (-e->J[1][0] * dx + e->J[0][0] * dy) / det;
}

/* P1 shape functions on the reference triangle */
static void phihat(const double xi[2], double phi[3])
{
    phi[0] = 1.0 - xi[0] - xi[1];
    phi[1] = xi[0];
    phi[2] = xi[1];
}

/* ------------------------------------------------------------------ */
/* kernel Psi(x, y) as an ncomp x ncomp matrix (row-major)             */
/*   constant:    c                       (s = -1, Sec. 3.1)           */
/*   inv_dist:    c / |x - y|             (s = -1/2, Sec. 3.1)         */
/*   peridynamic: c (x-y)(x-y)^T / |x-y|^3 (Sec. 3.2)                  */
/*   frac_half:   c / |x - y|^3           (s = 1/2, Sec. 3.1)          */

static void kernel(const orc_cfg *cf, const double x[2], const double y[2], double *out)
{
    double z0 = x[0] - y[0], z1 = x[1] - y[1];
    double r = sqrt(z0 * z0 + z1 * z1);
    switch (cf->kernel) {
    case ORC_K_CONSTANT:
        out[0] = cf->c;
        break;
    case ORC_K_INV_DIST:
        out[0] = cf->c / r;
        break;
    case ORC_K_FRAC_HALF:
        out[0] = cf->c / (r * r * r);
        break;
    default: {
        double r3 = r * r * r;
        out[0] = cf->c * z0 * z0 / r3;
        out[1] = cf->c * z0 * z1 / r3;
        out[2] = cf->c * z1 * z0 / r3;
        out[3] = cf->c * z1 * z1 / r3;
    }
    }
}

/* ------------------------------------------------------------------ */
/* Union-node local matrix.                                            */
/* The pair (k, l) touches the global nodes U = nodes(k) u nodes(l).   */
/* For a sample (x in T_k, y in T_l) and union nodes a, b, components  */
/* c, d the integrand (eq. def:integrand) for phi_i = phi_a e_c,       */
/* phi_j = phi_b e_d reads                                             */
/*   Phi = (phi_a(x) - phi_a(y)) (Psi_cd(x,y) phi_b(x) - Psi_cd(y,x) phi_b(y)). */

#define MAXU 6

typedef struct {
    int nu;
    int32_t node[MAXU];
    int ink[MAXU];   /* local index in k or -1 */
    int inl[MAXU];   /* local index in l or -1 */
} union_t;

static void make_union(const elem_t *k, const elem_t *l, union_t *u)
{
    u->nu = 0;
    for (int a = 0; a < 3; ++a) {
        u->node[u->nu] = k->node[a];
        u->ink[u->nu] = a;
        u->inl[u->nu] = -1;
        u->nu++;
    }
    for (int b = 0; b < 3; ++b) {
        int found = -1;
        for (int a = 0; a < u->nu; ++a)
            if (u->node[a] == l->node[b]) found = a;
        if (found >= 0) {
            u->inl[found] = b;
        } else {
            u->node[u->nu] = l->node[b];
            u->ink[u->nu] = -1;
            u->inl[u->nu] = b;
            u->nu++;
        }
    }
}

/* add weight * Phi(x, y) for all union index pairs into L[(a,c),(b,d)] */
static void add_sample(const orc_cfg *cf, const union_t *u, const elem_t *k, const elem_t *l,
                       const double xi[2], const double eta[2], double weight, double *L)
{
    const int n = cf->ncomp;
    const int dim = u->nu * n;
    double x[2], y[2], pk[3], pl[3], Kxy[4], Kyx[4];
    double fx[MAXU], fy[MAXU];
    to_phys(k, xi, x);
    to_phys(l, eta, y);
    /* Table 1, s <= 0 without the transforms (singular_n = 0): the rule
     * avoids x_p = y_q, i.e. a sample at the same point of both elements
     * (distance at rounding level against the element size) is left out */
    if (cf->kernel != ORC_K_CONSTANT && cf->singular_n == 0) {
        double z0 = x[0] - y[0], z1 = x[1] - y[1];
        double small = 1e-12 * (k->absdet < l->absdet ? k->absdet : l->absdet);
        if (z0 * z0 + z1 * z1 <= small) return;
    }
    phihat(xi, pk);
    phihat(eta, pl);
    for (int a = 0; a < u->nu; ++a) {
        fx[a] = u->ink[a] >= 0 ? pk[u->ink[a]] : 0.0;   /* phi_a(x), x in T_k */
        fy[a] = u->inl[a] >= 0 ? pl[u->inl[a]] : 0.0;   /* phi_a(y), y in T_l */
    }
    kernel(cf, x, y, Kxy);
    kernel(cf, y, x, Kyx);
    if (cf->n_materials > 0) {
        /* x in T_k, y in T_l */
        const double cxy = cf->material_c[k->mat * cf->n_materials + l->mat];
        const double cyx = cf->material_c[l->mat * cf->n_materials + k->mat];
        for (int i = 0; i < n * n; ++i) {
            Kxy[i] *= cxy;
            Kyx[i] *= cyx;
        }
    }
    for (int a = 0; a < u->nu; ++a)
        for (int c = 0; c < n; ++c)
            for (int b = 0; b < u->nu; ++b)
                for (int d = 0; d < n; ++d) {
                    double phi = (fx[a] - fy[a]) * (Kxy[c * n + d] * fx[b] - Kyx[c * n + d] * fy[b]);
                    L[(a * n + c) * dim + (b * n + d)] += weight * phi;
                }
}

/* ------------------------------------------------------------------ */
/* ball approximations                                                 */

/* barycentre rule: T_l counts for the outer point x iff |x - bary(T_l)| <= delta */
static int chi_bary(const orc_cfg *cf, const double x[2], const elem_t *l)
{
    double b[2];
    barycentre(l, b);
    double dx = x[0] - b[0];
    double dy = x[1] - b[1];
    return (dx * dx + dy * dy) <= cf->delta * cf->delta;
}

/* Regular N-gon inscribed in the circle of radius delta around x, vertices
 * q_j = x + delta * dir_j (CCW).  Sutherland-Hodgman clip of T_l against its
 * N edges.  A point v is inside edge j iff cross(q_{j+1} - q_j, v - q_j) >= 0;
 * the crossing point of segment a -> b is a + t (b - a), t = d_a/(d_a - d_b).
 * The infinity-norm ball (Def. 2.5) {y : |x - y|_inf <= delta} is the square
 * with corners x + delta (+-1, +-1), taken counter-clockwise from (+1, +1):
 * the same clip against its 4 edges is exact. */
#define MAXPOLY 80
static const double SQUARE_CORNERS[4][2] = {{1.0, 1.0}, {-1.0, 1.0}, {-1.0, -1.0}, {1.0, -1.0}};
static int clip_triangle(const orc_cfg *cf, const double x[2], const elem_t *l, double out[][2])
{
    double buf[2][MAXPOLY][2];
    int cnt = 3;
    for (int a = 0; a < 3; ++a) {
        buf[0][a][0] = l->v[a][0];
        buf[0][a][1] = l->v[a][1];
    }
    int cur = 0;
    const int square = cf->approach == ORC_A_INF;
    const int N = square ? 4 : cf->polygon_n;
    const double *dirs = square ? &SQUARE_CORNERS[0][0] : cf->polygon_dirs;
    for (int j = 0; j < N && cnt > 0; ++j) {
        int j1 = (j + 1) % N;
        double qa0 = x[0] + cf->delta * dirs[2 * j + 0];
        double qa1 = x[1] + cf->delta * dirs[2 * j + 1];
        double qb0 = x[0] + cf->delta * dirs[2 * j1 + 0];
        double qb1 = x[1] + cf->delta * dirs[2 * j1 + 1];
        double e0 = qb0 - qa0, e1 = qb1 - qa1;
        int nxt = 1 - cur, m = 0;
        for (int i = 0; i < cnt; ++i) {
            const double *p = buf[cur][i];
            const double *q = buf[cur][(i + 1) % cnt];
            double dp = e0 * (p[1] - qa1) - e1 * (p[0] - qa0);
            double dq = e0 * (q[1] - qa1) - e1 * (q[0] - qa0);
            int pin = dp >= 0.0, qin = dq >= 0.0;
            if (pin) {
                buf[nxt][m][0] = p[0];
                buf[nxt][m][1] = p[1];
                m++;
            }
            if (pin != qin) {
                double t = dp / (dp - dq);
                buf[nxt][m][0] = p[0] + t * (q[0] - p[0]);
                buf[nxt][m][1] = p[1] + t * (q[1] - p[1]);
                m++;
            }
        }
        cnt = m;
        cur = nxt;
    }
    for (int i = 0; i < cnt; ++i) {
        out[i][0] = buf[cur][i][0];
        out[i][1] = buf[cur][i][1];
    }
    return cnt;
}

static double shoelace(const double (*p)[2], int cnt)
{
    double s = 0.0;
    for (int i = 0; i < cnt; ++i) {
        int i1 = (i + 1) % cnt;
        s += p[i][0] * p[i1][1] - p[i1][0] * p[i][1];
    }
    return 0.5 * s;
}

/* The ball approximations of Def. 2.3 and 2.4 restricted to T_l.
 * nocaps: the convex hull of all crossings of the circle |y - x| = delta
 * with element edges.  Between two consecutive crossings (by angle) the arc
 * runs inside a single element, so the hull's chord between them lies in
 * that element, no vertex lies in the cut-off cap, and
 *   T_l n B^ncp(x) = conv(vertices of T_l in the closed disc
 *                         u crossings of the edges of T_l with the circle).
 * approxcaps adds, for every arc of the circle inside T_l, its midpoint (the
 * cap centre).  The region is convex; its boundary is walked counter-
 * clockwise: along each edge v_i -> v_i+1 the vertex v_i if inside, then
 * the crossings in order of the edge parameter t, from the roots of
 *   |v_i - x + t e|^2 = delta^2:  A t^2 + 2 B t + C = 0,
 *   A = e.e, B = (v_i - x).e, C = |v_i - x|^2 - delta^2, D = B^2 - A C;
 * leaving the disc (inside -> outside) t = (-B + sqrt D)/A, entering
 * t = (-B - sqrt D)/A (clamped to [0, 1]), and two crossings on an edge
 * with both ends outside iff D > 0 and 0 < -B < A.  With approxcaps the cap
 * centre follows every leaving crossing: the arc from it to the next
 * entering crossing lies inside T_l, and its midpoint is one of the two
 * points x +- delta m/|m| on the circle, m = u1 + u2 (u1, u2 the two
 * crossings minus x; u1 turned by +90 degrees when m = 0): the one deeper
 * inside T_l, i.e. with the larger smallest edge function
 * cross(v_i+1 - v_i, y - v_i) (ties to +; this also settles the degenerate
 * arc of a circle through a vertex, where the two crossings meet).  All
 * vertices inside: the triangle
 * itself.  No crossing otherwise: empty (also when the circle lies inside
 * T_l).  Returns the point count (<= 12). */
#define MAXCAPS 12
static int caps_polygon(const orc_cfg *cf, const double x[2], const elem_t *l, double out[][2])
{
    const double d2 = cf->delta * cf->delta;
    const double sa = (l->v[1][0] - l->v[0][0]) * (l->v[2][1] - l->v[0][1]) -
                      (l->v[2][0] - l->v[0][0]) * (l->v[1][1] - l->v[0][1]);
    const int ord[3] = {0, sa >= 0.0 ? 1 : 2, sa >= 0.0 ? 2 : 1};
    double P[3][2];
    int in[3];
    for (int i = 0; i < 3; ++i) {
        P[i][0] = l->v[ord[i]][0];
        P[i][1] = l->v[ord[i]][1];
        const double dx = P[i][0] - x[0], dy = P[i][1] - x[1];
        in[i] = dx * dx + dy * dy <= d2;
    }
    if (in[0] && in[1] && in[2]) {   /* the triangle itself, in stored order */
        for (int i = 0; i < 3; ++i) {
            out[i][0] = l->v[i][0];
            out[i][1] = l->v[i][1];
        }
        return 3;
    }
    double pt[MAXCAPS][2];
    int kind[MAXCAPS];   /* 0 vertex, 1 entering, 2 leaving */
    int n = 0, ncross = 0;
    for (int i = 0; i < 3; ++i) {
        const int i1 = (i + 1) % 3;
        if (in[i]) {
            pt[n][0] = P[i][0];
            pt[n][1] = P[i][1];
            kind[n++] = 0;
        }
        const double ex = P[i1][0] - P[i][0], ey = P[i1][1] - P[i][1];
        const double ax = P[i][0] - x[0], ay = P[i][1] - x[1];
        const double A = ex * ex + ey * ey;
        const double B = ax * ex + ay * ey;
        const double C = ax * ax + ay * ay - d2;
        const double D = B * B - A * C;
        const double sq = sqrt(D > 0.0 ? D : 0.0);
        double t[2];
        int k[2], m = 0;
        if (in[i] && !in[i1]) {
            t[0] = (-B + sq) / A;
            k[0] = 2;
            m = 1;
        } else if (!in[i] && in[i1]) {
            t[0] = (-B - sq) / A;
            k[0] = 1;
            m = 1;
        } else if (!in[i] && !in[i1] && D > 0.0 && -B > 0.0 && -B < A) {
            t[0] = (-B - sq) / A;
            t[1] = (-B + sq) / A;
            k[0] = 1;
            k[1] = 2;
            m = 2;
        }
        for (int c = 0; c < m; ++c) {
            const double tc = t[c] < 0.0 ? 0.0 : (t[c] > 1.0 ? 1.0 : t[c]);
            pt[n][0] = P[i][0] + tc * ex;
            pt[n][1] = P[i][1] + tc * ey;
            kind[n++] = k[c];
            ++ncross;
        }
    }
    if (ncross == 0) return 0;
    int cnt = 0;
    for (int j = 0; j < n; ++j) {
        out[cnt][0] = pt[j][0];
        out[cnt][1] = pt[j][1];
        ++cnt;
        if (cf->approach != ORC_A_APPROXCAPS || kind[j] != 2) continue;
        int jn = (j + 1) % n;
        while (kind[jn] != 1) jn = (jn + 1) % n;
        const double u1x = pt[j][0] - x[0], u1y = pt[j][1] - x[1];
        const double u2x = pt[jn][0] - x[0], u2y = pt[jn][1] - x[1];
        double mx = u1x + u2x, my = u1y + u2y;
        if (mx == 0.0 && my == 0.0) {
            mx = -u1y;
            my = u1x;
        }
        const double mn = sqrt(mx * mx + my * my);
        const double ux = cf->delta * (mx / mn), uy = cf->delta * (my / mn);
        double cand[2][2] = {{x[0] + ux, x[1] + uy}, {x[0] - ux, x[1] - uy}};
        double depth[2];
        for (int c = 0; c < 2; ++c) {
            depth[c] = 0.0;
            for (int i = 0; i < 3; ++i) {
                const int i1 = (i + 1) % 3;
                const double f = (P[i1][0] - P[i][0]) * (cand[c][1] - P[i][1]) -
                                 (P[i1][1] - P[i][1]) * (cand[c][0] - P[i][0]);
                if (i == 0 || f < depth[c]) depth[c] = f;
            }
        }
        const int pick = depth[0] >= depth[1] ? 0 : 1;
        out[cnt][0] = cand[pick][0];
        out[cnt][1] = cand[pick][1];
        ++cnt;
    }
    return cnt;
}

static int is_caps(const orc_cfg *cf) { return cf->approach == ORC_A_NOCAPS || cf->approach == ORC_A_APPROXCAPS; }

/* the polygon of T_l n B(x) for the clipped balls (N-gon, square, caps) */
static int ball_polygon(const orc_cfg *cf, const double x[2], const elem_t *l, double out[][2])
{
    return is_caps(cf) ? caps_polygon(cf, x, l, out) : clip_triangle(cf, x, l, out);
}

static int chi_poly(const orc_cfg *cf, const double x[2], const elem_t *l)
{
    double out[MAXPOLY][2];
    int cnt = ball_polygon(cf, x, l, out);
    if (cnt < 3) return 0;
    return fabs(shoelace((const double (*)[2])out, cnt)) > 0.0;
}

static int chi(const orc_cfg *cf, const double x[2], const elem_t *l)
{
    return cf->approach == ORC_A_BARY ? chi_bary(cf, x, l) : chi_poly(cf, x, l);
}

/* ------------------------------------------------------------------ */
/* pair classification                                                 */

static int shared_vertices(const elem_t *k, const elem_t *l)
{
    int s = 0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            s += k->node[a] == l->node[b];
    return s;
}

static int label_ok(const orc_mesh *m, int64_t k, int64_t l)
{
    int32_t lk = m->labels[k], ll = m->labels[l];
    if (lk != 1 && lk != 2) return 0;
    if (ll != 1 && ll != 2) return 0;
    return lk == 1 || ll == 1;
}

/* Geometric interaction test of the ordered pair (k, l).  Returns the class
 * (ORC_FAR .. ORC_IDENT) if the pair interacts, -1 otherwise.  Touching pairs
 * of a kernel treated as singular always interact (truncation is ignored
 * on them, Assumption 3); other pairs interact iff some outer point sees
 * T_l through the ball approximation. */
static int interact(const orc_mesh *m, const orc_cfg *cf, int64_t kk, int64_t ll)
{
    elem_t k, l;
    load_elem(m, kk, &k);
    load_elem(m, ll, &l);
    int s = shared_vertices(&k, &l);
    if (cf->singular_n > 0 && s > 0) return s;   /* 1 vertex, 2 edge, 3 identical */
    for (int p = 0; p < cf->P; ++p) {
        double x[2];
        to_phys(&k, &cf->pxi[2 * p], x);
        if (chi(cf, x, &l)) return ORC_FAR;
    }
    return -1;
}

/* Brute-force list of all interacting ordered pairs with admissible labels,
 * sorted by (k, l).  If elem_mask is given, only pairs with mask[k] or
 * mask[l] set are listed.  Returns the count; arrays are filled only when
 * cap is large enough. */
int64_t orc_pairs(const orc_mesh *m, const orc_cfg *cf, const uint8_t *elem_mask,
                  int32_t *k_out, int32_t *l_out, int8_t *cls_out, int64_t cap)
{
    const int64_t K = m->n_elements;
    int64_t *cnt = (int64_t *)calloc((size_t)K + 1, sizeof(int64_t));
    if (!cnt) return -1;
    /* with a mask, an unmasked k only meets the masked l (ascending) */
    int64_t nmask = 0, *mlist = NULL;
    if (elem_mask) {
        mlist = (int64_t *)malloc(sizeof(int64_t) * ((size_t)K + 1));
        if (!mlist) {
            free(cnt);
            return -1;
        }
        for (int64_t l = 0; l < K; ++l)
            if (elem_mask[l]) mlist[nmask++] = l;
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < K; ++k) {
        int64_t c = 0;
        const int all = !elem_mask || elem_mask[k];
        const int64_t nl = all ? K : nmask;
        for (int64_t t = 0; t < nl; ++t) {
            const int64_t l = all ? t : mlist[t];
            if (!label_ok(m, k, l)) continue;
            if (interact(m, cf, k, l) >= 0) c++;
        }
        cnt[k + 1] = c;
    }
    for (int64_t k = 0; k < K; ++k) cnt[k + 1] += cnt[k];
    int64_t total = cnt[K];
    if (cap >= total && total > 0) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t k = 0; k < K; ++k) {
            int64_t o = cnt[k];
            const int all = !elem_mask || elem_mask[k];
            const int64_t nl = all ? K : nmask;
            for (int64_t t = 0; t < nl; ++t) {
                const int64_t l = all ? t : mlist[t];
                if (!label_ok(m, k, l)) continue;
                int c = interact(m, cf, k, l);
                if (c >= 0) {
                    k_out[o] = (int32_t)k;
                    l_out[o] = (int32_t)l;
                    cls_out[o] = (int8_t)c;
                    o++;
                }
            }
        }
    }
    free(cnt);
    free(mlist);
    return total;
}

/* Alg. 2: truncated breadth-first traversal of the adjacency graph from each
 * element; a neighbour is queued iff the pair interacts.  The traversal uses
 * the geometric test only; the label filter applies when recording.  Output
 * is sorted by (k, l) through a per-k sort. */
static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

int64_t orc_pairs_bfs(const orc_mesh *m, const orc_cfg *cf,
                      int32_t *k_out, int32_t *l_out, int8_t *cls_out, int64_t cap)
{
    const int64_t K = m->n_elements, M = m->n_vertices;
    /* node -> element incidence */
    int64_t *nptr = (int64_t *)calloc((size_t)M + 1, sizeof(int64_t));
    int32_t *nel = (int32_t *)malloc(sizeof(int32_t) * (size_t)(3 * K));
    for (int64_t k = 0; k < K; ++k)
        for (int a = 0; a < 3; ++a) nptr[m->elements[3 * k + a] + 1]++;
    for (int64_t i = 0; i < M; ++i) nptr[i + 1] += nptr[i];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)M);
    for (int64_t i = 0; i < M; ++i) fill[i] = nptr[i];
    for (int64_t k = 0; k < K; ++k)
        for (int a = 0; a < 3; ++a) nel[fill[m->elements[3 * k + a]]++] = (int32_t)k;
    free(fill);

    int64_t total = 0;
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(K + 1));
    uint8_t *visited = (uint8_t *)calloc((size_t)K, 1);
    int32_t *found = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    for (int64_t k = 0; k < K; ++k) {
        int32_t lk = m->labels[k];
        if (lk != 1 && lk != 2) continue;
        int64_t head = 0, tail = 0, nf = 0;
        queue[tail++] = (int32_t)k;
        memset(visited, 0, (size_t)K);
        while (head < tail) {
            int32_t t = queue[head++];
            for (int a = 0; a < 3; ++a) {
                int32_t node = m->elements[3 * (int64_t)t + a];
                for (int64_t q = nptr[node]; q < nptr[node + 1]; ++q) {
                    int32_t l = nel[q];
                    if (visited[l]) continue;
                    int32_t ll = m->labels[l];
                    if (ll == 1 || ll == 2) {
                        if (interact(m, cf, k, l) >= 0) {
                            queue[tail++] = l;
                            if (label_ok(m, k, l)) found[nf++] = l;
                        }
                    }
                    visited[l] = 1;
                }
            }
        }
        qsort(found, (size_t)nf, sizeof(int32_t), cmp_i32);
        for (int64_t i = 0; i < nf; ++i) {
            if (total < cap) {
                k_out[total] = (int32_t)k;
                l_out[total] = found[i];
                cls_out[total] = (int8_t)interact(m, cf, k, found[i]);
            }
            total++;
        }
    }
    free(queue);
    free(visited);
    free(found);
    free(nptr);
    free(nel);
    return total;
}

/* ------------------------------------------------------------------ */
/* Regularising transforms for touching pairs (Sec. 2.4.2).            */
/* Each maps a point of (0,1)^4 to (xi, eta) in T^ x T^ and returns the */
/* Jacobian; summed with the tensor Gauss rule they integrate over      */
/* T^ x T^.  Element frames: see touch_frames().                        */

/* identical pair: z = eta - xi, sector j of the hexagon with corners
 * c_0..c_5 = (1,0),(0,1),(-1,1),(-1,0),(0,-1),(1,-1); z = rho((1-u)c_j + u c_j+1);
 * xi = o(z) + (1 - rho)(sigma, (1 - sigma) tau), o(z) = (max(0,-z1), max(0,-z2)). */
static const double HEX[6][2] = {{1, 0}, {0, 1}, {-1, 1}, {-1, 0}, {0, -1}, {1, -1}};

static double map_identical(int j, const double t[4], double xi[2], double eta[2])
{
    double rho = t[0], u = t[1], sg = t[2], tau = t[3];
    int j1 = (j + 1) % 6;
    double z0 = rho * ((1.0 - u) * HEX[j][0] + u * HEX[j1][0]);
    double z1 = rho * ((1.0 - u) * HEX[j][1] + u * HEX[j1][1]);
    double o0 = z0 < 0.0 ? -z0 : 0.0;
    double o1 = z1 < 0.0 ? -z1 : 0.0;
    xi[0] = o0 + (1.0 - rho) * sg;
    xi[1] = o1 + (1.0 - rho) * (1.0 - sg) * tau;
    eta[0] = xi[0] + z0;
    eta[1] = xi[1] + z1;
    return rho * (1.0 - rho) * (1.0 - rho) * (1.0 - sg);
}

/* edge pair: frames (P0,P1,A) and (P0,P1,B); v = (xi1 - eta1, xi2, eta2).
 * Faces of {max(v2 + v1+, v3 + v1-) <= 1, v2, v3 >= 0} with unit cone
 * Jacobian, triangles collapsed q -> (1-p) q:
 *   F0 (p, 1-p, q)  F1 (p, (1-p)q, 1)  F2 (-p, 1, (1-p)q)  F3 (-p, q, 1-p).
 * v = rho w, xi1 = max(0, v1) + (1 - rho) tau. */
static double map_edge(int f, const double t[4], double xi[2], double eta[2])
{
    double rho = t[0], p = t[1], q = t[2], tau = t[3];
    double w0, w1, w2, jf;
    switch (f) {
    case 0: w0 = p; w1 = 1.0 - p; w2 = q; jf = 1.0; break;
    case 1: w0 = p; w1 = (1.0 - p) * q; w2 = 1.0; jf = 1.0 - p; break;
    case 2: w0 = -p; w1 = 1.0; w2 = (1.0 - p) * q; jf = 1.0 - p; break;
    default: w0 = -p; w1 = q; w2 = 1.0 - p; jf = 1.0; break;
    }
    double v0 = rho * w0, v1 = rho * w1, v2 = rho * w2;
    xi[0] = (v0 > 0.0 ? v0 : 0.0) + (1.0 - rho) * tau;
    xi[1] = v1;
    eta[0] = xi[0] - v0;
    eta[1] = v2;
    return rho * rho * (1.0 - rho) * jf;
}

/* vertex pair: frames (P0,A1,A2), (P0,B1,B2); xi = s(1-a, a), eta = t(1-b, b);
 * region 0: t = s w, Jacobian s^3 w; region 1: s = t w, Jacobian t^3 w. */
static double map_vertex(int r, const double t4[4], double xi[2], double eta[2])
{
    double g = t4[0], w = t4[1], a = t4[2], b = t4[3];
    double s, t;
    if (r == 0) { s = g; t = g * w; }
    else { t = g; s = g * w; }
    xi[0] = s * (1.0 - a);
    xi[1] = s * a;
    eta[0] = t * (1.0 - b);
    eta[1] = t * b;
    return g * g * g * w;
}

static int n_pieces(int cls) { return cls == ORC_IDENT ? 6 : cls == ORC_EDGE ? 4 : 2; }

static double map_piece(int cls, int piece, const double t[4], double xi[2], double eta[2])
{
    if (cls == ORC_IDENT) return map_identical(piece, t, xi, eta);
    if (cls == ORC_EDGE) return map_edge(piece, t, xi, eta);
    return map_vertex(piece, t, xi, eta);
}

/* Vertex orders used by the transforms.
 * identical: the element's stored order.
 * edge: P0, P1 = shared vertices with P0 the smaller global node id;
 *       third vertex of each element last.
 * vertex: P0 = shared vertex, then the element's other two vertices in its
 *       cyclic order after P0. */
static void touch_frames(const orc_mesh *m, int64_t kk, int64_t ll, int cls,
                         int32_t ok[3], int32_t ol[3])
{
    const int32_t *ek = &m->elements[3 * kk], *el = &m->elements[3 * ll];
    if (cls == ORC_IDENT) {
        for (int a = 0; a < 3; ++a) ok[a] = ol[a] = ek[a];
        return;
    }
    if (cls == ORC_EDGE) {
        int32_t sh[2], ns = 0, ak = -1, bl = -1;
        for (int a = 0; a < 3; ++a) {
            int in = 0;
            for (int b = 0; b < 3; ++b) in |= ek[a] == el[b];
            if (in) sh[ns++] = ek[a];
            else ak = ek[a];
        }
        for (int b = 0; b < 3; ++b) {
            int in = 0;
            for (int a = 0; a < 3; ++a) in |= el[b] == ek[a];
            if (!in) bl = el[b];
        }
        int32_t p0 = sh[0] < sh[1] ? sh[0] : sh[1];
        int32_t p1 = sh[0] < sh[1] ? sh[1] : sh[0];
        ok[0] = p0; ok[1] = p1; ok[2] = ak;
        ol[0] = p0; ol[1] = p1; ol[2] = bl;
        return;
    }
    /* vertex */
    int ia = -1, ib = -1;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (ek[a] == el[b]) { ia = a; ib = b; }
    for (int s = 0; s < 3; ++s) {
        ok[s] = ek[(ia + s) % 3];
        ol[s] = el[(ib + s) % 3];
    }
}

/* Samples of the 4D rule in reference coordinates of the frames:
 * (xi, eta, weight) with weight = product Gauss weight x Jacobian. */
int64_t orc_duffy_samples(int cls, int n, const double *glx, const double *glw,
                          double *xi_out, double *eta_out, double *w_out, int64_t cap)
{
    int64_t c = 0;
    for (int piece = 0; piece < n_pieces(cls); ++piece)
        for (int i0 = 0; i0 < n; ++i0)
            for (int i1 = 0; i1 < n; ++i1)
                for (int i2 = 0; i2 < n; ++i2)
                    for (int i3 = 0; i3 < n; ++i3) {
                        double t[4] = {glx[i0], glx[i1], glx[i2], glx[i3]};
                        double xi[2], eta[2];
                        double jac = map_piece(cls, piece, t, xi, eta);
                        if (c < cap) {
                            xi_out[2 * c] = xi[0];
                            xi_out[2 * c + 1] = xi[1];
                            eta_out[2 * c] = eta[0];
                            eta_out[2 * c + 1] = eta[1];
                            w_out[c] = glw[i0] * glw[i1] * glw[i2] * glw[i3] * jac;
                        }
                        c++;
                    }
    return c;
}

/* ------------------------------------------------------------------ */
/* Inner quadrature of the truncated kernel (Sec. 2.4.1): samples        */
/* (eta in reference coordinates of T_l, weight incl. Jacobian) of        */
/*   int_{T_l n B(x)} g(y) dy  ~  sum_t w_t g(chi_l(eta_t)).               */
/* barycentre ball: the inner rule on all of T_l if |x - bary T_l| <= delta;*/
/* polygon: T_l unclipped if it lies inside the polygon, otherwise the fan  */
/* of the clipped polygon from its first vertex, the inner rule on every    */
/* sub-triangle and eta = chi_l^{-1}(y) (eq. discrete-inner).               */

static int inner_samples(const orc_cfg *cf, const double x[2], const elem_t *l,
                         double *eta, double *w)
{
    int cnt = 0;
    if (cf->approach == ORC_A_BARY) {
        if (!chi_bary(cf, x, l)) return 0;
        for (int q = 0; q < cf->Q; ++q) {
            eta[2 * cnt] = cf->qxi[2 * q];
            eta[2 * cnt + 1] = cf->qxi[2 * q + 1];
            w[cnt++] = cf->qw[q] * l->absdet;
        }
        return cnt;
    }
    double poly[MAXPOLY][2];
    int nv = ball_polygon(cf, x, l, poly);
    if (nv < 3) return 0;
    if (!(fabs(shoelace((const double (*)[2])poly, nv)) > 0.0)) return 0;
    int whole = nv == 3;
    for (int a = 0; a < 3 && whole; ++a)
        whole = poly[a][0] == l->v[a][0] && poly[a][1] == l->v[a][1];
    if (whole) {
        for (int q = 0; q < cf->Q; ++q) {
            eta[2 * cnt] = cf->qxi[2 * q];
            eta[2 * cnt + 1] = cf->qxi[2 * q + 1];
            w[cnt++] = cf->qw[q] * l->absdet;
        }
        return cnt;
    }
    for (int s = 1; s + 1 < nv; ++s) {
        elem_t S;
        for (int a = 0; a < 2; ++a) {
            S.v[0][a] = poly[0][a];
            S.v[1][a] = poly[s][a];
            S.v[2][a] = poly[s + 1][a];
        }
        S.J[0][0] = S.v[1][0] - S.v[0][0];
        S.J[0][1] = S.v[2][0] - S.v[0][0];
        S.J[1][0] = S.v[1][1] - S.v[0][1];
        S.J[1][1] = S.v[2][1] - S.v[0][1];
        S.absdet = fabs(S.J[0][0] * S.J[1][1] - S.J[0][1] * S.J[1][0]);
        for (int q = 0; q < cf->Q; ++q) {
            double y[2];
            to_phys(&S, &cf->qxi[2 * q], y);
            to_ref(l, y, &eta[2 * cnt]);
            w[cnt++] = cf->qw[q] * S.absdet;
        }
    }
    return cnt;
}

/* Moments of the inner integral for one outer point x and inner element l:
 * out = [int 1, int phi_a (3), int phi_a phi_b (9)] over T_l n B(x). */
int orc_inner_moments(const orc_cfg *cf, const orc_mesh *m, const double *x, int32_t ll, double *out)
{
    elem_t l;
    load_elem(m, ll, &l);
    double *eta = (double *)malloc(sizeof(double) * 2 * (size_t)MAXPOLY * (size_t)cf->Q);
    double *w = (double *)malloc(sizeof(double) * (size_t)MAXPOLY * (size_t)cf->Q);
    int ns = inner_samples(cf, x, &l, eta, w);
    memset(out, 0, sizeof(double) * 13);
    for (int t = 0; t < ns; ++t) {
        double ph[3];
        phihat(&eta[2 * t], ph);
        out[0] += w[t];
        for (int a = 0; a < 3; ++a) {
            out[1 + a] += w[t] * ph[a];
            for (int b = 0; b < 3; ++b) out[4 + 3 * a + b] += w[t] * ph[a] * ph[b];
        }
    }
    free(eta);
    free(w);
    return ns;
}

/* ------------------------------------------------------------------ */
/* local contribution A_kl over the union nodes                         */

/* Writes nodes[nu] and L[(nu*n)^2]; returns nu. */
static int local_matrix(const orc_mesh *m, const orc_cfg *cf, int64_t kk, int64_t ll, int cls,
                        int32_t *nodes, double *L)
{
    elem_t k, l;
    union_t u;
    const int n = cf->ncomp;
    if (cls != ORC_FAR && cf->singular_n > 0) {
        /* Alg. 1, first branch: intersecting pair, singular quadrature */
        int32_t ok[3], ol[3];
        touch_frames(m, kk, ll, cls, ok, ol);
        load_elem_ordered(m, ok, &k);
        load_elem_ordered(m, ol, &l);
        k.mat = material_of(m, kk);
        l.mat = material_of(m, ll);
        if (cf->dg) {
            dg_ids(m, kk, &k);
            dg_ids(m, ll, &l);
        }
        make_union(&k, &l, &u);
        memset(L, 0, sizeof(double) * (size_t)(u.nu * n) * (size_t)(u.nu * n));
        const int ns = cf->singular_n;
        for (int piece = 0; piece < n_pieces(cls); ++piece)
            for (int i0 = 0; i0 < ns; ++i0)
                for (int i1 = 0; i1 < ns; ++i1)
                    for (int i2 = 0; i2 < ns; ++i2)
                        for (int i3 = 0; i3 < ns; ++i3) {
                            double t[4] = {cf->gl_x[i0], cf->gl_x[i1], cf->gl_x[i2], cf->gl_x[i3]};
                            double xi[2], eta[2];
                            double jac = map_piece(cls, piece, t, xi, eta);
                            double wgt = cf->gl_w[i0] * cf->gl_w[i1] * cf->gl_w[i2] * cf->gl_w[i3] *
                                         jac * k.absdet * l.absdet;
                            add_sample(cf, &u, &k, &l, xi, eta, wgt, L);
                        }
    } else {
        /* Alg. 1, second branch: quadrature for kernel truncations */
        load_elem(m, kk, &k);
        load_elem(m, ll, &l);
        k.mat = material_of(m, kk);
        l.mat = material_of(m, ll);
        if (cf->dg) {
            dg_ids(m, kk, &k);
            dg_ids(m, ll, &l);
        }
        make_union(&k, &l, &u);
        memset(L, 0, sizeof(double) * (size_t)(u.nu * n) * (size_t)(u.nu * n));
        double *eta = (double *)malloc(sizeof(double) * 2 * (size_t)MAXPOLY * (size_t)cf->Q);
        double *w = (double *)malloc(sizeof(double) * (size_t)MAXPOLY * (size_t)cf->Q);
        for (int p = 0; p < cf->P; ++p) {
            double x[2];
            const double *xi = &cf->pxi[2 * p];
            to_phys(&k, xi, x);
            double wx = cf->pw[p] * k.absdet;
            int ns = inner_samples(cf, x, &l, eta, w);
            for (int t = 0; t < ns; ++t)
                add_sample(cf, &u, &k, &l, xi, &eta[2 * t], wx * w[t], L);
        }
        free(eta);
        free(w);
    }
    for (int a = 0; a < u.nu; ++a) nodes[a] = u.node[a];
    return u.nu;
}

int orc_local(const orc_mesh *m, const orc_cfg *cf, int32_t k, int32_t l, int cls,
              int32_t *nodes, double *L)
{
    return local_matrix(m, cf, k, l, cls, nodes, L);
}

/* signed area of T_l n polygon(x): used by tests of the clipping */
double orc_clip_area(const orc_cfg *cf, const double *x, const orc_mesh *m, int32_t ll, int32_t *cnt_out)
{
    elem_t l;
    double poly[MAXPOLY][2];
    load_elem(m, ll, &l);
    int cnt = ball_polygon(cf, x, &l, poly);
    *cnt_out = cnt;
    if (cnt < 3) return 0.0;
    return shoelace((const double (*)[2])poly, cnt);
}

/* ------------------------------------------------------------------ */
/* assembly: sum of local contributions over all listed ordered pairs    */
/* into a CSR pattern (eq. biFormApprox).  Row (n*node + comp) receives   */
/* entries only if node is a degree of freedom and, when rowsel is given, */
/* rowsel[node] is set.                                                 */

static int64_t find_slot(const int64_t *row_ptr, const int32_t *col, int64_t row, int32_t c)
{
    int64_t lo = row_ptr[row], hi = row_ptr[row + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (col[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    if (lo < row_ptr[row + 1] && col[lo] == c) return lo;
    return -1;
}

int orc_assemble(const orc_mesh *m, const orc_cfg *cf, int64_t npairs, const int32_t *pk,
                 const int32_t *pl, const int8_t *pcls, const uint8_t *isdof, const uint8_t *rowsel,
                 const int64_t *row_ptr, const int32_t *col, double *val)
{
    const int n = cf->ncomp;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < npairs; ++t) {
        int32_t nodes[MAXU];
        double L[(MAXU * 2) * (MAXU * 2)];
        int nu = local_matrix(m, cf, pk[t], pl[t], pcls[t], nodes, L);
        int dim = nu * n;
        for (int a = 0; a < nu; ++a) {
            if (!isdof[nodes[a]]) continue;
            if (rowsel && !rowsel[nodes[a]]) continue;
            for (int c = 0; c < n; ++c) {
                int64_t row = (int64_t)n * nodes[a] + c;
                for (int b = 0; b < nu; ++b)
                    for (int d = 0; d < n; ++d) {
                        int32_t cc = n * nodes[b] + d;
                        int64_t s = find_slot(row_ptr, col, row, cc);
                        if (s < 0) {
#pragma omp atomic write
                            err = 1;
                            continue;
                        }
                        double v = L[(a * n + c) * dim + (b * n + d)];
#pragma omp atomic
                        val[s] += v;
                    }
            }
        }
    }
    return err ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* load vector: b_(n i + c) = sum over Omega elements T containing node i of */
/* |J_T| sum_p d_p f_c(x_p) phi^_(loc i)(xi_p).  f is either given at the      */
/* outer quadrature points (fqp[K][P][n]) or affine:                         */
/* f_c(x) = aff[3c] + aff[3c+1] x_1 + aff[3c+2] x_2.                          */

int orc_rhs(const orc_mesh *m, const orc_cfg *cf, const double *fqp, const double *aff, double *b)
{
    const int n = cf->ncomp;
    const int64_t nunk = cf->dg ? 3 * m->n_elements : m->n_vertices;
    memset(b, 0, sizeof(double) * (size_t)(n * nunk));
    for (int64_t kk = 0; kk < m->n_elements; ++kk) {
        if (m->labels[kk] != 1) continue;
        elem_t k;
        load_elem(m, kk, &k);
        if (cf->dg) dg_ids(m, kk, &k);
        for (int p = 0; p < cf->P; ++p) {
            double x[2], ph[3];
            to_phys(&k, &cf->pxi[2 * p], x);
            phihat(&cf->pxi[2 * p], ph);
            for (int c = 0; c < n; ++c) {
                double f = fqp ? fqp[(kk * cf->P + p) * n + c]
                               : aff[3 * c] + aff[3 * c + 1] * x[0] + aff[3 * c + 2] * x[1];
                for (int a = 0; a < 3; ++a)
                    b[(int64_t)n * k.node[a] + c] += k.absdet * cf->pw[p] * f * ph[a];
            }
        }
    }
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

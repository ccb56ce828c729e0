// Interaction search (Sec. 2.5): all element pairs (e, f) that interact,
// found with a uniform bucket grid over the barycentres instead of the
// breadth-first traversal of Alg. 2.
//
// A block owns a tile of up to kTE elements of one grid cell and streams the
// elements of the (2 gr + 1)^2 neighbouring cells through LDS in chunks of
// kCH candidates.  Each wave takes one element e of the tile at a time and
// tests 64 candidates per step, one per lane; ballots give every lane its
// output position in e's scratch segment, whose length is the number of
// candidates the search visits for e (counted when the grid is filled), so a
// single pass writes the entries and counts them; the list sort compacts
// the segments.
//
// For every unordered pair both directions are tested at once:
//   status_p(e -> f) for the outer points x_p of e against T_f, and
//   status_q(f -> e) for the outer points of f against T_e,
// so the symmetric neighbour list S(e) = {f : (e,f) or (f,e) interacts}
// and the unordered lists used by the assembly are built in one pass.
//
// All decisions are FP64 without contraction and follow the operation
// order of the plain definition:
//   barycentre ball: (x - b).(x - b) <= delta^2,
//   polygon ball: Sutherland-Hodgman clip of T_f by the regular N-gon around
//   x (vertex j = x + delta dir_j), nonzero shoelace area; the clip is only
//   run when cheap bounds cannot decide (vertices well inside the inscribed
//   circle: whole; triangle well outside the circumscribed circle: empty).
#include "caps.h"
#include "nlfem_internal.h"

#pragma clang fp contract(off)

namespace nlfem {
namespace {

constexpr int kTE = 64;      // elements of a cell per block
constexpr int kCH = 128;     // candidates staged per chunk
constexpr int kBlock = 256;  // four waves
constexpr int kMaxNbr = 49;  // neighbour cells for gr <= 3

struct PairArgs {
    int64_t K, K1;
    const int32_t *E;
    const int32_t *lab;
    const double *V;
    const double2 *bary;
    const double2 *xp;
    const int64_t *cell_start;
    const int32_t *cell_elems;
    int32_t gnx, gny, gr, P;
    int32_t singular, poly;
    int32_t caps;                  // 1 nocaps, 2 approximate caps (caps.h), 0 polygon clip
    double delta, delta2, reach2, rin2, out2;
    int64_t *lcnt;          // [kLsLast][K1] per-element counts
    unsigned long long *maxClip;   // bound on the vertex count of any straddling clip
    const double *dir;             // [N][2] polygon directions (device copy)
    const int64_t *scr;     // [K + 1] start of each element's scratch segment
    int32_t *snbr;
    uint8_t *sflag;
    uint2 *smask;           // (status of e's points seeing f, status of f's points seeing e)
    SpecGate gate;
};

// ---- polygon ball -------------------------------------------------------

__device__ double point_segment_dist2(double px, double py, double ax, double ay, double bx, double by)
{
    double ex = bx - ax, ey = by - ay;
    double l2 = ex * ex + ey * ey;
    double t = l2 > 0.0 ? ((px - ax) * ex + (py - ay) * ey) / l2 : 0.0;
    t = fmin(1.0, fmax(0.0, t));
    double dx = px - (ax + t * ex), dy = py - (ay + t * ey);
    return dx * dx + dy * dy;
}

__device__ double point_triangle_dist2(double px, double py, const double2 v[3])
{
    double s0 = (v[1].x - v[0].x) * (py - v[0].y) - (v[1].y - v[0].y) * (px - v[0].x);
    double s1 = (v[2].x - v[1].x) * (py - v[1].y) - (v[2].y - v[1].y) * (px - v[1].x);
    double s2 = (v[0].x - v[2].x) * (py - v[2].y) - (v[0].y - v[2].y) * (px - v[2].x);
    if ((s0 >= 0 && s1 >= 0 && s2 >= 0) || (s0 <= 0 && s1 <= 0 && s2 <= 0)) return 0.0;
    double d = point_segment_dist2(px, py, v[0].x, v[0].y, v[1].x, v[1].y);
    d = fmin(d, point_segment_dist2(px, py, v[1].x, v[1].y, v[2].x, v[2].y));
    d = fmin(d, point_segment_dist2(px, py, v[2].x, v[2].y, v[0].x, v[0].y));
    return d;
}

// The Sutherland-Hodgman clip of the plain definition (vertex j of the
// polygon at (x, y) + delta * dir_j, a point inside edge j iff
// cross(q_{j+1} - q_j, v - q_j) >= 0, crossing a + t (b - a) with
// t = d_a / (d_a - d_b)), same operation order; returns the status.  A pass
// in which every current vertex is inside outputs the list unchanged, so it
// is skipped without touching the buffers.
__device__ __noinline__ uint32_t clip_status(double x, double y, const double2 v[3], const double *dir, int N,
                                             double delta)
{
    double bx[2][kMaxPoly + 4], by[2][kMaxPoly + 4];
    for (int a = 0; a < 3; ++a) {
        bx[0][a] = v[a].x;
        by[0][a] = v[a].y;
    }
    // passes that cannot change a polygon derived from the triangle: every
    // vertex inside edge j by 1e-9 C |e| (C bounds the coordinates), far
    // above the rounding of any point a pass produces; skipping them gives
    // the same polygon bit for bit
    uint64_t act = 0;
    {
        const double C = fmax(fmax(fmax(fabs(x), fabs(y)), fmax(fabs(v[0].x), fabs(v[0].y))),
                              fmax(fmax(fabs(v[1].x), fabs(v[1].y)), fmax(fabs(v[2].x), fabs(v[2].y)))) +
                         delta;
        for (int j = 0; j < N; ++j) {
            const int j1 = j + 1 == N ? 0 : j + 1;
            const double qa0 = x + delta * dir[2 * j], qa1 = y + delta * dir[2 * j + 1];
            const double qb0 = x + delta * dir[2 * j1], qb1 = y + delta * dir[2 * j1 + 1];
            const double e0 = qb0 - qa0, e1 = qb1 - qa1;
            const double tol = 1e-9 * C * (fabs(e0) + fabs(e1));
            const double d0 = e0 * (v[0].y - qa1) - e1 * (v[0].x - qa0);
            const double d1 = e0 * (v[1].y - qa1) - e1 * (v[1].x - qa0);
            const double d2 = e0 * (v[2].y - qa1) - e1 * (v[2].x - qa0);
            if (!(d0 > tol && d1 > tol && d2 > tol)) act |= 1ull << j;
        }
    }
    int cnt = 3, cur = 0;
    for (uint64_t rest = act; rest && cnt > 0; rest &= rest - 1) {
        const int j = __ffsll((unsigned long long)rest) - 1;
        int j1 = j + 1 == N ? 0 : j + 1;
        double qa0 = x + delta * dir[2 * j];
        double qa1 = y + delta * dir[2 * j + 1];
        double qb0 = x + delta * dir[2 * j1];
        double qb1 = y + delta * dir[2 * j1 + 1];
        double e0 = qb0 - qa0, e1 = qb1 - qa1;
        bool cuts = false;
        for (int i = 0; i < cnt; ++i)
            cuts |= !(e0 * (by[cur][i] - qa1) - e1 * (bx[cur][i] - qa0) >= 0.0);
        if (!cuts) continue;
        int nxt = 1 - cur, m = 0;
        for (int i = 0; i < cnt; ++i) {
            int i1 = i + 1 == cnt ? 0 : i + 1;
            double p0 = bx[cur][i], p1 = by[cur][i];
            double q0 = bx[cur][i1], q1 = by[cur][i1];
            double dp = e0 * (p1 - qa1) - e1 * (p0 - qa0);
            double dq = e0 * (q1 - qa1) - e1 * (q0 - qa0);
            bool pin = dp >= 0.0, qin = dq >= 0.0;
            if (pin) {
                bx[nxt][m] = p0;
                by[nxt][m] = p1;
                m++;
            }
            if (pin != qin) {
                double t = dp / (dp - dq);
                bx[nxt][m] = p0 + t * (q0 - p0);
                by[nxt][m] = p1 + t * (q1 - p1);
                m++;
            }
        }
        cnt = m;
        cur = nxt;
    }
    if (cnt < 3) return kOut;
    double s = 0.0;
    for (int i = 0; i < cnt; ++i) {
        int i1 = (i + 1) % cnt;
        s += bx[cur][i] * by[cur][i1] - bx[cur][i1] * by[cur][i];
    }
    double area = 0.5 * s;
    if (!(fabs(area) > 0.0)) return kOut;
    if (cnt == 3 && bx[cur][0] == v[0].x && by[cur][0] == v[0].y && bx[cur][1] == v[1].x &&
        by[cur][1] == v[1].y && bx[cur][2] == v[2].x && by[cur][2] == v[2].y)
        return kWhole;
    return kStraddle;
}

// sine of the triangle's angle at vertex a
__device__ inline double corner_sine(const double2 v[3], int a)
{
    const double2 p = v[a], q = v[a == 2 ? 0 : a + 1], r = v[a == 0 ? 2 : a - 1];
    const double ux = q.x - p.x, uy = q.y - p.y, wx = r.x - p.x, wy = r.y - p.y;
    return fabs(ux * wy - uy * wx) / (sqrt(ux * ux + uy * uy) * sqrt(wx * wx + wy * wy));
}

// Status of the outer point (x, y) for the triangle v under the polygon ball
// when poly_quick is unsure: the decisions of clip_status, taken from the
// edge tests of the original
// vertices (the clip's own arithmetic) wherever they fix the result:
//  - the clip returns the triangle unchanged iff every vertex passes every
//    edge test: whole;
//  - if all three vertices fail one edge test by a margin, every point the
//    clip can produce fails it (crossing points are convex combinations up
//    to rounding far below the margin): out;
//  - if one vertex passes every test by a margin and the triangle is no
//    sliver there, the clipped polygon keeps a corner of the triangle whose
//    area is orders of magnitude above the rounding of the area sum:
//    straddle.
// Otherwise the clip runs.  For straddling points *maxcnt is raised to
// 3 + 2 * (edges at which some vertex is not inside by the margin), a bound
// on every intermediate vertex count of the clip.
// The distance tests alone: whole if the triangle lies inside the inscribed
// circle, out if it is farther than delta; kUnsure otherwise.
constexpr uint32_t kUnsure = 3u;
template <bool CAPS>
__device__ inline uint32_t poly_quick(double x, double y, const double2 v[3], const PairArgs &a)
{
    double d0 = (v[0].x - x) * (v[0].x - x) + (v[0].y - y) * (v[0].y - y);
    double d1 = (v[1].x - x) * (v[1].x - x) + (v[1].y - y) * (v[1].y - y);
    double d2 = (v[2].x - x) * (v[2].x - x) + (v[2].y - y) * (v[2].y - y);
    // caps: whole exactly when every vertex lies in the closed disc (the
    // construction's own test)
    if (CAPS) {
        if (d0 <= a.delta2 && d1 <= a.delta2 && d2 <= a.delta2) return kWhole;
    } else if (d0 < a.rin2 && d1 < a.rin2 && d2 < a.rin2) {
        return kWhole;
    }
    if (point_triangle_dist2(x, y, v) > a.out2) return kOut;
    return kUnsure;
}

template <bool CAPS>
__device__ inline uint32_t poly_status(double x, double y, const double2 v[3], const PolyArgs &pg,
                                       const PairArgs &a, int *maxcnt)
{
    if constexpr (CAPS) {
        const double vx[3] = {v[0].x, v[1].x, v[2].x}, vy[3] = {v[0].y, v[1].y, v[2].y};
        double px[kMaxCaps], py[kMaxCaps];
        const int n = caps_polygon(x, y, vx, vy, a.delta, a.caps == 2, px, py);
        if (n < 3) return kOut;
        if (n == 3 && px[0] == vx[0] && py[0] == vy[0] && px[1] == vx[1] && py[1] == vy[1] && px[2] == vx[2] &&
            py[2] == vy[2])
            return kWhole;
        if (!(fabs(caps_area(px, py, n)) > 0.0)) return kOut;
        *maxcnt = max(*maxcnt, n);
        return kStraddle;
    } else {
        const double C = fmax(fabs(x), fabs(y)) + a.delta;
        const double m_out = 1e-9 * C, m_in = 1e-5 * C;   // margins as distances
        const int N = pg.N;
        bool all_in = true, sep = false, deep0 = true, deep1 = true, deep2 = true;
        int near = 0;
        // the directions and edge lengths from the kernel arguments (scalar
        // loads: j is uniform); vertex j + 1 of one edge is vertex j of the next
        double qa0 = x + a.delta * pg.dir[0][0];
        double qa1 = y + a.delta * pg.dir[0][1];
        for (int j = 0; j < N; ++j) {
            const int j1 = j + 1 == N ? 0 : j + 1;
            const double qb0 = x + a.delta * pg.dir[j1][0];
            const double qb1 = y + a.delta * pg.dir[j1][1];
            const double e0 = qb0 - qa0, e1 = qb1 - qa1;
            const double p0 = e0 * (v[0].y - qa1) - e1 * (v[0].x - qa0);
            const double p1 = e0 * (v[1].y - qa1) - e1 * (v[1].x - qa0);
            const double p2 = e0 * (v[2].y - qa1) - e1 * (v[2].x - qa0);
            // the edge length only scales the margins: the precomputed one
            const double el = pg.elen[j];
            const double tin = m_in * el, tout = m_out * el;
            all_in &= p0 >= 0.0 && p1 >= 0.0 && p2 >= 0.0;
            sep |= p0 < -tout && p1 < -tout && p2 < -tout;
            deep0 &= p0 > tin;
            deep1 &= p1 > tin;
            deep2 &= p2 > tin;
            near += (p0 < tout || p1 < tout || p2 < tout) ? 1 : 0;
            qa0 = qb0;
            qa1 = qb1;
        }
        if (all_in) return kWhole;
        if (sep) return kOut;
        const bool deep = (deep0 && corner_sine(v, 0) > 1e-3) || (deep1 && corner_sine(v, 1) > 1e-3) ||
                          (deep2 && corner_sine(v, 2) > 1e-3);
        const uint32_t st = deep ? kStraddle : clip_status(x, y, v, a.dir, N, a.delta);
        if (st == kStraddle) *maxcnt = max(*maxcnt, 3 + 2 * near);
        return st;
    }
}

// ---- the tile kernel --------------------------------------------------------

// MODE: 0 barycentre ball, 1 polygon clip (N-gon, square), 2 caps; the caps
// construction is compiled only into its own kernel (its arrays would
// otherwise raise the register count of the polygon kernel)
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_pairs(PairArgs a, PolyArgs pg)
{
    extern __shared__ __align__(16) unsigned char smem[];
    if (gated(a.gate)) return;
    const int64_t ncell = (int64_t)a.gnx * a.gny;
    const int64_t cell64 = xcd_item(blockIdx.x, ncell);   // grid.x is a multiple of 8
    if (cell64 >= ncell) return;
    constexpr bool POLY = MODE > 0, CAPS = MODE == 2;
    const int cell = (int)cell64;
    const int64_t cs = a.cell_start[cell], ce = a.cell_start[cell + 1];
    if (cs >= ce) return;
    const int cx = cell % a.gnx, cy = cell / a.gnx;

    double2 *c_b = (double2 *)smem;                       // [kCH]
    double2 *c_xp = c_b + kCH;                            // [P][kCH]
    double2 *c_v = c_xp + a.P * kCH;                      // [3][kCH] (polygon ball)
    int64_t *e_off = (int64_t *)(c_v + (POLY ? 3 * kCH : 0));   // [kTE][kLsLast]
    int32_t *c_id = (int32_t *)(e_off + kTE * kLsLast);   // [kCH]
    int32_t *c_lab = c_id + kCH;                          // [kCH]
    int32_t *c_nd = c_lab + kCH;                          // [3][kCH]
    __shared__ int64_t nb_start[kMaxNbr], nb_pre[kMaxNbr + 1];
    __shared__ int64_t e_scr[kTE];   // scratch segment of each tile element
    __shared__ int nb_n;
    // polygon ball: per wave, queue of unsure (candidate, direction, point)
    // items and the statuses they decide
    __shared__ int32_t pq_all[POLY ? kBlock / 64 : 1][POLY ? 64 * 2 * kMaxRule : 1];
    __shared__ uint32_t pm_all[POLY ? kBlock / 64 : 1][2][64];
    // per wave: the chunk positions of the candidates that can interact with
    // the wave's current element, in chunk order
    __shared__ int16_t cand_all[kBlock / 64][kCH];

    // the neighbour cells (row-major, clipped to the grid): one lane each, so
    // their counts load in parallel, then a prefix sum across the wave
    if (threadIdx.x < 64) {
        const int side = 2 * a.gr + 1;
        const int t = threadIdx.x;
        const int yy = cy - a.gr + t / side, xx = cx - a.gr + t % side;
        const bool in = t < side * side && yy >= 0 && yy < a.gny && xx >= 0 && xx < a.gnx;
        int64_t st = 0, cnt = 0;
        if (in) {
            const int c = yy * a.gnx + xx;
            st = a.cell_start[c];
            cnt = a.cell_start[c + 1] - st;
        }
        const unsigned long long bin = __ballot(in);
        const int slot = __popcll(bin & ((1ull << t) - 1ull));
        int64_t incl = cnt;
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(incl, o);
            if (t >= o) incl += y;
        }
        if (in) {
            nb_start[slot] = st;
            nb_pre[slot] = incl - cnt;
        }
        if (t == 63) {
            nb_n = __popcll(bin);
            nb_pre[__popcll(bin)] = incl;
        }
    }
    __syncthreads();
    const int64_t total = nb_pre[nb_n];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const unsigned long long lt = (1ull << lane) - 1ull;
    int clipmax = 0;
    int32_t *pq = pq_all[POLY ? wv : 0];
    uint32_t *pm_ef = pm_all[POLY ? wv : 0][0], *pm_fe = pm_all[POLY ? wv : 0][1];
    // the cell's elements in tiles of kTE
    for (int64_t t0 = cs; t0 < ce; t0 += kTE) {
        const int ne = (int)min((int64_t)kTE, ce - t0);
        for (int t = threadIdx.x; t < kTE * kLsLast; t += kBlock) e_off[t] = 0;
        if (threadIdx.x < ne) e_scr[threadIdx.x] = a.scr[a.cell_elems[t0 + threadIdx.x]];
        __syncthreads();

        for (int64_t c0 = 0; c0 < total; c0 += kCH) {
            const int nch = (int)min((int64_t)kCH, total - c0);
            if (threadIdx.x < nch) {
                const int64_t g = c0 + threadIdx.x;
                int j = 0;
                while (nb_pre[j + 1] <= g) ++j;
                const int32_t f = a.cell_elems[nb_start[j] + (g - nb_pre[j])];
                const int t = threadIdx.x;
                c_id[t] = f;
                c_lab[t] = a.lab[f];
                c_nd[t] = a.E[3 * (int64_t)f];
                c_nd[kCH + t] = a.E[3 * (int64_t)f + 1];
                c_nd[2 * kCH + t] = a.E[3 * (int64_t)f + 2];
                c_b[t] = a.bary[f];
                for (int p = 0; p < a.P; ++p) c_xp[p * kCH + t] = a.xp[(int64_t)f * a.P + p];
                if (POLY)
                    for (int v = 0; v < 3; ++v) {
                        int32_t n = c_nd[v * kCH + t];
                        c_v[v * kCH + t] = make_double2(a.V[2 * (int64_t)n], a.V[2 * (int64_t)n + 1]);
                    }
            }
            __syncthreads();
            for (int i = wv; i < ne; i += 4) {
                const int32_t e = a.cell_elems[t0 + i];
                const int32_t lab_e = a.lab[e];
                const int32_t ne0 = a.E[3 * (int64_t)e], ne1 = a.E[3 * (int64_t)e + 1],
                              ne2 = a.E[3 * (int64_t)e + 2];
                const double2 be = a.bary[e];
                double2 ve[3];
                if (POLY) {
                    ve[0] = make_double2(a.V[2 * (int64_t)ne0], a.V[2 * (int64_t)ne0 + 1]);
                    ve[1] = make_double2(a.V[2 * (int64_t)ne1], a.V[2 * (int64_t)ne1 + 1]);
                    ve[2] = make_double2(a.V[2 * (int64_t)ne2], a.V[2 * (int64_t)ne2 + 1]);
                }
                int64_t off[kLsLast];
                for (int k = 0; k < kLsLast; ++k) off[k] = e_off[i * kLsLast + k];

                // keep the candidates that are active and touching or within
                // reach of the barycentre, so the point tests below run on
                // full waves
                int16_t *cand = cand_all[wv];
                int ncand = 0;
                wave_sync();   // the previous element's reads of cand are done
                for (int jj = 0; jj < nch; jj += 64) {
                    const int j = jj + lane;
                    bool keep = false;
                    if (j < nch) {
                        const int32_t lab_f = c_lab[j];
                        const bool act = (lab_f == 1 || lab_f == 2) && (lab_e == 1 || lab_f == 1);
                        const int32_t f0 = c_nd[j], f1 = c_nd[kCH + j], f2 = c_nd[2 * kCH + j];
                        const bool sh = ne0 == f0 || ne0 == f1 || ne0 == f2 || ne1 == f0 || ne1 == f1 ||
                                        ne1 == f2 || ne2 == f0 || ne2 == f1 || ne2 == f2;
                        if (act && a.singular && sh) {
                            keep = true;
                        } else if (act) {
                            const double2 bf = c_b[j];
                            const double dbx = be.x - bf.x, dby = be.y - bf.y;
                            keep = dbx * dbx + dby * dby <= a.reach2;
                        }
                    }
                    const unsigned long long bk = __ballot(keep);
                    if (keep) cand[ncand + __popcll(bk & lt)] = (int16_t)j;
                    ncand += __popcll(bk);
                }
                wave_sync();
                for (int kb = 0; kb < ncand; kb += 64) {
                    const bool valid = kb + lane < ncand;
                    const int j = valid ? cand[kb + lane] : 0;
                    bool inS = false, inP = false, isUF = false;
                    int cls = 0;
                    uint32_t mef = 0, mfe = 0;
                    int32_t f = -1;
                    uint8_t flags = 0;
                    bool need = false;   // polygon ball: the point tests of this lane's candidate run
                    if (valid) {
                        f = c_id[j];
                        const int32_t lab_f = c_lab[j];
                        const bool act = (lab_f == 1 || lab_f == 2) && (lab_e == 1 || lab_f == 1);
                        const int32_t f0 = c_nd[j], f1 = c_nd[kCH + j], f2 = c_nd[2 * kCH + j];
                        const int shared = (ne0 == f0) + (ne0 == f1) + (ne0 == f2) + (ne1 == f0) +
                                           (ne1 == f1) + (ne1 == f2) + (ne2 == f0) + (ne2 == f1) +
                                           (ne2 == f2);
                        const bool touch = a.singular && shared > 0;
                        if (act && !touch) {
                            const double2 bf = c_b[j];
                            const double dbx = be.x - bf.x, dby = be.y - bf.y;
                            if (dbx * dbx + dby * dby <= a.reach2) {
                                if (!POLY) {
                                    for (int p = 0; p < a.P; ++p) {
                                        const double2 x = a.xp[(int64_t)e * a.P + p];
                                        const double dx = x.x - bf.x, dy = x.y - bf.y;
                                        if (dx * dx + dy * dy <= a.delta2) mef |= kWhole << (2 * p);
                                    }
                                    for (int q = 0; q < a.P; ++q) {
                                        const double2 x = c_xp[q * kCH + j];
                                        const double dx = x.x - be.x, dy = x.y - be.y;
                                        if (dx * dx + dy * dy <= a.delta2) mfe |= kWhole << (2 * q);
                                    }
                                } else {
                                    need = true;
                                }
                            }
                        }
                    }
                    if (POLY) {
                        // distance tests by all lanes in step (one point per step), the
                        // unsure (point, triangle) items appended to the wave's queue by
                        // ballot positions, then decided by all lanes at once
                        int nq = 0;
                        {
                            const int jn = need ? j : 0;
                            const double2 vf[3] = {c_v[jn], c_v[kCH + jn], c_v[2 * kCH + jn]};
                            for (int p = 0; p < a.P; ++p) {
                                uint32_t st = kOut;
                                if (need) {
                                    const double2 x = a.xp[(int64_t)e * a.P + p];
                                    st = poly_quick<CAPS>(x.x, x.y, vf, a);
                                }
                                const bool u = st == kUnsure;
                                const unsigned long long m = __ballot(u);
                                if (u) pq[nq + __popcll(m & lt)] = (lane << 5) | p;
                                else mef |= st << (2 * p);
                                nq += __popcll(m);
                            }
                            for (int q = 0; q < a.P; ++q) {
                                uint32_t st = kOut;
                                if (need) {
                                    const double2 x = c_xp[q * kCH + jn];
                                    st = poly_quick<CAPS>(x.x, x.y, ve, a);
                                }
                                const bool u = st == kUnsure;
                                const unsigned long long m = __ballot(u);
                                if (u) pq[nq + __popcll(m & lt)] = (lane << 5) | 16 | q;
                                else mfe |= st << (2 * q);
                                nq += __popcll(m);
                            }
                        }
                        // decide the queued items, one per lane
                        wave_sync();
                        pm_ef[lane] = 0u;
                        pm_fe[lane] = 0u;
                        wave_sync();
                        for (int it = lane; it < nq; it += 64) {
                            const int code = pq[it];
                            const int jl = code >> 5, fe_dir = code & 16, p = code & 15;
                            const int jc = cand[kb + jl];   // chunk slot of lane jl's candidate
                            uint32_t st;
                            if (!fe_dir) {
                                const double2 x = a.xp[(int64_t)e * a.P + p];
                                double2 vf[3] = {c_v[jc], c_v[kCH + jc], c_v[2 * kCH + jc]};
                                st = poly_status<CAPS>(x.x, x.y, vf, pg, a, &clipmax);
                                atomicOr(&pm_ef[jl], st << (2 * p));
                            } else {
                                const double2 x = c_xp[p * kCH + jc];
                                st = poly_status<CAPS>(x.x, x.y, ve, pg, a, &clipmax);
                                atomicOr(&pm_fe[jl], st << (2 * p));
                            }
                        }
                        wave_sync();
                        mef |= pm_ef[lane];
                        mfe |= pm_fe[lane];
                        wave_sync();
                    }
                    if (valid) {
                        const bool act = (c_lab[j] == 1 || c_lab[j] == 2) && (lab_e == 1 || c_lab[j] == 1);
                        const int32_t f0 = c_nd[j], f1 = c_nd[kCH + j], f2 = c_nd[2 * kCH + j];
                        const int shared = (ne0 == f0) + (ne0 == f1) + (ne0 == f2) + (ne1 == f0) +
                                           (ne1 == f1) + (ne1 == f2) + (ne2 == f0) + (ne2 == f1) +
                                           (ne2 == f2);
                        const bool touch = a.singular && shared > 0;
                        if (touch) cls = shared;
                        inS = act && (touch || (mef | mfe) != 0u);
                        inP = act && (touch || mef != 0u);
                        flags = (uint8_t)((touch ? 3 : ((mef != 0u) | ((mfe != 0u) << 1))) | (cls << 2));
                        isUF = inS && !touch && f >= e;
                    }
                    const unsigned long long bS = __ballot(inS);
                    const unsigned long long bP = __ballot(inP);
                    const unsigned long long bF = __ballot(isUF);
                    const unsigned long long bI = __ballot(inS && cls == 3);
                    const unsigned long long bE = __ballot(inS && cls == 2 && f > e);
                    const unsigned long long bV = __ballot(inS && cls == 1 && f > e);
                    if (inS) {
                        const int64_t o = e_scr[i] + off[kLsS] + __popcll(bS & lt);
                        a.snbr[o] = f;
                        a.sflag[o] = flags;
                        a.smask[o] = make_uint2(mef, mfe);
                    }
                    off[kLsS] += __popcll(bS);
                    off[kLsP] += __popcll(bP);
                    off[kLsUF] += __popcll(bF);
                    off[kLsUI] += __popcll(bI);
                    off[kLsUE] += __popcll(bE);
                    off[kLsUV] += __popcll(bV);
                }
                if (lane == 0)
                    for (int k = 0; k < kLsLast; ++k) e_off[i * kLsLast + k] = off[k];
            }
            __syncthreads();
        }
        for (int t = threadIdx.x; t < ne * kLsLast; t += kBlock) {
            int i = t / kLsLast, kind = t % kLsLast;
            a.lcnt[kind * a.K1 + a.cell_elems[t0 + i]] = e_off[t];
        }
        __syncthreads();
    }
    if (POLY && clipmax > 0) atomicMax(a.maxClip, (unsigned long long)clipmax);
}

// ---- grid build ---------------------------------------------------------------

// Per element: its three node -> element incidences and its grid cell (by
// barycentre; elements outside the domain labels get no cell).  Counting and
// filling use atomics, so the order within an incidence list or a cell is
// arbitrary; every consumer either sorts (neighbour lists, CSR columns) or
// does not depend on it.
struct BucketArgs {
    int64_t K, M;
    const int32_t *E, *lab;
    const double2 *bary;
    double x0, y0, h;
    int32_t nx, ny;
    int64_t *cell_cnt;
    const int64_t *cell_start;
    int32_t *cell_fill, *cell_elems, *cell_of;
    int64_t *inc_cnt;              // bucket count; cleared by the bucket fill
    const int64_t *inc_ptr;
    int32_t *inc_fill, *inc_list;
    const uint32_t *node_flags;    // 1: dof node
    const double *V;
    int32_t morton_bits;           // < 0: row-major cell index as the code
    int32_t *node_code;            // [M] code of a dof node, -1 otherwise
    int64_t *code_cnt;             // bucket count
    const int64_t *code_start;     // bucket fill
    int32_t *code_fill;
    int32_t *dof_list;
    int32_t gr;                    // neighbour-cell radius of the pair search
    int64_t *cand;                 // fill pass: [K] candidates of each element
    int64_t elem_blocks;           // blocks over elements, then over nodes
    SpecGate gate;
};

// interleaves the low 16 bits of v with zeros
__device__ inline uint32_t spread_bits(uint32_t v)
{
    v &= 0xffffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

// code of the grid cell of point (x, y): its position in the order of the rows
__device__ inline int32_t cell_code(const BucketArgs &a, double x, double y)
{
    int cx = (int)floor((x - a.x0) / a.h), cy = (int)floor((y - a.y0) / a.h);
    cx = min(max(cx, 0), a.nx - 1);
    cy = min(max(cy, 0), a.ny - 1);
    if (a.morton_bits < 0) return cy * a.nx + cx;
    return (int32_t)(spread_bits((uint32_t)cx) | (spread_bits((uint32_t)cy) << 1));
}

// count pass over the nodes: the dof nodes per code
__device__ void node_count(const BucketArgs &a, int64_t n)
{
    if (n >= a.M) return;
    int32_t code = -1;
    if (a.node_flags[n] == 1u) {
        code = cell_code(a, a.V[2 * n], a.V[2 * n + 1]);
        atomicAdd((unsigned long long *)&a.code_cnt[code], 1ull);
    }
    a.node_code[n] = code;
}

__global__ void __launch_bounds__(256) k_bucket_count(BucketArgs a)
{
    if (gated(a.gate)) return;
    if ((int64_t)blockIdx.x >= a.elem_blocks) {
        node_count(a, ((int64_t)blockIdx.x - a.elem_blocks) * 256 + threadIdx.x);
        return;
    }
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.K) return;
    for (int v = 0; v < 3; ++v) {
        const int32_t n = a.E[3 * k + v];
        if (n >= 0 && n < a.M) atomicAdd((unsigned long long *)&a.inc_cnt[n], 1ull);
    }
    const int32_t l = a.lab[k];
    if (l != 1 && l != 2) {
        a.cell_of[k] = -1;
        return;
    }
    const double2 b = a.bary[k];
    int cx = (int)floor((b.x - a.x0) / a.h), cy = (int)floor((b.y - a.y0) / a.h);
    cx = min(max(cx, 0), a.nx - 1);
    cy = min(max(cy, 0), a.ny - 1);
    const int c = cy * a.nx + cx;
    a.cell_of[k] = c;
    atomicAdd((unsigned long long *)&a.cell_cnt[c], 1ull);
}

// fill pass over the nodes: the dof list in code order (arbitrary within a
// code); also clears the CSR row lengths (the incidence counts, scanned by
// now) for the symbolic pass
__device__ void node_fill(const BucketArgs &a, int64_t n)
{
    if (n >= a.M) return;
    a.inc_cnt[n] = 0;
    const int32_t code = a.node_code[n];
    if (code < 0) return;
    const int32_t pos = atomicAdd(&a.code_fill[code], 1);
    a.dof_list[a.code_start[code] + pos] = (int32_t)n;
}

__global__ void __launch_bounds__(256) k_bucket_fill(BucketArgs a)
{
    if (gated(a.gate)) return;
    if ((int64_t)blockIdx.x >= a.elem_blocks) {
        node_fill(a, ((int64_t)blockIdx.x - a.elem_blocks) * 256 + threadIdx.x);
        return;
    }
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.K) return;
    for (int v = 0; v < 3; ++v) {
        const int32_t n = a.E[3 * k + v];
        if (n >= 0 && n < a.M) {
            const int32_t pos = atomicAdd(&a.inc_fill[n], 1);
            a.inc_list[a.inc_ptr[n] + pos] = (int32_t)k;
        }
    }
    const int c = a.cell_of[k];
    int64_t cand = 0;
    if (c >= 0) {
        const int32_t pos = atomicAdd(&a.cell_fill[c], 1);
        a.cell_elems[a.cell_start[c] + pos] = (int32_t)k;
        // the elements of the neighbour cells the pair search visits: a
        // bound on |S(k)| that sizes k's segment of the search's output
        const int cx = c % a.nx, cy = c / a.nx;
        for (int yy = max(cy - a.gr, 0); yy <= min(cy + a.gr, a.ny - 1); ++yy) {
            const int64_t r = (int64_t)yy * a.nx;
            const int x0 = max(cx - a.gr, 0), x1 = min(cx + a.gr, a.nx - 1);
            cand += a.cell_start[r + x1 + 1] - a.cell_start[r + x0];
        }
    }
    a.cand[k] = cand;
}

BucketArgs bucket_args(nlfem_pairs *h, const nlfem_mesh *m)
{
    BucketArgs a{};
    a.K = h->K;
    a.M = h->M;
    a.E = m->elements;
    a.lab = h->mesh_labels;
    a.bary = h->bary;
    a.x0 = h->gx0;
    a.y0 = h->gy0;
    a.h = h->gh;
    a.nx = h->gnx;
    a.ny = h->gny;
    a.cell_cnt = h->cell_cnt;
    a.cell_start = h->cell_start;
    a.cell_fill = h->cell_fill;
    a.cell_elems = h->cell_elems;
    a.cell_of = h->cell_of;
    a.inc_cnt = h->nlen;
    a.inc_ptr = h->ne_ptr;
    a.inc_fill = h->ne_fill;
    a.inc_list = h->ne_list;
    a.node_flags = h->node_flags;
    a.V = m->vertices;
    a.morton_bits = h->morton_bits;
    a.node_code = h->node_code;
    a.code_cnt = h->code_cnt;
    a.code_start = h->code_start;
    a.code_fill = h->code_fill;
    a.dof_list = h->dof_list;
    a.gr = h->gr;
    a.cand = h->cand;
    a.elem_blocks = grid_for(h->K, 256);
    a.gate = h->gate;
    return a;
}

}  // namespace

int launch_bucket_count(nlfem_pairs *h, const nlfem_mesh *m, hipStream_t s)
{
    const BucketArgs a = bucket_args(h, m);
    const int64_t blocks = a.elem_blocks + grid_for(h->M, 256);
    if (blocks > 0) hipLaunchKernelGGL(k_bucket_count, dim3((unsigned)blocks), dim3(256), 0, s, a);
    NLFEM_HIP(hipGetLastError());
    return NLFEM_OK;
}

int launch_bucket_fill(nlfem_pairs *h, const nlfem_mesh *m, hipStream_t s)
{
    const BucketArgs a = bucket_args(h, m);
    const int64_t blocks = a.elem_blocks + grid_for(h->M, 256);
    if (blocks > 0) hipLaunchKernelGGL(k_bucket_fill, dim3((unsigned)blocks), dim3(256), 0, s, a);
    NLFEM_HIP(hipGetLastError());
    return NLFEM_OK;
}

int launch_pairs(nlfem_pairs *h, const nlfem_mesh *m, hipStream_t s)
{
    const int64_t ncell = (int64_t)h->gnx * h->gny;
    if ((2 * h->gr + 1) * (2 * h->gr + 1) > kMaxNbr)
        return set_error(NLFEM_E_INVALID, "grid neighbour radius too large");
    PairArgs a{};
    a.K = h->K;
    a.K1 = h->K + 1;
    a.E = m->elements;
    a.lab = m->labels;
    a.V = m->vertices;
    a.bary = h->bary;
    a.xp = h->xp;
    a.cell_start = h->cell_start;
    a.cell_elems = h->cell_elems;
    a.gnx = h->gnx;
    a.gny = h->gny;
    a.gr = h->gr;
    a.P = h->rules.P;
    a.singular = h->singular;
    a.poly = clipped_ball(h->approach);
    a.caps = caps_mode(h->approach);
    a.delta = h->delta;
    a.delta2 = h->delta * h->delta;
    // conservative reach of a non-touching interaction between barycentres
    a.reach2 = h->far_reach * h->far_reach;
    const double rin = h->poly.r_in * (1.0 - 1e-12);
    a.rin2 = rin * rin;
    const double out = h->poly.r_out * (1.0 + 1e-12);   // the farthest polygon vertex
    a.out2 = out * out;
    a.lcnt = h->lcnt;
    a.maxClip = h->red + 10;
    a.dir = h->poly_dir;
    a.scr = h->scr_off;
    a.snbr = h->snbr_tmp;
    a.sflag = h->sflag_tmp;
    a.smask = h->smask_tmp;
    a.gate = h->gate;
    const size_t lds = sizeof(double2) * (size_t)kCH * (1 + a.P + (a.poly ? 3 : 0)) +
                       sizeof(int64_t) * kTE * kLsLast + sizeof(int32_t) * kCH * 5;
    dim3 grid(xcd_grid(ncell, INT32_MAX));
    if (a.caps) hipLaunchKernelGGL((k_pairs<2>), grid, dim3(kBlock), lds, s, a, h->poly);
    else if (a.poly) hipLaunchKernelGGL((k_pairs<1>), grid, dim3(kBlock), lds, s, a, h->poly);
    else hipLaunchKernelGGL((k_pairs<0>), grid, dim3(kBlock), lds, s, a, h->poly);
    NLFEM_HIP(hipGetLastError());
    return NLFEM_OK;
}

}  // namespace nlfem
